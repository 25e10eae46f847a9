"""FP64 CPU oracle of the DirectCF Lagrange–Remap step (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It loads ``liblr_ref.so`` built from
``lr_ref.c`` (``build.py`` in this folder) and shares no code with the GPU
library.
"""
from .ref import RefSolver, load, rect_halfplane_area, interface_offset  # noqa: F401
