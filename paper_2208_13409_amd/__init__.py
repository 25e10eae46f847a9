"""MI355X-native DirectCF multimaterial Lagrange–Remap step.

``paper_2208_13409_amd.lr`` is the ctypes binding of ``liblr.so`` (HIP kernels
for gfx950 behind the C-ABI declared in ``include/lr.h``);
``paper_2208_13409_amd.inputs`` holds the seeded synthetic workloads.  Nothing
is loaded at import time; the binding raises if the HIP library is missing.
"""
__all__ = ["lr", "inputs"]
