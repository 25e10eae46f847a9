"""Build the oracle shared libraries with the host C compiler.

Plain C99 at -O2 with floating-point contraction off, so that every
expression rounds in the order written.  ``liblr_ref.so`` is the
single-threaded build; ``liblr_ref_omp.so`` is the same source with OpenMP
over grid rows.  Every parallel loop writes only its own cell, node, face or
row entries (the gather form of the scheme), so both give the same bits.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "liblr_ref.so")
SO_OMP = os.path.join(HERE, "liblr_ref_omp.so")
FLAGS = ["-std=c99", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-Wall", "-Wextra"]


def _build_one(out, extra, verbose):
    src = os.path.join(HERE, "lr_ref.c")
    tmp = out + ".tmp"
    cmd = ["gcc", *FLAGS, *extra, "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build(verbose: bool = False) -> str:
    _build_one(SO_OMP, ["-fopenmp"], verbose)
    return _build_one(SO, ["-Wno-unknown-pragmas"], verbose)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
