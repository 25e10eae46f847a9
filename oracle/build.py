"""Build the oracle shared library ``liblr_ref.so`` with the host C compiler.

Plain C99 at -O2 with floating-point contraction off, so that every
expression rounds in the order written.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "liblr_ref.so")


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "lr_ref.c")
    tmp = SO + ".tmp"
    cmd = ["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, SO)
    return SO


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
