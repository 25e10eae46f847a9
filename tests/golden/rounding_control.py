"""Writes triple_point_448x192_rounding_control.json: how far the FP64 oracle
drifts from itself on the triple point (448 x 192, 3 materials, t_end 3.5)
when its initial state changes by one unit in the last place (every partial
density times 1 + 2^-52).  Relative L1 of density and pressure between the two
runs and the worst per-cell mass difference (against the cell's mass), every
100 steps.  Only the oracle runs here.

The roll-up of the triple point amplifies any perturbation, so this curve is
the floor that any implementation whose rounding differs from the oracle's
(another evaluation order, FMA contraction, another closed form) is held to
over the whole run.  Usage: python tests/golden/rounding_control.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import RefSolver  # noqa: E402
from paper_2208_13409_amd import inputs  # noqa: E402


def main():
    p = inputs.triple_point(1)
    a = RefSolver(p["nx"], p["ny"], p["gammas"], p["domain"], omp=True)
    b = RefSolver(p["nx"], p["ny"], p["gammas"], p["domain"], omp=True)
    a.set_state(0.0, p["k"], p["rho"], p["e"], p["ux"], p["uy"])
    b.set_state(0.0, p["k"], p["rho"] * (1.0 + 2.0 ** -52), p["e"], p["ux"], p["uy"])
    curve, n = [], 0
    while True:
        na, ta = a.run(p["t_end"], 100)
        nb, tb = b.run(p["t_end"], 100)
        n += na
        fa, fb = a.fields("rho", "p", "mass"), b.fields("rho", "p", "mass")
        l1 = [float(np.abs(fa[k] - fb[k]).sum() / np.abs(fa[k]).sum()) for k in ("rho", "p")]
        cell = np.maximum(np.abs(fa["mass"]).sum(0), 1e-300)
        worst = float((np.abs(fa["mass"] - fb["mass"]) / cell).max())
        curve.append(dict(step=n, t=ta, l1_rho=l1[0], l1_p=l1[1], worst_cell_mass=worst))
        print(curve[-1], flush=True)
        if na == 0 or ta >= p["t_end"]:
            break
    out = dict(workload="triple_point_448x192", perturbation="rho * (1 + 2**-52) at t = 0",
               oracle="oracle/lr_ref.c (OpenMP build, same bits as the single-threaded one)", curve=curve)
    with open(os.path.join(HERE, "triple_point_448x192_rounding_control.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
