"""Writes shock_bubble_64x64_fp32_state_control.json: how far the FP64
oracle drifts from itself on the smallest problem of the 256-problem
shock-bubble batch (64 x 64 cells, two materials, presence threshold 1e-6)
when its conserved state is stored in FP32 between steps (oracle/fp32_state.py),
and, as the harness check, when the same restarts run without the rounding.
Relative L1 of density and pressure against the plain oracle every 24 steps
up to 408 (the batch benchmark's length), and the first checkpoint at which
the two runs disagree on which materials are present in some cell.  Only the
oracle runs here.

FP32 storage perturbs every step by about 1e-7 of each value.  Traces of a
material near the presence threshold (V_a / A within a few percent of 1e-6)
then fall on either side of it in the two runs, a cell turns mixed or pure,
and its neighbours' regions switch between the order-2 and the order-1
reconstruction (§4.2): a local change of a few percent of the density, which
the shock-bubble's instability then carries.  This curve is the floor that any
FP32 bulk implementation is held to on this problem.
Usage: python tests/golden/fp32_state_control.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import RefSolver  # noqa: E402
from oracle.fp32_state import run_stored  # noqa: E402
from paper_2208_13409_amd import inputs  # noqa: E402

STEPS, EVERY, K_EPS = 408, 24, 1e-6


def problem():
    """the smallest problem of inputs.shock_bubble_batch(256)"""
    probs = inputs.shock_bubble_batch(256)
    i = min(range(len(probs)), key=lambda b: probs[b]["nx"] * probs[b]["ny"])
    return i, probs[i]


def main():
    idx, p = problem()
    marks = list(range(EVERY, STEPS + 1, EVERY))
    r = RefSolver(p["nx"], p["ny"], p["gammas"], p["domain"], k_eps=K_EPS)
    r.set_state(0.0, p["k"], p["rho"], p["e"], p["ux"], p["uy"])
    plain = {}
    for m in marks:
        r.run(1e30, max_steps=EVERY)
        plain[m] = r.fields("rho", "p", "vol")
    x0, x1, y0, y1 = p["domain"]
    A = (x1 - x0) * (y1 - y0) / (p["nx"] * p["ny"])
    out = {"problem": f"shock_bubble_batch(256)[{idx}]", "name": p["name"], "grid": [p["nx"], p["ny"]],
           "k_eps": K_EPS, "steps": marks}
    for key, rounding in (("fp32_state", True), ("harness_only", False)):
        runs = run_stored(p, STEPS, set(marks), K_EPS, rounding)
        l1 = {f: [float(np.abs(runs[m][f] - plain[m][f]).sum() / np.abs(plain[m][f]).sum()) for m in marks]
              for f in ("rho", "p")}
        flip = next((m for m in marks
                     if np.any((runs[m]["vol"] > K_EPS * A) != (plain[m]["vol"] > K_EPS * A))), None)
        out[key] = {"l1_rho": l1["rho"], "l1_p": l1["p"], "first_presence_difference": flip}
        print(key, " ".join(f"{x:.1e}" for x in l1["rho"]), "first flip", flip, flush=True)
    with open(os.path.join(HERE, "shock_bubble_64x64_fp32_state_control.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
