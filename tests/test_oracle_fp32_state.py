"""The FP32-storage control of the oracle (oracle/fp32_state.py), on the CPU.

The control restarts the oracle from its own fields after every step.  Without
the rounding those restarts must leave the run where the plain oracle goes
(they change a value by at most an ulp or so), so that what the rounded run
shows is the single-precision storage and nothing of the harness.  The stored
curve (tests/golden/shock_bubble_64x64_fp32_state_control.json, written by
fp32_state_control.py beside it from the oracle alone) must be reproduced."""
import json
import os

import numpy as np
import pytest

from oracle import RefSolver
from oracle.fp32_state import run_stored

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "shock_bubble_64x64_fp32_state_control.json")


def _problem():
    from tests.golden.fp32_state_control import problem
    return problem()[1]


def _plain(p, marks, k_eps):
    r = RefSolver(p["nx"], p["ny"], p["gammas"], p["domain"], k_eps=k_eps)
    r.set_state(0.0, p["k"], p["rho"], p["e"], p["ux"], p["uy"])
    out, n = {}, 0
    for m in marks:
        r.run(1e30, max_steps=m - n)
        n = m
        out[m] = r.fields("rho", "p", "vol")
    return out


def test_restarts_alone_follow_the_plain_oracle():
    p = _problem()
    marks = [24, 48, 96]
    plain = _plain(p, marks, 1e-6)
    runs = run_stored(p, 96, set(marks), 1e-6, rounding=False)
    for m in marks:
        for f in ("rho", "p"):
            l1 = np.abs(runs[m][f] - plain[m][f]).sum() / np.abs(plain[m][f]).sum()
            assert l1 < 1e-13, (m, f, l1)


def test_fp32_storage_is_a_single_precision_perturbation_before_any_flip():
    """Before the two runs disagree on a material's presence, FP32 storage
    moves the density by FP32-sized amounts only (L1 near 1e-7)."""
    p = _problem()
    marks = [24, 48, 96]
    plain = _plain(p, marks, 1e-6)
    runs = run_stored(p, 96, set(marks), 1e-6, rounding=True)
    for m in marks:
        l1 = np.abs(runs[m]["rho"] - plain[m]["rho"]).sum() / np.abs(plain[m]["rho"]).sum()
        assert 1e-9 < l1 < 1e-6, (m, l1)


@pytest.mark.slow
def test_stored_control_curve_is_reproduced():
    with open(GOLDEN) as f:
        g = json.load(f)
    p = _problem()
    assert p["name"] == g["name"]
    marks = g["steps"]
    plain = _plain(p, marks, g["k_eps"])
    runs = run_stored(p, marks[-1], set(marks), g["k_eps"], rounding=True)
    for m, want in zip(marks, g["fp32_state"]["l1_rho"]):
        l1 = np.abs(runs[m]["rho"] - plain[m]["rho"]).sum() / np.abs(plain[m]["rho"]).sum()
        assert l1 == pytest.approx(want, rel=1e-6, abs=1e-15), m
