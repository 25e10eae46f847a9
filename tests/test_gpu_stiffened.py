"""Stiffened gas (paper §5.2, p = (gamma-1) rho e - pi) on the GPU against the
FP64 oracle, whose stiffened form is pinned by the exact Riemann solution of
a water-air tube (tests/test_oracle_pins.py)."""
import sys

import numpy as np
import pytest

from oracle import RefSolver
from paper_2208_13409_amd import inputs
from paper_2208_13409_amd.lr import Solver

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_l1(a, b):
    return np.abs(a - b).sum() / max(np.abs(b).sum(), 1e-300)


def _pair(p, **kw):
    g = Solver(p["nx"], p["ny"], p["gammas"], p["domain"], pinfs=p["pinfs"], **kw)
    r = RefSolver(p["nx"], p["ny"], p["gammas"], p["domain"], pinfs=p["pinfs"], omp=True, **kw)
    for s in (g, r):
        s.set_state(0.0, p["k"], p["rho"], p["e"], p["ux"], p["uy"])
    return g, r


def _compare(g, r, tag):
    fg = g.fields("rho", "p", "vol", "mass", "ie", "ux", "uy")
    fr = r.fields("rho", "p", "vol", "mass", "ie", "ux", "uy")
    l1r, l1p = rel_l1(fg["rho"], fr["rho"]), rel_l1(fg["p"], fr["p"])
    worst = 0.0
    for key in ("vol", "mass", "ie"):
        cell = np.maximum(np.abs(fr[key]).sum(0), 1e-300)
        worst = max(worst, float((np.abs(fg[key] - fr[key]) / cell).max()))
    us = max(np.abs(fr["ux"]).max(), np.abs(fr["uy"]).max(), 1e-300)
    uerr = max(np.abs(fg["ux"] - fr["ux"]).max(), np.abs(fg["uy"] - fr["uy"]).max()) / us
    say(f"{tag}: L1 rho {l1r:.2e} p {l1p:.2e} cell {worst:.2e} u {uerr:.2e}")
    assert l1r <= 1e-10 and l1p <= 1e-10 and worst <= 1e-9 and uerr <= 1e-9, tag


def test_water_air_tube_to_t_end():
    """The water-air tube (water at 1e9 Pa against air) from rest to
    t_end = 1.2e-4 s: same step count and time, fields within 1e-10."""
    p = inputs.water_air_tube(400, 4)
    say("water-air tube 400x4 FP64 to t_end")
    g, r = _pair(p)
    ng, tg = g.run(p["t_end"])
    nr, tr = r.run(p["t_end"])
    assert ng == nr and tg == tr == p["t_end"], (ng, nr, tg, tr)
    _compare(g, r, f"water-air tube after {ng} steps")


def test_water_impact_steps():
    """The water-drop impact on the paper's 320x160 mesh (air at 1 km/s with
    the drop against a water wall at rest): 150 steps, fields within 1e-10,
    with mixed air-water cells at the drop's rim."""
    p = inputs.water_impact(1)
    say("water impact 320x160 FP64, 150 steps")
    g, r = _pair(p)
    g.run(1.0, max_steps=150)
    r.run(1.0, max_steps=150)
    assert r.counts()["mixed"] > 0
    _compare(g, r, "water impact after 150 steps")


def test_water_impact_in_batch_equals_alone():
    """A stiffened-gas problem in a batch gives the bits it gives alone."""
    from paper_2208_13409_amd.lr import LR_FP64, Batch
    p = inputs.water_impact(1)
    say("water impact in a batch of 2, FP64, 32 steps")
    g = Solver(p["nx"], p["ny"], p["gammas"], p["domain"], pinfs=p["pinfs"])
    g.set_state(0.0, p["k"], p["rho"], p["e"], p["ux"], p["uy"])
    g.run(1.0, max_steps=32)
    b = Batch(nmat=2, precision=LR_FP64, max_slots=4, pool_bytes=1 << 30, chunk_steps=16)
    other = inputs.random_mixed(7, 90, 70, nmat=2)
    ids = [b.submit(p, 1.0, max_steps=32), b.submit(other, 1.0, max_steps=32)]
    assert None not in ids
    while b.step() > 0:
        pass
    fb = b.fields(ids[0], "vol", "mass", "ie", "ux", "uy")
    fg = g.fields("vol", "mass", "ie", "ux", "uy")
    for key in fg:
        assert np.array_equal(fb[key], fg[key]), key
