"""The multidimensional least-squares reconstruction of §3.3 (recon_order 3)
on the GPU against the oracle, whose form of it is pinned by a closed form on
a translated linear field (tests/test_oracle_pins.py)."""
import sys

import numpy as np
import pytest

from oracle import RefSolver
from paper_2208_13409_amd import inputs
from paper_2208_13409_amd.lr import LR_FP32, Solver

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_l1(a, b):
    return np.abs(a - b).sum() / max(np.abs(b).sum(), 1e-300)


def _pair(p, **kw):
    g = Solver(p["nx"], p["ny"], p["gammas"], p["domain"], recon_order=3, **kw)
    kw.pop("precision", None)
    r = RefSolver(p["nx"], p["ny"], p["gammas"], p["domain"], recon_order=3, omp=True, **kw)
    for s in (g, r):
        s.set_state(0.0, p["k"], p["rho"], p["e"], p["ux"], p["uy"])
    return g, r


def _errors(g, r):
    fg = g.fields("rho", "p", "vol", "mass", "ie", "ux", "uy")
    fr = r.fields("rho", "p", "vol", "mass", "ie", "ux", "uy")
    worst = 0.0
    for key in ("vol", "mass", "ie"):
        cell = np.maximum(np.abs(fr[key]).sum(0), 1e-300)
        worst = max(worst, float((np.abs(fg[key] - fr[key]) / cell).max()))
    us = max(np.abs(fr["ux"]).max(), np.abs(fr["uy"]).max(), 1e-300)
    uerr = max(np.abs(fg["ux"] - fr["ux"]).max(), np.abs(fg["uy"] - fr["uy"]).max()) / us
    return rel_l1(fg["rho"], fr["rho"]), rel_l1(fg["p"], fr["p"]), worst, uerr


@pytest.mark.parametrize("nx,ny,nmat,seed,steps", [(90, 70, 2, 91, 20), (64, 48, 3, 92, 15),
                                                   (33, 9, 2, 93, 12)])
def test_lsq_random_mixed(nx, ny, nmat, seed, steps):
    p = inputs.random_mixed(seed, nx, ny, nmat=nmat)
    say(f"order 3 random mixed {nx}x{ny} nmat={nmat}, {steps} steps")
    g, r = _pair(p)
    g.run(1.0, max_steps=steps)
    r.run(1.0, max_steps=steps)
    l1r, l1p, worst, uerr = _errors(g, r)
    say(f"  L1 rho {l1r:.2e} p {l1p:.2e} cell {worst:.2e} u {uerr:.2e}")
    assert l1r <= 1e-10 and l1p <= 1e-10 and worst <= 1e-9 and uerr <= 1e-9


def test_lsq_triple_point_steps():
    p = inputs.triple_point(1)
    say("order 3 triple point 448x192, 60 steps")
    g, r = _pair(p)
    g.run(p["t_end"], max_steps=60)
    r.run(p["t_end"], max_steps=60)
    l1r, l1p, worst, uerr = _errors(g, r)
    say(f"  L1 rho {l1r:.2e} p {l1p:.2e} cell {worst:.2e} u {uerr:.2e}")
    assert l1r <= 1e-10 and l1p <= 1e-10 and worst <= 1e-8 and uerr <= 1e-8


@pytest.mark.parametrize("sx,sy", [(1, 1), (-1, 1)])
def test_lsq_closed_form_on_gpu(sx, sy):
    """The closed form of the oracle pin, on the GPU directly: a linear
    density translated by d on unit cells; every interior region carries its
    volume times a + g.x_D + phi g.(x_r - x_D - d), phi = min |g.e| / |g|."""
    n = 16
    a0, gr = 5.0, np.array([0.1, -0.07])
    d = np.array([sx * 0.3, sy * 0.2])
    xc = np.arange(n) + 0.5
    X, Y = np.meshgrid(xc, xc)
    say(f"order 3 closed form {sx},{sy}")
    g = Solver(n, n, [1.4], (0.0, n, 0.0, n), recon_order=3, kinematic=True, fixed_dt=1.0)
    g.set_state(0.0, np.ones((1, n, n)), (a0 + gr[0] * X + gr[1] * Y)[None], np.ones((1, n, n)),
                np.full((n + 1, n + 1), d[0]), np.full((n + 1, n + 1), d[1]))
    g.step()
    r2 = np.sqrt(2.0)
    phi = min(abs(gr[0]), abs(gr[1]), abs(gr.sum()) / r2, abs(gr[0] - gr[1]) / r2) / np.linalg.norm(gr)

    def value(donor, xr):
        xD = np.array(donor) + 0.5
        return a0 + gr @ xD + phi * (gr @ (xr - xD - d))

    muX, muY = g.stage("muX"), g.stage("muY")
    mu_c = g.stage("muD" if sx * sy > 0 else "muA")
    h = 1.0 - abs(d)
    for J in range(4, n - 4):
        for I in range(4, n - 4):
            D = (I - 1, J) if d[0] >= 0 else (I, J)
            xr = np.array([I + 0.5 * d[0], J + max(0.0, d[1]) + 0.5 * h[1]])
            assert muX[J, I] == pytest.approx(d[0] * h[1] * value(D, xr), rel=1e-13)
            D = (I, J - 1) if d[1] >= 0 else (I, J)
            xr = np.array([I + max(0.0, d[0]) + 0.5 * h[0], J + 0.5 * d[1]])
            assert muY[J, I] == pytest.approx(d[1] * h[0] * value(D, xr), rel=1e-13)
            D = (I - (d[0] >= 0), J - (d[1] >= 0))
            xr = np.array([I, J]) + 0.5 * d
            flux = abs(d[0] * d[1]) * value(D, xr)
            assert mu_c[J, I] == pytest.approx(flux if d[0] >= 0 else -flux, rel=1e-13)


def test_lsq_fp32_against_oracle():
    p = inputs.random_mixed(95, 96, 64, nmat=2)
    say("order 3 FP32 96x64, 20 steps")
    g, r = _pair(p, precision=LR_FP32, k_eps=1e-6)
    g.run(1.0, max_steps=20)
    r.run(1.0, max_steps=20)
    l1r, l1p, _, _ = _errors(g, r)
    say(f"  L1 rho {l1r:.2e} p {l1p:.2e}")
    assert l1r <= 1e-4 and l1p <= 1e-4
