"""The alternate-direction (AD) remap, the paper's comparator (§2.1.1,
§2.1.2, §4.2), on the GPU against the oracle's AD remap, whose pins are the
§3.1 corner-transport formula, the §3.2 single-node volume 1 + eps + eps^2/4,
equality with DirectCF for one-dimensional flow, conservation, bounds and the
second-order symmetry of the alternation (tests/test_oracle_pins.py)."""
import sys

import numpy as np
import pytest

from oracle import RefSolver
from paper_2208_13409_amd import inputs
from paper_2208_13409_amd.lr import LR_FP32, LR_REMAP_AD, LR_REMAP_DIRECTCF, Solver

pytestmark = pytest.mark.gpu
AD = LR_REMAP_AD


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_l1(a, b):
    return np.abs(a - b).sum() / max(np.abs(b).sum(), 1e-300)


def _pair(p, **kw):
    g = Solver(p["nx"], p["ny"], p["gammas"], p["domain"], remap=AD, **kw)
    kw.pop("precision", None)
    r = RefSolver(p["nx"], p["ny"], p["gammas"], p["domain"], remap=AD, omp=True, **kw)
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


def _check(g, r, tag, tol=1e-10, cell_tol=1e-9):
    l1r, l1p, worst, uerr = _errors(g, r)
    say(f"{tag}: L1 rho {l1r:.2e} p {l1p:.2e} cell {worst:.2e} u {uerr:.2e}")
    assert l1r <= tol and l1p <= tol and worst <= cell_tol and uerr <= cell_tol, tag


@pytest.mark.parametrize("nx,ny,nmat,seed,steps", [(90, 70, 2, 61, 21), (64, 48, 3, 62, 16),
                                                   (33, 9, 2, 63, 15), (40, 40, 4, 64, 10)])
def test_ad_random_mixed(nx, ny, nmat, seed, steps):
    """Random mixed states with interfaces, 2 to 4 materials, an odd and an
    even number of steps (both pass orders)."""
    p = inputs.random_mixed(seed, nx, ny, nmat=nmat)
    say(f"AD random mixed {nx}x{ny} nmat={nmat} seed={seed}, {steps} steps")
    g, r = _pair(p)
    g.run(1.0, max_steps=steps)
    r.run(1.0, max_steps=steps)
    assert r.counts()["mixed"] > 0
    _check(g, r, f"AD random {nx}x{ny}x{nmat}")


def test_ad_triple_point_steps():
    """The triple point 448x192, three materials, 100 steps of AD."""
    p = inputs.triple_point(1)
    say("AD triple point 448x192, 100 steps")
    g, r = _pair(p)
    ng, tg = g.run(p["t_end"], max_steps=100)
    nr, tr = r.run(p["t_end"], max_steps=100)
    assert ng == nr == 100 and tg == pytest.approx(tr, rel=1e-13)
    _check(g, r, "AD triple point")


@pytest.mark.parametrize("sx,sy", [(1, 1), (-1, -1), (1, -1), (-1, 1)])
def test_ad_corner_transport_formula(sx, sy):
    """§3.1 on the GPU: with a constant velocity and upwind values, each AD
    step (X-Y, then Y-X) is the bilinear corner-transport update."""
    nx, ny, ex, ey = 14, 12, 0.3, 0.2
    rng = np.random.default_rng(6)
    rho = rng.uniform(0.5, 2.0, size=(ny, nx))
    say(f"AD CTU {sx},{sy}")
    g = Solver(nx, ny, [1.4], (0.0, nx, 0.0, ny), recon_order=1, kinematic=True, fixed_dt=1.0, remap=AD)
    g.set_state(0.0, np.ones((1, ny, nx)), rho[None], np.ones((1, ny, nx)),
                np.full((ny + 1, nx + 1), sx * ex), np.full((ny + 1, nx + 1), sy * ey))

    def ctu(a):
        b = a.copy()
        for j in range(1, ny - 1):
            for i in range(1, nx - 1):
                b[j, i] = a[j, i] * (1 - ex) * (1 - ey) + a[j, i - sx] * ex * (1 - ey) + \
                    a[j - sy, i] * ey * (1 - ex) + a[j - sy, i - sx] * ex * ey
        return b

    want = rho
    for step in range(2):
        g.step()
        want = ctu(want)
        got = g.fields("mass")["mass"][0]
        lo = 2 + step
        np.testing.assert_allclose(got[lo:ny - lo, lo:nx - lo], want[lo:ny - lo, lo:nx - lo], rtol=1e-13)


def test_ad_square_advection_to_t_end():
    """§5.1 kinematic advection with AD, GPU against the oracle to the end:
    the two-material square advected at (5, 5) to t_end 0.02."""
    p = inputs.square_advection(80, nmat=2)
    say(f"AD advection {p['nx']}x{p['ny']} to t_end {p['t_end']}")
    g, r = _pair(p, kinematic=True)
    ng, tg = g.run(p["t_end"])
    nr, tr = r.run(p["t_end"])
    assert ng == nr and tg == tr == p["t_end"]
    _check(g, r, f"AD advection after {ng} steps")


@pytest.mark.parametrize("nmat", [1, 2])
def test_ad_solid_rotation_steps(nmat):
    """§5.1 kinematic solid rotation with AD, GPU against the oracle over 60
    steps (a tenth of a turn).  A prescribed field that is not divergence-
    free on the grid (here at the edge of the rotating disc, where the flow
    is cut off to stay tangent to the walls) makes the volume of a cell it
    keeps diverging drift from the cell area geometrically, since a pure
    cell's volume deviation is multiplied by Vol^{lag}/A every step (the same
    in the oracle); 60 steps keep that growth far from the rounding level."""
    p = inputs.solid_rotation(64, nmat=nmat)
    say(f"AD rotation {p['nx']}x{p['ny']} nmat={nmat}, 60 steps")
    g, r = _pair(p, kinematic=True)
    g.run(p["t_end"], max_steps=60)
    r.run(p["t_end"], max_steps=60)
    _check(g, r, f"AD rotation nmat={nmat}")


def test_directcf_keeps_the_diagonal_symmetry_ad_does_not():
    """§2.1.2 remark 3 and §5.1 on the GPU: for a problem symmetric about
    x = y, one DirectCF step stays symmetric to rounding and one AD step
    (X then Y) does not."""
    n = 40
    p = inputs.random_mixed(71, n, n, nmat=2)
    k = 0.5 * (p["k"] + p["k"].transpose(0, 2, 1))
    rho = 0.5 * (p["rho"] + p["rho"].transpose(0, 2, 1))
    e = 0.5 * (p["e"] + p["e"].transpose(0, 2, 1))
    rho = np.where(k > 0, np.where(rho > 0, rho, 1.0), 0.0)
    e = np.where(k > 0, np.where(e > 0, e, 1.0), 0.0)
    ux = 0.5 * (p["ux"] + p["uy"].T)
    uy = ux.T.copy()
    asym = {}
    for remap in (LR_REMAP_DIRECTCF, AD):
        g = Solver(n, n, p["gammas"], (0.0, 1.0, 0.0, 1.0), remap=remap)
        g.set_state(0.0, k, rho, e, ux, uy)
        g.step()
        m = g.fields("mass")["mass"]
        asym[remap] = float(np.abs(m - m.transpose(0, 2, 1)).max() / np.abs(m).max())
    say(f"asymmetry after one step: DirectCF {asym[LR_REMAP_DIRECTCF]:.2e}, AD {asym[AD]:.2e}")
    assert asym[LR_REMAP_DIRECTCF] <= 1e-13
    assert asym[AD] >= 1e-6


def test_ad_fp32_against_oracle():
    """The AD remap in FP32 (FP64 interface and clipping) within 1e-4 of the
    FP64 oracle over 20 steps of a two-material problem."""
    p = inputs.random_mixed(81, 96, 64, nmat=2)
    say("AD FP32 96x64, 20 steps")
    g, r = _pair(p, precision=LR_FP32, k_eps=1e-6)
    g.run(1.0, max_steps=20)
    r.run(1.0, max_steps=20)
    l1r, l1p, _, _ = _errors(g, r)
    say(f"AD FP32: L1 rho {l1r:.2e} p {l1p:.2e}")
    assert l1r <= 1e-4 and l1p <= 1e-4
