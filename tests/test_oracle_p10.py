"""The oracle against a second, independent reader of the step in 50-digit
arithmetic (tests/p10_mini_oracle.py), on grids of at most 6 x 6 cells over
1 to 3 steps: every conserved cell value within 1e-13 of its cell's total,
nodal velocities within 1e-13 of the largest speed.  The cases make the
oracle take its rare branches (three-material cells, clipping, degenerate
normals, the positivity guard, order 1, a stiffened gas), and the test
checks from the oracle's branch counters that they did."""
import numpy as np
import pytest

from oracle import RefSolver
from paper_2208_13409_amd import inputs

from .p10_mini_oracle import MiniStep

TOL = 1e-13


def _to_np(arr):
    return np.array([[[float(v) for v in row] for row in mat] for mat in arr])


def _compare(p, steps, **kw):
    r = RefSolver(p["nx"], p["ny"], p["gammas"], p["domain"], pinfs=p.get("pinfs"), **kw)
    r.set_state(0.0, p["k"], p["rho"], p["e"], p["ux"], p["uy"])
    m = MiniStep(p["nx"], p["ny"], p["gammas"], p["domain"], pinfs=p.get("pinfs"), **kw)
    m.set_state(p["k"], p["rho"], p["e"], p["ux"], p["uy"])
    for _ in range(steps):
        dr = r.step()
        dm = m.step()
        assert abs(dr - float(dm)) <= 1e-14 * dr
        f = r.fields("vol", "mass", "ie", "ux", "uy")
        for key, arr in (("vol", m.V), ("mass", m.M), ("ie", m.E)):
            a = _to_np(arr)
            cell = np.maximum(np.abs(a).sum(0), 1e-300)
            err = float((np.abs(f[key] - a) / cell).max())
            assert err <= TOL, (key, err)
        ux = np.array([[float(v) for v in row] for row in m.ux])
        uy = np.array([[float(v) for v in row] for row in m.uy])
        us = max(np.abs(ux).max(), np.abs(uy).max(), 1e-300)
        err = max(np.abs(f["ux"] - ux).max(), np.abs(f["uy"] - uy).max()) / us
        assert err <= TOL, ("u", err)
    return r.counts()


@pytest.mark.parametrize("nx,ny,nmat,seed,steps", [(6, 6, 2, 1, 3), (6, 5, 3, 2, 2), (4, 6, 3, 5, 3)])
def test_random_mixed_states(nx, ny, nmat, seed, steps):
    """random discs of two or three materials, smooth random fields: the
    interface, clipping and (with three materials) the per-material lines"""
    c = _compare(inputs.random_mixed(seed, nx, ny, nmat=nmat), steps)
    assert c["mixed"] > 0
    if nmat == 3:
        assert c["three_or_more"] > 0


def test_clipping_case():
    """a case whose donors send more of a material than they hold: clipping"""
    c = _compare(inputs.random_mixed(1, 6, 6, nmat=2), 3)
    assert c["clipped"] > 0


def test_first_order():
    c = _compare(inputs.random_mixed(3, 5, 6, nmat=2), 2, recon_order=1)
    assert c["mixed"] > 0


def test_degenerate_normals():
    """a uniform 30/70 mixture with a pressure pulse: every cell mixed with a
    Youngs gradient zero up to rounding, split in proportion (the pulse is
    20%: a weaker one leaves velocities that are differences of nearly equal
    pressures, whose rounding alone exceeds the bound)"""
    nx, ny = 6, 4
    g = (1.4, 3.0)
    x = (np.arange(nx) + 0.5) / nx
    pr = 1.0 + 0.2 * np.exp(-((x - 0.5) / 0.2) ** 2)
    k = np.stack([np.full((ny, nx), 0.3), np.full((ny, nx), 0.7)])
    rho = np.stack([np.ones((ny, nx)), 2.0 * np.ones((ny, nx))])
    e = np.stack([pr / ((g[a] - 1) * rho[a]) * np.ones((ny, 1)) for a in (0, 1)])
    z = np.zeros((ny + 1, nx + 1))
    p = dict(nx=nx, ny=ny, gammas=list(g), domain=(0.0, 1.0, 0.0, ny / nx), k=k, rho=rho, e=e, ux=z, uy=z)
    c = _compare(p, 2)
    assert c["degenerate_normal"] > 0


def test_positivity_guard():
    """a diagonal flow at Courant 0.49 through a density growing 55-fold per
    cell: order-2 outflows exceed the donor's mass and the guard fires"""
    n, lam, d = 6, 4.0, 0.49
    xc = np.arange(n) + 0.5
    X, Y = np.meshgrid(xc, xc)
    rho = np.exp(lam * (X + Y) - 20.0)[None]
    u = np.full((n + 1, n + 1), d)
    p = dict(nx=n, ny=n, gammas=[1.4], domain=(0.0, n, 0.0, n), k=np.ones((1, n, n)), rho=rho,
             e=np.ones((1, n, n)), ux=u, uy=u)
    c = _compare(p, 2, kinematic=True, fixed_dt=1.0)
    assert c["guard"] > 0


def test_stiffened_gas():
    """water (stiffened gas) next to air at rest with a pressure jump"""
    nx, ny = 6, 4
    x = (np.arange(nx) + 0.5) / nx
    left = (x < 0.5) * np.ones((ny, 1))
    k = np.stack([left, 1.0 - left])
    rho = np.stack([1000.0 * left, 50.0 * (1.0 - left)])
    e = np.stack([left * (1e9 + 2.1e9) / (6.0 * 1000.0), (1.0 - left) * 1e5 / (0.4 * 50.0)])
    z = np.zeros((ny + 1, nx + 1))
    p = dict(nx=nx, ny=ny, gammas=[7.0, 1.4], pinfs=[2.1e9, 0.0], domain=(0.0, 1.0, 0.0, ny / nx),
             k=k, rho=rho, e=e, ux=z, uy=z)
    _compare(p, 3)
