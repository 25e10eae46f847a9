"""The allocation-free entry point lr_run_noalloc against the allocating
path (lr_create, lr_set_state, lr_run, lr_get_fields) on the same inputs:
the same kernels on the same values, so the fields must agree bit for bit.
Two calls in a row, the second on a smaller problem (the workspace keeps the
first call's contents), in FP64 and FP32, then a problem too large for the
workspace, which must be refused."""
import numpy as np
import pytest

from paper_2208_13409_amd import inputs
from paper_2208_13409_amd.lr import LR_ENOMEM, LR_FP32, LR_FP64, LRError, Solver, run_noalloc

pytestmark = pytest.mark.gpu

NAMES = ("rho", "p", "k", "ux", "uy", "vol", "mass", "ie")


def _shape(name, p):
    nm, nx, ny = len(p["gammas"]), p["nx"], p["ny"]
    if name in ("k", "vol", "mass", "ie"):
        return (nm, ny, nx)
    if name in ("ux", "uy"):
        return (ny + 1, nx + 1)
    return (ny, nx)


def _both(p, steps, precision):
    import torch
    dev = torch.device("cuda:0")
    k_eps = 1e-6 if precision == LR_FP32 else 1e-10
    g = Solver(p["nx"], p["ny"], p["gammas"], p["domain"], precision=precision, k_eps=k_eps)
    g.set_state(0.0, p["k"], p["rho"], p["e"], p["ux"], p["uy"])
    n_a, t_a = g.run(10.0, max_steps=steps)
    ref = g.fields(*NAMES)
    ins = [torch.from_numpy(np.ascontiguousarray(p[n], dtype=np.float64)).to(dev)
           for n in ("k", "rho", "e", "ux", "uy")]
    outs = {n: torch.full(_shape(n, p), np.nan, dtype=torch.float64, device=dev) for n in NAMES}
    n_b, t_b = run_noalloc(p["nx"], p["ny"], p["gammas"], p["domain"], 10.0, *ins, NAMES, outs,
                           max_steps=steps, precision=precision, k_eps=k_eps)
    torch.cuda.synchronize()
    assert (n_a, t_a) == (n_b, t_b)
    for n in NAMES:
        got = outs[n].cpu().numpy()
        assert np.array_equal(got, ref[n]), (n, np.nanmax(np.abs(got - ref[n])))


@pytest.mark.parametrize("precision", [LR_FP64, LR_FP32])
def test_noalloc_matches_allocating_path(precision):
    big = inputs.random_mixed(301, 150, 110, nmat=3)
    small = inputs.random_mixed(302, 70, 45, nmat=2)
    print(f"noalloc precision={precision}: 150x110 3 materials, 40 steps", flush=True)
    _both(big, 40, precision)
    print(f"noalloc precision={precision}: 70x45 2 materials, 25 steps", flush=True)
    _both(small, 25, precision)


def test_noalloc_refuses_a_problem_beyond_the_workspace():
    import torch
    dev = torch.device("cuda:0")
    nx, ny, nm = 1024, 512, 3
    z = torch.zeros((nm, ny, nx), dtype=torch.float64, device=dev)
    u = torch.zeros((ny + 1, nx + 1), dtype=torch.float64, device=dev)
    with pytest.raises(LRError) as ex:
        run_noalloc(nx, ny, [1.4] * nm, (0.0, 2.0, 0.0, 1.0), 1.0, z, z, z, u, u, (), {})
    assert ex.value.code == LR_ENOMEM and "workspace" in str(ex.value)
