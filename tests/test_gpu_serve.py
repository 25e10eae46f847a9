"""The serving loop on the GPU: requests that overlap on the device, some
waiting for memory (a pool smaller than the whole stream), each result the
same as the request run alone."""
import numpy as np
import pytest

from paper_2208_13409_amd import inputs
from paper_2208_13409_amd.lr import LR_FP32, Batch, Solver
from paper_2208_13409_amd.serve import serve

pytestmark = pytest.mark.gpu


def test_serve_results_equal_alone():
    sizes = [64, 96, 64, 128, 96, 64, 160, 64]
    reqs = []
    for s, n in enumerate(sizes):
        p = inputs.four_quadrant(2014 + s, n=n)
        p["t_end"] = 0.02
        reqs.append(p)
    arrivals = np.zeros(len(reqs))  # all at once: admission is limited by memory
    probe = Batch(nmat=2, precision=LR_FP32, max_slots=8, pool_bytes=1 << 20)
    pool = sum(probe.footprint(n, n) for n in (160, 128, 64)) + 4096  # not all eight at once
    probe.close()
    b = Batch(nmat=2, precision=LR_FP32, max_slots=8, pool_bytes=pool, chunk_steps=4)
    out = serve(b, reqs, arrivals, fields=("rho", "p", "ux"), keep=True)
    assert all(rc == 0 for rc in out["rc"])
    assert 1 < out["max_running"] < len(reqs)  # overlapped, and some had to wait
    assert out["p99"] >= out["p50"] > 0
    for i, p in enumerate(reqs):
        g = Solver(p["nx"], p["ny"], p["gammas"], p["domain"], precision=LR_FP32, k_eps=1e-6)
        g.set_state(0.0, p["k"], p["rho"], p["e"], p["ux"], p["uy"])
        n, t = g.run(p["t_end"])
        assert t == p["t_end"] and n == out["steps"][i]
        ref = g.fields("rho", "p", "ux")
        for key in ("rho", "p", "ux"):
            assert np.array_equal(out["results"][i][key], ref[key]), (i, key)
