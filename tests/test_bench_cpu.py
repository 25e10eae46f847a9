"""Host-side pieces of bench.py: algorithmic bytes, the VALU roofline, the
counter records under profiles/, and the single-GPU contract.  No GPU."""
import json
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_kernel_bytes_per_launch():
    """Each kernel's algorithmic bytes: the arrays it must touch once (w-byte
    words; C cells, N nodes; a 4-byte mixed-cell index per cell)."""
    nx, ny, nmat, w = 448, 192, 3, 8
    C, N = nx * ny, (nx + 1) * (ny + 1)
    kb = bench.kernel_bytes(nx, ny, nmat, w)
    assert kb["k_lagrange"] == w * (4 * nmat * C + 7 * N)
    assert kb["k_mixed"] == w * nmat * C + 4 * C
    assert kb["k_remap"] == w * (2 * N + 6 * nmat * C + 4 * C) + 4 * C
    assert kb["k_dual"] == w * (7 * N + 4 * C)
    # the whole step: the persistent state read and written once
    assert bench.step_bytes(1, 1, 3, 8) == 176 and bench.step_bytes(1, 1, 2, 4) == 64


def test_valu_roofline_against_the_published_rates():
    """FP64: one wave64 instruction per SIMD every 4 cycles, FP32 every 2, on
    1024 SIMDs at 2.4 GHz (78.6 and 157.3 TFLOP/s counted as FMA)."""
    fp64 = bench.valu_roofline(1024 * 2400, 4e-6, fp32=False)  # 2400 instr per SIMD in 4 us
    assert fp64["peak"] == pytest.approx(39.3216)
    assert fp64["frac"] == pytest.approx(2400 * 4 / (4e-6 * 2.4e9))
    fp32 = bench.valu_roofline(1024 * 2400, 4e-6, fp32=True)
    assert fp32["peak"] == pytest.approx(2 * 39.3216)
    assert fp32["frac"] == pytest.approx(fp64["frac"] / 2)
    assert bench.valu_roofline(None, 1e-6, fp32=False) is None


def test_counter_records_follow_the_kernel_sources():
    """The dominant kernel's record gives traffic and VALU counts only while
    it names the current kernel sources' hash."""
    path = os.path.join(ROOT, "profiles", "k_remap_triple_point_448x192_fp64.md")
    rec = json.loads(re.search(r"```json\n(.*?)\n```", open(path).read(), re.S).group(1))
    traffic = bench.counted_traffic("k_remap", "triple_point_448x192", "fp64")
    valu = bench.counted_valu("k_remap", "triple_point_448x192", "fp64")
    if rec["kernel_sources_sha256"] == bench.kernel_sources_sha256():
        assert traffic == rec["traffic_bytes_per_launch"] > rec["algorithmic_bytes_per_launch"] * 0.5
        assert valu == rec["valu_instr_per_launch"] > 0
    else:
        assert traffic is None and valu is None
    assert bench.counted_traffic("k_remap", "no_such_workload", "fp64") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in r.stderr
