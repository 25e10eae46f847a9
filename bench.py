#!/usr/bin/env python3
"""Throughput of the DirectCF multimaterial Lagrange–Remap step on one MI355X.

A step is one pass of the whole hot path (CFL time step, staggered
Lagrangian phase, DirectCF remap with VOF partial fluxes, momentum remap)
over the grid.  The headline workload is the three-material triple point,
448 x 192 cells, FP64, one problem per context ("FP64 plain"), synthetic
initial state (no dataset); the metric is cell-updates per second = cells x
steps / wall time of the timed steps, with the state resident in device
memory.  The same JSON line carries

  "fp32_batched": 256 seeded two-material shock-bubble problems (grids from
      64x64 to 512x256) stepped together in FP32, every launch covering the
      tiles of all problems, under the launch schedule the batch's autotuner
      picked on the first chunks (persistent grid or not, graph replay or
      not), over a fixed window of steps;
  "serving": a seeded Poisson stream of four-quadrant Riemann problems
      (grids 128^2..1024^2, FP32, t_end 0.25) served with continuous
      batching; p50/p99 latency from arrival to result fields on the host;
  "roofline": the dominant kernel of the plain step, its algorithmic bytes
      per launch over its average duration, measured with start/stop HIP
      events recorded by each launch's dispatch on the kernel's stream;
      "traffic" is the HBM bytes per launch that rocprofv3 counted for the
      same kernel sources (profiles/), else null; "valu" the kernel's VALU
      issue (its counted VALU instructions per launch over the same measured
      duration, against the published FP32/FP64 vector rates), else null;
  "cpu_baseline": the FP64 oracle timed on a bounded sample of the plain
      workload on the host (one thread).
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
W64 = 8
KERNEL_SOURCES = ("paper_2208_13409_amd/csrc/lr_kernels.hip", "paper_2208_13409_amd/csrc/lr_device.hpp")


def kernel_sources_sha256():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def counted_traffic(kernel, workload, precision):
    """HBM bytes per launch of `kernel` from the rocprofv3 FETCH_SIZE and
    WRITE_SIZE passes recorded in profiles/<kernel>_<workload>_<precision>.md
    (each scaled by what the counter reads for a device copy of known size),
    or None when there is no record or the kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_{precision}.md")
    if not os.path.exists(path):
        return None
    m = re.search(r"```json\n(.*?)\n```", open(path).read(), re.S)
    if not m:
        return None
    rec = json.loads(m.group(1))
    if rec.get("kernel_sources_sha256") != kernel_sources_sha256():
        return None
    return rec.get("traffic_bytes_per_launch")


def counted_valu(kernel, workload, precision):
    """Wave64 VALU instructions per launch of `kernel` from the rocprofv3
    SQ_INSTS_VALU pass recorded beside the traffic, or None (no record, or
    the kernel sources changed since)."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_{precision}.md")
    if not os.path.exists(path):
        return None
    m = re.search(r"```json\n(.*?)\n```", open(path).read(), re.S)
    if not m:
        return None
    rec = json.loads(m.group(1))
    if rec.get("kernel_sources_sha256") != kernel_sources_sha256():
        return None
    return rec.get("valu_instr_per_launch")


def valu_roofline(instr, seconds, fp32):
    """VALU issue of a launch against the published vector rates: one wave64
    instruction per SIMD every 2 cycles in FP32 (157.3 TFLOP/s = 256 CUs x
    128 lanes x 2 x 2.4 GHz), every 4 in FP64 (78.6 TFLOP/s); 1024 SIMDs."""
    if instr is None:
        return None
    peak = 1024 * 64 * 2.4e9 / (2 if fp32 else 4) / 1e12
    achieved = instr * 64 / seconds / 1e12
    return {"achieved": achieved, "peak": peak, "unit": "T lane-instr/s", "frac": achieved / peak,
            "instr_per_launch": instr}


def kernel_bytes(nx, ny, nmat, w=W64):
    """Algorithmic bytes per launch of each kernel: every array the kernel has
    to read or write, touched once (C cells, N nodes; the per-cell int of the
    mixed-cell index is 4 bytes); the interface work of the mixed cells
    touches only those cells and is not counted."""
    C = nx * ny
    N = (nx + 1) * (ny + 1)
    return {
        # reads V, M, E and u; writes u^{n+1/2}, u^{lag}, m_p, e^{lag}
        "k_lagrange": w * (3 * nmat * C + 2 * N + 5 * N + nmat * C),
        # reads V (classification); writes the mixed-cell index
        "k_mixed": w * nmat * C + 4 * C,
        # reads u^{n+1/2}, V, M, e^{lag}, mixed index; writes V, M, E, sound
        # speed and the three region mass fluxes
        "k_remap": w * (2 * N + 3 * nmat * C + 3 * nmat * C + 4 * C) + 4 * C,
        # reads u^{lag}, u^{n+1/2}, m_p, the region mass fluxes, sound speed;
        # writes u
        "k_dual": w * (7 * N + 4 * C),
    }


def step_bytes(nx, ny, nmat, w=W64):
    """The per-cell-update figure of the whole step: the persistent state
    (V, M, E per material and the nodal velocity) read and written once."""
    return 2 * (3 * nmat + 2) * w * nx * ny


def workload(name):
    from paper_2208_13409_amd import inputs
    if name == "triple_point_448x192":
        return inputs.triple_point(1)
    if name == "triple_point_1792x768":
        return inputs.triple_point(4)
    if name == "sod_400x4":
        return inputs.sod(400, 4)
    raise SystemExit(f"unknown workload {name}")


def batch_leg(n_problems, steps, chunk=8):
    """FP32 shock-bubble batch: every problem runs one warm-up chunk, then
    `steps` timed steps (all problems take the same number of steps)."""
    from paper_2208_13409_amd import inputs
    from paper_2208_13409_amd.lr import LR_FP32, Batch
    probs = inputs.shock_bubble_batch(n_problems)
    steps = max(chunk, (steps // chunk) * chunk)
    probe = Batch(nmat=2, precision=LR_FP32, max_slots=1, pool_bytes=1 << 20)
    pool = sum(probe.footprint(p["nx"], p["ny"]) for p in probs) + (64 << 20)
    probe.close()
    b = Batch(nmat=2, precision=LR_FP32, max_slots=len(probs), pool_bytes=pool, chunk_steps=chunk,
              autotune=True)
    untimed = 5 * chunk  # four chunks timing the candidate schedules, one capturing the chosen one
    ids = [b.submit(p, 1e30, max_steps=untimed + steps, k_eps=1e-6) for p in probs]
    assert all(i is not None for i in ids)
    for _ in range(5):
        b.step()
    persistent, graph, rates = b.schedule()
    t0 = time.perf_counter()
    chunks = 0
    while b.step() > 0:
        chunks += 1
    wall = time.perf_counter() - t0
    chunks += 1
    for rid in ids:
        rc, st, _ = b.status(rid)
        assert rc == 0 and st == untimed + steps, (rid, rc, st)
    cells = sum(p["nx"] * p["ny"] for p in probs)
    value = cells * steps / wall
    bpc = step_bytes(1, 1, 2, 4)
    b.close()
    return {"value": value, "unit": "cell-updates/s", "dtype": "f32",
            "workload": f"shock_bubble_batch_{len(probs)}", "problems": len(probs), "cells": cells,
            "steps": steps, "ms_per_step": wall * 1e3 / steps, "chunks": chunks,
            "launch": ("persistent grids" if persistent else "one block per tile of every problem")
                      + (f", one HIP graph per chunk of {chunk} steps" if graph else
                         f", chunks of {chunk} steps launched directly"),
            "autotuner_cell_steps_per_ms": [round(float(r), 1) for r in rates] if rates is not None else None,
            "hbm_bytes_per_cell_update": bpc, "achieved_GBs": value * bpc / 1e9,
            "frac_hbm": value * bpc / 1e9 / HBM_PEAK_GBS}


def serve_leg(n_requests, rate):
    from paper_2208_13409_amd import inputs
    from paper_2208_13409_amd.lr import LR_FP32, Batch
    from paper_2208_13409_amd.serve import serve
    reqs = [inputs.four_quadrant(inputs.BASE_SEED + i) for i in range(n_requests)]
    arrivals = inputs.poisson_arrivals(n_requests, rate=rate)
    b = Batch(nmat=2, precision=LR_FP32, max_slots=64, pool_bytes=16 << 30, chunk_steps=8)
    out = serve(b, reqs, arrivals)
    b.close()
    served = sum(c * s for c, s in zip(out["cells"], out["steps"]))
    assert all(rc == 0 for rc in out["rc"])
    return {"p50_s": out["p50"], "p99_s": out["p99"], "requests": n_requests, "rate_per_s": rate,
            "cell_updates_per_s": out["cell_updates_per_s"], "wall_s": out["wall"],
            "gpu_busy": out["busy"], "max_running": out["max_running"],
            "offered_cell_updates_per_s": served / float(arrivals[-1]),
            "workload": f"four_quadrant stream, first {n_requests} requests, FP32"}


def cpu_baseline(p, steps):
    from oracle import RefSolver
    r = RefSolver(p["nx"], p["ny"], p["gammas"], p["domain"])
    r.set_state(0.0, p["k"], p["rho"], p["e"], p["ux"], p["uy"])
    t0 = time.perf_counter()
    n, _ = r.run(p["t_end"], max_steps=steps)
    el = time.perf_counter() - t0
    return {"value": p["nx"] * p["ny"] * n / el, "unit": "cell-updates/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{p['name']} FP64, the first {n} steps from t=0, single thread "
                      f"({el:.1f} s)"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="triple_point_448x192")
    ap.add_argument("--profile-steps", type=int, default=64,
                    help="steps run again with per-kernel HIP event pairs")
    ap.add_argument("--cpu-steps", type=int, default=150)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--batch-problems", type=int, default=256)
    ap.add_argument("--batch-steps", type=int, default=200)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=40)
    ap.add_argument("--serve-rate", type=float, default=50.0)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 8 device-to-device copies of MIB MiB (the reference kernel "
                         "that scales the HBM byte counters) and exit")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only: the library has no multi-GPU path "
              f"(asked for --gpus {args.gpus}, WORLD_SIZE {world}).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2208_13409_amd.lr import Solver

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    torch.cuda.set_device(0)
    if args.copy_calibration:
        nb = args.copy_calibration << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(8):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_each_way": nb, "copies": 8}), flush=True)
        return
    p = workload(args.workload)
    nx, ny, nmat = p["nx"], p["ny"], len(p["gammas"])
    cells = nx * ny
    stream = torch.cuda.Stream()
    fp32 = args.precision == "fp32"
    w = 4 if fp32 else 8
    g = Solver(nx, ny, p["gammas"], p["domain"], stream=stream, precision=1 if fp32 else 0)
    g.set_state(0.0, p["k"], p["rho"], p["e"], p["ux"], p["uy"])
    t_end = 1e30  # the timed steps follow the CFL step and never land on t_end

    nw, _ = g.run(t_end, max_steps=args.warmup)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    t0 = time.perf_counter()
    n, t = g.run(t_end, max_steps=args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    assert n == args.steps, f"only {n} of {args.steps} steps ran"

    # the same kind of steps again, with an event pair around every launch
    g.profile(True)
    g.run(t_end, max_steps=args.profile_steps)
    prof = g.profile_read()
    g.profile(False)
    kb = kernel_bytes(nx, ny, nmat, w)
    avg_us = {k: (ms / cnt * 1e3 if cnt else 0.0) for k, (ms, cnt) in prof.items()}
    dom = max(prof, key=lambda k: prof[k][0])
    dom_s = avg_us[dom] * 1e-6
    achieved = kb[dom] / dom_s / 1e9
    step_us = sum(avg_us.values())
    value = cells * n / wall
    out = {
        "metric": "cell-updates/s per step (FP32 batched vs FP64 plain, 1 GPU); p50/p99 solve latency",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": n,
        "warmup": nw,
        "ms_per_step": wall * 1e3 / n,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if fp32 else "f64",
        "data": "synthetic",
        "config": {"workload": p["name"], "nx": nx, "ny": ny, "nmat": nmat, "precision": args.precision,
                   "t_start": 0.0, "cfl": 0.5},
        "gpu_event_ms_per_step": gpu_ms / n,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": counted_traffic(dom, p["name"], args.precision),
                     "algorithmic_bytes_per_launch": kb[dom], "avg_launch_us": avg_us[dom],
                     "valu": valu_roofline(counted_valu(dom, p["name"], args.precision), dom_s, fp32)},
        "roofline_step": {"bytes_per_cell_update": step_bytes(1, 1, nmat, w),
                          "achieved_GBs": step_bytes(nx, ny, nmat, w) / (wall / n) / 1e9,
                          "frac": step_bytes(nx, ny, nmat, w) / (wall / n) / 1e9 / HBM_PEAK_GBS,
                          "sum_kernel_us": step_us},
        "kernels_avg_us": avg_us,
    }
    if not args.no_batch:
        out["fp32_batched"] = batch_leg(args.batch_problems, args.batch_steps)
        out["fp32_batched"]["vs_fp64_plain"] = out["fp32_batched"]["value"] / value
    if not args.no_serve:
        out["serving"] = serve_leg(args.serve_requests, args.serve_rate)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
