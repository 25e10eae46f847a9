#!/usr/bin/env python3
"""Throughput of the DirectCF multimaterial Lagrange–Remap step on one MI355X.

A step is one pass of the whole hot path (CFL time step, staggered
Lagrangian phase, DirectCF remap with VOF partial fluxes, momentum remap)
over the grid.  The headline workload is the three-material triple point,
448 x 192 cells, FP64, one problem per context ("FP64 plain"), synthetic
initial state (no dataset), timed in its developed state: the run first
reaches t = t_end / 2 = 1.75 (untimed), then takes the warm-up and the timed
steps.  The metric is cell-updates per second = cells x steps / wall time of
the timed steps, with the state resident in device memory.  The same JSON
line carries

  "from_rest": the same timing from t = 0 (most of the grid still at rest);
  "parity": relative L1 of density and pressure of the GPU against the FP64
      oracle after the oracle's sample steps from the same initial state;
  "fp32_batched": 256 seeded two-material shock-bubble problems (grids from
      64x64 to 512x256) stepped together in FP32, every launch covering the
      tiles of all problems, under the launch schedule the batch's autotuner
      picked, timed over a window that starts after every problem has run
      past half its end time; with the L1 of its smallest problem against
      the oracle (from the CPU-baseline leg), beside that of the oracle
      with its state stored in FP32 between steps;
  "triple_point_1792x768": the large triple point in FP64 and FP32 from its
      developed state (t = 1.75), and the L1 of FP32 against FP64 over the
      timed window from the same state;
  "ad_comparator_fp64": the paper's alternate-direction remap against the
      DirectCF remap, FP64, 100 steps from the same developed triple-point
      state, at 448x192 and 1792x768;
  "serving": a seeded Poisson stream of four-quadrant Riemann problems
      (grids 128^2..1024^2, FP32, t_end 0.25; 1000 requests at 50/s) served
      with continuous batching; p50/p99 latency from arrival to result fields
      on the host, overall and per quarter of the arrivals, with the served
      and the offered cell-updates/s;
  "roofline": the dominant kernel of the plain step: the step's algorithmic
      bytes per cell-update (the persistent state read and written once, 176 B
      for FP64 with three materials) times the cells one launch processes,
      over the kernel's average duration, measured with start/stop HIP events
      recorded by each launch's dispatch on the kernel's stream; "traffic" is
      the HBM bytes per launch that rocprofv3 counted for the same kernel
      sources (profiles/), else null; "valu" the kernel's VALU issue (its
      counted VALU instructions per launch over the same measured duration,
      against the published FP32/FP64 vector rates), else null;
  "cpu_baseline": the FP64 oracle timed on a bounded sample of the plain
      workload on the host's cores (OpenMP over grid rows), with the
      single-threaded figure, the core count and the CPU model beside it.
      This leg is the only one that runs the oracle: it also forms the
      other legs' L1 figures against it.
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
KERNEL_SOURCES = ("paper_2208_13409_amd/csrc/lr_step.hpp", "paper_2208_13409_amd/csrc/lr_device.hpp")


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


def batch_leg(n_problems, steps, chunk=8, prep_steps=200):
    """FP32 shock-bubble batch: `prep_steps` untimed steps, the autotuner's
    chunks among them (every problem past half its end time, 0.125, by then:
    the largest grid needs about 190 steps), then `steps` timed steps (all
    problems take the same number of steps).  Returns the leg's record and
    the smallest problem's fields, which the CPU-baseline leg compares with
    the FP64 oracle's after the same steps."""
    from paper_2208_13409_amd import inputs
    from paper_2208_13409_amd.lr import LR_FP32, LR_NSCHED, TILE_SHAPES, Batch
    probs = inputs.shock_bubble_batch(n_problems)
    steps = max(chunk, (steps // chunk) * chunk)
    prep_steps = (prep_steps // chunk) * chunk
    probe = Batch(nmat=2, precision=LR_FP32, max_slots=1, pool_bytes=1 << 20)
    pool = sum(probe.footprint(p["nx"], p["ny"]) for p in probs) + (64 << 20)
    probe.close()
    b = Batch(nmat=2, precision=LR_FP32, max_slots=len(probs), pool_bytes=pool, chunk_steps=chunk,
              autotune=True)
    # the autotuner times each schedule twice (forward, then in reverse); one
    # more chunk captures the chosen schedule's graph
    untimed = max(prep_steps, 2 * LR_NSCHED * chunk) + chunk
    ids = [b.submit(p, 1e30, max_steps=untimed + steps, k_eps=1e-6) for p in probs]
    assert all(i is not None for i in ids)
    for _ in range(untimed // chunk):
        b.step()
    persistent, graph, tile, rates = b.schedule()
    assert rates is not None, "the autotuner is still timing"
    t0 = time.perf_counter()
    chunks = 0
    while b.step() > 0:
        chunks += 1
    wall = time.perf_counter() - t0
    chunks += 1
    for rid in ids:
        rc, st, _ = b.status(rid)
        assert rc == 0 and st == untimed + steps, (rid, rc, st)
    small = min(range(len(probs)), key=lambda i: probs[i]["nx"] * probs[i]["ny"])
    ps = probs[small]
    check = {"problem": ps, "index": small, "steps": untimed + steps, "k_eps": 1e-6,
             "gpu": b.fields(ids[small], "rho", "p"), "fp32": True}
    cells = sum(p["nx"] * p["ny"] for p in probs)
    value = cells * steps / wall
    bpc = step_bytes(1, 1, 2, 4)
    b.close()
    return {"value": value, "unit": "cell-updates/s", "dtype": "f32",
            "workload": f"shock_bubble_batch_{len(probs)}", "problems": len(probs), "cells": cells,
            "steps": steps, "timed_from_step": untimed, "ms_per_step": wall * 1e3 / steps, "chunks": chunks,
            "launch": ("persistent grids" if persistent else "one block per tile of every problem")
                      + (f", one HIP graph per chunk of {chunk} steps" if graph else
                         f", chunks of {chunk} steps launched directly"),
            "tile": "%dx%d" % TILE_SHAPES[tile],
            "autotuner_cell_steps_per_ms": {
                "%dx%d%s%s" % (*TILE_SHAPES[c // 4], "+persistent" if c & 1 else "", "+graph" if c & 2 else ""):
                round(float(r_), 1) for c, r_ in enumerate(rates)},
            "hbm_bytes_per_cell_update": bpc, "achieved_GBs": value * bpc / 1e9,
            "frac_hbm": value * bpc / 1e9 / HBM_PEAK_GBS}, check


class FourQuadrantStream:
    """The serving workload's requests, built ahead of their admission by
    host threads (requests arrive built; the whole stream at once would take
    tens of GB of host memory).  Read in arrival order."""

    def __init__(self, n, ahead=48, workers=4):
        from concurrent.futures import ThreadPoolExecutor
        self.n, self.ahead = n, ahead
        self.pool = ThreadPoolExecutor(workers)
        self.futures = {}
        self.next = 0

    def _build(self, i):
        from paper_2208_13409_amd import inputs
        return inputs.four_quadrant(inputs.BASE_SEED + i)

    def __len__(self):
        return self.n

    def __getitem__(self, i):
        while self.next < min(self.n, i + self.ahead):
            self.futures[self.next] = self.pool.submit(self._build, self.next)
            self.next += 1
        return self.futures.pop(i).result()

    def warm(self, k):
        """start building, and wait for the first k"""
        while self.next < min(self.n, self.ahead):
            self.futures[self.next] = self.pool.submit(self._build, self.next)
            self.next += 1
        for i in range(min(k, self.n)):
            self.futures[i].result()

    def close(self):
        self.pool.shutdown(wait=False, cancel_futures=True)


def serve_leg(n_requests, rate, tile=None, max_slots=64, pool_gib=16):
    """The seeded Poisson stream of four-quadrant problems served with
    continuous batching: served and offered cell-updates/s (offered = the
    work of the stream over its arrival span), the share of wall time with a
    chunk in flight, p50/p99 latency overall and per quarter of the arrivals
    (a growing backlog shows as latencies growing from quarter to quarter)."""
    import numpy as np

    from paper_2208_13409_amd import inputs
    from paper_2208_13409_amd.lr import LR_FP32, LR_TILE_16x16, TILE_SHAPES, Batch
    from paper_2208_13409_amd.serve import percentile, serve
    # 16x16: the shape the batch autotuner keeps for FP32 two-material
    # launches (the stream's mix changes too often to time schedules on it)
    tile = LR_TILE_16x16 if tile is None else tile
    reqs = FourQuadrantStream(n_requests)
    reqs.warm(8)  # the first requests built before the clock starts
    arrivals = inputs.poisson_arrivals(n_requests, rate=rate)
    b = Batch(nmat=2, precision=LR_FP32, max_slots=max_slots, pool_bytes=pool_gib << 30, chunk_steps=8, tile=tile)
    out = serve(b, reqs, arrivals)
    b.close()
    reqs.close()
    # a failed request stops at its failing step: its steps count as served,
    # its latency is that of its error report
    failed = [{"request": i, "grid": int(round(c ** 0.5)), "rc": rc, "steps": st}
              for i, (rc, c, st) in enumerate(zip(out["rc"], out["cells"], out["steps"])) if rc != 0]
    work = np.array(out["cells"], dtype=float) * np.array(out["steps"], dtype=float)
    offered = float(work.sum() / arrivals[-1])
    lat = np.array(out["latency"])
    quarters = np.array_split(np.argsort(arrivals), 4)
    return {"p50_s": out["p50"], "p99_s": out["p99"], "requests": n_requests, "rate_per_s": rate,
            "cell_updates_per_s": out["cell_updates_per_s"], "offered_cell_updates_per_s": offered,
            "served_over_offered": out["cell_updates_per_s"] / offered, "wall_s": out["wall"],
            "arrival_span_s": float(arrivals[-1]), "gpu_busy": out["busy"], "max_running": out["max_running"],
            "latency_by_arrival_quarter": [{"p50_s": percentile(lat[q], 50), "p99_s": percentile(lat[q], 99)}
                                           for q in quarters],
            "failed_requests": failed, "tile": "%dx%d" % TILE_SHAPES[tile],
            "workload": f"four_quadrant stream, first {n_requests} requests of the seeded stream, FP32"}


def host_cpu():
    """CPU model name and logical CPUs of this host (lscpu, nproc)."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "nproc": len(os.sched_getaffinity(0))}


def cpu_baseline(p, steps):
    """The oracle on `steps` steps of the workload from t = 0, with OpenMP over
    grid rows on the host's cores and single-threaded; the fields it reaches
    are compared with the GPU's after the same steps from the same input."""
    import numpy as np

    from oracle import RefSolver
    from paper_2208_13409_amd.lr import Solver
    res = {}
    fields = None
    for omp in (True, False):
        r = RefSolver(p["nx"], p["ny"], p["gammas"], p["domain"], omp=omp)
        r.set_state(0.0, p["k"], p["rho"], p["e"], p["ux"], p["uy"])
        t0 = time.perf_counter()
        n, _ = r.run(p["t_end"], max_steps=steps)
        res[omp] = (p["nx"] * p["ny"] * n / (time.perf_counter() - t0), time.perf_counter() - t0, n)
        if fields is None:
            fields = r.fields("rho", "p")
    g = Solver(p["nx"], p["ny"], p["gammas"], p["domain"])
    g.set_state(0.0, p["k"], p["rho"], p["e"], p["ux"], p["uy"])
    ng, _ = g.run(p["t_end"], max_steps=steps)
    fg = g.fields("rho", "p")
    l1 = {k: float(np.abs(fg[k] - fields[k]).sum() / np.abs(fields[k]).sum()) for k in ("rho", "p")}
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    v, el, n = res[True]
    v1, el1, _ = res[False]
    host = host_cpu()
    return {"value": v, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{p['name']} FP64, the first {n} steps from t=0, OpenMP over rows on {threads} "
                      f"threads ({el:.1f} s); single thread {v1:.3g} cell-updates/s ({el1:.1f} s)",
            "single_thread": {"value": v1, "cores": 1, "seconds": el1},
            "host": host,
            "l1_vs_gpu": {"rho": l1["rho"], "p": l1["p"], "steps": n, "gpu_steps": ng}}


def oracle_check(chk):
    """Part of the CPU-baseline leg: the oracle on another leg's problem for
    the same steps, L1 of density and pressure of the GPU's fields against
    it; for an FP32 result also the oracle with its state stored in FP32
    between steps (oracle/fp32_state.py), the floor that single-precision
    storage sets through the presence-threshold branches."""
    import numpy as np

    from oracle import RefSolver
    from oracle.fp32_state import run_stored
    p, n = chk["problem"], chk["steps"]
    r = RefSolver(p["nx"], p["ny"], p["gammas"], p["domain"], k_eps=chk["k_eps"])
    r.set_state(0.0, p["k"], p["rho"], p["e"], p["ux"], p["uy"])
    r.run(1e30, max_steps=n)
    fr = r.fields("rho", "p")
    l1 = lambda a: {k: float(np.abs(a[k] - fr[k]).sum() / np.abs(fr[k]).sum()) for k in ("rho", "p")}
    out = {"problem": chk["index"], "grid": f"{p['nx']}x{p['ny']}", "steps": n, **l1(chk["gpu"])}
    if chk.get("fp32"):
        out["oracle_fp32_state_control"] = l1(run_stored(p, n, {n}, chk["k_eps"])[n])
    return out


def timed_window(g, stream, warmup, steps):
    """warm-up steps, then `steps` timed steps (wall clock and stream events)"""
    import torch
    t_far = 1e30  # the timed steps follow the CFL step and never land on an end time
    nw, _ = g.run(t_far, max_steps=warmup)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    t0 = time.perf_counter()
    n, _ = g.run(t_far, max_steps=steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    assert n == steps, f"only {n} of {steps} steps ran"
    return nw, n, wall, ev0.elapsed_time(ev1)


def large_leg(steps, warmup):
    """Triple point 1792x768 from its developed state: FP64 reaches t = 1.75;
    that state starts an FP64 and an FP32 solver, each timed over the same
    window; L1 of FP32 against FP64 after it."""
    import numpy as np
    import torch

    from paper_2208_13409_amd import inputs
    from paper_2208_13409_amd.lr import LR_FP32, Solver
    p = workload("triple_point_1792x768")
    nx, ny, nmat = p["nx"], p["ny"], len(p["gammas"])
    g = Solver(nx, ny, p["gammas"], p["domain"])
    g.set_state(0.0, p["k"], p["rho"], p["e"], p["ux"], p["uy"])
    t_dev = 0.5 * p["t_end"]
    n_prep, _ = g.run(t_dev)
    x0, x1, y0, y1 = p["domain"]
    st = inputs.restart_state(g.fields("vol", "mass", "ie", "ux", "uy"), (x1 - x0) / nx * (y1 - y0) / ny)
    g.close()
    out = {"workload": "triple_point_1792x768", "cells": nx * ny, "developed_from_step": n_prep,
           "t_start": t_dev}
    fields = {}
    for prec in ("fp64", "fp32"):
        stream = torch.cuda.Stream()
        h = Solver(nx, ny, p["gammas"], p["domain"], stream=stream,
                   precision=LR_FP32 if prec == "fp32" else 0, k_eps=1e-6 if prec == "fp32" else 1e-10)
        h.set_state(t_dev, *st)
        _, n, wall, _ = timed_window(h, stream, warmup, steps)
        w = 4 if prec == "fp32" else 8
        bpc = step_bytes(1, 1, nmat, w)
        v = nx * ny * n / wall
        out[prec] = {"value": v, "unit": "cell-updates/s", "steps": n, "ms_per_step": wall * 1e3 / n,
                     "bytes_per_cell_update": bpc, "frac_hbm_cache_resident": v * bpc / 1e9 / HBM_PEAK_GBS}
        fields[prec] = h.fields("rho", "p")
        h.close()
    out["fp32_l1_vs_fp64"] = {k: float(np.abs(fields["fp32"][k] - fields["fp64"][k]).sum()
                                       / np.abs(fields["fp64"][k]).sum()) for k in ("rho", "p")}
    return out


def ad_leg(steps, warmup):
    """The paper's comparator: the alternate-direction remap (an X and a Y
    pass per step, nine kernel launches) against the one-step DirectCF remap
    (four launches), FP64, each timed from the same developed state of the
    triple point (t = 1.75) at 448x192 and 1792x768."""
    import torch

    from paper_2208_13409_amd import inputs
    from paper_2208_13409_amd.lr import LR_REMAP_AD, LR_REMAP_DIRECTCF, LR_TILE_32x8, Solver
    out = {}
    for scale in (1, 4):
        p = inputs.triple_point(scale)
        nx, ny = p["nx"], p["ny"]
        g = Solver(nx, ny, p["gammas"], p["domain"])
        g.set_state(0.0, p["k"], p["rho"], p["e"], p["ux"], p["uy"])
        t_dev = 0.5 * p["t_end"]
        g.run(t_dev)
        x0, x1, y0, y1 = p["domain"]
        st = inputs.restart_state(g.fields("vol", "mass", "ie", "ux", "uy"), (x1 - x0) / nx * (y1 - y0) / ny)
        g.close()
        rec = {}
        for name, remap in (("directcf", LR_REMAP_DIRECTCF), ("ad", LR_REMAP_AD)):
            stream = torch.cuda.Stream()
            # both on the 32x8 tiles (the shape the alternate-direction
            # remap runs on), so that the two differ in the remap only
            h = Solver(nx, ny, p["gammas"], p["domain"], stream=stream, remap=remap, tile=LR_TILE_32x8)
            h.set_state(t_dev, *st)
            _, n, wall, _ = timed_window(h, stream, warmup, steps)
            rec[name] = {"us_per_step": wall * 1e6 / n, "value": nx * ny * n / wall}
            h.close()
        rec["directcf_speedup"] = rec["ad"]["us_per_step"] / rec["directcf"]["us_per_step"]
        out[f"triple_point_{nx}x{ny}"] = rec
    out["launches_per_step"] = {"directcf": 4, "ad": 9}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="triple_point_448x192")
    ap.add_argument("--develop", type=float, default=0.5,
                    help="fraction of t_end reached (untimed) before the timed window")
    ap.add_argument("--profile-steps", type=int, default=64,
                    help="steps run again with per-kernel HIP event pairs")
    ap.add_argument("--cpu-steps", type=int, default=150)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--batch-problems", type=int, default=256)
    ap.add_argument("--batch-steps", type=int, default=200)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--large-steps", type=int, default=100)
    ap.add_argument("--no-large", action="store_true")
    ap.add_argument("--no-ad", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=1000)
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
    from paper_2208_13409_amd.lr import TILE_SHAPES, Solver

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

    # from rest: most of the grid at rest, which the kernels skip
    g.set_state(0.0, p["k"], p["rho"], p["e"], p["ux"], p["uy"])
    nw0, n0, wall0, _ = timed_window(g, stream, args.warmup, args.steps)
    from_rest = {"value": cells * n0 / wall0, "steps": n0, "warmup": nw0, "ms_per_step": wall0 * 1e3 / n0,
                 "t_start": 0.0}

    # developed state: t = t_end / 2 reached untimed from rest
    t_dev = args.develop * p["t_end"]
    g.set_state(0.0, p["k"], p["rho"], p["e"], p["ux"], p["uy"])
    n_prep, t_prep = g.run(t_dev)
    nw, n, wall, gpu_ms = timed_window(g, stream, args.warmup, args.steps)

    # the same kind of steps again, with an event pair around every launch
    g.profile(True)
    g.run(1e30, max_steps=args.profile_steps)
    prof = g.profile_read()
    g.profile(False)
    kb = kernel_bytes(nx, ny, nmat, w)
    avg_us = {k: (ms / cnt * 1e3 if cnt else 0.0) for k, (ms, cnt) in prof.items()}
    dom = max(prof, key=lambda k: prof[k][0])
    dom_s = avg_us[dom] * 1e-6
    # the scope table's per-cell-update bytes times the cells of one launch
    alg = step_bytes(nx, ny, nmat, w)
    achieved = alg / dom_s / 1e9
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
                   "t_start": t_prep, "developed_from_step": n_prep, "cfl": 0.5,
                   "tile": "%dx%d" % TILE_SHAPES[int(g.stage("run")[3])]},
        "gpu_event_ms_per_step": gpu_ms / n,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": counted_traffic(dom, p["name"], args.precision),
                     "algorithmic_bytes_per_launch": alg,
                     "bytes_per_cell_update": step_bytes(1, 1, nmat, w),
                     "kernel_array_bytes_per_launch": kb[dom], "avg_launch_us": avg_us[dom],
                     "valu": valu_roofline(counted_valu(dom, p["name"], args.precision), dom_s, fp32)},
        "roofline_step": {"bytes_per_cell_update": step_bytes(1, 1, nmat, w),
                          "achieved_GBs": alg / (wall / n) / 1e9,
                          "frac": alg / (wall / n) / 1e9 / HBM_PEAK_GBS,
                          "sum_kernel_us": step_us},
        "kernels_avg_us": avg_us,
        "from_rest": from_rest,
    }
    checks = {}
    if not args.no_batch:
        out["fp32_batched"], checks["fp32_batched"] = batch_leg(args.batch_problems, args.batch_steps)
        out["fp32_batched"]["vs_fp64_plain"] = out["fp32_batched"]["value"] / value
    if not args.no_large:
        out["triple_point_1792x768"] = large_leg(args.large_steps, 10)
    if not args.no_ad:
        out["ad_comparator_fp64"] = ad_leg(100, 10)
    if not args.no_serve:
        out["serving"] = serve_leg(args.serve_requests, args.serve_rate)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, args.cpu_steps)
        out["parity"] = {"vs": "FP64 oracle", "l1_rho": out["cpu_baseline"]["l1_vs_gpu"]["rho"],
                         "l1_p": out["cpu_baseline"]["l1_vs_gpu"]["p"],
                         "steps": out["cpu_baseline"]["l1_vs_gpu"]["steps"], "t_start": 0.0}
        for key, chk in checks.items():
            out[key]["l1_vs_oracle"] = oracle_check(chk)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
