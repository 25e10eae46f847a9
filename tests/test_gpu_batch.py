"""Batched and device-input paths on the GPU, through the C-ABI.

A problem stepped inside a batch runs the same kernels on its own data with
its own time step, so its fields must equal those of the same problem run
alone in a single context (compared exactly, with the FP64 oracle as a
second reference for one member).  Covers graph replay and plain launches,
persistent and one-block-per-tile grids, admission while others run,
LR_EAGAIN when the pool or the slots are full, release and reuse, and
problems that finish at different steps."""
import sys

import numpy as np
import pytest

from oracle import RefSolver
from paper_2208_13409_amd import inputs
from paper_2208_13409_amd.lr import (LR_EAGAIN, LR_FP32, LR_FP64, LR_NSCHED, LR_OK, LR_TILE_16x16,
                                     LR_TILE_32x8, LR_TILE_32x12, LR_TILE_AUTO,
                                     LR_TILE_32x16, TILE_SHAPES, Batch, LRError, Solver)

pytestmark = pytest.mark.gpu

FIELDS = ("vol", "mass", "ie", "ux", "uy")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def problems(nmat=2, seeds=(11, 12, 13, 14), sizes=((40, 24), (72, 40), (33, 65), (96, 17))):
    return [inputs.random_mixed(s, nx, ny, nmat=nmat) for s, (nx, ny) in zip(seeds, sizes)]


def alone(p, precision, steps=None, t_end=None, tile=LR_TILE_AUTO):
    g = Solver(p["nx"], p["ny"], p["gammas"], p["domain"], precision=precision,
               k_eps=1e-6 if precision == LR_FP32 else 1e-10, tile=tile)
    g.set_state(0.0, p["k"], p["rho"], p["e"], p["ux"], p["uy"])
    n, t = g.run(t_end if t_end is not None else 1e30, max_steps=steps if steps is not None else 1 << 40)
    return g, n, t


def drain(b):
    """step until nothing runs; ids in the order they finished"""
    done = []
    for _ in range(100000):
        left = b.step()
        done += b.poll()
        if left == 0:
            break
    return done + b.poll()


def same_fields(a, b, tag):
    for key in FIELDS:
        d = np.abs(a[key] - b[key]).max()
        assert d == 0.0, f"{tag} {key}: batch and alone differ by {d:.3e}"


@pytest.mark.parametrize("precision,use_graph,persistent", [
    (LR_FP64, True, True), (LR_FP64, False, False), (LR_FP32, True, True), (LR_FP32, False, True)])
def test_batch_equals_alone(precision, use_graph, persistent):
    ps = problems()
    steps = [10, 24, 7, 18]  # different lengths: problems leave the launches at different chunks
    say(f"batch equals alone: precision {precision} graph {use_graph} persistent {persistent}")
    b = Batch(nmat=2, precision=precision, max_slots=8, pool_bytes=64 << 20, chunk_steps=4,
              use_graph=use_graph, persistent=persistent)
    kw = dict(k_eps=1e-6) if precision == LR_FP32 else {}
    ids = [b.submit(p, 1e30, max_steps=n, **kw) for p, n in zip(ps, steps)]
    assert all(i is not None for i in ids)
    done = drain(b)
    assert sorted(done) == sorted(ids)
    for p, rid, n in zip(ps, ids, steps):
        rc, st, t = b.status(rid)
        assert rc == LR_OK and st == n, (rc, st)
        g, na, ta = alone(p, precision, steps=n)
        assert na == n and t == ta
        same_fields(b.fields(rid, *FIELDS), g.fields(*FIELDS), p["name"])
        np.testing.assert_array_equal(b.totals(rid), g.totals())


def test_batch_member_matches_oracle():
    p = inputs.random_mixed(21, 50, 30, nmat=3)
    b = Batch(nmat=3, precision=LR_FP64, max_slots=4, pool_bytes=64 << 20, chunk_steps=6)
    rid = b.submit(p, 1e30, max_steps=12)
    drain(b)
    r = RefSolver(p["nx"], p["ny"], p["gammas"], p["domain"])
    r.set_state(0.0, p["k"], p["rho"], p["e"], p["ux"], p["uy"])
    r.run(1e30, max_steps=12)
    fb, fr = b.fields(rid, "vol", "mass", "ie", "rho", "p"), r.fields("vol", "mass", "ie", "rho", "p")
    for key in ("vol", "mass", "ie"):
        scale = np.abs(fr[key]).max()
        assert np.abs(fb[key] - fr[key]).max() <= 1e-9 * scale, key
    for key in ("rho", "p"):
        assert np.abs(fb[key] - fr[key]).sum() / np.abs(fr[key]).sum() <= 1e-10, key


def test_batch_t_end_lands_exactly():
    p = inputs.sod(120, 4)
    b = Batch(nmat=2, precision=LR_FP64, max_slots=2, pool_bytes=16 << 20, chunk_steps=8)
    rid = b.submit(p, 0.05)
    drain(b)
    rc, st, t = b.status(rid)
    g, n, ta = alone(p, LR_FP64, t_end=0.05)
    assert rc == LR_OK and t == 0.05 and ta == 0.05 and st == n
    same_fields(b.fields(rid, *FIELDS), g.fields(*FIELDS), "sod")


def test_continuous_admission_and_release():
    """Problems join while others run and reuse released slots and ranges;
    each result equals the problem alone."""
    ps = problems(seeds=(31, 32, 33, 34, 35, 36),
                  sizes=((48, 32), (64, 64), (40, 40), (80, 24), (32, 96), (56, 56)))
    b = Batch(nmat=2, precision=LR_FP32, max_slots=3, pool_bytes=64 << 20, chunk_steps=4)
    steps = [12, 20, 8, 16, 12, 4]
    pending = list(range(len(ps)))
    ids = {}
    finished = []
    for _ in range(1000):
        while pending:
            k = pending[0]
            rid = b.submit(ps[k], 1e30, max_steps=steps[k], k_eps=1e-6)
            if rid is None:
                break  # three slots taken
            ids[rid] = k
            pending.pop(0)
        b.step()
        for rid in b.poll():
            k = ids[rid]
            g, n, _ = alone(ps[k], LR_FP32, steps=steps[k])
            same_fields(b.fields(rid, *FIELDS), g.fields(*FIELDS), f"request {k}")
            b.release(rid)
            finished.append(k)
        if not pending and b.running() == 0:
            break
    assert sorted(finished) == list(range(len(ps)))


def test_admission_while_a_chunk_is_in_flight():
    """lr_batch_step_begin / _end: requests submitted and released while a
    chunk runs join at the next chunk; each result equals the problem alone,
    and a second begin while one is in flight is refused."""
    ps = problems(seeds=(41, 42, 43, 44, 45), sizes=((48, 32), (64, 40), (40, 40), (72, 24), (32, 56)))
    b = Batch(nmat=2, precision=LR_FP64, max_slots=3, pool_bytes=64 << 20, chunk_steps=4)
    steps = [12, 8, 16, 4, 8]
    pending = list(range(len(ps)))
    ids = {}
    finished = []
    rid = b.submit(ps[0], 1e30, max_steps=steps[0])
    ids[rid] = 0
    pending.pop(0)
    for _ in range(1000):
        b.step_begin()
        with pytest.raises(LRError):
            b.step_begin()
        while pending:  # admitted while the chunk runs
            k = pending[0]
            rid = b.submit(ps[k], 1e30, max_steps=steps[k])
            if rid is None:
                break
            ids[rid] = k
            pending.pop(0)
        b.step_end()
        for rid in b.poll():
            k = ids[rid]
            g, n, _ = alone(ps[k], LR_FP64, steps=steps[k])
            rc, st, _ = b.status(rid)
            assert rc == LR_OK and st == steps[k], (k, rc, st)
            same_fields(b.fields(rid, *FIELDS), g.fields(*FIELDS), f"request {k}")
            b.release(rid)
            finished.append(k)
        if not pending and b.running() == 0:
            break
    assert sorted(finished) == list(range(len(ps)))
    assert b.step_end() == 0  # none in flight: only counts


def test_admissions_and_results_overlap_a_chunk():
    """With a long chunk in flight, three requests are admitted (the staging
    ring holds their inputs: no submit waits for the chunk) and a request
    that finished before it is copied back and released (on the output
    stream); all of that takes a fraction of the chunk's time, and every
    result equals the problem alone.  (The batch's first copy during a chunk
    pays one-time set-up costs of the runtime and is not timed.)"""
    import time
    big = inputs.random_mixed(71, 1024, 768, nmat=2)
    small = [inputs.random_mixed(72 + s, 40, 32, nmat=2) for s in range(5)]
    probe = Batch(nmat=2, precision=LR_FP64, max_slots=1, pool_bytes=1 << 20)
    pool = probe.footprint(1024, 768) + 5 * probe.footprint(40, 32) + (16 << 20)
    probe.close()
    b = Batch(nmat=2, precision=LR_FP64, max_slots=6, pool_bytes=pool, chunk_steps=16)
    firsts = [b.submit(p, 1e30, max_steps=4) for p in small[:2]]
    rb = b.submit(big, 1e30, max_steps=64)
    b.step()  # chunk 1: the two small requests finish in it
    drained = b.poll()
    assert sorted(drained) == sorted(firsts)
    b.step_begin()  # chunk 2: the first copy during a chunk
    f0 = b.fields(firsts[0], *FIELDS)
    b.release(firsts[0])
    b.step_end()
    say("admissions and a result copy while a 16-step chunk of 1024x768 FP64 runs")
    b.step_begin()  # chunk 3, timed
    t0 = time.perf_counter()
    ids = [b.submit(p, 1e30, max_steps=8) for p in small[2:]]
    t_sub = time.perf_counter() - t0
    f1 = b.fields(firsts[1], *FIELDS)
    t_fld = time.perf_counter() - t0 - t_sub
    b.release(firsts[1])
    host = time.perf_counter() - t0
    t1 = time.perf_counter()
    b.step_end()
    wait = time.perf_counter() - t1
    say(f"submits {t_sub * 1e3:.2f} ms, fields {t_fld * 1e3:.2f} ms, all {host * 1e3:.2f} ms; "
        f"then the chunk's rest {wait * 1e3:.2f} ms")
    assert all(i is not None for i in ids)
    assert host < 0.5 * (host + wait), f"host work {host * 1e3:.1f} ms, chunk rest {wait * 1e3:.1f} ms"
    done = drain(b)
    assert sorted(done) == sorted(ids + [rb])
    for f, p in zip((f0, f1), small[:2]):
        g, _, _ = alone(p, LR_FP64, steps=4)
        same_fields(f, g.fields(*FIELDS), "request copied during a chunk")
    for p, rid in zip(small[2:], ids):
        g, _, _ = alone(p, LR_FP64, steps=8)
        same_fields(b.fields(rid, *FIELDS), g.fields(*FIELDS), p["name"])


def test_pool_full_is_eagain_then_fits_after_release():
    p = inputs.random_mixed(41, 64, 64)
    probe = Batch(nmat=2, precision=LR_FP32, max_slots=4, pool_bytes=1 << 20)
    f = probe.footprint(64, 64)
    probe.close()
    b = Batch(nmat=2, precision=LR_FP32, max_slots=4, pool_bytes=f + f // 2, chunk_steps=2)
    a = b.submit(p, 1e30, max_steps=4, k_eps=1e-6)
    assert a is not None
    assert b.submit(p, 1e30, max_steps=4, k_eps=1e-6) is None  # no range large enough
    b.release(a)
    c = b.submit(p, 1e30, max_steps=4, k_eps=1e-6)
    assert c is not None and c != a
    drain(b)
    assert b.status(c)[0] == LR_OK


def test_batch_rejects_bad_requests():
    p = inputs.random_mixed(51, 16, 16)
    b = Batch(nmat=2, precision=LR_FP64, max_slots=2, pool_bytes=16 << 20)
    q = dict(p)
    q["k"] = p["k"] * 0.5  # fractions no longer sum to 1
    with pytest.raises(LRError):
        b.submit(q, 1.0)
    with pytest.raises(LRError):
        b.submit(inputs.random_mixed(52, 16, 16, nmat=3), 1.0)  # nmat differs
    rid = b.submit(p, 1.0, max_steps=0)  # nothing to do: finished at once
    assert b.poll() == [rid] and b.status(rid)[0] == LR_OK and b.step() == 0
    with pytest.raises(LRError):
        b.status(rid + 100)


def test_set_state_device_equals_host():
    import torch
    p = inputs.random_mixed(61, 37, 29, nmat=2)
    a = Solver(p["nx"], p["ny"], p["gammas"], p["domain"])
    a.set_state(0.0, p["k"], p["rho"], p["e"], p["ux"], p["uy"])
    d = Solver(p["nx"], p["ny"], p["gammas"], p["domain"])
    dev = [torch.tensor(np.ascontiguousarray(p[n]), dtype=torch.float64, device="cuda")
           for n in ("k", "rho", "e", "ux", "uy")]
    d.set_state_device(0.0, *dev)
    for s in (a, d):
        s.run(1e30, max_steps=6)
    same_fields(d.fields(*FIELDS), a.fields(*FIELDS), "device input")
    bad = [x.clone() for x in dev]
    bad[0] *= 0.5
    with pytest.raises(LRError) as e:
        d.set_state_device(0.0, *bad)
    assert e.value.code == -8
    bad = [x.clone() for x in dev]
    bad[3][3, 3] = float("nan")
    with pytest.raises(LRError) as e:
        d.set_state_device(0.0, *bad)
    assert e.value.code == -5


def test_set_state_device_float32_inputs():
    """float32 device inputs are widened exactly: the same as the host call
    with the float-rounded values (pure cells, so the fractions stay exact)."""
    import torch
    p = inputs.sod(64, 4)
    names = ("k", "rho", "e", "ux", "uy")
    f32 = [torch.tensor(np.ascontiguousarray(p[n]), dtype=torch.float32, device="cuda") for n in names]
    d = Solver(p["nx"], p["ny"], p["gammas"], p["domain"])
    d.set_state_device(0.0, *f32)
    a = Solver(p["nx"], p["ny"], p["gammas"], p["domain"])
    a.set_state(0.0, *[x.double().cpu().numpy() for x in f32])
    for s in (a, d):
        s.run(1e30, max_steps=5)
    same_fields(d.fields(*FIELDS), a.fields(*FIELDS), "float32 device input")


def test_autotuned_schedule_keeps_results():
    """The autotuner times the twelve schedules (persistent grid x graph
    replay x tile shape) on the first chunks, forward then in reverse, and
    keeps the fastest; every schedule runs the same arithmetic, so the
    results equal the problems' alone, whatever it chose."""
    ps = problems()
    steps = 2 * 2 * LR_NSCHED + 6  # the tuning chunks of 2 steps, then three more
    b = Batch(nmat=2, precision=LR_FP32, max_slots=8, pool_bytes=64 << 20, chunk_steps=2, autotune=True)
    ids = [b.submit(p, 1e30, max_steps=steps, k_eps=1e-6) for p in ps]
    assert b.schedule()[3] is None  # still timing
    say(f"autotuner: {LR_NSCHED} schedules over {steps} steps of 4 problems")
    drain(b)
    persistent, graph, tile, rates = b.schedule()
    assert rates is not None and rates.shape == (LR_NSCHED,) and np.all(rates > 0)
    assert int(persistent) + 2 * int(graph) + 4 * tile == int(np.argmax(rates))
    for p, rid in zip(ps, ids):
        g, n, _ = alone(p, LR_FP32, steps=steps)
        same_fields(b.fields(rid, *FIELDS), g.fields(*FIELDS), p["name"])


@pytest.mark.parametrize("tile", [LR_TILE_16x16, LR_TILE_32x16, LR_TILE_32x12])
@pytest.mark.parametrize("precision,nmat,persistent", [(LR_FP64, 3, False), (LR_FP32, 2, True)])
def test_tile_shapes_give_the_same_bits(tile, precision, nmat, persistent):
    """The step kernels on 16x16, 32x16 and 32x12 tiles give the bits of the
    default 32x8 tiles of a problem alone, on ragged grids smaller and larger
    than one tile and on one of more than 1024 tiles (where the launches skip
    material at rest)."""
    sizes = ((40, 24), (33, 65), (96, 17), (15, 9), (700, 400))
    ps = [inputs.random_mixed(60 + i, nx, ny, nmat=nmat) for i, (nx, ny) in enumerate(sizes)]
    steps = 10
    say(f"tile {TILE_SHAPES[tile]} precision {precision} nmat {nmat} persistent {persistent}: against alone")
    probe = Batch(nmat=nmat, precision=precision, max_slots=1, pool_bytes=1 << 20)
    pool = sum(probe.footprint(p["nx"], p["ny"]) for p in ps) + (16 << 20)
    probe.close()
    b = Batch(nmat=nmat, precision=precision, max_slots=len(ps), pool_bytes=pool, chunk_steps=4,
              tile=tile, persistent=persistent)
    kw = dict(k_eps=1e-6) if precision == LR_FP32 else {}
    ids = [b.submit(p, 1e30, max_steps=steps, **kw) for p in ps]
    drain(b)
    assert b.schedule()[2] == tile
    for p, rid in zip(ps, ids):
        rc, st, _ = b.status(rid)
        assert rc == LR_OK and st == steps
        g, n, _ = alone(p, precision, steps=steps)
        same_fields(b.fields(rid, *FIELDS), g.fields(*FIELDS), f"{p['name']} on tile {TILE_SHAPES[tile]}")


@pytest.mark.parametrize("precision,nmat", [(LR_FP64, 3), (LR_FP32, 2), (LR_FP64, 1)])
def test_single_problem_tile_shapes_give_the_same_bits(precision, nmat):
    """A problem alone on each tile shape (the FP64 32x12 launches with two
    threads per cell in the Lagrange and dual kernels, as 32x8) gives the bits
    of 32x8, on ragged grids; the automatic choice keeps 32x8 for a grid whose
    32x8 node tiles fit on the 256 CUs, takes 32x12 for one whose 32x12 ones do,
    and 32x16 beyond."""
    steps = 12
    auto = {(70, 37): LR_TILE_32x8, (448, 192): LR_TILE_32x12, (130, 250): LR_TILE_32x8,
            (700, 400): LR_TILE_32x16}
    for i, (nx, ny) in enumerate(auto):
        p = inputs.random_mixed(70 + i, nx, ny, nmat=nmat)
        g0, n0, _ = alone(p, precision, steps=steps, tile=LR_TILE_32x8)
        assert n0 == steps and g0.stage("run")[3] == LR_TILE_32x8
        ref = g0.fields(*FIELDS)
        for tile in (LR_TILE_16x16, LR_TILE_32x16, LR_TILE_32x12, LR_TILE_AUTO):
            say(f"{nx}x{ny} precision {precision} nmat {nmat} alone on tile {tile}")
            g, n, _ = alone(p, precision, steps=steps, tile=tile)
            assert n == steps
            if tile == LR_TILE_AUTO:
                assert g.stage("run")[3] == auto[(nx, ny)]
            same_fields(g.fields(*FIELDS), ref, f"{nx}x{ny} on tile {tile}")


@pytest.mark.parametrize("nmat", [2, 3])
def test_wide_and_narrow_tiles_give_the_same_bits(nmat):
    """Small FP64 launches run the Lagrange and dual tiles with 512 threads,
    large ones with 256: the same problem alone (a small launch) and beside
    a large one in a batch (more than 1024 tiles) must give the same bits."""
    small = inputs.random_mixed(51, 100, 70, nmat=nmat)
    big = inputs.random_mixed(52, 700, 500, nmat=nmat)
    steps = 12
    g, n, _ = alone(small, LR_FP64, steps=steps)
    ref = g.fields(*FIELDS)
    probe = Batch(nmat=nmat, precision=LR_FP64, max_slots=2, pool_bytes=1 << 20)
    pool = probe.footprint(100, 70) + probe.footprint(700, 500) + (16 << 20)
    probe.close()
    b = Batch(nmat=nmat, precision=LR_FP64, max_slots=2, pool_bytes=pool, chunk_steps=4)
    rs = b.submit(small, 1e30, max_steps=steps)
    b.submit(big, 1e30, max_steps=steps)
    say(f"100x70 beside 700x500 (FP64, {nmat} materials): 256-thread tiles, against the problem alone")
    drain(b)
    rc, st, _ = b.status(rs)
    assert rc == LR_OK and st == steps
    same_fields(b.fields(rs, *FIELDS), ref, "small problem")


def test_at_rest_skips_give_the_same_bits():
    """Only launches of more than 1024 tiles skip the work of material at rest
    (remap regions of zero volume and cells whose four nodes are at rest,
    dual regions without mass flux).  The triple point, whose shock has not
    yet reached most of the grid, alone (a small FP64 launch, no skips) and
    beside a large problem in a batch (with the skips) must give the same
    fields."""
    tp = inputs.triple_point(1)
    big = inputs.random_mixed(53, 700, 500, nmat=3)
    steps = 40
    g, n, _ = alone(tp, LR_FP64, steps=steps)
    assert n == steps
    ref = g.fields(*FIELDS)
    assert np.count_nonzero(ref["ux"] == 0.0) > ref["ux"].size // 2  # mostly at rest still
    probe = Batch(nmat=3, precision=LR_FP64, max_slots=2, pool_bytes=1 << 20)
    pool = probe.footprint(tp["nx"], tp["ny"]) + probe.footprint(700, 500) + (16 << 20)
    probe.close()
    b = Batch(nmat=3, precision=LR_FP64, max_slots=2, pool_bytes=pool, chunk_steps=4)
    rs = b.submit(tp, 1e30, max_steps=steps)
    b.submit(big, 1e30, max_steps=steps)
    say("triple point 448x192 beside 700x500 (FP64): at-rest skips, against the problem alone")
    drain(b)
    rc, st, _ = b.status(rs)
    assert rc == LR_OK and st == steps
    same_fields(b.fields(rs, *FIELDS), ref, "triple point")


@pytest.mark.parametrize("precision", [LR_FP64, LR_FP32])
def test_mixed_list_grows_and_the_step_runs_again(precision):
    """A problem whose list of mixed cells starts at 16 entries (far fewer
    than its mixed cells) stops at its first step, grows the list to the
    count the step found and runs the step again: alone and in a batch its
    fields equal those of the problem run with room from the start."""
    p = inputs.random_mixed(81, 90, 70, nmat=3)
    k = p["k"]
    assert ((k > 1e-6).sum(0) >= 2).sum() > 200
    kw = dict(k_eps=1e-6) if precision == LR_FP32 else {}
    say(f"mixed-cell list of 16 entries, 90x70, 3 materials, precision {precision}")
    ref = Solver(p["nx"], p["ny"], p["gammas"], p["domain"], precision=precision, **kw)
    ref.set_state(0.0, p["k"], p["rho"], p["e"], p["ux"], p["uy"])
    ref.run(1e30, max_steps=12)
    want = ref.fields(*FIELDS)
    small = Solver(p["nx"], p["ny"], p["gammas"], p["domain"], precision=precision, mix_list=16, **kw)
    small.set_state(0.0, p["k"], p["rho"], p["e"], p["ux"], p["uy"])
    n, _ = small.run(1e30, max_steps=5)
    for _ in range(7):  # and one step at a time
        small.step()
    assert n == 5
    same_fields(small.fields(*FIELDS), want, "alone with a growing list")
    b = Batch(nmat=3, precision=precision, max_slots=2, pool_bytes=64 << 20, chunk_steps=4)
    rid = b.submit(p, 1e30, max_steps=12, mix_list=16, **kw)
    drain(b)
    rc, st, _ = b.status(rid)
    assert rc == LR_OK and st == 12
    same_fields(b.fields(rid, *FIELDS), want, "in a batch with a growing list")
    # a list just large enough for the initial state: it overflows later, as
    # the bubble's interface lengthens, in the middle of a chunk
    q = inputs.shock_bubble(83, grid=(96, 64))
    nmix0 = int(((q["k"] > 1e-6).sum(0) >= 2).sum())
    ref = Solver(q["nx"], q["ny"], q["gammas"], q["domain"], precision=precision, **kw)
    ref.set_state(0.0, q["k"], q["rho"], q["e"], q["ux"], q["uy"])
    ref.run(1e30, max_steps=60)
    b = Batch(nmat=2, precision=precision, max_slots=2, pool_bytes=64 << 20, chunk_steps=4)
    rid = b.submit(q, 1e30, max_steps=60, mix_list=nmix0 + 1, **kw)
    drain(b)
    rc, st, _ = b.status(rid)
    assert rc == LR_OK and st == 60
    same_fields(b.fields(rid, *FIELDS), ref.fields(*FIELDS), "shock-bubble with a list that grows mid-chunk")
