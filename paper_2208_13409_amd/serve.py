"""Request loop serving many solves on one GPU with continuous batching.

Requests arrive over time.  Each is admitted into a ``Batch`` as soon as a
slot and a range of its device pool are free (admission by device-memory
footprint: ``submit`` declines while the request does not fit).  It then
runs in the shared launches with whatever else is running, and its result
fields are copied to the host when it finishes, after which its slot and
memory are released for the next one.

The device is kept busy: admissions (host-side checks and staging of the
inputs) run while a chunk of steps is in flight, and as soon as a chunk
ends the next one is launched, before the results of the requests that
finished in it are copied back (the batch copies them on a stream of its
own).  Latency is measured from a request's arrival to its fields being on
the host.  ``requests`` may be any indexable sequence (a lazy one builds
each request when it is admitted).
"""
import collections
import time

import numpy as np


def percentile(xs, q):
    return float(np.percentile(np.asarray(xs, dtype=float), q)) if len(xs) else float("nan")


def serve(batch, requests, arrivals, fields=("rho", "p"), keep=False):
    """Serve ``requests`` (problem dicts with ``t_end``) arriving at
    ``arrivals`` seconds after the start, in real time.

    Returns a dict: per-request latency, steps, cells and admission time,
    the fields when ``keep``, the wall time, the cell-updates served per
    second, the share of the wall time with a chunk of steps in flight, and
    p50/p99 latency."""
    n = len(requests)
    order = sorted(range(n), key=lambda i: arrivals[i])
    lat, steps, rcs = [None] * n, [0] * n, [None] * n
    cells, admitted = [0] * n, [None] * n
    results = {}
    queue = collections.deque()
    head = {}  # the built request at the head of the queue, not yet admitted
    ids = {}
    nxt, done = 0, 0
    busy = 0.0
    max_running = 0
    t0 = time.perf_counter()

    def clock():
        return time.perf_counter() - t0

    def admit(may_idle):
        """submit queued requests while they fit"""
        while queue:
            i = queue[0]
            r = head.get(i)
            if r is None:
                r = head[i] = requests[i]
            rid = batch.submit(r, r["t_end"])
            if rid is None:
                if may_idle and batch.running() == 0 and not ids:
                    raise RuntimeError(f"request {i} does not fit in an empty batch")
                return
            ids[rid] = i
            cells[i] = r["nx"] * r["ny"]
            admitted[i] = clock()
            del head[i]
            queue.popleft()

    def collect(finished):
        """fields of the finished requests to the host, then their release"""
        nonlocal done
        for rid in finished:
            i = ids.pop(rid)
            rc, st, _ = batch.status(rid)
            rcs[i], steps[i] = rc, st
            out = batch.fields(rid, *fields) if rc == 0 else None
            lat[i] = clock() - arrivals[i]
            if keep:
                results[i] = out
            batch.release(rid)
            done += 1

    inflight = False  # a chunk launched and not yet waited for
    t_launch = 0.0
    while done < n:
        now = clock()
        while nxt < n and arrivals[order[nxt]] <= now:
            queue.append(order[nxt])
            nxt += 1
        admit(may_idle=not inflight)  # with a chunk in flight: overlaps it
        if inflight:
            batch.step_end()
            busy += clock() - t_launch
            inflight = False
            finished = batch.poll()
            running = batch.running()
            max_running = max(max_running, running)
            if running:  # the next chunk at once; the results come back meanwhile
                t_launch = clock()
                batch.step_begin()
                inflight = True
            collect(finished)
            continue
        running = batch.running()
        max_running = max(max_running, running)
        if running:
            t_launch = clock()
            batch.step_begin()
            inflight = True
        else:
            collect(batch.poll())  # requests that finished at admission (nothing to step)
            if not ids and not queue and nxt < n:  # idle until the next arrival
                time.sleep(max(0.0, arrivals[order[nxt]] - clock()))
    wall = clock()
    served = float(sum(c * s for c, s in zip(cells, steps)))
    return dict(latency=lat, steps=steps, rc=rcs, cells=cells, admitted=admitted, wall=wall,
                cell_updates_per_s=served / wall if wall > 0 else float("nan"),
                busy=busy / wall if wall > 0 else float("nan"), max_running=max_running,
                p50=percentile(lat, 50), p99=percentile(lat, 99), results=results)
