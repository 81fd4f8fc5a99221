"""Serving loop: solve requests (tau*omega, geometry, size) arrive over time,
are admitted against an HBM budget, keep their lattices on the device, and
are advanced together by the batch API (one fused launch per step over every
resident lattice).  Requests join the running batch as memory frees up and
leave it when their step count is reached (continuous batching).

The comparison is the plain loop: the same requests, first come first
served, one solver at a time stepped alone.

    python -m paper_0904_4504_amd.serve --rate 2.0 --requests 40 [--plain]
"""
import argparse
import collections
import json
import os
import sys
import time

import numpy as np

from . import lbm as L


class Request:
    __slots__ = ("rid", "arrival", "solve", "bytes", "solver", "admitted", "done", "result")

    def __init__(self, rid, arrival, solve):
        self.rid = rid
        self.arrival = arrival
        self.solve = solve
        self.bytes = 0
        self.solver = None
        self.admitted = None
        self.done = None
        self.result = None


def _summary(reqs, wall, mode, host_s=None):
    lat = np.array([r.done - r.arrival for r in reqs])
    out = {
        "mode": mode,
        "requests": len(reqs),
        "wall_s": wall,
        "solves_per_s": len(reqs) / wall if wall > 0 else float("nan"),
        "latency_p50_s": float(np.percentile(lat, 50)),
        "latency_p99_s": float(np.percentile(lat, 99)),
        "latency_mean_s": float(lat.mean()),
    }
    if host_s is not None:
        # time the loop spent on the host between device chunks (admission,
        # solver creation, retirement, read-out), while the device idled
        out["host_s"] = host_s
        out["host_fraction"] = host_s / wall if wall > 0 else float("nan")
    return out


def _progress(tag, done, total, t0, clock):
    if done % 20 == 0 or done == total:
        print(f"[{tag}] {done}/{total} requests done, {clock() - t0:.1f} s", file=sys.stderr,
              flush=True)


def _finish(req):
    req.result = req.solver.impedance()
    req.solver.close()
    req.solver = None


def serve(trace, budget_bytes=200e9, chunk=256, stream=None, clock=time.perf_counter,
          max_resident=4096, progress=None):
    """Continuous batching.  trace: [(arrival_s, lbm_inputs.Solve)] sorted by
    arrival.  Each device chunk runs `chunk` steps or up to the next
    completion, whichever comes first, so a finished request is retired (and
    its memory freed for the queue) at the step it ends.  Returns (requests
    with results and timestamps, summary)."""
    import torch
    stream = stream or torch.cuda.Stream()
    pending = collections.deque(Request(i, t, s) for i, (t, s) in enumerate(trace))
    waiting = collections.deque()
    resident = []
    used = 0
    done = []
    batch = L.Batch(stream)
    t0 = clock()
    host_s = 0.0
    th = clock()
    try:
        while pending or waiting or resident:
            now = clock() - t0
            while pending and pending[0].arrival <= now:
                r = pending.popleft()
                # the solvers start from rest: no population-load buffer
                r.bytes = L.required_bytes(L.params_from_solve(r.solve, loads=False)) + 512
                if r.bytes > budget_bytes:
                    raise ValueError(f"request {r.rid} needs {r.bytes} B > budget")
                waiting.append(r)
            # admit first come first served while memory and slots allow
            while waiting and used + waiting[0].bytes <= budget_bytes and \
                    len(resident) < max_resident:
                r = waiting.popleft()
                r.solver = L.Solver(L.params_from_solve(r.solve, loads=False), stream=stream)
                batch.add(r.solver)
                r.admitted = clock() - t0
                used += r.bytes
                resident.append(r)
            if not resident:
                if pending:
                    time.sleep(max(0.0, min(0.01, pending[0].arrival - (clock() - t0))))
                th = clock()  # idle waiting for arrivals is not host work
                continue
            left = min(r.solve.nsteps - r.solver.steps_done for r in resident)
            host_s += clock() - th
            batch.step(min(chunk, left))
            batch.synchronize()
            th = clock()
            still = []
            for r in resident:
                if r.solver.steps_done >= r.solve.nsteps:
                    batch.remove(r.solver)
                    _finish(r)
                    r.done = clock() - t0
                    used -= r.bytes
                    done.append(r)
                    if progress:
                        _progress(progress, len(done), len(trace), t0, clock)
                else:
                    still.append(r)
            resident = still
        wall = clock() - t0
    finally:
        for r in resident:
            if r.solver is not None:
                r.solver.close()
        batch.close()
    done.sort(key=lambda r: r.rid)
    return done, _summary(done, wall, "batched", host_s)


def serve_plain(trace, stream=None, clock=time.perf_counter, progress=None):
    """The plain loop: one request at a time, in arrival order, stepped alone."""
    import torch
    stream = stream or torch.cuda.Stream()
    reqs = [Request(i, t, s) for i, (t, s) in enumerate(trace)]
    t0 = clock()
    for r in reqs:
        now = clock() - t0
        if r.arrival > now:
            time.sleep(r.arrival - now)
        r.admitted = clock() - t0
        r.solver = L.Solver(L.params_from_solve(r.solve, loads=False), stream=stream)
        r.solver.step(r.solve.nsteps)
        r.solver.synchronize()
        _finish(r)
        r.done = clock() - t0
        if progress:
            _progress(progress, r.rid + 1, len(reqs), t0, clock)
    wall = clock() - t0
    return reqs, _summary(reqs, wall, "plain")


def main(argv=None):
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import lbm_inputs as W
    ap = argparse.ArgumentParser()
    ap.add_argument("--rate", type=float, default=2.0, help="arrivals per second")
    ap.add_argument("--requests", type=int, default=40)
    ap.add_argument("--warmup-requests", type=int, default=4)
    ap.add_argument("--period", type=int, default=1024)
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--chunk", type=int, default=256)
    ap.add_argument("--plain", action="store_true", help="also run the plain loop")
    ap.add_argument("--seed", type=int, default=5)
    a = ap.parse_args(argv)
    import torch
    torch.cuda.set_device(0)
    n = a.requests + a.warmup_requests
    trace = W.serving_trace(a.rate, n, seed=a.seed, period=a.period)
    out = {}
    reqs, summ = serve(trace, a.budget_gb * 1e9, a.chunk)
    keep = reqs[a.warmup_requests:]
    out["batched"] = dict(_summary(keep, max(r.done for r in keep) - keep[0].arrival, "batched"),
                          rate=a.rate)
    if a.plain:
        reqs_p, _ = serve_plain(trace)
        keep_p = reqs_p[a.warmup_requests:]
        out["plain"] = dict(_summary(keep_p, max(r.done for r in keep_p) - keep_p[0].arrival,
                                     "plain"), rate=a.rate)
        dz = max(abs(x.result["Z"] - y.result["Z"]) / abs(y.result["Z"])
                 for x, y in zip(reqs, reqs_p))
        out["max_rel_dZ_batched_vs_plain"] = dz
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
