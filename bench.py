#!/usr/bin/env python3
"""Benchmark of the lattice-BGK hot path on one MI355X.

Default workload (batch): the 256 uneven solves of the batched sweep (sides
256-2048 cells, aspect 1:1, 2:1, 4:1, a plate or a rectangle of 8-64 cells
per side, tau*omega log-uniform in [1e-2, 1e2], U0 = 1e-3, D2Q37, FP32
deviation storage with FP64 force and lock-in), drawn from one seeded PCG64
stream, advanced together as one batch with the tile the autotuner picks.
Every member keeps its state as the six H2 coefficients per cell (48 B per
update in FP32): 13.5 GB of state, 53 times the 256 MB last-level cache, so
every step streams it from HBM.  One step = one stream-collide launch over
the tiles of all 256 lattices (pull advection of the 37 populations from the
coefficients, bounce-back with the moving-wall term, moments, H2
equilibrium, regularized collision) plus one launch that computes each
solve's FP64 momentum-exchange force, appends it to the history and
accumulates the lock-in sums.  The state is created and warmed up on the
device before the timed steps.

Other workloads: beam_box (3 x 1024^2 with the 32 x 16 body; its 151 MB of
coefficient state stays in the last-level cache between steps, so its
bandwidth is not an HBM figure), plate_sweep (5 plates of 4 x 2048).

Prints one JSON line: MLUPS (fluid-cell updates per second); the dominant
kernel against its roofline (each launch of it records its own start and stop
events over a second pass of K steps); and the CPU oracle timed on a bounded
sample of the workload on this host, on all its cores and on one.

The rate depends on the run's length: a short run (--steps 20) runs at the
GPU's boost shader clock, while over about 600 steps of this streaming load
the clock settles some 9 % lower under the board's power management and the
batch step slows by as much (2.78 to 3.02 ms); the default 1000 + 1000 steps
report that sustained rate.

    python bench.py [--steps K] [--warmup W] [--workload batch|beam_box|plate_sweep]
    python bench.py --workload batch_sweep   # sweep solves/s, batched vs plain loop
    python bench.py --workload serving       # p50/p99 latency, batched vs plain loop
"""
import argparse
import dataclasses
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("MLUPS & HBM GB/s (%peak); sweep solves/s + p50/p99 latency vs plain loop")
HBM_PEAK_GBS = 8000.0
CSRC = os.path.join(ROOT, "paper_0904_4504_amd", "csrc")
# dominant kernel per device representation: (name, source file)
KERNELS = {
    1: ("lbm::step_kernel<D2Q37, float, false, false, 256, false>", "kernels.hip"),
    2: ("lbm::coef_kernel<D2Q37, float, {rb}, false>", "coef.hip"),
}
# committed rocprofv3 counters per (representation, workload)
COUNTERS = {
    (1, "beam_box"): "step_kernel_beam_box_counters.json",
    (2, "beam_box"): "coef_kernel_beam_box_counters.json",
    (2, "batch"): "coef_kernel_batch_counters.json",
}
# FP32 arithmetic per lattice update of the coefficient kernel (D2Q37) by
# cells per thread K, counted on the compiled kernel without its wall-link
# path (FMA = 2, add or multiply = 1, per lane over K): forming the 37
# streamed populations from their source cells' coefficients and gathering
# their six moments (source-cell terms shared by the K cells of a lane,
# per-row sums and the scatter), plus 28 for the collision.
COEF_FLOPS_PER_LU = {1: 469, 2: 423, 3: 401}
COEF_K_DEFAULT = 3  # the library's tile when none is given
# FP32 vector peak without packed FP32 (which this build does not use):
# 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz
FP32_VALU_PEAK_TFLOPS = 78.6
# host sources that shape what a kernel's counters measure besides its own
# file: the work order, tile sizes and layout
ORDER_SOURCES = ("api.cpp", "batch.cpp", "internal.hpp", "solver.hpp")


def sources_hash(src):
    """sha256 (16 hex) over the kernel's source file and ORDER_SOURCES."""
    h = hashlib.sha256()
    for name in (src,) + ORDER_SOURCES:
        with open(os.path.join(CSRC, name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def workload(name, steps, warmup):
    import lbm_inputs as W
    n = warmup + steps
    if name == "batch":
        solves = W.batch_sweep()
        desc = ("batch: the 256 seeded solves of the batched sweep (sides 256-2048, aspect "
                "1/2/4, plate or 8-64-cell rectangle, tau*omega 1e-2..1e2, U0 1e-3), D2Q37 "
                "FP32-deviation storage, FP64 force + lock-in, one batch, autotuned tile")
    elif name == "beam_box":
        solves = [W.beam_box(tw) for tw in W.BEAM_TAU_OMEGA]
        desc = ("beam_box: 1024x1024 domain, 32x16 body centred, rest-equilibrium far field, "
                "D2Q37 FP32-deviation storage, FP64 force + lock-in, tau*omega {0.1, 1, 10} "
                "as one batch")
    elif name == "plate_sweep":
        solves = [W.plate_sweep(tw) for tw in W.PLATE_SWEEP_TAU_OMEGA]
        desc = ("plate_sweep: 4x2048 plates, stationary far wall, D2Q37 FP32-deviation, "
                "tau*omega {0.01, 0.1, 1, 10, 100} as one batch")
    else:
        raise SystemExit(f"unknown workload {name}")
    # the timed steps form the lock-in window, so every step runs the whole
    # path; a second pass of as many steps (kernel timing) follows the window
    solves = [dataclasses.replace(s, nsteps=n + steps, window_first=warmup, window_count=steps)
              for s in solves]
    return solves, desc


def copy_ceiling(stream, nbytes=1 << 31, reps=5):
    """Measured copy ceilings on this GPU, next to the 8 TB/s datasheet peak:
    bytes read plus written per second (GB/s) of two device copies of nbytes,
    torch's device-to-device copy (a DMA-style copy) and an elementwise
    kernel (dst = src * 1), which streams like a plain one-vector-per-thread
    copy kernel (6.2 against 6.3 TB/s for the best hand-written copy over
    13 GB on the same GPU; the DMA-style copy 5.0 TB/s)."""
    import torch
    out = {}
    with torch.cuda.stream(stream):
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for name, fn in (("memcpy", lambda: dst.copy_(src)),
                         ("elementwise", lambda: torch.mul(src, 1.0, out=dst))):
            fn()
            t0 = torch.cuda.Event(enable_timing=True)
            t1 = torch.cuda.Event(enable_timing=True)
            t0.record(stream)
            for _ in range(reps):
                fn()
            t1.record(stream)
            torch.cuda.synchronize()
            out[name] = 2 * nbytes / (t0.elapsed_time(t1) / reps / 1e3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return out


def traffic_from_profile(repr_, name):
    """HBM bytes per launch from committed rocprofv3 counters of this kernel
    and workload, if they were taken on the current kernel and host sources;
    else None."""
    _, src = KERNELS[repr_]
    counters = COUNTERS.get((repr_, name))
    if counters is None:
        return None
    try:
        with open(os.path.join(ROOT, "profiles", counters)) as fh:
            prof = json.load(fh)
    except (OSError, ValueError):
        return None
    if prof.get("sources_sha256_16") != sources_hash(src):
        return None
    return prof.get("hbm_bytes_per_launch")


def _oracle_rate(solve, threads, budget_s):
    """(MLUPS, steps, seconds) of the FP64 oracle on `threads` threads over
    about budget_s seconds of steps of `solve` from rest."""
    import oracle as O
    import lbm_inputs as W
    p = O.OracleParams(
        Q=solve.Q, nx=solve.nx, ny=solve.ny, tau=solve.tau, omega=solve.omega, u0=solve.u0,
        geometry=O.GEOM_BOX if solve.geometry == W.BOX else O.GEOM_PLATE,
        far=O.FAR_EQ if solve.far == W.FAR_EQ else O.FAR_WALL,
        box_x0=solve.box[0], box_y0=solve.box[1], box_lx=solve.box[2], box_ly=solve.box[3],
        nthreads=threads)
    O.run(p, 1)  # first call: page in, thread pool
    t0 = time.perf_counter()
    O.run(p, 2)
    per_step = (time.perf_counter() - t0) / 2
    nsteps = max(2, min(4000, int(budget_s / max(per_step, 1e-6))))
    t0 = time.perf_counter()
    O.run(p, nsteps)
    dt = time.perf_counter() - t0
    return solve.fluid_cells * nsteps / dt / 1e6, nsteps, dt


def cpu_baseline(solve, budget_s):
    """The FP64 oracle on a bounded sample of the workload (one of its solves
    from rest), on all of this host's cores and on one core."""
    cores = len(os.sched_getaffinity(0))
    mlups, n, dt = _oracle_rate(solve, cores, budget_s)
    mlups1, n1, dt1 = _oracle_rate(solve, 1, budget_s / 3)
    return {"value": mlups, "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "value_1core": mlups1,
            "sample": f"{solve.name}: one {solve.nx}x{solve.ny} lattice of the workload from "
                      f"rest, FP64 oracle, OpenMP over rows: {n} steps on {cores} threads in "
                      f"{dt:.1f} s; {n1} steps on 1 thread in {dt1:.1f} s"}


def sweep_mode(a):
    """Batched sweep vs the plain one-solve-at-a-time loop on the 256-solve
    batch workload (or the first `--sweep-solves` solves of the seeded draw),
    each run for `--sweep-steps` steps (lock-in over the second half; 20 480 =
    10 periods of transient and 10 of window).  Prints solves/s and MLUPS of
    both and the largest relative impedance difference between them."""
    import torch
    import lbm_inputs as W
    import paper_0904_4504_amd as P
    from paper_0904_4504_amd import autotune
    solves = [s.scaled(a.sweep_steps, a.sweep_steps // 2)
              for s in W.batch_sweep(count=a.sweep_solves)]
    cells = sum(s.fluid_cells for s in solves) * a.sweep_steps
    stream = torch.cuda.Stream()
    out = {}
    with torch.cuda.stream(stream):
        # tile chosen by the autotuner on the largest solves of the sample
        tile, tile_ms = autotune.tune(solves, stream=stream)
        # warm-up: one small solve through both paths (code objects, graphs)
        warm = solves[0].scaled(64, 32)
        with P.Solver(P.params_from_solve(warm), stream=stream) as sv:
            sv.step(64)
            sv.synchronize()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        solvers = [P.Solver(P.params_from_solve(s, tile=tile, loads=False), stream=stream)
                   for s in solves]
        batch = P.Batch(stream)
        for sv in solvers:
            batch.add(sv)
        for done in range(0, a.sweep_steps, 2048):
            batch.step(min(2048, a.sweep_steps - done))
            batch.synchronize()
            print(f"[batched] {min(done + 2048, a.sweep_steps)}/{a.sweep_steps} steps, "
                  f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
        zb = [sv.impedance() for sv in solvers]
        batch.close()
        for sv in solvers:
            sv.close()
        tb = time.perf_counter() - t0
        t0 = time.perf_counter()
        zp = []
        for k, s in enumerate(solves):
            with P.Solver(P.params_from_solve(s, tile=tile, loads=False), stream=stream) as sv:
                sv.step(a.sweep_steps)
                sv.synchronize()
                zp.append(sv.impedance())
            if (k + 1) % 16 == 0:
                print(f"[plain] {k + 1}/{len(solves)} solves, {time.perf_counter() - t0:.1f} s",
                      file=sys.stderr, flush=True)
        tp = time.perf_counter() - t0
    dz = max(abs(x["Z"] - y["Z"]) / abs(y["Z"]) for x, y in zip(zb, zp))
    out = {"metric": "sweep solves/s (batched vs plain loop)", "value": len(solves) / tb,
           "unit": "solves/s", "n_gpus": 1, "higher_is_better": True, "data": "synthetic",
           "plain_value": len(solves) / tp, "speedup": tp / tb,
           "batched_mlups": cells / tb / 1e6, "plain_mlups": cells / tp / 1e6,
           "max_rel_dZ_batched_vs_plain": dz,
           "config": {"workload": f"batch_sweep sample: first {len(solves)} of the seeded "
                                  f"256-solve draw (sides 256-2048, aspect 1/2/4, plate or box, "
                                  f"tau*omega 1e-2..1e2), {a.sweep_steps} steps each, D2Q37 FP32",
                      "wall_s_batched": tb, "wall_s_plain": tp,
                      "solver_create_included": True,
                      "tile": tile, "autotune_ms_per_step": tile_ms}}
    print(json.dumps(out), flush=True)


def serving_mode(a):
    """Continuous batching vs the plain loop on the serving mix (1 box : 4
    plates), drive period `--serve-period` steps (10 + 10 periods per
    request).  Capacity is measured with every request queued at t = 0; the
    Poisson traces then run at 0.5, 0.8 and 0.95 of it through both paths.
    Each trace has `--serve-warmup` + `--serve-requests` requests; latencies
    and solves/s are taken over the requests after the warm-up ones."""
    import torch
    import lbm_inputs as W
    from paper_0904_4504_amd import serve as S
    from paper_0904_4504_amd.serve import _summary
    torch.cuda.set_device(0)
    warm, n = a.serve_warmup, a.serve_requests
    total = warm + n

    def after_warmup(reqs, mode):
        keep = reqs[warm:]
        wall = max(r.done for r in keep) - keep[0].arrival
        return _summary(keep, wall, mode)

    burst = [(0.0, s) for _, s in W.serving_trace(1.0, total, period=a.serve_period)]
    S.serve(burst[:4], chunk=a.serve_chunk)  # warm-up: code objects, graphs
    _, cap = S.serve(burst, chunk=a.serve_chunk, progress="capacity")
    capacity = cap["solves_per_s"]
    rates = []
    keys = ("solves_per_s", "latency_p50_s", "latency_p99_s", "wall_s")
    for f in (0.5, 0.8, 0.95):
        trace = W.serving_trace(f * capacity, total, period=a.serve_period)
        rb, sb = S.serve(trace, chunk=a.serve_chunk, progress=f"batched {f}")
        rp, _ = S.serve_plain(trace, progress=f"plain {f}")
        dz = max(abs(x.result["Z"] - y.result["Z"]) / abs(y.result["Z"]) for x, y in zip(rb, rp))
        b, p = after_warmup(rb, "batched"), after_warmup(rp, "plain")
        rates.append({"load": f, "rate_per_s": f * capacity,
                      "batched": dict({k: b[k] for k in keys}, host_fraction=sb["host_fraction"]),
                      "plain": {k: p[k] for k in keys},
                      "max_rel_dZ_batched_vs_plain": dz})
    out = {"metric": "serving solves/s and p50/p99 latency (continuous batching vs plain loop)",
           "value": capacity, "unit": "solves/s", "n_gpus": 1, "higher_is_better": True,
           "data": "synthetic", "rates": rates,
           "capacity_host_fraction": cap["host_fraction"],
           "config": {"workload": f"serving mix: {warm} warm-up + {n} requests per rate, 1 box "
                                  f"(1024x1024, body 32x16) : 4 plates (4 x 1024..8192), "
                                  f"tau*omega 1e-3..1e3, period {a.serve_period} steps, "
                                  f"10 + 10 periods per request, D2Q37 FP32, HBM budget 200 GB",
                      "chunk_steps": a.serve_chunk}}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="batch")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--representation", type=int, default=0,
                    help="0 automatic, 1 populations, 2 (3: without loads) H2 coefficients")
    ap.add_argument("--tile", type=int, default=0,
                    help="kernel tile (cells per thread of the population or the coefficient "
                         "kernel); 0 = library default")
    ap.add_argument("--sweep-solves", type=int, default=256)
    ap.add_argument("--sweep-steps", type=int, default=20480)
    ap.add_argument("--serve-requests", type=int, default=400)
    ap.add_argument("--serve-warmup", type=int, default=40)
    ap.add_argument("--serve-period", type=int, default=1024)
    ap.add_argument("--serve-chunk", type=int, default=1024)
    a = ap.parse_args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the solves of a sweep are independent and would "
              "be split across GPUs by solve, which this build does not do; use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_0904_4504_amd as P

    torch.cuda.set_device(0)
    if a.workload == "batch_sweep":
        return sweep_mode(a)
    if a.workload == "serving":
        return serving_mode(a)
    solves, desc = workload(a.workload, a.steps, a.warmup)
    stream = torch.cuda.Stream()
    tile, tile_ms = a.tile, None
    with torch.cuda.stream(stream):
        if a.workload == "batch" and not a.tile and a.representation == 0:
            # the batched sweep runs with the tile the autotuner picks
            from paper_0904_4504_amd import autotune
            tile, tile_ms = autotune.tune(solves, stream=stream)
        # the runs start from rest: coefficient members need no population buffer
        solvers = [P.Solver(P.params_from_solve(s, representation=a.representation,
                                                tile=tile, loads=False),
                            stream=stream) for s in solves]
        reprs = {sv.representation for sv in solvers}
        if len(reprs) != 1:
            raise SystemExit(f"members in several representations {reprs}")
        repr_ = reprs.pop()
        batch = P.Batch(stream)
        for sv in solvers:
            batch.add(sv)
        batch.step(a.warmup)
        batch.synchronize()
        # the timed steps run as the batch runs them in production (HIP graphs)
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0.record(stream)
        batch.step(a.steps)
        t1.record(stream)
        torch.cuda.synchronize()
        batch.synchronize()
        elapsed_ms = t0.elapsed_time(t1)
        # then as many steps again, eagerly, each launch of the step kernel
        # recording its own start and stop events: its average duration for
        # the roofline
        batch.timing(True)
        batch.step(a.steps)
        batch.synchronize()
        kern_ms, launches = batch.kernel_time()
        batch.timing(False)
        state_bytes = sum(P.required_bytes(sv.p) for sv in solvers)
        batch.close()
        for sv in solvers:
            sv.close()
        del solvers
        torch.cuda.empty_cache()

    cells = sum(s.fluid_cells for s in solves)
    Q = solves[0].Q
    # algorithmic bytes per lattice update: read and write the stored state
    # once -- the Q populations, or the six H2 coefficients that hold the
    # regularized state exactly
    bytes_per_lu = 2 * (Q if repr_ == 1 else 6) * 4
    mlups = cells * a.steps / (elapsed_ms / 1e3) / 1e6
    avg_kernel_s = kern_ms / 1e3 / launches
    launch_bytes = bytes_per_lu * cells
    hbm_gbs = launch_bytes / avg_kernel_s / 1e9
    traffic = traffic_from_profile(repr_, a.workload)
    copy_gbs = copy_ceiling(stream)
    # the state read and written by one step: 2 buffers of the device state
    # (coefficients or populations) of every member; above the 256 MB
    # last-level cache it streams from HBM every step
    resident = "hbm" if state_bytes > (256 << 20) else "last-level cache (256 MB)"
    hbm = {"achieved": hbm_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": hbm_gbs / HBM_PEAK_GBS,
           "copy_ceiling": dict(copy_gbs, unit="GB/s", bytes_each_way=1 << 31),
           "frac_of_copy_ceiling": hbm_gbs / max(copy_gbs.values()),
           "algorithmic_bytes_per_launch": launch_bytes, "traffic": traffic,
           "device_bytes": state_bytes, "state_streams_from": resident}
    kernel = KERNELS[repr_][0].format(rb=tile or COEF_K_DEFAULT)
    roofline = dict(hbm, bound="hbm")
    if repr_ != 1:
        # coefficients: 48 B and 401-469 flop per update (8.4-9.8 flop/B), at or
        # below the ridge of the FP32 vector units over HBM (78.6 / 8.0 =
        # 9.8 flop/B), so the roofline bound is HBM; the vector-ALU figures go
        # alongside
        flops = COEF_FLOPS_PER_LU[tile or COEF_K_DEFAULT]
        tflops = flops * cells / avg_kernel_s / 1e12
        roofline["alu"] = {"achieved": tflops, "peak": FP32_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                           "frac": tflops / FP32_VALU_PEAK_TFLOPS, "flops_per_update": flops}
        # the same updates on the Q populations (2 Q s bytes each): the HBM
        # rate a population kernel would need to match this one
        pop_gbs = 2 * Q * 4 * cells / avg_kernel_s / 1e9
        roofline["population_form"] = {"bytes_per_update": 2 * Q * 4, "equivalent": pop_gbs,
                                       "unit": "GB/s", "over_peak": pop_gbs / HBM_PEAK_GBS}
    roofline.update({"kernel": kernel, "avg_kernel_ms": avg_kernel_s * 1e3, "launches": launches,
                     "kernel_timing": "start and stop events recorded by each launch itself "
                                      "(extended launch), a second pass of the same number of "
                                      "steps after the timed one"})
    out = {
        "metric": METRIC,
        "value": mlups,
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": elapsed_ms / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": desc,
            "lattice": f"D2Q{Q}",
            "solves": len(solves),
            "fluid_cells": cells,
            "algorithmic_bytes_per_update": bytes_per_lu,
            "representation": {1: "populations", 2: "H2 coefficients"}[repr_],
            "force_and_lockin": "f64",
            "tile": tile or (COEF_K_DEFAULT if repr_ != 1 else 1),
            "autotune_ms_per_step": tile_ms,
        },
        "roofline": roofline,
    }
    if not a.no_cpu:
        # a median-size solve of the workload
        pick = sorted(solves, key=lambda s: s.fluid_cells)[len(solves) // 2]
        out["cpu_baseline"] = cpu_baseline(pick.scaled(2, 0), a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
