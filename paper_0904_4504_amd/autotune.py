"""Tile autotuner: picks the kernel tile for a set of solves by timing it.

The library has a few tiles per device representation (cells per thread of
the population kernel: 1, 2, 4; of the coefficient kernel: 1, 2, 3).  Which
one is fastest depends on the lattice sizes, the storage and the mix of a
batch.  `tune` builds throw-away solvers for a sample of the solves with each
candidate tile, advances them together as one batch (the way they will run),
times a fixed number of steps with HIP events on the batch's stream and
returns the fastest tile.  Results are cached per (lattice, storage,
representation, size class) for the life of the process.
"""
import math

from . import lbm as L

_CACHE = {}


def candidates(representation):
    """Tiles the library accepts for a device representation."""
    return (1, 2, 3) if representation == L.REPR_COEFFICIENTS else (1, 2, 4)


def _key(solves, representation):
    cells = sum(s.nx * s.ny for s in solves)
    return (solves[0].Q, solves[0].storage, representation, len(solves),
            int(round(math.log2(max(cells, 1)))))


def tune(solves, representation=L.REPR_AUTO, steps=64, warmup=8, sample=8, stream=None,
         use_cache=True):
    """Fastest tile for advancing `solves` (lbm_inputs.Solve, all kept in the
    same representation) as one batch.  Returns (tile, {tile: ms per step}).

    Times at most `sample` of the solves (the largest ones, which dominate the
    step time) for `steps` steps after `warmup` steps; the solves' own state
    is untouched (the timing uses separate solvers)."""
    import torch
    if not solves:
        raise ValueError("no solves to tune for")
    stream = stream or torch.cuda.current_stream()
    pick = sorted(solves, key=lambda s: s.nx * s.ny, reverse=True)[:sample]
    # the representation the library picks for these solves
    with L.Solver(L.params_from_solve(pick[0].scaled(warmup + steps, 0),
                                      representation=representation), stream=stream) as probe:
        repr_ = probe.representation
    key = _key(pick, repr_)
    if use_cache and key in _CACHE:
        return _CACHE[key]
    times = {}
    for tile in candidates(repr_):
        solvers = [L.Solver(L.params_from_solve(s.scaled(warmup + steps, 0), tile=tile,
                                                representation=repr_), stream=stream)
                   for s in pick]
        batch = L.Batch(stream)
        try:
            for sv in solvers:
                batch.add(sv)
            batch.step(warmup)
            batch.synchronize()
            t0 = torch.cuda.Event(enable_timing=True)
            t1 = torch.cuda.Event(enable_timing=True)
            t0.record(stream)
            batch.step(steps)
            t1.record(stream)
            batch.synchronize()
            times[tile] = t0.elapsed_time(t1) / steps
        finally:
            batch.close()
            for sv in solvers:
                sv.close()
    best = min(times, key=times.get)
    _CACHE[key] = (best, times)
    return best, times
