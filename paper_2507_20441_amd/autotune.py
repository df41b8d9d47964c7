"""Autotuner for the schedule of the batched kernels.

The batched persistent kernels take four knobs (tm_batch_options): samples
per tile -- the unit of work pulled from the device counter, so also the
samples each of a workgroup's 256 lanes takes (tile / 256) -- the grid size
(how many workgroups, hence wavefronts, share the jobs at once), the LDS
bytes that stage a job's interval prefix for its root draws, and the pass
limit (left at its default: it only splits a batch).  Results never depend
on them -- every sample is keyed by (seed, sample id) -- so the tuner times
the real batch under each candidate, checks that every result is unchanged,
and keeps the fastest: a grid over (tile, grid), then the LDS staging at the
best pair.
"""
import time

from . import timest as T


def candidates(cus):
    tiles = (2048, 8192, 32768)
    grids = (0, 4 * cus, 16 * cus)
    return [(t, b) for t in tiles for b in grids]


LDS_CANDIDATES = (0, 24 * 1024, 64 * 1024)


def _time(weights, ks, seeds, repeats):
    import torch
    best, out = None, None
    for _ in range(repeats):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = T.sample_batch(weights, ks, seeds)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) * 1e3
        best = dt if best is None else min(best, dt)
    return best, [(r.acc2.value, r.acc2_sq.value, r.n_valid) for r in out]


def tune(weights, ks, seeds, cus, repeats=2, cands=None):
    """Time tm_sample_batch over the given weight sets for each (tile,
    blocks) candidate, then each LDS staging size at the best pair; set the
    fastest schedule and return it as (tile, blocks, root_lds) with all
    timings (ms) keyed by the same triples."""
    cands = cands or candidates(cus)
    prev = T.batch_options()
    times = {}
    ref = None
    lds0 = prev["root_lds"]
    for tile, blocks in cands:
        T.batch_options(tile=tile, blocks=blocks, root_lds=lds0)
        dt, sig = _time(weights, ks, seeds, repeats)
        if ref is None:
            ref = sig
        elif sig != ref:
            T.batch_options(**prev)
            raise AssertionError(f"schedule {tile},{blocks} changed a result")
        times[(tile, blocks, lds0)] = dt
    tile, blocks, _ = min(times, key=times.get)
    for lds in LDS_CANDIDATES:
        if (tile, blocks, lds) in times:
            continue
        T.batch_options(tile=tile, blocks=blocks, root_lds=lds)
        dt, sig = _time(weights, ks, seeds, repeats)
        if sig != ref:
            T.batch_options(**prev)
            raise AssertionError(f"root_lds {lds} changed a result")
        times[(tile, blocks, lds)] = dt
    choice = min(times, key=times.get)
    T.batch_options(tile=choice[0], blocks=choice[1], root_lds=choice[2])
    return choice, times
