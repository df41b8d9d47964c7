"""Autotuner for the schedule of the batched kernels.

The batched sampler's persistent kernels take two knobs: samples per tile
(the unit of work pulled from the device counter) and the grid size.  Results
never depend on them -- every sample is keyed by (seed, sample id) -- so the
tuner simply times the real batch under each candidate and keeps the fastest.
"""
import time

from . import timest as T


def candidates(cus):
    return [(2048, 0), (8192, 0), (32768, 0), (8192, 4 * cus), (8192, 16 * cus),
            (32768, 16 * cus), (131072, 0)]


def tune(weights, ks, seeds, cus, repeats=2, cands=None):
    """Time tm_sample_batch over the given weight sets for each (tile,
    blocks) candidate; set and return the fastest with all timings (ms)."""
    import torch
    cands = cands or candidates(cus)
    times = {}
    ref = None
    for tile, blocks in cands:
        T.batch_config(tile, blocks)
        best = None
        for _ in range(repeats):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = T.sample_batch(weights, ks, seeds)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) * 1e3
            best = dt if best is None else min(best, dt)
        sig = [(r.acc2.value, r.n_valid) for r in out]
        if ref is None:
            ref = sig
        elif sig != ref:
            raise AssertionError(f"schedule {tile},{blocks} changed a result")
        times[(tile, blocks)] = best
    choice = min(times, key=times.get)
    T.batch_config(*choice)
    return choice, times
