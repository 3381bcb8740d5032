"""Autotuner for the batched TOA pass.

Times each candidate launch shape of the TOA pass (16-TOA tiles per chunk,
waves per workgroup, placement: launch order, XCD-grouped or balanced) on
the caller's data set and chain count with the library's event-timed stage
profiler, and keeps the fastest.
The choice is cached per data-set shape (pulsar count, TOA count, basis sizes,
chain count) so that a request always runs with the same tuning, which keeps
its results reproducible: the reduction order depends only on the tuning.
"""
from __future__ import annotations

import numpy as np

CANDIDATES = tuple((tpc, wpb, xcd) for tpc in (8, 12, 16, 24, 32, 64) for wpb in (1, 2, 4)
                   for xcd in (0, 1))


def round_fitting_tpcs(toa_offsets, n_chains, n_cu, wpb=1, rounds=(1, 2), waves_per_simd=(1, 2, 3, 4)):
    """Tiles per chunk at which the TOA pass's waves (chunks x 16-chain blocks
    x wpb waves per workgroup) just fit a whole number of rounds of the
    device's wave slots (n_cu x 4 SIMDs x waves per SIMD): the smallest such
    chunk for each round count and occupancy.  Chunks of a pulsar are split
    evenly, so these launches run in full rounds of near-equal waves."""
    off = np.asarray(toa_offsets, dtype=np.int64)
    tiles = (np.diff(off) + 15) // 16
    n_cb = (int(n_chains) + 15) // 16 * int(wpb)
    out = set()
    for r in rounds:
        for occ in waves_per_simd:
            slots = r * int(n_cu) * 4 * occ
            lo, hi = 1, max(1, int(tiles.max()))
            if int(np.maximum(1, -(-tiles // hi)).sum()) * n_cb > slots:
                continue
            while lo < hi:                      # smallest tpc with waves <= slots
                mid = (lo + hi) // 2
                if int(np.maximum(1, -(-tiles // mid)).sum()) * n_cb <= slots:
                    hi = mid
                else:
                    lo = mid + 1
            out.add(lo)
    return sorted(out)

_cache: dict = {}


def serving_tuning(toa_offsets, n_chains, n_cu):
    """TOA-pass tuning of a served request as a fixed function of its shape
    (no timing, so the choice, and with it the reduction order and the
    request's bits, cannot depend on what else runs on the device): one-wave
    workgroups, XCD-aware placement, and the chunk length at which the
    request's waves fill one round of the device at two waves per SIMD (the
    one-wave form's occupancy), kept between 4 and 32 tiles; the balanced
    placement where that launch fills whole rounds (else the XCD-grouped one)."""
    fit = round_fitting_tpcs(toa_offsets, n_chains, n_cu, wpb=1, rounds=(1,), waves_per_simd=(2,))
    tpc = fit[0] if fit else 32
    return (int(min(32, max(4, tpc))), 1, 2)


def shape_key(ds, n_chains):
    lay = ds.layout
    return (int(lay.n_psr), int(lay.n_toa), int(lay.k_coef), int(lay.k_dm), int(lay.d),
            int(n_chains))


def tune(ds, x, reps=5, candidates=None, use_cache=True):
    """Pick the fastest tuning for evaluating ``x`` on ``ds``; returns
    (tuning, log) and leaves the data set set to that tuning.  The default
    candidates are CANDIDATES plus the round-fitting chunk sizes."""
    if candidates is None:
        import torch
        n_cu = torch.cuda.get_device_properties(x.device).multi_processor_count
        fit = [(tpc, 1) for tpc in round_fitting_tpcs(ds.toa_offsets, x.shape[0], n_cu)]
        fit += [(tpc, 4) for tpc in round_fitting_tpcs(ds.toa_offsets, x.shape[0], n_cu, wpb=4,
                                                        waves_per_simd=(2, 3))]
        # (round-fitting launches also with the balanced placement, xcd 2)
        candidates = CANDIDATES + tuple((tpc, wpb, xcd) for tpc, wpb in fit for xcd in (0, 1, 2)
                                        if (tpc, wpb, xcd) not in CANDIDATES)
    key = shape_key(ds, x.shape[0])
    if use_cache and key in _cache:
        best = _cache[key]
        ds.ptafs_set_tuning(*best)
        return best, {"cached": True}
    timings = []
    ds.ptafs_set_tuning(*candidates[0])
    ds.ptafs_profile_stages(x, reps=2)              # warm up
    for cand in candidates:
        ds.ptafs_set_tuning(*cand)
        st = ds.ptafs_profile_stages(x, reps=reps)
        timings.append((st["toa"] + st["reduce"], cand))
    timings.sort()
    best = timings[0][1]
    ds.ptafs_set_tuning(*best)
    _cache[key] = best
    log = {"cached": False, "best": list(best), "best_ms": round(timings[0][0], 5),
           "worst_ms": round(timings[-1][0], 5), "n_candidates": len(timings)}
    return best, log
