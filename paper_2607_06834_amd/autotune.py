"""Autotuner for the batched TOA pass.

Times each candidate launch shape of the TOA pass (16-TOA tiles per chunk,
waves per workgroup, XCD-aware placement) on the caller's data set and chain
count with the library's event-timed stage profiler, and keeps the fastest.
The choice is cached per data-set shape (pulsar count, TOA count, basis sizes,
chain count) so that a request always runs with the same tuning, which keeps
its results reproducible: the reduction order depends only on the tuning.
"""
from __future__ import annotations

CANDIDATES = tuple((tpc, wpb, xcd) for tpc in (8, 12, 16, 24, 32, 64) for wpb in (1, 2, 4)
                   for xcd in (0, 1))

_cache: dict = {}


def shape_key(ds, n_chains):
    lay = ds.layout
    return (int(lay.n_psr), int(lay.n_toa), int(lay.k_coef), int(lay.k_dm), int(lay.d),
            int(n_chains))


def tune(ds, x, reps=5, candidates=CANDIDATES, use_cache=True):
    """Pick the fastest tuning for evaluating ``x`` on ``ds``; returns
    (tuning, log) and leaves the data set set to that tuning."""
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
