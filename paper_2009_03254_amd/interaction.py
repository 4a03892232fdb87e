"""Interaction benchmarks of the paper's evaluation (Sec. 4.6.1,
tab:mc_benchmark_table): sequences of isovalues extracted one after another
on one volume, so that the block cache carries over from surface to surface.

* Random: isovalues drawn uniformly (seeded) over a value range, the
  cache-unfriendly exploratory case;
* Sweep Up / Sweep Down: evenly spaced isovalues over the same range in
  ascending / descending order, the cache-friendly cases.

As in the paper, the first extraction of a sequence is discarded from the
averages.  Each extraction is the full path (cull, cache update, decode of the
new blocks, marching cubes, count readback); the driver only issues the calls
and collects the library's per-call statistics.
"""
from __future__ import annotations

import time

import numpy as np

KINDS = ("random", "sweep_up", "sweep_down")

# indices of bcmc_stats.stage_ms
STAGES = {"cull": 0, "cache_update": 1, "decode": 2, "mc_count": 3, "emit": 5}


def isovalues(kind, lo, hi, n=100, seed=0):
    """The n isovalues of a benchmark over [lo, hi] (float32 values)."""
    if kind == "random":
        v = np.random.default_rng(seed).uniform(lo, hi, n)
    elif kind == "sweep_up":
        v = np.linspace(lo, hi, n)
    elif kind == "sweep_down":
        v = np.linspace(hi, lo, n)
    else:
        raise ValueError(f"unknown benchmark {kind!r}")
    return v.astype(np.float32)


def run(vol, isos, out, profile=False, on_call=None):
    """Extract every isovalue of `isos` in order on `vol` (its cache carries
    over) into the preallocated buffer `out`; returns one record per call:
    host time (ms, count readback included) and the library's statistics.
    With profile, HIP events time every stage (a few microseconds each)."""
    from . import BcmcError, lib
    vol.set_profiling(bool(profile))
    recs = []
    try:
        for k, iso in enumerate(isos):
            t0 = time.perf_counter()
            rc, T = vol.extract_into(float(iso), out)
            ms = (time.perf_counter() - t0) * 1e3
            if rc != 0:
                raise BcmcError(rc, lib().bcmc_last_error().decode())
            st = vol.stats()
            recs.append({"iso": float(iso), "ms": ms, **st})
            if on_call is not None:
                on_call(k, st)
    finally:
        vol.set_profiling(False)
    return recs


def summarise(recs, n_blocks, discard_first=True):
    """Averages over a sequence's calls (the first discarded): extraction
    time per isovalue, hit rate, share of the volume's blocks decoded per
    surface, triangles; and, for profiled calls, each stage's share of the
    summed stage times."""
    r = recs[1:] if discard_first and len(recs) > 1 else recs
    out = {
        "n_isovalues": len(r),
        "mean_ms": float(np.mean([x["ms"] for x in r])),
        "hit_rate": float(np.mean([x["hit_rate"] for x in r])),
        "decoded_per_surface": float(np.mean([x["n_new"] for x in r])) / n_blocks,
        "active_per_surface": float(np.mean([x["n_active"] for x in r])) / n_blocks,
        "mean_triangles": float(np.mean([x["n_triangles"] for x in r])),
        "max_slots": int(max(x["n_slots"] for x in r)),
    }
    tot = {k: float(np.sum([x["stage_ms"][i] for x in r])) for k, i in STAGES.items()}
    s = sum(tot.values())
    if s > 0:
        out["stage_share"] = {k: round(v / s, 4) for k, v in tot.items()}
        out["stage_mean_ms"] = {k: round(v / len(r), 4) for k, v in tot.items()}
    return out
