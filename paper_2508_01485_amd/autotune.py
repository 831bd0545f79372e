"""Autotuner of the scoring pass's static schedule (tile sizes and degree bins).

The pass cuts a graph's vertices into row tiles, score tiles and hubs at load
time (``rs_tiling`` in ``include/rs.h``); which cut-offs run fastest depends on
the degree distribution.  ``tune`` keys a graph (or a batch of graphs) by a
signature of its degree histogram, looks the signature up in a cache file,
and on a miss searches the cut-offs one at a time (coordinate descent:
every value of one cut-off with the others fixed, keeping the fastest, over
all cut-offs, twice) with ``rs_autotune``, which re-cuts the schedule and
times passes on the device.  The winner is stored in the cache and left on
the graph.

The search's timing, re-cutting and passes are native (``rs_autotune``);
this module holds the signature, the search order and the cache.
"""
from __future__ import annotations

import hashlib
import json
import os
import time

import numpy as np

DEFAULT = {"row_entries": 2048, "row_vertices": 512, "score_pairs": 256, "score_vertices": 256, "hub_list": 1024}
SPACE = {
    "row_entries": (512, 1024, 2048),
    "row_vertices": (128, 256, 512),
    "score_pairs": (64, 128, 256),
    "score_vertices": (64, 128, 256),
    "hub_list": (256, 512, 1024),
}
ORDER = ("row_entries", "score_pairs", "row_vertices", "score_vertices", "hub_list")


def default_cache_path() -> str:
    return os.environ.get("RS_TUNE_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "paper_2508_01485_amd", "tiling.json")


def degree_signature(row_offsets, n_graphs: int = 1) -> str:
    """Signature of a degree distribution: the share of vertices in each
    power-of-two degree bin (rounded to 1/100), the mean degree (rounded to a
    tenth of a power of two) and the power-of-two sizes of the vertex count
    and the graph count.  Independent of vertex order and ids."""
    off = np.asarray(row_offsets, dtype=np.int64)
    n = off.size - 1
    deg = np.diff(off)
    bins = np.bincount(np.floor(np.log2(deg + 1)).astype(np.int64), minlength=24)[:24] if n else np.zeros(24)
    share = np.round(bins / max(n, 1), 2).tolist()
    mean = float(deg.mean()) if n else 0.0
    key = {"share": share, "log2_mean_deg": round(float(np.log2(mean + 1)), 1),
           "log2_n": int(np.log2(n + 1)), "log2_graphs": int(np.log2(max(n_graphs, 1)))}
    return hashlib.sha256(json.dumps(key, sort_keys=True).encode()).hexdigest()[:16]


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path, cache):
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def search(g, reps: int = 3, rounds: int = 2):
    """Coordinate descent over SPACE from the graph's current cut-offs;
    returns (best cut-offs, best pass ms, number of candidates timed)."""
    import paper_2508_01485_amd as rs
    cur = rs.rs_get_tiling(g)
    best_ms, timed = None, 0
    for _ in range(rounds):
        changed = False
        for name in ORDER:
            cands = [dict(cur, **{name: v}) for v in SPACE[name]]
            if cur not in cands:
                cands.append(dict(cur))
            i, ms = rs.rs_autotune(g, cands, reps)
            timed += len(cands)
            if cands[i] != cur:
                changed = True
            cur, best_ms = cands[i], float(ms[i])
        if not changed:
            break
    return cur, best_ms, timed


def tune(g, row_offsets, n_graphs: int = 1, cache_path: str | None = None, reps: int = 3):
    """Cut-offs for the graph g (loaded from row_offsets): from the cache when
    its degree signature is known, else by search (then cached).  The graph
    keeps the chosen cut-offs and must be scored again."""
    import paper_2508_01485_amd as rs
    path = cache_path or default_cache_path()
    sig = degree_signature(row_offsets, n_graphs)
    cache = _load(path)
    t0 = time.perf_counter()
    if sig in cache:
        tiling = cache[sig]["tiling"]
        rs.rs_set_tiling(g, tiling)
        return {"signature": sig, "tiling": tiling, "cached": True, "seconds": time.perf_counter() - t0}
    tiling, ms, timed = search(g, reps)
    cache[sig] = {"tiling": tiling, "pass_ms": ms, "candidates_timed": timed}
    _store(path, cache)
    return {"signature": sig, "tiling": tiling, "cached": False, "pass_ms": ms, "candidates_timed": timed,
            "seconds": time.perf_counter() - t0}
