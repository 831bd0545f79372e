"""CPU oracle for the robust-spanner scoring pass -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never loads it, and it
shares no code with the GPU library.

``rs_oracle.c`` is the plain fp64 reference (direct entropy sums, a literal loop
over the ordered pairs of Eq. RSI); this module builds it with gcc, loads it
with ctypes, and wraps it for numpy arrays.  ``brute`` holds an independent
pure-Python enumeration used to pin the C oracle on tiny graphs.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "rs_oracle.c")
LIB = os.path.join(HERE, "librs_oracle.so")

ALG2_LITERAL = 1

_P = ctypes.c_void_p
_I64 = ctypes.c_int64


def build(extra_flags=(), out=LIB) -> str:
    """Compile the oracle with gcc (always recompiles)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
           "-std=c11", "-Wall", "-Wextra", *extra_flags, "-o", out, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return out


_lib = None


def load(path=LIB):
    global _lib
    if path == LIB and _lib is not None:
        return _lib
    if not os.path.exists(path):
        build(out=path)
    lib = ctypes.CDLL(path)
    lib.rso_validate.argtypes = [_I64, _P, _P, _P]
    lib.rso_validate.restype = ctypes.c_int
    lib.rso_weight.argtypes = [_I64, _P, _P, ctypes.c_int32, ctypes.c_uint]
    lib.rso_weight.restype = ctypes.c_double
    lib.rso_triad_term.argtypes = [ctypes.c_double] * 3
    lib.rso_triad_term.restype = ctypes.c_double
    lib.rso_rsi_from_terms.argtypes = [_I64, _I64, _P, _P, _P, ctypes.c_double]
    lib.rso_rsi_from_terms.restype = ctypes.c_double
    lib.rso_score.argtypes = [_I64, _P, _P, _P, _P, _I64, ctypes.c_uint, ctypes.c_int] + [_P] * 16
    lib.rso_score.restype = ctypes.c_int
    lib.rso_triads.argtypes = [_I64, _P, _P, _P, _I64, _I64, _P, _P, _P]
    lib.rso_triads.restype = _I64
    lib.rso_topk.argtypes = [_I64, _P, _P, _I64, _P, _P, _P]
    lib.rso_topk.restype = ctypes.c_int
    if path == LIB:
        _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _graph_arrays(g):
    off = np.ascontiguousarray(g.off, dtype=np.int64)
    col = np.ascontiguousarray(g.col, dtype=np.int32)
    lab = np.ascontiguousarray(g.labels, dtype=np.int32)
    return off, col, lab


def validate(g, lib=None) -> int:
    lib = lib or load()
    off, col, lab = _graph_arrays(g)
    return lib.rso_validate(g.n, _ptr(off), _ptr(col), _ptr(lab))


def weight(counts: dict, ref: int, flags: int = 0, lib=None) -> float:
    """w for the neighbour multiset ``counts`` {community: frequency} toward ``ref``."""
    lib = lib or load()
    comms = np.array(list(counts.keys()), dtype=np.int32)
    cnts = np.array(list(counts.values()), dtype=np.int64)
    return lib.rso_weight(comms.size, _ptr(comms), _ptr(cnts), int(ref), flags)


def triad_term(a: float, b: float, c: float, lib=None) -> float:
    lib = lib or load()
    return lib.rso_triad_term(a, b, c)


def rsi_from_terms(d: int, triples, omega_max: float, lib=None) -> float:
    lib = lib or load()
    t = np.asarray(triples, dtype=np.float64).reshape(-1, 3)
    a, b, c = (np.ascontiguousarray(t[:, i]) for i in range(3))
    return lib.rso_rsi_from_terms(d, t.shape[0], _ptr(a), _ptr(b), _ptr(c), omega_max)


def score(g, subset=None, flags: int = 0, nthreads: int = 0, rows: bool = False, lib=None) -> dict:
    """Run the oracle; returns a dict of numpy arrays and scalars."""
    lib = lib or load()
    off, col, lab = _graph_arrays(g)
    n = g.n
    nn = max(n, 1)
    out = {
        "R": np.zeros(nn), "raw": np.zeros(nn), "border": np.zeros(nn, np.uint8),
        "ell": np.zeros(nn, np.int32), "dprime": np.zeros(nn, np.int32),
        "tI": np.zeros(nn, np.int64), "tII": np.zeros(nn, np.int64),
        "tII_closed": np.zeros(nn, np.int64), "w_own": np.zeros(nn),
    }
    if rows:
        out["hist_off"] = np.zeros(n + 1, np.int64)
        cap = max(int(off[-1]), 1)
        out["hist_comm"] = np.zeros(cap, np.int32)
        out["hist_cnt"] = np.zeros(cap, np.int64)
        out["hist_w"] = np.zeros(cap)
    sub = None if subset is None else np.ascontiguousarray(subset, dtype=np.int64)
    omax = ctypes.c_double(0.0)
    nb = ctypes.c_int64(0)
    mx = ctypes.c_int64(0)
    rc = lib.rso_score(
        n, _ptr(off), _ptr(col), _ptr(lab), _ptr(sub), 0 if sub is None else sub.size,
        flags, nthreads,
        _ptr(out["R"]), _ptr(out["raw"]), _ptr(out["border"]), _ptr(out["ell"]),
        _ptr(out["dprime"]), _ptr(out["tI"]), _ptr(out["tII"]), _ptr(out["tII_closed"]),
        _ptr(out["w_own"]), _ptr(out.get("hist_off")), _ptr(out.get("hist_comm")),
        _ptr(out.get("hist_cnt")), _ptr(out.get("hist_w")),
        ctypes.byref(omax), ctypes.byref(nb), ctypes.byref(mx))
    if rc != 0:
        raise RuntimeError(f"oracle rso_score failed with code {rc}")
    for k in ("R", "raw", "border", "ell", "dprime", "tI", "tII", "tII_closed", "w_own"):
        out[k] = out[k][:n]
    if rows:
        tot = int(out["hist_off"][-1])
        for k in ("hist_comm", "hist_cnt", "hist_w"):
            out[k] = out[k][:tot]
    out["omega_max"] = omax.value
    out["n_border"] = nb.value
    out["m_inter"] = mx.value
    return out


def topk(R, K: int, alive=None, lib=None):
    lib = lib or load()
    R = np.ascontiguousarray(R, dtype=np.float64)
    n = R.size
    al = None if alive is None else np.ascontiguousarray(alive, dtype=np.uint8)
    ids = np.zeros(max(K, 1), np.int32)
    sc = np.zeros(max(K, 1))
    cnt = ctypes.c_int64(0)
    rc = lib.rso_topk(n, _ptr(R), _ptr(al), K, _ptr(ids), _ptr(sc), ctypes.byref(cnt))
    if rc != 0:
        raise RuntimeError(f"oracle rso_topk failed with code {rc}")
    return ids[: cnt.value].copy(), sc[: cnt.value].copy()


def triads(g, u: int, lib=None):
    """Every triad counted at u as (w, v, kind); kind 1 type-I, 2 open type-II, 3 closed type-II."""
    lib = lib or load()
    off, col, lab = _graph_arrays(g)
    k = lib.rso_triads(g.n, _ptr(off), _ptr(col), _ptr(lab), u, 0, None, None, None)
    w = np.zeros(max(k, 1), np.int64)
    v = np.zeros(max(k, 1), np.int64)
    kind = np.zeros(max(k, 1), np.int32)
    lib.rso_triads(g.n, _ptr(off), _ptr(col), _ptr(lab), u, k, _ptr(w), _ptr(v), _ptr(kind))
    return [(int(w[i]), int(v[i]), int(kind[i])) for i in range(k)]


class _Graph:
    """Plain container (n, off, col, labels) for graphs built here."""

    def __init__(self, n, off, col, labels):
        self.n, self.off, self.col, self.labels = int(n), off, col, labels


def target_communities(labels, k_c: int):
    """Target-community mode (Section VI-A, the considered communities;
    Section VII-C, the k largest by member count): the labels of the k_c
    communities with the most members, ties broken by the smaller label."""
    labs, counts = np.unique(np.asarray(labels), return_counts=True)
    order = np.lexsort((labs, -counts))
    return labs[order[:k_c]]


def restrict_to_targets(g, k_c: int):
    """(graph, keep): the subgraph induced by the target communities' members
    (every edge with an endpoint outside them dropped, those vertices left
    isolated with their labels) and the mask of the kept vertices.  Counts,
    T = sum of f over the considered communities, degrees and triads of the
    scoring pass then involve the targets only."""
    keep = np.isin(g.labels, target_communities(g.labels, k_c))
    src = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.off))
    dst = np.asarray(g.col, dtype=np.int64)
    ok = keep[src] & keep[dst]
    off = np.zeros(g.n + 1, np.int64)
    np.cumsum(np.bincount(src[ok], minlength=g.n), out=off[1:])
    return _Graph(g.n, off, dst[ok].astype(np.int32), np.asarray(g.labels, dtype=np.int32)), keep


def reachable_communities(g, sources, alive=None):
    """|zeta(v)| after a disruption, for the absolute AWCC of the robustness
    experiments (Section VII-B): for each source, a breadth-first search over
    the current graph, and the number of distinct communities among the
    vertices it reaches other than the source itself.  A removed source
    (alive False) reaches nothing."""
    from collections import deque
    off = np.asarray(g.off, dtype=np.int64)
    col = np.asarray(g.col, dtype=np.int64)
    lab = np.asarray(g.labels)
    out = np.zeros(len(sources), np.int64)
    for i, s in enumerate(sources):
        s = int(s)
        if alive is not None and not alive[s]:
            continue
        seen = {s}
        queue = deque([s])
        comms = set()
        while queue:
            x = queue.popleft()
            for e in range(off[x], off[x + 1]):
                y = int(col[e])
                if y not in seen:
                    seen.add(y)
                    comms.add(int(lab[y]))
                    queue.append(y)
        # the source's own community counts when another member is reached
        out[i] = len(comms)
    return out
