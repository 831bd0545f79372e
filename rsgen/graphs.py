"""Seeded generators of community-structured undirected graphs (inputs only).

Every generator draws from numpy's PCG64 stream (``numpy.random.default_rng``)
seeded by the caller, so the same seed yields the same arrays on every machine.
Outputs are canonical CSR graphs: symmetric, rows sorted ascending, no
self-loops, no duplicate edges, ``int64`` row offsets, ``int32`` column indices
and ``int32`` community labels.

Workload recipes (stand-ins for the paper's real social graphs, which are not
available here):

* ``sbm``: stochastic block model.  Each unordered vertex pair is an edge with
  probability ``p_in`` (same block) or ``p_out`` (different blocks).  The edge
  count of each kind is drawn from its binomial law and the edges themselves
  are a uniform random subset of the eligible pairs, which is the same
  distribution as independent Bernoulli trials.  Vertex ids and community ids
  are randomly permuted afterwards so the input is not community sorted.
* ``lfr``: an LFR-style benchmark written from the published model description
  (power-law degrees, power-law community sizes, a mixing fraction ``mu`` of
  each vertex's edges leaving its community).  Readings where the model is
  infeasible or loose are listed in the function docstring.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

_PAR_MIN = 1 << 22  # arrays shorter than this are sorted in one call


def _sort_keys(x, hi: int):
    """Ascending copy of non-negative int64 keys below ``hi`` (same result as
    ``np.sort``).  Large arrays are split into 64 value ranges by a stable
    radix pass on the top key bits and the ranges are sorted in threads."""
    x = np.asarray(x, dtype=np.int64)
    threads = max(1, min(16, os.cpu_count() or 1))
    if x.size < _PAR_MIN or threads == 1 or hi <= 64:
        return np.sort(x)
    shift = max(0, int(hi - 1).bit_length() - 6)
    bucket = (x >> shift).astype(np.uint8)
    cnt = np.bincount(bucket, minlength=64)
    order = np.argsort(bucket, kind="stable")
    del bucket
    xs = x[order]
    del order
    ends = np.cumsum(cnt)
    starts = ends - cnt
    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(lambda i: xs[starts[i]:ends[i]].sort(), range(64)))
    return xs


def _take(a, idx):
    """``a[idx]`` for a 1-D array and an index array; large gathers run in
    threads over index chunks (same result)."""
    idx = np.asarray(idx)
    threads = max(1, min(16, os.cpu_count() or 1))
    if idx.size < _PAR_MIN or threads == 1:
        return a[idx]
    out = np.empty(idx.size, dtype=a.dtype)
    bounds = np.linspace(0, idx.size, 4 * threads + 1).astype(np.int64)
    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(lambda i: np.take(a, idx[bounds[i]:bounds[i + 1]], out=out[bounds[i]:bounds[i + 1]]),
                    range(4 * threads)))
    return out


def _unique_keys(x, hi: int):
    """Sorted distinct values of non-negative int64 keys below ``hi``."""
    s = _sort_keys(x, hi)
    if s.size < 2:
        return s
    keep = np.empty(s.size, dtype=bool)
    keep[0] = True
    np.not_equal(s[1:], s[:-1], out=keep[1:])
    return s[keep]


@dataclass
class Graph:
    """Undirected simple graph in CSR form plus community labels."""

    n: int
    off: np.ndarray  # int64 [n+1]
    col: np.ndarray  # int32 [nnz], rows sorted ascending
    labels: np.ndarray  # int32 [n], non-negative community ids
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.off[-1])

    @property
    def m(self) -> int:
        return self.nnz // 2

    def edges(self):
        """Return (u, v) arrays of the undirected edges with u < v."""
        src = np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.off))
        dst = self.col.astype(np.int64)
        keep = src < dst
        return src[keep], dst[keep]


def canonical_csr(n: int, u, v, say=None):
    """Symmetrise, drop self-loops and duplicates, sort rows; return (off, col)."""
    say = say if say is not None else (lambda msg: None)
    u = np.asarray(u, dtype=np.int64).ravel()
    v = np.asarray(v, dtype=np.int64).ravel()
    keep = u != v
    u = u[keep]
    v = v[keep]
    a = np.minimum(u, v)
    b = np.maximum(u, v)
    del u, v, keep
    key = _unique_keys(a * n + b, n * n)
    del a, b
    say(f"csr: {key.size} distinct edges")
    a = key // n
    b = key - a * n
    del key
    both = _sort_keys(np.concatenate([a * n + b, b * n + a]), n * n)
    del a, b
    say(f"csr: {both.size} entries sorted")
    src = both // n
    dst = (both - src * n).astype(np.int32)
    del both
    off = np.zeros(n + 1, dtype=np.int64)
    if src.size:
        np.cumsum(np.bincount(src, minlength=n), out=off[1:])
    return off, dst


def _relabel(rng, n, off, col, labels, say=None):
    """Randomly permute vertex ids and community ids (keeps the graph isomorphic)."""
    perm = rng.permutation(n).astype(np.int64)  # old -> new
    src = np.repeat(perm, np.diff(off))
    dst = _take(perm, col)
    off2, col2 = canonical_csr(n, src, dst, say)
    lab_new = np.empty(n, dtype=np.int64)
    lab_new[perm] = labels
    uniq = np.unique(lab_new)
    cperm = rng.permutation(uniq.size)
    remap = np.empty(int(uniq.max()) + 1 if uniq.size else 0, dtype=np.int64)
    remap[uniq] = cperm
    lab2 = remap[lab_new].astype(np.int32) if n else np.zeros(0, np.int32)
    return off2, col2, lab2


def _distinct(rng, m, draw):
    """Draw exactly ``m`` distinct int64 keys, each uniformly from ``draw``'s support."""
    got = np.zeros(0, dtype=np.int64)
    while got.size < m:
        need = m - got.size
        got = np.unique(np.concatenate([got, draw(int(need * 1.05) + 16)]))
    if got.size > m:
        got = rng.permutation(got)[:m]
    return got


def sbm(block_sizes, p_in: float, p_out: float, seed: int, permute: bool = True) -> Graph:
    """Stochastic block model with the given block sizes."""
    rng = np.random.default_rng(seed)
    sizes = np.asarray(block_sizes, dtype=np.int64)
    starts = np.concatenate([[0], np.cumsum(sizes)])
    n = int(starts[-1])
    block_of = np.repeat(np.arange(sizes.size, dtype=np.int64), sizes)
    pair_in = sizes * (sizes - 1) // 2
    n_in = int(pair_in.sum())
    n_all = n * (n - 1) // 2
    n_out = n_all - n_in
    m_in = int(rng.binomial(n_in, p_in)) if n_in and p_in > 0 else 0
    m_out = int(rng.binomial(n_out, p_out)) if n_out and p_out > 0 else 0
    cdf_in = np.cumsum(pair_in) / max(n_in, 1)

    def draw_in(k):
        blk = np.searchsorted(cdf_in, rng.random(k), side="right")
        blk = np.minimum(blk, sizes.size - 1)
        s = sizes[blk]
        ok = s >= 2
        blk, s = blk[ok], s[ok]
        i = (rng.random(blk.size) * s).astype(np.int64)
        j = (rng.random(blk.size) * (s - 1)).astype(np.int64)
        j = j + (j >= i)
        gi = starts[blk] + i
        gj = starts[blk] + j
        return np.minimum(gi, gj) * n + np.maximum(gi, gj)

    def draw_out(k):
        a = rng.integers(0, n, size=k)
        b = rng.integers(0, n, size=k)
        ok = block_of[a] != block_of[b]
        a, b = a[ok], b[ok]
        return np.minimum(a, b) * n + np.maximum(a, b)

    keys = np.concatenate([
        _distinct(rng, m_in, draw_in) if m_in else np.zeros(0, np.int64),
        _distinct(rng, m_out, draw_out) if m_out else np.zeros(0, np.int64),
    ])
    u = keys // n if n else keys
    v = keys - u * n if n else keys
    off, col = canonical_csr(n, u, v)
    labels = block_of.astype(np.int32)
    if permute and n:
        off, col, labels = _relabel(rng, n, off, col, labels)
    return Graph(n, off, col, labels, meta={
        "kind": "sbm", "seed": seed, "blocks": int(sizes.size), "p_in": p_in, "p_out": p_out})


def _powerlaw_int(rng, size, lo, hi, expo):
    vals = np.arange(lo, hi + 1, dtype=np.float64)
    w = vals ** (-expo)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    idx = np.searchsorted(cdf, rng.random(size), side="right")
    return (lo + np.minimum(idx, vals.size - 1)).astype(np.int64)


def _floor_powerlaw_pmf(x0, hi, expo):
    """pmf of floor(X) for X with density ~x^-expo on [x0, hi+1)."""
    a = x0 ** (1.0 - expo)
    b = (hi + 1.0) ** (1.0 - expo)
    ks = np.arange(int(np.floor(x0)), hi + 1, dtype=np.float64)
    lo_edge = np.maximum(ks, x0)
    hi_edge = ks + 1.0
    cdf_lo = (a - lo_edge ** (1.0 - expo)) / (a - b)
    cdf_hi = (a - hi_edge ** (1.0 - expo)) / (a - b)
    return ks, cdf_hi - cdf_lo


def _solve_x0(mean_deg, hi, expo):
    """x0 such that floor(X) (X ~ x^-expo on [x0, hi+1)) has the requested mean."""
    lo_x, hi_x = 1.0, float(hi)
    for _ in range(80):
        mid = 0.5 * (lo_x + hi_x)
        ks, p = _floor_powerlaw_pmf(mid, hi, expo)
        if float((ks * p).sum()) < mean_deg:
            lo_x = mid
        else:
            hi_x = mid
    return 0.5 * (lo_x + hi_x)


def _floor_powerlaw(rng, size, x0, hi, expo):
    a = x0 ** (1.0 - expo)
    b = (hi + 1.0) ** (1.0 - expo)
    x = (a - rng.random(size) * (a - b)) ** (1.0 / (1.0 - expo))
    return np.minimum(np.floor(x), hi).astype(np.int64)


def _pair_internal(rng, stubs, comm, say=None):
    """Pair stubs uniformly at random inside each community; return edge keys (a<b)."""
    say = say if say is not None else (lambda msg: None)
    if stubs.size < 2:
        return np.zeros(0, np.int64)
    n = comm.size
    stubs = _take(stubs, rng.permutation(stubs.size))
    say(f"lfr: {stubs.size} internal stubs shuffled")
    key = _take(comm, stubs)
    if comm.size and int(comm.max()) < 65536:
        key = key.astype(np.uint16)  # the stable sort of 16-bit keys is a radix sort
    order = np.argsort(key, kind="stable")
    del key
    say("lfr: internal stubs ordered by community")
    stubs = _take(stubs, order)
    del order
    sc = _take(comm, stubs)
    gstart = np.flatnonzero(np.r_[True, sc[1:] != sc[:-1]])
    glen = np.diff(np.r_[gstart, sc.size])
    pos = np.arange(sc.size) - np.repeat(gstart, glen)
    last = np.repeat(glen, glen)
    first = np.flatnonzero((pos % 2 == 0) & (pos + 1 < last))
    a, b = stubs[first], stubs[first + 1]
    ok = a != b
    a, b = a[ok], b[ok]
    return np.minimum(a, b) * n + np.maximum(a, b)


def _pair_external(rng, stubs, comm, rounds):
    """Pair stubs uniformly across communities, redrawing same-community pairs."""
    n = comm.size
    out = []
    for _ in range(rounds):
        if stubs.size < 2:
            break
        stubs = stubs[rng.permutation(stubs.size)]
        h = stubs.size // 2
        a, b = stubs[:h], stubs[h:2 * h]
        ok = comm[a] != comm[b]
        out.append(np.minimum(a[ok], b[ok]) * n + np.maximum(a[ok], b[ok]))
        stubs = np.concatenate([a[~ok], b[~ok], stubs[2 * h:]])
    keys = np.concatenate(out) if out else np.zeros(0, np.int64)
    return keys, stubs.size


def _union_keys(keys, add, n):
    """Sorted union of edge-key sets (duplicates dropped)."""
    if add.size == 0:
        return keys
    add = _unique_keys(add, n * n)
    if keys.size == 0:
        return add
    pos = np.searchsorted(keys, add)
    pos_c = np.minimum(pos, keys.size - 1)
    new = keys[pos_c] != add
    # both sorted and disjoint: insert the new keys at their positions
    return np.insert(keys, pos[new], add[new])


def lfr(n: int, mean_deg: float, max_deg: int, mu: float, seed: int,
        tau1: float = 2.5, tau2: float = 1.5, cmin: int = 50, cmax: int = 20000,
        ext_rounds: int = 12, repair_rounds: int = 4, log=None) -> Graph:
    """LFR-style graph.

    Steps: (1) degrees i.i.d. as floor(X), X from the power law x^-tau1 on
    [x_min, max_deg+1), x_min solved so the degree law's mean is ``mean_deg``; (2) each vertex's
    external degree is mu*d rounded stochastically, the rest is internal;
    (3) community sizes i.i.d. from s^-tau2 on [cmin, cmax] until they cover n
    (the last one is trimmed); (4) each vertex joins a random community,
    chosen with probability proportional to size among communities larger than
    its internal degree (all communities if none is larger); (5) internal
    degree is capped at (realised community size - 1) and the excess becomes
    external (the only way to honour max_deg when it exceeds the largest
    community); (6) internal stubs are paired uniformly at random inside each
    community, external stubs uniformly at random across the graph with
    same-community pairs rejected and redrawn for a bounded number of rounds;
    (7) self-loops and multi-edges are removed; (8) vertex ids and community
    ids are randomly permuted.  Realised statistics go to ``meta``.  ``log``,
    if given, is called with a short message after each stage.
    """
    say = log if log is not None else (lambda msg: None)
    rng = np.random.default_rng(seed)
    x0 = _solve_x0(mean_deg, max_deg, tau1)
    deg = _floor_powerlaw(rng, n, x0, max_deg, tau1)
    k_ext = np.floor(mu * deg + rng.random(n)).astype(np.int64)
    k_in = deg - k_ext

    # community sizes
    sizes = []
    total = 0
    est = max(16, int(2 * n / max(cmin, 1)))
    while total < n:
        s = _powerlaw_int(rng, est, cmin, cmax, tau2)
        cs = np.cumsum(s) + total
        cut = int(np.searchsorted(cs, n, side="left"))
        if cut < s.size:
            take = s[: cut + 1].copy()
            take[-1] -= int(cs[cut] - n)
            sizes.append(take)
            total = n
        else:
            sizes.append(s)
            total = int(cs[-1])
    sizes = np.concatenate(sizes) if sizes else np.zeros(0, np.int64)
    sizes = sizes[sizes > 0]
    nc = sizes.size
    order = np.argsort(-sizes, kind="stable")
    sizes_desc = sizes[order]
    csum = np.cumsum(sizes_desc).astype(np.float64)
    elig = np.searchsorted(-sizes_desc, -k_in, side="left")  # communities with size > k_in
    elig = np.maximum(elig, 1)
    pick = np.searchsorted(csum, rng.random(n) * csum[elig - 1], side="right")
    pick = np.minimum(pick, elig - 1)
    comm = order[pick].astype(np.int64)
    real = np.bincount(comm, minlength=nc)
    cap = np.maximum(real[comm] - 1, 0)
    over = np.maximum(k_in - cap, 0)
    k_in = k_in - over
    k_ext = k_ext + over

    say(f"lfr: degrees and {nc} communities drawn")
    keys = _union_keys(np.zeros(0, np.int64),
                       _pair_internal(rng, np.repeat(np.arange(n, dtype=np.int64), k_in), comm, say), n)
    say(f"lfr: {keys.size} internal edges paired")
    ext_keys, left = _pair_external(rng, np.repeat(np.arange(n, dtype=np.int64), k_ext), comm, ext_rounds)
    keys = _union_keys(keys, ext_keys, n)
    say(f"lfr: {keys.size} edges after external pairing")
    # repair rounds: stubs lost to self-loops / multi-edges are paired again
    for _ in range(repair_rounds):
        a = keys // n
        b = keys - a * n
        same = _take(comm, a) == _take(comm, b)
        r_in = np.bincount(a[same], minlength=n) + np.bincount(b[same], minlength=n)
        r_ext = np.bincount(a[~same], minlength=n) + np.bincount(b[~same], minlength=n)
        del a, b, same
        def_in = np.maximum(k_in - r_in, 0)
        def_ext = np.maximum(k_ext - r_ext, 0)
        if def_in.sum() + def_ext.sum() < 2:
            break
        add = _pair_internal(rng, np.repeat(np.arange(n, dtype=np.int64), def_in), comm)
        add_e, _ = _pair_external(rng, np.repeat(np.arange(n, dtype=np.int64), def_ext), comm, ext_rounds)
        keys = _union_keys(keys, np.concatenate([add, add_e]), n)
        say(f"lfr: {keys.size} edges after a repair round")
    u = keys // n
    v = keys - u * n
    del keys
    off, col = canonical_csr(n, u, v, say)
    del u, v
    say("lfr: CSR built")
    off, col, labels = _relabel(rng, n, off, col, comm.astype(np.int32), say)
    say("lfr: ids permuted")
    g = Graph(n, off, col, labels, meta={
        "kind": "lfr", "seed": seed, "n": n, "mean_deg_target": mean_deg, "max_deg": max_deg,
        "mu_target": mu, "x_min": x0, "communities": int(nc)})
    g.meta.update(graph_stats(g))
    return g


def random_small(n: int, p: float, k: int, seed: int, label_values=None) -> Graph:
    """Erdos-Renyi G(n, p) with uniform random labels in [0, k) (tiny test graphs).

    ``label_values`` optionally maps the k labels to arbitrary non-negative ids.
    """
    rng = np.random.default_rng(seed)
    iu, ju = np.triu_indices(n, 1)
    keep = rng.random(iu.size) < p
    off, col = canonical_csr(n, iu[keep], ju[keep])
    lab = rng.integers(0, max(k, 1), size=n)
    if label_values is not None:
        lab = np.asarray(label_values, dtype=np.int64)[lab]
    return Graph(n, off, col, lab.astype(np.int32), meta={"kind": "gnp", "seed": seed})


def from_edges(n: int, edges, labels) -> Graph:
    """Build a Graph from an explicit undirected edge list."""
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    off, col = canonical_csr(n, e[:, 0], e[:, 1])
    return Graph(n, off, col, np.asarray(labels, dtype=np.int32), meta={"kind": "explicit"})


def graph_stats(g: Graph) -> dict:
    """Realised size statistics of a graph (counts only, no scoring arithmetic)."""
    deg = np.diff(g.off)
    src = np.repeat(np.arange(g.n, dtype=np.int64), deg)
    inter = int(np.count_nonzero(g.labels[src] != g.labels[g.col])) // 2 if g.n else 0
    return {
        "n_real": g.n,
        "m_real": g.m,
        "mean_deg_real": float(deg.mean()) if g.n else 0.0,
        "max_deg_real": int(deg.max()) if g.n else 0,
        "m_inter": inter,
        "mu_real": inter / g.m if g.m else 0.0,
        "communities_real": int(np.unique(g.labels).size) if g.n else 0,
    }


def cached(name: str, make, cache_dir=None, log=None) -> Graph:
    """The graph ``name`` from ``cache_dir`` if an earlier call stored it there,
    else ``make()``, stored there.  ``cache_dir`` defaults to the environment
    variable RS_GRAPH_CACHE; without one nothing is cached.  Arrays are plain
    .npy files (loaded without pickle) and the metadata is JSON."""
    import json
    cache_dir = cache_dir if cache_dir is not None else os.environ.get("RS_GRAPH_CACHE", "")
    say = log if log is not None else (lambda msg: None)
    if not cache_dir:
        return make()
    base = os.path.join(cache_dir, name)
    parts = ("off", "col", "labels")
    if all(os.path.exists(f"{base}.{p}.npy") for p in parts) and os.path.exists(f"{base}.json"):
        arr = {p: np.load(f"{base}.{p}.npy", allow_pickle=False) for p in parts}
        with open(f"{base}.json") as f:
            meta = json.load(f)
        say(f"graph {name} loaded from {cache_dir}")
        return Graph(int(arr["off"].size - 1), arr["off"], arr["col"], arr["labels"], meta=meta)
    g = make()
    os.makedirs(cache_dir, exist_ok=True)
    for p in parts:
        np.save(f"{base}.{p}.npy", getattr(g, p), allow_pickle=False)
    with open(f"{base}.json", "w") as f:
        json.dump(g.meta, f)
    say(f"graph {name} stored in {cache_dir}")
    return g


# Named workloads.  Sizes follow the benchmark configurations: a small SBM the
# oracle scores in well under a second, an LFR-style graph of one million
# vertices (~10M edges) and one of twenty million vertices (~300M edges).

def cfg_sbm_small(seed: int = 0) -> Graph:
    """SBM: n=2,000 in 20 planted communities of 100, p_in=0.05, p_out=0.001."""
    return sbm([100] * 20, 0.05, 0.001, seed)


def cfg_lfr_1m(seed: int = 0, log=None) -> Graph:
    """LFR-style: n=1e6, degree law exponent 2.5, mean 20, max 5,000, sizes
    exponent 1.5 on [50, 20,000], mixing 0.1."""
    return lfr(1_000_000, 20.0, 5000, 0.1, seed, log=log)


def cfg_lfr_20m(seed: int = 0, log=None) -> Graph:
    """LFR-style: n=2e7, mean degree 30, max 100,000, mixing 0.15 (same size law)."""
    return lfr(20_000_000, 30.0, 100_000, 0.15, seed, log=log)


def cfg_batch_graph(index: int, seed_base: int = 1000) -> Graph:
    """One graph of the batched workload (seed seed_base + index): n
    log-uniform on [200, 50,000], mean degree U[8, 40], U{5..500} communities
    (at most n/10), mixing U[0.05, 0.3]; with probability 1/2 an SBM with
    equal blocks, else LFR-style with max degree min(1,000, n/4) and community
    sizes on [m/4, 4m] around m = n / communities (the s^-1.5 law's mean on
    [a, b] is sqrt(ab) = m)."""
    seed = seed_base + index
    rng = np.random.default_rng(seed)
    n = int(round(np.exp(rng.uniform(np.log(200), np.log(50_000)))))
    mean_deg = float(rng.uniform(8.0, 40.0))
    k = int(min(rng.integers(5, 501), max(n // 10, 1)))
    mu = float(rng.uniform(0.05, 0.3))
    if rng.random() < 0.5:
        sizes = np.full(k, n // k, np.int64)
        sizes[: n % k] += 1
        s = n / k
        p_in = min(1.0, (1.0 - mu) * mean_deg / max(s - 1.0, 1.0))
        p_out = min(1.0, mu * mean_deg / max(n - s, 1.0))
        g = sbm(sizes, p_in, p_out, seed)
    else:
        m = n / k
        g = lfr(n, mean_deg, min(1000, n // 4), mu, seed, cmin=max(2, int(m / 4)), cmax=max(3, int(4 * m)))
    g.meta.update({"batch_index": index, "mean_deg_target": mean_deg, "communities_target": k, "mu_target": mu})
    return g


def _batch_one(args):
    return cfg_batch_graph(*args)


def cfg_batch(n_graphs: int = 4096, seed_base: int = 1000, workers: int = 1) -> list:
    """The batched workload's graphs 0..n_graphs-1 (in index order)."""
    jobs = [(i, seed_base) for i in range(n_graphs)]
    if workers <= 1:
        return [_batch_one(j) for j in jobs]
    import multiprocessing as mp
    with mp.get_context("spawn").Pool(workers) as pool:
        return pool.map(_batch_one, jobs, chunksize=8)


def pack_batch(graphs):
    """Disjoint union of graphs: (vertex_offsets [G+1] int64, row_offsets
    int64, col int32 with global ids, labels int32 as given per graph)."""
    vo = np.zeros(len(graphs) + 1, np.int64)
    vo[1:] = np.cumsum([g.n for g in graphs])
    eo = np.zeros(len(graphs) + 1, np.int64)
    eo[1:] = np.cumsum([g.nnz for g in graphs])
    off = np.zeros(int(vo[-1]) + 1, np.int64)
    col = np.empty(int(eo[-1]), np.int32)
    lab = np.empty(int(vo[-1]), np.int32)
    for i, g in enumerate(graphs):
        off[vo[i] + 1: vo[i + 1] + 1] = g.off[1:] + eo[i]
        col[eo[i]: eo[i + 1]] = g.col + np.int32(vo[i])
        lab[vo[i]: vo[i + 1]] = g.labels
    return vo, off, col, lab
