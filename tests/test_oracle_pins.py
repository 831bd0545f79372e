"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these compare the oracle with itself: each checks a printed value of
the paper, a closed form, an identity, a special case, an invariant, or an
independent brute force.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import brute
from rsgen import cfg_sbm_small, from_edges, random_small

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "worked_example.json")))


# ---------------------------------------------------------------- printed --

def test_worked_example_weight(oracle_lib):
    ex = GOLD["weight_example"]
    counts = {int(k): v for k, v in ex["counts"].items()}
    w = oracle.weight(counts, ex["reference"], lib=oracle_lib)
    assert w == pytest.approx(ex["omega_unnormalized"], abs=1e-15)
    # |L| = 2 communities remain after removing the reference, so H = w / 2
    assert w / 2 == pytest.approx(ex["H"], abs=1e-15)


def test_worked_example_normalization(oracle_lib):
    ex = GOLD["normalization_example"]
    # Three equally frequent communities other than the reference: H = log2 3, |L| = 3.
    wmax = oracle.weight({2: 1, 3: 1, 4: 1}, 1, lib=oracle_lib)
    assert abs(wmax - ex["omega_max_printed"]) < ex["print_unit"]["omega_max"]
    w_u = oracle.weight({1: 1, 2: 1, 3: 1}, 1, lib=oracle_lib)
    assert abs(w_u / wmax - ex["normalized_printed"]) < ex["print_unit"]["normalized"]
    # Algorithm 2's uniform L_all - 1 would give 2 log2 3 = 3.17 here, far from the print
    assert abs(oracle.weight({2: 1, 3: 1, 4: 1}, 1, flags=oracle.ALG2_LITERAL, lib=oracle_lib)
               - ex["omega_max_printed"]) > 1.0


def test_worked_example_rsi(oracle_lib):
    ex = GOLD["rsi_example"]
    r = oracle.rsi_from_terms(ex["degree"], ex["normalized_triads"], 1.0, lib=oracle_lib)
    tol = ex["print_unit"]
    assert abs(r - ex["R_printed"]) < tol
    # the alternatives a plausible slip would give are all outside the printed value
    t = [oracle.triad_term(*x, lib=oracle_lib) for x in ex["normalized_triads"]]
    assert abs(sum(t) / 9 - ex["R_printed"]) > tol          # d^2
    assert abs(sum(t[:2]) / 6 - ex["R_printed"]) > tol      # one orientation only
    prod = [a * b * c for a, b, c in ex["normalized_triads"]]
    assert abs(sum(prod) / 6 - ex["R_printed"]) > tol      # no cube root


# ------------------------------------------------------------ closed forms --

def test_k4_four_communities_closed_form(oracle_lib):
    """K4 with four distinct labels: every neighbour-community weight is 2 (H=1,
    |L|=2), every own weight 3 log2 3, w_max = 3 log2 3; six ordered type-I pairs
    of term cbrt(8) = 2 each, so R = 12 / (w_max * 3 * 2) = 2 / (3 log2 3)."""
    g = from_edges(4, [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)], [7, 1, 5, 3])
    o = oracle.score(g, rows=True, lib=oracle_lib)
    wmax = 3 * math.log2(3)
    assert o["omega_max"] == pytest.approx(wmax, rel=1e-15)
    np.testing.assert_allclose(o["R"], 2 / wmax, rtol=1e-14)
    np.testing.assert_allclose(o["raw"], 2.0, rtol=1e-14)
    assert list(o["tI"]) == [6] * 4 and list(o["tII"]) == [0] * 4
    np.testing.assert_allclose(o["hist_w"], 2.0, rtol=1e-15)
    np.testing.assert_allclose(o["w_own"], wmax, rtol=1e-15)


def test_entropy_two_to_one(oracle_lib):
    """{A:3, B:1, C:2} toward A: p = (1/3, 2/3), H = log2 3 - 2/3, w = 2H."""
    h = math.log2(3) - 2.0 / 3.0
    assert oracle.weight({0: 3, 1: 1, 2: 2}, 0, lib=oracle_lib) == pytest.approx(2 * h, rel=1e-15)


def test_entropy_uniform_and_single(oracle_lib):
    for k in range(1, 12):
        counts = {c: 5 for c in range(k)}
        # reference absent: H = log2 k, |L| = k
        assert oracle.weight(counts, 99, lib=oracle_lib) == pytest.approx(k * math.log2(k), rel=1e-14, abs=0)
        # reference present: H = log2(k-1), |L| = k-1
        exp = (k - 1) * math.log2(k - 1) if k > 1 else 0.0
        assert oracle.weight(counts, 0, lib=oracle_lib) == pytest.approx(exp, rel=1e-14, abs=0)
    # a single remaining community carries no diversity: exactly zero
    assert oracle.weight({0: 4, 1: 9}, 0, lib=oracle_lib) == 0.0


def _h_optimal(counts, ref):
    """Eq. H_optimal, written out: H(L_i) = -(1/(T-f_i)) (X - T log2(T-f_i) - f_i log2(f_i/(T-f_i)))."""
    f = np.array([c for c in counts.values() if c > 0], dtype=np.float64)
    T = f.sum()
    X = float((f * np.log2(f)).sum())
    fi = float(counts.get(ref, 0))
    Y = T - fi
    if Y <= 0:
        return 0.0
    last = fi * math.log2(fi / Y) if fi > 0 else 0.0
    return -(X - T * math.log2(Y) - last) / Y


def test_eq_h_optimal_identity(oracle_lib):
    """The shared-term closed form equals the direct entropy sum."""
    rng = np.random.default_rng(1)
    for _ in range(2000):
        k = int(rng.integers(1, 12))
        counts = {int(c): int(rng.integers(1, 200)) for c in rng.choice(50, k, replace=False)}
        ref = int(rng.choice(list(counts))) if rng.random() < 0.7 else 1000
        L = len([c for c in counts if c != ref])
        w = oracle.weight(counts, ref, lib=oracle_lib)
        exp = _h_optimal(counts, ref) * L if L >= 2 else 0.0
        assert w == pytest.approx(exp, rel=1e-12, abs=1e-12)


# ---------------------------------------------------------- special cases --

def test_at_most_two_labels_scores_zero(oracle_lib):
    for s in range(20):
        g = random_small(14, 0.4, 2, s)
        o = oracle.score(g, lib=oracle_lib)
        assert o["omega_max"] == 0.0
        assert np.all(o["R"] == 0.0)


def test_non_border_vertex_scores_zero(oracle_lib):
    for s in range(30):
        g = random_small(14, 0.35, 4, 100 + s)
        o = oracle.score(g, lib=oracle_lib)
        nb = o["border"] == 0
        assert np.all(o["R"][nb] == 0.0)
        assert np.all(o["tI"][nb] == 0) and np.all(o["tII"][nb] == 0)


def test_single_foreign_community_neighbourhood(oracle_lib):
    """u whose neighbours all lie in one foreign community: u's weights are all
    zero (|L| <= 1) and it has no type-I triad."""
    # u=0 in community 0; neighbours 1,2,3 in community 1; they connect onward.
    edges = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 4), (2, 5), (3, 6), (4, 5), (5, 6), (6, 7), (3, 7)]
    labels = [0, 1, 1, 1, 0, 2, 0, 3]
    g = from_edges(8, edges, labels)
    o = oracle.score(g, rows=True, lib=oracle_lib)
    lo, hi = o["hist_off"][0], o["hist_off"][1]
    assert o["w_own"][0] == 0.0 and np.all(o["hist_w"][lo:hi] == 0.0)
    assert o["tI"][0] == 0
    # R(0) comes only from type-II triads (v in community 0 reached through 1,2,3)
    assert o["tII"][0] > 0


def test_degree_one_and_isolated(oracle_lib):
    # vertex 3 has degree 1 with a type-II triad available; vertex 4 isolated
    edges = [(0, 1), (1, 2), (0, 2), (3, 1)]
    labels = [0, 1, 2, 0, 1]
    g = from_edges(5, edges, labels)
    o = oracle.score(g, lib=oracle_lib)
    assert o["R"][3] == 0.0 and o["tII"][3] == 1
    assert o["R"][4] == 0.0 and o["border"][4] == 0


def test_empty_graphs(oracle_lib):
    g = from_edges(0, np.zeros((0, 2)), [])
    o = oracle.score(g, lib=oracle_lib)
    assert o["R"].size == 0 and o["omega_max"] == 0.0
    g = from_edges(6, np.zeros((0, 2)), [0, 1, 2, 3, 4, 5])
    o = oracle.score(g, lib=oracle_lib)
    assert np.all(o["R"] == 0) and o["n_border"] == 0


# -------------------------------------------------------------- invariants --

def test_community_relabelling_invariance(oracle_lib):
    rng = np.random.default_rng(7)
    for s in range(40):
        g = random_small(15, 0.3, 5, 200 + s)
        o1 = oracle.score(g, lib=oracle_lib)
        perm = rng.permutation(5) * 1000 + rng.integers(0, 999, 5)  # arbitrary new ids
        g2 = from_edges(g.n, np.stack(g.edges(), 1), perm[g.labels])
        o2 = oracle.score(g2, lib=oracle_lib)
        for k in ("tI", "tII", "ell", "dprime", "border"):
            assert np.array_equal(o1[k], o2[k])
        np.testing.assert_allclose(o2["R"], o1["R"], rtol=1e-12, atol=0)


def test_vertex_relabelling_equivariance(oracle_lib):
    rng = np.random.default_rng(8)
    for s in range(40):
        g = random_small(15, 0.3, 4, 300 + s)
        o1 = oracle.score(g, lib=oracle_lib)
        p = rng.permutation(g.n)
        u, v = g.edges()
        lab2 = np.empty_like(g.labels)
        lab2[p] = g.labels
        g2 = from_edges(g.n, np.stack([p[u], p[v]], 1), lab2)
        o2 = oracle.score(g2, lib=oracle_lib)
        assert np.array_equal(o2["tI"][p], o1["tI"]) and np.array_equal(o2["tII"][p], o1["tII"])
        np.testing.assert_allclose(o2["R"][p], o1["R"], rtol=1e-12, atol=0)


def test_omega_max_unchanged_without_border_restriction(oracle_lib):
    """Non-border vertices carry only zero weights, so the max over every vertex
    equals the max over border vertices (the V_b restriction changes nothing)."""
    for s in range(30):
        g = random_small(14, 0.3, 4, 400 + s)
        o = oracle.score(g, rows=True, lib=oracle_lib)
        allmax = max([0.0] + list(o["w_own"]) + list(o["hist_w"]))
        assert allmax == o["omega_max"]


def test_lemmas_1_to_3(oracle_lib):
    """Lemma 1: w_v(u) depends on v and C(u) only; Lemma 3: at most eta_v distinct
    weights leave v (one per community of N(v) plus its own)."""
    for s in range(20):
        g = random_small(13, 0.4, 4, 500 + s)
        adj = brute.adjacency(g)
        C = [int(c) for c in g.labels]
        for v in range(g.n):
            ws = {}
            for u in range(g.n):
                if u == v:
                    continue
                w = brute.omega(adj, C, C[u], v)
                if C[u] in ws:
                    assert ws[C[u]] == w  # Lemma 1
                ws[C[u]] = w
            o = oracle.score(g, rows=True, lib=oracle_lib)
            lo, hi = o["hist_off"][v], o["hist_off"][v + 1]
            eta = len(set(o["hist_comm"][lo:hi]) | {C[v]})
            relevant = {c: ws[c] for c in ws if c in set(o["hist_comm"][lo:hi]) | {C[v]}}
            assert len(set(relevant.values())) <= eta  # Lemma 3


# ------------------------------------------------------------- brute force --

def test_brute_force_agrees(oracle_lib):
    """>= 1000 random tiny graphs: the C oracle equals an independent O(n^3)
    enumeration with explicit multisets."""
    worst = 0.0
    for s in range(1000):
        rng = np.random.default_rng(10_000 + s)
        n = int(rng.integers(1, 13))
        k = int(rng.integers(1, 7))
        g = random_small(n, float(rng.uniform(0.1, 0.9)), k, 10_000 + s)
        o = oracle.score(g, lib=oracle_lib)
        R, tI, tII, wmax = brute.scores(g)
        assert list(o["tI"]) == tI and list(o["tII"]) == tII, s
        assert o["omega_max"] == pytest.approx(wmax, rel=1e-13, abs=0), s
        for a, b in zip(o["R"], R):
            assert (a == 0.0) == (b == 0.0), s
            if b:
                worst = max(worst, abs(a - b) / b)
    assert worst <= 1e-12


def _factorized_scores(g, o):
    """The per-(vertex, community) factorisation of Eq. RSI used by the GPU design:
    d(d-1) R(u) w_max = sum_{w in N'(u)} [ w_w(Cu)^(2/3) (S_w(Cu) - a_u)
                                         + w_w(Cu)^(1/3) sum_{v in N'(u) & N'(w)} cbrt(w_v(Cu) w_w(Cv)) ]
    with a_x = cbrt(w_x(C(x))) and S_w(c) = sum of a_v over v in N(w), C(v) = c."""
    C = g.labels
    rows = {}
    for v in range(g.n):
        lo, hi = o["hist_off"][v], o["hist_off"][v + 1]
        rows[v] = dict(zip(o["hist_comm"][lo:hi].tolist(), o["hist_w"][lo:hi].tolist()))

    def wt(x, c):
        return o["w_own"][x] if c == C[x] else rows[x][c]

    nbr = [set(g.col[g.off[v]:g.off[v + 1]].tolist()) for v in range(g.n)]
    fn = [{x for x in nbr[v] if C[x] != C[v]} for v in range(g.n)]
    a = np.cbrt(o["w_own"])
    R = np.zeros(g.n)
    for u in range(g.n):
        acc = 0.0
        for w in fn[u]:
            W = wt(w, C[u])
            S = sum(a[v] for v in nbr[w] if C[v] == C[u])
            acc += np.cbrt(W) ** 2 * (S - a[u])
            for v in fn[u] & fn[w]:
                acc += np.cbrt(W) * np.cbrt(wt(v, C[u]) * wt(w, C[v]))
        d = len(nbr[u])
        if d >= 2 and o["omega_max"] > 0:
            R[u] = acc / o["omega_max"] / (d * (d - 1))
    return R


def test_factorized_form_equals_triple_loop(oracle_lib):
    for s in range(300):
        rng = np.random.default_rng(20_000 + s)
        g = random_small(int(rng.integers(2, 15)), float(rng.uniform(0.15, 0.8)),
                         int(rng.integers(2, 7)), 20_000 + s)
        o = oracle.score(g, rows=True, lib=oracle_lib)
        np.testing.assert_allclose(_factorized_scores(g, o), o["R"], rtol=1e-12, atol=1e-15)


def _reaches(adj_edges, src, dst, allowed):
    """BFS from src to dst over ``adj_edges`` restricted to vertices in ``allowed``."""
    seen = {src}
    stack = [src]
    while stack:
        x = stack.pop()
        if x == dst:
            return True
        for y in adj_edges.get(x, ()):
            if y in allowed and y not in seen:
                seen.add(y)
                stack.append(y)
    return False


def test_bfs_robustness_of_counted_triads(oracle_lib):
    """Information flow in a triad (Section IV-A): after removing any single
    real edge of a counted triad (u, w, v), community C(w) still reaches u --
    directly over (w, u), or over w -> v and then v's path to u (a real edge for
    type-I, a path inside C(u) for type-II).  Graphs have internally connected
    communities; every counted triad of every vertex is checked."""
    checked = 0
    for s in range(60):
        rng = np.random.default_rng(30_000 + s)
        n, k = 14, int(rng.integers(2, 5))
        lab = rng.integers(0, k, n)
        edges = set()
        for c in range(k):  # a spanning path inside every community
            mem = np.flatnonzero(lab == c)
            for a, b in zip(mem[:-1], mem[1:]):
                edges.add((int(a), int(b)))
        iu, ju = np.triu_indices(n, 1)
        for a, b in zip(iu, ju):
            if rng.random() < 0.25:
                edges.add((int(a), int(b)))
        g = from_edges(n, sorted(edges), lab)
        adj = brute.adjacency(g)
        for u in range(n):
            for w, v, kind in oracle.triads(g, u, lib=oracle_lib):
                real = [(u, w), (w, v)] + ([(u, v)] if kind in (1, 3) else [])
                cu = {x for x in range(n) if lab[x] == lab[u]}
                for e in real:
                    sub = {x: set(adj[x]) for x in range(n)}
                    sub[e[0]].discard(e[1])
                    sub[e[1]].discard(e[0])
                    # the triad's own route: w, v and (type-II) C(u)'s members
                    allowed = {u, w, v} | (cu if kind in (2, 3) else set())
                    assert _reaches(sub, w, u, allowed), (s, u, w, v, kind, e)
                    checked += 1
    assert checked > 500


# ---------------------------------------------------------------- top-k ----

def test_topk_ties_and_bounds(oracle_lib):
    R = np.array([0.5, 0.7, 0.5, 0.0, 0.7, 0.1])
    ids, sc = oracle.topk(R, 4, lib=oracle_lib)
    assert list(ids) == [1, 4, 0, 2]
    ids, _ = oracle.topk(R, 100, lib=oracle_lib)
    assert list(ids) == [1, 4, 0, 2, 5, 3]
    alive = np.array([1, 0, 1, 1, 1, 1], np.uint8)
    ids, _ = oracle.topk(R, 3, alive=alive, lib=oracle_lib)
    assert list(ids) == [4, 0, 2]


# ------------------------------------------------------------- statistics --

def test_lemma4_border_fraction_sbm():
    """Lemma 4 on the planted SBM (20 blocks of 100, p_out = 0.001): a vertex is
    a border vertex with probability 1 - (1 - p_out)^(n - n_c); the realised
    fraction must lie within 4 sigma, and inside Lemma 4's exponential bounds
    widened by the same 4 sigma."""
    g = cfg_sbm_small(0)
    o = oracle.score(g)
    frac = o["n_border"] / g.n
    p = 1 - (1 - 0.001) ** (2000 - 100)
    sigma = math.sqrt(p * (1 - p) / g.n)
    assert abs(frac - p) <= 4 * sigma
    lo = 1 - math.exp(-(2000 - 100) * 0.001)
    assert lo - 4 * sigma <= frac <= lo + 4 * sigma


# -------------------------------------------------------------- validation --

@pytest.mark.parametrize("case", ["asym", "unsorted", "dup", "self", "neglabel", "range", "offsets"])
def test_validate_rejects(case, oracle_lib):
    """Each case breaks exactly one property of a simple undirected graph."""
    from rsgen.graphs import Graph
    # path 0-1-2-3 plus edge 0-2: rows 0:[1,2] 1:[0,2] 2:[0,1,3] 3:[2]
    off = np.array([0, 2, 4, 7, 8], np.int64)
    col = np.array([1, 2, 0, 2, 0, 1, 3, 2], np.int32)
    lab = np.array([0, 1, 0, 1], np.int32)
    good = Graph(4, off.copy(), col.copy(), lab.copy())
    if case == "asym":
        col[7] = 1                      # 3->1 without 1->3
    elif case == "unsorted":
        col[4], col[5] = col[5], col[4]  # row 2 becomes [1,0,3]
    elif case == "dup":
        col[1] = 1                      # row 0 becomes [1,1]
    elif case == "self":               # a symmetric self-loop and nothing else wrong
        off = np.array([0, 3, 5, 8, 9], np.int64)
        col = np.array([0, 1, 2, 0, 2, 0, 1, 3, 2], np.int32)
    elif case == "neglabel":
        lab[3] = -1
    elif case == "range":
        col[7] = 9
    elif case == "offsets":
        off[2], off[1] = off[1], off[2]
    assert oracle.validate(Graph(4, off, col, lab), lib=oracle_lib) == 2
    assert oracle.validate(good, lib=oracle_lib) == 0


def test_triad_kinds_on_a_hand_built_graph(oracle_lib):
    """The oracle's triad labels and its closed type-II count (Section II,
    the triad types; reading A7) on a graph small enough to list by hand:
    u and v1, v2 in community A, w in B, x in C; edges u-w, u-v1, u-x, w-v1,
    w-v2, w-x.  At u: (w, v1) is a closed type-II triad (v1 shares u's
    community and is u's neighbour), (w, v2) an open one, and the triangle
    {u, w, x} gives the two type-I triads (w, x) and (x, w)."""
    U, W, V1, V2, X = range(5)
    g = from_edges(5, [(U, W), (U, V1), (U, X), (W, V1), (W, V2), (W, X)], [0, 1, 0, 0, 2])
    got = sorted(oracle.triads(g, U, lib=oracle_lib))
    assert got == sorted([(W, V1, 3), (W, V2, 2), (W, X, 1), (X, W, 1)])
    o = oracle.score(g, lib=oracle_lib)
    assert (o["tI"][U], o["tII"][U], o["tII_closed"][U]) == (2, 2, 1)
    # v2 sees w only, with w's other neighbours u and v1 in v2's own
    # community: two open type-II triads and no closed one
    assert sorted(oracle.triads(g, V2, lib=oracle_lib)) == [(W, U, 2), (W, V1, 2)]
    assert (o["tI"][V2], o["tII"][V2], o["tII_closed"][V2]) == (0, 2, 0)
