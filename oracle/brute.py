"""Pure-Python brute force of the robust spanning index -- TEST INFRASTRUCTURE ONLY.

An independent, deliberately naive second reading of the paper used to pin the C
oracle on tiny graphs (n <= ~16).  It shares nothing with ``rs_oracle.c``:

* L(u, v) is an explicit ``collections.Counter`` over N(v) minus C(u)
  (Eq. cont); H and the weight follow Eq. entropy / Eq. weight with log2.
* Triads are classified from the definitions of Section III-A: type-I is a
  closed triangle over three distinct communities, type-II an open triad
  (u, v not adjacent) with C(u) = C(v) != C(w); the closed triangle with
  C(u) = C(v) != C(w) is counted once as type-II (reading A7).
* w_max is found by the literal double loop of Algorithm 1, Step 2: every pair
  of border vertices (u, v) with C(u) = C(v) or v in N(u) and |L(u, v)| > 1
  adds the directed edge v -> u with weight w_v(u) to E_b.
* R(u) sums over every ordered (w, v) in V x V with w in N(u), v in N(w), and
  divides each term by w_max and the sum by d(u)(d(u)-1) (Algorithm 1, Step 3).
"""
from __future__ import annotations

import math
from collections import Counter


def adjacency(g):
    adj = [set() for _ in range(g.n)]
    for u in range(g.n):
        for e in range(int(g.off[u]), int(g.off[u + 1])):
            adj[u].add(int(g.col[e]))
    return adj


def L_multiset(adj, C, u_comm, v):
    return Counter(C[x] for x in adj[v] if C[x] != u_comm)


def entropy(counter):
    total = sum(counter.values())
    h = 0.0
    for f in counter.values():
        p = f / total
        h -= p * math.log2(p)
    return h


def omega(adj, C, u_comm, v):
    L = L_multiset(adj, C, u_comm, v)
    if not L:
        return 0.0
    return entropy(L) * len(L)


def triad_kind(adj, C, u, w, v):
    """0 none, 1 type-I, 2 type-II open, 3 type-II closed (definitions of Section III-A)."""
    if len({u, w, v}) < 3:
        return 0
    if w not in adj[u] or v not in adj[w]:
        return 0
    if len({C[u], C[w], C[v]}) == 3 and v in adj[u]:
        return 1
    if C[u] == C[v] and C[w] != C[u]:
        return 3 if v in adj[u] else 2
    return 0


def indicator(adj, C, u, w, v):
    k = triad_kind(adj, C, u, w, v)
    return k != 0 and C[v] != C[w] and C[u] != C[w]


def border_set(adj, C):
    return {u for u in range(len(adj)) if any(C[x] != C[u] for x in adj[u])}


def omega_max(adj, C):
    Vb = border_set(adj, C)
    best = 0.0
    for u in Vb:
        for v in Vb:
            if C[u] == C[v] or v in adj[u]:
                L = L_multiset(adj, C, C[u], v)
                if len(L) > 1:
                    best = max(best, entropy(L) * len(L))
    return best


def scores(g):
    """Return (R, tI, tII, omega_max) lists for a tiny graph."""
    adj = adjacency(g)
    C = [int(c) for c in g.labels]
    n = g.n
    wmax = omega_max(adj, C)
    R, tI, tII = [0.0] * n, [0] * n, [0] * n
    for u in range(n):
        acc = 0.0
        for w in range(n):
            for v in range(n):
                if w not in adj[u] or v not in adj[w]:
                    continue
                if not indicator(adj, C, u, w, v):
                    continue
                if triad_kind(adj, C, u, w, v) == 1:
                    tI[u] += 1
                else:
                    tII[u] += 1
                prod = omega(adj, C, C[u], v) * omega(adj, C, C[v], w) * omega(adj, C, C[u], w)
                if wmax > 0:
                    acc += prod ** (1.0 / 3.0) / wmax
        d = len(adj[u])
        R[u] = acc / (d * (d - 1)) if d >= 2 and wmax > 0 else 0.0
    return R, tI, tII, wmax
