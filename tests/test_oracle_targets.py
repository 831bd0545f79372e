"""Pins of the oracle's target-community mode (Section VI-A: the interaction
matrix spans the considered communities only, with T summed over them;
Section VII-C: the k largest communities by member count).  Reading: the
pass runs on the subgraph induced by the members of the k_c largest
communities (ties: the smaller label), every other vertex isolated."""
from collections import Counter

import numpy as np
import pytest

import oracle
from oracle import brute
from rsgen import from_edges, random_small


@pytest.fixture(scope="module")
def oracle_lib():
    return oracle.load()


def test_selection_by_size_then_label():
    lab = [5, 5, 5, 2, 2, 9, 9, 7]  # sizes 5:3, 2:2, 9:2, 7:1
    assert list(oracle.target_communities(lab, 1)) == [5]
    assert list(oracle.target_communities(lab, 2)) == [5, 2]  # 2 and 9 tie: the smaller label
    assert list(oracle.target_communities(lab, 3)) == [5, 2, 9]
    assert sorted(oracle.target_communities(lab, 10)) == [2, 5, 7, 9]


def _induced_by_hand(g, k_c):
    """The targets by counting with a Counter, and the induced edge list by
    looping over the rows (independent of the oracle's numpy masks)."""
    cnt = Counter(int(c) for c in g.labels)
    ranked = sorted(cnt, key=lambda c: (-cnt[c], c))[:k_c]
    keep = [int(c) in ranked for c in g.labels]
    edges = []
    for u in range(g.n):
        for e in range(int(g.off[u]), int(g.off[u + 1])):
            v = int(g.col[e])
            if u < v and keep[u] and keep[v]:
                edges.append((u, v))
    return from_edges(g.n, np.array(edges, np.int64).reshape(-1, 2), g.labels), np.array(keep)


def test_restricted_scores_equal_brute_force_on_induced_subgraph(oracle_lib):
    """300 random tiny graphs, k_c in 1..4: the oracle on its restricted
    graph equals the brute force on the subgraph built by hand."""
    worst = 0.0
    for s in range(300):
        rng = np.random.default_rng(20_000 + s)
        n = int(rng.integers(1, 13))
        g = random_small(n, float(rng.uniform(0.2, 0.9)), int(rng.integers(1, 7)), 20_000 + s)
        k_c = int(rng.integers(1, 5))
        gr, keep = oracle.restrict_to_targets(g, k_c)
        gh, keep_h = _induced_by_hand(g, k_c)
        assert np.array_equal(keep, keep_h), s
        assert np.array_equal(gr.off, gh.off) and np.array_equal(gr.col, gh.col), s
        o = oracle.score(gr, lib=oracle_lib)
        R, tI, tII, wmax = brute.scores(gh)
        assert list(o["tI"]) == tI and list(o["tII"]) == tII, s
        assert o["omega_max"] == pytest.approx(wmax, rel=1e-13, abs=0), s
        for a, b in zip(o["R"], R):
            assert (a == 0.0) == (b == 0.0), s
            if b:
                worst = max(worst, abs(a - b) / b)
        # vertices outside the targets have no edges left and score 0
        assert np.all(np.diff(gr.off)[~keep] == 0) and np.all(o["R"][~keep] == 0.0), s
    assert worst <= 1e-12


def test_all_communities_is_the_plain_pass(oracle_lib):
    g = random_small(14, 0.5, 4, 31)
    gr, keep = oracle.restrict_to_targets(g, 4)
    assert keep.all()
    assert np.array_equal(gr.off, g.off) and np.array_equal(gr.col, g.col)


def test_target_mode_changes_weights_through_T(oracle_lib):
    """A vertex with neighbours in three communities, one of them outside the
    targets: its weights follow the counts over the two considered ones.
    Star centre 0 (community 0) with leaves in communities 1, 1, 2, 3, 3, 3
    and a four-member community 0 filler: targets (k_c = 2) are 0 and 3, so
    centre 0's row reduces to {3: 3} and every L has at most one community."""
    lab = [0, 1, 1, 2, 3, 3, 3, 0, 0, 0]
    edges = [(0, i) for i in range(1, 7)] + [(7, 8), (8, 9), (0, 7)]
    g = from_edges(10, edges, lab)
    assert sorted(oracle.target_communities(lab, 2)) == [0, 3]
    gr, keep = oracle.restrict_to_targets(g, 2)
    o = oracle.score(gr, lib=oracle_lib, rows=True)
    # centre's considered neighbours: three in community 3 and one (7) in its own
    assert np.diff(gr.off)[0] == 4
    # with only two considered communities no weight is positive (|L| <= 1)
    assert o["omega_max"] == 0.0 and np.all(o["R"] == 0.0)
    full = oracle.score(g, lib=oracle_lib)
    assert full["omega_max"] > 0.0
