"""Pins of the oracle's reachable-community count (absolute AWCC, Section
VII-B): |zeta(v)| = distinct communities among the other vertices that paths
from v reach."""
import numpy as np
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import connected_components

import oracle
from rsgen import from_edges, random_small


def test_hand_example():
    # component {0,1,2,3}: labels 0,1,1,2; component {4,5}: labels 0,0; 6 isolated
    g = from_edges(7, [(0, 1), (1, 2), (2, 3), (4, 5)], [0, 1, 1, 2, 0, 0, 3])
    got = oracle.reachable_communities(g, [0, 1, 3, 4, 6])
    # 0 reaches 1,2,3 -> {1, 2}; 1 reaches 0,2,3 -> {0, 1, 2}; 3 -> {0, 1};
    # 4 reaches 5 -> {0} (its own community, through another member); 6 -> none
    assert list(got) == [2, 3, 2, 1, 0]
    alive = np.ones(7, bool)
    alive[1] = False
    assert oracle.reachable_communities(g, [1], alive=alive)[0] == 0


def test_equals_component_labels_by_scipy():
    """Against connected components from scipy (a different algorithm)."""
    for s in range(60):
        rng = np.random.default_rng(700 + s)
        n = int(rng.integers(1, 80))
        g = random_small(n, float(rng.uniform(0.0, 0.08)), int(rng.integers(1, 9)), 700 + s)
        a = csr_matrix((np.ones(g.nnz), g.col, g.off), shape=(n, n))
        _, comp = connected_components(a, directed=False)
        src = rng.choice(n, min(n, 10), replace=False)
        exp = []
        for v in src:
            members = np.flatnonzero(comp == comp[v])
            members = members[members != v]
            exp.append(len(set(g.labels[members].tolist())))
        assert list(oracle.reachable_communities(g, src)) == exp, s
