"""Target-community mode on the GPU (the k_c largest communities only):
every output equals the oracle on the subgraph the targets induce, and the
restricted handle reproduces a fresh load of that subgraph."""
import sys

import numpy as np
import pytest

import oracle
from rsgen import lfr, random_small, sbm
from tests.parity import compare, gpu_run, rel_close

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[targets]", *a, flush=True)
    sys.stdout.flush()


CASES = [
    ("lfr_8k", lambda: lfr(8000, 14.0, 300, 0.3, seed=41, cmin=20, cmax=1500), (1, 3, 5, 7)),
    ("sbm_uneven", lambda: sbm([400, 300, 300, 200, 120, 80, 40], 0.05, 0.01, seed=42), (2, 4, 7)),
    ("gnp_ties", lambda: random_small(300, 0.05, 6, 43), (1, 2, 6)),
]


@pytest.mark.parametrize("name,make,kcs", CASES, ids=[c[0] for c in CASES])
def test_targets_match_oracle(name, make, kcs):
    g = make()
    for k_c in kcs:
        _say(f"{name} k_c={k_c}")
        gr, keep = oracle.restrict_to_targets(g, k_c)
        gpu = gpu_run(g, 100, targets=k_c)
        ora = oracle.score(gr, rows=True)
        d = compare(gr, gpu, ora, 100, alive=keep)
        assert gpu["counts"]["n_alive"] == int(keep.sum())
        assert set(gpu["ids"].tolist()) <= set(np.flatnonzero(keep).tolist())
        _say(f"{name} k_c={k_c}: ok {d}")


def test_targets_equal_fresh_load_of_induced_graph():
    import paper_2508_01485_amd as rs
    g = lfr(8000, 14.0, 300, 0.3, seed=41, cmin=20, cmax=1500)
    gr, keep = oracle.restrict_to_targets(g, 4)
    h = rs.rs_load_graph(g.off, g.col, g.labels)
    try:
        res = rs.rs_restrict_to_targets(h, 4)
        R1 = rs.rs_read_scores(h)
        c1 = rs.rs_read_vertex_counts(h)
        again = rs.rs_restrict_to_targets(h, 6)  # a wider set keeps the intersection: nothing more goes
        assert again["vertices_removed"] == 0
        assert rs.rs_read_scores(h).tobytes() == R1.tobytes()
    finally:
        h.free()
    assert res["vertices_removed"] == int((~keep).sum())
    h2 = rs.rs_load_graph(gr.off, gr.col, gr.labels)
    try:
        rs.rs_score(h2)
        R2 = rs.rs_read_scores(h2)
        c2 = rs.rs_read_vertex_counts(h2)
    finally:
        h2.free()
    rel_close(R1, R2, 1e-12)
    for key in ("border", "ell", "dprime", "tI", "tII"):
        assert np.array_equal(c1[key], c2[key]), key


def test_targets_covering_every_community_change_nothing():
    import paper_2508_01485_amd as rs
    g = sbm([200, 150, 100], 0.06, 0.01, seed=44)
    h = rs.rs_load_graph(g.off, g.col, g.labels)
    try:
        res = rs.rs_restrict_to_targets(h, 3)  # also runs the first pass
        R1 = rs.rs_read_scores(h)
        rs.rs_score(h)
        assert rs.rs_read_scores(h).tobytes() == R1.tobytes()
        assert res == {"edges_removed": 0, "edges_ignored": 0, "vertices_removed": 0, "affected": 0}
        with pytest.raises(rs.RSError, match="k_c < 1"):
            rs.rs_restrict_to_targets(h, 0)
    finally:
        h.free()
