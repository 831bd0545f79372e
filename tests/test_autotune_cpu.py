"""The autotuner's degree signature (CPU): it depends on the degree
distribution, not on vertex order or ids, and separates different shapes."""
import numpy as np

from rsgen import lfr, sbm


def _permuted_offsets(g, seed):
    deg = np.diff(g.off)
    perm = np.random.default_rng(seed).permutation(g.n)
    off = np.zeros(g.n + 1, np.int64)
    np.cumsum(deg[perm], out=off[1:])
    return off


def test_signature_ignores_order_and_separates_shapes():
    from paper_2508_01485_amd.autotune import SPACE, DEFAULT, degree_signature
    a = lfr(5000, 12.0, 300, 0.2, seed=1, cmin=10, cmax=300)
    b = sbm([500] * 10, 0.02, 0.002, seed=2)
    sa = degree_signature(a.off)
    assert sa == degree_signature(_permuted_offsets(a, 3))
    assert sa != degree_signature(b.off)
    assert sa != degree_signature(a.off, n_graphs=64)
    assert all(DEFAULT[k] in v for k, v in SPACE.items())
