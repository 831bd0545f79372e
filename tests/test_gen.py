"""Statistics and format checks of the seeded input generators."""
import hashlib
import math

import numpy as np

import oracle
from rsgen import canonical_csr, cfg_sbm_small, graph_stats, lfr, sbm


def _sha(g):
    h = hashlib.sha256()
    for a in (g.off, g.col, g.labels):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def test_canonical_csr_properties():
    rng = np.random.default_rng(0)
    u = rng.integers(0, 50, 400)
    v = rng.integers(0, 50, 400)
    off, col = canonical_csr(50, u, v)
    for x in range(50):
        row = col[off[x]:off[x + 1]]
        assert np.all(np.diff(row) > 0) and not np.any(row == x)
        for y in row:
            assert x in col[off[y]:off[y + 1]]


def test_sbm_small_config_statistics():
    g = cfg_sbm_small(0)
    assert g.n == 2000 and oracle.validate(g) == 0
    # E[m] = 20 * C(100,2) * 0.05 + C(20,2) * 100^2 * 0.001 = 4950 + 1900
    var = 20 * 4950 * 0.05 * 0.95 + 190 * 10000 * 0.001 * 0.999
    assert abs(g.m - 6850) <= 4 * math.sqrt(var)
    st = graph_stats(g)
    assert abs(st["m_inter"] - 1900) <= 4 * math.sqrt(190 * 10000 * 0.001)
    assert np.bincount(g.labels).tolist() == [100] * 20
    assert _sha(g) == _sha(cfg_sbm_small(0))
    assert _sha(g) != _sha(cfg_sbm_small(1))


def test_sbm_uneven_blocks():
    g = sbm([30, 70, 5, 200], 0.2, 0.01, 3)
    assert oracle.validate(g) == 0
    assert sorted(np.bincount(g.labels).tolist()) == [5, 30, 70, 200]


def test_lfr_statistics_small():
    g = lfr(20000, 20.0, 500, 0.1, seed=5, cmin=20, cmax=1000)
    assert oracle.validate(g) == 0
    st = g.meta
    assert abs(st["mean_deg_real"] - 20.0) < 1.5
    assert abs(st["mu_real"] - 0.1) < 0.02
    assert st["max_deg_real"] <= 500
    deg = np.diff(g.off)
    # heavy tail: the top 1 % of degrees sits far above the mean
    assert np.percentile(deg, 99) > 4 * deg.mean()


def test_graph_cache_round_trip(tmp_path):
    from rsgen import cached
    calls = []

    def make():
        calls.append(1)
        return lfr(3000, 10.0, 100, 0.2, seed=5, cmin=20, cmax=300)

    g1 = cached("lfr3k", make, cache_dir=str(tmp_path))
    g2 = cached("lfr3k", make, cache_dir=str(tmp_path))
    assert len(calls) == 1
    for a, b in ((g1.off, g2.off), (g1.col, g2.col), (g1.labels, g2.labels)):
        assert a.dtype == b.dtype and np.array_equal(a, b)
    assert g2.meta["m_real"] == g1.meta["m_real"]
    g3 = cached("lfr3k", make, cache_dir="")  # no cache directory: always generated
    assert len(calls) == 2 and np.array_equal(g3.col, g1.col)


def test_large_array_helpers_match_numpy():
    """The threaded sort / gather helpers give numpy's own results."""
    from rsgen.graphs import _sort_keys, _take, _unique_keys
    rng = np.random.default_rng(3)
    x = rng.integers(0, 10**12, 5_000_000)
    assert np.array_equal(_sort_keys(x, 10**12), np.sort(x))
    y = rng.integers(0, 1000, 5_000_000)
    assert np.array_equal(_unique_keys(y, 1000), np.unique(y))
    idx = rng.integers(0, x.size, 5_000_000)
    assert np.array_equal(_take(x, idx), x[idx])
