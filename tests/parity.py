"""Comparison of the HIP path with the CPU oracle (test helper).

Rules: every integer output bit-exact (border, ell, dprime, tI, tII, the
interaction-matrix rows (community, count), G'); fp64 weights and scores
within REL of the oracle, and a value is exactly zero iff the oracle's is;
top-k identical position by position except inside near-tie classes of the
oracle (neighbouring sorted scores within TIE_REL), where any order is valid.
"""
import numpy as np

import oracle

REL = 1e-6       # scores (fp64, different summation order and log2/cbrt rounding)
W_REL = 1e-9     # weights: closed form of Eq. H_optimal vs the direct entropy sum
TIE_REL = 1e-9


def gpu_run(g, k, stream=None, flags=0, targets=None):
    """Load, score (or, with targets = k_c, restrict to the k_c largest
    communities) and read every output."""
    import paper_2508_01485_amd as rs
    h = rs.rs_load_graph(g.off, g.col, g.labels, stream=stream, flags=flags)
    try:
        if targets is None:
            rs.rs_score(h)
        else:
            rs.rs_restrict_to_targets(h, targets)
        ids, sc = rs.rs_topk(h, k)
        out = {"ids": ids, "scores": sc, "R": rs.rs_read_scores(h), "raw": rs.rs_read_scores(h, raw=True),
               "counts": rs.rs_read_counts(h)}
        out.update(rs.rs_read_vertex_counts(h))
        out["rows"] = rs.rs_read_rows(h)
        out["gprime"] = rs.rs_read_gprime(h)
    finally:
        h.free()
    return out


def rel_close(a, b, rel):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    assert a.shape == b.shape
    zero_a, zero_b = a == 0.0, b == 0.0
    bad_zero = np.flatnonzero(zero_a != zero_b)
    assert bad_zero.size == 0, f"zero pattern differs at {bad_zero[:10]}: {a[bad_zero[:5]]} vs {b[bad_zero[:5]]}"
    nz = ~zero_b
    if nz.any():
        err = np.abs(a[nz] - b[nz]) / np.maximum(np.abs(a[nz]), np.abs(b[nz]))
        worst = float(err.max())
        assert worst <= rel, f"max relative error {worst} > {rel} at {np.flatnonzero(nz)[err.argmax()]}"
        return worst
    return 0.0


def topk_matches(gpu_ids, ora_ids, ora_R_all, k, alive=None):
    """Position-by-position equality outside oracle near-tie classes."""
    gpu_ids = np.asarray(gpu_ids)
    ora_ids = np.asarray(ora_ids)
    assert gpu_ids.size == ora_ids.size
    if gpu_ids.size == 0:
        return 0
    # the oracle's full order, to know each class's members beyond position k
    order_ids, order_sc = oracle.topk(ora_R_all, len(ora_R_all), alive=alive)
    cls = np.zeros(order_sc.size, np.int64)
    for i in range(1, order_sc.size):
        a, b = order_sc[i - 1], order_sc[i]
        same = (a == b) or (max(abs(a), abs(b)) > 0 and abs(a - b) <= TIE_REL * max(abs(a), abs(b)))
        cls[i] = cls[i - 1] + (0 if same else 1)
    cls_of = dict(zip(order_ids.tolist(), cls.tolist()))
    exempt = 0
    for pos, (gi, oi) in enumerate(zip(gpu_ids.tolist(), ora_ids.tolist())):
        if gi == oi:
            continue
        assert gi in cls_of, f"gpu id {gi} not a live vertex"
        assert cls_of[gi] == cls[pos], f"position {pos}: gpu {gi} vs oracle {oi} are not near-tied"
        exempt += 1
    return exempt


def compare(g, gpu, ora, k, alive=None):
    """Full comparison; returns a dict of diagnostics.  alive: the live
    vertices when some were removed (the oracle's top-k skips the others)."""
    n = g.n
    for key in ("ell", "dprime", "tI", "tII"):
        assert np.array_equal(np.asarray(gpu[key], np.int64), np.asarray(ora[key], np.int64)), key
    assert np.array_equal(gpu["border"].astype(np.uint8), ora["border"]), "border"
    c = gpu["counts"]
    assert c["n_border"] == ora["n_border"]
    assert c["m_inter"] == ora["m_inter"]
    assert c["sum_ell"] == int(ora["ell"].sum())
    assert c["sum_tI"] == int(ora["tI"].sum()) and c["sum_tII"] == int(ora["tII"].sum())
    # interaction matrix rows
    off, comm, cnt, w = gpu["rows"]
    assert np.array_equal(off, ora["hist_off"])
    assert np.array_equal(comm, ora["hist_comm"])
    assert np.array_equal(cnt.astype(np.int64), ora["hist_cnt"])
    wr = rel_close(w, ora["hist_w"], W_REL)
    wo = rel_close(gpu["w_own"], ora["w_own"], W_REL)
    om = ora["omega_max"]
    assert (c["omega_max"] == 0.0) == (om == 0.0)
    if om:
        assert abs(c["omega_max"] - om) <= W_REL * om
    # G' = edges whose endpoints have different labels
    goff, gcol = gpu["gprime"]
    src = np.repeat(np.arange(n), np.diff(g.off))
    keep = g.labels[src] != g.labels[g.col]
    exp_off = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(src[keep], minlength=n), out=exp_off[1:])
    assert np.array_equal(goff, exp_off) and np.array_equal(gcol, g.col[keep])
    rr = rel_close(gpu["R"], ora["R"], REL)
    rel_close(gpu["raw"], ora["raw"], REL)
    ora_ids, ora_sc = oracle.topk(ora["R"], k, alive=alive)
    ex = topk_matches(gpu["ids"], ora_ids, ora["R"], k, alive=alive)
    rel_close(gpu["scores"], gpu["R"][gpu["ids"]], 0.0)
    return {"w_rel": wr, "w_own_rel": wo, "R_rel": rr, "tie_exempt": ex}
