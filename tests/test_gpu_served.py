"""The served form: requests on several resident graphs, run concurrently by
the server's workers (and, under a small HBM budget, with evictions and
reloads), give exactly the results of applying each graph's batches one by
one to a lone handle, and each request's top-k is the CPU oracle's on that
graph's mutated state."""
import sys

import numpy as np
import pytest

from rsgen import lfr

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[served]", *a, flush=True)
    sys.stdout.flush()


def _graphs():
    return [lfr(n, 12.0, 200, 0.25, seed=60 + i, cmin=10, cmax=300) for i, n in enumerate((3000, 5000, 4000, 6000))]


def _requests(graphs, count, seed):
    """(graph index, edges or None, vertices or None) in submission order."""
    rng = np.random.default_rng(seed)
    alive = [np.ones(g.edges()[0].size, bool) for g in graphs]
    out = []
    for _ in range(count):
        gi = int(rng.integers(len(graphs)))
        g = graphs[gi]
        u, v = g.edges()
        if rng.random() < 0.6:
            live = np.flatnonzero(alive[gi])
            pick = rng.choice(live, min(int(rng.integers(1, 80)), live.size), replace=False)
            alive[gi][pick] = False
            out.append((gi, np.stack([u[pick], v[pick]], 1), None))
        else:
            out.append((gi, None, rng.choice(g.n, int(rng.integers(1, 6)), replace=False)))
    return out


def _alone(rs, graphs, reqs, k):
    """Each graph's batches applied in order to a lone handle."""
    handles = []
    for g in graphs:
        h = rs.rs_load_graph(g.off, g.col, g.labels)
        rs.rs_score(h)
        handles.append(h)
    res = []
    for gi, e, v in reqs:
        rs.rs_apply_removals(handles[gi], edges=e, vertices=v)
        res.append(rs.rs_topk(handles[gi], k))
    for h in handles:
        h.free()
    return res


def _served(rs, graphs, reqs, k, slots, budget):
    srv = rs.RSServer(slots=slots, hbm_budget=budget)
    try:
        gids = [srv.add_graph(g.off, g.col, g.labels) for g in graphs]
        rids = [srv.submit(gids[gi], k, edges=e, vertices=v) for gi, e, v in reqs]
        out = [srv.wait(r) for r in rids]
        return out, srv.stats()
    finally:
        srv.free()


def _compare(alone, served):
    for i, ((ia, sa), (ib, sb, info)) in enumerate(zip(alone, served)):
        assert np.array_equal(ia, ib), i
        assert sa.tobytes() == sb.tobytes(), i
        assert info["t_submit"] <= info["t_start"] <= info["t_done"]


def test_served_requests_equal_alone():
    import paper_2508_01485_amd as rs
    graphs = _graphs()
    reqs = _requests(graphs, 40, 1)
    alone = _alone(rs, graphs, reqs, 50)
    served, st = _served(rs, graphs, reqs, 50, slots=3, budget=0)
    _compare(alone, served)
    assert st["requests_done"] == 40 and st["loads"] == len(graphs) and st["evictions"] == 0, st
    _say("mix of 40 requests on 4 graphs, 3 slots: identical to alone", st)


def test_served_under_budget_evicts_and_reloads():
    """A budget of about two graphs: graphs are evicted and reloaded with
    their removal history, and every result is still the lone one."""
    import paper_2508_01485_amd as rs
    graphs = _graphs()
    reqs = _requests(graphs, 40, 2)
    alone = _alone(rs, graphs, reqs, 30)
    big = max(48 * g.nnz + 360 * g.n + (8 << 20) for g in graphs)
    served, st = _served(rs, graphs, reqs, 30, slots=2, budget=2 * big)
    _compare(alone, served)
    assert st["evictions"] > 0 and st["loads"] > len(graphs), st
    assert st["peak_device_bytes"] <= 2 * big, st
    _say("budget of two graphs: identical to alone", st)


def test_served_submit_while_waiting():
    """Requests submitted from one thread while another waits for earlier
    ones (the request table grows during the waits); results equal alone."""
    import threading

    import paper_2508_01485_amd as rs
    graphs = _graphs()
    reqs = _requests(graphs, 120, 3)
    alone = _alone(rs, graphs, reqs, 20)
    srv = rs.RSServer(slots=3, hbm_budget=0)
    try:
        gids = [srv.add_graph(g.off, g.col, g.labels) for g in graphs]
        rids, out = [], []
        cv = threading.Condition()

        def waiter():
            i = 0
            while i < len(reqs):
                with cv:
                    while i >= len(rids):
                        cv.wait()
                    rid = rids[i]
                out.append(srv.wait(rid))
                i += 1

        th = threading.Thread(target=waiter)
        th.start()
        for gi, e, v in reqs:
            rid = srv.submit(gids[gi], 20, edges=e, vertices=v)
            with cv:
                rids.append(rid)
                cv.notify()
        th.join()
    finally:
        srv.free()
    _compare(alone, out)
    _say("120 requests submitted while waiting: identical to alone")


def test_served_request_on_an_invalid_graph_fails_cleanly():
    """A graph is validated on its first load: a request on an asymmetric
    graph fails with RS_ERR_GRAPH through wait, and a valid graph served
    beside it is unaffected."""
    import paper_2508_01485_amd as rs
    good = _graphs()[0]
    bad_col = good.col.copy()
    bad_col[0] = bad_col[0] + 1 if bad_col[0] + 1 < good.n else bad_col[0] - 1  # breaks symmetry (or sorting)
    srv = rs.RSServer(slots=2, hbm_budget=0)
    try:
        gb = srv.add_graph(good.off, bad_col, good.labels)
        gg = srv.add_graph(good.off, good.col, good.labels)
        rb = srv.submit(gb, 10, vertices=[0])
        rg = srv.submit(gg, 10, vertices=[0])
        with pytest.raises(rs.RSError) as ei:
            srv.wait(rb)
        assert ei.value.status == 2, ei.value
        ids, sc, info = srv.wait(rg)
        assert ids.size == 10
        with pytest.raises(rs.RSError):  # and again on a later request
            srv.wait(srv.submit(gb, 5))
    finally:
        srv.free()
    ref = _alone(rs, [good], [(0, None, np.array([0]))], 10)[0]
    assert np.array_equal(ids, ref[0]) and sc.tobytes() == ref[1].tobytes()


def _oracle_results(graphs, reqs, k):
    """Each request's top-k from the oracle on the graph's state after that
    request: the edges and vertices removed so far (a removed vertex loses
    its edges and leaves the ranking)."""
    import oracle
    from rsgen import from_edges
    state = []
    for g in graphs:
        u, v = g.edges()
        state.append({"idx": {(int(a), int(b)): i for i, (a, b) in enumerate(zip(u, v))},
                      "e": np.ones(u.size, bool), "v": np.ones(g.n, bool), "u": u, "w": v})
    out = []
    for gi, e, vs in reqs:
        s, g = state[gi], graphs[gi]
        if e is not None:
            for a, b in np.asarray(e).tolist():
                s["e"][s["idx"][(min(a, b), max(a, b))]] = False
        if vs is not None:
            s["v"][np.asarray(vs)] = False
            s["e"] &= s["v"][s["u"]] & s["v"][s["w"]]
        cur = from_edges(g.n, np.stack([s["u"][s["e"]], s["w"][s["e"]]], 1), g.labels)
        o = oracle.score(cur)
        ids, sc = oracle.topk(o["R"], k, alive=s["v"].astype(np.uint8))
        out.append((ids, sc, o["R"], s["v"].copy()))
    return out


def _compare_oracle(ora, served, k):
    from tests.parity import REL, rel_close, topk_matches
    exempt = 0
    for i, ((oi, osc, oR, alive), (ib, sb, _)) in enumerate(zip(ora, served)):
        assert ib.size == oi.size, i
        exempt += topk_matches(ib, oi, oR, k, alive=alive.astype(np.uint8))
        rel_close(sb, oR[ib], REL)
    return exempt


def test_served_requests_match_oracle():
    """Every request served in the mix (4 graphs, 3 slots, then a budget of
    about two graphs with evictions and reloads) returns the top-k of the
    oracle run on that graph's mutated state."""
    import paper_2508_01485_amd as rs
    graphs = _graphs()
    for seed, slots, budget_graphs in ((4, 3, 0), (5, 2, 2)):
        reqs = _requests(graphs, 30, seed)
        big = max(48 * g.nnz + 360 * g.n + (8 << 20) for g in graphs)
        served, st = _served(rs, graphs, reqs, 25, slots=slots, budget=budget_graphs * big)
        ex = _compare_oracle(_oracle_results(graphs, reqs, 25), served, 25)
        _say(f"{len(reqs)} served requests equal the oracle's top-25 ({ex} near-tie positions)", st)
