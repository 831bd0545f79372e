// rs_serve.hip -- the served form: a request loop over several resident
// graphs (host code; every request runs the library's own calls on the
// graph's own stream).
//
// A request applies one removal batch to one graph (the removal model of
// Section VII-B), re-scores incrementally and reads the top-k.  Worker threads
// take requests in submission order, skipping requests whose graph is busy,
// so the requests of one graph run one at a time in order while those of
// different graphs overlap on the device.  Graphs are loaded on demand within
// an HBM budget; an idle graph may be evicted (least recently used first) and
// is later reloaded from its validated, renumbered host form (built on its
// first load) with its whole removal history applied as one batch, which
// gives the same graph and the same bits (the result of a
// removal is the graph minus the union of removed edges and vertices, and a
// re-score equals a full pass on it).
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "rs_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

struct ServedGraph {
    int64_t n = 0, nnz = 0;
    std::vector<int64_t> off;
    std::vector<int32_t> col, lab;
    // removal history (caller ids): edges as (src, dst) pairs, vertices
    std::vector<int32_t> hist_src, hist_dst, hist_vert;
    rs_graph *h = nullptr;
    rs::Prebuilt *pre = nullptr;  // validated, renumbered host form (built on the first load)
    int64_t bytes = 0;     // device bytes counted in the budget while resident
    int64_t estimate = 0;  // device bytes expected before the first load
    int64_t known = 0;     // device bytes measured at the last residency (0: never loaded)
    bool busy = false;
    int64_t last_use = 0;
};

struct Request {
    int32_t gid = 0;
    int64_t k = 0;
    std::vector<int32_t> src, dst, verts;
    std::vector<int32_t> ids;
    std::vector<double> scores;
    int64_t count = 0;
    rs_status status = RS_OK;
    std::string error;
    rs_request_info info = {};
    bool done = false;
};

// Device bytes of a graph before it is first loaded: an upper bound from the
// resident layout (per entry: col, record key and data, pair facts; per
// vertex: offsets, cards, scores, top-k lists, marks; per G' entry: links).
int64_t estimate_bytes(int64_t n, int64_t nnz) {
    return 48 * nnz + 360 * n + (8 << 20);
}

}  // namespace

struct rs_server {
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<ServedGraph> graphs;  // workers keep references across unlocks
    std::deque<int64_t> queue;
    std::unordered_map<int64_t, Request> reqs;
    std::vector<std::thread> workers;
    int64_t next_id = 0;
    int64_t budget = 0, used = 0, peak = 0;
    int64_t loads = 0, evictions = 0, done_count = 0;
    bool stop = false;
    Clock::time_point t0 = Clock::now();
    int64_t tick = 0;

    int64_t now_ns() const {
        return (int64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(Clock::now() - t0).count();
    }

    // Under mu: the first queued request whose graph is idle.
    bool take(int64_t &rid) {
        for (auto it = queue.begin(); it != queue.end(); ++it) {
            const Request &r = reqs[*it];
            if (!graphs[r.gid].busy) {
                rid = *it;
                queue.erase(it);
                return true;
            }
        }
        return false;
    }

    // Under mu: make room for `need` more bytes by evicting idle resident
    // graphs, least recently used first.  False if that is not possible now.
    bool make_room(int64_t need, int32_t keep) {
        if (budget <= 0) return true;
        while (used + need > budget) {
            int32_t victim = -1;
            for (int32_t i = 0; i < (int32_t)graphs.size(); ++i) {
                const ServedGraph &sg = graphs[i];
                if (i != keep && !sg.busy && sg.h && (victim < 0 || sg.last_use < graphs[victim].last_use))
                    victim = i;
            }
            if (victim < 0) return false;
            ServedGraph &sg = graphs[victim];
            rs_free_graph(sg.h);
            sg.h = nullptr;
            used -= sg.bytes;
            sg.known = sg.bytes;
            sg.bytes = 0;
            ++evictions;
        }
        return true;
    }

    void worker() {
        std::unique_lock<std::mutex> lk(mu);
        while (true) {
            int64_t rid = -1;
            cv_work.wait(lk, [&] { return stop || take(rid); });
            if (stop && rid < 0) return;
            Request &r = reqs[rid];
            ServedGraph &sg = graphs[r.gid];
            sg.busy = true;
            r.info.t_start = now_ns();
            // residency: reserve the graph's bytes, evicting idle graphs
            bool fresh = false;
            if (!sg.h) {
                const int64_t need = sg.known > 0 ? sg.known : sg.estimate;
                if (budget > 0 && need > budget) {
                    r.status = RS_ERR_NOMEM;
                    r.error = "graph larger than the whole HBM budget";
                } else {
                    cv_work.wait(lk, [&] { return make_room(need, r.gid); });
                    used += need;
                    sg.bytes = need;
                    fresh = true;
                }
            }
            // sg is busy from here on: no other worker frees or replaces
            // its handle, and the handle is only published under mu
            rs_graph *h = sg.h;
            lk.unlock();
            rs_status st = r.status;
            if (st == RS_OK && fresh) {
                st = load(sg, &h);
                if (st == RS_OK) {
                    lk.lock();
                    sg.h = h;
                    // the reservation becomes the measured size; idle graphs
                    // make way if the estimate was short, else the request fails
                    used += h->dev_bytes - sg.bytes;
                    sg.bytes = h->dev_bytes;
                    sg.known = sg.bytes;
                    if (!make_room(0, r.gid)) {
                        rs_free_graph(h);
                        sg.h = h = nullptr;
                        used -= sg.bytes;
                        sg.bytes = 0;
                        st = RS_ERR_NOMEM;
                        r.error = "the graph's device footprint exceeds the HBM budget left by busy graphs";
                    }
                    lk.unlock();
                }
            }
            if (st == RS_OK) st = serve(sg, h, r);
            if (st != RS_OK && r.error.empty()) r.error = rs_last_error();
            lk.lock();
            if (fresh) {
                if (!sg.h) {  // the load failed: give the reservation back
                    used -= sg.bytes;
                    sg.bytes = 0;
                }
                r.info.loaded = sg.h ? 1 : 0;
                if (sg.h) ++loads;
            }
            if (sg.h) {  // staging grown by this request counts too
                used += sg.h->dev_bytes - sg.bytes;
                sg.bytes = sg.known = sg.h->dev_bytes;
            }
            peak = std::max(peak, used);
            r.status = st;
            r.info.t_done = now_ns();
            r.done = true;
            sg.busy = false;
            sg.last_use = ++tick;
            ++done_count;
            cv_done.notify_all();
            cv_work.notify_all();
        }
    }

    // Load a graph and bring it to its current state: a full pass, then its
    // removal history as one batch.  The first load validates and renumbers
    // the host copy once and keeps that form (the copy itself is dropped);
    // a reload after an eviction only uploads it.
    rs_status load(ServedGraph &sg, rs_graph **out) {
        rs_status st = RS_OK;
        if (!sg.pre) {
            rs_csr c;
            c.n = sg.n;
            c.nnz = sg.nnz;
            c.offset_bytes = 8;
            c.on_device = 0;
            c.row_offsets = sg.off.data();
            c.col = sg.col.data();
            c.labels = sg.lab.data();
            st = rs::prebuild_graph(&c, &sg.pre);
            if (st != RS_OK) return st;
            std::vector<int64_t>().swap(sg.off);
            std::vector<int32_t>().swap(sg.col);
            std::vector<int32_t>().swap(sg.lab);
        }
        rs_graph *h = nullptr;
        st = rs::load_prebuilt(sg.pre, nullptr, &h);
        if (st == RS_OK) st = rs_score(h);
        if (st == RS_OK && (!sg.hist_src.empty() || !sg.hist_vert.empty())) {
            rs_removals b;
            b.n_edges = (int64_t)sg.hist_src.size();
            b.src = sg.hist_src.data();
            b.dst = sg.hist_dst.data();
            b.n_vertices = (int64_t)sg.hist_vert.size();
            b.vertices = sg.hist_vert.data();
            st = rs_apply_removals(h, &b, nullptr);
        }
        if (st != RS_OK) {
            rs_free_graph(h);
            return st;
        }
        *out = h;
        return RS_OK;
    }

    // One request on a resident graph: removals, then the top-k.
    rs_status serve(ServedGraph &sg, rs_graph *h, Request &r) {
        rs_removals b;
        b.n_edges = (int64_t)r.src.size();
        b.src = r.src.data();
        b.dst = r.dst.data();
        b.n_vertices = (int64_t)r.verts.size();
        b.vertices = r.verts.data();
        rs_removal_result res = {};
        rs_status st = RS_OK;
        if (b.n_edges > 0 || b.n_vertices > 0) st = rs_apply_removals(h, &b, &res);
        if (st != RS_OK) return st;
        sg.hist_src.insert(sg.hist_src.end(), r.src.begin(), r.src.end());
        sg.hist_dst.insert(sg.hist_dst.end(), r.dst.begin(), r.dst.end());
        sg.hist_vert.insert(sg.hist_vert.end(), r.verts.begin(), r.verts.end());
        r.info.affected = res.affected;
        r.info.edges_removed = res.edges_removed;
        r.ids.resize((size_t)std::max<int64_t>(r.k, 1));
        r.scores.resize((size_t)std::max<int64_t>(r.k, 1));
        return rs_topk(h, r.k, r.ids.data(), r.scores.data(), &r.count);
    }
};

extern "C" {

rs_status rs_server_create(int32_t n_slots, int64_t hbm_budget, rs_server **out) {
    if (!out) return rs::fail(RS_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (n_slots < 1) return rs::fail(RS_ERR_ARG, "n_slots < 1");
    rs_server *s = new (std::nothrow) rs_server();
    if (!s) return rs::fail(RS_ERR_NOMEM, "server allocation failed");
    s->budget = hbm_budget;
    try {
        for (int32_t i = 0; i < n_slots; ++i) s->workers.emplace_back([s] { s->worker(); });
    } catch (...) {
        rs_server_free(s);
        return rs::fail(RS_ERR_NOMEM, "worker threads could not be started");
    }
    *out = s;
    return RS_OK;
}

rs_status rs_server_add_graph(rs_server *s, const rs_csr *csr, int32_t *graph_id) {
    if (!s || !csr || !graph_id) return rs::fail(RS_ERR_ARG, "server, csr or graph_id is NULL");
    if (csr->on_device) return rs::fail(RS_ERR_ARG, "a served graph is registered from host arrays");
    if (csr->n < 0 || csr->nnz < 0) return rs::fail(RS_ERR_ARG, "negative n or nnz");
    if (csr->offset_bytes != 4 && csr->offset_bytes != 8) return rs::fail(RS_ERR_ARG, "offset_bytes must be 4 or 8");
    if (!csr->row_offsets || (csr->n > 0 && !csr->labels) || (csr->nnz > 0 && !csr->col))
        return rs::fail(RS_ERR_ARG, "null CSR array");
    ServedGraph sg;
    try {
        sg.n = csr->n;
        sg.nnz = csr->nnz;
        sg.off.resize(csr->n + 1);
        for (int64_t i = 0; i <= csr->n; ++i)
            sg.off[i] = csr->offset_bytes == 8 ? ((const int64_t *)csr->row_offsets)[i]
                                               : (int64_t)((const int32_t *)csr->row_offsets)[i];
        sg.col.assign(csr->col, csr->col + csr->nnz);
        sg.lab.assign(csr->labels, csr->labels + csr->n);
    } catch (const std::bad_alloc &) {
        return rs::fail(RS_ERR_NOMEM, "host copy of the graph failed");
    }
    sg.estimate = estimate_bytes(sg.n, sg.nnz);
    std::lock_guard<std::mutex> lk(s->mu);
    *graph_id = (int32_t)s->graphs.size();
    s->graphs.push_back(std::move(sg));
    return RS_OK;
}

rs_status rs_server_submit(rs_server *s, int32_t graph_id, const rs_removals *batch, int64_t k, int64_t *request_id) {
    if (!s || !request_id) return rs::fail(RS_ERR_ARG, "server or request_id is NULL");
    if (k < 0) return rs::fail(RS_ERR_ARG, "k < 0");
    Request r;
    r.k = k;
    r.gid = graph_id;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (graph_id < 0 || graph_id >= (int32_t)s->graphs.size()) return rs::fail(RS_ERR_RANGE, "unknown graph id");
    }
    if (batch) {
        if (batch->n_edges < 0 || batch->n_vertices < 0) return rs::fail(RS_ERR_ARG, "negative batch size");
        if ((batch->n_edges > 0 && (!batch->src || !batch->dst)) || (batch->n_vertices > 0 && !batch->vertices))
            return rs::fail(RS_ERR_ARG, "null batch array");
        r.src.assign(batch->src, batch->src + batch->n_edges);
        r.dst.assign(batch->dst, batch->dst + batch->n_edges);
        r.verts.assign(batch->vertices, batch->vertices + batch->n_vertices);
    }
    std::lock_guard<std::mutex> lk(s->mu);
    const int64_t n = s->graphs[graph_id].n;
    for (int32_t x : r.src)
        if (x < 0 || x >= n) return rs::fail(RS_ERR_RANGE, "edge endpoint out of range");
    for (int32_t x : r.dst)
        if (x < 0 || x >= n) return rs::fail(RS_ERR_RANGE, "edge endpoint out of range");
    for (int32_t x : r.verts)
        if (x < 0 || x >= n) return rs::fail(RS_ERR_RANGE, "vertex id out of range");
    r.info.t_submit = s->now_ns();
    const int64_t id = s->next_id++;
    s->reqs.emplace(id, std::move(r));
    s->queue.push_back(id);
    *request_id = id;
    s->cv_work.notify_all();  // a waiter for memory must not absorb the wake-up
    return RS_OK;
}

rs_status rs_server_wait(rs_server *s, int64_t request_id, int32_t *ids, double *scores, int64_t *count,
                         rs_request_info *info) {
    if (!s) return rs::fail(RS_ERR_ARG, "server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(request_id);
    if (it == s->reqs.end()) return rs::fail(RS_ERR_ARG, "unknown request id");
    // submissions may rehash the map while this thread waits: keep a pointer
    // to the element (stable), not the iterator (invalidated by a rehash)
    Request *rq = &it->second;
    s->cv_done.wait(lk, [&] { return rq->done; });
    Request r = std::move(*rq);
    s->reqs.erase(request_id);
    lk.unlock();
    if (r.status != RS_OK) return rs::fail(r.status, r.error);
    if (count) *count = r.count;
    if (r.count > 0 && (!ids || !scores)) return rs::fail(RS_ERR_ARG, "ids or scores is NULL");
    if (r.count > 0) {
        std::copy(r.ids.begin(), r.ids.begin() + r.count, ids);
        std::copy(r.scores.begin(), r.scores.begin() + r.count, scores);
    }
    if (info) *info = r.info;
    return RS_OK;
}

rs_status rs_server_stats(rs_server *s, rs_server_stats_t *st) {
    if (!s || !st) return rs::fail(RS_ERR_ARG, "server or stats is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    st->requests_done = s->done_count;
    st->loads = s->loads;
    st->evictions = s->evictions;
    st->device_bytes = s->used;
    st->peak_device_bytes = s->peak;
    return RS_OK;
}

void rs_server_free(rs_server *s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    for (auto &t : s->workers)
        if (t.joinable()) t.join();
    for (auto &sg : s->graphs) {
        if (sg.h) rs_free_graph(sg.h);
        rs::free_prebuilt(sg.pre);
    }
    delete s;
}

}  // extern "C"
