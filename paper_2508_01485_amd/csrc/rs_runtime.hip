// rs_runtime.hip -- host side of the RS library: the C ABI of include/rs.h.
//
// rs_load_graph validates the caller's CSR (a simple undirected graph,
// Section II), renumbers it so that every community is a contiguous id range
// (labels ascending, caller ids ascending inside a community), re-sorts the
// rows, bins the vertices by degree for the row kernel and uploads everything
// to device memory owned by the handle.  All later calls run kernels on the
// graph's stream (rs_kernels.hip); the host only marshals arguments, sizes
// launches and copies results.
#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <cstring>
#include <new>
#include <thread>

#include "rs_internal.h"

namespace rs {

static thread_local std::string g_err;

rs_status fail(rs_status s, const std::string &msg) {
    g_err = msg;
    return s;
}

rs_status hip_fail(hipError_t e, const char *what) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return (e == hipErrorOutOfMemory) ? RS_ERR_NOMEM : RS_ERR_HIP;
}

void clear_error() { g_err.clear(); }

// ------------------------------------------------------------ host threads
template <class F>
static void parallel_for(int64_t n, int64_t grain, F &&f) {
    unsigned nt = std::thread::hardware_concurrency();
    nt = std::max(1u, std::min(nt, 16u));
    if (n <= grain || nt == 1) {
        f((int64_t)0, n);
        return;
    }
    std::atomic<int64_t> next{0};
    auto work = [&]() {
        for (;;) {
            int64_t s = next.fetch_add(grain);
            if (s >= n) break;
            f(s, std::min(n, s + grain));
        }
    };
    std::vector<std::thread> th;
    th.reserve(nt - 1);
    for (unsigned i = 1; i < nt; ++i) th.emplace_back(work);
    work();
    for (auto &t : th) t.join();
}

// ------------------------------------------------------------ allocation
// Optional fault injection for tests of the error paths: RS_FAULT_ALLOC=N
// makes the N-th device allocation of every rs_load_graph call fail.
static hipError_t dev_alloc(rs_graph *g, void **p, size_t bytes) {
    *p = nullptr;
    const long long idx = (long long)g->allocations.size() + 1;
    if (const char *f = std::getenv("RS_FAULT_ALLOC")) {
        if (std::atoll(f) == idx) return hipErrorOutOfMemory;
    }
    hipError_t e = hipMalloc(p, bytes ? bytes : 16);
    if (e == hipSuccess) {
        g->allocations.push_back({*p, bytes ? bytes : 16});
        g->dev_bytes += (int64_t)(bytes ? bytes : 16);
    }
    return e;
}

// Free one buffer of the graph (the stream must be idle).
static void dev_free(rs_graph *g, void **p) {
    if (!*p) return;
    for (size_t i = 0; i < g->allocations.size(); ++i)
        if (g->allocations[i].first == *p) {
            g->dev_bytes -= (int64_t)g->allocations[i].second;
            g->allocations.erase(g->allocations.begin() + (long)i);
            break;
        }
    (void)hipFree(*p);
    *p = nullptr;
}

static void release(rs_graph *g) {
    if (!g) return;
    if (g->stream) (void)hipStreamSynchronize(g->stream);
    release_replays(g);
    for (auto &a : g->allocations) (void)hipFree(a.first);
    g->allocations.clear();
    if (g->hpin) (void)hipHostFree(g->hpin);
    g->hpin = nullptr;
    g->hpin_cap = 0;
    if (g->rem_buf) (void)hipFree(g->rem_buf);
    if (g->rem_host) (void)hipHostFree(g->rem_host);
    if (g->rem_cnt_host) (void)hipHostFree(g->rem_cnt_host);
    if (g->rem_ev) (void)hipEventDestroy(g->rem_ev);
    g->rem_ev = nullptr;
    if (g->reach_hflag) (void)hipHostFree(g->reach_hflag);
    g->reach_hflag = nullptr;
    g->reach_comp = g->reach_src = nullptr;
    g->reach_bits = g->reach_flag = nullptr;
    g->rem_buf = g->rem_host = nullptr;
    g->rem_cnt_host = nullptr;
    g->rem_cap = g->rem_host_cap = 0;
    for (hipEvent_t e : g->timing.pool) (void)hipEventDestroy(e);
    for (auto &pe : g->timing.pending) {
        (void)hipEventDestroy(pe.second.first);
        (void)hipEventDestroy(pe.second.second);
    }
    g->timing.pool.clear();
    g->timing.pending.clear();
    if (g->own_stream && g->stream) (void)hipStreamDestroy(g->stream);
    g->stream = nullptr;
}

// ------------------------------------------------------------ timing
static hipEvent_t take_event(rs_graph *g) {
    hipEvent_t e = nullptr;
    if (!g->timing.pool.empty()) {
        e = g->timing.pool.back();
        g->timing.pool.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
        e = nullptr;
    }
    return e;
}

void timing_begin(rs_graph *g, int kid, hipEvent_t *ev) {
    (void)kid;
    *ev = nullptr;
    if (!g->timing.on) return;
    *ev = take_event(g);
    if (*ev) (void)hipEventRecord(*ev, g->stream);
}

void timing_end(rs_graph *g, int kid, hipEvent_t ev) {
    if (!g->timing.on || !ev) return;
    hipEvent_t e2 = take_event(g);
    if (!e2) {
        g->timing.pool.push_back(ev);
        return;
    }
    (void)hipEventRecord(e2, g->stream);
    g->timing.pending.push_back({kid, {ev, e2}});
}

// ------------------------------------------------------------ validation
template <class OffIn>
static rs_status validate_graph(int64_t n, int64_t nnz, const OffIn *off, const int32_t *col, const int32_t *lab) {
    if ((int64_t)off[0] != 0) return fail(RS_ERR_GRAPH, "row_offsets[0] != 0");
    for (int64_t u = 0; u < n; ++u)
        if ((int64_t)off[u + 1] < (int64_t)off[u])
            return fail(RS_ERR_GRAPH, "row_offsets decrease at vertex " + std::to_string(u));
    if ((int64_t)off[n] != nnz) return fail(RS_ERR_GRAPH, "row_offsets[n] != nnz");
    for (int64_t u = 0; u < n; ++u)
        if (lab[u] < 0) return fail(RS_ERR_GRAPH, "negative label at vertex " + std::to_string(u));
    for (int64_t i = 0; i < nnz; ++i)
        if (col[i] < 0 || col[i] >= n) return fail(RS_ERR_RANGE, "neighbour id out of range at entry " + std::to_string(i));
    std::atomic<int> bad{0};
    std::atomic<int64_t> bad_at{-1};
    parallel_for(n, 4096, [&](int64_t lo, int64_t hi) {
        for (int64_t u = lo; u < hi && !bad.load(std::memory_order_relaxed); ++u) {
            const int64_t b = (int64_t)off[u], e = (int64_t)off[u + 1];
            for (int64_t i = b; i < e; ++i) {
                const int32_t v = col[i];
                int why = 0;
                if (v < 0 || v >= n)
                    why = 3;
                else if (v == u)
                    why = 1;
                else if (i > b && col[i - 1] >= v)
                    why = 2;
                else {
                    const int32_t *rb = col + (int64_t)off[v], *re = col + (int64_t)off[v + 1];
                    const int32_t *it = std::lower_bound(rb, re, (int32_t)u);
                    if (it == re || *it != (int32_t)u) why = 4;
                }
                if (why) {
                    int expected = 0;
                    if (bad.compare_exchange_strong(expected, why)) bad_at.store(u);
                    return;
                }
            }
        }
    });
    switch (bad.load()) {
        case 0: return RS_OK;
        case 1: return fail(RS_ERR_GRAPH, "self-loop at vertex " + std::to_string(bad_at.load()));
        case 2: return fail(RS_ERR_GRAPH, "row not strictly ascending (unsorted or duplicate) at vertex " +
                                              std::to_string(bad_at.load()));
        case 3: return fail(RS_ERR_RANGE, "neighbour id out of range in row " + std::to_string(bad_at.load()));
        default: return fail(RS_ERR_GRAPH, "asymmetric adjacency at vertex " + std::to_string(bad_at.load()));
    }
}

// ------------------------------------------------------------ load
// The static schedule of a graph under one Tiling: row tiles and hub rows,
// score tiles, score hubs and their chunks, and the blocks of each vertex.
struct HostTiles {
    std::vector<int2> rtv, stiles, schunk;
    std::vector<RowTile> rtiles;
    std::vector<int32_t> vrowb, vscore;  // the row block and score unit of each vertex
    std::vector<int32_t> rhubs, shubs, sfirst;
    std::vector<int32_t> gblk_off, gblk;  // batches: the row blocks of each graph
    int n_chunks_lds = 0;
    int n_hubs_lds = 0;  // score hubs whose foreign list fits in LDS (listed first)
};

struct HostGraph : HostTiles {
    std::vector<int64_t> off;   // internal offsets
    std::vector<int32_t> col;   // internal rows
    std::vector<int32_t> lab;   // internal community per internal vertex
    std::vector<int32_t> new2old, old2new, comm2orig;
    std::vector<int64_t> oo, goff;
    std::vector<int32_t> outl, cstart;
};

// Greedy cut of the vertex sequence into tiles of consecutive vertices: a
// tile closes when the next vertex would push its weight past wcap or its
// vertex count past vcap, and at every vertex listed in cuts (ascending).  A
// vertex heavier than wcap is a hub.
static void cut_tiles(int64_t n, const std::vector<int64_t> &weight, int64_t wcap, int64_t vcap,
                      std::vector<int2> &tiles, std::vector<int32_t> &hubs,
                      const std::vector<int64_t> &cuts = std::vector<int64_t>()) {
    int64_t lo = 0, w = 0;
    size_t ci = 0;
    for (int64_t v = 0; v < n; ++v) {
        if (ci < cuts.size() && cuts[ci] <= v) {
            while (ci < cuts.size() && cuts[ci] <= v) ++ci;
            if (v > lo) tiles.push_back(make_int2((int)lo, (int)v));
            lo = v;
            w = 0;
        }
        const int64_t x = weight[v];
        if (x > wcap) {
            if (v > lo) tiles.push_back(make_int2((int)lo, (int)v));
            hubs.push_back((int32_t)v);
            lo = v + 1;
            w = 0;
            continue;
        }
        if (w + x > wcap || v - lo == vcap) {
            tiles.push_back(make_int2((int)lo, (int)v));
            lo = v;
            w = 0;
        }
        w += x;
    }
    if (n > lo) tiles.push_back(make_int2((int)lo, (int)n));
}

// Cut the static schedule for the tiling T from the internal row offsets,
// each vertex's row capacity and load-time foreign degree (vstart: a batch's
// graph starts; tiles never span two graphs).
static void cut_all(int64_t n, const std::vector<int64_t> &off, const std::vector<int64_t> &cap,
                    const std::vector<int64_t> &fgn, const std::vector<int64_t> &vstart, const Tiling &T,
                    HostTiles &H) {
    H = HostTiles();
    cut_tiles(n, cap, T.row_entries, T.row_vertices, H.rtv, H.rhubs, vstart);
    H.rtiles.resize(H.rtv.size());
    for (size_t t = 0; t < H.rtv.size(); ++t) {
        RowTile &rt = H.rtiles[t];
        rt.v0 = H.rtv[t].x;
        rt.v1 = H.rtv[t].y;
        rt.e0 = off[rt.v0];
        rt.te = (int)(off[rt.v1] - off[rt.v0]);
        rt.pad = 0;
    }
    cut_tiles(n, fgn, T.score_pairs, T.score_vertices, H.stiles, H.shubs);
    // a score hub's pairs are processed kScoreTileP at a time, one chunk per workgroup
    // hubs whose foreign list fits in LDS are listed (and chunked) first
    std::stable_partition(H.shubs.begin(), H.shubs.end(), [&](int32_t v) { return fgn[v] <= T.hub_list; });
    H.sfirst.assign(1, 0);
    H.n_chunks_lds = 0;
    H.n_hubs_lds = 0;
    for (size_t h = 0; h < H.shubs.size(); ++h) {
        if (fgn[H.shubs[h]] <= T.hub_list) H.n_hubs_lds = (int)h + 1;
        const int64_t nch = (fgn[H.shubs[h]] + kScoreTileP - 1) / kScoreTileP;
        for (int64_t c = 0; c < nch; ++c) H.schunk.push_back(make_int2((int)h, (int)c));
        H.sfirst.push_back((int32_t)H.schunk.size());
        if (fgn[H.shubs[h]] <= T.hub_list) H.n_chunks_lds = (int)H.schunk.size();
    }
    // the block of the full launch that handles each vertex: hubs take
    // the first blocks, tile t of XCD x = t / per runs at block
    // hubs + 8 (t % per) + ((x - hubs) mod 8) (the inverse of the
    // kernels' block-to-tile map)
    auto tile_block = [](int64_t t, int64_t n_tiles, int64_t hubs) {
        const int64_t per = (n_tiles + 7) / 8, x = t / per, q = t % per;
        return (int32_t)(hubs + 8 * q + (((x - hubs) % 8 + 8) % 8));
    };
    H.vrowb.assign(n, 0);
    for (size_t h = 0; h < H.rhubs.size(); ++h) H.vrowb[H.rhubs[h]] = (int32_t)h;
    for (size_t t = 0; t < H.rtv.size(); ++t)
        for (int v = H.rtv[t].x; v < H.rtv[t].y; ++v)
            H.vrowb[v] = tile_block((int64_t)t, (int64_t)H.rtv.size(), (int64_t)H.rhubs.size());
    H.vscore.assign(n, 0);
    for (size_t h = 0; h < H.shubs.size(); ++h) H.vscore[H.shubs[h]] = -1 - (int32_t)h;
    for (size_t t = 0; t < H.stiles.size(); ++t)
        for (int v = H.stiles[t].x; v < H.stiles[t].y; ++v)
            H.vscore[v] = tile_block((int64_t)t, (int64_t)H.stiles.size(), (int64_t)H.n_chunks_lds);
    if (!vstart.empty()) {
        // each row block lies in one graph (tiles are cut at the graph
        // starts): list the blocks of every graph, for its w_max
        const int64_t G = (int64_t)vstart.size() - 1;
        auto graph_of = [&](int64_t v) {
            return (int64_t)(std::upper_bound(vstart.begin(), vstart.end(), v) - vstart.begin()) - 1;
        };
        std::vector<std::pair<int32_t, int32_t>> bg;  // (graph, block)
        for (size_t h = 0; h < H.rhubs.size(); ++h) bg.emplace_back((int32_t)graph_of(H.rhubs[h]), (int32_t)h);
        for (size_t t = 0; t < H.rtv.size(); ++t)
            bg.emplace_back((int32_t)graph_of(H.rtv[t].x),
                            tile_block((int64_t)t, (int64_t)H.rtv.size(), (int64_t)H.rhubs.size()));
        std::sort(bg.begin(), bg.end());
        H.gblk_off.assign(G + 1, 0);
        H.gblk.resize(bg.size());
        for (size_t i = 0; i < bg.size(); ++i) {
            ++H.gblk_off[bg[i].first + 1];
            H.gblk[i] = bg[i].second;
        }
        for (int64_t gi = 0; gi < G; ++gi) H.gblk_off[gi + 1] += H.gblk_off[gi];
    }
}

// vstart: for a batch, the first vertex of each graph and n (a graph's
// vertices keep one contiguous id range through the renumbering, since its
// labels are ranked above those of the graphs before it); empty otherwise.
template <class OffIn>
static rs_status build_internal(int64_t n, int64_t nnz, const OffIn *off, const int32_t *col, const int32_t *lab,
                                const std::vector<int64_t> &vstart, HostGraph &H) {
    try {
        // communities: ascending caller label -> internal id 0..k-1
        H.comm2orig.assign(lab, lab + n);
        std::sort(H.comm2orig.begin(), H.comm2orig.end());
        H.comm2orig.erase(std::unique(H.comm2orig.begin(), H.comm2orig.end()), H.comm2orig.end());
        const int64_t k = (int64_t)H.comm2orig.size();
        std::vector<int32_t> cid(n);
        parallel_for(n, 1 << 16, [&](int64_t lo, int64_t hi) {
            for (int64_t v = lo; v < hi; ++v)
                cid[v] = (int32_t)(std::lower_bound(H.comm2orig.begin(), H.comm2orig.end(), lab[v]) -
                                   H.comm2orig.begin());
        });
        // vertices: counting sort by community, stable in caller id
        std::vector<int64_t> start(k + 1, 0);
        for (int64_t v = 0; v < n; ++v) ++start[cid[v] + 1];
        for (int64_t c = 0; c < k; ++c) start[c + 1] += start[c];
        H.new2old.resize(n);
        H.old2new.resize(n);
        H.lab.resize(n);
        {
            std::vector<int64_t> fill(start.begin(), start.end() - 1);
            for (int64_t v = 0; v < n; ++v) {
                const int64_t nv = fill[cid[v]]++;
                H.new2old[nv] = (int32_t)v;
                H.old2new[v] = (int32_t)nv;
                H.lab[nv] = cid[v];
            }
        }
        // rows in internal ids, sorted
        H.off.assign(n + 1, 0);
        for (int64_t nv = 0; nv < n; ++nv) {
            const int64_t v = H.new2old[nv];
            H.off[nv + 1] = H.off[nv] + ((int64_t)off[v + 1] - (int64_t)off[v]);
        }
        H.col.resize(nnz);
        parallel_for(n, 1024, [&](int64_t lo, int64_t hi) {
            for (int64_t nv = lo; nv < hi; ++nv) {
                const int64_t v = H.new2old[nv];
                const int64_t b = (int64_t)off[v], e = (int64_t)off[v + 1];
                int32_t *dst = H.col.data() + H.off[nv];
                for (int64_t i = b; i < e; ++i) dst[i - b] = H.old2new[col[i]];
                std::sort(dst, dst + (e - b));
            }
        });
        // tiles: row tiles bound the row capacity, score tiles the foreign
        // entries (own-community neighbours form the id range of the community)
        std::vector<int64_t> cap(n), fgn(n);
        parallel_for(n, 4096, [&](int64_t lo, int64_t hi) {
            for (int64_t nv = lo; nv < hi; ++nv) {
                const int32_t *b = H.col.data() + H.off[nv], *e = H.col.data() + H.off[nv + 1];
                const int32_t c = H.lab[nv];
                const int64_t own = std::lower_bound(b, e, (int32_t)start[c + 1]) - std::lower_bound(b, e, (int32_t)start[c]);
                cap[nv] = e - b;
                fgn[nv] = (e - b) - own;
            }
        });
        // out-lists: foreign neighbours of higher rank (foreign degree, id)
        H.oo.assign(n + 1, 0);
        auto higher = [&](int64_t x, int32_t y) { return fgn[y] > fgn[x] || (fgn[y] == fgn[x] && y > x); };
        auto foreign = [&](int64_t x, int32_t y) { return H.lab[y] != H.lab[x]; };
        parallel_for(n, 4096, [&](int64_t lo, int64_t hi) {
            for (int64_t x = lo; x < hi; ++x) {
                int64_t c = 0;
                for (int64_t j = H.off[x]; j < H.off[x + 1]; ++j) {
                    const int32_t y = H.col[j];
                    if (foreign(x, y) && higher(x, y)) ++c;
                }
                H.oo[x + 1] = c;
            }
        });
        for (int64_t x = 0; x < n; ++x) H.oo[x + 1] += H.oo[x];
        H.outl.resize(H.oo[n]);
        parallel_for(n, 4096, [&](int64_t lo, int64_t hi) {
            for (int64_t x = lo; x < hi; ++x) {
                int64_t o = H.oo[x];
                for (int64_t j = H.off[x]; j < H.off[x + 1]; ++j) {
                    const int32_t y = H.col[j];
                    if (foreign(x, y) && higher(x, y)) H.outl[o++] = y;
                }
            }
        });
        // link slots: u's foreign entries in row order (the links themselves
        // are built on the device)
        H.goff.assign(n + 1, 0);
        for (int64_t x = 0; x < n; ++x) H.goff[x + 1] = H.goff[x] + fgn[x];
        if (H.oo[n] > (int64_t)INT32_MAX) return fail(RS_ERR_RANGE, "out-lists exceed 32-bit offsets");
        H.cstart.resize(k + 1);
        for (int64_t c = 0; c <= k; ++c) H.cstart[c] = (int32_t)start[c];
        cut_all(n, H.off, cap, fgn, vstart, Tiling(), H);
    } catch (const std::bad_alloc &) {
        return fail(RS_ERR_NOMEM, "host allocation failed while renumbering the graph");
    }
    return RS_OK;
}

// keep: H stays intact for later uploads (its host maps are copied, not moved)
// Allocate and fill the schedule's device arrays, freeing any earlier
// ones: tiles and hubs, the per-block partials, the incremental re-score's
// unit flags and lists, and each vertex's row block and score unit.  Leaves
// the copies queued on the graph's stream.
static rs_status upload_tiles(rs_graph *g, const HostTiles &H) {
    DeviceGraph &D = g->d;
    void **tile_arrays[] = {(void **)&D.rtiles, (void **)&D.rhubs, (void **)&D.stiles, (void **)&D.shubs,
                            (void **)&D.shub_first, (void **)&D.shub_chunk, (void **)&D.hub_part,
                            (void **)&D.rflag, (void **)&D.cflag, (void **)&D.hflag, (void **)&D.rlist,
                            (void **)&D.slist, (void **)&D.hlist, (void **)&D.part_rows, (void **)&D.wmax_part,
                            (void **)&D.vrowb, (void **)&D.vscore, (void **)&D.hfilter};
    for (void **p : tile_arrays) dev_free(g, p);
    const size_t N = (size_t)std::max<int64_t>(D.n, 1);
    g->n_rtiles = (int)H.rtiles.size();
    g->n_rhubs = (int)H.rhubs.size();
    g->n_stiles = (int)H.stiles.size();
    g->n_shubs = (int)H.shubs.size();
    g->n_schunks = (int)H.schunk.size();
    g->n_schunks_lds = H.n_chunks_lds;
    g->n_shubs_lds = H.n_hubs_lds;
    g->grid_rows = tile_grid(g->n_rhubs, g->n_rtiles);
    g->grid_score = tile_grid(g->n_schunks, g->n_stiles);
    const size_t nch = std::max<size_t>(H.schunk.size(), 1);
    const size_t nrt = std::max<size_t>(H.rtiles.size(), 1), nrh = std::max<size_t>(H.rhubs.size(), 1);
    const size_t nst = std::max<size_t>(H.stiles.size(), 1), nsh = std::max<size_t>(H.shubs.size(), 1);
    const size_t gr = (size_t)std::max(g->grid_rows, 1), gs = (size_t)std::max(g->grid_score, 1);
    struct Req {
        void **p;
        size_t bytes;
    } reqs[] = {
        {(void **)&D.rtiles, sizeof(RowTile) * nrt},
        {(void **)&D.rhubs, 4 * nrh},
        {(void **)&D.stiles, sizeof(int2) * nst},
        {(void **)&D.shubs, 4 * nsh},
        {(void **)&D.shub_first, 4 * (nsh + 1)},
        {(void **)&D.shub_chunk, sizeof(int2) * nch},
        {(void **)&D.hub_part, sizeof(HubPart) * nch},
        {(void **)&D.rflag, gr},
        {(void **)&D.cflag, nch},
        {(void **)&D.hflag, nsh},
        {(void **)&D.rlist, 4 * gr},
        {(void **)&D.slist, 4 * gs},
        {(void **)&D.hlist, 4 * nch},
        {(void **)&D.part_rows, sizeof(RowPart) * gr},
        {(void **)&D.wmax_part, 8 * gr},
        {(void **)&D.vrowb, 4 * N},
        {(void **)&D.vscore, 4 * N},
        {(void **)&D.hfilter, 4 * (size_t)kFilterWords * std::max<size_t>(H.shubs.size() - H.n_hubs_lds, 1)},
    };
    for (auto &r : reqs) {
        hipError_t e = dev_alloc(g, r.p, r.bytes);
        if (e != hipSuccess) return hip_fail(e, "device allocation");
    }
    hipStream_t s = g->stream;
    hipError_t e = hipSuccess;
    auto put = [&](void *dst, const void *src, size_t bytes) {
        if (e == hipSuccess && bytes) e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s);
    };
    put(D.rtiles, H.rtiles.data(), sizeof(RowTile) * H.rtiles.size());
    put(D.rhubs, H.rhubs.data(), 4 * H.rhubs.size());
    put(D.stiles, H.stiles.data(), sizeof(int2) * H.stiles.size());
    put(D.shubs, H.shubs.data(), 4 * H.shubs.size());
    put(D.shub_first, H.sfirst.data(), 4 * H.sfirst.size());
    put(D.shub_chunk, H.schunk.data(), sizeof(int2) * H.schunk.size());
    put(D.vrowb, H.vrowb.data(), 4 * H.vrowb.size());
    put(D.vscore, H.vscore.data(), 4 * H.vscore.size());
    if (e == hipSuccess) e = hipMemsetAsync(D.rflag, 0, gr, s);
    if (e == hipSuccess) e = hipMemsetAsync(D.cflag, 0, nch, s);
    if (e == hipSuccess) e = hipMemsetAsync(D.hflag, 0, nsh, s);
    return e == hipSuccess ? RS_OK : hip_fail(e, "schedule upload");
}

static rs_status upload(rs_graph *g, HostGraph &H, int64_t n, int64_t nnz, bool keep = false) {
    DeviceGraph &D = g->d;
    D.n = n;
    D.nnz = nnz;
    D.k = (int32_t)H.comm2orig.size();
    D.off64 = nnz > (int64_t)INT32_MAX || g->wide_offsets;
    if (H.outl.size() >= ((size_t)1 << 30))
        return fail(RS_ERR_RANGE, "more than 2^30 edges between communities (out-list positions are 30-bit in hit records)");
    g->n_out = (int64_t)H.outl.size();
    const size_t N = (size_t)std::max<int64_t>(n, 1), Z = (size_t)std::max<int64_t>(nnz, 1);
    const size_t offb = D.off64 ? 8 : 4;
    struct Req {
        void **p;
        size_t bytes;
    } reqs[] = {
        {&D.off, offb * (N + 1)},
        {(void **)&D.deg, 4 * N},
        {(void **)&D.col, 4 * Z},
        {(void **)&D.clab, 4 * Z},
        {(void **)&D.lab, 4 * N},
        {(void **)&D.new2old, 4 * N},
        {(void **)&D.alive, N},
        {(void **)&D.oo, 8 * (N + 1)},
        {(void **)&D.goff, 8 * (N + 1)},
        {(void **)&D.prec, sizeof(PairRec) * Z},
        {(void **)&D.plink, sizeof(PairLink) * std::max<size_t>((size_t)H.goff[n], 1)},
        {(void **)&D.cstart, 4 * H.cstart.size()},
        {(void **)&D.wpart, 8 * (size_t)kWorkBlocks},
        {(void **)&D.raw, 8 * N},
        {(void **)&D.vmark, 4 * N},
        {(void **)&D.elist, 4 * N},
        {(void **)&D.ucnt, 4 * (size_t)kUnitRows * kUnitGroups},
        {(void **)&D.abin, 4 * N},
        {(void **)&D.echunk, sizeof(int2) * (N + Z / 64 + 1)},
        {(void **)&D.ictr, 8 * (size_t)kIcCount},
        {(void **)&D.wblk, 8 * 64},
        {(void **)&D.wticket, 8},
        {(void **)&g->rem_cnt, 8 * 4},
        {(void **)&D.outl, 4 * std::max<size_t>(H.outl.size(), 1)},
        {(void **)&D.oe, sizeof(OutEnt) * std::max<size_t>(H.outl.size(), 1)},
        {(void **)&D.reckey, 4 * Z},
        {(void **)&D.recdat, sizeof(RecDat) * Z},
        {(void **)&D.card, sizeof(VCard) * N},
        {(void **)&D.wown, 8 * N},
        {(void **)&D.av, 8 * N},
        {(void **)&D.R, 8 * N},
        {(void **)&D.tI, 8 * N},
        {(void **)&D.tII, 8 * N},
        {(void **)&D.ctr, sizeof(DevCounters)},
        {(void **)&D.thist, 4 * (size_t)kTopkBins},
        {(void **)&D.thist_c, 4 * 256},
        {(void **)&D.tstate, sizeof(TopkState)},
        {(void **)&D.tfinal, sizeof(TopkKey) * N},
        {(void **)&D.ttie, sizeof(TopkKey) * N},
        {(void **)&D.ttie2, sizeof(TopkKey) * N},
        {(void **)&D.tout_ids, 4 * N},
        {(void **)&D.tout_sc, 8 * N},
        {(void **)&D.scratch_d, 8 * N},
        {(void **)&D.tblk, 16 + 16 * N},
        {(void **)&D.scratch_u, 8 * 8},
    };
    for (auto &r : reqs) {
        hipError_t e = dev_alloc(g, r.p, r.bytes);
        if (e != hipSuccess) return hip_fail(e, "device allocation");
    }
    {
        const hipError_t eh = hipHostMalloc((void **)&g->rem_cnt_host, 8 * (4 + (size_t)kIcCount), hipHostMallocDefault);
        if (eh != hipSuccess) {
            g->rem_cnt_host = nullptr;
            return hip_fail(eh, "pinned counters");
        }
        const hipError_t ee = hipEventCreateWithFlags(&g->rem_ev, hipEventDisableTiming);
        if (ee != hipSuccess) {
            g->rem_ev = nullptr;
            return hip_fail(ee, "removal event");
        }
    }
    std::vector<int32_t> off32, deg(n);
    for (int64_t v = 0; v < n; ++v) deg[v] = (int32_t)(H.off[v + 1] - H.off[v]);
    const void *offsrc = H.off.data();
    if (!D.off64) {
        off32.resize(n + 1);
        for (int64_t v = 0; v <= n; ++v) off32[v] = (int32_t)H.off[v];
        offsrc = off32.data();
    }
    hipStream_t s = g->stream;
    hipError_t e = hipMemcpyAsync(D.off, offsrc, offb * (n + 1), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && n) e = hipMemcpyAsync(D.deg, deg.data(), 4 * n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && nnz) e = hipMemcpyAsync(D.col, H.col.data(), 4 * nnz, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && n) e = hipMemcpyAsync(D.lab, H.lab.data(), 4 * n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && n) e = hipMemcpyAsync(D.new2old, H.new2old.data(), 4 * n, hipMemcpyHostToDevice, s);
    auto put = [&](void *dst, const void *src, size_t bytes) {
        if (e == hipSuccess && bytes) e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s);
    };
    put(D.oo, H.oo.data(), 8 * H.oo.size());
    put(D.goff, H.goff.data(), 8 * H.goff.size());
    put(D.cstart, H.cstart.data(), 4 * H.cstart.size());
    std::vector<VCard> cards;
    try {
        cards.resize(n);
    } catch (const std::bad_alloc &) {
        return fail(RS_ERR_NOMEM, "host allocation failed while building vertex cards");
    }
    for (int64_t v = 0; v < n; ++v) {
        VCard &c = cards[v];
        memset(&c, 0, sizeof(c));
        c.off = H.off[v];
        c.goff = H.goff[v];
        c.lab = H.lab[v];
    }
    put(D.card, cards.data(), sizeof(VCard) * cards.size());
    if (e == hipSuccess && n) e = hipStreamSynchronize(s);  // the host cards must outlive the copy
    put(D.outl, H.outl.data(), 4 * H.outl.size());
    if (e == hipSuccess) e = hipMemsetAsync(D.alive, 1, N, s);
    if (e == hipSuccess) e = hipMemsetAsync(D.vmark, 0, 4 * N, s);
    if (e == hipSuccess) e = hipMemsetAsync(D.thist, 0, 4 * (size_t)kTopkBins, s);
    if (e == hipSuccess) e = hipMemsetAsync(D.thist_c, 0, 4 * 256, s);
    if (e == hipSuccess) e = hipMemsetAsync(D.ctr, 0, sizeof(DevCounters), s);
    if (e == hipSuccess) e = hipMemsetAsync(D.wticket, 0, 8, s);
    if (e == hipSuccess) e = hipMemsetAsync(D.tstate, 0, sizeof(TopkState), s);
    if (e != hipSuccess) return hip_fail(e, "graph upload");
    const rs_status tst = upload_tiles(g, H);
    if (tst != RS_OK) return tst;
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "graph upload");
    const rs_status lst = launch_col_labels(g);  // each entry's neighbour community
    if (lst != RS_OK) return lst;
    const rs_status rst = launch_links(g);  // each G' entry's reverse entry and out-list range
    if (rst != RS_OK) return rst;
    const rs_status ost = launch_out_entries(g);  // each out-list entry's two row entries
    if (ost != RS_OK) return ost;
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "pair-slot map");
    if (keep) {
        try {
            g->h_new2old = H.new2old;
            g->h_old2new = H.old2new;
            g->h_comm2orig = H.comm2orig;
        } catch (const std::bad_alloc &) {
            return fail(RS_ERR_NOMEM, "host maps");
        }
    } else {
        g->h_new2old.swap(H.new2old);
        g->h_old2new.swap(H.old2new);
        g->h_comm2orig.swap(H.comm2orig);
    }
    g->n_alive = n;
    return RS_OK;
}

template <class OffIn>
static rs_status load_t(const rs_csr *csr, rs_graph *g) {
    const int64_t n = csr->n, nnz = csr->nnz;
    const OffIn *off = (const OffIn *)csr->row_offsets;
    const int32_t *col = csr->col, *lab = csr->labels;
    std::vector<OffIn> h_off;
    std::vector<int32_t> h_col, h_lab;
    if (csr->on_device) {
        try {
            h_off.resize(n + 1);
            h_col.resize(nnz);
            h_lab.resize(n);
        } catch (const std::bad_alloc &) {
            return fail(RS_ERR_NOMEM, "host staging allocation failed");
        }
        hipError_t e = hipMemcpy(h_off.data(), off, sizeof(OffIn) * (n + 1), hipMemcpyDeviceToHost);
        if (e == hipSuccess && nnz) e = hipMemcpy(h_col.data(), col, 4 * nnz, hipMemcpyDeviceToHost);
        if (e == hipSuccess && n) e = hipMemcpy(h_lab.data(), lab, 4 * n, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "copying the device-resident input graph");
        off = h_off.data();
        col = h_col.data();
        lab = h_lab.data();
    }
    rs_status st = validate_graph<OffIn>(n, nnz, off, col, lab);
    if (st != RS_OK) return st;
    HostGraph H;
    st = build_internal<OffIn>(n, nnz, off, col, lab, g->h_vstart, H);
    if (st != RS_OK) return st;
    g->h_gblk_off.swap(H.gblk_off);
    g->h_gblk.swap(H.gblk);
    hipError_t e = hipGetDevice(&g->device);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (!g->stream) {
        e = hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
        g->own_stream = true;
    }
    return upload(g, H, n, nnz);
}

// A validated, renumbered and tiled host form of a graph, kept by the
// request server so that a graph evicted from device memory is reloaded by
// an upload alone.
struct Prebuilt {
    HostGraph H;
    int64_t n = 0, nnz = 0;
};

rs_status prebuild_graph(const rs_csr *csr, Prebuilt **out) {
    if (!out || !csr) return fail(RS_ERR_ARG, "csr or out is NULL");
    *out = nullptr;
    if (csr->on_device || csr->offset_bytes != 8) return fail(RS_ERR_ARG, "prebuilt graphs take host int64 offsets");
    if (csr->n < 0 || csr->nnz < 0 || csr->n > (int64_t)INT32_MAX - 1) return fail(RS_ERR_RANGE, "n or nnz out of range");
    if (!csr->row_offsets || (csr->n > 0 && !csr->labels) || (csr->nnz > 0 && !csr->col))
        return fail(RS_ERR_ARG, "null CSR array");
    const int64_t *off = (const int64_t *)csr->row_offsets;
    rs_status st = validate_graph<int64_t>(csr->n, csr->nnz, off, csr->col, csr->labels);
    if (st != RS_OK) return st;
    Prebuilt *P = new (std::nothrow) Prebuilt();
    if (!P) return fail(RS_ERR_NOMEM, "prebuilt graph");
    st = build_internal<int64_t>(csr->n, csr->nnz, off, csr->col, csr->labels, std::vector<int64_t>(), P->H);
    if (st != RS_OK) {
        delete P;
        return st;
    }
    P->n = csr->n;
    P->nnz = csr->nnz;
    *out = P;
    return RS_OK;
}

rs_status load_prebuilt(Prebuilt *P, void *hip_stream, rs_graph **out) {
    if (!P || !out) return fail(RS_ERR_ARG, "prebuilt graph or out is NULL");
    *out = nullptr;
    rs_graph *g = new (std::nothrow) rs_graph();
    if (!g) return fail(RS_ERR_NOMEM, "handle allocation failed");
    g->stream = (hipStream_t)hip_stream;
    if (const char *gv = std::getenv("RS_GRAPHS")) g->graphs_off = gv[0] == '0';
    hipError_t e = hipGetDevice(&g->device);
    rs_status st = e == hipSuccess ? RS_OK : hip_fail(e, "hipGetDevice");
    if (st == RS_OK && !g->stream) {
        e = hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking);
        if (e == hipSuccess)
            g->own_stream = true;
        else
            st = hip_fail(e, "hipStreamCreate");
    }
    if (st == RS_OK) st = upload(g, P->H, P->n, P->nnz, true);
    if (st != RS_OK) {
        std::string keep = g_err;
        release(g);
        delete g;
        g_err = keep;
        return st;
    }
    *out = g;
    return RS_OK;
}

void free_prebuilt(Prebuilt *P) { delete P; }

template <class T>
static hipError_t d2h(std::vector<T> &dst, const void *src, int64_t count);

// The last pass's row facts {deg, ell, p, q} of every vertex (internal ids).
static hipError_t read_meta(rs_graph *g, std::vector<VMeta> &meta) {
    std::vector<VCard> cards;
    const hipError_t e = d2h(cards, g->d.card, g->d.n);
    if (e != hipSuccess) return e;
    meta.resize(cards.size());
    for (size_t v = 0; v < cards.size(); ++v) meta[v] = cards[v].m;
    return hipSuccess;
}

template <class T>
static hipError_t d2h(std::vector<T> &dst, const void *src, int64_t count) {
    dst.resize(count);
    if (!count) return hipSuccess;
    return hipMemcpy(dst.data(), src, sizeof(T) * count, hipMemcpyDeviceToHost);
}

static hipError_t read_offsets(rs_graph *g, std::vector<int64_t> &off) {
    const int64_t n = g->d.n;
    if (g->d.off64) return d2h(off, g->d.off, n + 1);
    std::vector<int32_t> o32;
    hipError_t e = d2h(o32, g->d.off, n + 1);
    off.assign(o32.begin(), o32.end());
    return e;
}

}  // namespace rs

using namespace rs;

// ================================================================== C ABI
// ------------------------------------------------------------ tiling
static rs_status check_tiling(const rs_tiling *t) {
    if (!t) return fail(RS_ERR_ARG, "tiling is NULL");
    if (t->row_entries < 64 || t->row_entries > kRowTile || t->row_vertices < 1 || t->row_vertices > kRowTileV ||
        t->score_pairs < 1 || t->score_pairs > kScoreTileP || t->score_vertices < 1 ||
        t->score_vertices > kScoreTileV || t->hub_list < 1 || t->hub_list > kHubList)
        return fail(RS_ERR_ARG, "tiling out of range: row_entries 64.." + std::to_string(kRowTile) +
                                    ", row_vertices 1.." + std::to_string(kRowTileV) + ", score_pairs 1.." +
                                    std::to_string(kScoreTileP) + ", score_vertices 1.." +
                                    std::to_string(kScoreTileV) + ", hub_list 1.." + std::to_string(kHubList));
    return RS_OK;
}

static Tiling to_tiling(const rs_tiling *t) {
    Tiling T;
    T.row_entries = t->row_entries;
    T.row_vertices = t->row_vertices;
    T.score_pairs = t->score_pairs;
    T.score_vertices = t->score_vertices;
    T.hub_list = t->hub_list;
    return T;
}

// Re-cut the schedule of a resident graph for the tiling T.  The cut needs
// each vertex's row capacity and load-time foreign degree, which the device
// keeps as the capacity layout and the pair-slot offsets; the tiles are cut
// on the host and the schedule's arrays replaced.  Captured replays are
// dropped (their grids change), and the graph must be scored again.
static rs_status retile(rs_graph *g, const Tiling &T) {
    DeviceGraph &D = g->d;
    const int64_t n = D.n;
    hipError_t e = hipStreamSynchronize(g->stream);
    if (e != hipSuccess) return hip_fail(e, "retile");
    std::vector<int64_t> off, goff, cap, fgn;
    HostTiles X;
    try {
        off.resize(n + 1);
        goff.resize(n + 1);
        cap.resize(n);
        fgn.resize(n);
        if (D.off64) {
            e = hipMemcpy(off.data(), D.off, 8 * (size_t)(n + 1), hipMemcpyDeviceToHost);
        } else {
            std::vector<int32_t> o32(n + 1);
            e = hipMemcpy(o32.data(), D.off, 4 * (size_t)(n + 1), hipMemcpyDeviceToHost);
            for (int64_t v = 0; v <= n; ++v) off[v] = o32[v];
        }
        if (e == hipSuccess) e = hipMemcpy(goff.data(), D.goff, 8 * (size_t)(n + 1), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "retile: reading the capacity layout");
        for (int64_t v = 0; v < n; ++v) {
            cap[v] = off[v + 1] - off[v];
            fgn[v] = goff[v + 1] - goff[v];
        }
        cut_all(n, off, cap, fgn, g->h_vstart, T, X);
    } catch (const std::bad_alloc &) {
        return fail(RS_ERR_NOMEM, "host allocation failed while cutting tiles");
    }
    release_replays(g);
    rs_status st = upload_tiles(g, X);
    if (st == RS_OK && g->n_graphs > 0) {  // a batch's row blocks of each graph
        dev_free(g, (void **)&D.gblk_off);
        dev_free(g, (void **)&D.gblk);
        e = dev_alloc(g, (void **)&D.gblk_off, 4 * X.gblk_off.size());
        if (e == hipSuccess) e = dev_alloc(g, (void **)&D.gblk, 4 * std::max<size_t>(X.gblk.size(), 1));
        if (e == hipSuccess)
            e = hipMemcpyAsync(D.gblk_off, X.gblk_off.data(), 4 * X.gblk_off.size(), hipMemcpyHostToDevice, g->stream);
        if (e == hipSuccess && !X.gblk.empty())
            e = hipMemcpyAsync(D.gblk, X.gblk.data(), 4 * X.gblk.size(), hipMemcpyHostToDevice, g->stream);
        if (e != hipSuccess) st = hip_fail(e, "retile: batch row blocks");
        g->h_gblk_off.swap(X.gblk_off);
        g->h_gblk.swap(X.gblk);
    }
    if (st == RS_OK) {
        e = hipStreamSynchronize(g->stream);
        if (e != hipSuccess) st = hip_fail(e, "retile");
    }
    g->tiling = T;
    g->scored = false;
    return st;
}

extern "C" {

const char *rs_status_string(rs_status s) {
    switch (s) {
        case RS_OK: return "RS_OK";
        case RS_ERR_ARG: return "RS_ERR_ARG";
        case RS_ERR_GRAPH: return "RS_ERR_GRAPH";
        case RS_ERR_RANGE: return "RS_ERR_RANGE";
        case RS_ERR_NOMEM: return "RS_ERR_NOMEM";
        case RS_ERR_HIP: return "RS_ERR_HIP";
        case RS_ERR_STATE: return "RS_ERR_STATE";
        default: return "RS_ERR_UNKNOWN";
    }
}

const char *rs_last_error(void) { return g_err.c_str(); }

// A batch passes its graph starts (n_graphs + 1 entries), else vstart is NULL.
static rs_status load_graph(const rs_csr *csr, void *hip_stream, uint32_t flags, const int64_t *vstart,
                            int32_t n_graphs, rs_graph **out) {
    if (!out) return fail(RS_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!csr) return fail(RS_ERR_ARG, "csr is NULL");
    if ((flags & ~RS_LOAD_WIDE_OFFSETS) != 0) return fail(RS_ERR_ARG, "unknown flags");
    if (csr->n < 0 || csr->nnz < 0) return fail(RS_ERR_ARG, "negative n or nnz");
    if (csr->offset_bytes != 4 && csr->offset_bytes != 8) return fail(RS_ERR_ARG, "offset_bytes must be 4 or 8");
    if (csr->on_device != 0 && csr->on_device != 1) return fail(RS_ERR_ARG, "on_device must be 0 or 1");
    if (!csr->row_offsets) return fail(RS_ERR_ARG, "row_offsets is NULL");
    if (csr->n > 0 && !csr->labels) return fail(RS_ERR_ARG, "labels is NULL");
    if (csr->nnz > 0 && !csr->col) return fail(RS_ERR_ARG, "col is NULL");
    if (csr->n > (int64_t)INT32_MAX - 1) return fail(RS_ERR_RANGE, "n does not fit int32 vertex ids");
    if (csr->offset_bytes == 4 && csr->nnz > (int64_t)INT32_MAX)
        return fail(RS_ERR_RANGE, "nnz overflows 4-byte row offsets");
    rs_graph *g = new (std::nothrow) rs_graph();
    if (!g) return fail(RS_ERR_NOMEM, "handle allocation failed");
    g->stream = (hipStream_t)hip_stream;  // NULL: created after validation
    g->wide_offsets = (flags & RS_LOAD_WIDE_OFFSETS) != 0;
    if (const char *gv = std::getenv("RS_GRAPHS")) g->graphs_off = gv[0] == '0';
    if (vstart) {
        g->n_graphs = n_graphs;
        g->h_vstart.assign(vstart, vstart + n_graphs + 1);
    }
    rs_status st = csr->offset_bytes == 8 ? load_t<int64_t>(csr, g) : load_t<int32_t>(csr, g);
    if (st != RS_OK) {
        std::string keep = g_err;
        release(g);
        delete g;
        g_err = keep;
        return st;
    }
    *out = g;
    return RS_OK;
}

rs_status rs_load_graph(const rs_csr *csr, void *hip_stream, uint32_t flags, rs_graph **out) {
    clear_error();
    return load_graph(csr, hip_stream, flags, nullptr, 0, out);
}

rs_status rs_load_batch(int32_t n_graphs, const int64_t *vertex_offsets, const rs_csr *csr, void *hip_stream,
                        uint32_t flags, rs_graph **out) {
    clear_error();
    if (!out) return fail(RS_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (n_graphs < 1 || !vertex_offsets || !csr) return fail(RS_ERR_ARG, "n_graphs < 1, or a NULL array");
    if (csr->on_device) return fail(RS_ERR_ARG, "a batch is loaded from host arrays");
    if (csr->n < 0 || csr->nnz < 0) return fail(RS_ERR_ARG, "negative n or nnz");
    if (csr->offset_bytes != 4 && csr->offset_bytes != 8) return fail(RS_ERR_ARG, "offset_bytes must be 4 or 8");
    if (!csr->row_offsets || (csr->n > 0 && !csr->labels) || (csr->nnz > 0 && !csr->col))
        return fail(RS_ERR_ARG, "null CSR array");
    const int64_t n = csr->n;
    if (vertex_offsets[0] != 0 || vertex_offsets[n_graphs] != n) return fail(RS_ERR_ARG, "vertex_offsets must run 0..n");
    for (int32_t gi = 0; gi < n_graphs; ++gi)
        if (vertex_offsets[gi + 1] < vertex_offsets[gi]) return fail(RS_ERR_ARG, "vertex_offsets decrease");
    auto rowoff = [&](int64_t v) {
        return csr->offset_bytes == 8 ? ((const int64_t *)csr->row_offsets)[v]
                                      : (int64_t)((const int32_t *)csr->row_offsets)[v];
    };
    // the row offsets first: the scan below walks every row
    if (rowoff(0) != 0) return fail(RS_ERR_GRAPH, "row_offsets[0] != 0");
    for (int64_t v = 0; v < n; ++v)
        if (rowoff(v + 1) < rowoff(v)) return fail(RS_ERR_GRAPH, "row_offsets decrease at vertex " + std::to_string(v));
    if (rowoff(n) != csr->nnz) return fail(RS_ERR_GRAPH, "row_offsets[n] != nnz");
    // every edge stays inside its graph; labels are ranked per graph and
    // offset so that no community spans two graphs (the ranks keep each
    // graph's label order, hence its internal numbering)
    std::vector<int32_t> lab2;
    try {
        lab2.resize(n);
        int64_t base = 0;
        for (int32_t gi = 0; gi < n_graphs; ++gi) {
            const int64_t a = vertex_offsets[gi], b = vertex_offsets[gi + 1];
            for (int64_t v = a; v < b; ++v)
                for (int64_t e = rowoff(v); e < rowoff(v + 1); ++e)
                    if (csr->col[e] < a || csr->col[e] >= b) return fail(RS_ERR_GRAPH, "an edge joins two graphs of the batch");
            std::vector<int32_t> u(csr->labels + a, csr->labels + b);
            std::sort(u.begin(), u.end());
            u.erase(std::unique(u.begin(), u.end()), u.end());
            for (int64_t v = a; v < b; ++v) {
                if (csr->labels[v] < 0) return fail(RS_ERR_GRAPH, "negative label");
                lab2[v] = (int32_t)(base + (std::lower_bound(u.begin(), u.end(), csr->labels[v]) - u.begin()));
            }
            base += (int64_t)u.size();
            if (base > (int64_t)INT32_MAX) return fail(RS_ERR_RANGE, "too many communities in the batch");
        }
    } catch (const std::bad_alloc &) {
        return fail(RS_ERR_NOMEM, "host staging of the batch failed");
    }
    rs_csr c = *csr;
    c.labels = lab2.data();
    rs_graph *g = nullptr;
    rs_status st = load_graph(&c, hip_stream, flags, vertex_offsets, n_graphs, &g);
    if (st != RS_OK) return st;
    DeviceGraph &D = g->d;
    std::vector<int32_t> vg(n);
    for (int32_t gi = 0; gi < n_graphs; ++gi)
        for (int64_t v = vertex_offsets[gi]; v < vertex_offsets[gi + 1]; ++v) vg[v] = gi;
    const size_t N = (size_t)std::max<int64_t>(n, 1), G = (size_t)n_graphs;
    struct Req {
        void **p;
        size_t bytes;
    } reqs[] = {
        {(void **)&D.vstart, 8 * (G + 1)},
        {(void **)&D.vgraph, 4 * N},
        {(void **)&D.gwmax, 8 * G},
        {(void **)&D.gblk_off, 4 * (G + 1)},
        {(void **)&D.gorder, 4 * G},
        {(void **)&D.gblk, 4 * std::max<size_t>(g->h_gblk.size(), 1)},
        {(void **)&D.bids, 4 * G * kBatchK},
        {(void **)&D.bscores, 8 * G * kBatchK},
        {(void **)&D.bcounts, 8 * G},
    };
    hipError_t e = hipSuccess;
    for (auto &r : reqs) {
        e = dev_alloc(g, r.p, r.bytes);
        if (e != hipSuccess) break;
    }
    if (e == hipSuccess) e = hipMemcpyAsync(D.vstart, vertex_offsets, 8 * (G + 1), hipMemcpyHostToDevice, g->stream);
    if (e == hipSuccess && n) e = hipMemcpyAsync(D.vgraph, vg.data(), 4 * n, hipMemcpyHostToDevice, g->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(D.gblk_off, g->h_gblk_off.data(), 4 * (G + 1), hipMemcpyHostToDevice, g->stream);
    // top-k segments, when every graph has at most kSegMax of them
    int64_t nmax = 0;
    for (size_t i = 0; i < G; ++i) nmax = std::max<int64_t>(nmax, vertex_offsets[i + 1] - vertex_offsets[i]);
    std::vector<int32_t> seg_g, sfirst(G + 1, 0);
    if (nmax <= (int64_t)kSegVerts * kSegMax) {
        for (size_t i = 0; i < G; ++i) {
            const int64_t ns = (vertex_offsets[i + 1] - vertex_offsets[i] + kSegVerts - 1) / kSegVerts;
            for (int64_t j = 0; j < ns; ++j) seg_g.push_back((int32_t)i);
            sfirst[i + 1] = (int32_t)seg_g.size();
        }
    }
    const size_t S = seg_g.size();
    if (e == hipSuccess && S > 0) {
        struct Req2 {
            void **p;
            size_t bytes;
        } more[] = {
            {(void **)&D.seg_g, 4 * S},
            {(void **)&D.sfirst, 4 * (G + 1)},
            {(void **)&D.c_hi, 8 * S * kBatchK},
            {(void **)&D.c_lo, 4 * S * kBatchK},
            {(void **)&D.c_cnt, 4 * S},
        };
        for (auto &r : more) {
            e = dev_alloc(g, r.p, r.bytes);
            if (e != hipSuccess) break;
        }
        if (e == hipSuccess) e = hipMemcpyAsync(D.seg_g, seg_g.data(), 4 * S, hipMemcpyHostToDevice, g->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(D.sfirst, sfirst.data(), 4 * (G + 1), hipMemcpyHostToDevice, g->stream);
        if (e == hipSuccess) g->n_segs = (int32_t)S;
    }
    std::vector<int32_t> order(G);
    for (size_t i = 0; i < G; ++i) order[i] = (int32_t)i;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        return vertex_offsets[a + 1] - vertex_offsets[a] > vertex_offsets[b + 1] - vertex_offsets[b];
    });
    if (e == hipSuccess) e = hipMemcpyAsync(D.gorder, order.data(), 4 * G, hipMemcpyHostToDevice, g->stream);
    if (e == hipSuccess && !g->h_gblk.empty())
        e = hipMemcpyAsync(D.gblk, g->h_gblk.data(), 4 * g->h_gblk.size(), hipMemcpyHostToDevice, g->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    if (e != hipSuccess) {
        st = hip_fail(e, "batch upload");
        std::string keep = g_err;
        rs_free_graph(g);
        g_err = keep;
        return st;
    }
    *out = g;
    return RS_OK;
}

rs_status rs_topk_batch(rs_graph *g, int64_t k, int32_t *ids, double *scores, int64_t *counts) {
    clear_error();
    if (!g || !ids || !scores || !counts) return fail(RS_ERR_ARG, "graph or an output is NULL");
    if (g->n_graphs <= 0) return fail(RS_ERR_STATE, "not a batch");
    if (k < 1 || k > kBatchK) return fail(RS_ERR_ARG, "k must be 1.." + std::to_string(kBatchK));
    if (!g->scored) return fail(RS_ERR_STATE, "rs_topk_batch before rs_score");
    rs_status st = launch_topk_graphs(g, k, g->d.bids, g->d.bscores, g->d.bcounts);
    if (st != RS_OK) return st;
    const size_t G = (size_t)g->n_graphs;
    hipError_t e = hipMemcpyAsync(ids, g->d.bids, 4 * G * (size_t)k, hipMemcpyDeviceToHost, g->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(scores, g->d.bscores, 8 * G * (size_t)k, hipMemcpyDeviceToHost, g->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(counts, g->d.bcounts, 8 * G, hipMemcpyDeviceToHost, g->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    return e == hipSuccess ? RS_OK : hip_fail(e, "batched top-k copy");
}

void rs_free_graph(rs_graph *g) {
    if (!g) return;
    if (g->stream) (void)hipStreamSynchronize(g->stream);
    release(g);
    delete g;
}

rs_status rs_score(rs_graph *g) {
    clear_error();
    if (!g) return fail(RS_ERR_ARG, "graph is NULL");
    rs_status st = launch_score_pass(g);
    if (st == RS_OK) g->scored = true;
    return st;
}

rs_status rs_topk(rs_graph *g, int64_t k, int32_t *ids, double *scores, int64_t *count) {
    clear_error();
    if (!g || !count) return fail(RS_ERR_ARG, "graph or count is NULL");
    if (k < 0) return fail(RS_ERR_ARG, "k < 0");
    if (k > 0 && (!ids || !scores)) return fail(RS_ERR_ARG, "ids or scores is NULL");
    if (!g->scored) return fail(RS_ERR_STATE, "rs_topk before rs_score");
    int64_t cnt = 0;
    rs_status st = launch_topk(g, k, ids, scores, &cnt);
    if (st != RS_OK) return st;
    *count = cnt;
    return RS_OK;
}

rs_status rs_apply_removals(rs_graph *g, const rs_removals *b, rs_removal_result *res) {
    clear_error();
    if (!g || !b) return fail(RS_ERR_ARG, "graph or batch is NULL");
    if (!g->scored) return fail(RS_ERR_STATE, "rs_apply_removals before rs_score");
    if (g->n_graphs > 0) return fail(RS_ERR_STATE, "removals are not applied to a batch of graphs");
    if (b->n_edges < 0 || b->n_vertices < 0) return fail(RS_ERR_ARG, "negative batch size");
    if (b->n_edges > 0 && (!b->src || !b->dst)) return fail(RS_ERR_ARG, "edge arrays are NULL");
    if (b->n_vertices > 0 && !b->vertices) return fail(RS_ERR_ARG, "vertex array is NULL");
    const int64_t n = g->d.n;
    std::vector<int32_t> es, ed, vs;
    try {
        es.resize(b->n_edges);
        ed.resize(b->n_edges);
        vs.resize(b->n_vertices);
    } catch (const std::bad_alloc &) {
        return fail(RS_ERR_NOMEM, "host staging allocation failed");
    }
    for (int64_t i = 0; i < b->n_edges; ++i) {
        const int32_t a = b->src[i], c = b->dst[i];
        if (a < 0 || a >= n || c < 0 || c >= n) return fail(RS_ERR_RANGE, "edge endpoint out of range");
        es[i] = g->h_old2new[a];
        ed[i] = g->h_old2new[c];
    }
    for (int64_t i = 0; i < b->n_vertices; ++i) {
        const int32_t x = b->vertices[i];
        if (x < 0 || x >= n) return fail(RS_ERR_RANGE, "vertex id out of range");
        vs[i] = g->h_old2new[x];
    }
    std::sort(vs.begin(), vs.end());
    vs.erase(std::unique(vs.begin(), vs.end()), vs.end());
    const int64_t m = b->n_edges, nv = (int64_t)vs.size();
    const int64_t need = std::max<int64_t>(2 * m + nv, 1);
    // staging kept between calls: grown (never shrunk) before anything is mutated
    if (need > g->rem_cap || need > g->rem_host_cap) {
        const int64_t cap = std::max<int64_t>(2 * need, 4096);
        int32_t *nb = nullptr, *nh = nullptr;
        hipError_t ea = hipMalloc((void **)&nb, 4 * (size_t)cap);
        if (ea == hipSuccess) ea = hipHostMalloc((void **)&nh, 4 * (size_t)cap, hipHostMallocDefault);
        if (ea != hipSuccess) {
            if (nb) (void)hipFree(nb);
            return hip_fail(ea, "removal staging");
        }
        if (g->rem_buf) (void)hipFree(g->rem_buf);
        if (g->rem_host) (void)hipHostFree(g->rem_host);
        g->dev_bytes += 4 * (cap - g->rem_cap);  // the device staging counts toward the graph's footprint
        g->rem_buf = nb;
        g->rem_host = nh;
        g->rem_cap = g->rem_host_cap = cap;
    }
    std::copy(es.begin(), es.end(), g->rem_host);
    std::copy(ed.begin(), ed.end(), g->rem_host + m);
    std::copy(vs.begin(), vs.end(), g->rem_host + 2 * m);
    int32_t *d_buf = g->rem_buf;
    unsigned long long *d_cnt = g->rem_cnt;
    hipError_t e = hipMemcpyAsync(d_buf, g->rem_host, 4 * (size_t)(2 * m + nv), hipMemcpyHostToDevice, g->stream);
    if (e == hipSuccess) e = hipMemsetAsync(d_cnt, 0, 4 * sizeof(unsigned long long), g->stream);
    if (e == hipSuccess) e = hipMemsetAsync(g->d.ictr, 0, 8 * (size_t)kIcCount, g->stream);
    rs_status st = e == hipSuccess ? RS_OK : hip_fail(e, "removal upload");
    // remove (marking the rows that change), then compact those rows, find
    // what must be recomputed and rerun only that
    if (st == RS_OK) st = launch_remove_edges(g, d_buf, d_buf + m, m, d_cnt);
    if (st == RS_OK) st = launch_remove_vertices(g, d_buf + 2 * m, nv, d_cnt + 2);
    if (st == RS_OK) st = launch_incremental_marks(g);
    // The counts reach pinned host memory behind an event, and the pass
    // (sized on the device) is queued right after it: the host waits for the
    // counts while the GPU goes on.
    unsigned long long *cnt = g->rem_cnt_host, *ic = g->rem_cnt_host + 4;
    if (st == RS_OK) {
        e = hipMemcpyAsync(cnt, d_cnt, 4 * sizeof(unsigned long long), hipMemcpyDeviceToHost, g->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(ic, g->d.ictr, 8 * (size_t)kIcCount, hipMemcpyDeviceToHost, g->stream);
        if (e == hipSuccess) e = hipEventRecord(g->rem_ev, g->stream);
        if (e != hipSuccess) st = hip_fail(e, "incremental counts");
    }
    if (st == RS_OK) st = launch_score_incremental(g);
    if (st == RS_OK) {
        e = hipEventSynchronize(g->rem_ev);
        if (e != hipSuccess) st = hip_fail(e, "incremental counts");
    }
    // the re-score stays queued on the graph's stream (as rs_score's pass)
    if (st != RS_OK) return st;
    g->n_alive -= (int64_t)cnt[3];
    if (res) {
        res->edges_removed = (int64_t)(cnt[0] + cnt[2]);
        res->edges_ignored = m - (int64_t)cnt[0];
        res->vertices_removed = (int64_t)cnt[3];
        res->affected = (int64_t)ic[kIcAffected];
    }
    return RS_OK;
}

rs_status rs_restrict_to_targets(rs_graph *g, int32_t k_c, rs_removal_result *res) {
    clear_error();
    if (!g) return fail(RS_ERR_ARG, "graph is NULL");
    if (k_c < 1) return fail(RS_ERR_ARG, "k_c < 1");
    if (g->n_graphs > 0) return fail(RS_ERR_STATE, "target mode is not applied to a batch of graphs");
    // internal communities are numbered in ascending caller label, so a
    // stable sort by decreasing size breaks ties by the smaller label
    const int64_t k = g->d.k;
    std::vector<int32_t> cs, order, drop;
    hipError_t e = d2h(cs, g->d.cstart, k + 1);
    if (e != hipSuccess) return hip_fail(e, "community ranges");
    try {
        order.resize(k);
        for (int64_t c = 0; c < k; ++c) order[c] = (int32_t)c;
        std::stable_sort(order.begin(), order.end(),
                         [&](int32_t a, int32_t b) { return cs[a + 1] - cs[a] > cs[b + 1] - cs[b]; });
        for (int64_t i = k_c; i < k; ++i)
            for (int32_t v = cs[order[i]]; v < cs[order[i] + 1]; ++v) drop.push_back(g->h_new2old[v]);
    } catch (const std::bad_alloc &) {
        return fail(RS_ERR_NOMEM, "host staging allocation failed");
    }
    if (!g->scored) {
        rs_status st = launch_score_pass(g);
        if (st != RS_OK) return st;
        g->scored = true;
    }
    if (drop.empty()) {
        if (res) *res = rs_removal_result{0, 0, 0, 0};
        return RS_OK;
    }
    rs_removals b{0, nullptr, nullptr, (int64_t)drop.size(), drop.data()};
    return rs_apply_removals(g, &b, res);
}

rs_status rs_reachable_communities(rs_graph *g, int64_t n_sources, const int32_t *sources, int64_t *counts) {
    clear_error();
    if (!g) return fail(RS_ERR_ARG, "graph is NULL");
    if (n_sources < 0 || n_sources > kMaxReachSources)
        return fail(RS_ERR_ARG, "n_sources must be 0.." + std::to_string(kMaxReachSources));
    if (n_sources > 0 && (!sources || !counts)) return fail(RS_ERR_ARG, "sources or counts is NULL");
    const int64_t n = g->d.n;
    std::vector<int32_t> src((size_t)n_sources);
    for (int64_t i = 0; i < n_sources; ++i) {
        if (sources[i] < 0 || sources[i] >= n) return fail(RS_ERR_RANGE, "source id out of range");
        src[i] = g->h_old2new[sources[i]];
    }
    if (n_sources == 0) return RS_OK;
    const int words = std::max(1, (int)((g->d.k + 31) / 32));
    const size_t nb = 4 * (size_t)n_sources * words;
    // buffers kept by the handle from the first call (sized for the largest
    // source count, 1,024)
    hipError_t e = hipSuccess;
    if (!g->reach_comp) {
        const size_t cap_bits = 4 * (size_t)kMaxReachSources * words;
        e = dev_alloc(g, (void **)&g->reach_comp, 4 * (size_t)std::max<int64_t>(n, 1));
        if (e == hipSuccess) e = dev_alloc(g, (void **)&g->reach_src, 4 * (size_t)kMaxReachSources);
        if (e == hipSuccess) e = dev_alloc(g, (void **)&g->reach_bits, cap_bits);
        if (e == hipSuccess) e = dev_alloc(g, (void **)&g->reach_flag, sizeof(unsigned int));
        if (e == hipSuccess) e = hipHostMalloc((void **)&g->reach_hflag, sizeof(unsigned int), hipHostMallocDefault);
        if (e != hipSuccess) {
            g->reach_comp = nullptr;  // (device buffers stay tracked and are freed with the handle)
            return hip_fail(e, "reach buffers");
        }
    }
    e = hipMemcpyAsync(g->reach_src, src.data(), 4 * (size_t)n_sources, hipMemcpyHostToDevice, g->stream);
    rs_status st = e == hipSuccess ? RS_OK : hip_fail(e, "reach upload");
    if (st == RS_OK)
        st = launch_reach(g, g->reach_src, (int)n_sources, g->reach_comp, g->reach_bits, words, g->reach_flag,
                          g->reach_hflag);
    std::vector<unsigned int> hb;
    if (st == RS_OK) {
        hb.resize(nb / 4);
        e = hipMemcpyAsync(hb.data(), g->reach_bits, nb, hipMemcpyDeviceToHost, g->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
        if (e != hipSuccess) st = hip_fail(e, "reach copy");
    }
    if (st == RS_OK)
        for (int64_t i = 0; i < n_sources; ++i) {
            int64_t c = 0;
            for (int w = 0; w < words; ++w) c += __builtin_popcount(hb[(size_t)i * words + w]);
            counts[i] = c;
        }
    return st;
}

// Scratch layout of rs_reachable_communities_static (offsets from the
// device's static array, each 256-byte aligned): the hook flag, the counts,
// the sources, the community bitmaps, the component labels.
static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

rs_status rs_reachable_communities_static(rs_graph *g, int64_t n_sources, const int32_t *sources, int64_t *counts) {
    clear_error();
    if (!g) return fail(RS_ERR_ARG, "graph is NULL");
    if (n_sources < 0 || n_sources > kMaxReachSources)
        return fail(RS_ERR_ARG, "n_sources must be 0.." + std::to_string(kMaxReachSources));
    if (n_sources > 0 && (!sources || !counts)) return fail(RS_ERR_ARG, "sources or counts is NULL");
    const int64_t n = g->d.n;
    int32_t src[kMaxReachSources];
    for (int64_t i = 0; i < n_sources; ++i) {
        if (sources[i] < 0 || sources[i] >= n) return fail(RS_ERR_RANGE, "source id out of range");
        src[i] = g->h_old2new[sources[i]];
    }
    if (n_sources == 0) return RS_OK;
    const int words = std::max(1, (int)((g->d.k + 31) / 32));
    const size_t o_cnt = 256, o_src = o_cnt + align256(8 * (size_t)n_sources),
                 o_bits = o_src + align256(4 * (size_t)n_sources),
                 o_comp = o_bits + align256(4 * (size_t)n_sources * words),
                 need = o_comp + 4 * (size_t)std::max<int64_t>(n, 1);
    if (need > kStaticScratchBytes)
        return fail(RS_ERR_RANGE, "graph too large for the static scratch: needs " + std::to_string(need) +
                                      " bytes (4 per vertex plus the bitmaps), at most " +
                                      std::to_string(kStaticScratchBytes));
    void *base = nullptr;
    rs_status st = static_scratch(g->device, &base);
    if (st != RS_OK) return st;
    char *b = (char *)base;
    unsigned int *d_flag = (unsigned int *)b;
    long long *d_cnt = (long long *)(b + o_cnt);
    int32_t *d_src = (int32_t *)(b + o_src);
    unsigned int *d_bits = (unsigned int *)(b + o_bits);
    int32_t *d_comp = (int32_t *)(b + o_comp);
    hipError_t e = hipMemcpyAsync(d_src, src, 4 * (size_t)n_sources, hipMemcpyHostToDevice, g->stream);
    if (e != hipSuccess) return hip_fail(e, "reach upload");
    unsigned int h_flag = 0;  // written by the component rounds' flag copies
    st = launch_reach(g, d_src, (int)n_sources, d_comp, d_bits, words, d_flag, &h_flag);
    if (st == RS_OK) st = launch_reach_counts(g, d_bits, (int)n_sources, words, d_cnt);
    if (st == RS_OK) {
        e = hipMemcpyAsync(counts, d_cnt, 8 * (size_t)n_sources, hipMemcpyDeviceToHost, g->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
        if (e != hipSuccess) st = hip_fail(e, "reach copy");
    } else {
        (void)hipStreamSynchronize(g->stream);  // the source upload reads this frame's array
    }
    return st;
}

rs_status rs_get_tiling(rs_graph *g, rs_tiling *t) {
    clear_error();
    if (!g || !t) return fail(RS_ERR_ARG, "graph or tiling is NULL");
    t->row_entries = g->tiling.row_entries;
    t->row_vertices = g->tiling.row_vertices;
    t->score_pairs = g->tiling.score_pairs;
    t->score_vertices = g->tiling.score_vertices;
    t->hub_list = g->tiling.hub_list;
    return RS_OK;
}

rs_status rs_set_tiling(rs_graph *g, const rs_tiling *t) {
    clear_error();
    if (!g) return fail(RS_ERR_ARG, "graph is NULL");
    rs_status st = check_tiling(t);
    if (st != RS_OK) return st;
    return retile(g, to_tiling(t));
}

rs_status rs_autotune(rs_graph *g, int32_t n_cand, const rs_tiling *cand, int32_t reps, int32_t *best, double *ms) {
    clear_error();
    if (!g || !cand || !best || !ms) return fail(RS_ERR_ARG, "graph, candidates, best or ms is NULL");
    if (n_cand < 1 || reps < 1) return fail(RS_ERR_ARG, "n_cand and reps must be >= 1");
    for (int32_t i = 0; i < n_cand; ++i) {
        const rs_status st = check_tiling(&cand[i]);
        if (st != RS_OK) return st;
    }
    const bool was_scored = g->scored;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    rs_status st = e == hipSuccess ? RS_OK : hip_fail(e, "autotune events");
    int32_t b = -1;
    for (int32_t i = 0; i < n_cand && st == RS_OK; ++i) {
        st = retile(g, to_tiling(&cand[i]));
        if (st == RS_OK) st = launch_score_pass(g);  // warm-up (and the replay's capture)
        if (st != RS_OK) break;
        e = hipEventRecord(e0, g->stream);
        for (int32_t r = 0; r < reps && st == RS_OK && e == hipSuccess; ++r) st = launch_score_pass(g);
        if (e == hipSuccess) e = hipEventRecord(e1, g->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float t = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
        if (e != hipSuccess && st == RS_OK) st = hip_fail(e, "autotune timing");
        ms[i] = (double)t / reps;
        if (st == RS_OK && (b < 0 || ms[i] < ms[b])) b = i;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st != RS_OK) return st;
    *best = b;
    st = retile(g, to_tiling(&cand[b]));
    if (st == RS_OK && was_scored) {
        st = launch_score_pass(g);
        if (st == RS_OK) g->scored = true;
    }
    return st;
}

rs_status rs_read_scores(rs_graph *g, double *out, int64_t n, int32_t raw) {
    clear_error();
    if (!g || (!out && n > 0)) return fail(RS_ERR_ARG, "graph or out is NULL");
    if (n != g->d.n) return fail(RS_ERR_ARG, "n does not match the graph");
    if (!g->scored) return fail(RS_ERR_STATE, "rs_read_scores before rs_score");
    if (n == 0) return RS_OK;
    rs_status st = launch_gather_scores(g, g->d.scratch_d, raw ? 1 : 0);
    if (st != RS_OK) return st;
    hipError_t e = hipMemcpyAsync(out, g->d.scratch_d, 8 * n, hipMemcpyDeviceToHost, g->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    return e == hipSuccess ? RS_OK : hip_fail(e, "score copy");
}

rs_status rs_read_counts(rs_graph *g, rs_counts *c) {
    clear_error();
    if (!g || !c) return fail(RS_ERR_ARG, "graph or counts is NULL");
    if (g->scored) {
        const rs_status st = launch_reduce_counts(g);
        if (st != RS_OK) return st;
    }
    DevCounters dc;
    hipError_t e = hipMemcpyAsync(&dc, g->d.ctr, sizeof(dc), hipMemcpyDeviceToHost, g->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    if (e != hipSuccess) return hip_fail(e, "counter copy");
    std::vector<int32_t> deg(g->d.n);
    if (g->d.n) {
        e = hipMemcpy(deg.data(), g->d.deg, 4 * g->d.n, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "degree copy");
    }
    int64_t live = 0;
    for (int32_t d : deg) live += d;
    c->n = g->d.n;
    c->nnz = live;
    c->n_alive = g->n_alive;
    c->n_communities = g->d.k;
    c->n_border = (int64_t)dc.n_border;
    c->m_inter = (int64_t)dc.sum_dprime / 2;
    c->sum_ell = (int64_t)dc.sum_ell;
    c->sum_ell_x = (int64_t)dc.sum_ell_x;
    c->sum_tI = (int64_t)dc.sum_tI;
    c->sum_tII = (int64_t)dc.sum_tII;
    c->sum_work_I = (int64_t)dc.sum_workI;
    double w;
    std::memcpy(&w, &dc.wmax_bits, sizeof(w));
    c->omega_max = w;
    return RS_OK;
}

rs_status rs_read_vertex_counts(rs_graph *g, int32_t *border, int32_t *ell, int32_t *dprime, int64_t *tI,
                                int64_t *tII, double *w_own) {
    clear_error();
    if (!g) return fail(RS_ERR_ARG, "graph is NULL");
    if (!g->scored) return fail(RS_ERR_STATE, "read before rs_score");
    const int64_t n = g->d.n;
    hipError_t e = hipStreamSynchronize(g->stream);
    std::vector<VMeta> meta;
    std::vector<long long> htI, htII;
    std::vector<double> hw;
    if (e == hipSuccess) e = read_meta(g, meta);
    if (e == hipSuccess) e = d2h(htI, g->d.tI, n);
    if (e == hipSuccess) e = d2h(htII, g->d.tII, n);
    if (e == hipSuccess) e = d2h(hw, g->d.wown, n);
    if (e != hipSuccess) return hip_fail(e, "vertex count copy");
    for (int64_t v = 0; v < n; ++v) {
        const VMeta &m = meta[g->h_old2new[v]];
        const int32_t dp = m.deg - (m.q - m.p);
        const int32_t x = g->h_old2new[v];
        if (border) border[v] = dp > 0;
        if (ell) ell[v] = m.ell;
        if (dprime) dprime[v] = dp;
        if (tI) tI[v] = dp > 0 ? htI[x] : 0;
        if (tII) tII[v] = dp > 0 ? htII[x] : 0;
        if (w_own) w_own[v] = hw[x];
    }
    return RS_OK;
}

rs_status rs_read_rows(rs_graph *g, int64_t *row_off, int32_t *comm, int32_t *count, double *weight) {
    clear_error();
    if (!g || !row_off) return fail(RS_ERR_ARG, "graph or row_off is NULL");
    if (!g->scored) return fail(RS_ERR_STATE, "read before rs_score");
    const int64_t n = g->d.n;
    hipError_t e = hipStreamSynchronize(g->stream);
    std::vector<VMeta> meta;
    std::vector<int64_t> off;
    if (e == hipSuccess) e = read_meta(g, meta);
    if (e == hipSuccess) e = read_offsets(g, off);
    if (e != hipSuccess) return hip_fail(e, "row copy");
    row_off[0] = 0;
    for (int64_t v = 0; v < n; ++v) row_off[v + 1] = row_off[v] + meta[g->h_old2new[v]].ell;
    if (!comm && !count && !weight) return RS_OK;
    std::vector<int32_t> key;
    std::vector<RecDat> dat;
    e = d2h(key, g->d.reckey, g->d.nnz);
    if (e == hipSuccess) e = d2h(dat, g->d.recdat, g->d.nnz);
    if (e != hipSuccess) return hip_fail(e, "row copy");
    for (int64_t v = 0; v < n; ++v) {
        const int32_t x = g->h_old2new[v];
        const int64_t rb = off[x];
        const VMeta &m = meta[x];
        for (int32_t r = 0; r < m.ell; ++r) {
            const int64_t o = row_off[v] + r;
            if (comm) comm[o] = g->h_comm2orig[key[rb + r]];
            if (count) count[o] = dat[rb + r].f;
            if (weight) weight[o] = dat[rb + r].w;
        }
    }
    return RS_OK;
}

rs_status rs_read_gprime(rs_graph *g, int64_t *goff, int32_t *gcol) {
    clear_error();
    if (!g || !goff) return fail(RS_ERR_ARG, "graph or off is NULL");
    if (!g->scored) return fail(RS_ERR_STATE, "read before rs_score");
    const int64_t n = g->d.n;
    hipError_t e = hipStreamSynchronize(g->stream);
    std::vector<VMeta> meta;
    std::vector<int32_t> hcol;
    std::vector<int64_t> off;
    if (e == hipSuccess) e = read_meta(g, meta);
    if (e == hipSuccess) e = read_offsets(g, off);
    if (e != hipSuccess) return hip_fail(e, "G' copy");
    goff[0] = 0;
    for (int64_t v = 0; v < n; ++v) {
        const VMeta &m = meta[g->h_old2new[v]];
        goff[v + 1] = goff[v] + m.deg - (m.q - m.p);
    }
    if (!gcol) return RS_OK;
    e = d2h(hcol, g->d.col, g->d.nnz);
    if (e != hipSuccess) return hip_fail(e, "G' copy");
    for (int64_t v = 0; v < n; ++v) {
        const int32_t x = g->h_old2new[v];
        const VMeta &m = meta[x];
        const int64_t rb = off[x];
        int64_t o = goff[v];
        for (int32_t j = 0; j < m.deg; ++j) {
            if (j >= m.p && j < m.q) continue;
            gcol[o++] = g->h_new2old[hcol[rb + j]];
        }
        std::sort(gcol + goff[v], gcol + goff[v + 1]);
    }
    return RS_OK;
}

static const char *kKernelNames[K_COUNT] = {
    "k_rows", "k_wmax", "k_score_hub", "k_score", "k_topk_hist", "k_topk_find", "k_topk_collect", "k_tie_rank", "k_final_order",
    "k_hub_sum", "k_topk_graphs", "k_wmax_graphs", "k_hub_filters"};

const char *rs_kernel_name(int32_t id) { return (id >= 0 && id < K_COUNT) ? kKernelNames[id] : nullptr; }

rs_status rs_set_timing(rs_graph *g, int32_t on) {
    clear_error();
    if (!g) return fail(RS_ERR_ARG, "graph is NULL");
    g->timing.on = on != 0;
    return RS_OK;
}

rs_status rs_read_timings(rs_graph *g, int32_t cap, double *ms, int64_t *launches, int32_t *n_kernels) {
    clear_error();
    if (!g) return fail(RS_ERR_ARG, "graph is NULL");
    hipError_t e = hipStreamSynchronize(g->stream);
    if (e != hipSuccess) return hip_fail(e, "timing sync");
    drain_replays(g);
    for (auto &pe : g->timing.pending) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, pe.second.first, pe.second.second) == hipSuccess) {
            g->timing.ms[pe.first] += t;
            g->timing.launches[pe.first] += 1;
        }
        g->timing.pool.push_back(pe.second.first);
        g->timing.pool.push_back(pe.second.second);
    }
    g->timing.pending.clear();
    for (int i = 0; i < K_COUNT && i < cap; ++i) {
        if (ms) ms[i] = g->timing.ms[i];
        if (launches) launches[i] = g->timing.launches[i];
    }
    for (int i = 0; i < K_COUNT; ++i) {
        g->timing.ms[i] = 0;
        g->timing.launches[i] = 0;
    }
    if (n_kernels) *n_kernels = K_COUNT;
    return RS_OK;
}

}  // extern "C"
