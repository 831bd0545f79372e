// rs_internal.h -- device layout and launch interface of the RS library.
//
// Resident layout of one graph in HBM (internal ids):
//   * Vertices are renumbered so that every community is a contiguous id
//     range (communities in ascending caller-label order, vertices inside a
//     community in ascending caller-id order), and each CSR row is sorted by
//     internal id.  A row therefore lists its neighbours community by
//     community, and the neighbours in the vertex's own community form one
//     contiguous sub-range [p, q) of the row.
//   * off[n+1] is the row capacity layout fixed at load time (OffT = int32
//     or int64); deg[n] is the current row length (removals shrink rows in
//     place, keeping them sorted).
//   * The interaction matrix is stored sparse, one record per (vertex,
//     neighbour community) in the row's own slot range [off[v], off[v] + ell):
//     reckey[] holds the community (ascending within a vertex), recdat[] the
//     first row position of that community's run, its length f and the weight
//     w_v(c).
//   * meta[v] = {deg, ell, p, q} of the last pass.  G' (the edges between
//     communities) is implicit: v's foreign neighbours are the row positions
//     outside [p, q), in ascending id order.
//   * Out-lists orient G': vertices are ranked by (load-time foreign degree,
//     id), and out(v) lists v's foreign neighbours of higher rank.  Every
//     triangle of G' is {u, x, y} with y in out(x) for exactly one ordering of
//     its other two vertices, and the lists are short (a hub's foreign
//     neighbours are mostly of lower rank).  Removals tombstone entries (~id).
//   * Pair facts: every foreign row entry e = (w, u) gets prec[e], written by
//     w's row pass: w_w(C(u)) and the run of C(u) in w's row.  The G' entries
//     (u, w) of u have link slots [goff[u], goff[u + 1]) in foreign-list order
//     (goff is the prefix of the load-time foreign degrees; removals only
//     shrink the lists): plink[s] = the index of the reverse entry (w, u) and
//     w's out-list range.  The score pass reads u's links as one contiguous
//     stream and each pair's facts with one independent load.
//   * Work is cut at load time into static tiles of consecutive vertices: row
//     tiles bound the row capacity they cover, score tiles the number of
//     foreign entries (removals only shrink both).  Vertices too large for a
//     tile are hubs and get a workgroup of their own.  No kernel of a pass
//     uses a same-address atomic; each workgroup writes its own partials.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/rs.h"

namespace rs {

constexpr int kBlock = 256;          // threads per workgroup of the per-vertex kernels
constexpr int kRowTile = 2048;       // row capacity (entries) covered by one row tile
constexpr int kRowTileV = 512;       // vertices of one row tile
constexpr int kScoreTileP = 256;     // foreign entries (load-time bound) of one score tile (one per thread)
constexpr int kScoreTileV = 256;     // vertices of one score tile (one per thread)
constexpr int kHubKeys = 1024;       // score hubs with at most this many records keep their keys in LDS
constexpr int kHubList = 1024;       // score hubs with at most this many foreign entries stage them in LDS
constexpr int kFilterBits = 18;      // a big hub's neighbour filter: 2^18 bits (32 KB), one hash
constexpr int kFilterWords = (1 << kFilterBits) / 32;
constexpr int kTopkBins = 65536;     // 16-bit digits of the 96-bit ranking key
constexpr int kHistChunk = 49152;    // keys per block of the histogram kernel (< 2^16)
constexpr int kTieCap = 16384;       // largest tie class ranked through sorted chunks
constexpr int kSortCap = 2048;       // final lists up to this size are bitonic-sorted in LDS
constexpr int kSmallCap = 4096;      // fewest candidates (final list + threshold bin) the common path ranks
constexpr int kWorkBlocks = 1024;    // blocks (and partials) of the on-demand W1 count
constexpr int kMaxReachSources = 1024;  // sources per rs_reachable_communities call
constexpr size_t kStaticScratchBytes = size_t(32) << 20;  // per-device array of rs_reachable_communities_static
constexpr int kMaxDevices = 64;
constexpr int kBatchK = 32;
constexpr int kSegVerts = 1024;   // vertices per batched top-k segment (64 lanes x 16 keys)
constexpr int kSegMax = 64;       // segments per graph merged by one wavefront          // largest k of the per-graph top-k of a batch

// An incremental re-score whose units exceed this many tenths of the full
// pass's workgroups runs the full pass instead.
constexpr int kFullPassTenths = 6;
// Tile and bin cut-offs of a graph's static schedule: chosen at load (the
// defaults) or by the autotuner.  Each is at most the compile-time size the
// kernels' LDS is laid out for.
struct Tiling {
    int row_entries = kRowTile;        // row capacity one row tile covers; a longer row is a hub row
    int row_vertices = kRowTileV;      // vertices of one row tile
    int score_pairs = kScoreTileP;     // foreign entries of one score tile; more make a score hub
    int score_vertices = kScoreTileV;  // vertices of one score tile
    int hub_list = kHubList;           // score hubs with at most this many foreign entries stage them in LDS
};

// Vertex marks of an incremental re-score (after removals).
constexpr unsigned int kRowChanged = 1u;   // the row lost entries
constexpr unsigned int kAffected = 2u;     // the score must be recomputed
// Counters of an incremental re-score (ictr[]).
// Affected tile vertices are rescored in units built per pass: bin b holds
// the vertices with a load-time foreign degree in (2^(b-1), 2^b] (bin 0: at
// most 1), and a unit of bin b takes 256 >> b of them (<= 256 pairs).
constexpr int kScoreBins = 9;
// The units are found over contiguous vertex ranges, one per workgroup (at
// most kUnitGroups), each counting its tile vertices per bin and its
// affected vertices (kUnitRows counts per range).
constexpr int kUnitGroups = 1024;
constexpr int kUnitRows = kScoreBins + 1;
enum IncCounter {
    kIcChanged = 0, kIcLinkRows, kIcRows, kIcMain, kIcBig, kIcAffected, kIcWmaxOld, kIcChunks, kIcAList,
    kIcBins,  // kScoreBins counts
    kIcCount = kIcBins + kScoreBins
};

// Grid of a tiled launch: one workgroup per hub, then the tiles rounded up to
// a multiple of the 8 XCDs.
inline int tile_grid(int hubs, int tiles) { return hubs + 8 * ((tiles + 7) / 8); }

enum KernelId {
    K_ROWS = 0,
    K_WMAX,
    K_SCORE_HUB,
    K_SCORE,
    K_TOPK_HIST,
    K_TOPK_FIND,
    K_TOPK_COLLECT,
    K_TOPK_TIE,
    K_TOPK_RANK,
    K_HUB_SUM,
    K_TOPK_GRAPHS,
    K_WMAX_GRAPHS,
    K_HUB_FILTERS,
    K_COUNT
};

struct __align__(16) RecDat {
    int pos;   // first row position of the community's run
    int f;     // run length = number of neighbours in the community
    double w;  // w_v(community)
};

struct __align__(16) VMeta {
    int deg, ell, p, q;
};

// Everything a pass needs about a vertex, in one 64-byte card (one memory
// line for a gathered vertex): the static row start, pair-slot start and
// community, and the last pass's row facts, a_v and the first record keys
// (INT_MAX past ell).
struct __align__(64) VCard {
    long long off;   // row start
    long long goff;  // first pair slot
    VMeta m;         // {deg, ell, p, q} of the last pass
    int pad;
    int lab;         // community
    double a;        // cbrt(own-community weight) of the last pass
    int key[4];      // first record keys of the last pass
};

// The facts of the pair (u, w) at w's row entry (w, u), written by w's row
// pass: w_w(C(u)), the length f of C(u)'s run in w's row and the distance
// from the entry back to the run's first entry.
struct __align__(16) PairRec {
    double w;
    int f;
    int back;
};

// An out-list entry x -> y: the indices of the row entries (x, y) in x's row
// and (y, x) in y's row (a type-I hit reads the pair facts at both).
struct __align__(16) OutEnt {
    long long xy, yx;
};

// A link slot (u, w): the index of the row entry (w, u) and w's out-list
// range (tombstones included).
struct __align__(16) PairLink {
    long long e;
    int oo;
    int on;
};
static_assert(sizeof(VCard) == 64, "one card per 64 bytes");

// A row tile: vertices [v0, v1) whose rows occupy entries [e0, e0 + te).
struct __align__(16) RowTile {
    long long e0;
    int v0, v1, te, pad;
};

// Per-block partial results of the row kernels (no atomics).
struct RowPart {
    unsigned long long wmax_bits, n_border, sum_dprime, sum_ell, sum_ell_x, pad[3];
};
// Partial sum of one chunk of a score hub's pairs.
struct HubPart {
    double raw;
    long long tI, tII, pad;
};

// Totals of a pass, reduced from the partials.
struct DevCounters {
    unsigned long long wmax_bits;  // w_max as the bit pattern of a non-negative double
    unsigned long long n_border;
    unsigned long long sum_dprime;
    unsigned long long sum_ell;
    unsigned long long sum_ell_x;
    unsigned long long sum_tI;
    unsigned long long sum_tII;
    unsigned long long sum_workI;
};

// Ranking key: score bits (a non-negative double orders like its bits) and
// the complement of the caller id, so that a larger key ranks first.
struct __align__(16) TopkKey {
    unsigned long long hi;  // bits of the score
    unsigned int lo;        // 0xffffffff - caller id
    int v;                  // internal vertex id
};

// State of one top-k selection (device memory).
struct TopkState {
    long long k;           // requested count (clamped to live vertices)
    unsigned int digit;    // current digit index (0..5)
    unsigned int thresh;   // threshold digit value of the current level
    long long above;       // keys already placed in the final list before this level
    long long take;        // keys still needed from the threshold bin
    long long binsize;     // keys in the threshold bin
    unsigned long long n_final;  // final-list fill counter
    unsigned long long n_tie;    // tie-list fill counter
    unsigned int overflow;       // tie class too large for the pairwise ranker
    unsigned int done;           // threshold bin taken whole
    unsigned int small;          // spare
};

struct DeviceGraph {
    int64_t n = 0, nnz = 0;
    int32_t k = 0;
    bool off64 = false;
    void *off = nullptr;        // OffT[n+1]
    int32_t *deg = nullptr;     // [n] current degree
    int32_t *col = nullptr;     // [nnz]
    int32_t *clab = nullptr;    // [nnz] the community of each entry's neighbour (-1: removed tail), the row pass's input
    int32_t *lab = nullptr;     // [n] internal community id
    int32_t *new2old = nullptr; // [n]
    uint8_t *alive = nullptr;   // [n]
    RowTile *rtiles = nullptr;  // row tiles
    int32_t *rhubs = nullptr;   // vertices whose row capacity exceeds kRowTile
    int2 *stiles = nullptr;     // score tiles
    int32_t *shubs = nullptr;   // vertices with more than kScoreTileP foreign entries
    int32_t *shub_first = nullptr;  // [hubs + 1] first chunk of each score hub
    int2 *shub_chunk = nullptr;     // [chunks] (hub, chunk index within the hub)
    HubPart *hub_part = nullptr;    // [chunks] chunk partials
    int64_t *oo = nullptr;      // [n+1] out-list offsets
    int64_t *goff = nullptr;    // [n+1] pair-slot offsets
    PairRec *prec = nullptr;    // [nnz] pair facts at foreign row entries
    PairLink *plink = nullptr;  // [link slots]
    int32_t *cstart = nullptr;  // [k+1] first internal id of each community
    unsigned long long *wpart = nullptr;  // [kWorkBlocks] partials of the on-demand W1 count
    // incremental re-score
    unsigned int *vmark = nullptr;          // [n] kRowChanged | kAffected
    int32_t *vrowb = nullptr;               // [n] row block of each vertex
    int32_t *vscore = nullptr;              // [n] score tile block, or -1 - score hub index
    unsigned long long *wblk = nullptr;  // [64] per-workgroup maxima of k_wmax
    unsigned int *wticket = nullptr;     // k_wmax's finishing ticket (zero between passes)
    OutEnt *oe = nullptr;         // [out-list entries] row entries of each out-list entry's edge
    uint32_t *hfilter = nullptr;  // [big hubs][kFilterWords] membership filter of each big hub's foreign neighbours
    uint8_t *rflag = nullptr, *cflag = nullptr, *hflag = nullptr;  // flags: row blocks, score-hub chunks, score hubs (whole)
    int32_t *elist = nullptr, *abin = nullptr;  // [n] changed rows; affected tile vertices by bin
    int32_t *ucnt = nullptr;                    // [kUnitRows * kUnitGroups] per-range counts, then slots
    int2 *echunk = nullptr;                 // [n + nnz / 64] chunks of 64 entries of the changed rows
    int32_t *rlist = nullptr, *slist = nullptr, *hlist = nullptr; // block lists
    unsigned long long *ictr = nullptr;     // [kIcCount]
    // batched graphs (a disjoint union of n_graphs graphs, each a contiguous id range)
    int64_t *vstart = nullptr;              // [n_graphs + 1] first vertex of each graph
    int32_t *vgraph = nullptr;              // [n] graph of each vertex
    unsigned long long *gwmax = nullptr;    // [n_graphs] w_max of each graph (bits)
    int32_t *gblk_off = nullptr, *gblk = nullptr;  // the row blocks of each graph
    int32_t *gorder = nullptr;              // graphs by decreasing vertex count (top-k order of work)
    int32_t *seg_g = nullptr, *sfirst = nullptr;  // top-k segments: graph of each, first of each graph
    unsigned long long *c_hi = nullptr;     // [segments * kBatchK] segment top-k keys (score bits)
    unsigned int *c_lo = nullptr;           // [segments * kBatchK] segment top-k keys (low words)
    int32_t *c_cnt = nullptr;               // [segments] keys per segment list
    int32_t *bids = nullptr;                // [n_graphs * kBatchK] per-graph top-k
    double *bscores = nullptr;
    int64_t *bcounts = nullptr;             // [n_graphs]
    int32_t *outl = nullptr;    // [m'] out-lists: foreign neighbours of higher rank, ascending (removed: ~id)
    int32_t *reckey = nullptr;  // [nnz] interaction-matrix record keys
    RecDat *recdat = nullptr;   // [nnz] interaction-matrix record data
    VCard *card = nullptr;      // [n]
    double *wown = nullptr, *R = nullptr;
    double *av = nullptr;       // [n] a_v = cbrt(own-community weight) of the last pass
    double *raw = nullptr;      // [n] Eq. RSI sums before the w_max and d(d-1) division
    long long *tI = nullptr, *tII = nullptr;
    RowPart *part_rows = nullptr;    // [row grid]
    unsigned long long *wmax_part = nullptr;  // [row grid] w_max bits per block
    DevCounters *ctr = nullptr;
    // top-k
    unsigned int *thist = nullptr;  // [kTopkBins]
    unsigned int *thist_c = nullptr;  // [256] coarse histogram (sums of 256 bins)
    TopkState *tstate = nullptr;
    TopkKey *tfinal = nullptr, *ttie = nullptr, *ttie2 = nullptr;  // [n] each
    int32_t *tout_ids = nullptr;
    double *tout_sc = nullptr;
    double *scratch_d = nullptr;    // [n] doubles (readers)
    char *tblk = nullptr;           // [16 + 16 n] top-k output block: flag | ids | scores
    unsigned long long *scratch_u = nullptr;  // [8] small counters
};

// A fixed launch sequence captured once into a HIP graph and replayed: the
// score pass, or the common path of top-k for one k.  With timing on, the
// timing events are captured too; their times are read after a replay has
// completed (unread until then).
struct Replay {
    hipGraphExec_t exec = nullptr;
    long long key = -1;
    bool timed = false;
    bool unread = false;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> events;
};

struct Timing {
    bool on = false;
    std::vector<hipEvent_t> pool;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
    double ms[K_COUNT] = {};
    long long launches[K_COUNT] = {};
};

}  // namespace rs

struct rs_graph {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool scored = false;
    bool wide_offsets = false;  // 64-bit device edge offsets even for nnz <= INT32_MAX
    int64_t n_alive = 0;
    int64_t dev_bytes = 0;  // device memory held by the graph
    int n_rtiles = 0, n_rhubs = 0, n_stiles = 0, n_shubs = 0, n_schunks = 0;
    int n_schunks_lds = 0;               // chunks of hubs whose foreign list fits in LDS (listed first)
    int n_shubs_lds = 0;                 // those hubs (the big hubs follow)
    int64_t n_out = 0;                   // out-list entries (G' edges)
    int grid_rows = 0, grid_score = 0;   // hubs first, then the tiles in XCD-major order
    std::vector<int32_t> h_new2old, h_old2new, h_comm2orig;
    rs::DeviceGraph d;
    rs::Timing timing;
    rs::Replay pass_rep, topk_rep;
    bool graphs_off = false;  // eager launches only (RS_GRAPHS=0, or a capture failed)
    int32_t n_graphs = 0;     // > 0: a batch of graphs loaded as one disjoint union
    std::vector<int64_t> h_vstart;
    std::vector<int32_t> h_gblk_off, h_gblk;
    int32_t n_segs = 0;       // batched top-k segments (0: the one-wavefront-per-graph form)
    int32_t *reach_comp = nullptr, *reach_src = nullptr;  // reachable-community buffers (first use)
    unsigned int *reach_bits = nullptr, *reach_flag = nullptr, *reach_hflag = nullptr;
    std::vector<std::pair<void *, size_t>> allocations;  // device buffers and their sizes
    rs::Tiling tiling;
    // pinned host buffer of the common top-k path: [flag | ids | scores]
    void *hpin = nullptr;
    int64_t hpin_cap = 0;
    // removal batches: device staging kept between calls (grown on demand),
    // pinned host staging of the batch and of the counts read back
    int32_t *rem_buf = nullptr;
    int64_t rem_cap = 0;
    int32_t *rem_host = nullptr;
    int64_t rem_host_cap = 0;
    unsigned long long *rem_cnt = nullptr;       // device [4]: edges removed, -, edges of removed vertices, vertices
    unsigned long long *rem_cnt_host = nullptr;  // pinned [4 + kIcCount]
    hipEvent_t rem_ev = nullptr;                 // the removal counts have reached rem_cnt_host
};

namespace rs {

// Error plumbing (rs_runtime.hip).
rs_status fail(rs_status s, const std::string &msg);
rs_status hip_fail(hipError_t e, const char *what);
void clear_error();

// Timing helpers (rs_runtime.hip).
void timing_begin(rs_graph *g, int kid, hipEvent_t *ev);
void timing_end(rs_graph *g, int kid, hipEvent_t ev);

// Kernel launchers (rs_kernels.hip).  All enqueue on g->stream.
rs_status launch_score_pass(rs_graph *g);
// An incremental pass after launch_incremental_marks, sized on the device:
// the row blocks, main score blocks and big-hub chunks listed by the marks
// (indices of the full launches; every index when the units exceed
// kFullPassTenths of the full pass) and the units of the affected tile
// vertices, then w_max from every block's partial and, if it moved, every
// score rescaled.  No host round trip.
rs_status launch_score_incremental(rs_graph *g);
rs_status launch_topk(rs_graph *g, int64_t k, int32_t *ids, double *scores, int64_t *count);
// Read the timing events of completed replays into the timing totals.
void drain_replays(rs_graph *g);
void release_replays(rs_graph *g);
rs_status launch_reduce_counts(rs_graph *g);
rs_status launch_remove_edges(rs_graph *g, const int32_t *d_src, const int32_t *d_dst, int64_t m,
                              unsigned long long *d_removed);
rs_status launch_remove_vertices(rs_graph *g, const int32_t *d_verts, int64_t nv,
                                 unsigned long long *d_removed_edges);
rs_status launch_links(rs_graph *g);
rs_status launch_col_labels(rs_graph *g);
rs_status launch_out_entries(rs_graph *g);
rs_status launch_incremental_marks(rs_graph *g);
rs_status launch_topk_graphs(rs_graph *g, int64_t k, int32_t *d_ids, double *d_scores, int64_t *d_counts);
rs_status launch_gather_scores(rs_graph *g, double *d_out, int raw);
// Host-built graphs kept for reloads (the request server).
struct Prebuilt;
rs_status prebuild_graph(const rs_csr *csr, Prebuilt **out);
rs_status load_prebuilt(Prebuilt *P, void *hip_stream, rs_graph **out);
void free_prebuilt(Prebuilt *P);
rs_status launch_reach(rs_graph *g, const int32_t *d_src, int ns, int32_t *comp, unsigned int *bits, int words,
                       unsigned int *d_changed, unsigned int *h_changed);
rs_status launch_zero_u64(rs_graph *g, unsigned long long *p, int count);
// The device address of this library's static scratch array on `device`
// (taken once per device with hipGetSymbolAddress), and the per-source
// bit counts of reach bitmaps.
rs_status static_scratch(int device, void **out);
rs_status launch_reach_counts(rs_graph *g, const unsigned int *bits, int ns, int words, long long *d_counts);

}  // namespace rs
