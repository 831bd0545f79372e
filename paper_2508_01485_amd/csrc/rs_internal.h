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
//   * The interaction matrix is stored sparse, one 16-byte record per
//     (vertex, neighbour community) in the row's own slot range
//     [off[v], off[v] + ell): community, first row position of that
//     community's run, weight w_v(c).  A run's length is the next record's
//     position minus its own (the last run ends at deg[v]).
//   * meta[v] = {deg, ell, p, q} of the last pass.  G' (the edges between
//     communities) is implicit: v's foreign neighbours are the row positions
//     outside [p, q), in ascending id order.
//   * Vertices are grouped at load time into degree bins (sched); every
//     kernel walks the bins with a persistent grid, so no work list is built
//     during a pass and no kernel uses a same-address atomic.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/rs.h"

namespace rs {

// Degree bins (load-time degree d):
//   A  d <= 16        rows: one thread per vertex; scores: one thread per vertex
//   B  16 < d <= 64   rows: one thread per vertex; scores: 4 lanes per vertex
//   C  64 < d <= 512  rows and scores: 16 lanes per vertex
//   D  d > 512        rows: one block per vertex (streamed); scores: a wavefront
constexpr int kBins = 4;
constexpr int kBinMaxDeg[kBins - 1] = {16, 64, 512};

constexpr int kBlock = 256;          // threads per block of the per-vertex kernels
constexpr int kGridRows = 2048;      // persistent grid of the thread-per-vertex row kernel (multiple of 8)
constexpr int kGridMid = 1024;       // persistent grid of the 16-lane row kernel (multiple of 8)
constexpr int kGridScore = 2048;     // persistent grid of the small-vertex score kernel
constexpr int kGridBig = 2048;       // persistent grid of the large-vertex score kernel
constexpr int kCapB = 64;            // LDS staging of N'(u) for the 4-lane teams of bin B
constexpr int kCapC = 256;           // ... 16-lane teams of bin C
constexpr int kCapD = 1024;          // ... wavefront teams of bin D (larger lists stay in HBM)
constexpr int kTopkBins = 65536;     // 16-bit digits of the 96-bit ranking key
constexpr int kHistChunk = 49152;    // keys per block of the histogram kernel (< 2^16)
constexpr int kTieCap = 16384;       // largest tie class ranked by pairwise compare
constexpr int kSortCap = 2048;       // final lists up to this size are bitonic-sorted in LDS

enum KernelId {
    K_ROWS_HUB = 0,
    K_ROWS_MID,
    K_ROWS,
    K_WMAX,
    K_SCORE,
    K_SCORE_BIG,
    K_TOPK_HIST,
    K_TOPK_FIND,
    K_TOPK_COLLECT,
    K_TOPK_TIE,
    K_TOPK_RANK,
    K_COUNT
};

struct __align__(16) Rec {
    int key;   // community (internal id)
    int pos;   // first row position of the community's run
    double w;  // w_v(key)
};

struct __align__(16) VMeta {
    int deg, ell, p, q;
};

// Per-block partial results of the row kernels (no atomics).
struct RowPart {
    unsigned long long wmax_bits, n_border, sum_dprime, sum_ell, sum_ell_x, pad[3];
};
struct ScorePart {
    unsigned long long tI, tII, workI, pad;
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
};

struct DeviceGraph {
    int64_t n = 0, nnz = 0;
    int32_t k = 0;
    bool off64 = false;
    void *off = nullptr;        // OffT[n+1]
    int32_t *deg = nullptr;     // [n] current degree
    int32_t *col = nullptr;     // [nnz]
    int32_t *lab = nullptr;     // [n] internal community id
    int32_t *new2old = nullptr; // [n]
    uint8_t *alive = nullptr;   // [n]
    int32_t *sched = nullptr;   // [n] vertices grouped by degree bin
    Rec *rec = nullptr;         // [nnz] interaction-matrix records
    VMeta *meta = nullptr;      // [n]
    double *wown = nullptr, *a = nullptr, *R = nullptr;
    long long *tI = nullptr, *tII = nullptr;
    RowPart *part_rows = nullptr;    // [kGridRows + kGridMid + hub blocks]
    ScorePart *part_score = nullptr; // [kGridScore + kGridBig]
    DevCounters *ctr = nullptr;
    // top-k
    unsigned int *thist = nullptr;  // [kTopkBins]
    TopkState *tstate = nullptr;
    TopkKey *tfinal = nullptr, *ttie = nullptr, *ttie2 = nullptr;  // [n] each
    int32_t *tout_ids = nullptr;
    double *tout_sc = nullptr;
    double *scratch_d = nullptr;    // [n] doubles (readers)
    unsigned long long *scratch_u = nullptr;  // [8] small counters
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
    int64_t n_alive = 0;
    int64_t bin_lo[rs::kBins + 1] = {};  // start of each degree bin in sched
    int hub_grid = 0;                    // blocks of the hub row kernel
    std::vector<int32_t> h_new2old, h_old2new, h_comm2orig;
    rs::DeviceGraph d;
    rs::Timing timing;
    std::vector<void *> allocations;
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
rs_status launch_topk(rs_graph *g, int64_t k, int64_t *count);
rs_status launch_reduce_counts(rs_graph *g);
rs_status launch_remove_edges(rs_graph *g, const int32_t *d_src, const int32_t *d_dst, int64_t m,
                              unsigned long long *d_removed);
rs_status launch_remove_vertices(rs_graph *g, const int32_t *d_verts, int64_t nv,
                                 unsigned long long *d_removed_edges);
rs_status launch_compact_rows(rs_graph *g);
rs_status launch_gather_scores(rs_graph *g, double *d_out, int raw);
rs_status launch_zero_u64(rs_graph *g, unsigned long long *p, int count);

}  // namespace rs
