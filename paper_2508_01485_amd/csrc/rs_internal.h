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
//     neighbour community), in the row's own slot range [off[v], off[v]+ell):
//     hkey (community), hpos (first row position of that community's run),
//     hw (weight w_v(c)), hS (sum of a_x over the run, foreign runs only).
//     Run lengths are differences of consecutive hpos (the last run ends at
//     deg[v]).
//   * G' (edges between communities) is implicit: the foreign neighbours of
//     v are the row positions outside [p, q).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/rs.h"

namespace rs {

// Degree bins for the per-vertex row kernel: team size (lanes per vertex).
// A vertex of (load-time) degree d goes to the smallest team >= d, capped at
// a wavefront; rows longer than the team loop over chunks.
constexpr int kRowBins = 4;
constexpr int kRowTeam[kRowBins] = {8, 16, 32, 64};

// Foreign-degree bins for the S-aggregation and score kernels (filled by the
// row kernel each pass): team sizes.
constexpr int kScoreBins = 3;
constexpr int kScoreTeam[kScoreBins] = {4, 16, 64};
constexpr int kScoreBinMax[kScoreBins - 1] = {4, 16};  // d' <= 4, d' <= 16, else

constexpr int kBlock = 256;          // threads per block of the vertex kernels
constexpr int kTopkBins = 65536;     // 16-bit digits of the 96-bit ranking key
constexpr int kTieCap = 16384;       // largest tie class ranked by pairwise compare

// Kernel ids for timing.
enum KernelId {
    K_INIT = 0,
    K_ROWS,
    K_SAGG,
    K_SCORE,
    K_TOPK_HIST,
    K_TOPK_FIND,
    K_TOPK_COLLECT,
    K_TOPK_TIE,
    K_TOPK_RANK,
    K_MUTATE,
    K_UTIL,
    K_COUNT
};

// Counters written by the kernels of one pass (device memory, cleared by the
// init kernel at the start of each pass).
struct DevCounters {
    unsigned long long wmax_bits;  // w_max as the bit pattern of a non-negative double
    unsigned long long n_border;
    unsigned long long sum_dprime;
    unsigned long long sum_ell;
    unsigned long long sum_ell_x;  // records of foreign communities
    unsigned long long sum_tI;
    unsigned long long sum_tII;
    unsigned long long sum_workI;
    unsigned int bcount[kScoreBins];  // border vertices per foreign-degree bin
    unsigned int pad;
};

// Ranking key: score bits (a non-negative double orders like its bits) and
// the complement of the caller id, so that a larger key ranks first.
struct TopkKey {
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
    void *off = nullptr;       // OffT[n+1]
    int32_t *deg = nullptr;    // [n]
    int32_t *col = nullptr;    // [nnz]
    int32_t *lab = nullptr;    // [n] internal community id
    int32_t *new2old = nullptr;// [n]
    uint8_t *alive = nullptr;  // [n]
    int32_t *sched = nullptr;  // [n] vertices grouped by row bin
    // interaction matrix records
    int32_t *hkey = nullptr, *hpos = nullptr;
    double *hw = nullptr, *hS = nullptr;
    // per-vertex results
    int32_t *ell = nullptr, *pq = nullptr;  // pq: 2 ints per vertex (p, q)
    double *wown = nullptr, *a = nullptr, *R = nullptr;
    long long *tI = nullptr, *tII = nullptr;
    int32_t *blist = nullptr;  // [kScoreBins * n] border vertices by foreign-degree bin
    DevCounters *ctr = nullptr;
    // top-k
    unsigned int *thist = nullptr;  // [kTopkBins]
    TopkState *tstate = nullptr;
    TopkKey *tfinal = nullptr, *ttie = nullptr, *ttie2 = nullptr;  // [n] each
    int32_t *tout_ids = nullptr;
    double *tout_sc = nullptr;
    // scratch for removals and readers
    int32_t *scratch_i = nullptr;   // [max(n, nnz)] ints
    double *scratch_d = nullptr;    // [n] doubles
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
    int64_t row_bin_lo[rs::kRowBins + 1] = {};  // start of each row bin in sched
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
rs_status launch_remove_edges(rs_graph *g, const int32_t *d_src, const int32_t *d_dst, int64_t m,
                              unsigned long long *d_removed);
rs_status launch_remove_vertices(rs_graph *g, const int32_t *d_verts, int64_t nv,
                                 unsigned long long *d_removed_edges);
rs_status launch_compact_rows(rs_graph *g);
rs_status launch_gather_scores(rs_graph *g, double *d_out, int raw);

}  // namespace rs
