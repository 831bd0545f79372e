// rs_kernels.hip -- HIP kernels of the robust-spanner scoring pass (gfx950, wave64).
//
// One pass (rs_score) is three kernels over the resident graph:
//   k_rows   Algorithm 1 Steps 1-2 fused: for every vertex, gather the labels
//            of its neighbours, run-length count them into interaction-matrix
//            records (community, count), detect the border vertex, compute the
//            Algorithm 2 / Eq. H_optimal weights of every record and the
//            vertex's own-community weight, and reduce w_max.  Teams of 8..64
//            lanes per vertex by (load-time) degree bin.
//   k_sagg   type-II aggregate: for every foreign record (w, c) of a border
//            vertex, S_w(c) = sum of a_x = cbrt(w_x(C(x))) over the run.
//   k_score  Eq. RSI per border vertex u, in the per-(vertex, community)
//            factorised form (Lemmas 1-2): every type-II triad through w
//            contributes w_w(C(u))^(2/3) a_v, and the type-I triads are the
//            common foreign neighbours of u and w, found by sorted-list
//            intersection (Section IV, Step 3).  One owner per vertex, fixed
//            summation order, no floating-point atomics.
// Top-k (Algorithm 1 Step 4) is an exact radix select on the 96-bit key
// (score bits, complement of the caller id) with 16-bit digits.
#include <climits>

#include "rs_internal.h"

namespace rs {

// ------------------------------------------------------------ team helpers
template <int T>
struct Team {
    int lane;  // lane within the team
    int base;  // first wavefront lane of the team
    __device__ __forceinline__ Team() {
        int l = (int)__lane_id();
        lane = l & (T - 1);
        base = l & ~(T - 1);
    }
    __device__ __forceinline__ unsigned long long ballot(bool p) const {
        unsigned long long m = __ballot(p);
        if (T == 64) return m;
        return (m >> base) & ((1ull << T) - 1ull);
    }
    template <class V>
    __device__ __forceinline__ V bcast(V v, int src) const { return __shfl(v, src, T); }
    template <class V>
    __device__ __forceinline__ V up1(V v) const { return __shfl_up(v, 1, T); }
    __device__ __forceinline__ double sum(double x) const {
#pragma unroll
        for (int o = T / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, T);
        return x;
    }
    __device__ __forceinline__ long long sum(long long x) const {
#pragma unroll
        for (int o = T / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, T);
        return x;
    }
    __device__ __forceinline__ int imax(int x) const {
#pragma unroll
        for (int o = T / 2; o > 0; o >>= 1) x = max(x, __shfl_xor(x, o, T));
        return x;
    }
    __device__ __forceinline__ double dmax(double x) const {
#pragma unroll
        for (int o = T / 2; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o, T));
        return x;
    }
};

__device__ __forceinline__ unsigned long long dbits(double x) {
    return (unsigned long long)__double_as_longlong(x);
}

// ------------------------------------------------------------ weights
// Eq. H_optimal with Algorithm 2's shared terms: for a vertex of degree d
// whose neighbour-community counts have X = sum f log2 f over ell distinct
// communities, the weight toward a community with count f > 0 is
//   H = -(X - d log2(d - f) - f log2(f / (d - f))) / (d - f),  w = H (ell - 1),
// and toward a community absent from the neighbourhood (f = 0, only the own
// community can be) H = log2 d - X / d with |L| = ell (Eq. weight).
// |L| <= 1 means a single remaining community: H = 0 exactly.
__device__ __forceinline__ double weight_present(int d, double X, int ell, int f) {
    int L = ell - 1;
    if (L < 2) return 0.0;
    double Y = (double)(d - f);
    double fd = (double)f;
    double H = -(X - (double)d * log2(Y) - fd * log2(fd / Y)) / Y;
    return H * (double)L;
}

__device__ __forceinline__ double weight_absent(int d, double X, int ell) {
    if (ell < 2) return 0.0;
    double Y = (double)d;
    double H = -(X - Y * log2(Y)) / Y;
    return H * (double)ell;
}

__device__ __forceinline__ double flogf(int f) { return f > 1 ? (double)f * log2((double)f) : 0.0; }

// ------------------------------------------------------------ init
__global__ void k_init(DevCounters *c) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        c->wmax_bits = 0;
        c->n_border = 0;
        c->sum_dprime = 0;
        c->sum_ell = 0;
        c->sum_ell_x = 0;
        c->sum_tI = 0;
        c->sum_tII = 0;
        c->sum_workI = 0;
        for (int b = 0; b < kScoreBins; ++b) c->bcount[b] = 0;
    }
}

// ------------------------------------------------------------ k_rows
template <typename OffT>
struct RowArgs {
    const OffT *off;
    const int32_t *deg, *col, *lab, *sched;
    int32_t *hkey, *hpos;
    double *hw;
    int32_t *ell, *pq;
    double *wown, *a, *R;
    long long *tI, *tII;
    int32_t *blist;
    long long n;
    DevCounters *ctr;
    long long bin_lo[kRowBins + 1];  // vertex ranges of the bins in sched
    int blk_lo[kRowBins + 1];        // block ranges of the bins in the grid
};

struct RowResult {
    int ell, p, q;
    double wown, lmax;
};

// A row that fits one team pass (d <= T): everything stays in registers.
template <int T, typename OffT>
__device__ __forceinline__ RowResult row_single(const RowArgs<OffT> &A, const Team<T> &tm, OffT rb,
                                                int d, int cv) {
    const int i = tm.lane;
    const bool valid = i < d;
    const int c = valid ? A.lab[A.col[rb + i]] : INT_MAX;
    int pc = tm.up1(c);
    if (i == 0) pc = -1;
    const bool start = valid && c != pc;
    const unsigned long long m = tm.ballot(start);
    const int ell = __popcll(m);
    int f = 0;
    if (start) {
        unsigned long long rest = (i + 1 < T) ? (m >> (i + 1)) : 0ull;
        int nxt = rest ? (i + 1 + __builtin_ctzll(rest)) : d;
        f = nxt - i;
    }
    const double X = tm.sum(start ? flogf(f) : 0.0);
    const unsigned long long mo = tm.ballot(start && c == cv);
    RowResult r;
    r.ell = ell;
    int fown;
    if (mo) {
        int ol = __builtin_ctzll(mo);
        fown = tm.bcast(f, ol);
        r.p = ol;
    } else {
        fown = 0;
        r.p = __popcll(tm.ballot(valid && c < cv));
    }
    r.q = r.p + fown;
    double lmax = 0.0;
    if (start) {
        const double w = weight_present(d, X, ell, f);
        const int slot = __popcll(m & ((1ull << i) - 1ull));
        A.hkey[rb + slot] = c;
        A.hpos[rb + slot] = i;
        A.hw[rb + slot] = w;
        lmax = w;
    }
    r.wown = fown > 0 ? weight_present(d, X, ell, fown) : weight_absent(d, X, ell);
    r.lmax = fmax(tm.dmax(lmax), r.wown);
    return r;
}

// A longer row: run starts are written to the record slots, then re-read.
template <int T, typename OffT>
__device__ __forceinline__ RowResult row_multi(const RowArgs<OffT> &A, const Team<T> &tm, OffT rb,
                                               int d, int cv) {
    int nruns = 0, prev = -1;
    for (int b = 0; b < d; b += T) {
        const int i = b + tm.lane;
        const bool valid = i < d;
        const int c = valid ? A.lab[A.col[rb + i]] : INT_MAX;
        int pc = tm.up1(c);
        if (tm.lane == 0) pc = prev;
        const bool start = valid && c != pc;
        const unsigned long long m = tm.ballot(start);
        if (start) {
            const int slot = nruns + __popcll(m & ((1ull << tm.lane) - 1ull));
            A.hkey[rb + slot] = c;
            A.hpos[rb + slot] = i;
        }
        nruns += __popcll(m);
        prev = tm.bcast(c, T - 1);
    }
    __threadfence_block();
    const int ell = nruns;
    double xp = 0.0;
    int fown = 0, pown = -1, pend = 0;
    for (int r = tm.lane; r < ell; r += T) {
        const int s = A.hpos[rb + r];
        const int e = (r + 1 < ell) ? A.hpos[rb + r + 1] : d;
        const int c = A.hkey[rb + r];
        xp += flogf(e - s);
        if (c == cv) {
            fown = e - s;
            pown = s;
        }
        if (c < cv) pend = max(pend, e);
    }
    const double X = tm.sum(xp);
    fown = tm.imax(fown);
    pown = tm.imax(pown);
    pend = tm.imax(pend);
    RowResult res;
    res.ell = ell;
    res.p = fown > 0 ? pown : pend;
    res.q = res.p + fown;
    double lmax = 0.0;
    for (int r = tm.lane; r < ell; r += T) {
        const int s = A.hpos[rb + r];
        const int e = (r + 1 < ell) ? A.hpos[rb + r + 1] : d;
        const double w = weight_present(d, X, ell, e - s);
        A.hw[rb + r] = w;
        lmax = fmax(lmax, w);
    }
    res.wown = fown > 0 ? weight_present(d, X, ell, fown) : weight_absent(d, X, ell);
    res.lmax = fmax(tm.dmax(lmax), res.wown);
    return res;
}

__device__ __forceinline__ int score_bin_of(int dprime) {
    return dprime <= kScoreBinMax[0] ? 0 : (dprime <= kScoreBinMax[1] ? 1 : 2);
}

// Blocks are dealt round-robin to the 8 XCDs; remap so that each XCD works on
// a contiguous eighth of the bin (neighbouring vertex ids share communities,
// so their label and record reads share that XCD's L2).
__device__ __forceinline__ int xcd_remap(int blk, int nblk) {
    const int x = blk & 7, j = blk >> 3;
    const int per = nblk >> 3, rem = nblk & 7;
    return x * per + min(x, rem) + j;
}

template <int T, typename OffT>
__device__ void rows_bin(const RowArgs<OffT> &A, int bin, int blk, int nblk) {
    __shared__ unsigned long long s_wmax, s_nb, s_dp, s_ell, s_ellx;
    __shared__ unsigned int s_cnt[kScoreBins], s_base[kScoreBins];
    if (threadIdx.x == 0) {
        s_wmax = 0;
        s_nb = s_dp = s_ell = s_ellx = 0;
        for (int b = 0; b < kScoreBins; ++b) s_cnt[b] = 0;
    }
    __syncthreads();
    const Team<T> tm;
    const int lb = xcd_remap(blk, nblk);
    const long long idx = A.bin_lo[bin] + (long long)lb * (kBlock / T) + threadIdx.x / T;
    const bool has = idx < A.bin_lo[bin + 1];
    int v = -1, sbin = -1, lpos = 0;
    if (has) {
        v = A.sched[idx];
        const OffT rb = A.off[v];
        const int d = A.deg[v];
        const int cv = A.lab[v];
        const RowResult r = (d <= T) ? row_single<T, OffT>(A, tm, rb, d, cv) : row_multi<T, OffT>(A, tm, rb, d, cv);
        if (tm.lane == 0) {
            const int dprime = d - (r.q - r.p);
            A.ell[v] = r.ell;
            A.pq[2 * (long long)v] = r.p;
            A.pq[2 * (long long)v + 1] = r.q;
            A.wown[v] = r.wown;
            A.a[v] = cbrt(r.wown);
            atomicMax(&s_wmax, dbits(r.lmax));
            atomicAdd(&s_ell, (unsigned long long)r.ell);
            atomicAdd(&s_ellx, (unsigned long long)(r.ell - (r.q > r.p ? 1 : 0)));
            if (dprime > 0) {
                atomicAdd(&s_nb, 1ull);
                atomicAdd(&s_dp, (unsigned long long)dprime);
                sbin = score_bin_of(dprime);
                lpos = (int)atomicAdd(&s_cnt[sbin], 1u);
            } else {
                A.R[v] = 0.0;
                A.tI[v] = 0;
                A.tII[v] = 0;
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        atomicMax(&A.ctr->wmax_bits, s_wmax);
        atomicAdd(&A.ctr->n_border, s_nb);
        atomicAdd(&A.ctr->sum_dprime, s_dp);
        atomicAdd(&A.ctr->sum_ell, s_ell);
        atomicAdd(&A.ctr->sum_ell_x, s_ellx);
        for (int b = 0; b < kScoreBins; ++b)
            s_base[b] = s_cnt[b] ? atomicAdd(&A.ctr->bcount[b], s_cnt[b]) : 0u;
    }
    __syncthreads();
    if (sbin >= 0) A.blist[(long long)sbin * A.n + s_base[sbin] + lpos] = v;
}

template <typename OffT>
__global__ __launch_bounds__(kBlock) void k_rows(RowArgs<OffT> A) {
    const int b = blockIdx.x;
    if (b < A.blk_lo[1])
        rows_bin<8, OffT>(A, 0, b - A.blk_lo[0], A.blk_lo[1] - A.blk_lo[0]);
    else if (b < A.blk_lo[2])
        rows_bin<16, OffT>(A, 1, b - A.blk_lo[1], A.blk_lo[2] - A.blk_lo[1]);
    else if (b < A.blk_lo[3])
        rows_bin<32, OffT>(A, 2, b - A.blk_lo[2], A.blk_lo[3] - A.blk_lo[2]);
    else
        rows_bin<64, OffT>(A, 3, b - A.blk_lo[3], A.blk_lo[4] - A.blk_lo[3]);
}

// ------------------------------------------------------------ shared args
template <typename OffT>
struct PassArgs {
    const OffT *off;
    const int32_t *deg, *col, *lab;
    const int32_t *hkey, *hpos;
    const double *hw;
    double *hS;
    const int32_t *ell, *pq;
    const double *a;
    double *R;
    long long *tI, *tII;
    const int32_t *blist;
    long long n;
    DevCounters *ctr;
};

// ------------------------------------------------------------ k_sagg
// S_w(c) for every foreign record of a border vertex w: one lane per run,
// summing a_x over the run's row positions in order.
template <int T, typename OffT>
__device__ __forceinline__ void sagg_vertex(const PassArgs<OffT> &A, const Team<T> &tm, int w) {
    const OffT rb = A.off[w];
    const int d = A.deg[w];
    const int ell = A.ell[w];
    const int cw = A.lab[w];
    for (int r = tm.lane; r < ell; r += T) {
        if (A.hkey[rb + r] == cw) continue;
        const int s = A.hpos[rb + r];
        const int e = (r + 1 < ell) ? A.hpos[rb + r + 1] : d;
        double acc = 0.0;
        for (int i = s; i < e; ++i) acc += A.a[A.col[rb + i]];
        A.hS[rb + r] = acc;
    }
}

template <int T, typename OffT>
__device__ __forceinline__ void sagg_bin(const PassArgs<OffT> &A, int bin) {
    const Team<T> tm;
    const long long cnt = A.ctr->bcount[bin];
    const int per = kBlock / T;
    for (long long i = (long long)blockIdx.x * per + threadIdx.x / T; i < cnt; i += (long long)gridDim.x * per)
        sagg_vertex<T, OffT>(A, tm, A.blist[(long long)bin * A.n + i]);
}

template <typename OffT>
__global__ __launch_bounds__(kBlock) void k_sagg(PassArgs<OffT> A) {
    sagg_bin<4, OffT>(A, 0);
    sagg_bin<16, OffT>(A, 1);
    sagg_bin<64, OffT>(A, 2);
}

// ------------------------------------------------------------ k_score
// Position of community c among the records of x (c is known to be present).
template <typename OffT>
__device__ __forceinline__ int find_rec(const PassArgs<OffT> &A, OffT rb, int ell, int c) {
    int lo = 0, hi = ell - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (A.hkey[rb + mid] < c)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// The foreign neighbours of x are its row minus the own-community sub-range
// [p, q); j-th foreign neighbour, ascending.
struct Foreign {
    long long rb;
    int p, h, n;  // p, q - p, number of foreign neighbours
};

template <typename OffT>
__device__ __forceinline__ Foreign foreign_of(const PassArgs<OffT> &A, int x) {
    Foreign f;
    f.rb = (long long)A.off[x];
    f.p = A.pq[2 * (long long)x];
    f.h = A.pq[2 * (long long)x + 1] - f.p;
    f.n = A.deg[x] - f.h;
    return f;
}

template <typename OffT>
__device__ __forceinline__ int fget(const PassArgs<OffT> &A, const Foreign &f, int j) {
    return A.col[f.rb + (j < f.p ? j : j + f.h)];
}

// Lower bound of value y in the foreign list f, searching [lo, f.n).
template <typename OffT>
__device__ __forceinline__ int flower(const PassArgs<OffT> &A, const Foreign &f, int lo, int y) {
    int hi = f.n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (fget(A, f, mid) < y)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

template <typename OffT>
__device__ __forceinline__ double weight_of(const PassArgs<OffT> &A, int x, int c) {
    const OffT rb = A.off[x];
    return A.hw[rb + find_rec(A, rb, A.ell[x], c)];
}

template <int T, typename OffT>
__device__ __forceinline__ void score_vertex(const PassArgs<OffT> &A, const Team<T> &tm, int u, double wmax,
                                             long long &wI) {
    const int cu = A.lab[u];
    const int du = A.deg[u];
    const double au = A.a[u];
    const Foreign fu = foreign_of(A, u);
    double acc = 0.0;
    long long cI = 0, cII = 0;
    for (int j = tm.lane; j < fu.n; j += T) {
        const int w = fget(A, fu, j);
        const OffT rbw = A.off[w];
        const int ellw = A.ell[w];
        const int s = find_rec(A, rbw, ellw, cu);
        const double W = A.hw[rbw + s];
        const double S = A.hS[rbw + s];
        const int F = ((s + 1 < ellw) ? A.hpos[rbw + s + 1] : A.deg[w]) - A.hpos[rbw + s];
        cII += F - 1;
        const double c1 = cbrt(W);
        acc += c1 * c1 * (S - au);
        // type-I: common foreign neighbours of u and w
        const Foreign fw = foreign_of(A, w);
        const bool u_short = fu.n <= fw.n;
        const Foreign &fs = u_short ? fu : fw;
        const Foreign &fl = u_short ? fw : fu;
        wI += fs.n;
        int lo = 0;
        for (int t = 0; t < fs.n && lo < fl.n; ++t) {
            const int y = fget(A, fs, t);
            lo = flower(A, fl, lo, y);
            if (lo < fl.n && fget(A, fl, lo) == y) {
                const double wv = weight_of(A, y, cu);
                const double wwv = A.hw[rbw + find_rec(A, rbw, ellw, A.lab[y])];
                acc += cbrt(W * wv * wwv);
                ++cI;
                ++lo;
            }
        }
    }
    acc = tm.sum(acc);
    cI = tm.sum(cI);
    cII = tm.sum(cII);
    if (tm.lane == 0) {
        A.R[u] = (du >= 2 && wmax > 0.0) ? acc / wmax / (double)((long long)du * (du - 1)) : 0.0;
        A.tI[u] = cI;
        A.tII[u] = cII;
    }
}

template <int T, typename OffT>
__device__ __forceinline__ void score_bin(const PassArgs<OffT> &A, int bin, double wmax, long long &cI,
                                          long long &cII, long long &wI) {
    const Team<T> tm;
    const long long cnt = A.ctr->bcount[bin];
    const int per = kBlock / T;
    for (long long i = (long long)blockIdx.x * per + threadIdx.x / T; i < cnt; i += (long long)gridDim.x * per) {
        const int u = A.blist[(long long)bin * A.n + i];
        score_vertex<T, OffT>(A, tm, u, wmax, wI);
        if (tm.lane == 0) {
            cI += A.tI[u];
            cII += A.tII[u];
        }
    }
}

template <typename OffT>
__global__ __launch_bounds__(kBlock) void k_score(PassArgs<OffT> A) {
    const double wmax = __longlong_as_double((long long)A.ctr->wmax_bits);
    long long cI = 0, cII = 0, wI = 0;
    score_bin<4, OffT>(A, 0, wmax, cI, cII, wI);
    score_bin<16, OffT>(A, 1, wmax, cI, cII, wI);
    score_bin<64, OffT>(A, 2, wmax, cI, cII, wI);
    __shared__ unsigned long long s[3];
    if (threadIdx.x == 0) s[0] = s[1] = s[2] = 0;
    __syncthreads();
    for (int o = 32; o > 0; o >>= 1) {
        cI += __shfl_xor(cI, o);
        cII += __shfl_xor(cII, o);
        wI += __shfl_xor(wI, o);
    }
    if (__lane_id() == 0) {
        atomicAdd(&s[0], (unsigned long long)cI);
        atomicAdd(&s[1], (unsigned long long)cII);
        atomicAdd(&s[2], (unsigned long long)wI);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (s[0]) atomicAdd(&A.ctr->sum_tI, s[0]);
        if (s[1]) atomicAdd(&A.ctr->sum_tII, s[1]);
        if (s[2]) atomicAdd(&A.ctr->sum_workI, s[2]);
    }
}

// ------------------------------------------------------------ pass launcher
static inline int grid_for(long long items, int per_block, int cap) {
    long long g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

template <typename OffT>
static rs_status score_pass_t(rs_graph *g) {
    DeviceGraph &D = g->d;
    hipEvent_t ev;
    timing_begin(g, K_INIT, &ev);
    hipLaunchKernelGGL(k_init, dim3(1), dim3(64), 0, g->stream, D.ctr);
    timing_end(g, K_INIT, ev);

    RowArgs<OffT> A;
    A.off = (const OffT *)D.off;
    A.deg = D.deg;
    A.col = D.col;
    A.lab = D.lab;
    A.sched = D.sched;
    A.hkey = D.hkey;
    A.hpos = D.hpos;
    A.hw = D.hw;
    A.ell = D.ell;
    A.pq = D.pq;
    A.wown = D.wown;
    A.a = D.a;
    A.R = D.R;
    A.tI = D.tI;
    A.tII = D.tII;
    A.blist = D.blist;
    A.n = D.n;
    A.ctr = D.ctr;
    int blocks = 0;
    for (int b = 0; b < kRowBins; ++b) {
        A.bin_lo[b] = g->row_bin_lo[b];
        A.blk_lo[b] = blocks;
        long long cnt = g->row_bin_lo[b + 1] - g->row_bin_lo[b];
        int per = kBlock / kRowTeam[b];
        // a multiple of 8 blocks per bin keeps xcd_remap's grouping aligned
        // with the hardware's round-robin block-to-XCD assignment
        blocks += (int)(((cnt + per - 1) / per + 7) / 8 * 8);
    }
    A.bin_lo[kRowBins] = g->row_bin_lo[kRowBins];
    A.blk_lo[kRowBins] = blocks;
    if (blocks > 0) {
        timing_begin(g, K_ROWS, &ev);
        hipLaunchKernelGGL(k_rows<OffT>, dim3(blocks), dim3(kBlock), 0, g->stream, A);
        timing_end(g, K_ROWS, ev);
    }

    PassArgs<OffT> P;
    P.off = (const OffT *)D.off;
    P.deg = D.deg;
    P.col = D.col;
    P.lab = D.lab;
    P.hkey = D.hkey;
    P.hpos = D.hpos;
    P.hw = D.hw;
    P.hS = D.hS;
    P.ell = D.ell;
    P.pq = D.pq;
    P.a = D.a;
    P.R = D.R;
    P.tI = D.tI;
    P.tII = D.tII;
    P.blist = D.blist;
    P.n = D.n;
    P.ctr = D.ctr;
    const int grid = grid_for(D.n, kBlock / 4, 2048);
    timing_begin(g, K_SAGG, &ev);
    hipLaunchKernelGGL(k_sagg<OffT>, dim3(grid), dim3(kBlock), 0, g->stream, P);
    timing_end(g, K_SAGG, ev);
    timing_begin(g, K_SCORE, &ev);
    hipLaunchKernelGGL(k_score<OffT>, dim3(grid), dim3(kBlock), 0, g->stream, P);
    timing_end(g, K_SCORE, ev);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "score pass launch");
    return RS_OK;
}

rs_status launch_score_pass(rs_graph *g) {
    return g->d.off64 ? score_pass_t<long long>(g) : score_pass_t<int32_t>(g);
}

// ------------------------------------------------------------ top-k
__device__ __forceinline__ bool key_gt(const TopkKey &a, const TopkKey &b) {
    return a.hi > b.hi || (a.hi == b.hi && a.lo > b.lo);
}

__device__ __forceinline__ unsigned int key_digit(const TopkKey &k, int j) {
    switch (j) {
        case 0: return (unsigned int)(k.hi >> 48);
        case 1: return (unsigned int)(k.hi >> 32) & 0xffffu;
        case 2: return (unsigned int)(k.hi >> 16) & 0xffffu;
        case 3: return (unsigned int)k.hi & 0xffffu;
        case 4: return k.lo >> 16;
        default: return k.lo & 0xffffu;
    }
}

__device__ __forceinline__ TopkKey make_key(const double *R, const int32_t *new2old, int v) {
    TopkKey k;
    k.hi = dbits(R[v]) & 0x7fffffffffffffffull;  // scores are >= 0; never rank a -0.0 first
    k.lo = 0xffffffffu - (unsigned int)new2old[v];
    k.v = v;
    return k;
}

// Wavefront-aggregated histogram increment.
__device__ __forceinline__ void hist_add(unsigned int *hist, bool act, unsigned int dig) {
    unsigned long long live = __ballot(act);
    while (live) {
        const int leader = __builtin_ctzll(live);
        const unsigned int dl = __shfl(dig, leader);
        const unsigned long long same = __ballot(act && dig == dl) & live;
        if ((int)__lane_id() == leader) atomicAdd(&hist[dl], (unsigned int)__popcll(same));
        live &= ~same;
    }
}

// Append the lanes with `act` to list[*counter ...] (wavefront-aggregated).
__device__ __forceinline__ void list_push(TopkKey *list, unsigned long long *counter, bool act, const TopkKey &k) {
    const unsigned long long m = __ballot(act);
    if (!m) return;
    const int leader = __builtin_ctzll(m);
    unsigned long long base = 0;
    if ((int)__lane_id() == leader) base = atomicAdd(counter, (unsigned long long)__popcll(m));
    base = __shfl(base, leader);
    if (act) list[base + __popcll(m & ((1ull << __lane_id()) - 1ull))] = k;
}

// Level-0 histogram over every live vertex.
__global__ __launch_bounds__(kBlock) void k_topk_hist(const double *R, const int32_t *new2old, const uint8_t *alive,
                                                      long long n, unsigned int *hist) {
    for (long long base = (long long)blockIdx.x * kBlock; base < n; base += (long long)gridDim.x * kBlock) {
        const long long v = base + threadIdx.x;
        const bool act = v < n && alive[v];
        unsigned int dig = 0;
        if (act) dig = key_digit(make_key(R, new2old, (int)v), 0);
        hist_add(hist, act, dig);
    }
}

// Histogram of digit j over a key list.
__global__ __launch_bounds__(kBlock) void k_list_hist(const TopkKey *list, const unsigned long long *count, int j,
                                                      unsigned int *hist) {
    const long long n = (long long)*count;
    for (long long base = (long long)blockIdx.x * kBlock; base < n; base += (long long)gridDim.x * kBlock) {
        const long long i = base + threadIdx.x;
        const bool act = i < n;
        unsigned int dig = 0;
        if (act) dig = key_digit(list[i], j);
        hist_add(hist, act, dig);
    }
}

// One block of 1024 threads: find the threshold digit of the current level,
// record it, and clear the histogram for the next use.
__global__ __launch_bounds__(1024) void k_topk_find(unsigned int *hist, TopkState *st, int level) {
    __shared__ long long s_scan[1024];
    __shared__ long long s_total;
    const int t = threadIdx.x;
    const long long need = st->take;
    // thread t owns bins [hiB - 63, hiB] with hiB = 65535 - 64 t (descending order)
    const int hiB = kTopkBins - 1 - 64 * t;
    long long mine = 0;
    for (int b = 0; b < 64; ++b) mine += hist[hiB - b];
    s_scan[t] = mine;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {  // inclusive scan
        long long x = t >= o ? s_scan[t - o] : 0;
        __syncthreads();
        s_scan[t] += x;
        __syncthreads();
    }
    const long long incl = s_scan[t];
    const long long excl = incl - mine;
    if (t == 1023) s_total = incl;
    __syncthreads();
    if (excl < need && need <= incl) {
        long long cum = excl;
        for (int b = 0; b < 64; ++b) {
            const long long h = hist[hiB - b];
            if (cum + h >= need) {
                st->digit = level;
                st->thresh = (unsigned int)(hiB - b);
                st->above += cum;
                st->take = need - cum;
                st->binsize = h;
                st->done = (need - cum == h) ? 1u : 0u;
                break;
            }
            cum += h;
        }
    }
    if (t == 0 && !(need > 0 && s_total >= need)) {  // cannot happen for need <= live keys: take all
        st->digit = level;
        st->thresh = 0;
        st->take = 0;
        st->binsize = 0;
        st->done = 1u;
    }
    __syncthreads();
    for (int b = 0; b < 64; ++b) hist[hiB - b] = 0;
}

__global__ __launch_bounds__(kBlock) void k_topk_collect(const double *R, const int32_t *new2old, const uint8_t *alive,
                                                         long long n, TopkState *st, TopkKey *fin, TopkKey *tie) {
    const unsigned int th = st->thresh;
    const bool done = st->done != 0u;
    for (long long base = (long long)blockIdx.x * kBlock; base < n; base += (long long)gridDim.x * kBlock) {
        const long long v = base + threadIdx.x;
        const bool act = v < n && alive[v];
        TopkKey k;
        unsigned int dig = 0;
        if (act) {
            k = make_key(R, new2old, (int)v);
            dig = key_digit(k, 0);
        }
        const bool to_final = act && (dig > th || (dig == th && done));
        const bool to_tie = act && dig == th && !done;
        list_push(fin, &st->n_final, to_final, k);
        list_push(tie, &st->n_tie, to_tie, k);
    }
}

__global__ __launch_bounds__(kBlock) void k_list_collect(const TopkKey *list, const unsigned long long *count,
                                                         TopkState *st, TopkKey *fin, TopkKey *tie,
                                                         unsigned long long *tie_count) {
    const long long n = (long long)*count;
    const int j = st->digit;
    const unsigned int th = st->thresh;
    const bool done = st->done != 0u;
    for (long long base = (long long)blockIdx.x * kBlock; base < n; base += (long long)gridDim.x * kBlock) {
        const long long i = base + threadIdx.x;
        const bool act = i < n;
        TopkKey k;
        unsigned int dig = 0;
        if (act) {
            k = list[i];
            dig = key_digit(k, j);
        }
        list_push(fin, &st->n_final, act && (dig > th || (dig == th && done)), k);
        list_push(tie, tie_count, act && dig == th && !done, k);
    }
}

// Rank every key of `list` among the keys of `list` by pairwise comparison.
// mode 0 (tie class): keys ranked below st->take are appended to the final list.
// mode 1 (final list): key of rank r is written to the output at position r.
__global__ __launch_bounds__(kBlock) void k_pair_rank(const TopkKey *list, const unsigned long long *count,
                                                      TopkState *st, int mode, TopkKey *fin,
                                                      const double *R, const int32_t *new2old, int32_t *out_ids,
                                                      double *out_sc) {
    __shared__ TopkKey tile[kBlock];
    const long long n = (long long)*count;
    if (mode == 0 && (st->done || n > kTieCap)) {
        if (mode == 0 && !st->done && n > kTieCap && blockIdx.x == 0 && threadIdx.x == 0) st->overflow = 1u;
        return;
    }
    if (mode == 1 && st->overflow) return;
    for (long long base = (long long)blockIdx.x * kBlock; base < n; base += (long long)gridDim.x * kBlock) {
        const long long i = base + threadIdx.x;
        TopkKey me;
        me.hi = 0;
        me.lo = 0;
        me.v = -1;
        if (i < n) me = list[i];
        long long rank = 0;
        for (long long t0 = 0; t0 < n; t0 += kBlock) {
            __syncthreads();
            if (t0 + threadIdx.x < n) tile[threadIdx.x] = list[t0 + threadIdx.x];
            __syncthreads();
            const int lim = (int)min((long long)kBlock, n - t0);
            for (int jj = 0; jj < lim; ++jj) rank += key_gt(tile[jj], me) ? 1 : 0;
        }
        if (i < n) {
            if (mode == 0) {
                if (rank < st->take) {
                    const unsigned long long pos = atomicAdd(&st->n_final, 1ull);
                    fin[pos] = me;
                }
            } else {
                out_ids[rank] = new2old[me.v];
                out_sc[rank] = R[me.v];
            }
        }
    }
}

__global__ void k_topk_setup(TopkState *st, long long k) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->k = k;
        st->digit = 0;
        st->thresh = 0;
        st->above = 0;
        st->take = k;
        st->binsize = 0;
        st->n_final = 0;
        st->n_tie = 0;
        st->overflow = 0;
        st->done = 0;
    }
}

__global__ void k_zero_u64(unsigned long long *p) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0;
}

rs_status launch_topk(rs_graph *g, int64_t k, int64_t *count) {
    DeviceGraph &D = g->d;
    const long long keff = k < g->n_alive ? k : g->n_alive;
    *count = keff;
    if (keff <= 0) return RS_OK;
    hipEvent_t ev;
    const int grid_n = grid_for(D.n, kBlock, 4096);
    hipLaunchKernelGGL(k_topk_setup, dim3(1), dim3(64), 0, g->stream, D.tstate, keff);
    timing_begin(g, K_TOPK_HIST, &ev);
    hipLaunchKernelGGL(k_topk_hist, dim3(grid_n), dim3(kBlock), 0, g->stream, D.R, D.new2old, D.alive, D.n, D.thist);
    timing_end(g, K_TOPK_HIST, ev);
    timing_begin(g, K_TOPK_FIND, &ev);
    hipLaunchKernelGGL(k_topk_find, dim3(1), dim3(1024), 0, g->stream, D.thist, D.tstate, 0);
    timing_end(g, K_TOPK_FIND, ev);
    timing_begin(g, K_TOPK_COLLECT, &ev);
    hipLaunchKernelGGL(k_topk_collect, dim3(grid_n), dim3(kBlock), 0, g->stream, D.R, D.new2old, D.alive, D.n,
                       D.tstate, D.tfinal, D.ttie);
    timing_end(g, K_TOPK_COLLECT, ev);
    const unsigned long long *n_tie = &D.tstate->n_tie;
    const unsigned long long *n_fin = &D.tstate->n_final;
    timing_begin(g, K_TOPK_TIE, &ev);
    hipLaunchKernelGGL(k_pair_rank, dim3(kTieCap / kBlock), dim3(kBlock), 0, g->stream, D.ttie, n_tie, D.tstate, 0,
                       D.tfinal, D.R, D.new2old, D.tout_ids, D.tout_sc);
    timing_end(g, K_TOPK_TIE, ev);
    const int grid_k = grid_for(keff, kBlock, 4096);
    timing_begin(g, K_TOPK_RANK, &ev);
    hipLaunchKernelGGL(k_pair_rank, dim3(grid_k), dim3(kBlock), 0, g->stream, D.tfinal, n_fin, D.tstate, 1, D.tfinal,
                       D.R, D.new2old, D.tout_ids, D.tout_sc);
    timing_end(g, K_TOPK_RANK, ev);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "top-k launch");

    TopkState st;
    e = hipMemcpyAsync(&st, D.tstate, sizeof(st), hipMemcpyDeviceToHost, g->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    if (e != hipSuccess) return hip_fail(e, "top-k state read");
    if (!st.overflow) return RS_OK;

    // A tie class larger than the pairwise ranker: refine it digit by digit.
    TopkKey *cur = D.ttie, *nxt = D.ttie2;
    unsigned long long *cnt_dev = nullptr;
    e = hipMalloc(&cnt_dev, 2 * sizeof(unsigned long long));
    if (e != hipSuccess) return hip_fail(e, "top-k refine counter");
    e = hipMemcpyAsync(cnt_dev, &st.n_tie, sizeof(unsigned long long), hipMemcpyHostToDevice, g->stream);
    for (int j = 1; j <= 5 && e == hipSuccess; ++j) {
        long long cur_n = 0;
        e = hipMemcpyAsync(&cur_n, cnt_dev, sizeof(long long), hipMemcpyDeviceToHost, g->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
        if (e != hipSuccess) break;
        const int grid_l = grid_for(cur_n, kBlock, 4096);
        hipLaunchKernelGGL(k_list_hist, dim3(grid_l), dim3(kBlock), 0, g->stream, cur, cnt_dev, j, D.thist);
        hipLaunchKernelGGL(k_topk_find, dim3(1), dim3(1024), 0, g->stream, D.thist, D.tstate, j);
        hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, g->stream, cnt_dev + 1);
        hipLaunchKernelGGL(k_list_collect, dim3(grid_l), dim3(kBlock), 0, g->stream, cur, cnt_dev, D.tstate,
                           D.tfinal, nxt, cnt_dev + 1);
        e = hipMemcpyAsync(cnt_dev, cnt_dev + 1, sizeof(unsigned long long), hipMemcpyDeviceToDevice, g->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(&st, D.tstate, sizeof(st), hipMemcpyDeviceToHost, g->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
        if (e != hipSuccess) break;
        TopkKey *tmp = cur;
        cur = nxt;
        nxt = tmp;
        if (st.done) break;
    }
    if (e == hipSuccess) {
        TopkState fix = st;
        fix.overflow = 0;
        e = hipMemcpyAsync(D.tstate, &fix, sizeof(fix), hipMemcpyHostToDevice, g->stream);
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_pair_rank, dim3(grid_k), dim3(kBlock), 0, g->stream, D.tfinal, n_fin, D.tstate, 1,
                           D.tfinal, D.R, D.new2old, D.tout_ids, D.tout_sc);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    (void)hipFree(cnt_dev);
    if (e != hipSuccess) return hip_fail(e, "top-k refine");
    return RS_OK;
}

// ------------------------------------------------------------ removals
// A removed CSR entry is marked by complementing it (~x < 0), which keeps
// every row ordered on the decoded value until the compaction below.
__device__ __forceinline__ int decode(int x) { return x < 0 ? ~x : x; }

template <typename OffT>
__device__ __forceinline__ long long find_entry(const OffT *off, const int32_t *deg, const int32_t *col, int u, int v) {
    long long lo = (long long)off[u], hi = lo + deg[u];
    while (lo < hi) {
        const long long mid = (lo + hi) >> 1;
        const int x = decode(col[mid]);
        if (x < v)
            lo = mid + 1;
        else if (x > v)
            hi = mid;
        else
            return mid;
    }
    return -1;
}

// Delete the undirected edge {a, b}; the entry in the row of min(a, b) is
// the owner and decides which request wins.  Returns 1 if deleted here.
template <typename OffT>
__device__ __forceinline__ int delete_edge(const OffT *off, const int32_t *deg, int32_t *col, int a, int b) {
    const int x = min(a, b), y = max(a, b);
    const long long e = find_entry(off, deg, col, x, y);
    if (e < 0) return 0;
    if (atomicCAS(&col[e], y, ~y) != y) return 0;
    const long long f = find_entry(off, deg, col, y, x);
    if (f >= 0) col[f] = ~x;
    return 1;
}

template <typename OffT>
__global__ void k_remove_edges(const OffT *off, const int32_t *deg, int32_t *col, const int32_t *src,
                               const int32_t *dst, long long m, unsigned long long *removed) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (long long)gridDim.x * blockDim.x) {
        const int a = src[i], b = dst[i];
        if (a != b && delete_edge(off, deg, col, a, b)) atomicAdd(removed, 1ull);
    }
}

// One wavefront per removed vertex: delete every incident edge, then mark the
// vertex dead.  removed[0] counts edges, removed[1] newly dead vertices.
template <typename OffT>
__global__ void k_remove_vertices(const OffT *off, const int32_t *deg, int32_t *col, uint8_t *alive,
                                  const int32_t *verts, long long nv, unsigned long long *removed) {
    const long long wave = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const long long nwave = ((long long)gridDim.x * blockDim.x) >> 6;
    for (long long i = wave; i < nv; i += nwave) {
        const int x = verts[i];
        const long long rb = (long long)off[x];
        const int d = deg[x];
        unsigned long long cnt = 0;
        for (int j = (int)__lane_id(); j < d; j += 64) {
            const int y = col[rb + j];
            if (y >= 0) cnt += (unsigned long long)delete_edge(off, deg, col, x, y);
        }
        for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o);
        if (__lane_id() == 0) {
            if (cnt) atomicAdd(&removed[0], cnt);
            if (alive[x]) {
                alive[x] = 0;
                atomicAdd(&removed[1], 1ull);
            }
        }
    }
}

// Squeeze the marked entries out of every row (order kept), updating deg.
template <typename OffT>
__global__ void k_compact(const OffT *off, int32_t *deg, int32_t *col, long long n) {
    for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (long long)gridDim.x * blockDim.x) {
        const long long rb = (long long)off[v];
        const int d = deg[v];
        int w = 0;
        for (int j = 0; j < d; ++j) {
            const int x = col[rb + j];
            if (x >= 0) col[rb + (w++)] = x;
        }
        deg[v] = w;
    }
}

rs_status launch_remove_edges(rs_graph *g, const int32_t *d_src, const int32_t *d_dst, int64_t m,
                              unsigned long long *d_removed) {
    if (m <= 0) return RS_OK;
    const int grid = grid_for(m, 256, 4096);
    if (g->d.off64)
        hipLaunchKernelGGL(k_remove_edges<long long>, dim3(grid), dim3(256), 0, g->stream,
                           (const long long *)g->d.off, g->d.deg, g->d.col, d_src, d_dst, (long long)m, d_removed);
    else
        hipLaunchKernelGGL(k_remove_edges<int32_t>, dim3(grid), dim3(256), 0, g->stream,
                           (const int32_t *)g->d.off, g->d.deg, g->d.col, d_src, d_dst, (long long)m, d_removed);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? RS_OK : hip_fail(e, "remove edges launch");
}

rs_status launch_remove_vertices(rs_graph *g, const int32_t *d_verts, int64_t nv, unsigned long long *d_removed) {
    if (nv <= 0) return RS_OK;
    const int grid = grid_for(nv, 4, 4096);
    if (g->d.off64)
        hipLaunchKernelGGL(k_remove_vertices<long long>, dim3(grid), dim3(256), 0, g->stream,
                           (const long long *)g->d.off, g->d.deg, g->d.col, g->d.alive, d_verts, (long long)nv,
                           d_removed);
    else
        hipLaunchKernelGGL(k_remove_vertices<int32_t>, dim3(grid), dim3(256), 0, g->stream,
                           (const int32_t *)g->d.off, g->d.deg, g->d.col, g->d.alive, d_verts, (long long)nv,
                           d_removed);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? RS_OK : hip_fail(e, "remove vertices launch");
}

rs_status launch_compact_rows(rs_graph *g) {
    const int grid = grid_for(g->d.n, 256, 8192);
    if (g->d.off64)
        hipLaunchKernelGGL(k_compact<long long>, dim3(grid), dim3(256), 0, g->stream, (const long long *)g->d.off,
                           g->d.deg, g->d.col, (long long)g->d.n);
    else
        hipLaunchKernelGGL(k_compact<int32_t>, dim3(grid), dim3(256), 0, g->stream, (const int32_t *)g->d.off,
                           g->d.deg, g->d.col, (long long)g->d.n);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? RS_OK : hip_fail(e, "compact launch");
}

// ------------------------------------------------------------ readers
__global__ void k_gather_scores(const double *R, const int32_t *new2old, const DevCounters *ctr, long long n, int raw,
                                double *out) {
    const double wmax = __longlong_as_double((long long)ctr->wmax_bits);
    for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (long long)gridDim.x * blockDim.x)
        out[new2old[v]] = raw ? R[v] * wmax : R[v];
}

rs_status launch_gather_scores(rs_graph *g, double *d_out, int raw) {
    const int grid = grid_for(g->d.n, 256, 8192);
    hipLaunchKernelGGL(k_gather_scores, dim3(grid), dim3(256), 0, g->stream, g->d.R, g->d.new2old, g->d.ctr,
                       (long long)g->d.n, raw, d_out);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? RS_OK : hip_fail(e, "gather launch");
}

}  // namespace rs
