// rs_kernels.hip -- HIP kernels of the robust-spanner scoring pass (gfx950, wave64).
//
// One pass (rs_score):
//   k_rows_hub, k_rows
//            Algorithm 1 Steps 1-2 fused, per vertex: gather the labels of the
//            neighbours, run-length count them into interaction-matrix records
//            (rows are community-sorted, so every community is one run),
//            detect the border vertex, compute every record's weight with
//            Algorithm 2's shared terms (Eq. H_optimal) and the vertex's
//            own-community weight, and a per-block maximum for w_max.
//   k_wmax   reduce the per-block partials (w_max and pass totals).
//   k_score_small, k_score_big
//            Eq. RSI per border vertex u in the per-(vertex, community)
//            factorised form of Lemmas 1-2: the type-II triads through a
//            foreign neighbour w contribute w_w(C(u))^(2/3) a_v for every other
//            neighbour v of w in C(u) (a_v = cbrt(w_v(C(v)))), and the type-I
//            triads are the common foreign neighbours of u and w, found by
//            sorted-list search (Section IV, Step 3).  One owner per vertex,
//            fixed summation order, no floating-point atomics.
// Top-k (Algorithm 1 Step 4) is an exact radix select on the 96-bit key
// (score bits, complement of the caller id) with 16-bit digits.
//
// No kernel of a pass uses a same-address global atomic: per-block results go
// to partial arrays.  Vertex work is walked by persistent grids over static
// degree bins, each bin split into 8 contiguous ranges, one per XCD.
#include <climits>

#include "rs_internal.h"

namespace rs {

// ------------------------------------------------------------ helpers
template <int T>
struct Team {
    int lane;  // lane within the team
    int base;  // first wavefront lane of the team
    __device__ __forceinline__ Team() {
        const int l = (int)__lane_id();
        lane = l & (T - 1);
        base = l & ~(T - 1);
    }
    __device__ __forceinline__ unsigned long long ballot(bool p) const {
        const unsigned long long m = __ballot(p);
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
    __device__ __forceinline__ int isum(int x) const {
#pragma unroll
        for (int o = T / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, T);
        return x;
    }
    __device__ __forceinline__ double dmax(double x) const {
#pragma unroll
        for (int o = T / 2; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o, T));
        return x;
    }
    __device__ __forceinline__ int imax(int x) const {
#pragma unroll
        for (int o = T / 2; o > 0; o >>= 1) x = max(x, __shfl_xor(x, o, T));
        return x;
    }
    // exclusive prefix sum over the team's lanes
    __device__ __forceinline__ int excl_scan(int x) const {
        int incl = x;
#pragma unroll
        for (int o = 1; o < T; o <<= 1) {
            const int y = __shfl_up(incl, o, T);
            if (lane >= o) incl += y;
        }
        return incl - x;
    }
};

__device__ __forceinline__ unsigned long long dbits(double x) { return (unsigned long long)__double_as_longlong(x); }
__device__ __forceinline__ double bitsd(unsigned long long b) { return __longlong_as_double((long long)b); }

// Item range of this block for a bin of `cnt` items, `per` items per block
// step: the bin is split into 8 contiguous ranges (one per XCD; blocks are
// dealt to the XCDs round-robin, so block b runs on XCD b % 8) and the blocks
// of an XCD stride through its range.  gridDim.x is a multiple of 8.
struct Span {
    long long first, hi, step;
};
__device__ __forceinline__ Span xcd_span(long long cnt, int per) {
    const int x = (int)(blockIdx.x & 7u), j = (int)(blockIdx.x >> 3), nx = (int)(gridDim.x >> 3);
    Span s;
    const long long lo = cnt * x / 8;
    s.hi = cnt * (x + 1) / 8;
    s.first = lo + (long long)j * per;
    s.step = (long long)nx * per;
    return s;
}

// ------------------------------------------------------------ weights
// Eq. H_optimal with Algorithm 2's shared terms: for a vertex of degree d
// whose neighbour-community counts have X = sum f log2 f over ell distinct
// communities, the weight toward a community with count f > 0 is
//   H = -(X - d log2(d - f) - f log2(f / (d - f))) / (d - f),  w = H (ell - 1),
// and toward a community absent from the neighbourhood (f = 0; only the own
// community can be) H = log2 d - X / d with |L| = ell (Eq. weight).
// |L| <= 1 leaves a single community: H = 0 exactly.
__device__ __forceinline__ double flogf(int f);
__device__ __forceinline__ double weight_present(int d, double X, int ell, int f) {
    const int L = ell - 1;
    if (L < 2) return 0.0;
    const double Y = (double)(d - f);
    return (log2(Y) + (flogf(f) - X) / Y) * (double)L;  // = -(X - d log2 Y - f log2(f/Y)) / Y
}

__device__ __forceinline__ double weight_absent(int d, double X, int ell) {
    if (ell < 2) return 0.0;
    const double Y = (double)d;
    return (log2(Y) - X / Y) * (double)ell;
}

__device__ __forceinline__ double flogf(int f) { return f > 1 ? (double)f * log2((double)f) : 0.0; }

constexpr int kNone = 1 << 30;  // no run start in the rest of a chunk

// ============================================================ row kernels
template <typename OffT>
struct RowArgs {
    const OffT *off;
    const int32_t *deg, *col, *lab, *sched;
    Rec *rec;
    VMeta *meta;
    double *wown, *a, *R;
    long long *tI, *tII;
    RowPart *part;
    long long bin_lo[kBins + 1];
};

struct RowResult {
    int ell, p, q;
    double wown, lmax;
};

struct RowAcc {
    double wmax;
    unsigned long long nb, dp, ell, ellx;
};

template <typename OffT>
__device__ __forceinline__ void finish_row(const RowArgs<OffT> &A, int v, int d, const RowResult &r, RowAcc &acc) {
    const int fown = r.q - r.p;
    const int dprime = d - fown;
    VMeta m;
    m.deg = d;
    m.ell = r.ell;
    m.p = r.p;
    m.q = r.q;
    A.meta[v] = m;
    A.wown[v] = r.wown;
    A.a[v] = cbrt(r.wown);
    acc.wmax = fmax(acc.wmax, r.lmax);
    acc.ell += (unsigned long long)r.ell;
    acc.ellx += (unsigned long long)(r.ell - (fown > 0 ? 1 : 0));
    if (dprime > 0) {
        acc.nb += 1;
        acc.dp += (unsigned long long)dprime;
    } else {
        A.R[v] = 0.0;
        A.tI[v] = 0;
        A.tII[v] = 0;
    }
}

__device__ void block_reduce_row(RowAcc acc, RowPart *out) {
    __shared__ unsigned long long s_u[5][kBlock / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        acc.wmax = fmax(acc.wmax, __shfl_xor(acc.wmax, o));
        acc.nb += __shfl_xor(acc.nb, o);
        acc.dp += __shfl_xor(acc.dp, o);
        acc.ell += __shfl_xor(acc.ell, o);
        acc.ellx += __shfl_xor(acc.ellx, o);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s_u[0][w] = dbits(acc.wmax);
        s_u[1][w] = acc.nb;
        s_u[2][w] = acc.dp;
        s_u[3][w] = acc.ell;
        s_u[4][w] = acc.ellx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        RowPart p = {};
        for (int i = 0; i < kBlock / 64; ++i) {
            p.wmax_bits = max(p.wmax_bits, s_u[0][i]);
            p.n_border += s_u[1][i];
            p.sum_dprime += s_u[2][i];
            p.sum_ell += s_u[3][i];
            p.sum_ell_x += s_u[4][i];
        }
        *out = p;
    }
}

// Small-value tables for the thread path (d <= kTab): log2 y, y log2 y, 1/y.
constexpr int kTab = 64;
struct Tables {
    double lg[kTab + 1], fl[kTab + 1], rc[kTab + 1];
};
__device__ __forceinline__ void fill_tables(Tables &t) {
    for (int i = threadIdx.x; i <= kTab; i += blockDim.x) {
        const double x = (double)i;
        t.lg[i] = i > 0 ? log2(x) : 0.0;
        t.fl[i] = flogf(i);
        t.rc[i] = i > 0 ? 1.0 / x : 0.0;
    }
    __syncthreads();
}

// Eq. H_optimal rearranged: with Y = d - f,
//   H = -(X - d log2 Y - f log2(f/Y)) / Y = log2 Y - (X - f log2 f) / Y.
__device__ __forceinline__ double weight_present_t(const Tables &t, int d, double X, int ell, int f) {
    const int L = ell - 1;
    if (L < 2) return 0.0;
    const int Y = d - f;
    return (t.lg[Y] + (t.fl[f] - X) * t.rc[Y]) * (double)L;
}
__device__ __forceinline__ double weight_absent_t(const Tables &t, int d, double X, int ell) {
    if (ell < 2) return 0.0;
    return (t.lg[d] - X * t.rc[d]) * (double)ell;
}

template <int PASS, typename OffT>
__device__ __forceinline__ void row_close_t(const RowArgs<OffT> &A, const Tables &tb, OffT rb, int d, int cv,
                                            double X, int ell, int label, int start, int slot, int f, double &xs,
                                            int &fown, int &pown, double &lmax) {
    if (PASS == 1) {
        xs += tb.fl[f];
        if (label == cv) {
            fown = f;
            pown = start;
        }
    } else {
        Rec rc;
        rc.key = label;
        rc.pos = start;
        rc.w = weight_present_t(tb, d, X, ell, f);
        A.rec[rb + slot] = rc;
        lmax = fmax(lmax, rc.w);
    }
}

// Bins A and B (d <= 64): one thread per vertex, the row read 16 entries at
// a time into registers.  Pass 1 counts the runs and X = sum f log2 f, pass
// 2 re-reads the row (cache-hot) and writes the weighted records.
template <int PASS, typename OffT>
__device__ __forceinline__ void row_thread_pass(const RowArgs<OffT> &A, const Tables &tb, OffT rb, int d, int cv,
                                                double X, int ell, double &xs, int &fown, int &pown, int &below,
                                                int &nruns, double &lmax) {
    int cur = -1, s = 0, slot = 0;
    for (int base = 0; base < d; base += 16) {
        int c[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) c[i] = base + i < d ? A.col[rb + base + i] : 0;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            c[i] = base + i < d ? A.lab[c[i]] : INT_MAX;
            if (PASS == 1 && base + i < d && c[i] < cv) ++below;
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int pos = base + i;
            if (pos < d) {
                if (pos > 0 && c[i] != cur) {
                    row_close_t<PASS>(A, tb, rb, d, cv, X, ell, cur, s, slot, pos - s, xs, fown, pown, lmax);
                    ++slot;
                    s = pos;
                }
                cur = c[i];
            }
        }
    }
    if (d > 0) {
        row_close_t<PASS>(A, tb, rb, d, cv, X, ell, cur, s, slot, d - s, xs, fown, pown, lmax);
        ++slot;
    }
    nruns = slot;
}

template <typename OffT>
__device__ __forceinline__ RowResult row_thread(const RowArgs<OffT> &A, const Tables &tb, OffT rb, int d, int cv) {
    double xs = 0.0, lmax = 0.0;
    int fown = 0, pown = 0, below = 0, nr = 0;
    row_thread_pass<1, OffT>(A, tb, rb, d, cv, 0.0, 0, xs, fown, pown, below, nr, lmax);
    const double X = xs;
    const int ell = nr;
    row_thread_pass<2, OffT>(A, tb, rb, d, cv, X, ell, xs, fown, pown, below, nr, lmax);
    RowResult r;
    r.ell = ell;
    r.p = fown > 0 ? pown : below;
    r.q = r.p + fown;
    r.wown = fown > 0 ? weight_present_t(tb, d, X, ell, fown) : weight_absent_t(tb, d, X, ell);
    r.lmax = fmax(lmax, r.wown);
    return r;
}

template <int PASS, typename OffT>
__device__ __forceinline__ void row_close_d(const RowArgs<OffT> &A, OffT rb, int d, int cv, double X, int ell,
                                            int label, int start, int slot, int f, double &xs, int &fown, int &pown,
                                            double &lmax) {
    if (PASS == 1) {
        xs += flogf(f);
        if (label == cv) {
            fown = f;
            pown = start;
        }
    } else {
        Rec rc;
        rc.key = label;
        rc.pos = start;
        rc.w = weight_present(d, X, ell, f);
        A.rec[rb + slot] = rc;
        lmax = fmax(lmax, rc.w);
    }
}

// Bin C: T lanes per vertex, the row streamed in chunks of T*U entries
// (entry base + k*T + lane in register c[k]); run starts are team ballots and
// the run still open at a chunk's end is carried into the next chunk.
template <int T, int U, int PASS, typename OffT>
__device__ __forceinline__ void row_team_pass(const RowArgs<OffT> &A, const Team<T> &tm, OffT rb, int d, int cv,
                                              double X, int ell, double &xs, int &fown, int &pown, int &below,
                                              int &nruns, double &lmax) {
    constexpr int CH = T * U;
    int open_label = -1, open_start = 0, open_slot = 0;
    int nr = 0;
    const unsigned long long lt = (1ull << tm.lane) - 1ull;
    for (int base = 0; base < d; base += CH) {
        int c[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int i = base + k * T + tm.lane;
            c[k] = i < d ? A.col[rb + i] : 0;
        }
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int i = base + k * T + tm.lane;
            c[k] = i < d ? A.lab[c[k]] : INT_MAX;
            if (PASS == 1 && i < d && c[k] < cv) ++below;
        }
        unsigned long long m[U];
        int bef[U];
        int cnt = 0;
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int i = base + k * T + tm.lane;
            const int last_prev = (k == 0) ? open_label : tm.bcast(c[k - 1], T - 1);
            int pc = tm.up1(c[k]);
            if (tm.lane == 0) pc = last_prev;
            m[k] = tm.ballot(i < d && c[k] != pc);
            bef[k] = cnt;
            cnt += __popcll(m[k]);
        }
        const bool last_chunk = base + CH >= d;
        int first[U + 1];
        first[U] = last_chunk ? d - base : kNone;
#pragma unroll
        for (int k = U - 1; k >= 0; --k) first[k] = m[k] ? k * T + __builtin_ctzll(m[k]) : first[k + 1];
        if (open_label >= 0 && first[0] != kNone) {
            if (tm.lane == 0)
                row_close_d<PASS>(A, rb, d, cv, X, ell, open_label, open_start, open_slot,
                                  base + first[0] - open_start, xs, fown, pown, lmax);
            open_label = -1;
        }
        int nl = -1, ns = 0, nsl = 0;
#pragma unroll
        for (int k = 0; k < U; ++k) {
            if ((m[k] >> tm.lane) & 1ull) {
                const unsigned long long rest = (tm.lane + 1 < T) ? (m[k] >> (tm.lane + 1)) : 0ull;
                const int nxt = rest ? k * T + tm.lane + 1 + __builtin_ctzll(rest) : first[k + 1];
                const int slot = nr + bef[k] + __popcll(m[k] & lt);
                if (nxt != kNone) {
                    row_close_d<PASS>(A, rb, d, cv, X, ell, c[k], base + k * T + tm.lane, slot,
                                      nxt - (k * T + tm.lane), xs, fown, pown, lmax);
                } else {
                    nl = c[k];
                    ns = base + k * T + tm.lane;
                    nsl = slot;
                }
            }
        }
        const unsigned long long owner = tm.ballot(nl >= 0);
        if (owner) {
            const int ol = __builtin_ctzll(owner);
            open_label = tm.bcast(nl, ol);
            open_start = tm.bcast(ns, ol);
            open_slot = tm.bcast(nsl, ol);
        }
        nr += cnt;
    }
    nruns = nr;
}

template <int T, int U, typename OffT>
__device__ __forceinline__ RowResult row_team(const RowArgs<OffT> &A, const Team<T> &tm, OffT rb, int d, int cv) {
    double xs = 0.0, lmax = 0.0;
    int fown = 0, pown = -1, below = 0, nr = 0;
    row_team_pass<T, U, 1, OffT>(A, tm, rb, d, cv, 0.0, 0, xs, fown, pown, below, nr, lmax);
    const double X = tm.sum(xs);
    fown = tm.imax(fown);
    pown = tm.imax(pown);
    below = tm.isum(below);
    const int ell = nr;
    row_team_pass<T, U, 2, OffT>(A, tm, rb, d, cv, X, ell, xs, fown, pown, below, nr, lmax);
    RowResult r;
    r.ell = ell;
    r.p = fown > 0 ? pown : below;
    r.q = r.p + fown;
    r.wown = fown > 0 ? weight_present(d, X, ell, fown) : weight_absent(d, X, ell);
    r.lmax = fmax(tm.dmax(lmax), r.wown);
    return r;
}

template <int T, int U, typename OffT>
__device__ __forceinline__ void rows_team_bin(const RowArgs<OffT> &A, int bin, RowAcc &acc) {
    const Team<T> tm;
    constexpr int per = kBlock / T;
    const Span s = xcd_span(A.bin_lo[bin + 1] - A.bin_lo[bin], per);
    for (long long base = s.first; base < s.hi; base += s.step) {
        const long long it = base + threadIdx.x / T;
        if (it < s.hi) {
            const int v = A.sched[A.bin_lo[bin] + it];
            const int d = A.deg[v];
            const RowResult r = row_team<T, U, OffT>(A, tm, A.off[v], d, A.lab[v]);
            if (tm.lane == 0) finish_row(A, v, d, r, acc);
        }
    }
}

// Bin C: 16 lanes per vertex.
template <typename OffT>
__global__ __launch_bounds__(kBlock) void k_rows_mid(RowArgs<OffT> A) {
    RowAcc acc = {0.0, 0, 0, 0, 0};
    rows_team_bin<16, 8, OffT>(A, 2, acc);
    block_reduce_row(acc, &A.part[blockIdx.x]);
}

// Bins A and B: one thread per vertex.
template <typename OffT>
__global__ __launch_bounds__(kBlock) void k_rows(RowArgs<OffT> A) {
    __shared__ Tables tb;
    fill_tables(tb);
    RowAcc acc = {0.0, 0, 0, 0, 0};
    {
        // bins A and B are adjacent in sched: one thread per vertex
        const Span s = xcd_span(A.bin_lo[2] - A.bin_lo[0], kBlock);
        for (long long base = s.first; base < s.hi; base += s.step) {
            const long long it = base + threadIdx.x;
            if (it < s.hi) {
                const int v = A.sched[A.bin_lo[0] + it];
                const int d = A.deg[v];
                const RowResult r = row_thread<OffT>(A, tb, A.off[v], d, A.lab[v]);
                finish_row(A, v, d, r, acc);
            }
        }
    }
    block_reduce_row(acc, &A.part[blockIdx.x]);
}

// ------------------------------------------------------------ hub rows
// Bin D: one block per vertex; the row is streamed in groups of kHubG
// entries (entry g0 + k*256 + tid in register c[k]) twice: the first pass
// counts the runs and X, the second writes the weighted records.  A run that
// crosses a group boundary stays open in the block's shared state.
constexpr int kHubU = 8;
constexpr int kHubG = kBlock * kHubU;
constexpr int kHubW = kBlock / 64;            // wavefronts per block
constexpr int kHubM = kHubU * kHubW;          // ballot masks per group

struct HubState {
    int prev;                                  // label of the previous group's last entry
    int open_start, open_label, open_slot;     // run open at the group boundary (open_start < 0: none)
    int nruns;                                 // runs started before the current group
    int fown, pown;                            // the own community's run (pass 1)
    int next_prev;
};

struct HubShared {
    int lab[kHubG];
    unsigned long long mask[kHubM];
    int pre[kHubM + 1];
    int first[kHubM + 1];
    HubState st;
    double red[kHubW];
    int ired[kHubW];
};

template <int PASS, typename OffT>
__device__ __forceinline__ void hub_close(const RowArgs<OffT> &A, HubShared &S, OffT rb, int d, int cv, double X,
                                          int ell, int start, int label, int slot, int f, double &xpart, double &lmax) {
    if (PASS == 1) {
        xpart += flogf(f);
        if (label == cv) {
            S.st.fown = f;
            S.st.pown = start;
        }
    } else {
        Rec rc;
        rc.key = label;
        rc.pos = start;
        rc.w = weight_present(d, X, ell, f);
        A.rec[rb + slot] = rc;
        lmax = fmax(lmax, rc.w);
    }
}

template <int PASS, typename OffT>
__device__ void hub_stream(const RowArgs<OffT> &A, HubShared &S, OffT rb, int d, int cv, double X, int ell,
                           double &xpart, int &below, double &lmax) {
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    if (tid == 0) {
        S.st.prev = -1;
        S.st.open_start = -1;
        S.st.nruns = 0;
    }
    for (int g0 = 0; g0 < d; g0 += kHubG) {
        int c[kHubU];
#pragma unroll
        for (int k = 0; k < kHubU; ++k) {
            const int i = g0 + k * kBlock + tid;
            c[k] = i < d ? A.col[rb + i] : 0;
        }
#pragma unroll
        for (int k = 0; k < kHubU; ++k) {
            const int i = g0 + k * kBlock + tid;
            c[k] = i < d ? A.lab[c[k]] : INT_MAX;
            if (PASS == 1 && i < d && c[k] < cv) ++below;
        }
        __syncthreads();  // previous group done with S.lab; S.st updated
#pragma unroll
        for (int k = 0; k < kHubU; ++k) S.lab[k * kBlock + tid] = c[k];
        __syncthreads();
        const int prev = S.st.prev;
        bool st[kHubU];
#pragma unroll
        for (int k = 0; k < kHubU; ++k) {
            const int li = k * kBlock + tid;
            const int pc = li > 0 ? S.lab[li - 1] : prev;
            st[k] = (g0 + li < d) && c[k] != pc;
            const unsigned long long mk = __ballot(st[k]);
            if (lane == 0) S.mask[k * kHubW + wave] = mk;
        }
        __syncthreads();
        if (tid == 0) {
            int acc = 0;
            for (int mi = 0; mi < kHubM; ++mi) {
                S.pre[mi] = acc;
                acc += __popcll(S.mask[mi]);
            }
            S.pre[kHubM] = acc;
            int nxt = kNone;
            S.first[kHubM] = kNone;
            for (int mi = kHubM - 1; mi >= 0; --mi) {
                if (S.mask[mi]) nxt = (mi / kHubW) * kBlock + (mi % kHubW) * 64 + __builtin_ctzll(S.mask[mi]);
                S.first[mi] = nxt;
            }
            if (S.st.open_start >= 0 && S.first[0] != kNone) {
                hub_close<PASS>(A, S, rb, d, cv, X, ell, S.st.open_start, S.st.open_label, S.st.open_slot,
                                g0 + S.first[0] - S.st.open_start, xpart, lmax);
                S.st.open_start = -1;
            }
            S.st.next_prev = S.lab[kHubG - 1];
        }
        __syncthreads();
        const int nr0 = S.st.nruns;
        const bool last_group = g0 + kHubG >= d;
#pragma unroll
        for (int k = 0; k < kHubU; ++k) {
            if (st[k]) {
                const int li = k * kBlock + tid;
                const int mi = k * kHubW + wave;
                const unsigned long long mk = S.mask[mi];
                const unsigned long long rest = lane + 1 < 64 ? (mk >> (lane + 1)) : 0ull;
                const int nxt = rest ? li + 1 + __builtin_ctzll(rest) : S.first[mi + 1];
                const int slot = nr0 + S.pre[mi] + __popcll(mk & ((1ull << lane) - 1ull));
                if (nxt != kNone)
                    hub_close<PASS>(A, S, rb, d, cv, X, ell, g0 + li, c[k], slot, nxt - li, xpart, lmax);
                else if (last_group)
                    hub_close<PASS>(A, S, rb, d, cv, X, ell, g0 + li, c[k], slot, d - (g0 + li), xpart, lmax);
                else {
                    S.st.open_start = g0 + li;
                    S.st.open_label = c[k];
                    S.st.open_slot = slot;
                }
            }
        }
        __syncthreads();
        if (tid == 0) {
            S.st.nruns = nr0 + S.pre[kHubM];
            S.st.prev = S.st.next_prev;
        }
    }
    __syncthreads();
    if (tid == 0 && S.st.open_start >= 0) {
        hub_close<PASS>(A, S, rb, d, cv, X, ell, S.st.open_start, S.st.open_label, S.st.open_slot,
                        d - S.st.open_start, xpart, lmax);
        S.st.open_start = -1;
    }
    __syncthreads();
}

__device__ __forceinline__ double block_sum_d(double x, double *red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < kHubW; ++i) t += red[i];
    __syncthreads();
    return t;
}

__device__ __forceinline__ double block_max_d(double x, double *red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < kHubW; ++i) t = fmax(t, red[i]);
    __syncthreads();
    return t;
}

__device__ __forceinline__ int block_sum_i(int x, int *red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
    __syncthreads();
    int t = 0;
    for (int i = 0; i < kHubW; ++i) t += red[i];
    __syncthreads();
    return t;
}

template <typename OffT>
__global__ __launch_bounds__(kBlock) void k_rows_hub(RowArgs<OffT> A) {
    __shared__ HubShared S;
    RowAcc acc = {0.0, 0, 0, 0, 0};
    const long long cnt = A.bin_lo[4] - A.bin_lo[3];
    for (long long h = blockIdx.x; h < cnt; h += gridDim.x) {
        const int v = A.sched[A.bin_lo[3] + h];
        const OffT rb = A.off[v];
        const int d = A.deg[v];
        const int cv = A.lab[v];
        if (threadIdx.x == 0) {
            S.st.fown = 0;
            S.st.pown = -1;
        }
        double xpart = 0.0, lmax = 0.0;
        int below = 0;
        hub_stream<1, OffT>(A, S, rb, d, cv, 0.0, 0, xpart, below, lmax);
        const double X = block_sum_d(xpart, S.red);
        const int nbelow = block_sum_i(below, S.ired);
        const int ell = S.st.nruns;
        const int fown = S.st.fown;
        const int p = fown > 0 ? S.st.pown : nbelow;
        __syncthreads();  // everyone has read pass 1's totals before pass 2 resets them
        hub_stream<2, OffT>(A, S, rb, d, cv, X, ell, xpart, below, lmax);
        const double lm = block_max_d(lmax, S.red);
        if (threadIdx.x == 0) {
            RowResult r;
            r.ell = ell;
            r.p = p;
            r.q = p + fown;
            r.wown = fown > 0 ? weight_present(d, X, ell, fown) : weight_absent(d, X, ell);
            r.lmax = fmax(lm, r.wown);
            finish_row(A, v, d, r, acc);
        }
        __syncthreads();
    }
    block_reduce_row(acc, &A.part[blockIdx.x]);
}

// Reduce the row partials of a pass into the counters (one block).
__global__ __launch_bounds__(1024) void k_wmax(const RowPart *part, int np, DevCounters *c) {
    __shared__ unsigned long long s[5][16];
    unsigned long long w = 0, nb = 0, dp = 0, ell = 0, ellx = 0;
    for (int i = threadIdx.x; i < np; i += blockDim.x) {
        const RowPart p = part[i];
        w = max(w, p.wmax_bits);
        nb += p.n_border;
        dp += p.sum_dprime;
        ell += p.sum_ell;
        ellx += p.sum_ell_x;
    }
    for (int o = 32; o > 0; o >>= 1) {
        w = max(w, (unsigned long long)__shfl_xor(w, o));
        nb += __shfl_xor(nb, o);
        dp += __shfl_xor(dp, o);
        ell += __shfl_xor(ell, o);
        ellx += __shfl_xor(ellx, o);
    }
    if ((threadIdx.x & 63) == 0) {
        s[0][threadIdx.x >> 6] = w;
        s[1][threadIdx.x >> 6] = nb;
        s[2][threadIdx.x >> 6] = dp;
        s[3][threadIdx.x >> 6] = ell;
        s[4][threadIdx.x >> 6] = ellx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        DevCounters r = {};
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
            r.wmax_bits = max(r.wmax_bits, s[0][i]);
            r.n_border += s[1][i];
            r.sum_dprime += s[2][i];
            r.sum_ell += s[3][i];
            r.sum_ell_x += s[4][i];
        }
        *c = r;
    }
}

// ============================================================ score kernels
template <typename OffT>
struct ScoreArgs {
    const OffT *off;
    const int32_t *col, *lab, *sched;
    const Rec *rec;
    const VMeta *meta;
    const double *a;
    double *R;
    long long *tI, *tII;
    const DevCounters *ctr;
    ScorePart *part;
    long long bin_lo[kBins + 1];
};

// Index of community c among the records of a vertex (c is present).
__device__ __forceinline__ int find_rec(const Rec *rec, long long rb, int ell, int c) {
    int lo = 0, hi = ell - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (rec[rb + mid].key < c)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// The foreign neighbours of x: its row minus the own-community sub-range
// [p, q), ascending.
struct Flist {
    long long rb;
    int p, h, n;
};
__device__ __forceinline__ Flist make_flist(long long rb, const VMeta &m) {
    Flist f;
    f.rb = rb;
    f.p = m.p;
    f.h = m.q - m.p;
    f.n = m.deg - f.h;
    return f;
}
__device__ __forceinline__ int fat(const int32_t *col, const Flist &f, int j) {
    return col[f.rb + (j < f.p ? j : j + f.h)];
}
__device__ __forceinline__ bool fcontains(const int32_t *col, const Flist &f, int y) {
    int lo = 0, hi = f.n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (fat(col, f, mid) < y)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo < f.n && fat(col, f, lo) == y;
}

// Foreign neighbour w of u: its weight toward C(u), and the type-II triads
// through w: the other neighbours v of w in C(u) (count F, sum of a_v).
struct WInfo {
    double W, S;
    int F;
};
template <typename OffT>
__device__ __forceinline__ WInfo w_info(const ScoreArgs<OffT> &A, int u, int cu, long long rbw, const VMeta &mw) {
    const int s = find_rec(A.rec, rbw, mw.ell, cu);
    const Rec r = A.rec[rbw + s];
    const int e = (s + 1 < mw.ell) ? A.rec[rbw + s + 1].pos : mw.deg;
    WInfo o;
    o.W = r.w;
    o.F = e - r.pos - 1;
    double S = 0.0;
#pragma unroll 4
    for (int i = r.pos; i < e; ++i) {
        const int x = A.col[rbw + i];
        if (x != u) S += A.a[x];
    }
    o.S = S;
    return o;
}

template <typename OffT>
__device__ __forceinline__ double weight_toward(const ScoreArgs<OffT> &A, int x, int c) {
    const long long rb = (long long)A.off[x];
    return A.rec[rb + find_rec(A.rec, rb, A.meta[x].ell, c)].w;
}

struct ScoreAcc {
    long long tI, tII, workI;
};

template <typename OffT>
__device__ __forceinline__ void score_store(const ScoreArgs<OffT> &A, int u, int d, double acc, long long cI,
                                            long long cII, double wmax, ScoreAcc &sa) {
    A.R[u] = (d >= 2 && wmax > 0.0) ? acc / wmax / (double)((long long)d * (d - 1)) : 0.0;
    A.tI[u] = cI;
    A.tII[u] = cII;
    sa.tI += cI;
    sa.tII += cII;
}

// Membership of y in a sorted LDS column of n entries (stride kBlock).
__device__ __forceinline__ bool lds_member(const int *colv, int n, int y) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (colv[mid * kBlock] < y)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo < n && colv[lo * kBlock] == y;
}

// Bin A: one thread per vertex (d <= 16).  N'(u) is kept (ascending) in an
// LDS column of this thread.  For every foreign neighbour w, the type-I
// partners are N'(u) & N'(w): the shorter list is walked, the longer probed.
template <typename OffT>
__device__ __forceinline__ void score_thread(const ScoreArgs<OffT> &A, int u, double wmax, int *colv,
                                             ScoreAcc &sa) {
    const VMeta mu = A.meta[u];
    const Flist fu = make_flist((long long)A.off[u], mu);
    if (fu.n == 0) return;
    const int cu = A.lab[u];
    double acc = 0.0;
    long long cII = 0, cI = 0, work = 0;
    for (int j0 = 0; j0 < fu.n; j0 += 4) {
        int w[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) w[t] = j0 + t < fu.n ? fat(A.col, fu, j0 + t) : -1;
        long long rbw[4];
        VMeta mw[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            rbw[t] = 0;
            mw[t].deg = mw[t].ell = mw[t].p = mw[t].q = 0;
            if (w[t] >= 0) {
                rbw[t] = (long long)A.off[w[t]];
                mw[t] = A.meta[w[t]];
            }
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            if (w[t] >= 0) {
                colv[(j0 + t) * kBlock] = w[t];
                const WInfo wi = w_info(A, u, cu, rbw[t], mw[t]);
                const double c1 = cbrt(wi.W);
                acc += c1 * c1 * wi.S;
                cII += wi.F;
            }
        }
    }
    for (int j = 0; j < fu.n; ++j) {
        const int w = colv[j * kBlock];
        const long long rbw = (long long)A.off[w];
        const VMeta mw = A.meta[w];
        const Flist fw = make_flist(rbw, mw);
        work += min(fu.n, fw.n);
        double Ww = -1.0;
        if (fw.n <= fu.n) {
            for (int t0 = 0; t0 < fw.n; t0 += 8) {
                int y[8];
#pragma unroll
                for (int t = 0; t < 8; ++t) y[t] = t0 + t < fw.n ? fat(A.col, fw, t0 + t) : -1;
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    if (y[t] >= 0 && lds_member(colv, fu.n, y[t])) {
                        if (Ww < 0.0) Ww = A.rec[rbw + find_rec(A.rec, rbw, mw.ell, cu)].w;
                        const double Wy = weight_toward(A, y[t], cu);
                        const double Wwy = A.rec[rbw + find_rec(A.rec, rbw, mw.ell, A.lab[y[t]])].w;
                        acc += cbrt(Ww * Wy * Wwy);
                        ++cI;
                    }
                }
            }
        } else {
            for (int k = 0; k < fu.n; ++k) {
                const int y = colv[k * kBlock];
                if (fcontains(A.col, fw, y)) {
                    if (Ww < 0.0) Ww = A.rec[rbw + find_rec(A.rec, rbw, mw.ell, cu)].w;
                    const double Wy = weight_toward(A, y, cu);
                    const double Wwy = A.rec[rbw + find_rec(A.rec, rbw, mw.ell, A.lab[y])].w;
                    acc += cbrt(Ww * Wy * Wwy);
                    ++cI;
                }
            }
        }
    }
    sa.workI += work;
    score_store(A, u, mu.deg, acc, cI, cII, wmax, sa);
}

// Bins B-D: T lanes per vertex.  N'(u) is staged in LDS when it fits (CAP).
// The foreign neighbours w are dealt to the lanes in chunks of T; each lane
// computes w's weight and type-II sum, then the chunk's type-I searches are
// flattened over the team: item t of w iterates the shorter of N'(u), N'(w)
// and probes the other.
template <int T, int CAP, typename OffT>
__device__ __forceinline__ void score_team(const ScoreArgs<OffT> &A, const Team<T> &tm, int u, const VMeta &mu,
                                           const Flist &fu, double wmax, const int *nl, ScoreAcc &sa) {
    const int cu = A.lab[u];
    const bool staged = fu.n <= CAP;
    double acc = 0.0;
    long long cI = 0, cII = 0, work = 0;
    for (int jb = 0; jb < fu.n; jb += T) {
        const int j = jb + tm.lane;
        const bool has = j < fu.n;
        Flist fw;
        fw.rb = 0;
        fw.p = fw.h = fw.n = 0;
        double W = 0.0;
        int wl = 0;
        if (has) {
            const int w = staged ? nl[j] : fat(A.col, fu, j);
            const long long rbw = (long long)A.off[w];
            const VMeta mw = A.meta[w];
            fw = make_flist(rbw, mw);
            const WInfo wi = w_info(A, u, cu, rbw, mw);
            W = wi.W;
            const double c1 = cbrt(W);
            acc += c1 * c1 * wi.S;
            cII += wi.F;
            wl = mw.ell;
        }
        // type-I: flattened over the chunk
        const int myw = has ? min(fu.n, fw.n) : 0;
        const int ex = tm.excl_scan(myw);
        const int total = tm.isum(myw);
        work += myw;
        for (int b = 0; b < total; b += T) {
            const int it = b + tm.lane;
            // owner: the largest lane whose exclusive prefix is <= it
            int lo = 0;
#pragma unroll
            for (int step = T / 2; step > 0; step >>= 1) {
                const int cand = lo + step;
                const int e = tm.bcast(ex, cand);
                if (e <= it) lo = cand;
            }
            const int o = lo;
            const int t = it - tm.bcast(ex, o);
            Flist fo;
            fo.rb = tm.bcast(fw.rb, o);
            fo.p = tm.bcast(fw.p, o);
            fo.h = tm.bcast(fw.h, o);
            fo.n = tm.bcast(fw.n, o);
            const double oW = tm.bcast(W, o);
            const int owl = tm.bcast(wl, o);
            if (it < total) {
                int y;
                bool found;
                if (fo.n <= fu.n) {
                    y = fat(A.col, fo, t);
                    if (staged) {
                        int l2 = 0, h2 = fu.n;
                        while (l2 < h2) {
                            const int mid = (l2 + h2) >> 1;
                            if (nl[mid] < y)
                                l2 = mid + 1;
                            else
                                h2 = mid;
                        }
                        found = l2 < fu.n && nl[l2] == y;
                    } else {
                        found = fcontains(A.col, fu, y);
                    }
                } else {
                    y = staged ? nl[t] : fat(A.col, fu, t);
                    found = fcontains(A.col, fo, y);
                }
                if (found) {
                    const double Wv = weight_toward(A, y, cu);
                    const double Wwv = A.rec[fo.rb + find_rec(A.rec, fo.rb, owl, A.lab[y])].w;
                    acc += cbrt(oW * Wv * Wwv);
                    ++cI;
                }
            }
        }
    }
    acc = tm.sum(acc);
    cI = tm.sum(cI);
    cII = tm.sum(cII);
    if (tm.lane == 0) score_store(A, u, mu.deg, acc, cI, cII, wmax, sa);
    sa.workI += work;
}

template <int T, int CAP, typename OffT>
__device__ __forceinline__ void score_team_bin(const ScoreArgs<OffT> &A, int bin, double wmax, int *lds,
                                               ScoreAcc &sa) {
    const Team<T> tm;
    const int teams = (int)blockDim.x / T;
    const Span s = xcd_span(A.bin_lo[bin + 1] - A.bin_lo[bin], teams);
    int *nl = lds + (threadIdx.x / T) * CAP;
    for (long long base = s.first; base < s.hi; base += s.step) {
        const long long it = base + threadIdx.x / T;
        const bool has = it < s.hi;
        int u = 0;
        VMeta mu;
        mu.deg = mu.ell = mu.p = mu.q = 0;
        Flist fu;
        fu.rb = 0;
        fu.p = fu.h = fu.n = 0;
        if (has) {
            u = A.sched[A.bin_lo[bin] + it];
            mu = A.meta[u];
            fu = make_flist((long long)A.off[u], mu);
            if (fu.n <= CAP)
                for (int j = tm.lane; j < fu.n; j += T) nl[j] = fat(A.col, fu, j);
        }
        __syncthreads();
        if (has && fu.n > 0) score_team<T, CAP, OffT>(A, tm, u, mu, fu, wmax, nl, sa);
        __syncthreads();
    }
}

__device__ void block_reduce_score(ScoreAcc sa, ScorePart *out) {
    __shared__ unsigned long long s_u[3][16];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        sa.tI += __shfl_xor(sa.tI, o);
        sa.tII += __shfl_xor(sa.tII, o);
        sa.workI += __shfl_xor(sa.workI, o);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s_u[0][w] = (unsigned long long)sa.tI;
        s_u[1][w] = (unsigned long long)sa.tII;
        s_u[2][w] = (unsigned long long)sa.workI;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        ScorePart p = {};
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
            p.tI += s_u[0][i];
            p.tII += s_u[1][i];
            p.workI += s_u[2][i];
        }
        *out = p;
    }
}

// Bins A (one thread per vertex) and B (4 lanes per vertex).
template <typename OffT>
__global__ __launch_bounds__(kBlock) void k_score_small(ScoreArgs<OffT> A) {
    __shared__ int lds[16 * kBlock];  // bin A: 16-entry column per thread; bin B: kCapB entries per team
    const double wmax = bitsd(A.ctr->wmax_bits);
    ScoreAcc sa = {0, 0, 0};
    score_team_bin<4, kCapB, OffT>(A, 1, wmax, lds, sa);
    {
        const Span s = xcd_span(A.bin_lo[1] - A.bin_lo[0], kBlock);
        for (long long base = s.first; base < s.hi; base += s.step) {
            const long long it = base + threadIdx.x;
            if (it < s.hi) score_thread<OffT>(A, A.sched[A.bin_lo[0] + it], wmax, lds + threadIdx.x, sa);
        }
    }
    block_reduce_score(sa, &A.part[blockIdx.x]);
}

// Bins C (16 lanes per vertex) and D (a wavefront per vertex).
template <typename OffT>
__global__ __launch_bounds__(kBlock) void k_score_big(ScoreArgs<OffT> A) {
    __shared__ int lds[16 * kBlock];  // bin C: 16 teams x kCapC; bin D: 4 teams x kCapD
    const double wmax = bitsd(A.ctr->wmax_bits);
    ScoreAcc sa = {0, 0, 0};
    score_team_bin<64, kCapD, OffT>(A, 3, wmax, lds, sa);
    score_team_bin<16, kCapC, OffT>(A, 2, wmax, lds, sa);
    block_reduce_score(sa, &A.part[kGridScore + blockIdx.x]);
}

__global__ __launch_bounds__(1024) void k_reduce_score(const ScorePart *part, int np, DevCounters *c) {
    __shared__ unsigned long long s[3][16];
    unsigned long long a = 0, b = 0, w = 0;
    for (int i = threadIdx.x; i < np; i += blockDim.x) {
        a += part[i].tI;
        b += part[i].tII;
        w += part[i].workI;
    }
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o);
        b += __shfl_xor(b, o);
        w += __shfl_xor(w, o);
    }
    if ((threadIdx.x & 63) == 0) {
        s[0][threadIdx.x >> 6] = a;
        s[1][threadIdx.x >> 6] = b;
        s[2][threadIdx.x >> 6] = w;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long x = 0, y = 0, z = 0;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
            x += s[0][i];
            y += s[1][i];
            z += s[2][i];
        }
        c->sum_tI = x;
        c->sum_tII = y;
        c->sum_workI = z;
    }
}

// ------------------------------------------------------------ pass launcher
template <typename OffT>
static rs_status score_pass_t(rs_graph *g) {
    DeviceGraph &D = g->d;
    hipEvent_t ev;
    RowArgs<OffT> A;
    A.off = (const OffT *)D.off;
    A.deg = D.deg;
    A.col = D.col;
    A.lab = D.lab;
    A.sched = D.sched;
    A.rec = D.rec;
    A.meta = D.meta;
    A.wown = D.wown;
    A.a = D.a;
    A.R = D.R;
    A.tI = D.tI;
    A.tII = D.tII;
    for (int b = 0; b <= kBins; ++b) A.bin_lo[b] = g->bin_lo[b];
    // partials: [k_rows | k_rows_mid | k_rows_hub]
    if (g->hub_grid > 0) {
        A.part = D.part_rows + kGridRows + kGridMid;
        timing_begin(g, K_ROWS_HUB, &ev);
        hipLaunchKernelGGL(k_rows_hub<OffT>, dim3(g->hub_grid), dim3(kBlock), 0, g->stream, A);
        timing_end(g, K_ROWS_HUB, ev);
    }
    A.part = D.part_rows + kGridRows;
    timing_begin(g, K_ROWS_MID, &ev);
    hipLaunchKernelGGL(k_rows_mid<OffT>, dim3(kGridMid), dim3(kBlock), 0, g->stream, A);
    timing_end(g, K_ROWS_MID, ev);
    A.part = D.part_rows;
    timing_begin(g, K_ROWS, &ev);
    hipLaunchKernelGGL(k_rows<OffT>, dim3(kGridRows), dim3(kBlock), 0, g->stream, A);
    timing_end(g, K_ROWS, ev);
    timing_begin(g, K_WMAX, &ev);
    hipLaunchKernelGGL(k_wmax, dim3(1), dim3(1024), 0, g->stream, D.part_rows, kGridRows + kGridMid + g->hub_grid,
                       D.ctr);
    timing_end(g, K_WMAX, ev);

    ScoreArgs<OffT> S;
    S.off = (const OffT *)D.off;
    S.col = D.col;
    S.lab = D.lab;
    S.sched = D.sched;
    S.rec = D.rec;
    S.meta = D.meta;
    S.a = D.a;
    S.R = D.R;
    S.tI = D.tI;
    S.tII = D.tII;
    S.ctr = D.ctr;
    S.part = D.part_score;
    for (int b = 0; b <= kBins; ++b) S.bin_lo[b] = g->bin_lo[b];
    timing_begin(g, K_SCORE, &ev);
    hipLaunchKernelGGL(k_score_small<OffT>, dim3(kGridScore), dim3(kBlock), 0, g->stream, S);
    timing_end(g, K_SCORE, ev);
    timing_begin(g, K_SCORE_BIG, &ev);
    hipLaunchKernelGGL(k_score_big<OffT>, dim3(kGridBig), dim3(kBlock), 0, g->stream, S);
    timing_end(g, K_SCORE_BIG, ev);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "score pass launch");
    return RS_OK;
}

rs_status launch_score_pass(rs_graph *g) {
    return g->d.off64 ? score_pass_t<long long>(g) : score_pass_t<int32_t>(g);
}

rs_status launch_reduce_counts(rs_graph *g) {
    hipLaunchKernelGGL(k_reduce_score, dim3(1), dim3(1024), 0, g->stream, g->d.part_score, kGridScore + kGridBig,
                       g->d.ctr);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? RS_OK : hip_fail(e, "reduce launch");
}

// ============================================================ top-k
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

// Level-0 histogram: each block counts a contiguous chunk (< 2^16 keys) in an
// LDS histogram of 16-bit counters packed two per word, then adds its
// non-zero bins to the global histogram.
__global__ __launch_bounds__(kBlock) void k_topk_hist(const double *R, const int32_t *new2old, const uint8_t *alive,
                                                      long long n, long long chunk, unsigned int *hist) {
    __shared__ unsigned int sh[kTopkBins / 2];
    for (int i = threadIdx.x; i < kTopkBins / 2; i += kBlock) sh[i] = 0u;
    __syncthreads();
    const long long lo = (long long)blockIdx.x * chunk;
    const long long hi = min(n, lo + chunk);
    for (long long v = lo + threadIdx.x; v < hi; v += kBlock) {
        if (alive[v]) {
            const unsigned int dig = key_digit(make_key(R, new2old, (int)v), 0);
            atomicAdd(&sh[dig >> 1], 1u << ((dig & 1u) * 16u));
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kTopkBins / 2; i += kBlock) {
        const unsigned int x = sh[i];
        if (x & 0xffffu) atomicAdd(&hist[2 * i], x & 0xffffu);
        if (x >> 16) atomicAdd(&hist[2 * i + 1], x >> 16);
    }
}

// Histogram of digit j over a key list (refinement of a large tie class).
__global__ __launch_bounds__(kBlock) void k_list_hist(const TopkKey *list, const unsigned long long *count, int j,
                                                      unsigned int *hist) {
    const long long n = (long long)*count;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock)
        atomicAdd(&hist[key_digit(list[i], j)], 1u);
}

// One block of 1024 threads: find the threshold digit of the current level,
// record it, and clear the histogram for the next use.
__global__ __launch_bounds__(1024) void k_topk_find(unsigned int *hist, TopkState *st, int level) {
    __shared__ long long s_scan[1024];
    __shared__ long long s_total;
    const int t = threadIdx.x;
    const long long need = st->take;
    // thread t owns bins [base, base + 63]; bins descend with t
    const int base = kTopkBins - 64 * (t + 1);
    const uint4 *h4 = (const uint4 *)(hist + base);
    long long mine = 0;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const uint4 x = h4[i];
        mine += (long long)x.x + x.y + x.z + x.w;
    }
    s_scan[t] = mine;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const long long x = t >= o ? s_scan[t - o] : 0;
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
        for (int i = 63; i >= 0; --i) {
            const long long h = hist[base + i];
            if (cum + h >= need) {
                st->digit = (unsigned int)level;
                st->thresh = (unsigned int)(base + i);
                st->above += cum;
                st->take = need - cum;
                st->binsize = h;
                st->done = (need - cum == h) ? 1u : 0u;
                break;
            }
            cum += h;
        }
    }
    __syncthreads();
    if (t == 0 && !(need > 0 && s_total >= need)) {  // cannot happen for need <= live keys: take all
        st->digit = (unsigned int)level;
        st->thresh = 0;
        st->take = 0;
        st->binsize = 0;
        st->done = 1u;
    }
    uint4 *w4 = (uint4 *)(hist + base);
#pragma unroll
    for (int i = 0; i < 16; ++i) w4[i] = make_uint4(0u, 0u, 0u, 0u);
}

// Block-aggregated append of the flagged threads' keys to list[*counter...].
__device__ __forceinline__ void block_push(TopkKey *list, unsigned long long *counter, bool act, const TopkKey &k,
                                           unsigned int *s_cnt, unsigned long long *s_base) {
    const unsigned long long m = __ballot(act);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) s_cnt[w] = (unsigned int)__popcll(m);
    __syncthreads();
    unsigned int before = 0, total = 0;
    for (int i = 0; i < kBlock / 64; ++i) {
        if (i < w) before += s_cnt[i];
        total += s_cnt[i];
    }
    if (threadIdx.x == 0 && total) *s_base = atomicAdd(counter, (unsigned long long)total);
    __syncthreads();
    if (act) list[*s_base + before + __popcll(m & ((1ull << __lane_id()) - 1ull))] = k;
    __syncthreads();
}

__global__ __launch_bounds__(kBlock) void k_topk_collect(const double *R, const int32_t *new2old, const uint8_t *alive,
                                                         long long n, TopkState *st, TopkKey *fin, TopkKey *tie) {
    __shared__ unsigned int s_cnt[kBlock / 64];
    __shared__ unsigned long long s_base;
    const unsigned int th = st->thresh;
    const bool done = st->done != 0u;
    for (long long base = (long long)blockIdx.x * kBlock; base < n; base += (long long)gridDim.x * kBlock) {
        const long long v = base + threadIdx.x;
        const bool act = v < n && alive[v];
        TopkKey k;
        k.hi = 0;
        k.lo = 0;
        k.v = -1;
        unsigned int dig = 0;
        if (act) {
            k = make_key(R, new2old, (int)v);
            dig = key_digit(k, 0);
        }
        const bool to_final = act && (dig > th || (dig == th && done));
        const bool to_tie = act && dig == th && !done;
        if (__syncthreads_or(to_final)) block_push(fin, &st->n_final, to_final, k, s_cnt, &s_base);
        if (__syncthreads_or(to_tie)) block_push(tie, &st->n_tie, to_tie, k, s_cnt, &s_base);
    }
}

__global__ __launch_bounds__(kBlock) void k_list_collect(const TopkKey *list, const unsigned long long *count,
                                                         TopkState *st, TopkKey *fin, TopkKey *tie,
                                                         unsigned long long *tie_count) {
    __shared__ unsigned int s_cnt[kBlock / 64];
    __shared__ unsigned long long s_base;
    const long long n = (long long)*count;
    const int j = (int)st->digit;
    const unsigned int th = st->thresh;
    const bool done = st->done != 0u;
    for (long long base = (long long)blockIdx.x * kBlock; base < n; base += (long long)gridDim.x * kBlock) {
        const long long i = base + threadIdx.x;
        const bool act = i < n;
        TopkKey k;
        k.hi = 0;
        k.lo = 0;
        k.v = -1;
        unsigned int dig = 0;
        if (act) {
            k = list[i];
            dig = key_digit(k, j);
        }
        const bool to_final = act && (dig > th || (dig == th && done));
        const bool to_tie = act && dig == th && !done;
        if (__syncthreads_or(to_final)) block_push(fin, &st->n_final, to_final, k, s_cnt, &s_base);
        if (__syncthreads_or(to_tie)) block_push(tie, tie_count, to_tie, k, s_cnt, &s_base);
    }
}

// Rank the tie class pairwise; the key of rank r < take goes to the final
// list at position above + r (the final list then holds `above` keys).
__global__ __launch_bounds__(kBlock) void k_tie_rank(const TopkKey *list, TopkState *st, TopkKey *fin) {
    __shared__ TopkKey tile[kBlock];
    const long long n = (long long)st->n_tie;
    if (st->done || n > kTieCap) {
        if (!st->done && n > kTieCap && blockIdx.x == 0 && threadIdx.x == 0) st->overflow = 1u;
        return;
    }
    const long long above = (long long)st->n_final;
    const long long take = st->take;
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
        if (i < n && rank < take) fin[above + rank] = me;
    }
}

// Final order of `count` keys (count <= kSortCap): bitonic sort, descending,
// in LDS by one block of 1024 threads.
__global__ __launch_bounds__(1024) void k_final_sort(const TopkKey *fin, long long count, const TopkState *st,
                                                     const double *R, const int32_t *new2old, int32_t *out_ids,
                                                     double *out_sc) {
    __shared__ TopkKey s[kSortCap];
    // the final list holds n_final keys, plus `take` ranked ties when the threshold bin was split
    const long long have = (long long)st->n_final + (st->done ? 0 : st->take);
    if (st->overflow || have != count) return;  // list incomplete: refinement pending
    int n2 = 1;
    while (n2 < count) n2 <<= 1;
    for (int i = threadIdx.x; i < n2; i += blockDim.x) {
        if (i < count) {
            s[i] = fin[i];
        } else {
            s[i].hi = 0;
            s[i].lo = 0;  // below every real key (a real key has lo >= 2^31)
            s[i].v = -1;
        }
    }
    __syncthreads();
    for (int k = 2; k <= n2; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < n2; i += blockDim.x) {
                const int l = i ^ j;
                if (l > i) {
                    const bool desc = (i & k) == 0;
                    const TopkKey x = s[i], y = s[l];
                    if (desc ? key_gt(y, x) : key_gt(x, y)) {
                        s[i] = y;
                        s[l] = x;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < count; i += blockDim.x) {
        out_ids[i] = new2old[s[i].v];
        out_sc[i] = R[s[i].v];
    }
}

// Final order of a longer list: each key's rank by pairwise comparison.
__global__ __launch_bounds__(kBlock) void k_final_rank(const TopkKey *fin, long long n, const TopkState *st,
                                                       const double *R, const int32_t *new2old, int32_t *out_ids,
                                                       double *out_sc) {
    __shared__ TopkKey tile[kBlock];
    const long long have = (long long)st->n_final + (st->done ? 0 : st->take);
    if (st->overflow || have != n) return;  // list incomplete: refinement pending
    for (long long base = (long long)blockIdx.x * kBlock; base < n; base += (long long)gridDim.x * kBlock) {
        const long long i = base + threadIdx.x;
        TopkKey me;
        me.hi = 0;
        me.lo = 0;
        me.v = -1;
        if (i < n) me = fin[i];
        long long rank = 0;
        for (long long t0 = 0; t0 < n; t0 += kBlock) {
            __syncthreads();
            if (t0 + threadIdx.x < n) tile[threadIdx.x] = fin[t0 + threadIdx.x];
            __syncthreads();
            const int lim = (int)min((long long)kBlock, n - t0);
            for (int jj = 0; jj < lim; ++jj) rank += key_gt(tile[jj], me) ? 1 : 0;
        }
        if (i < n) {
            out_ids[rank] = new2old[me.v];
            out_sc[rank] = R[me.v];
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

__global__ void k_zero_u64(unsigned long long *p, int count) {
    for (int i = threadIdx.x; i < count; i += blockDim.x) p[i] = 0ull;
}

static inline int grid_for(long long items, int per_block, int cap) {
    long long g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

static rs_status final_order(rs_graph *g, long long keff) {
    DeviceGraph &D = g->d;
    hipEvent_t ev;
    timing_begin(g, K_TOPK_RANK, &ev);
    if (keff <= kSortCap)
        hipLaunchKernelGGL(k_final_sort, dim3(1), dim3(1024), 0, g->stream, D.tfinal, keff, D.tstate, D.R,
                           D.new2old, D.tout_ids, D.tout_sc);
    else
        hipLaunchKernelGGL(k_final_rank, dim3(grid_for(keff, kBlock, 4096)), dim3(kBlock), 0, g->stream, D.tfinal,
                           keff, D.tstate, D.R, D.new2old, D.tout_ids, D.tout_sc);
    timing_end(g, K_TOPK_RANK, ev);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? RS_OK : hip_fail(e, "top-k order launch");
}

rs_status launch_topk(rs_graph *g, int64_t k, int64_t *count) {
    DeviceGraph &D = g->d;
    const long long keff = k < g->n_alive ? k : g->n_alive;
    *count = keff;
    if (keff <= 0) return RS_OK;
    hipEvent_t ev;
    long long chunk = (D.n + 255) / 256;
    if (chunk < 4096) chunk = 4096;
    if (chunk > kHistChunk) chunk = kHistChunk;
    const int grid_h = (int)((D.n + chunk - 1) / chunk);
    hipLaunchKernelGGL(k_topk_setup, dim3(1), dim3(64), 0, g->stream, D.tstate, keff);
    timing_begin(g, K_TOPK_HIST, &ev);
    hipLaunchKernelGGL(k_topk_hist, dim3(grid_h), dim3(kBlock), 0, g->stream, D.R, D.new2old, D.alive, D.n, chunk,
                       D.thist);
    timing_end(g, K_TOPK_HIST, ev);
    timing_begin(g, K_TOPK_FIND, &ev);
    hipLaunchKernelGGL(k_topk_find, dim3(1), dim3(1024), 0, g->stream, D.thist, D.tstate, 0);
    timing_end(g, K_TOPK_FIND, ev);
    timing_begin(g, K_TOPK_COLLECT, &ev);
    hipLaunchKernelGGL(k_topk_collect, dim3(grid_for(D.n, kBlock, 1024)), dim3(kBlock), 0, g->stream, D.R,
                       D.new2old, D.alive, D.n, D.tstate, D.tfinal, D.ttie);
    timing_end(g, K_TOPK_COLLECT, ev);
    timing_begin(g, K_TOPK_TIE, &ev);
    hipLaunchKernelGGL(k_tie_rank, dim3(kTieCap / kBlock), dim3(kBlock), 0, g->stream, D.ttie, D.tstate, D.tfinal);
    timing_end(g, K_TOPK_TIE, ev);
    rs_status rs_st = final_order(g, keff);
    if (rs_st != RS_OK) return rs_st;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "top-k launch");

    TopkState st;
    e = hipMemcpyAsync(&st, D.tstate, sizeof(st), hipMemcpyDeviceToHost, g->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    if (e != hipSuccess) return hip_fail(e, "top-k state read");
    if (!st.overflow) return RS_OK;

    // A tie class larger than the pairwise ranker: refine it digit by digit.
    // The final list already holds the keys above the tie class.
    unsigned long long *cnt = D.scratch_u;  // [0] current list size, [1] next list size
    TopkKey *cur = D.ttie, *nxt = D.ttie2;
    e = hipMemcpyAsync(cnt, &D.tstate->n_tie, sizeof(unsigned long long), hipMemcpyDeviceToDevice, g->stream);
    for (int j = 1; j <= 5 && e == hipSuccess; ++j) {
        unsigned long long cur_n = 0;
        e = hipMemcpyAsync(&cur_n, cnt, sizeof(cur_n), hipMemcpyDeviceToHost, g->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
        if (e != hipSuccess) break;
        const int grid_l = grid_for((long long)cur_n, kBlock, 4096);
        hipLaunchKernelGGL(k_list_hist, dim3(grid_l), dim3(kBlock), 0, g->stream, cur, cnt, j, D.thist);
        hipLaunchKernelGGL(k_topk_find, dim3(1), dim3(1024), 0, g->stream, D.thist, D.tstate, j);
        hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, g->stream, cnt + 1, 1);
        hipLaunchKernelGGL(k_list_collect, dim3(grid_l), dim3(kBlock), 0, g->stream, cur, cnt, D.tstate, D.tfinal,
                           nxt, cnt + 1);
        e = hipMemcpyAsync(cnt, cnt + 1, sizeof(unsigned long long), hipMemcpyDeviceToDevice, g->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(&st, D.tstate, sizeof(st), hipMemcpyDeviceToHost, g->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
        if (e != hipSuccess) break;
        TopkKey *tmp = cur;
        cur = nxt;
        nxt = tmp;
        if (st.done) break;
    }
    if (e == hipSuccess) e = hipMemsetAsync(&D.tstate->overflow, 0, sizeof(unsigned int), g->stream);
    if (e != hipSuccess) return hip_fail(e, "top-k refine");
    rs_st = final_order(g, keff);
    if (rs_st != RS_OK) return rs_st;
    e = hipStreamSynchronize(g->stream);
    return e == hipSuccess ? RS_OK : hip_fail(e, "top-k refine");
}

// ============================================================ removals
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
    unsigned long long cnt = 0;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (long long)gridDim.x * blockDim.x) {
        const int a = src[i], b = dst[i];
        if (a != b) cnt += (unsigned long long)delete_edge(off, deg, col, a, b);
    }
    for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o);
    if (__lane_id() == 0 && cnt) atomicAdd(removed, cnt);
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
        hipLaunchKernelGGL(k_remove_edges<int32_t>, dim3(grid), dim3(256), 0, g->stream, (const int32_t *)g->d.off,
                           g->d.deg, g->d.col, d_src, d_dst, (long long)m, d_removed);
    const hipError_t e = hipGetLastError();
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
        hipLaunchKernelGGL(k_remove_vertices<int32_t>, dim3(grid), dim3(256), 0, g->stream, (const int32_t *)g->d.off,
                           g->d.deg, g->d.col, g->d.alive, d_verts, (long long)nv, d_removed);
    const hipError_t e = hipGetLastError();
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
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? RS_OK : hip_fail(e, "compact launch");
}

// ============================================================ readers
__global__ void k_gather_scores(const double *R, const int32_t *new2old, const DevCounters *ctr, long long n, int raw,
                                double *out) {
    const double wmax = bitsd(ctr->wmax_bits);
    for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (long long)gridDim.x * blockDim.x)
        out[new2old[v]] = raw ? R[v] * wmax : R[v];
}

rs_status launch_gather_scores(rs_graph *g, double *d_out, int raw) {
    const int grid = grid_for(g->d.n, 256, 8192);
    hipLaunchKernelGGL(k_gather_scores, dim3(grid), dim3(256), 0, g->stream, g->d.R, g->d.new2old, g->d.ctr,
                       (long long)g->d.n, raw, d_out);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? RS_OK : hip_fail(e, "gather launch");
}

rs_status launch_zero_u64(rs_graph *g, unsigned long long *p, int count) {
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, g->stream, p, count);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? RS_OK : hip_fail(e, "zero launch");
}

}  // namespace rs
