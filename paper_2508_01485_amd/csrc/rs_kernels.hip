// rs_kernels.hip -- HIP kernels of the robust-spanner scoring pass (gfx950, wave64).
//
// One pass (rs_score):
//   k_rows   Algorithm 1 Steps 1-2 fused, per vertex: gather the labels of the
//            neighbours, run-length count them into interaction-matrix records
//            (rows are community-sorted, so every community is one run),
//            detect the border vertex, compute every record's weight with
//            Algorithm 2's shared terms (Eq. H_optimal) and the vertex's
//            own-community weight, and a per-block maximum for w_max.
//   k_wmax   reduce the per-block maxima to w_max (the other pass totals are
//            reduced when a reader asks).
//   k_score  Eq. RSI per border vertex u, one lane per pair (u, w) with w a
//            foreign neighbour, in the per-(vertex, community) factorised form
//            of Lemmas 1-2 (Section IV, Step 3).  One owner per vertex, fixed
//            summation order, no floating-point atomics.  Hubs too large for
//            LDS staging run in k_score_hub; k_hub_sum adds each hub's chunk
//            partials.
// Top-k (Algorithm 1 Step 4) is an exact radix select on the 96-bit key
// (score bits, complement of the caller id) with 16-bit digits.
//
// Work is cut into static tiles of consecutive vertices (and hub vertices
// with a workgroup each); a launch has one workgroup per tile, so the
// hardware dispatcher balances the uneven tiles.
#include <climits>
#include <cstring>

#include <mutex>

#include "rs_internal.h"

namespace rs {

// ------------------------------------------------------------ helpers
// Blocks for a grid-stride loop over `items`: one per per_block items, at
// least 1 and at most cap.
static inline int grid_for(long long items, int per_block, int cap) {
    long long g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

__device__ __forceinline__ unsigned long long dbits(double x) { return (unsigned long long)__double_as_longlong(x); }
__device__ __forceinline__ double bitsd(unsigned long long b) { return __longlong_as_double((long long)b); }

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

// The same terms with small arguments (<= kTab) read from LDS tables of
// log2 y, y log2 y and 1/y (most run lengths and degrees are small).
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
}
__device__ __forceinline__ double flogf_t(const Tables &t, int f) { return f <= kTab ? t.fl[f] : flogf(f); }
__device__ __forceinline__ double weight_present_t(const Tables &t, int d, double X, int ell, int f) {
    const int L = ell - 1;
    if (L < 2) return 0.0;
    const int Y = d - f;
    if (Y <= kTab) return (t.lg[Y] + (flogf_t(t, f) - X) * t.rc[Y]) * (double)L;
    return weight_present(d, X, ell, f);
}
__device__ __forceinline__ double weight_absent_t(const Tables &t, int d, double X, int ell) {
    if (ell < 2) return 0.0;
    if (d <= kTab) return (t.lg[d] - X * t.rc[d]) * (double)ell;
    return weight_absent(d, X, ell);
}


// ============================================================ row pass
template <typename OffT>
struct RowArgs {
    const OffT *off;
    const int32_t *deg, *col, *lab;
    const int32_t *clab;  // the community of each entry's neighbour (read in place of col and lab)
    const RowTile *tiles;
    const int32_t *hubs;
    int n_tiles, n_hubs, tiles_per_xcd;
    int32_t *reckey;
    RecDat *recdat;
    VCard *card;
    const int64_t *goff;
    PairRec *prec;     // pair facts at the foreign row entries, written by this pass
    const int *blist;  // incremental pass: the listed blocks (k_rows_inc)
    double *wown, *R, *raw;
    double *av;  // [n] a_v = cbrt(own-community weight), dense for the score pass's run sums
    long long *tI, *tII;
    RowPart *part;
    unsigned long long *wmax_part;  // [grid] w_max bits of each block (dense copy for k_wmax)
};

struct RowResult {
    int ell, p, q;
    double wown, lmax;
};

struct RowAcc {
    double wmax;
    unsigned long long nb, dp, ell, ellx;
};

// The vertex's row facts of this pass: its card (row facts, a_v, first four
// record keys k4), own weight, and zero scores for a non-border vertex.
template <typename OffT>
__device__ __forceinline__ void finish_row(const RowArgs<OffT> &A, int v, int d, const RowResult &r, int4 k4,
                                           long long off, long long goff, int lab, RowAcc &acc) {
    const int fown = r.q - r.p;
    const int dprime = d - fown;
    VCard c;  // written whole: one aligned 64-byte store, no partial lines
    c.off = off;
    c.goff = goff;
    c.m.deg = d;
    c.m.ell = r.ell;
    c.m.p = r.p;
    c.m.q = r.q;
    c.pad = 0;
    c.lab = lab;
    c.a = cbrt(r.wown);
    A.av[v] = c.a;
    c.key[0] = k4.x;
    c.key[1] = k4.y;
    c.key[2] = k4.z;
    c.key[3] = k4.w;
    A.card[v] = c;
    A.wown[v] = r.wown;
    acc.wmax = fmax(acc.wmax, r.lmax);
    acc.ell += (unsigned long long)r.ell;
    acc.ellx += (unsigned long long)(r.ell - (fown > 0 ? 1 : 0));
    if (dprime > 0) {
        acc.nb += 1;
        acc.dp += (unsigned long long)dprime;
    } else {
        A.R[v] = 0.0;
        A.raw[v] = 0.0;
        A.tI[v] = 0;
        A.tII[v] = 0;
    }
}

__device__ void block_reduce_row(RowAcc acc, RowPart *out, unsigned long long *wmax_out) {
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
        *wmax_out = p.wmax_bits;
    }
}

// Tile of the grid's block b: hubs take the first blocks; the tiles follow,
// the tiles of one XCD contiguous (blocks are dealt to the XCDs round-robin,
// so block b runs on XCD b % 8 and consecutive tiles share that XCD's L2).
__device__ __forceinline__ int tile_of_block(int b, int n_hubs, int per_xcd) {
    return (b & 7) * per_xcd + ((b - n_hubs) >> 3);
}

// ------------------------------------------------------------ row tiles
// A row tile is a run of consecutive vertices whose rows (capacity <=
// kRowTile entries, a contiguous slice of col) are processed flat:
//   1. every entry's neighbour label is gathered (coalesced col reads);
//   2. an entry starts a run if it starts a row or its label differs from
//      the previous entry's (rows are community-sorted, so each run is one
//      interaction-matrix record); run starts are ranked with wavefront
//      ballots and a block prefix;
//   3. one thread per vertex walks its runs in LDS: ell, X = sum f log2 f,
//      the own community's run and the entries below it (p, q);
//   4. the records' weights (Eq. H_optimal) are computed flat over runs.
// A removed entry is -1 (after compaction): such a tail forms a run that is
// skipped.
constexpr int kRowW = kBlock / 64;      // wavefronts per workgroup
constexpr int kRowU = kRowTile / kBlock; // entries per thread
constexpr int kRowM = kRowTile / 64;     // ballot words per tile
static_assert(kRowTile % kBlock == 0 && kRowTile <= 65535 && kRowTileV % kBlock == 0, "row tile size");

// Streaming state of a hub row (one workgroup).
struct HubSeg {
    int prev, next_prev;                     // label before the segment / of its last entry
    int open_start, open_label, open_slot;   // run open at the segment boundary (open_start < 0: none)
    int nruns;                               // runs started before the segment
    double red[kRowW];
    int ired[kRowW];
};

struct RowTileShared {
    HubSeg hub;
    Tables tab;
    unsigned int bm[kRowTile / 32];      // row-start bits
    unsigned long long mask[kRowM];      // run-start bits
    int mbase[kRowM];                    // run starts before each mask word
    int wlast[kRowW], wcnt[kRowW];
    unsigned short runpos[kRowTile + 1]; // tile-local entry of each run start (+ end)
    unsigned short runv[kRowTile];       // tile-local vertex of each run
    int runlab[kRowTile];                // label of each run (-1: removed tail)
    double vX[kRowTileV];
    int vd[kRowTileV], vell[kRowTileV], vlab[kRowTileV];
    unsigned short vrf[kRowTileV], vo[kRowTileV];
};

__device__ __forceinline__ int run_index(const RowTileShared &S, int e) {
    return S.mbase[e >> 6] + __popcll(S.mask[e >> 6] & ((1ull << (e & 63)) - 1ull));
}

template <typename OffT>
__device__ void row_tile(const RowArgs<OffT> &A, RowTileShared &S, int t, RowAcc &acc) {
    constexpr int kVU = kRowTileV / kBlock;  // vertices per thread
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const RowTile tl = A.tiles[t];
    const int v0 = tl.v0, nv = tl.v1 - tl.v0;
    const OffT e0 = (OffT)tl.e0;
    const int TE = tl.te;
    for (int x = tid; x < kRowTile / 32; x += kBlock) S.bm[x] = 0u;
    // the tile's entries and the facts of this thread's vertices, all
    // independent loads issued together (the tables are filled while they
    // are in flight)
    int L[kRowU];
#pragma unroll
    for (int i = 0; i < kRowU; ++i) {
        const int e = wave * (kRowTile / kRowW) + i * 64 + lane;
        L[i] = e < TE ? A.clab[e0 + e] : -2;
    }
    int vo[kVU], vc[kVU], vdeg[kVU], vlab[kVU];
    long long vgo[kVU];
#pragma unroll
    for (int j = 0; j < kVU; ++j) {
        // a slot past the tile loads the tile's first vertex (tiles are never
        // empty), and every use below skips it: no branch around the loads,
        // which would wait for them before the next slot's
        const int i = tid + j * kBlock;
        const int ic = i < nv ? i : 0;
        const OffT a0 = A.off[v0 + ic], a1 = A.off[v0 + ic + 1];
        vo[j] = (int)(a0 - e0);
        vc[j] = (int)(a1 - a0);
        vdeg[j] = A.deg[v0 + ic];
        vlab[j] = A.lab[v0 + ic];
        vgo[j] = A.goff[v0 + ic];
    }
    fill_tables(S.tab);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kVU; ++j)
        if (tid + j * kBlock < nv && vc[j] > 0) atomicOr(&S.bm[vo[j] >> 5], 1u << (vo[j] & 31));
    if (lane == 63) S.wlast[wave] = L[kRowU - 1];
    __syncthreads();
    unsigned long long m[kRowU];
    int cnt = 0;
#pragma unroll
    for (int i = 0; i < kRowU; ++i) {
        const int e = wave * (kRowTile / kRowW) + i * 64 + lane;
        int lp = __shfl_up(L[i], 1);
        const int carry = i > 0 ? __shfl(L[i > 0 ? i - 1 : 0], 63) : (wave > 0 ? S.wlast[wave > 0 ? wave - 1 : 0] : INT_MIN);
        if (lane == 0) lp = carry;
        const bool rs = (S.bm[e >> 5] >> (e & 31)) & 1u;
        m[i] = __ballot(e < TE && (rs || L[i] != lp));
        cnt += __popcll(m[i]);
    }
    if (lane == 0) S.wcnt[wave] = cnt;
    __syncthreads();
    int base = 0, total = 0;
#pragma unroll
    for (int x = 0; x < kRowW; ++x) {
        const int c = S.wcnt[x];
        if (x < wave) base += c;
        total += c;
    }
    const unsigned long long lt = (1ull << lane) - 1ull;
#pragma unroll
    for (int i = 0; i < kRowU; ++i) {
        const int e = wave * (kRowTile / kRowW) + i * 64 + lane;
        if (lane == 0) {
            S.mask[e >> 6] = m[i];
            S.mbase[e >> 6] = base;
        }
        if ((m[i] >> lane) & 1ull) {
            const int r = base + __popcll(m[i] & lt);
            S.runpos[r] = (unsigned short)e;
            S.runlab[r] = L[i];
        }
        base += __popcll(m[i]);
    }
    if (tid == 0) S.runpos[total] = (unsigned short)TE;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kVU; ++j) {
        const int i = tid + j * kBlock;
        if (i >= nv) continue;
        const int o = vo[j], c = vc[j], d = vdeg[j], cv = vlab[j];
        int rf = 0, re = 0;
        if (c > 0) {
            rf = run_index(S, o);
            re = o + c >= TE ? total : run_index(S, o + c);
        }
        double X = 0.0;
        int ell = 0, fown = 0, below = 0;
        for (int r = rf; r < re; ++r) {
            const int lb = S.runlab[r];
            if (lb < 0) break;
            const int f = (int)S.runpos[r + 1] - (int)S.runpos[r];
            X += flogf_t(S.tab, f);
            ++ell;
            S.runv[r] = (unsigned short)i;
            if (lb == cv)
                fown = f;
            else if (lb < cv)
                below += f;
        }
        S.vX[i] = X;
        S.vd[i] = d;
        S.vlab[i] = cv;
        S.vell[i] = ell;
        S.vrf[i] = (unsigned short)rf;
        S.vo[i] = (unsigned short)o;
        RowResult res;
        res.ell = ell;
        res.p = below;
        res.q = below + fown;
        res.wown = fown > 0 ? weight_present_t(S.tab, d, X, ell, fown) : weight_absent_t(S.tab, d, X, ell);
        res.lmax = res.wown;
        int4 k4;  // the first record keys: the labels of the first valid runs
        k4.x = ell > 0 ? S.runlab[rf] : INT_MAX;
        k4.y = ell > 1 ? S.runlab[rf + 1] : INT_MAX;
        k4.z = ell > 2 ? S.runlab[rf + 2] : INT_MAX;
        k4.w = ell > 3 ? S.runlab[rf + 3] : INT_MAX;
        finish_row(A, v0 + i, d, res, k4, (long long)e0 + o, vgo[j], cv, acc);
    }
    __syncthreads();
    for (int r = tid; r < total; r += kBlock) {
        const int lb = S.runlab[r];
        if (lb < 0) continue;
        const int i = S.runv[r];
        const int f = (int)S.runpos[r + 1] - (int)S.runpos[r];
        const double w = weight_present_t(S.tab, S.vd[i], S.vX[i], S.vell[i], f);
        const int o = S.vo[i];
        const OffT idx = e0 + (OffT)(o + (r - (int)S.vrf[i]));
        A.reckey[idx] = lb;
        RecDat rd;
        rd.pos = (int)S.runpos[r] - o;
        rd.f = f;
        rd.w = w;
        A.recdat[idx] = rd;
        acc.wmax = fmax(acc.wmax, w);
        // pair facts at the run's entries when it is another community's:
        // entry (w, u) gets the record of C(u) in w's row (the weight computed
        // once per run; neighbouring threads' runs are neighbouring entries)
        if (lb != S.vlab[i]) {
            const int p0 = (int)S.runpos[r];
            PairRec pr;
            pr.w = w;
            pr.f = f;
            for (int t = 0; t < f; ++t) {
                pr.back = t;
                A.prec[e0 + (OffT)(p0 + t)] = pr;
            }
        }
    }
}

// ------------------------------------------------------------ hub rows
// A vertex whose row capacity exceeds kRowTile gets a workgroup: its row is
// streamed in segments of kRowTile entries with the tile's flat machinery
// (labels, run starts by ballot, runs closed flat over LDS), twice: the first
// pass counts the runs, X and the own run, the second writes the weighted
// records.  The run still open at a segment's end is carried to the next.
template <int PASS, typename OffT>
__device__ __forceinline__ void hub_run(const RowArgs<OffT> &A, OffT rb, int d, int cv, double X, int ell, int label,
                                        int start, int f, int slot, double &xpart, int &below, int &fown,
                                        double &lmax) {
    if (PASS == 1) {
        xpart += flogf(f);
        if (label == cv)
            fown = f;
        else if (label < cv)
            below += f;
        A.reckey[rb + slot] = label;
        RecDat rd;
        rd.pos = start;
        rd.f = f;
        rd.w = 0.0;  // set by the second pass, once X and ell are known
        A.recdat[rb + slot] = rd;
    } else {
        const double w = weight_present(d, X, ell, f);
        A.recdat[rb + slot].w = w;
        lmax = fmax(lmax, w);
    }
}

template <int PASS, typename OffT>
__device__ void hub_pass(const RowArgs<OffT> &A, RowTileShared &S, OffT rb, int d, int cv, double X, int ell,
                         double &xpart, int &below, int &fown, double &lmax) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    HubSeg &H = S.hub;
    if (tid == 0) {
        H.prev = INT_MIN;
        H.open_start = -1;
        H.nruns = 0;
    }
    for (int seg0 = 0; seg0 < d; seg0 += kRowTile) {
        const int TE = min(kRowTile, d - seg0);
        int L[kRowU];
#pragma unroll
        for (int i = 0; i < kRowU; ++i) {
            const int e = wave * (kRowTile / kRowW) + i * 64 + lane;
            L[i] = e < TE ? A.clab[rb + seg0 + e] : -2;
        }
        __syncthreads();  // the previous segment is done with S
        if (lane == 63) S.wlast[wave] = L[kRowU - 1];
#pragma unroll
        for (int i = 0; i < kRowU; ++i)
            if (wave * (kRowTile / kRowW) + i * 64 + lane == TE - 1) H.next_prev = L[i];
        __syncthreads();
        unsigned long long m[kRowU];
        int cnt = 0;
#pragma unroll
        for (int i = 0; i < kRowU; ++i) {
            const int e = wave * (kRowTile / kRowW) + i * 64 + lane;
            int lp = __shfl_up(L[i], 1);
            const int carry = i > 0 ? __shfl(L[i > 0 ? i - 1 : 0], 63) : (wave > 0 ? S.wlast[wave > 0 ? wave - 1 : 0] : H.prev);
            if (lane == 0) lp = carry;
            m[i] = __ballot(e < TE && L[i] != lp);
            cnt += __popcll(m[i]);
        }
        if (lane == 0) S.wcnt[wave] = cnt;
        __syncthreads();
        int base = 0, total = 0;
#pragma unroll
        for (int x = 0; x < kRowW; ++x) {
            const int c = S.wcnt[x];
            if (x < wave) base += c;
            total += c;
        }
        const unsigned long long lt = (1ull << lane) - 1ull;
#pragma unroll
        for (int i = 0; i < kRowU; ++i) {
            const int e = wave * (kRowTile / kRowW) + i * 64 + lane;
            if ((m[i] >> lane) & 1ull) {
                const int r = base + __popcll(m[i] & lt);
                S.runpos[r] = (unsigned short)e;
                S.runlab[r] = L[i];
            }
            base += __popcll(m[i]);
        }
        if (tid == 0) S.runpos[total] = (unsigned short)TE;
        __syncthreads();
        const bool last = seg0 + TE >= d;
        const int nr0 = H.nruns;
        if (PASS == 2) {
            // pair facts at this segment's foreign entries: the entry's run
            // (the one carried in, or the last run start at or before it)
            // and that run's record from the first pass
#pragma unroll
            for (int i = 0; i < kRowU; ++i) {
                const int e = wave * (kRowTile / kRowW) + i * 64 + lane;
                if (e >= TE || L[i] < 0 || L[i] == cv) continue;
                int lo = 0, hi = total;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if ((int)S.runpos[mid] <= e)
                        lo = mid + 1;
                    else
                        hi = mid;
                }
                const int slot = lo == 0 ? H.open_slot : nr0 + lo - 1;
                const RecDat rd = A.recdat[rb + slot];
                PairRec pr;
                pr.w = weight_present(d, X, ell, rd.f);
                pr.f = rd.f;
                pr.back = seg0 + e - rd.pos;
                A.prec[rb + seg0 + e] = pr;
            }
        }
        // the run carried from the previous segment closes at this segment's
        // first run start (or at the row's end)
        if (tid == 0 && H.open_start >= 0 && (total > 0 || last)) {
            const int end = total > 0 ? seg0 + (int)S.runpos[0] : d;
            hub_run<PASS, OffT>(A, rb, d, cv, X, ell, H.open_label, H.open_start, end - H.open_start, H.open_slot,
                                xpart, below, fown, lmax);
            H.open_start = -1;
        }
        const int closed = last ? total : total - 1;  // the segment's last run stays open unless the row ends
        for (int r = tid; r < closed; r += kBlock) {
            const int f = (int)S.runpos[r + 1] - (int)S.runpos[r];
            hub_run<PASS, OffT>(A, rb, d, cv, X, ell, S.runlab[r], seg0 + (int)S.runpos[r], f, nr0 + r, xpart,
                                below, fown, lmax);
        }
        __syncthreads();
        if (tid == 0) {
            if (!last && total > 0) {
                H.open_start = seg0 + (int)S.runpos[total - 1];
                H.open_label = S.runlab[total - 1];
                H.open_slot = nr0 + total - 1;
            }
            H.nruns = nr0 + total;
            H.prev = H.next_prev;
        }
    }
    __syncthreads();
}

__device__ __forceinline__ double block_sum_d(double x, double *red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < kRowW; ++i) t += red[i];
    __syncthreads();
    return t;
}

__device__ __forceinline__ double block_max_d(double x, double *red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < kRowW; ++i) t = fmax(t, red[i]);
    __syncthreads();
    return t;
}

__device__ __forceinline__ int block_sum_i(int x, int *red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
    __syncthreads();
    int t = 0;
    for (int i = 0; i < kRowW; ++i) t += red[i];
    __syncthreads();
    return t;
}

template <typename OffT>
__device__ void hub_row(const RowArgs<OffT> &A, RowTileShared &S, int v, RowAcc &acc) {
    const OffT rb = A.off[v];
    const int d = A.deg[v];
    const int cv = A.lab[v];
    double xpart = 0.0, lmax = 0.0;
    int below = 0, fown = 0;
    hub_pass<1, OffT>(A, S, rb, d, cv, 0.0, 0, xpart, below, fown, lmax);
    const double X = block_sum_d(xpart, S.hub.red);
    const int p = block_sum_i(below, S.hub.ired);
    const int fo = block_sum_i(fown, S.hub.ired);  // one thread holds the own run's length
    const int ell = S.hub.nruns;
    __syncthreads();  // everyone has read pass 1's totals before pass 2 resets them
    hub_pass<2, OffT>(A, S, rb, d, cv, X, ell, xpart, below, fown, lmax);
    const double lm = block_max_d(lmax, S.hub.red);  // (its barriers order pass 2's record writes)
    if (threadIdx.x == 0) {
        RowResult r;
        r.ell = ell;
        r.p = p;
        r.q = p + fo;
        r.wown = fo > 0 ? weight_present(d, X, ell, fo) : weight_absent(d, X, ell);
        r.lmax = fmax(lm, r.wown);
        int4 k4;
        k4.x = ell > 0 ? A.reckey[rb + 0] : INT_MAX;
        k4.y = ell > 1 ? A.reckey[rb + 1] : INT_MAX;
        k4.z = ell > 2 ? A.reckey[rb + 2] : INT_MAX;
        k4.w = ell > 3 ? A.reckey[rb + 3] : INT_MAX;
        finish_row(A, v, d, r, k4, (long long)rb, A.goff[v], cv, acc);
    }
}

// Reduce the row partials of a pass into the counters (one workgroup; the
// loads of four partials per thread are in flight together).
__device__ void reduce_row_parts(const RowPart *part, int np, DevCounters *c) {
    __shared__ unsigned long long s[5][kBlock / 64];
    unsigned long long w = 0, nb = 0, dp = 0, ell = 0, ellx = 0;
    for (int i0 = threadIdx.x; i0 < np; i0 += 4 * kBlock) {
        RowPart q[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int i = i0 + j * kBlock;
            if (i < np) {
                q[j] = part[i];
            } else {
                q[j] = RowPart{};
            }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            w = max(w, q[j].wmax_bits);
            nb += q[j].n_border;
            dp += q[j].sum_dprime;
            ell += q[j].sum_ell;
            ellx += q[j].sum_ell_x;
        }
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
        DevCounters r = *c;
        r.wmax_bits = r.n_border = r.sum_dprime = r.sum_ell = r.sum_ell_x = 0;
        for (int i = 0; i < kBlock / 64; ++i) {
            r.wmax_bits = max(r.wmax_bits, s[0][i]);
            r.n_border += s[1][i];
            r.sum_dprime += s[2][i];
            r.sum_ell += s[3][i];
            r.sum_ell_x += s[4][i];
        }
        *c = r;
    }
}

// Algorithm 1 Steps 1-2 for every vertex: hub rows first, then the tiles.
template <typename OffT>
__global__ __launch_bounds__(kBlock) void k_rows(RowArgs<OffT> A) {
    __shared__ RowTileShared S;
    RowAcc acc = {0.0, 0, 0, 0, 0};
    const int b = (int)blockIdx.x;
    if (b < A.n_hubs) {
        hub_row(A, S, A.hubs[b], acc);
    } else {
        const int t = tile_of_block(b, A.n_hubs, A.tiles_per_xcd);
        if (t < A.n_tiles) row_tile(A, S, t, acc);
    }
    block_reduce_row(acc, &A.part[b], &A.wmax_part[b]);
}

// Whether an incremental pass runs every block of the full launches: its
// units (listed row blocks, main score blocks and big-hub chunks, and the
// units of the affected tile vertices) exceed kFullPassTenths of the full
// pass's workgroups (a removed hub touches much of the graph; full launches
// run faster per unit, and the bits are the same).  Every kernel of the
// pass decides alike from the marks' counters.
__device__ __forceinline__ bool inc_full(const unsigned long long *ictr, int grid_rows, int grid_score) {
    long long u = (long long)ictr[kIcRows] + (long long)ictr[kIcMain] + (long long)ictr[kIcBig];
#pragma unroll
    for (int b = 0; b < kScoreBins; ++b) u += ((long long)ictr[kIcBins + b] + (kBlock >> b) - 1) / (kBlock >> b);
    return 10 * u > (long long)kFullPassTenths * ((long long)grid_rows + grid_score);
}

// The incremental pass's row blocks: block i of a capped grid takes the
// listed blocks i, i + gridDim.x, ... (every block of the full launch in a
// full pass), each exactly as k_rows runs it.
template <typename OffT>
__global__ __launch_bounds__(kBlock) void k_rows_inc(RowArgs<OffT> A, const unsigned long long *ictr, int grid_rows,
                                                     int grid_score) {
    __shared__ RowTileShared S;
    const bool full = inc_full(ictr, grid_rows, grid_score);
    const long long cnt = full ? (long long)grid_rows : (long long)ictr[kIcRows];
    for (long long i = blockIdx.x; i < cnt; i += gridDim.x) {
        RowAcc acc = {0.0, 0, 0, 0, 0};
        const int b = full ? (int)i : A.blist[i];
        if (b < A.n_hubs) {
            hub_row(A, S, A.hubs[b], acc);
        } else {
            const int t = tile_of_block(b, A.n_hubs, A.tiles_per_xcd);
            if (t < A.n_tiles) row_tile(A, S, t, acc);
        }
        block_reduce_row(acc, &A.part[b], &A.wmax_part[b]);
        __syncthreads();  // the next block's LDS
    }
}

// w_max of a pass from the dense per-block maxima of the row kernel: up to
// kWmaxBlocks workgroups of 1,024 threads each take a contiguous slice
// (eight loads per thread in flight together) and store its maximum; the
// workgroup that finishes last (a ticket) takes the maximum of those and
// resets the ticket.  A maximum does not depend on the order, so the bits are
// those of a single workgroup's.  The other row totals are reduced only when
// a reader asks for them.
constexpr int kWmaxBlocks = 64;
__global__ __launch_bounds__(1024) void k_wmax(const unsigned long long *wpart, int np, unsigned long long *wblk,
                                               unsigned int *ticket, DevCounters *c) {
    __shared__ unsigned long long s[16];
    __shared__ bool last;
    const int per = (np + gridDim.x - 1) / gridDim.x;
    const int lo = blockIdx.x * per, hi = min(np, lo + per);
    unsigned long long w = 0;
    for (int i0 = lo + threadIdx.x; i0 < hi; i0 += 8 * 1024) {
        unsigned long long q[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int i = i0 + j * 1024;
            q[j] = i < hi ? wpart[i] : 0ull;
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) w = max(w, q[j]);
    }
    for (int o = 32; o > 0; o >>= 1) w = max(w, (unsigned long long)__shfl_xor(w, o));
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = w;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long m = 0;
        for (int i = 0; i < 16; ++i) m = max(m, s[i]);
        wblk[blockIdx.x] = m;
        __threadfence();
        last = atomicAdd(ticket, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (last && threadIdx.x == 0) {
        __threadfence();
        unsigned long long m = 0;
        for (unsigned int i = 0; i < gridDim.x; ++i) m = max(m, ((volatile unsigned long long *)wblk)[i]);
        c->wmax_bits = m;
        *ticket = 0u;
    }
}

// Batched graphs: each graph's w_max, the maximum of the w_max of its row
// blocks (row tiles never span two graphs), one wavefront per graph.  The
// block values are fp64 bits maximised as integers, as for the whole-graph
// w_max, so a graph's w_max has the bits it has when the graph is alone.
__global__ __launch_bounds__(kBlock) void k_wmax_graphs(const unsigned long long *wpart, const int32_t *gblk_off,
                                                        const int32_t *gblk, int n_graphs,
                                                        unsigned long long *gwmax) {
    const int gi = (int)blockIdx.x * (kBlock / 64) + (int)(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (gi >= n_graphs) return;  // whole wavefronts leave; no barrier follows
    unsigned long long m = 0;
    for (int i = gblk_off[gi] + lane; i < gblk_off[gi + 1]; i += 64) m = max(m, wpart[gblk[i]]);
    for (int o = 32; o > 0; o >>= 1) m = max(m, (unsigned long long)__shfl_xor(m, o));
    if (lane == 0) gwmax[gi] = m;
}

// All row totals of the last pass (for the counter readers).
__global__ __launch_bounds__(kBlock) void k_reduce_rows(const RowPart *part, int np, DevCounters *c) {
    reduce_row_parts(part, np, c);
}

// ============================================================ score pass
template <typename OffT>
struct ScoreArgs {
    const OffT *off;
    const int32_t *col, *lab;
    const int2 *tiles;
    const int32_t *hubs;
    int n_tiles, n_hubs, tiles_per_xcd;
    const int32_t *hub_first;
    const int2 *hub_chunk;
    int n_chunks, n_chunks_lds;
    HubPart *hub_part;
    const int32_t *outl;
    const int64_t *oo;      // out-list offsets
    const int32_t *reckey;
    const RecDat *recdat;
    const VCard *card;
    const PairRec *prec;    // pair facts at the foreign row entries, written by the row pass
    const uint32_t *hfilter;  // big hubs' neighbour filters (hub n_hubs_lds + i at i * kFilterWords)
    const OutEnt *oe;         // each out-list entry's row entries (x, y) and (y, x)
    int n_hubs_lds;
    const PairLink *plink;  // link slots: reverse entry and out-list range of each G' entry
    const double *av;       // [n] a_v of the row pass
    const int *blist;       // unused by the score kernels (the incremental lists are arguments)
    const unsigned long long *gwmax;  // batched graphs: w_max bits of each graph, else null
    const int32_t *vgraph;            // batched graphs: graph of each vertex
    double *R, *raw;
    long long *tI, *tII;
    const DevCounters *ctr;
};

// Sorted-range helpers on LDS arrays.
__device__ __forceinline__ int lds_lower(const int *a, int lo, int hi, int x) {
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] < x)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}
__device__ __forceinline__ bool lds_has(const int *a, int lo, int hi, int x) {
    const int i = lds_lower(a, lo, hi, x);
    return i < hi && a[i] == x;
}

// Out-lists keep removed entries complemented (~id) in place, so a list is
// ascending in the decoded id.
__device__ __forceinline__ int out_id(int x) { return x < 0 ? ~x : x; }

// Position of the live id x among the n out-list entries a[0..n) in LDS, or -1.
__device__ __forceinline__ int lds_find_out(const int *a, int n, int x) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (out_id(a[mid]) < x)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo < n && a[lo] == x ? lo : -1;
}

// Whether the n out-list entries a[0..n) in LDS hold the live id x.
__device__ __forceinline__ bool lds_has_out(const int *a, int n, int x) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (out_id(a[mid]) < x)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo < n && a[lo] == x;
}

// Position of the live id t in the sorted out-list outl[o0, o1) in HBM
// (removed ids are complemented and keep their place), or -1: a 16-ary
// search on the decoded ids, each step 15 loads issued together (a list of up
// to 16 entries is one step).  Probes past the range load its last entry and
// are discarded after the load: a test before the load would make each
// probe wait for the previous one.
__device__ __forceinline__ long long out_find(const int32_t *outl, long long o0, long long o1, int t) {
    long long lo = o0, hi = o1;
    if (hi <= lo) return -1;
    while (hi - lo > 16) {
        const long long st = (hi - lo + 15) >> 4;
        int y[15];
#pragma unroll
        for (int j = 1; j < 16; ++j) y[j - 1] = outl[min(lo + j * st, hi - 1)];
        int cnt = 0;
#pragma unroll
        for (int j = 1; j < 16; ++j) cnt += (int)((lo + j * st < hi) & (out_id(y[j - 1]) <= t));
        lo += cnt * st;
        hi = min(hi, lo + st);
    }
    int y[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) y[j] = outl[min(lo + j, hi - 1)];
    long long f = -1;
#pragma unroll
    for (int j = 0; j < 16; ++j)
        if (lo + j < hi && y[j] == t) f = lo + j;
    return f;
}

__device__ __forceinline__ bool out_has(const int32_t *outl, long long o0, long long o1, int t) {
    return out_find(outl, o0, o1, t) >= 0;
}

// The type-II terms of the pair (u, w), w a foreign neighbour of u (Lemma 2,
// unnormalised weights), from the pair's facts at w's entry for u (W =
// w_w(C(u)) and the run of C(u) in w's row): W^(2/3) times the sum of a_v
// over the other members v of that run (v in C(u), v adjacent to w; counted
// whether or not v ~ u), and the count f_w(C(u)) - 1.
template <typename OffT>
__device__ __forceinline__ double type2_pair(const ScoreArgs<OffT> &A, int u, const PairRec &pr, long long e) {
    if (pr.f <= 1) return 0.0;
    double S = 0.0;
    const int32_t *run = A.col + (e - pr.back);
    for (int i = 0; i < pr.f; i += 8) {
        int x[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) x[t] = i + t < pr.f ? run[i + t] : u;
        double av[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) av[t] = x[t] != u ? A.av[x[t]] : 0.0;
#pragma unroll
        for (int t = 0; t < 8; ++t) S += av[t];
    }
    const double c1 = cbrt(pr.w);
    return c1 * c1 * S;
}

// R of Algorithm 1: the raw sum over w_max and d(d-1); 0 when d < 2 or w_max = 0.
__device__ __forceinline__ double score_value(double acc, int d, double wmax) {
    return (d >= 2 && wmax > 0.0) ? acc / wmax / (double)((long long)d * (d - 1)) : 0.0;
}

template <typename OffT>
__device__ __forceinline__ void score_store(const ScoreArgs<OffT> &A, int u, int d, double acc, long long cI,
                                            long long cII, double wmax) {
    A.R[u] = score_value(acc, d, A.gwmax ? bitsd(A.gwmax[A.vgraph[u]]) : wmax);
    A.raw[u] = acc;
    A.tI[u] = cI;
    A.tII[u] = cII;
}

// Exclusive prefix of one int per thread over the block; total to *total.
__device__ __forceinline__ int block_excl_scan(int x, int *ws, int &total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int incl = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(incl, o);
        if (lane >= o) incl += y;
    }
    if (lane == 63) ws[wave] = incl;
    __syncthreads();
    int base = 0;
    total = 0;
#pragma unroll
    for (int i = 0; i < kBlock / 64; ++i) {
        const int c = ws[i];
        if (i < wave) base += c;
        total += c;
    }
    return base + incl - x;
}

// Store a hub chunk's partial; the chunk finishing last adds the partials
// of the hub in chunk order and writes its score (one thread).
// A hub chunk's partial (its pair terms and counts, summed over the block in a
// fixed tree order) goes to its slot; k_hub_sum adds the chunks of each hub in
// chunk order once the score kernels are done.  The chunk's counts also go to
// the block totals.
template <typename OffT>
__device__ void hub_chunk_store(const ScoreArgs<OffT> &A, const double *red, const long long (*ired)[kBlock / 64],
                                int hub, int chunk) {
    HubPart hp;
    hp.raw = 0.0;
    hp.tI = hp.tII = 0;
    hp.pad = 0;
    for (int i = 0; i < kBlock / 64; ++i) {
        hp.raw += red[i];
        hp.tI += ired[0][i];
        hp.tII += ired[1][i];
    }
    A.hub_part[A.hub_first[hub] + chunk] = hp;
}

// Per-pair facts of a unit's type-I scan, and the hits found so far.
constexpr int kScanR = 2;                  // work items per lane per round
constexpr int kWaveHitCap = 192;           // hits a wavefront holds before evaluating them
constexpr int kHitCap = kWaveHitCap * (kBlock / 64);
static_assert(kWaveHitCap >= 64 * kScanR, "a round's hits always fit after a flush");
struct TypeIShared {
    int ibeg[kBlock];      // first work item of each pair within its wavefront's list
    int ioo[kBlock];       // out-list start of each pair's w
    int pv[kBlock];        // u of each pair
    int pcu[kBlock];       // C(u)
    int pw[kBlock];        // w
    double pW[kBlock];     // w_w(C(u))
};
struct HitBuf {
    int hitp[kHitCap];     // pair of each hit (per wavefront: ascending)
    int hitc[kHitCap];     // where the edge test found (u, v): the edge test's code
    int hito[kHitCap];     // the out-list position of v (the entry w -> v)
    double hitv[kHitCap];  // the hit's two ordered triads
};

// Lanes of one wavefront exchange data through LDS: the writes must be
// complete and visible before other lanes read them.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The terms of a wavefront's nb held hits (from slot h0), then each pair's
// own lane adds its hits (a contiguous range of the list) in list order.
template <class Edge, typename OffT>
__device__ __forceinline__ void typeI_flush(const ScoreArgs<OffT> &A, const TypeIShared &T, HitBuf &H, const Edge &edge,
                                            int h0, int nb, int lane, int me, bool mine, double &val, int &t1) {
    for (int h = lane; h < nb; h += 64) {
        // the weights of the triangle {u, w, v} are the pair facts at its
        // row entries: w_v(C(u)) at (v, u), w_w(C(v)) at (w, v), w_v(C(w))
        // at (v, w) (the out-list entry w -> v holds the last two indices)
        const int q = H.hitp[h0 + h];
        const double W = T.pW[q];
        const OutEnt e = A.oe[H.hito[h0 + h]];
        const double w_wv = A.prec[e.xy].w;
        const double w_vw = A.prec[e.yx].w;
        const double w_vu = edge.wvu(A, T, H.hitc[h0 + h]);
        H.hitv[h0 + h] = cbrt(w_vu * w_wv * W) + cbrt(W * w_vw * w_vu);
    }
    wave_sync();
    if (mine) {
        int a = 0, b = nb;
        while (a < b) {
            const int mid = (a + b) >> 1;
            if (H.hitp[h0 + mid] < me)
                a = mid + 1;
            else
                b = mid;
        }
        for (int h = a; h < nb && H.hitp[h0 + h] == me; ++h) {
            val += H.hitv[h0 + h];
            t1 += 2;
        }
    }
    wave_sync();
}

// Type-I triads of a unit's pairs (Eq. RSI with v adjacent to u and C(v) !=
// C(u): the triangles of G').  The pair (u, w) finds the triangles {u, w, v}
// with v in out(w) (each triangle at u is found by exactly one of its two
// pairs).  Every position of every pair's out-list is one work item.  Each
// wavefront works through the items of its own 64 pairs, kScanR items per
// lane per round with their loads in flight together (consecutive lanes read
// consecutive entries of one list, and no lane scans a long list alone); the
// wavefronts of the block do not wait for each other.  A live entry v with
// edge(p, v) closes a triangle.  Hits are appended in item order, so each
// pair's hits stay contiguous and in out-list order; when the wavefront's
// list is nearly full (and at the end) every held hit's two ordered triads
// (w, v) and (v, w),
//   cbrt(w_v(C(u)) w_w(C(v)) W) + cbrt(W w_v(C(w)) w_v(C(u))),  W = w_w(C(u)),
// are evaluated, one lane per hit, and the pair's own lane adds them to its
// sum in list order (so the sum's order is fixed).  `items` is the lane's
// out-list length (0 without a pair), and T.ioo, T.pv, T.pcu, T.pw, T.pW hold
// the lane's pair; they must be visible block-wide (a barrier) before the call.
template <class Edge, typename OffT>
__device__ void typeI_scan(const ScoreArgs<OffT> &A, TypeIShared &T, HitBuf &H, int items, const Edge &edge,
                           double &val, int &t1) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int w0 = wave * 64;          // the wavefront's first pair
    const int h0 = wave * kWaveHitCap;  // and its hit slots
    int incl = items;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(incl, o);
        if (lane >= o) incl += y;
    }
    const int total = __shfl(incl, 63);
    T.ibeg[tid] = incl - items;
    wave_sync();
    int nb = 0;  // held hits of this wavefront
    for (int base = 0; base < total; base += 64 * kScanR) {
        int y[kScanR], p[kScanR], op[kScanR];
#pragma unroll
        for (int r = 0; r < kScanR; ++r) {
            const int i = base + r * 64 + lane;
            p[r] = w0;
            y[r] = -1;
            op[r] = 0;
            if (i < total) {
                int lo = 0, hi = 64;  // the last pair of the wavefront whose first item is <= i
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (T.ibeg[w0 + mid] <= i)
                        lo = mid;
                    else
                        hi = mid;
                }
                p[r] = w0 + lo;
                op[r] = T.ioo[w0 + lo] + (i - T.ibeg[w0 + lo]);
                y[r] = A.outl[op[r]];
            }
        }
#pragma unroll
        for (int r = 0; r < kScanR; ++r) {
            int code = 0;
            const bool hit = y[r] >= 0 && y[r] != T.pv[p[r]] && edge(p[r], y[r], code);
            const unsigned long long m = __ballot(hit);
            if (hit) {
                const int s = nb + __popcll(m & ((1ull << lane) - 1ull));
                H.hitp[h0 + s] = p[r];
                H.hitc[h0 + s] = code;
                H.hito[h0 + s] = op[r];
            }
            nb += __popcll(m);
        }
        if (nb > kWaveHitCap - 64 * kScanR || (base + 64 * kScanR >= total && nb > 0)) {
            wave_sync();
            typeI_flush(A, T, H, edge, h0, nb, lane, tid, items > 0, val, t1);
            nb = 0;
        }
    }
}

// ------------------------------------------------------------ score units
// A score unit is either a tile -- <= kScoreTileV consecutive vertices with
// at most kScoreTileP foreign entries -- or one chunk of kScoreTileP pairs of
// a score hub whose foreign list fits in LDS.  Either way the foreign
// neighbours w of the unit's vertices are laid out in LDS (a vertex's
// entries ascending), one lane takes one pair (u, w), and the pair terms are
// summed in a fixed order: per vertex in pair order for a tile, in a tree
// over the chunk for a hub (k_hub_sum then adds a hub's chunk partials in a
// fixed order).
static_assert(kScoreTileV == kBlock && kScoreTileP == kBlock, "score unit size: one vertex and one pair per thread");

// A score unit's LDS: kW foreign neighbours (a tile's at most kScoreTileP,
// an LDS hub's at most kHubList); tiles launch with the smaller form, which
// leaves room for one more workgroup per CU.
template <int kW>
struct ScoreUnitSharedT {
    static constexpr int kWords = kW;
    int w[kW];                       // foreign neighbours
    int pb[kScoreTileV + 1];         // tile: first pair of each vertex
    unsigned short pu[kScoreTileP];  // tile: vertex of each pair
    int ws[kBlock / 64];
    double red[kBlock / 64];
    long long ired[2][kBlock / 64];
    TypeIShared ti;
    union {  // three phases that never overlap
        struct {  // prologue: the tile's vertices
            long long ou[kScoreTileV], go[kScoreTileV];  // row start and first pair slot
            int cu[kScoreTileV], p[kScoreTileV], h[kScoreTileV];
        } v;
        HitBuf hits;  // type-I scan
        struct {      // epilogue: the lanes' pair terms
            double val[kBlock];
            int t2[kBlock], t1[kBlock];
        } e;
    } u;
};
using ScoreUnitShared = ScoreUnitSharedT<kHubList>;
using ScoreTileShared = ScoreUnitSharedT<kScoreTileP>;

// A hub chunk's partial: block tree sum of the lanes' terms (thread 0 gets it).
__device__ __forceinline__ void chunk_tree(double x, long long y1, long long y2, double *red,
                                           long long (*ired)[kBlock / 64]) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        x += __shfl_xor(x, o);
        y1 += __shfl_xor(y1, o);
        y2 += __shfl_xor(y2, o);
    }
    if (lane == 0) {
        red[wave] = x;
        ired[0][wave] = y1;
        ired[1][wave] = y2;
    }
    __syncthreads();
}

// Edge tests of a unit's type-I scan: u's foreign list is in LDS (a tile
// vertex's slice, or a hub's whole list).
template <class SU>
// Each also gives a code for its hits, from which wvu() reads w_v(C(u)),
// the pair fact at the row entry (v, u).
struct TileEdge {
    const SU *S;
    __device__ __forceinline__ bool operator()(int p, int y, int &code) const {
        const int i = S->pu[p];
        const int k = lds_lower(S->w, S->pb[i], S->pb[i + 1], y);
        code = k;  // (u, v) is the unit's pair k: its W is w_v(C(u))
        return k < S->pb[i + 1] && S->w[k] == y;
    }
    template <typename OffT>
    __device__ __forceinline__ double wvu(const ScoreArgs<OffT> &, const TypeIShared &T, int code) const {
        return T.pW[code];
    }
};
struct HubListEdge {
    const int *w;
    int n;
    int cbase, ccnt;  // the chunk's pairs: list positions [cbase, cbase + ccnt)
    long long go;     // the hub's first link slot
    __device__ __forceinline__ bool operator()(int, int y, int &code) const {
        const int k = lds_lower(w, 0, n, y);
        code = k;  // (u, v) is the hub's pair k
        return k < n && w[k] == y;
    }
    template <typename OffT>
    __device__ __forceinline__ double wvu(const ScoreArgs<OffT> &A, const TypeIShared &T, int code) const {
        if (code >= cbase && code < cbase + ccnt) return T.pW[code - cbase];
        return A.prec[A.plink[go + code].e].w;
    }
};

// vl: a unit of listed vertices vl[0, vn) (the incremental pass's rescored
// vertices) instead of the tile idx.
template <typename OffT, class SU>
__device__ void score_unit(const ScoreArgs<OffT> &A, SU &S, bool hub_unit_arg, int idx, double wmax,
                           const int32_t *vl = nullptr, int vn = 0) {
    // a hub chunk needs room for the hub's whole foreign list
    const bool hub_unit = SU::kWords >= kHubList && hub_unit_arg;
    const int tid = threadIdx.x;
    // ---- prologue: lay out the unit's pairs
    int v0 = 0, nv = 0, total = 0, dp = 0, deg = 0, pb = 0;    // tile
    int hub = 0, chunk = 0, hu = 0, hdp = 0, hcu = 0;  // hub chunk
    long long hgo = 0;
    if (hub_unit) {
        const int2 hc = A.hub_chunk[idx];
        hub = hc.x;
        chunk = hc.y;
        hu = A.hubs[hub];
        const VCard ch = A.card[hu];
        const VMeta m = ch.m;
        const long long ou = ch.off;
        const int h = m.q - m.p;
        hdp = m.deg - h;  // <= the load-time count, which fits kHubList
        hcu = ch.lab;
        hgo = ch.goff;
        for (int j = tid; j < hdp; j += kBlock) S.w[j] = A.col[ou + (j < m.p ? j : j + h)];
        total = min(kBlock, max(0, hdp - chunk * kBlock));
        __syncthreads();
    } else {
        if (vl) {
            nv = vn;
        } else {
            const int2 tl = A.tiles[idx];
            v0 = tl.x;
            nv = tl.y - tl.x;
        }
        if (tid < nv) {
            const int v = vl ? vl[tid] : v0 + tid;
            const VCard cv = A.card[v];
            const VMeta m = cv.m;
            deg = m.deg;
            dp = m.deg - (m.q - m.p);
            S.u.v.ou[tid] = cv.off;
            S.u.v.go[tid] = cv.goff;
            S.u.v.cu[tid] = cv.lab;
            S.u.v.p[tid] = m.p;
            S.u.v.h[tid] = m.q - m.p;
        }
        pb = block_excl_scan(dp, S.ws, total);
        if (tid < nv) {
            S.pb[tid] = pb;
            for (int k = pb; k < pb + dp; ++k) S.pu[k] = (unsigned short)tid;
        }
        if (tid == 0) S.pb[nv] = total;
        __syncthreads();
        if (tid < total) {
            const int i = S.pu[tid];
            const int j = tid - S.pb[i];
            S.w[tid] = A.col[S.u.v.ou[i] + (j < S.u.v.p[i] ? j : j + S.u.v.h[i])];
        }
        __syncthreads();
    }
    // ---- the lane's pair: type II
    const bool has = tid < total;
    double val = 0.0;
    int t2 = 0, t1 = 0, items = 0;
    if (has) {
        int u, cu, w;
        long long slot;
        if (hub_unit) {
            const int k = chunk * kBlock + tid;
            u = hu;
            cu = hcu;
            w = S.w[k];
            slot = hgo + k;
        } else {
            const int i = S.pu[tid];
            u = vl ? vl[i] : v0 + i;
            cu = S.u.v.cu[i];
            w = S.w[tid];
            slot = S.u.v.go[i] + (tid - S.pb[i]);
        }
        const PairLink pl = A.plink[slot];
        const PairRec pr = A.prec[pl.e];
        val = type2_pair(A, u, pr, pl.e);
        t2 = pr.f - 1;
        items = pl.on;
        S.ti.ioo[tid] = pl.oo;
        S.ti.pv[tid] = u;
        S.ti.pcu[tid] = cu;
        S.ti.pw[tid] = w;
        S.ti.pW[tid] = pr.w;
    }
    // ---- type I (the hit lists overlay the prologue's vertex facts)
    __syncthreads();
    if (hub_unit) {
        HubListEdge E;
        E.w = S.w;
        E.n = hdp;
        E.cbase = chunk * kBlock;
        E.ccnt = total;
        E.go = hgo;
        typeI_scan(A, S.ti, S.u.hits, items, E, val, t1);
    } else {
        TileEdge<SU> E;
        E.S = &S;
        typeI_scan(A, S.ti, S.u.hits, items, E, val, t1);
    }
    // ---- epilogue: sums in a fixed order (its terms overlay the hit lists)
    __syncthreads();
    if (!hub_unit) {
        S.u.e.val[tid] = val;
        S.u.e.t2[tid] = t2;
        S.u.e.t1[tid] = t1;
        __syncthreads();
        if (tid < nv && dp > 0) {
            double acc = 0.0;
            long long c1 = 0, c2 = 0;
            for (int q = pb; q < pb + dp; ++q) {
                acc += S.u.e.val[q];
                c2 += S.u.e.t2[q];
                c1 += S.u.e.t1[q];
            }
            score_store(A, vl ? vl[tid] : v0 + tid, deg, acc, c1, c2, wmax);
        }
        return;
    }
    chunk_tree(val, t1, t2, S.red, S.ired);
    if (tid == 0) hub_chunk_store(A, S.red, S.ired, hub, chunk);
}

// A hub whose foreign list exceeds kHubList: u's list stays in HBM.  The
// type-I edge test of (u, y) uses the out-lists instead: the edge is in
// exactly one of out(u) (staged in LDS when it fits) and out(y).
constexpr int kHubOutStage = 1024;
struct ScoreHubBigShared {
    double red[kBlock / 64];
    long long ired[2][kBlock / 64];
    int outu[kHubOutStage];
    TypeIShared ti;
    HitBuf hits;
};

// A big hub's neighbour filter: bit h(y) is set for every current foreign
// neighbour y of the hub (one multiplicative hash into 2^kFilterBits bits,
// built at the start of the score pass).  A clear bit proves that y is no
// neighbour; a set bit is checked exactly.
__device__ __forceinline__ uint32_t filter_hash(int y) {
    return ((uint32_t)y * 2654435761u) >> (32 - kFilterBits);
}

struct HubOutEdge {
    const int *stage;      // out(u) in LDS (n_stage entries), or null
    int n_stage;
    const int32_t *outl;
    const int64_t *oo;
    long long uo0, uo1;    // out(u) in HBM
    const uint32_t *filt;  // u's neighbour filter
    int u;
    // code: the out-list position of the edge, times two, plus 1 when it is
    // the entry v -> u (else u -> v)
    __device__ __forceinline__ bool operator()(int, int y, int &code) const {
        const uint32_t h = filter_hash(y);
        if (!((filt[h >> 5] >> (h & 31)) & 1u)) return false;
        long long o = -1;
        if (stage) {
            const int k = lds_find_out(stage, n_stage, y);
            if (k >= 0) o = uo0 + k;
        } else {
            o = out_find(outl, uo0, uo1, y);
        }
        if (o >= 0) {
            code = (int)(o << 1);
            return true;
        }
        o = out_find(outl, oo[y], oo[y + 1], u);
        code = (int)(o << 1) | 1;
        return o >= 0;
    }
    template <typename OffT>
    __device__ __forceinline__ double wvu(const ScoreArgs<OffT> &A, const TypeIShared &, int code) const {
        const OutEnt e = A.oe[code >> 1];
        return A.prec[(code & 1) ? e.xy : e.yx].w;
    }
};

template <typename OffT>
__device__ void score_hub_big(const ScoreArgs<OffT> &A, ScoreHubBigShared &S, int hub, int chunk, double wmax) {
    const int tid = threadIdx.x;
    const int u = A.hubs[hub];
    const VCard cu_ = A.card[u];
    const VMeta m = cu_.m;
    const long long ou = cu_.off;
    const int h = m.q - m.p;
    const int dp = m.deg - h;
    const int cu = cu_.lab;
    const long long uo0 = A.oo[u], uo1 = A.oo[u + 1];
    const int n_out = (int)(uo1 - uo0);
    const bool staged = n_out <= kHubOutStage;
    if (staged)
        for (int j = tid; j < n_out; j += kBlock) S.outu[j] = A.outl[uo0 + j];
    const int k = chunk * kScoreTileP + tid;
    double val = 0.0;
    int t2 = 0, t1 = 0, items = 0;
    if (k < dp) {
        const int w = A.col[ou + (k < m.p ? k : k + h)];
        const PairLink pl = A.plink[cu_.goff + k];
        const PairRec pr = A.prec[pl.e];
        val = type2_pair(A, u, pr, pl.e);
        t2 = pr.f - 1;
        items = pl.on;
        S.ti.ioo[tid] = pl.oo;
        S.ti.pv[tid] = u;
        S.ti.pcu[tid] = cu;
        S.ti.pw[tid] = w;
        S.ti.pW[tid] = pr.w;
    }
    HubOutEdge E;
    E.stage = staged ? S.outu : nullptr;
    E.n_stage = n_out;
    E.outl = A.outl;
    E.oo = A.oo;
    E.uo0 = uo0;
    E.uo1 = uo1;
    E.filt = A.hfilter + (size_t)(hub - A.n_hubs_lds) * kFilterWords;
    E.u = u;
    __syncthreads();  // the staged out-list
    typeI_scan(A, S.ti, S.hits, items, E, val, t1);
    chunk_tree(val, t1, t2, S.red, S.ired);
    if (tid == 0) hub_chunk_store(A, S.red, S.ired, hub, chunk);
}

// Each big hub's neighbour filter from its current foreign list (after the
// row pass: the card's own run [p, q)): built in LDS by one workgroup per
// hub, then written out whole.
template <typename OffT>
__global__ __launch_bounds__(kBlock) void k_hub_filters(const int32_t *hubs, int h0, const VCard *card,
                                                        const int32_t *col, uint32_t *filters) {
    __shared__ uint32_t f[kFilterWords];
    const int h = h0 + (int)blockIdx.x;
    for (int i = threadIdx.x; i < kFilterWords; i += kBlock) f[i] = 0u;
    __syncthreads();
    const VCard c = card[hubs[h]];
    const int hp = c.m.q - c.m.p;
    const int dp = c.m.deg - hp;
    for (int j = threadIdx.x; j < dp; j += kBlock) {
        const uint32_t x = filter_hash(col[c.off + (j < c.m.p ? j : j + hp)]);
        atomicOr(&f[x >> 5], 1u << (x & 31));
    }
    __syncthreads();
    uint32_t *out = filters + (size_t)blockIdx.x * kFilterWords;
    for (int i = threadIdx.x; i < kFilterWords; i += kBlock) out[i] = f[i];
}

// Algorithm 1 Step 3 (Eq. RSI) for every border vertex of the LDS-sized
// score hubs (one chunk of 256 pairs per workgroup) ...
template <typename OffT>
__global__ __launch_bounds__(kBlock) void k_score_lds_hubs(ScoreArgs<OffT> A) {
    __shared__ ScoreUnitShared S;
    score_unit(A, S, true, (int)blockIdx.x, bitsd(A.ctr->wmax_bits));
}

// ... and of the score tiles (tile t of XCD x = t / per runs on a block of
// that XCD: blocks are dealt to the XCDs round-robin, so consecutive tiles
// share an L2).
template <typename OffT>
__global__ __launch_bounds__(kBlock) void k_score(ScoreArgs<OffT> A) {
    __shared__ ScoreTileShared S;
    const int idx = tile_of_block((int)blockIdx.x, 0, A.tiles_per_xcd);
    if (idx < A.n_tiles) score_unit(A, S, false, idx, bitsd(A.ctr->wmax_bits));
}

// Both in one launch (the LDS hubs' chunks first, so they start early, then
// the tiles), with the larger LDS form for every workgroup: used when the
// LDS hubs are few, where a launch of their own would end on one chunk's
// latency with nothing beside it.
constexpr int kSplitHubChunks = 4096;
template <typename OffT>
__global__ __launch_bounds__(kBlock) void k_score_all(ScoreArgs<OffT> A) {
    __shared__ ScoreUnitShared S;
    const int b = (int)blockIdx.x;
    const bool hub_unit = b < A.n_chunks_lds;
    const int idx = hub_unit ? b : tile_of_block(b, A.n_chunks_lds, A.tiles_per_xcd);
    if (hub_unit || idx < A.n_tiles) score_unit(A, S, hub_unit, idx, bitsd(A.ctr->wmax_bits));
}

// ... and of the hubs too large for LDS (chunks n_chunks_lds ...); partials
// summed by k_hub_sum after the score kernels.
template <typename OffT>
__global__ __launch_bounds__(kBlock) void k_score_hub(ScoreArgs<OffT> A) {
    __shared__ ScoreHubBigShared S;
    const double wmax = bitsd(A.ctr->wmax_bits);
    const int b = (int)blockIdx.x;
    const int2 hc = A.hub_chunk[A.n_chunks_lds + b];
    score_hub_big(A, S, hc.x, hc.y, wmax);
}

// The incremental pass's score work in one launch (the parts are
// independent and overlap): block i of a capped grid takes the work items
// i, i + gridDim.x, ... of one queue,
//   1. the listed big-hub chunks (all of them in a full pass),
//   2. the listed main blocks, LDS-hub chunks and tiles (all in a full pass),
//   3. the units of the affected tile vertices, largest bin first: 256 >> b
//      listed vertices of bin b per unit, so at most 256 pairs (none in a
//      full pass, whose tiles run whole).
// Every item runs as in the full launches; a unit's values are those of its
// vertices' tiles (a vertex's sum does not depend on the unit's others).
template <typename OffT>
__global__ __launch_bounds__(kBlock) void k_score_inc(ScoreArgs<OffT> A, const int32_t *big, const int32_t *main_,
                                                      const int32_t *abin, const unsigned long long *ictr,
                                                      uint8_t *hflag, int grid_rows, int grid_score, int grid_main) {
    __shared__ union {
        ScoreUnitShared u;
        ScoreHubBigShared h;
    } S;
    // the whole-hub flags of the marks were turned into lists: clear them
    for (int h = blockIdx.x * kBlock + threadIdx.x; h < A.n_hubs; h += gridDim.x * kBlock) hflag[h] = 0;
    const double wmax = bitsd(A.ctr->wmax_bits);
    const bool full = inc_full(ictr, grid_rows, grid_score);
    const long long n_big = full ? (long long)(A.n_chunks - A.n_chunks_lds) : (long long)ictr[kIcBig];
    const long long n_main = full ? (long long)grid_main : (long long)ictr[kIcMain];
    // units of bin b: ufirst[b] after the bins above b
    long long ufirst[kScoreBins], voff[kScoreBins], vcnt[kScoreBins], n_units = 0, off = 0;
#pragma unroll
    for (int b = 0; b < kScoreBins; ++b) {
        vcnt[b] = full ? 0 : (long long)ictr[kIcBins + b];
        voff[b] = off;
        off += vcnt[b];
    }
#pragma unroll
    for (int b = kScoreBins - 1; b >= 0; --b) {
        ufirst[b] = n_units;
        n_units += (vcnt[b] + (kBlock >> b) - 1) / (kBlock >> b);
    }
    const long long total = n_big + n_main + n_units;
    for (long long i = blockIdx.x; i < total; i += gridDim.x) {
        if (i < n_big) {
            const int c = full ? (int)i : big[i];
            const int2 hc = A.hub_chunk[A.n_chunks_lds + c];
            score_hub_big(A, S.h, hc.x, hc.y, wmax);
        } else if (i < n_big + n_main) {
            const long long j = i - n_big;
            const int bl = full ? (int)j : main_[j];
            const bool hub_unit = bl < A.n_chunks_lds;
            const int idx = hub_unit ? bl : tile_of_block(bl, A.n_chunks_lds, A.tiles_per_xcd);
            if (hub_unit || idx < A.n_tiles) score_unit(A, S.u, hub_unit, idx, wmax);
        } else {
            const long long u = i - n_big - n_main;
            int b = 0;  // units of bin b are [ufirst[b], ufirst[b - 1]); ufirst[kScoreBins - 1] = 0
            while (ufirst[b] > u) ++b;
            const int vpu = kBlock >> b;
            const long long start = voff[b] + (u - ufirst[b]) * vpu;
            const int nv = (int)min((long long)vpu, voff[b] + vcnt[b] - start);
            score_unit(A, S.u, false, -1, wmax, abin + start, nv);
        }
        __syncthreads();  // the next item's LDS
    }
}

// Each hub's score from its chunk partials (one wavefront per hub: lane l
// sums chunks l, l + 64, ... in order, then a fixed shuffle tree).  A hub
// whose foreign list became empty keeps the zeros the row pass wrote.
__global__ __launch_bounds__(kBlock) void k_hub_sum(const int32_t *hubs, const int32_t *hub_first,
                                                    const HubPart *hub_part, int n_hubs, const VCard *card,
                                                    const DevCounters *ctr, const unsigned long long *gwmax,
                                                    const int32_t *vgraph, double *R, double *raw,
                                                    long long *tI, long long *tII) {
    const int hub = (int)blockIdx.x * (kBlock / 64) + (int)(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (hub >= n_hubs) return;
    const int first = hub_first[hub], nch = hub_first[hub + 1] - first;
    double acc = 0.0;
    long long c1 = 0, c2 = 0;
    for (int c = lane; c < nch; c += 64) {
        const HubPart q = hub_part[first + c];
        acc += q.raw;
        c1 += q.tI;
        c2 += q.tII;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        acc += __shfl_xor(acc, o);
        c1 += __shfl_xor(c1, o);
        c2 += __shfl_xor(c2, o);
    }
    if (lane == 0) {
        const int u = hubs[hub];
        const VMeta m = card[u].m;
        if (m.deg - (m.q - m.p) > 0) {
            R[u] = score_value(acc, m.deg, bitsd(gwmax ? gwmax[vgraph[u]] : ctr->wmax_bits));
            raw[u] = acc;
            tI[u] = c1;
            tII[u] = c2;
        }
    }
}

// The pass's triad totals from the per-vertex counts (read on demand: the
// incremental pass reruns vertices in units of its own, so per-workgroup
// partials of the full launch would go stale).
__global__ __launch_bounds__(1024) void k_reduce_score(const long long *tI, const long long *tII, long long n,
                                                       DevCounters *c) {
    __shared__ unsigned long long s[2][16];
    unsigned long long a = 0, b = 0;
    for (long long i = threadIdx.x; i < n; i += blockDim.x) {
        a += (unsigned long long)tI[i];
        b += (unsigned long long)tII[i];
    }
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o);
        b += __shfl_xor(b, o);
    }
    if ((threadIdx.x & 63) == 0) {
        s[0][threadIdx.x >> 6] = a;
        s[1][threadIdx.x >> 6] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long x = 0, y = 0;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
            x += s[0][i];
            y += s[1][i];
        }
        c->sum_tI = x;
        c->sum_tII = y;
    }
}

// W1 = sum over G' pairs (u, w) of min(d'(u), d'(w)), the list elements a
// merge intersection would scan (reported for the algorithmic-byte count;
// computed when a reader asks, from the last pass's row facts).  One
// wavefront per vertex; per-block partials in wpart.
template <typename OffT>
__global__ __launch_bounds__(kBlock) void k_work_I(const OffT *off, const int32_t *col, const VCard *card, long long n,
                                                   unsigned long long *wpart) {
    __shared__ unsigned long long s[kBlock / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    unsigned long long acc = 0;
    for (long long x = (long long)blockIdx.x * (kBlock / 64) + wave; x < n; x += (long long)gridDim.x * (kBlock / 64)) {
        const VMeta m = card[x].m;
        const int dpx = m.deg - (m.q - m.p);
        if (dpx == 0) continue;
        const OffT rb = off[x];
        for (int j = lane; j < m.deg; j += 64) {
            if (j >= m.p && j < m.q) continue;
            const VMeta my = card[col[rb + j]].m;
            acc += (unsigned long long)min(dpx, my.deg - (my.q - my.p));
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (lane == 0) s[wave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int i = 0; i < kBlock / 64; ++i) t += s[i];
        wpart[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(kBlock) void k_reduce_work(const unsigned long long *wpart, DevCounters *c) {
    __shared__ unsigned long long s[kBlock / 64];
    unsigned long long t = 0;
    for (int i = threadIdx.x; i < kWorkBlocks; i += kBlock) t += wpart[i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long z = 0;
        for (int i = 0; i < kBlock / 64; ++i) z += s[i];
        c->sum_workI = z;
    }
}

// ------------------------------------------------------------ link slots
// For a row entry e = (x, y) with y foreign to x: plink[goff[x] + k] = {the
// index of the entry (y, x), y's out-list range}, k = y's index among x's
// foreign entries (x's row without its own-community id range).  Rows are
// sorted, so positions are binary searches.  Run at load and after removals
// (compaction shifts rows).
// Lower bounds (first position holding an id >= key) of N keys, key i in the
// sorted row row[i][0, d[i]), found together: binary searches in lockstep,
// each step one independent load per key still searching.  DEC: removed
// entries (complemented in place, the row still ordered on the original
// ids) compare by their id.
template <int N, bool DEC>
__device__ __forceinline__ void lower_n(const int32_t *const *row, const int *d, const int *key, int *pos) {
    int lo[N], hi[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
        lo[i] = 0;
        hi[i] = d[i];
    }
    for (;;) {
        bool more = false;
#pragma unroll
        for (int i = 0; i < N; ++i) more |= lo[i] < hi[i];
        if (!more) break;
        int mid[N], y[N];
#pragma unroll
        for (int i = 0; i < N; ++i) {
            mid[i] = (lo[i] + hi[i]) >> 1;
            y[i] = lo[i] < hi[i] ? row[i][mid[i]] : 0;
        }
#pragma unroll
        for (int i = 0; i < N; ++i) {
            if (lo[i] < hi[i]) {
                const int yi = DEC && y[i] < 0 ? ~y[i] : y[i];
                if (yi < key[i])
                    lo[i] = mid[i] + 1;
                else
                    hi[i] = mid[i];
            }
        }
    }
#pragma unroll
    for (int i = 0; i < N; ++i) pos[i] = lo[i];
}

template <typename OffT>
struct LinkArgs {
    const OffT *off;
    const int32_t *deg, *col, *lab, *cstart;
    const int64_t *goff, *oo;
    PairLink *plink;
    const int32_t *outl;        // out-lists (tombstones complemented)
    OutEnt *oe;                 // each out-list entry's row entries
    const unsigned int *vmark;  // after removals: kRowChanged marks the rows that changed
    const VCard *card;          // the last pass's own-run bounds [p, q) of the unchanged rows
};

// The link of x's row entry j (if it is a current foreign entry).
template <typename OffT>
__device__ __forceinline__ void link_entry(const LinkArgs<OffT> &L, int x, int j) {
    if (j >= L.deg[x]) return;  // removed tail
    const int y = L.col[(long long)L.off[x] + j];
    const int cx = L.lab[x];
    if (L.lab[y] == cx) return;  // own community
    // first position in a's row (length da) holding an id >= key
    auto lower = [&](int a, int da, int key) {
        const int32_t *row = L.col + L.off[a];
        int l = 0, h = da;
        while (l < h) {
            const int mid = (l + h) >> 1;
            if (row[mid] < key)
                l = mid + 1;
            else
                h = mid;
        }
        return l;
    };
    const int dx = L.deg[x];
    int kx = j;
    if (y >= L.cstart[cx + 1]) kx -= lower(x, dx, L.cstart[cx + 1]) - lower(x, dx, L.cstart[cx]);
    PairLink pl;
    pl.e = (long long)L.off[y] + lower(y, L.deg[y], x);
    pl.oo = (int)L.oo[y];
    pl.on = (int)(L.oo[y + 1] - L.oo[y]);
    L.plink[L.goff[x] + kx] = pl;
}

// Every entry (at load): the owning row is the last x with off[x] <= e.
template <typename OffT>
__global__ __launch_bounds__(kBlock) void k_links(LinkArgs<OffT> L, long long n, long long nnz) {
    for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < nnz; e += (long long)gridDim.x * kBlock) {
        long long lo = 0, hi = n;
        while (hi - lo > 1) {
            const long long mid = (lo + hi) >> 1;
            if ((long long)L.off[mid] <= e)
                lo = mid;
            else
                hi = mid;
        }
        link_entry(L, (int)lo, (int)(e - (long long)L.off[lo]));
    }
}

template <typename OffT>
static LinkArgs<OffT> link_args(rs_graph *g) {
    DeviceGraph &D = g->d;
    LinkArgs<OffT> L;
    L.off = (const OffT *)D.off;
    L.deg = D.deg;
    L.col = D.col;
    L.lab = D.lab;
    L.cstart = D.cstart;
    L.goff = D.goff;
    L.oo = D.oo;
    L.vmark = D.vmark;
    L.card = D.card;
    L.plink = D.plink;
    L.outl = D.outl;
    L.oe = D.oe;
    return L;
}

template <typename OffT>
static rs_status links_t(rs_graph *g) {
    DeviceGraph &D = g->d;
    if (D.nnz == 0) return RS_OK;
    const long long grid = std::min<long long>((D.nnz + kBlock - 1) / kBlock, 65536);
    hipLaunchKernelGGL(k_links<OffT>, dim3((int)grid), dim3(kBlock), 0, g->stream, link_args<OffT>(g),
                       (long long)D.n, (long long)D.nnz);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? RS_OK : hip_fail(e, "link-slot launch");
}

rs_status launch_links(rs_graph *g) { return g->d.off64 ? links_t<long long>(g) : links_t<int32_t>(g); }

// Each out-list entry x -> y (at load): the indices of the row entries
// (x, y) and (y, x); the owner x is the last with oo[x] <= o.
template <typename OffT>
__global__ __launch_bounds__(kBlock) void k_out_entries(LinkArgs<OffT> L, long long n, long long n_out) {
    for (long long o = (long long)blockIdx.x * kBlock + threadIdx.x; o < n_out; o += (long long)gridDim.x * kBlock) {
        long long lo = 0, hi = n;
        while (hi - lo > 1) {
            const long long mid = (lo + hi) >> 1;
            if (L.oo[mid] <= o)
                lo = mid;
            else
                hi = mid;
        }
        const int x = (int)lo;
        const int y = out_id(L.outl[o]);
        const long long xb = (long long)L.off[x], yb = (long long)L.off[y];
        const int32_t *rows[2] = {L.col + xb, L.col + yb};
        const int ds[2] = {L.deg[x], L.deg[y]};
        const int keys[2] = {y, x};
        int k[2];
        lower_n<2, true>(rows, ds, keys, k);
        OutEnt e;
        e.xy = xb + k[0];
        e.yx = yb + k[1];
        L.oe[o] = e;
    }
}

template <typename OffT>
static rs_status out_entries_t(rs_graph *g) {
    DeviceGraph &D = g->d;
    const long long n_out = g->n_out;
    if (n_out == 0) return RS_OK;
    hipLaunchKernelGGL(k_out_entries<OffT>, dim3(grid_for(n_out, kBlock, 65536)), dim3(kBlock), 0, g->stream,
                       link_args<OffT>(g), (long long)D.n, n_out);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? RS_OK : hip_fail(e, "out-entry launch");
}

rs_status launch_out_entries(rs_graph *g) {
    return g->d.off64 ? out_entries_t<long long>(g) : out_entries_t<int32_t>(g);
}

// Each entry's neighbour community (once at load; compaction moves it with
// the entry): the row pass reads it in place of the id and its label.
__global__ __launch_bounds__(kBlock) void k_col_labels(const int32_t *col, const int32_t *lab, long long nnz,
                                                       int32_t *clab) {
    for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < nnz; e += (long long)gridDim.x * kBlock) {
        const int x = col[e];
        clab[e] = x >= 0 ? lab[x] : -1;
    }
}

rs_status launch_col_labels(rs_graph *g) {
    DeviceGraph &D = g->d;
    if (D.nnz == 0) return RS_OK;
    hipLaunchKernelGGL(k_col_labels, dim3(grid_for(D.nnz, kBlock, 65536)), dim3(kBlock), 0, g->stream, D.col, D.lab,
                       (long long)D.nnz, D.clab);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? RS_OK : hip_fail(e, "entry label launch");
}


__global__ void k_zero_u64(unsigned long long *p, int count) {
    for (int i = threadIdx.x; i < count; i += blockDim.x) p[i] = 0ull;
}

// After an incremental pass: when w_max changed, every R is recomputed from
// its raw sum (the same expression as the pass, so the bits equal a full
// pass's).  Raw sums are 0 for vertices without foreign neighbours.
__global__ __launch_bounds__(kBlock) void k_rescale(const unsigned long long *wmax_old, const DevCounters *ctr,
                                                    const VCard *card, const double *raw, double *R, long long n) {
    const unsigned long long wb = ctr->wmax_bits;
    if (wb == *wmax_old) return;
    const double wmax = bitsd(wb);
    for (long long u = (long long)blockIdx.x * kBlock + threadIdx.x; u < n; u += (long long)gridDim.x * kBlock) {
        const VMeta m = card[u].m;
        R[u] = m.deg - (m.q - m.p) > 0 ? score_value(raw[u], m.deg, wmax) : 0.0;
    }
}

// ------------------------------------------------------------ graph replay
static void drain_one(rs_graph *g, Replay &R) {
    if (!R.unread) return;
    if (!R.events.empty()) (void)hipEventSynchronize(R.events.back().second.second);
    for (auto &pe : R.events) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, pe.second.first, pe.second.second) == hipSuccess) {
            g->timing.ms[pe.first] += t;
            g->timing.launches[pe.first] += 1;
        }
    }
    R.unread = false;
}

void drain_replays(rs_graph *g) {
    drain_one(g, g->pass_rep);
    drain_one(g, g->topk_rep);
}

static void drop_replay(rs_graph *g, Replay &R) {
    drain_one(g, R);
    if (R.exec) (void)hipGraphExecDestroy(R.exec);
    R.exec = nullptr;
    R.key = -1;
    for (auto &pe : R.events) {
        g->timing.pool.push_back(pe.second.first);
        g->timing.pool.push_back(pe.second.second);
    }
    R.events.clear();
}

void release_replays(rs_graph *g) {
    drop_replay(g, g->pass_rep);
    drop_replay(g, g->topk_rep);
}

// Enqueue a fixed launch sequence on the graph's stream through a replayed
// HIP graph (captured on first use, and again when the key changes), or
// eagerly when graphs are off, when per-kernel timing is on (its events are
// recorded around eager launches), when the stream is the null stream, or
// when the caller is capturing the stream itself.
template <class F>
static rs_status replay(rs_graph *g, Replay &R, long long key, F enqueue) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (g->graphs_off || g->timing.on || !g->stream || hipStreamIsCapturing(g->stream, &cs) != hipSuccess ||
        cs != hipStreamCaptureStatusNone)
        return enqueue();
    if (!R.exec || R.key != key) {
        drop_replay(g, R);
        const size_t p0 = g->timing.pending.size();
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamBeginCapture(g->stream, hipStreamCaptureModeRelaxed);
        rs_status st = RS_OK;
        if (e == hipSuccess) {
            st = enqueue();
            e = hipStreamEndCapture(g->stream, &graph);
        }
        if (e == hipSuccess && st == RS_OK) e = hipGraphInstantiate(&R.exec, graph, nullptr, nullptr, 0);
        if (graph) (void)hipGraphDestroy(graph);
        // the events captured in the sequence now belong to the replay
        R.events.assign(g->timing.pending.begin() + (long)p0, g->timing.pending.end());
        g->timing.pending.resize(p0);
        if (e != hipSuccess || st != RS_OK) {
            (void)hipGetLastError();
            drop_replay(g, R);
            g->graphs_off = true;  // this stream cannot be captured: stay eager
            return enqueue();
        }
        R.key = key;
        R.timed = g->timing.on;
    }
    drain_one(g, R);  // a previous replay's times, before its events are recorded again
    const hipError_t e = hipGraphLaunch(R.exec, g->stream);
    if (e != hipSuccess) return hip_fail(e, "graph launch");
    R.unread = R.timed;
    return RS_OK;
}

// ------------------------------------------------------------ pass launcher
// Workgroups of an incremental pass's launches (each loops over its list):
// enough to fill the chip, few enough that an empty list costs little.
constexpr int kIncGrid = 2048;

template <typename OffT>
static rs_status score_pass_t(rs_graph *g, bool inc) {
    DeviceGraph &D = g->d;
    hipEvent_t ev;
    RowArgs<OffT> A;
    A.off = (const OffT *)D.off;
    A.deg = D.deg;
    A.col = D.col;
    A.lab = D.lab;
    A.clab = D.clab;
    A.tiles = D.rtiles;
    A.hubs = D.rhubs;
    A.n_tiles = g->n_rtiles;
    A.n_hubs = g->n_rhubs;
    A.tiles_per_xcd = (g->n_rtiles + 7) / 8;
    A.reckey = D.reckey;
    A.recdat = D.recdat;
    A.card = D.card;
    A.goff = D.goff;
    A.prec = D.prec;
    A.blist = inc ? D.rlist : nullptr;
    A.wown = D.wown;
    A.av = D.av;
    A.R = D.R;
    A.raw = D.raw;
    A.tI = D.tI;
    A.tII = D.tII;
    A.part = D.part_rows;
    A.wmax_part = D.wmax_part;
    const int n_big = g->n_schunks - g->n_schunks_lds;
    const int grid_main = g->grid_score - n_big;
    if (inc) {
        timing_begin(g, K_ROWS, &ev);
        hipLaunchKernelGGL(k_rows_inc<OffT>, dim3(std::max(1, std::min(g->grid_rows, kIncGrid))), dim3(kBlock), 0,
                           g->stream, A, (const unsigned long long *)D.ictr, g->grid_rows, g->grid_score);
        timing_end(g, K_ROWS, ev);
    } else if (g->grid_rows > 0) {
        timing_begin(g, K_ROWS, &ev);
        hipLaunchKernelGGL(k_rows<OffT>, dim3(g->grid_rows), dim3(kBlock), 0, g->stream, A);
        timing_end(g, K_ROWS, ev);
    }
    timing_begin(g, K_WMAX, &ev);
    hipLaunchKernelGGL(k_wmax, dim3(std::max(1, std::min(kWmaxBlocks, (g->grid_rows + 8191) / 8192))), dim3(1024), 0,
                       g->stream, D.wmax_part, g->grid_rows, D.wblk, D.wticket, D.ctr);
    timing_end(g, K_WMAX, ev);
    if (g->n_graphs > 0) {
        timing_begin(g, K_WMAX_GRAPHS, &ev);
        hipLaunchKernelGGL(k_wmax_graphs, dim3((g->n_graphs + kBlock / 64 - 1) / (kBlock / 64)), dim3(kBlock), 0,
                           g->stream, D.wmax_part, D.gblk_off, D.gblk, g->n_graphs, D.gwmax);
        timing_end(g, K_WMAX_GRAPHS, ev);
    }

    ScoreArgs<OffT> S;
    S.off = (const OffT *)D.off;
    S.col = D.col;
    S.lab = D.lab;
    S.tiles = D.stiles;
    S.hubs = D.shubs;
    S.n_tiles = g->n_stiles;
    S.n_hubs = g->n_shubs;
    S.tiles_per_xcd = (g->n_stiles + 7) / 8;
    S.hub_first = D.shub_first;
    S.hub_chunk = D.shub_chunk;
    S.n_chunks = g->n_schunks;
    S.n_chunks_lds = g->n_schunks_lds;
    S.hub_part = D.hub_part;
    S.outl = D.outl;
    S.oo = D.oo;
    S.reckey = D.reckey;
    S.recdat = D.recdat;
    S.card = D.card;
    S.prec = D.prec;
    S.hfilter = D.hfilter;
    S.oe = D.oe;
    S.n_hubs_lds = g->n_shubs_lds;
    S.plink = D.plink;
    S.av = D.av;
    S.R = D.R;
    S.raw = D.raw;
    S.gwmax = g->n_graphs > 0 ? D.gwmax : nullptr;
    S.vgraph = D.vgraph;
    S.tI = D.tI;
    S.tII = D.tII;
    S.ctr = D.ctr;
    const int n_big_hubs = g->n_shubs - g->n_shubs_lds;
    if (n_big_hubs > 0) {  // the big hubs' neighbour filters for the edge tests below
        timing_begin(g, K_HUB_FILTERS, &ev);
        hipLaunchKernelGGL(k_hub_filters<OffT>, dim3(n_big_hubs), dim3(kBlock), 0, g->stream, D.shubs,
                           g->n_shubs_lds, D.card, D.col, D.hfilter);
        timing_end(g, K_HUB_FILTERS, ev);
    }
    const unsigned long long *ictr = D.ictr;
    if (inc) {
        S.blist = nullptr;
        timing_begin(g, K_SCORE, &ev);
        hipLaunchKernelGGL(k_score_inc<OffT>, dim3(kIncGrid), dim3(kBlock), 0, g->stream, S, (const int32_t *)D.hlist,
                           (const int32_t *)D.slist, (const int32_t *)D.abin, ictr, D.hflag, g->grid_rows,
                           g->grid_score, grid_main);
        timing_end(g, K_SCORE, ev);
    } else {
        if (n_big > 0) {
            S.blist = nullptr;
            timing_begin(g, K_SCORE_HUB, &ev);
            hipLaunchKernelGGL(k_score_hub<OffT>, dim3(n_big), dim3(kBlock), 0, g->stream, S);
            timing_end(g, K_SCORE_HUB, ev);
        }
        S.blist = nullptr;
        const int grid_tiles = grid_main - g->n_schunks_lds;  // the tiles, rounded up to the 8 XCDs
        timing_begin(g, K_SCORE, &ev);
        if (g->n_schunks_lds >= kSplitHubChunks) {  // many LDS hubs: tiles with the smaller LDS form
            hipLaunchKernelGGL(k_score_lds_hubs<OffT>, dim3(g->n_schunks_lds), dim3(kBlock), 0, g->stream, S);
            if (grid_tiles > 0) hipLaunchKernelGGL(k_score<OffT>, dim3(grid_tiles), dim3(kBlock), 0, g->stream, S);
        } else if (grid_main > 0) {
            hipLaunchKernelGGL(k_score_all<OffT>, dim3(grid_main), dim3(kBlock), 0, g->stream, S);
        }
        timing_end(g, K_SCORE, ev);
    }
    if (g->n_shubs > 0) {
        timing_begin(g, K_HUB_SUM, &ev);
        hipLaunchKernelGGL(k_hub_sum, dim3((g->n_shubs + kBlock / 64 - 1) / (kBlock / 64)), dim3(kBlock), 0,
                           g->stream, D.shubs, D.shub_first, D.hub_part, g->n_shubs, D.card, D.ctr, D.gwmax,
                           D.vgraph, D.R, D.raw, D.tI, D.tII);
        timing_end(g, K_HUB_SUM, ev);
    }
    if (inc && D.n > 0)  // w_max moved: every score is rescaled from its raw sum
        hipLaunchKernelGGL(k_rescale, dim3(grid_for(D.n, kBlock, 4096)), dim3(kBlock), 0, g->stream,
                           (const unsigned long long *)&D.ictr[kIcWmaxOld], D.ctr, D.card, D.raw, D.R, (long long)D.n);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "score pass launch");
    return RS_OK;
}

rs_status launch_score_pass(rs_graph *g) {
    return replay(g, g->pass_rep, 0, [g]() {
        return g->d.off64 ? score_pass_t<long long>(g, false) : score_pass_t<int32_t>(g, false);
    });
}

rs_status launch_score_incremental(rs_graph *g) {
    return g->d.off64 ? score_pass_t<long long>(g, true) : score_pass_t<int32_t>(g, true);
}

rs_status launch_reduce_counts(rs_graph *g) {
    DeviceGraph &D = g->d;
    hipLaunchKernelGGL(k_reduce_rows, dim3(1), dim3(kBlock), 0, g->stream, D.part_rows, g->grid_rows, D.ctr);
    hipLaunchKernelGGL(k_reduce_score, dim3(1), dim3(1024), 0, g->stream, D.tI, D.tII, (long long)D.n, D.ctr);
    if (D.off64)
        hipLaunchKernelGGL(k_work_I<long long>, dim3(kWorkBlocks), dim3(kBlock), 0, g->stream,
                           (const long long *)D.off, D.col, D.card, (long long)D.n, D.wpart);
    else
        hipLaunchKernelGGL(k_work_I<int32_t>, dim3(kWorkBlocks), dim3(kBlock), 0, g->stream, (const int32_t *)D.off,
                           D.col, D.card, (long long)D.n, D.wpart);
    hipLaunchKernelGGL(k_reduce_work, dim3(1), dim3(kBlock), 0, g->stream, D.wpart, D.ctr);
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

// A vertex's ranking key is (score bits, 0xffffffff - caller id), compared
// as one 96-bit number.  Scores are >= 0; the sign bit is cleared so that a
// -0.0 could never rank first.
__device__ __forceinline__ unsigned long long score_bits(double r) {
    return dbits(r) & 0x7fffffffffffffffull;
}

// Level-0 digit: the top 16 bits of the key (score bits only).
__device__ __forceinline__ unsigned int digit0_of(double r) { return (unsigned int)(score_bits(r) >> 48); }

// Level-0 bins: a score key's sign bit is clear, so its top 16 bits take
// values below 2^15.
constexpr int kHist0Bins = 32768;

// Level-0 histogram: each block (1024 threads) counts a contiguous chunk
// (< 2^16 keys) in an LDS histogram of 16-bit counters packed two per word
// (digit 0, which holds every zero score, is counted in registers), then adds
// its non-zero bins to the global histogram, and its sums of 256 consecutive
// bins to a 256-bin coarse histogram.  Few large blocks keep the number of
// global atomics (one per non-zero bin per block) small.
constexpr int kHistThreads = 1024;
constexpr int kHistPer = 16;  // keys per thread per step, loads all in flight together

// Global slot of level-0 bin b: consecutive bins 256 bytes apart (bin
// hi * 1024 + lo at lo * 64 + hi, a bijection of [0, 65536)).  Scores share
// their leading bits, so a pass fills a few hundred neighbouring bins, and
// every workgroup adds into all of them: spread over separate cache lines,
// those atomics no longer queue on a handful of lines.
__device__ __forceinline__ unsigned int hperm(unsigned int b) { return ((b & 1023u) << 6) | (b >> 10); }

// Loads of one step of a chunk scan [lo, hi) (hi > lo): kPer keys per thread,
// kThreads apart from v0.  Indexes past the chunk load its last key, which
// the caller skips, so no branch or select touches a loaded value before its
// use (either would wait for the load).  The flags are kept one per register:
// packed bytes would wait for their loads too.
template <int kPer, int kThreads>
__device__ __forceinline__ void load_keys(const double *R, const uint8_t *alive, long long v0, long long hi,
                                          double (&r)[kPer], unsigned int (&al)[kPer]) {
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const long long v = v0 + (long long)j * kThreads;
        const long long vc = v < hi ? v : hi - 1;
        r[j] = R[vc];
        al[j] = alive[vc];
    }
}

// Block 0 also resets the selection's list counters for the collect kernel.
__global__ __launch_bounds__(kHistThreads) void k_topk_hist(const double *R, const uint8_t *alive, long long n,
                                                            long long chunk, unsigned int *hist,
                                                            unsigned int *coarse, TopkState *st) {
    __shared__ uint4 sh4[kHist0Bins / 8];
    __shared__ unsigned int s_zero[kHistThreads / 64];
    unsigned int *sh = (unsigned int *)sh4;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->n_final = 0;
        st->n_tie = 0;
        st->overflow = 0;
    }
    const long long lo = (long long)blockIdx.x * chunk;
    const long long hi = min(n, lo + chunk);
    constexpr long long kStep = (long long)kHistPer * kHistThreads;
    const int steps = (int)((hi - lo + kStep - 1) / kStep);
    if (steps <= 0) return;  // (uniform; the grid never holds an empty chunk)
    unsigned int zeros = 0;
    for (int s = 0; s < steps; ++s) {
        const long long v0 = lo + (long long)s * kStep + threadIdx.x;
        double r[kHistPer];
        unsigned int al[kHistPer];
        load_keys<kHistPer, kHistThreads>(R, alive, v0, hi, r, al);
        if (s == 0) {  // clear the LDS histogram while the first loads are in flight
            for (int i = threadIdx.x; i < kHist0Bins / 8; i += kHistThreads) sh4[i] = make_uint4(0u, 0u, 0u, 0u);
            __syncthreads();
        }
#pragma unroll
        for (int j = 0; j < kHistPer; ++j) {
            if (v0 + (long long)j * kHistThreads >= hi || !al[j]) continue;
            const unsigned int dig = digit0_of(r[j]);
            if (dig == 0u)
                ++zeros;
            else
                atomicAdd(&sh[dig >> 1], 1u << ((dig & 1u) * 16u));
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) zeros += __shfl_xor(zeros, o);
    if ((threadIdx.x & 63) == 0) s_zero[threadIdx.x >> 6] = zeros;
    __syncthreads();
    // flush: thread t takes the 16-byte words t, t + 1024, ... (8 bins each);
    // the 32 words of a coarse bin are 32 consecutive lanes of one wavefront,
    // whose sums a shuffle reduction adds.  Wavefronts whose words are all
    // zero (most: scores fill a few hundred bins) skip both.
    static_assert(kHist0Bins / 8 % kHistThreads == 0, "whole wavefronts per flush step");
    for (int i = threadIdx.x; i < kHist0Bins / 8; i += kHistThreads) {
        const uint4 x = sh4[i];
        unsigned int w[4] = {x.x, x.y, x.z, x.w};
        if (i == 0) {  // bin 0 (the low half of word 0) holds no LDS count: the zeros (< 2^16: the chunk is smaller)
            unsigned int z = 0;
            for (int q = 0; q < kHistThreads / 64; ++q) z += s_zero[q];
            w[0] += z;
        }
        unsigned int cs = 0;
#pragma unroll
        for (int t = 0; t < 4; ++t) cs += (w[t] & 0xffffu) + (w[t] >> 16);
        if (!__any(cs != 0u)) continue;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            if (w[t] & 0xffffu) atomicAdd(&hist[hperm(8 * i + 2 * t)], w[t] & 0xffffu);
            if (w[t] >> 16) atomicAdd(&hist[hperm(8 * i + 2 * t + 1)], w[t] >> 16);
        }
#pragma unroll
        for (int o = 16; o > 0; o >>= 1) cs += __shfl_xor(cs, o);
        if ((threadIdx.x & 31) == 0 && cs) atomicAdd(&coarse[i >> 5], cs);
    }
}

// The level-0 threshold, found by wavefront 0 of every block of the collect
// kernel from the finished histograms, with no barrier: lane l holds the
// positions 4l .. 4l + 3 of 256 counts in descending bin order.  wave_find
// returns, in every lane, the position where the running count reaches k,
// the count above it and the count at it (k <= the total; the caller checks).
struct Thresh0 {
    unsigned int bin;
    bool done;  // the bin is taken whole
};

__device__ __forceinline__ void wave_find(const long long (&c)[4], long long k, int &pos, long long &above,
                                          long long &at, long long &total) {
    const int lane = threadIdx.x & 63;
    const long long s = c[0] + c[1] + c[2] + c[3];
    long long incl = s;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const long long y = __shfl_up(incl, o);
        if (lane >= o) incl += y;
    }
    total = __shfl(incl, 63);
    const long long excl = incl - s;
    const unsigned long long m = __ballot(excl < k && k <= incl);
    const int L = m ? __ffsll((long long)m) - 1 : 0;
    long long a = __shfl(excl, L);
    long long q[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) q[j] = __shfl(c[j], L);
    int j = 0;
    while (j < 3 && a + q[j] < k) a += q[j++];
    pos = 4 * L + j;
    above = a;
    at = q[j];
}

// Wavefront 0 of a 1024-thread block: the coarse bin where the count from
// the top reaches k (cc: its lane's four coarse counts, loaded by the caller
// before anything else so that waiting for them waits for no later load),
// then the fine bin inside it.  Block 0 records the selection state for the
// later kernels.  Returns through LDS after one barrier of the whole block.
__device__ Thresh0 find_threshold0(const long long (&cc)[4], const unsigned int *hist, TopkState *st,
                                   long long k) {
    __shared__ Thresh0 s_res;
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        const bool publish = blockIdx.x == 0 && lane == 0;
        int pc;
        long long ac, mc, tot;
        wave_find(cc, k, pc, ac, mc, tot);
        Thresh0 res;
        if (tot < k) {  // cannot happen for k <= live keys: take all
            res.bin = 0u;
            res.done = true;
            if (publish) {
                st->k = k;
                st->digit = 0;
                st->thresh = 0;
                st->above = 0;
                st->take = 0;
                st->binsize = 0;
                st->done = 1u;
            }
        } else {
            const int c = 255 - pc;
            long long fc[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) fc[j] = hist[hperm((unsigned int)(256 * c + 255 - (4 * lane + j)))];
            int pf;
            long long af, mf, tf;
            wave_find(fc, k - ac, pf, af, mf, tf);
            const long long above = ac + af;
            res.bin = (unsigned int)(256 * c + 255 - pf);
            res.done = k == above + mf;
            if (publish) {
                st->k = k;
                st->digit = 0;
                st->thresh = res.bin;
                st->above = above;
                st->take = k - above;
                st->binsize = mf;
                st->done = res.done ? 1u : 0u;
            }
        }
        if (lane == 0) s_res = res;
    }
    __syncthreads();
    return s_res;
}

// Histogram of digit j over a key list (refinement of a large tie class).
// The refine levels are launched back to back with no host round trip: a
// level whose predecessor already took its threshold bin whole (done, at an
// earlier digit) does nothing.
__device__ __forceinline__ bool refine_finished(const TopkState *st, int level) {
    return st->done != 0u && (int)st->digit < level;
}

__global__ __launch_bounds__(kBlock) void k_list_hist(const TopkKey *list, const unsigned long long *count, int j,
                                                      const TopkState *st, unsigned int *hist) {
    __shared__ unsigned int s_d, s_c;  // the workgroup's aggregated digit and its count
    if (refine_finished(st, j)) return;
    const long long n = (long long)*count;
    if (threadIdx.x == 0) {
        s_d = 0xffffffffu;
        s_c = 0u;
    }
    __syncthreads();
    // keys of one wavefront that share a digit (common: a class of equal
    // scores shares every score digit, and ids share their high digits) are
    // added at once, into the workgroup's counter when the digit is the
    // workgroup's, so a class of equal keys costs one global atomic per
    // workgroup
    for (long long base = (long long)blockIdx.x * kBlock; base < n; base += (long long)gridDim.x * kBlock) {
        const long long i = base + threadIdx.x;
        const bool act = i < n;
        const unsigned int d = act ? key_digit(list[i], j) : 0u;
        const int lane = threadIdx.x & 63;
        unsigned long long pend = __ballot(act);
        // up to four digits shared by several lanes are added by one lane
        // each; the lanes left over add their own
        for (int r = 0; r < 4 && pend; ++r) {
            const int leader = __ffsll((long long)pend) - 1;
            const unsigned int dl = (unsigned int)__shfl((int)d, leader);
            const unsigned long long mm = __ballot(act && d == dl);
            if (lane == leader) {
                const unsigned int prev = atomicCAS(&s_d, 0xffffffffu, dl);
                if (prev == 0xffffffffu || prev == dl)
                    atomicAdd(&s_c, (unsigned int)__popcll(mm));
                else
                    atomicAdd(&hist[dl], (unsigned int)__popcll(mm));
            }
            pend &= ~mm;
        }
        if ((pend >> lane) & 1ull) atomicAdd(&hist[d], 1u);
    }
    __syncthreads();
    if (threadIdx.x == 0 && s_c) atomicAdd(&hist[s_d], s_c);
}

// One block of 1024 threads: find the threshold digit of the current level,
// record it, and clear the histogram for the next use.
__global__ __launch_bounds__(1024) void k_topk_find(unsigned int *hist, TopkState *st, int level) {
    __shared__ long long s_scan[1024];
    __shared__ long long s_total;
    if (refine_finished(st, level)) return;  // (uniform; the histogram is still clear)
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

// Level-0 collect: keys above the threshold bin go to the final list, keys in
// it to the tie list.  Each block (1024 threads) issues its first loads, finds
// the threshold from the histograms while they are in flight, scans one
// contiguous chunk and stages its keys in LDS, then reserves room in each
// list with one atomic (keys beyond the staging capacity are reserved one by
// one).  The histograms are cleared by the ranking kernel that follows.
constexpr int kCollThreads = 1024;
constexpr int kCollPer = 8;       // keys per thread per step, loads all in flight together
constexpr int kCollStage = 2048;  // staged keys per list and block
__global__ __launch_bounds__(kCollThreads) void k_topk_collect(const double *R, const int32_t *new2old,
                                                               const uint8_t *alive, long long n, long long chunk,
                                                               long long k, const unsigned int *hist,
                                                               const unsigned int *coarse, TopkState *st,
                                                               TopkKey *fin, TopkKey *tie) {
    __shared__ TopkKey sf[kCollStage], stl[kCollStage];
    __shared__ unsigned int s_nf, s_nt;
    __shared__ unsigned long long s_bf, s_bt;
    if (threadIdx.x == 0) {
        s_nf = 0u;
        s_nt = 0u;
    }
    const long long lo = (long long)blockIdx.x * chunk;
    const long long hi = min(n, lo + chunk);
    constexpr long long kStep = (long long)kCollPer * kCollThreads;
    const int steps = (int)((hi - lo + kStep - 1) / kStep);
    if (steps <= 0) return;  // (uniform; the grid never holds an empty chunk, and block 0 starts at key 0)
    // the coarse counts first (wavefront 0 searches them; every lane loads
    // its four, no branch), then the first step's keys
    long long cc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) cc[j] = (long long)coarse[255 - (4 * (threadIdx.x & 63) + j)];
    double r[kCollPer];
    unsigned int al[kCollPer];
    load_keys<kCollPer, kCollThreads>(R, alive, lo + threadIdx.x, hi, r, al);
    __builtin_amdgcn_sched_barrier(0);  // no use of the loaded keys moves above the search
    const Thresh0 t0 = find_threshold0(cc, hist, st, k);
    const unsigned int th = t0.bin;
    const bool done = t0.done;
    for (int s = 0;;) {
        const long long v0 = lo + (long long)s * kStep + threadIdx.x;
#pragma unroll
        for (int j = 0; j < kCollPer; ++j) {
            if (v0 + (long long)j * kCollThreads >= hi || !al[j]) continue;
            const unsigned int dig = digit0_of(r[j]);
            const bool f = dig > th || (dig == th && done);
            const bool t = dig == th && !done;
            if (!f && !t) continue;
            const long long v = v0 + (long long)j * kCollThreads;
            TopkKey key;
            key.hi = score_bits(r[j]);
            key.lo = 0xffffffffu - (unsigned int)new2old[v];
            key.v = (int)v;
            const unsigned int i = atomicAdd(f ? &s_nf : &s_nt, 1u);
            if (i < (unsigned int)kCollStage)
                (f ? sf : stl)[i] = key;
            else if (f)
                fin[atomicAdd(&st->n_final, 1ull)] = key;
            else
                tie[atomicAdd(&st->n_tie, 1ull)] = key;
        }
        if (++s >= steps) break;
        load_keys<kCollPer, kCollThreads>(R, alive, lo + (long long)s * kStep + threadIdx.x, hi, r, al);
    }
    __syncthreads();
    const unsigned int cf = min(s_nf, (unsigned int)kCollStage), ct = min(s_nt, (unsigned int)kCollStage);
    if (threadIdx.x == 0) {
        if (cf) s_bf = atomicAdd(&st->n_final, (unsigned long long)cf);
        if (ct) s_bt = atomicAdd(&st->n_tie, (unsigned long long)ct);
    }
    __syncthreads();
    for (unsigned int i = threadIdx.x; i < cf; i += kCollThreads) fin[s_bf + i] = sf[i];
    for (unsigned int i = threadIdx.x; i < ct; i += kCollThreads) tie[s_bt + i] = stl[i];
}

__global__ __launch_bounds__(kBlock) void k_list_collect(const TopkKey *list, const unsigned long long *count,
                                                         int level, TopkState *st, TopkKey *fin, TopkKey *tie,
                                                         unsigned long long *tie_count) {
    __shared__ unsigned int s_cnt[kBlock / 64];
    __shared__ unsigned long long s_base;
    if (refine_finished(st, level)) return;
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

// ------------------------------------------------------------ rank by counting
// Ranking of a list of unique keys (the caller id is part of the key): a
// key's rank is the number of keys above it.  A workgroup of 1024 threads
// takes 64 keys (one per lane) and its 16 wavefronts each count over every
// 16th key of the list, staged in LDS tiles that every lane of a wavefront
// reads at the same place (broadcast); the 16 counts are summed.  Sixteen
// wavefronts per group keep enough of them on every CU to hide the LDS
// latency of the comparisons.
constexpr int kCountKeys = 64;
constexpr int kCountThreads = 1024;
constexpr int kCountSubs = kCountThreads / 64;
constexpr int kCountTile = 2048;
constexpr int kRankMax = 65536;  // longest list ranked here (final lists beyond: k_final_rank)

// 1 if the key (hi, lo) ranks above `me`, both halves compared without a
// branch: a short-circuit test waits for the score half's LDS read before
// issuing the id half's, which costs more than the extra read in the
// latency-bound ranking of a few thousand candidates (k_topk_rank).  The long
// lists of k_count_rank, bound by LDS issue instead, keep the short circuit.
__device__ __forceinline__ int key_above(unsigned long long hi, unsigned int lo, const TopkKey &me) {
    return (int)((hi > me.hi) | ((hi == me.hi) & (lo > me.lo)));
}

// The list a rank pass works on, and whether it is needed: the tie class of
// the threshold bin (mode 0, skipped when the bin was taken whole or is too
// large), or the final list of keff keys (mode 1, skipped while the list is
// incomplete).
__device__ __forceinline__ long long rank_count(const TopkState *st, int mode, long long keff) {
    if (mode == 0) {
        const long long n = (long long)st->n_tie;
        return (st->done || n > kTieCap) ? -1 : n;
    }
    const long long have = (long long)st->n_final + (st->done ? 0 : st->take);
    return (st->overflow || have != keff) ? -1 : keff;
}

// Mode 0: a tie key of rank r < take goes to the final list after the keys
// above the bin (a class too large to rank here is flagged for refinement
// digit by digit); mode 1: the key of rank r is the r-th output.
__global__ __launch_bounds__(kCountThreads) void k_count_rank(const TopkKey *list, TopkState *st, int mode,
                                                              long long keff, TopkKey *fin, const double *R,
                                                              const int32_t *new2old, int32_t *out_ids,
                                                              double *out_sc) {
    __shared__ unsigned long long s_hi[kCountTile];
    __shared__ unsigned int s_lo[kCountTile];
    __shared__ int s_part[kCountSubs][kCountKeys];
    const long long n = rank_count(st, mode, keff);
    if (mode == 0 && n < 0 && !st->done && blockIdx.x == 0 && threadIdx.x == 0) st->overflow = 1u;
    if (n < 0) return;
    const int lane = threadIdx.x & 63, sub = threadIdx.x >> 6;
    for (long long base = (long long)blockIdx.x * kCountKeys; base < n; base += (long long)gridDim.x * kCountKeys) {
        const long long i = base + lane;
        TopkKey me;
        me.hi = 0;
        me.lo = 0;
        me.v = -1;
        if (i < n) me = list[i];
        int cnt = 0;
        for (long long t0 = 0; t0 < n; t0 += kCountTile) {
            const int lim = (int)min((long long)kCountTile, n - t0);
            __syncthreads();  // the previous tile (and group) is done with LDS
            for (int j = threadIdx.x; j < lim; j += kCountThreads) {
                const TopkKey x = list[t0 + j];
                s_hi[j] = x.hi;
                s_lo[j] = x.lo;
            }
            __syncthreads();
#pragma unroll 8
            for (int j = sub; j < lim; j += kCountSubs)
                cnt += (s_hi[j] > me.hi || (s_hi[j] == me.hi && s_lo[j] > me.lo)) ? 1 : 0;
        }
        s_part[sub][lane] = cnt;
        __syncthreads();
        if (sub == 0 && i < n) {
            long long rank = 0;
#pragma unroll
            for (int q = 0; q < kCountSubs; ++q) rank += s_part[q][lane];
            if (mode == 0) {
                if (rank < st->take) fin[(long long)st->n_final + rank] = me;
            } else {
                out_ids[rank] = new2old[me.v];
                out_sc[rank] = R[me.v];
            }
        }
    }
}

// Common case: the final list and the threshold bin's keys together, at most
// `cap` candidates (the grid's 64 keys per workgroup), ordered by counting in
// the same layout as k_count_rank.  The final list's keys all lie above the
// bin's and keys are unique, so a candidate's place among all candidates is
// its place in the top-k; places below keff are written as ids and scores,
// recovered from the key (key = (score bits, 0xffffffff - caller id), scores
// >= +0), into the compact output block.  No selection inside the bin is
// needed.  flag = 1 when ranked here, 0 when the general path must run.
__global__ __launch_bounds__(kCountThreads) void k_topk_rank(const TopkState *st, const TopkKey *fin,
                                                             const TopkKey *tie, long long keff, long long cap,
                                                             int32_t *out_ids, double *out_sc, unsigned int *flag,
                                                             unsigned int *hist, unsigned int *coarse) {
    __shared__ unsigned long long s_hi[kCountTile];
    __shared__ unsigned int s_lo[kCountTile];
    __shared__ int s_part[kCountSubs][kCountKeys];
    // the level-0 histograms are no longer read: clear them for the next
    // call (and for the refinement levels of the general path)
    for (long long i = (long long)blockIdx.x * kCountThreads + threadIdx.x; i < kTopkBins / 4;
         i += (long long)gridDim.x * kCountThreads)
        ((uint4 *)hist)[i] = make_uint4(0u, 0u, 0u, 0u);
    if (blockIdx.x == 0 && threadIdx.x < 256) coarse[threadIdx.x] = 0u;
    const long long nf = (long long)st->n_final;
    const long long n = nf + (st->done ? 0 : (long long)st->n_tie);
    const bool ok = n <= cap && n >= keff;
    if (blockIdx.x == 0 && threadIdx.x == 0) *flag = ok ? 1u : 0u;
    const long long base = (long long)blockIdx.x * kCountKeys;
    if (!ok || base >= n) return;  // uniform per workgroup
    const int lane = threadIdx.x & 63, sub = threadIdx.x >> 6;
    const long long i = base + lane;
    TopkKey me;
    me.hi = 0;
    me.lo = 0;
    me.v = -1;
    if (i < n) me = i < nf ? fin[i] : tie[i - nf];
    int cnt = 0;
    for (long long t0 = 0; t0 < n; t0 += kCountTile) {
        const int lim = (int)min((long long)kCountTile, n - t0);
        if (t0) __syncthreads();  // the previous tile is done with LDS
        for (int j = threadIdx.x; j < lim; j += kCountThreads) {
            const long long q = t0 + j;
            const TopkKey x = q < nf ? fin[q] : tie[q - nf];
            s_hi[j] = x.hi;
            s_lo[j] = x.lo;
        }
        __syncthreads();
#pragma unroll 8
        for (int j = sub; j < lim; j += kCountSubs) cnt += key_above(s_hi[j], s_lo[j], me);
    }
    s_part[sub][lane] = cnt;
    __syncthreads();
    if (sub == 0 && i < n) {
        long long rank = 0;
#pragma unroll
        for (int q = 0; q < kCountSubs; ++q) rank += s_part[q][lane];
        if (rank < keff) {
            out_ids[rank] = (int32_t)(0xffffffffu - me.lo);
            out_sc[rank] = __longlong_as_double((long long)me.hi);
        }
    }
}

// Candidates the common path ranks at most: the kSmallCap floor, or twice the
// requested count (the bin holding the k-th key rarely holds as many keys as
// lie above it), in whole workgroups.  Counting costs the square of the
// candidates, so beyond kUnionMax the general path (the threshold bin ranked
// alone, then the final list) is cheaper: 0, and the ranking kernel runs as
// one workgroup that only clears the histograms and sends the host there.
constexpr long long kUnionMax = 20480;
static long long rank_cap(long long keff) {
    long long cap = std::max<long long>(kSmallCap, 2 * keff);
    cap = (cap + kCountKeys - 1) / kCountKeys * kCountKeys;
    return cap <= kUnionMax ? cap : 0;
}

static rs_status final_order(rs_graph *g, long long keff) {
    DeviceGraph &D = g->d;
    hipEvent_t ev;
    timing_begin(g, K_TOPK_RANK, &ev);
    if (keff <= kSortCap) {
        hipLaunchKernelGGL(k_final_sort, dim3(1), dim3(1024), 0, g->stream, D.tfinal, keff, D.tstate, D.R,
                           D.new2old, D.tout_ids, D.tout_sc);
    } else if (keff <= kRankMax) {
        hipLaunchKernelGGL(k_count_rank, dim3((int)((keff + kCountKeys - 1) / kCountKeys)), dim3(kCountThreads), 0,
                           g->stream, (const TopkKey *)D.tfinal, D.tstate, 1, keff, (TopkKey *)nullptr, D.R,
                           D.new2old, D.tout_ids, D.tout_sc);
    } else {
        hipLaunchKernelGGL(k_final_rank, dim3(grid_for(keff, kBlock, 4096)), dim3(kBlock), 0, g->stream, D.tfinal,
                           keff, D.tstate, D.R, D.new2old, D.tout_ids, D.tout_sc);
    }
    timing_end(g, K_TOPK_RANK, ev);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? RS_OK : hip_fail(e, "top-k order launch");
}

static hipError_t copy_out(rs_graph *g, long long keff, int32_t *ids, double *scores) {
    hipError_t e = hipMemcpyAsync(ids, g->d.tout_ids, 4 * (size_t)keff, hipMemcpyDeviceToHost, g->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(scores, g->d.tout_sc, 8 * (size_t)keff, hipMemcpyDeviceToHost, g->stream);
    return e;
}

// The common path of top-k: the histogram, the collect (each block finds the
// threshold itself), and the ranking of the candidates by counting across
// workgroups into a compact device block [flag | ids | scores], copied once
// into pinned host memory.
static rs_status topk_common(rs_graph *g, long long keff) {
    DeviceGraph &D = g->d;
    hipEvent_t ev;
    long long chunk = (D.n + 63) / 64;  // about 64 blocks, each < 2^16 keys
    if (chunk < 16384) chunk = 16384;
    if (chunk > kHistChunk) chunk = kHistChunk;
    const int grid_h = (int)((D.n + chunk - 1) / chunk);
    timing_begin(g, K_TOPK_HIST, &ev);
    hipLaunchKernelGGL(k_topk_hist, dim3(grid_h), dim3(kHistThreads), 0, g->stream, D.R, D.alive, D.n, chunk,
                       D.thist, D.thist_c, D.tstate);
    timing_end(g, K_TOPK_HIST, ev);
    timing_begin(g, K_TOPK_COLLECT, &ev);
    long long cchunk = (D.n + 255) / 256;  // 64 to 256 blocks
    if (cchunk < 16384) cchunk = 16384;
    hipLaunchKernelGGL(k_topk_collect, dim3((int)((D.n + cchunk - 1) / cchunk)), dim3(kCollThreads), 0, g->stream,
                       D.R, D.new2old, D.alive, D.n, cchunk, keff, D.thist, D.thist_c, D.tstate, D.tfinal, D.ttie);
    timing_end(g, K_TOPK_COLLECT, ev);
    const size_t sc_off = 16 + ((4 * (size_t)keff + 7) & ~(size_t)7);
    char *dblk = D.tblk;
    const long long cap = rank_cap(keff);
    timing_begin(g, K_TOPK_RANK, &ev);
    hipLaunchKernelGGL(k_topk_rank, dim3((int)std::max<long long>(cap / kCountKeys, 1)), dim3(kCountThreads), 0,
                       g->stream, D.tstate, D.tfinal, D.ttie, keff, cap, (int32_t *)(dblk + 16),
                       (double *)(dblk + sc_off), (unsigned int *)dblk, D.thist, D.thist_c);
    timing_end(g, K_TOPK_RANK, ev);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(g->hpin, dblk, sc_off + 8 * (size_t)keff, hipMemcpyDeviceToHost, g->stream);
    return e == hipSuccess ? RS_OK : hip_fail(e, "top-k");
}

rs_status launch_topk(rs_graph *g, int64_t k, int32_t *ids, double *scores, int64_t *count) {
    DeviceGraph &D = g->d;
    const long long keff = k < g->n_alive ? k : g->n_alive;
    *count = keff;
    if (keff <= 0) return RS_OK;
    hipEvent_t ev;
    if (g->hpin_cap < keff) {
        drop_replay(g, g->topk_rep);  // it copies into the buffer being replaced
        if (g->hpin) (void)hipHostFree(g->hpin);
        g->hpin = nullptr;
        g->hpin_cap = 0;
        const hipError_t ea = hipHostMalloc(&g->hpin, 16 + 16 * (size_t)keff, hipHostMallocDefault);
        if (ea != hipSuccess) {
            g->hpin = nullptr;
            return hip_fail(ea, "pinned top-k buffer");
        }
        g->hpin_cap = keff;
    }
    const size_t sc_off = 16 + ((4 * (size_t)keff + 7) & ~(size_t)7);
    rs_status cst = replay(g, g->topk_rep, keff, [g, keff]() { return topk_common(g, keff); });
    if (cst != RS_OK) return cst;
    hipError_t e = hipStreamSynchronize(g->stream);
    if (e != hipSuccess) return hip_fail(e, "top-k");
    drain_replays(g);
    if (*(const unsigned int *)g->hpin) {
        memcpy(ids, (const char *)g->hpin + 16, 4 * (size_t)keff);
        memcpy(scores, (const char *)g->hpin + sc_off, 8 * (size_t)keff);
        return RS_OK;
    }
    TopkState st;

    // General path: rank the tie class (by counting), then order the final list.
    timing_begin(g, K_TOPK_TIE, &ev);
    static_assert(kTieCap <= kRankMax, "a rankable tie class fits the counting ranker");
    hipLaunchKernelGGL(k_count_rank, dim3(kTieCap / kCountKeys), dim3(kCountThreads), 0, g->stream,
                       (const TopkKey *)D.ttie, D.tstate, 0, 0ll, D.tfinal, D.R, D.new2old, D.tout_ids, D.tout_sc);
    timing_end(g, K_TOPK_TIE, ev);
    rs_status rs_st = final_order(g, keff);
    if (rs_st != RS_OK) return rs_st;
    e = hipMemcpyAsync(&st, D.tstate, sizeof(st), hipMemcpyDeviceToHost, g->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    if (e != hipSuccess) return hip_fail(e, "top-k state read");
    if (st.overflow) {
        // A tie class larger than the pairwise ranker: refine it digit by
        // digit.  The final list already holds the keys above the tie class.
        // All levels are enqueued at once; the lists only shrink, so the
        // tie count bounds every level's grid, and the levels after the one
        // that finishes return at once.
        unsigned long long *cnt = D.scratch_u;  // [0] current list size, [1] next list size
        TopkKey *cur = D.ttie, *nxt = D.ttie2;
        const int grid_l = grid_for((long long)st.n_tie, 16 * kBlock, 4096);
        e = hipMemcpyAsync(cnt, &D.tstate->n_tie, sizeof(unsigned long long), hipMemcpyDeviceToDevice, g->stream);
        for (int j = 1; j <= 5 && e == hipSuccess; ++j) {
            timing_begin(g, K_TOPK_FIND, &ev);
            hipLaunchKernelGGL(k_list_hist, dim3(grid_l), dim3(kBlock), 0, g->stream, cur, cnt, j, D.tstate, D.thist);
            hipLaunchKernelGGL(k_topk_find, dim3(1), dim3(1024), 0, g->stream, D.thist, D.tstate, j);
            timing_end(g, K_TOPK_FIND, ev);
            hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, g->stream, cnt + 1, 1);
            hipLaunchKernelGGL(k_list_collect, dim3(grid_l), dim3(kBlock), 0, g->stream, cur, cnt, j, D.tstate,
                               D.tfinal, nxt, cnt + 1);
            e = hipMemcpyAsync(cnt, cnt + 1, sizeof(unsigned long long), hipMemcpyDeviceToDevice, g->stream);
            TopkKey *tmp = cur;
            cur = nxt;
            nxt = tmp;
        }
        if (e == hipSuccess) e = hipMemsetAsync(&D.tstate->overflow, 0, sizeof(unsigned int), g->stream);
        if (e != hipSuccess) return hip_fail(e, "top-k refine");
        rs_st = final_order(g, keff);
        if (rs_st != RS_OK) return rs_st;
    }
    e = copy_out(g, keff, ids, scores);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    return e == hipSuccess ? RS_OK : hip_fail(e, "top-k copy");
}

// ------------------------------------------------------------ batched top-k
// Top-k of every graph of a batch (k <= kBatchK), one wavefront per graph,
// the largest graphs first: each lane keeps the k best keys of its strided
// share of the graph's vertices, sorted, in its own LDS column (k * 64 keys
// per wavefront: lanes hit distinct banks and no barrier is needed).  Keys
// below a lower bound of the graph's k-th key are dropped with a register
// compare: first the k-th largest of the lanes' maximum keys (a first pass
// over the scores; k lanes hold a key at least that large), then, as lists
// fill, the largest k-th key over the lanes whose lists are full (that lane
// alone holds k keys at least as large).  The union of the lane
// lists holds the graph's top-k, which k rounds of a wavefront maximum over
// the list heads take out in order.  Scores are loaded kTopkGU per lane at a
// time so their latencies overlap.  Keys are (score bits, 0xffffffff - the
// caller's id within its graph); ids are distinct, so no two keys tie.
constexpr int kTopkGU = 16;

__device__ __forceinline__ bool key_gt(unsigned long long ah, unsigned int al, unsigned long long bh, unsigned int bl) {
    return ah > bh || (ah == bh && al > bl);
}

// Wavefront maximum of (flag, hi, lo) keys; lanes without a key pass flag 0.
__device__ __forceinline__ void wave_max_key(bool &f, unsigned long long &h, unsigned int &l, int &who) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long oh = (unsigned long long)__shfl_xor((long long)h, o);
        const unsigned int ol = (unsigned int)__shfl_xor((int)l, o);
        const int ow = __shfl_xor(who, o);
        const bool of = __shfl_xor((int)f, o) != 0;
        if (of && (!f || key_gt(oh, ol, h, l))) {
            h = oh;
            l = ol;
            who = ow;
            f = true;
        }
    }
}

__global__ __launch_bounds__(64) void k_topk_graphs(const double *R, const int32_t *new2old, const uint8_t *alive,
                                                    const int64_t *vstart, const int32_t *gorder, int n_graphs, int k,
                                                    int32_t *ids, double *scores, int64_t *counts) {
    extern __shared__ unsigned long long topk_lds[];  // [k][64] score bits, then [k][64] low keys
    unsigned long long *lhi = topk_lds;
    unsigned int *llo = (unsigned int *)(topk_lds + 64 * k);
    const int lane = threadIdx.x;
    for (int oi = blockIdx.x; oi < n_graphs; oi += gridDim.x) {
        const int gi = gorder[oi];
        const long long v0 = vstart[gi], v1 = vstart[gi + 1];
        // first pass: each lane's largest key, then the k-th largest of those
        bool mf = false;
        unsigned long long mh = 0;
        unsigned int ml = 0;
        for (long long base = v0; base < v1; base += 64 * kTopkGU) {
#pragma unroll
            for (int j = 0; j < kTopkGU; ++j) {
                const long long v = base + 64 * j + lane;
                if (v < v1 && alive[v]) {
                    const unsigned long long h = score_bits(R[v]);
                    const unsigned int l = 0xffffffffu - (unsigned int)(new2old[v] - (int)v0);
                    if (!mf || key_gt(h, l, mh, ml)) {
                        mh = h;
                        ml = l;
                        mf = true;
                    }
                }
            }
        }
        int rank = 0, nfull = 0;
        for (int m = 0; m < 64; ++m) {
            const unsigned long long oh = (unsigned long long)__shfl((long long)mh, m);
            const unsigned int ol = (unsigned int)__shfl((int)ml, m);
            const bool of = __shfl((int)mf, m) != 0;
            nfull += of;
            rank += of && key_gt(oh, ol, mh, ml);
        }
        const unsigned long long at_k = __ballot(mf && rank == k - 1);
        const bool have_lb = nfull >= k && at_k != 0ull;  // (uniform)
        unsigned long long lbh = 0;
        unsigned int lbl = 0;
        if (have_lb) {
            const int src = __ffsll((long long)at_k) - 1;
            lbh = (unsigned long long)__shfl((long long)mh, src);
            lbl = (unsigned int)__shfl((int)ml, src);
        }
        int cnt = 0;
        unsigned long long th = 0, tl_h = 0;  // wavefront bound; this lane's k-th key
        unsigned int tl = 0, tl_l = 0;
        bool have_th = false;
        for (long long base = v0; base < v1; base += 64 * kTopkGU) {
            unsigned long long hi[kTopkGU];
            unsigned int lo[kTopkGU];
            bool ok[kTopkGU];
#pragma unroll
            for (int j = 0; j < kTopkGU; ++j) {
                const long long v = base + 64 * j + lane;
                ok[j] = v < v1;
                hi[j] = 0;
                lo[j] = 0;
                if (ok[j]) {
                    ok[j] = alive[v] != 0;
                    hi[j] = score_bits(R[v]);
                    lo[j] = 0xffffffffu - (unsigned int)(new2old[v] - (int)v0);
                }
            }
#pragma unroll
            for (int j = 0; j < kTopkGU; ++j) {
                if (!ok[j]) continue;
                if (have_lb && key_gt(lbh, lbl, hi[j], lo[j])) continue;
                if (have_th && !key_gt(hi[j], lo[j], th, tl)) continue;
                if (cnt == k && !key_gt(hi[j], lo[j], tl_h, tl_l)) continue;
                int p = cnt < k ? cnt++ : k - 1;
                while (p > 0 && key_gt(hi[j], lo[j], lhi[64 * (p - 1) + lane], llo[64 * (p - 1) + lane])) {
                    lhi[64 * p + lane] = lhi[64 * (p - 1) + lane];
                    llo[64 * p + lane] = llo[64 * (p - 1) + lane];
                    --p;
                }
                lhi[64 * p + lane] = hi[j];
                llo[64 * p + lane] = lo[j];
                if (cnt == k) {
                    tl_h = lhi[64 * (k - 1) + lane];
                    tl_l = llo[64 * (k - 1) + lane];
                }
            }
            bool f = cnt == k;
            unsigned long long h = f ? tl_h : 0ull;
            unsigned int l = f ? tl_l : 0u;
            int who = lane;
            wave_max_key(f, h, l, who);
            if (f) {
                have_th = true;
                th = h;
                tl = l;
            }
        }
        int ptr = 0, taken = 0;
        for (int r = 0; r < k; ++r) {
            bool f = ptr < cnt;
            unsigned long long hh = f ? lhi[64 * ptr + lane] : 0ull;
            unsigned int hl = f ? llo[64 * ptr + lane] : 0u;
            int who = lane;
            wave_max_key(f, hh, hl, who);
            if (!f) break;  // fewer live vertices than k (uniform across the wavefront)
            if (lane == who) ++ptr;
            if (lane == 0) {
                ids[(long long)gi * k + r] = (int32_t)(0xffffffffu - hl);
                scores[(long long)gi * k + r] = __longlong_as_double((long long)hh);
            }
            ++taken;
        }
        if (lane == 0) counts[gi] = taken;
    }
}

// Segmented form, for batches whose graphs have at most 64 segments of
// kSegKeys = 64 * kTopkGU vertices: one wavefront per segment holds its keys
// in registers (kTopkGU per lane) and takes out the segment's top-k by k
// rounds of a wavefront maximum over the lanes' best remaining keys; then one
// wavefront per graph merges the graph's segment lists (one per lane, staged
// in its LDS column) by k rounds over the list heads.  The latency of a
// graph is then that of one segment plus one merge, whatever its size.
constexpr int kSegKeys = 64 * kTopkGU;
static_assert(kSegKeys == kSegVerts, "a segment is one key per lane and register slot");

__global__ __launch_bounds__(kBlock) void k_topk_seg(const double *R, const int32_t *new2old, const uint8_t *alive,
                                                     const int64_t *vstart, const int32_t *seg_g,
                                                     const int32_t *sfirst, int n_segs, int k,
                                                     unsigned long long *c_hi, unsigned int *c_lo, int32_t *c_cnt) {
    const int seg = (int)blockIdx.x * (kBlock / 64) + (int)(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (seg >= n_segs) return;  // whole wavefronts leave; no barrier follows
    const int gi = seg_g[seg];
    const long long gv0 = vstart[gi];
    const long long s0 = gv0 + (long long)(seg - sfirst[gi]) * kSegKeys;
    const long long s1 = min(s0 + (long long)kSegKeys, (long long)vstart[gi + 1]);
    unsigned long long hi[kTopkGU];
    unsigned int lo[kTopkGU];
    unsigned int valid = 0u;
#pragma unroll
    for (int j = 0; j < kTopkGU; ++j) {
        const long long v = s0 + 64 * j + lane;
        hi[j] = 0ull;
        lo[j] = 0u;
        if (v < s1 && alive[v]) {
            hi[j] = score_bits(R[v]);
            lo[j] = 0xffffffffu - (unsigned int)(new2old[v] - (int)gv0);
            valid |= 1u << j;
        }
    }
    int r = 0;
#pragma unroll 1
    for (; r < k; ++r) {
        bool f = false;
        unsigned long long bh = 0ull;
        unsigned int bl = 0u;
        int bj = 0;
#pragma unroll
        for (int j = 0; j < kTopkGU; ++j) {
            const bool ok = ((valid >> j) & 1u) != 0u;
            const bool better = ok && (!f || key_gt(hi[j], lo[j], bh, bl));
            bh = better ? hi[j] : bh;
            bl = better ? lo[j] : bl;
            bj = better ? j : bj;
            f = f || ok;
        }
        int who = lane;
        wave_max_key(f, bh, bl, who);
        if (!f) break;  // the segment has fewer live vertices than k (uniform)
        if (lane == who) valid &= ~(1u << bj);
        if (lane == 0) {
            c_hi[(long long)seg * k + r] = bh;
            c_lo[(long long)seg * k + r] = bl;
        }
    }
    if (lane == 0) c_cnt[seg] = r;
}

__global__ __launch_bounds__(64) void k_topk_merge(const unsigned long long *c_hi, const unsigned int *c_lo,
                                                   const int32_t *c_cnt, const int32_t *sfirst, int n_graphs, int k,
                                                   int32_t *ids, double *scores, int64_t *counts) {
    extern __shared__ unsigned long long topk_lds[];  // [k][64] score bits, then [k][64] low keys
    unsigned long long *lhi = topk_lds;
    unsigned int *llo = (unsigned int *)(topk_lds + 64 * k);
    const int lane = threadIdx.x;
    for (int gi = blockIdx.x; gi < n_graphs; gi += gridDim.x) {
        const int sa = sfirst[gi], ns = sfirst[gi + 1] - sa;  // ns <= 64
        const int cnt = lane < ns ? c_cnt[sa + lane] : 0;
        for (int r = 0; r < cnt; ++r) {
            lhi[64 * r + lane] = c_hi[(long long)(sa + lane) * k + r];
            llo[64 * r + lane] = c_lo[(long long)(sa + lane) * k + r];
        }
        int ptr = 0, taken = 0;
        for (int r = 0; r < k; ++r) {
            bool f = ptr < cnt;
            unsigned long long hh = f ? lhi[64 * ptr + lane] : 0ull;
            unsigned int hl = f ? llo[64 * ptr + lane] : 0u;
            int who = lane;
            wave_max_key(f, hh, hl, who);
            if (!f) break;
            if (lane == who) ++ptr;
            if (lane == 0) {
                ids[(long long)gi * k + r] = (int32_t)(0xffffffffu - hl);
                scores[(long long)gi * k + r] = __longlong_as_double((long long)hh);
            }
            ++taken;
        }
        if (lane == 0) counts[gi] = taken;
    }
}

rs_status launch_topk_graphs(rs_graph *g, int64_t k, int32_t *d_ids, double *d_scores, int64_t *d_counts) {
    DeviceGraph &D = g->d;
    if (g->n_graphs <= 0) return RS_OK;
    hipEvent_t ev = nullptr;
    timing_begin(g, K_TOPK_GRAPHS, &ev);
    if (g->n_segs > 0) {
        hipLaunchKernelGGL(k_topk_seg, dim3((g->n_segs + kBlock / 64 - 1) / (kBlock / 64)), dim3(kBlock), 0,
                           g->stream, D.R, D.new2old, D.alive, D.vstart, D.seg_g, D.sfirst, g->n_segs, (int)k,
                           D.c_hi, D.c_lo, D.c_cnt);
        hipLaunchKernelGGL(k_topk_merge, dim3(grid_for(g->n_graphs, 1, 1 << 20)), dim3(64), (size_t)(12 * 64 * k),
                           g->stream, D.c_hi, D.c_lo, D.c_cnt, D.sfirst, g->n_graphs, (int)k, d_ids, d_scores,
                           d_counts);
    } else {
        hipLaunchKernelGGL(k_topk_graphs, dim3(grid_for(g->n_graphs, 1, 1 << 20)), dim3(64), (size_t)(12 * 64 * k),
                           g->stream, D.R, D.new2old, D.alive, D.vstart, D.gorder, g->n_graphs, (int)k, d_ids,
                           d_scores, d_counts);
    }
    timing_end(g, K_TOPK_GRAPHS, ev);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? RS_OK : hip_fail(e, "batched top-k launch");
}

// ============================================================ removals
// A removed CSR entry is marked by complementing it (~x < 0), which keeps
// every row ordered on the decoded value until the compaction below.
__device__ __forceinline__ int decode(int x) { return x < 0 ? ~x : x; }

// The out-lists that a removal must update, and the marks of the vertices
// whose rows change (bit kRowChanged).
struct OutLists {
    const int32_t *lab;
    const int64_t *oo;
    int32_t *outl;
    unsigned int *vmark;
};

// Tombstone y in out(x), if there; returns whether it was found.  Only the
// request that deleted the edge gets here, so the store does not race.
__device__ __forceinline__ bool out_drop(const OutLists &O, int x, int y) {
    const long long o0 = O.oo[x];
    const int32_t *row[1] = {O.outl + o0};
    const int d[1] = {(int)(O.oo[x + 1] - o0)};
    const int key[1] = {y};
    int k[1];
    lower_n<1, true>(row, d, key, k);
    if (k[0] >= d[0] || O.outl[o0 + k[0]] != y) return false;
    O.outl[o0 + k[0]] = ~y;
    return true;
}

// Delete the undirected edge {a, b}; the entry in the row of min(a, b) is
// the owner and decides which request wins.  Returns 1 if deleted here; nx
// and ny tell whether the rows of min(a, b) and max(a, b) were marked changed
// here first.  A deleted edge between communities also leaves the out-list
// that holds it.
template <typename OffT>
__device__ __forceinline__ int delete_edge(const OffT *off, const int32_t *deg, int32_t *col, const OutLists &O,
                                           int a, int b, bool &nx, bool &ny) {
    const int x = min(a, b), y = max(a, b);
    // y in x's row and x in y's row, searched together (entries keep their
    // places until the compaction, so the second position stays valid)
    const long long xb = (long long)off[x], yb = (long long)off[y];
    const int32_t *rows[2] = {col + xb, col + yb};
    const int ds[2] = {deg[x], deg[y]};
    const int keys[2] = {y, x};
    int k[2];
    lower_n<2, true>(rows, ds, keys, k);
    if (k[0] >= ds[0] || decode(col[xb + k[0]]) != y) return 0;
    if (atomicCAS(&col[xb + k[0]], y, ~y) != y) return 0;
    if (k[1] < ds[1] && decode(col[yb + k[1]]) == x) col[yb + k[1]] = ~x;
    nx = (atomicOr(&O.vmark[x], kRowChanged) & kRowChanged) == 0u;
    ny = (atomicOr(&O.vmark[y], kRowChanged) & kRowChanged) == 0u;
    if (O.lab[x] != O.lab[y] && !out_drop(O, x, y)) out_drop(O, y, x);
    return 1;
}

// The rows first marked changed by a wavefront's lanes, appended to the list
// of changed rows (any order; one atomic per wavefront).  All lanes call it.
__device__ __forceinline__ void append_changed(int x, bool nx, int y, bool ny, int32_t *list,
                                               unsigned long long *count) {
    const int lane = (int)__lane_id();
    const unsigned long long mx = __ballot(nx), my = __ballot(ny);
    const int tot = __popcll(mx) + __popcll(my);
    if (tot == 0) return;
    unsigned long long first = 0;
    if (lane == 0) first = atomicAdd(count, (unsigned long long)tot);
    first = __shfl(first, 0);
    const unsigned long long below = (1ull << lane) - 1ull;
    if (nx) list[first + __popcll(mx & below)] = x;
    if (ny) list[first + __popcll(mx) + __popcll(my & below)] = y;
}

template <typename OffT>
__global__ void k_remove_edges(const OffT *off, const int32_t *deg, int32_t *col, OutLists O, const int32_t *src,
                               const int32_t *dst, long long m, unsigned long long *removed, int32_t *changed,
                               unsigned long long *n_changed) {
    const int lane = (int)__lane_id();
    unsigned long long cnt = 0;
    for (long long base = (long long)blockIdx.x * blockDim.x + threadIdx.x - lane; base < m;
         base += (long long)gridDim.x * blockDim.x) {
        const long long i = base + lane;
        int a = 0, b = 0;
        bool nx = false, ny = false;
        if (i < m) {
            a = src[i];
            b = dst[i];
            if (a != b) cnt += (unsigned long long)delete_edge(off, deg, col, O, a, b, nx, ny);
        }
        append_changed(min(a, b), nx, max(a, b), ny, changed, n_changed);
    }
    for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o);
    if (lane == 0 && cnt) atomicAdd(removed, cnt);
}

// One wavefront per removed vertex: delete every incident edge, then mark the
// vertex dead.  removed[0] counts edges, removed[1] newly dead vertices.
template <typename OffT>
__global__ void k_remove_vertices(const OffT *off, const int32_t *deg, int32_t *col, OutLists O, uint8_t *alive,
                                  const int32_t *verts, long long nv, unsigned long long *removed, int32_t *changed,
                                  unsigned long long *n_changed) {
    const long long wave = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const long long nwave = ((long long)gridDim.x * blockDim.x) >> 6;
    const int lane = (int)__lane_id();
    for (long long i = wave; i < nv; i += nwave) {
        const int x = verts[i];
        const long long rb = (long long)off[x];
        const int d = deg[x];
        unsigned long long cnt = 0;
        for (int j0 = 0; j0 < d; j0 += 64) {
            const int j = j0 + lane;
            const int y = j < d ? col[rb + j] : -1;
            bool nx = false, ny = false;
            if (y >= 0) cnt += (unsigned long long)delete_edge(off, deg, col, O, x, y, nx, ny);
            append_changed(min(x, y), nx, max(x, y), ny, changed, n_changed);
        }
        for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o);
        if (lane == 0) {
            if (cnt) atomicAdd(&removed[0], cnt);
            if (alive[x]) {
                alive[x] = 0;
                atomicAdd(&removed[1], 1ull);
            }
        }
    }
}

static OutLists out_lists(rs_graph *g) {
    OutLists O;
    O.lab = g->d.lab;
    O.oo = g->d.oo;
    O.outl = g->d.outl;
    O.vmark = g->d.vmark;
    return O;
}

rs_status launch_remove_edges(rs_graph *g, const int32_t *d_src, const int32_t *d_dst, int64_t m,
                              unsigned long long *d_removed) {
    if (m <= 0) return RS_OK;
    const int grid = grid_for(m, 256, 4096);
    if (g->d.off64)
        hipLaunchKernelGGL(k_remove_edges<long long>, dim3(grid), dim3(256), 0, g->stream,
                           (const long long *)g->d.off, g->d.deg, g->d.col, out_lists(g), d_src, d_dst, (long long)m,
                           d_removed, g->d.elist, &g->d.ictr[kIcChanged]);
    else
        hipLaunchKernelGGL(k_remove_edges<int32_t>, dim3(grid), dim3(256), 0, g->stream, (const int32_t *)g->d.off,
                           g->d.deg, g->d.col, out_lists(g), d_src, d_dst, (long long)m, d_removed, g->d.elist,
                           &g->d.ictr[kIcChanged]);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? RS_OK : hip_fail(e, "remove edges launch");
}

rs_status launch_remove_vertices(rs_graph *g, const int32_t *d_verts, int64_t nv, unsigned long long *d_removed) {
    if (nv <= 0) return RS_OK;
    const int grid = grid_for(nv, 4, 4096);
    if (g->d.off64)
        hipLaunchKernelGGL(k_remove_vertices<long long>, dim3(grid), dim3(256), 0, g->stream,
                           (const long long *)g->d.off, g->d.deg, g->d.col, out_lists(g), g->d.alive, d_verts,
                           (long long)nv, d_removed, g->d.elist, &g->d.ictr[kIcChanged]);
    else
        hipLaunchKernelGGL(k_remove_vertices<int32_t>, dim3(grid), dim3(256), 0, g->stream, (const int32_t *)g->d.off,
                           g->d.deg, g->d.col, out_lists(g), g->d.alive, d_verts, (long long)nv, d_removed,
                           g->d.elist, &g->d.ictr[kIcChanged]);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? RS_OK : hip_fail(e, "remove vertices launch");
}


// ------------------------------------------------------------ incremental re-score
// After a removal batch only some results change.  With E the vertices whose
// rows changed (endpoints of removed edges), a vertex u needs a new score iff
//   u is in E, or u has a foreign neighbour in E (u's pair facts, type-I
//   weights or out-lists involve it), or u is in the community of some v in
//   E and adjacent to a foreign neighbour w of v (u's pair (u, w) sums a_v);
// rows need recomputing only for E, and links only for E's entries and the
// neighbours' links back to E.  The removal kernels list E as they mark it.
// The row tiles and hub chunks that hold changed rows or affected hubs are
// rerun whole, with the block indices of the full launch, and the affected
// tile vertices are rescored in units built for the pass; every result and
// every partial is what a full pass would give.

// Compact the listed changed rows (removed entries are complemented, < 0):
// one wavefront per row, kCompactGroups groups of 64 entries loaded at once
// (a hub's long row takes one round trip per 1,024 entries), each group
// packed by a ballot and prefix; the freed tail of the capacity is set to -1.
constexpr int kCompactGroups = 16;
template <typename OffT>
__global__ __launch_bounds__(kBlock) void k_compact_rows(const OffT *off, int32_t *deg, int32_t *col, int32_t *clab,
                                                         const int32_t *list, const unsigned long long *count) {
    const long long nl = (long long)*count;
    const int lane = threadIdx.x & 63;
    for (long long i = ((long long)blockIdx.x * kBlock + threadIdx.x) >> 6; i < nl;
         i += ((long long)gridDim.x * kBlock) >> 6) {
        const int v = list[i];
        const long long rb = (long long)off[v];
        const int d = deg[v];
        int w = 0;
        for (int j0 = 0; j0 < d; j0 += 64 * kCompactGroups) {  // groups of 64 entries loaded at once
            int x[kCompactGroups], c[kCompactGroups];
#pragma unroll
            for (int t = 0; t < kCompactGroups; ++t) {
                const int j = j0 + 64 * t + lane;
                x[t] = j < d ? col[rb + j] : -1;
                c[t] = j < d ? clab[rb + j] : -1;
            }
#pragma unroll
            for (int t = 0; t < kCompactGroups; ++t) {
                const unsigned long long m = __ballot(x[t] >= 0);
                if (x[t] >= 0) {
                    const long long to = rb + w + __popcll(m & ((1ull << lane) - 1ull));
                    col[to] = x[t];
                    clab[to] = c[t];
                }
                w += __popcll(m);
            }
        }
        for (int j = w + lane; j < d; j += 64) {
            col[rb + j] = -1;
            clab[rb + j] = -1;
        }
        if (lane == 0) deg[v] = w;
    }
}

// The listed (changed, compacted) rows cut into chunks of 64 entries, at
// least one per row: (row's list index, chunk).  One slot per wavefront in
// the chunk counter (a wavefront prefix orders its lanes' chunks).
__global__ __launch_bounds__(kBlock) void k_row_chunks(const int32_t *deg, const int32_t *list,
                                                       const unsigned long long *count, int2 *chunks,
                                                       unsigned long long *n_chunks) {
    const long long nl = (long long)*count;
    const int lane = threadIdx.x & 63;
    for (long long base = (long long)blockIdx.x * kBlock + (threadIdx.x & ~63); base < nl;
         base += (long long)gridDim.x * kBlock) {
        const long long i = base + lane;
        const int nc = i < nl ? max(1, (deg[list[i]] + 63) >> 6) : 0;
        int incl = nc;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int t = __shfl_up(incl, o);
            if (lane >= o) incl += t;
        }
        unsigned long long first = 0;
        if (lane == 63) first = atomicAdd(n_chunks, (unsigned long long)incl);
        first = __shfl(first, 63);
        for (int c = 0; c < nc; ++c) chunks[first + (incl - nc) + c] = make_int2((int)i, c);
    }
}

// The marks of the pair (x, w) of a member x of C(v) in the row of v's
// foreign neighbour w (the pair sums a_v): a score hub whose row did not
// change flags the chunk holding the pair (w's place in x's foreign list);
// any other x is affected whole.
template <typename OffT>
__device__ __forceinline__ void mark_run_member(const LinkArgs<OffT> &L, unsigned int *vmark, const int32_t *vscore,
                                                const int32_t *hub_first, uint8_t *cflag, int x, int w) {
    const int sx = vscore[x];
    if (sx < 0 && !(L.vmark[x] & kRowChanged)) {
        const int32_t *row[1] = {L.col + L.off[x]};
        const int d[1] = {L.deg[x]};
        const int key[1] = {w};
        int k[1];
        lower_n<1, false>(row, d, key, k);
        const VMeta m = L.card[x].m;
        const int kx = k[0] < m.p ? k[0] : k[0] - (m.q - m.p);
        cflag[hub_first[-1 - sx] + kx / kScoreTileP] = 1;
    } else {
        atomicOr(&vmark[x], kAffected);
    }
}

// Item g of a wavefront's flattened work: its owner lane (pre: the lanes'
// inclusive item counts, in LDS) and its index among the owner's items.
__device__ __forceinline__ int flat_owner(const int *pre, int g, int &idx) {
    int lo = 0, hi = 63;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (pre[mid] > g)
            hi = mid;
        else
            lo = mid + 1;
    }
    idx = g - (lo > 0 ? pre[lo - 1] : 0);
    return lo;
}

// Longest changed row whose triangles at a hub neighbour are listed pair by
// pair; a hub next to a longer changed row is rescored whole.
constexpr int kTriRow = 512;

// After removals, one wavefront per chunk of 64 entries of a changed
// (compacted) row v (chunks: k_row_chunks), for each entry (v, w) with w in
// another community:
// * links: v's link for the entry (the reverse entry and w's out-list), and
//   the index of the entry (v, w), which moved with v's row, in w's link
//   back to v;
// * marks: v is affected whole.  The pairs whose terms read v's row are
//   (a) (w, v) itself (w's pair facts, out-list scan, a-run),
//   (b) (w, y) for each y adjacent to both, in a third community (the
//       triangle {w, y, v} reads v's record weights),
//   (c) (x, w) for each member x of C(v) in w's row (its a-run sums a_v).
//   A tile vertex with such a pair is affected whole (its unit reruns); a
//   score hub whose own row did not change flags only the chunks holding the
//   pairs (the others keep their partials), so a changed vertex next to a
//   hub costs a few chunks, not the hub.
// The long lists of (b) and (c) are worked by the whole wavefront (items
// flattened over the lanes).  Only the kRowChanged bits, set by the
// removals before, are read.
template <typename OffT>
__global__ __launch_bounds__(kBlock) void k_mark_link(LinkArgs<OffT> L, unsigned int *vmark, const int32_t *vscore,
                                                      const int32_t *hub_first, uint8_t *cflag, const int32_t *rows,
                                                      const int2 *chunks, const unsigned long long *n_chunks) {
    __shared__ int s_pre[kBlock / 64][64];
    const long long nc = (long long)*n_chunks;
    const int lane = threadIdx.x & 63;
    int *pre = s_pre[threadIdx.x >> 6];
    for (long long q = ((long long)blockIdx.x * kBlock + threadIdx.x) >> 6; q < nc;
         q += ((long long)gridDim.x * kBlock) >> 6) {
        const int2 it = chunks[q];
        const int v = rows[it.x];
        if (it.y == 0 && lane == 0) atomicOr(&vmark[v], kAffected);
        const long long rb = (long long)L.off[v];
        const int dv = L.deg[v];
        const int cv = L.lab[v];
        const int id0 = L.cstart[cv], id1 = L.cstart[cv + 1];
        const int j = it.y * 64 + lane;
        int w = 0, cw = cv;
        if (j < dv) {
            w = L.col[rb + j];
            cw = L.lab[w];
        }
        const bool fw = j < dv && cw != cv;
        long long wb = 0;
        int dw = 0, k0 = 0, k1 = 0, wh = 0, pw = 0, qw = 0;
        bool whub = false;  // w: a score hub with its row unchanged
        if (fw) {
            wb = (long long)L.off[w];
            dw = L.deg[w];
            const int32_t *roww = L.col + wb;
            // in w's row: C(v)'s run [k[0], k[1]) and the entry (w, v) at
            // k[2]; in v's row: v's own run [k[3], k[4])
            const int32_t *rws[5] = {roww, roww, roww, L.col + rb, L.col + rb};
            const int ds[5] = {dw, dw, dw, dv, dv};
            const int keys[5] = {id0, id1, v, id0, id1};
            int k[5];
            lower_n<5, false>(rws, ds, keys, k);
            k0 = k[0];
            k1 = k[1];
            const int pv = k[3], qv = k[4], ew = k[2];
            PairLink pl;
            pl.e = wb + ew;
            pl.oo = (int)L.oo[w];
            pl.on = (int)(L.oo[w + 1] - L.oo[w]);
            L.plink[L.goff[v] + (j < pv ? j : j - (qv - pv))] = pl;
            // w's own run is its card's when w's row did not change
            const bool wch = (L.vmark[w] & kRowChanged) != 0u;
            if (wch) {
                const int32_t *rw2[2] = {roww, roww};
                const int dw2[2] = {dw, dw};
                const int kw2[2] = {L.cstart[cw], L.cstart[cw + 1]};
                int pq[2];
                lower_n<2, false>(rw2, dw2, kw2, pq);
                pw = pq[0];
                qw = pq[1];
            } else {
                const VMeta m = L.card[w].m;
                pw = m.p;
                qw = m.q;
            }
            const int kw = ew < pw ? ew : ew - (qw - pw);
            L.plink[L.goff[w] + kw].e = rb + j;
            {
                // the out-list entry of {v, w} (in the list of the lower
                // rank: load-time foreign degree, then id) gets both entries
                const long long fv = L.goff[v + 1] - L.goff[v], fw = L.goff[w + 1] - L.goff[w];
                const bool v_low = fv < fw || (fv == fw && v < w);
                const int a = v_low ? v : w, bkey = v_low ? w : v;
                const long long o0 = L.oo[a];
                const int32_t *orow[1] = {L.outl + o0};
                const int od[1] = {(int)(L.oo[a + 1] - o0)};
                const int okey[1] = {bkey};
                int ok[1];
                lower_n<1, true>(orow, od, okey, ok);
                if (ok[0] < od[0] && L.outl[o0 + ok[0]] == bkey) {
                    OutEnt e;
                    e.xy = v_low ? rb + j : wb + ew;
                    e.yx = v_low ? wb + ew : rb + j;
                    L.oe[o0 + ok[0]] = e;
                }
            }
            const int sw = vscore[w];
            whub = sw < 0 && !wch;
            if (whub) {
                wh = -1 - sw;
                cflag[hub_first[wh] + kw / kScoreTileP] = 1;  // (a)
            } else {
                atomicOr(&vmark[w], kAffected);
            }
        }
        // (c) the runs of C(v) in the foreign neighbours' rows
        {
            const int cnt = fw ? k1 - k0 : 0;
            int incl = cnt;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int y = __shfl_up(incl, o);
                if (lane >= o) incl += y;
            }
            pre[lane] = incl;
            const int total = __shfl(incl, 63);
            wave_sync();
            for (int g0 = 0; g0 < total; g0 += 64) {
                const int g = g0 + lane;
                int idx = 0, l = 0;
                if (g < total) l = flat_owner(pre, g, idx);
                const int wl = __shfl(w, l), kl = __shfl(k0, l);
                const long long wbl = ((long long)__shfl((int)(wb >> 32), l) << 32) | (unsigned int)__shfl((int)wb, l);
                if (g < total) mark_run_member(L, vmark, vscore, hub_first, cflag, L.col[wbl + kl + idx], wl);
            }
            wave_sync();
        }
        // (b) the triangles {w, y, v} at the hub neighbours w: the pairs
        // (w, y) for the foreign neighbours y of v in a third community
        const unsigned long long hubs = __ballot(whub);
        if (hubs) {
            if (dv > kTriRow) {  // too long to intersect: the hub reruns whole
                if (whub) atomicOr(&vmark[w], kAffected);
            } else {
                const int cnt = whub ? dv : 0;
                int incl = cnt;
#pragma unroll
                for (int o = 1; o < 64; o <<= 1) {
                    const int y = __shfl_up(incl, o);
                    if (lane >= o) incl += y;
                }
                pre[lane] = incl;
                const int total = __shfl(incl, 63);
                wave_sync();
                for (int g0 = 0; g0 < total; g0 += 64) {
                    const int g = g0 + lane;
                    int t = 0, l = 0;
                    if (g < total) l = flat_owner(pre, g, t);
                    const int cwl = __shfl(cw, l), hl = __shfl(wh, l), pwl = __shfl(pw, l), qwl = __shfl(qw, l),
                              dwl = __shfl(dw, l);
                    const long long wbl =
                        ((long long)__shfl((int)(wb >> 32), l) << 32) | (unsigned int)__shfl((int)wb, l);
                    if (g < total) {
                        const int y = L.col[rb + t];
                        const int cy = L.lab[y];
                        if (cy != cv && cy != cwl) {
                            const int32_t *row[1] = {L.col + wbl};
                            const int d[1] = {dwl};
                            const int key[1] = {y};
                            int k[1];
                            lower_n<1, false>(row, d, key, k);
                            if (k[0] < dwl && L.col[wbl + k[0]] == y) {
                                const int ky = k[0] < pwl ? k[0] : k[0] - (qwl - pwl);
                                cflag[hub_first[hl] + ky / kScoreTileP] = 1;
                            }
                        }
                    }
                }
                wave_sync();
            }
        }
    }
}

// Marks -> units: a changed row flags its row block; an affected hub flags
// all chunks of its score hub; an affected tile vertex is placed in abin,
// grouped by the bin of its load-time foreign degree (units of rescored
// vertices are built per pass, so scattered affected vertices do not rerun
// whole tiles).  Three steps over contiguous vertex ranges, one range per
// workgroup, so that no counter in global memory is shared: count per range
// and bin (LDS atomics), an exclusive scan of the counts bin after bin (one
// workgroup), and placement at the scanned offsets.  The scan also counts the
// affected vertices and keeps w_max before the pass; placement clears the
// marks.
__device__ __forceinline__ int score_bin(long long fgn) {
    int b = 0;
    while (b < kScoreBins - 1 && (1ll << b) < fgn) ++b;
    return b;
}

__device__ __forceinline__ void unit_range(long long n, long long &lo, long long &hi) {
    const long long per = ((n + gridDim.x - 1) / gridDim.x + 63) & ~63ll;
    lo = min(n, (long long)blockIdx.x * per);
    hi = min(n, lo + per);
}

// The marks of kMarkPer vertices of a range per thread, loaded together (a
// loop that tests each mark before loading the next waits for every load):
// slots past the range load its last mark and are skipped by the caller.
constexpr int kMarkPer = 8;
__device__ __forceinline__ void load_marks(const unsigned int *vmark, long long v0, long long hi,
                                           unsigned int (&mk)[kMarkPer]) {
#pragma unroll
    for (int j = 0; j < kMarkPer; ++j) {
        const long long v = v0 + (long long)j * kBlock;
        mk[j] = vmark[v < hi ? v : hi - 1];
    }
}

// ucnt[r * gridDim.x + range]: rows 0..kScoreBins-1 tile vertices per bin,
// row kScoreBins affected vertices.
__global__ __launch_bounds__(kBlock) void k_units_count(const unsigned int *vmark, const int32_t *vrowb,
                                                        const int32_t *vscore, const int64_t *goff, long long n,
                                                        uint8_t *rflag, uint8_t *hflag, int32_t *ucnt) {
    __shared__ int s_cnt[kUnitRows];
    if (threadIdx.x < kUnitRows) s_cnt[threadIdx.x] = 0;
    __syncthreads();
    long long lo, hi;
    unit_range(n, lo, hi);
    int aff = 0;
    for (long long v0 = lo + threadIdx.x; v0 < hi; v0 += (long long)kMarkPer * kBlock) {
        unsigned int mk[kMarkPer];
        load_marks(vmark, v0, hi, mk);
#pragma unroll
        for (int j = 0; j < kMarkPer; ++j) {
            const long long v = v0 + (long long)j * kBlock;
            const unsigned int m = mk[j];
            if (v >= hi || !m) continue;
            if (m & kRowChanged) rflag[vrowb[v]] = 1;
            if (m & kAffected) {
                ++aff;
                const int sc = vscore[v];
                if (sc >= 0)
                    atomicAdd(&s_cnt[score_bin(goff[v + 1] - goff[v])], 1);
                else
                    hflag[-1 - sc] = 1;
            }
        }
    }
    if (aff) atomicAdd(&s_cnt[kScoreBins], aff);
    __syncthreads();
    if (threadIdx.x < kUnitRows) ucnt[threadIdx.x * gridDim.x + blockIdx.x] = s_cnt[threadIdx.x];
}

// One workgroup: each bin's per-range counts become the ranges' first slots
// in abin (bins in order); bin totals, the listed total and the affected
// count go to the counters.  Thread t holds ranges 4t..4t+3 of every row
// (all loads issued at once), and one block scan serves all bins.
static_assert(kUnitGroups == 4 * kBlock, "k_units_scan holds four ranges per thread");
__global__ __launch_bounds__(kBlock) void k_units_scan(int32_t *ucnt, int groups, unsigned long long *ictr,
                                                       const DevCounters *ctr) {
    __shared__ int ws[kUnitRows][kBlock / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int j0 = 4 * threadIdx.x;
    int x[kUnitRows][4], incl[kUnitRows];
#pragma unroll
    for (int r = 0; r < kUnitRows; ++r) {
#pragma unroll
        for (int i = 0; i < 4; ++i) x[r][i] = j0 + i < groups ? ucnt[r * groups + j0 + i] : 0;
    }
#pragma unroll
    for (int r = 0; r < kUnitRows; ++r) {
        int t = x[r][0] + x[r][1] + x[r][2] + x[r][3];
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(t, o);
            if (lane >= o) t += y;
        }
        incl[r] = t;
        if (lane == 63) ws[r][wave] = t;
    }
    __syncthreads();
    int base = 0;
#pragma unroll
    for (int r = 0; r < kScoreBins; ++r) {
        int before = 0, total = 0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) {
            if (w < wave) before += ws[r][w];
            total += ws[r][w];
        }
        int pos = base + before + incl[r] - (x[r][0] + x[r][1] + x[r][2] + x[r][3]);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if (j0 + i < groups) ucnt[r * groups + j0 + i] = pos;
            pos += x[r][i];
        }
        if (threadIdx.x == 0) ictr[kIcBins + r] = (unsigned long long)total;
        base += total;
    }
    if (threadIdx.x == 0) {
        long long aff = 0;
        for (int w = 0; w < kBlock / 64; ++w) aff += ws[kScoreBins][w];
        ictr[kIcAffected] = (unsigned long long)aff;
        ictr[kIcAList] = (unsigned long long)base;
        ictr[kIcWmaxOld] = ctr->wmax_bits;
    }
}

// Each range's affected tile vertices to their bins' slots (any order inside
// a range and bin; a vertex's score does not depend on its unit); the marks
// are cleared.
__global__ __launch_bounds__(kBlock) void k_units_place(unsigned int *vmark, const int32_t *vscore,
                                                        const int64_t *goff, long long n, const int32_t *ucnt,
                                                        int32_t *abin) {
    __shared__ int s_cur[kScoreBins];
    if (threadIdx.x < kScoreBins) s_cur[threadIdx.x] = ucnt[threadIdx.x * gridDim.x + blockIdx.x];
    __syncthreads();
    long long lo, hi;
    unit_range(n, lo, hi);
    for (long long v0 = lo + threadIdx.x; v0 < hi; v0 += (long long)kMarkPer * kBlock) {
        unsigned int mk[kMarkPer];
        load_marks(vmark, v0, hi, mk);
#pragma unroll
        for (int j = 0; j < kMarkPer; ++j) {
            const long long v = v0 + (long long)j * kBlock;
            const unsigned int m = mk[j];
            if (v >= hi || !m) continue;
            vmark[v] = 0u;
            if ((m & kAffected) && vscore[v] >= 0)
                abin[atomicAdd(&s_cur[score_bin(goff[v + 1] - goff[v])], 1)] = (int32_t)v;
        }
    }
}

// Append the lanes' values whose pred holds to list (one atomic per
// wavefront; all lanes call it).
__device__ __forceinline__ void wave_append(bool pred, int val, int32_t *list, unsigned long long *count) {
    const int lane = threadIdx.x & 63;
    const unsigned long long m = __ballot(pred);
    if (!m) return;
    unsigned long long first = 0;
    if (lane == 0) first = atomicAdd(count, (unsigned long long)__popcll(m));
    first = __shfl(first, 0);
    if (pred) list[first + __popcll(m & ((1ull << lane) - 1ull))] = val;
}

// Flags -> the incremental launches' lists (indices of the full launches):
// the flagged row blocks, and the score-hub chunks to rerun, each chunk of a
// hub flagged whole and each chunk flagged by itself (the main list takes
// the LDS-hub chunks, the big list the others).  Clears the row and chunk
// flags; the hub flags are cleared by the score pass that follows.
__global__ __launch_bounds__(kBlock) void k_unit_lists(uint8_t *rflag, int n_rows, uint8_t *cflag,
                                                       const uint8_t *hflag, const int2 *hub_chunk, int n_chunks,
                                                       int n_chunks_lds, int32_t *rlist, int32_t *slist,
                                                       int32_t *hlist, unsigned long long *ictr) {
    const int lane = threadIdx.x & 63;
    const int top = max(n_rows, n_chunks);
    for (int base = blockIdx.x * kBlock + (threadIdx.x & ~63); base < top; base += gridDim.x * kBlock) {
        const int i = base + lane;
        const bool r = i < n_rows && rflag[i] != 0;
        if (r) rflag[i] = 0;
        bool c = false;
        if (i < n_chunks) {
            const bool own = cflag[i] != 0;
            if (own) cflag[i] = 0;
            c = own || hflag[hub_chunk[i].x] != 0;
        }
        wave_append(r, i, rlist, &ictr[kIcRows]);
        wave_append(c && i < n_chunks_lds, i, slist, &ictr[kIcMain]);
        wave_append(c && i >= n_chunks_lds, i - n_chunks_lds, hlist, &ictr[kIcBig]);
    }
}

template <typename OffT>
static rs_status incremental_marks_t(rs_graph *g) {
    DeviceGraph &D = g->d;
    if (D.n == 0) return RS_OK;
    const OffT *off = (const OffT *)D.off;
    const int gn = grid_for(D.n, kBlock, 1024);
    hipLaunchKernelGGL(k_compact_rows<OffT>, dim3(gn), dim3(kBlock), 0, g->stream, off, D.deg, D.col, D.clab,
                       D.elist, &D.ictr[kIcChanged]);
    hipLaunchKernelGGL(k_row_chunks, dim3(gn), dim3(kBlock), 0, g->stream, D.deg, D.elist, &D.ictr[kIcChanged],
                       D.echunk, &D.ictr[kIcChunks]);
    hipLaunchKernelGGL(k_mark_link<OffT>, dim3(gn), dim3(kBlock), 0, g->stream, link_args<OffT>(g), D.vmark,
                       (const int32_t *)D.vscore, (const int32_t *)D.shub_first, D.cflag, D.elist, D.echunk,
                       &D.ictr[kIcChunks]);
    const int ug = grid_for(D.n, kBlock, kUnitGroups);
    hipLaunchKernelGGL(k_units_count, dim3(ug), dim3(kBlock), 0, g->stream, D.vmark, D.vrowb, D.vscore, D.goff,
                       (long long)D.n, D.rflag, D.hflag, D.ucnt);
    hipLaunchKernelGGL(k_units_scan, dim3(1), dim3(kBlock), 0, g->stream, D.ucnt, ug, D.ictr, D.ctr);
    hipLaunchKernelGGL(k_units_place, dim3(ug), dim3(kBlock), 0, g->stream, D.vmark, D.vscore, D.goff,
                       (long long)D.n, D.ucnt, D.abin);
    const int top = std::max(g->grid_rows, g->n_schunks);
    hipLaunchKernelGGL(k_unit_lists, dim3(grid_for(top, kBlock, 4096)), dim3(kBlock), 0, g->stream, D.rflag,
                       g->grid_rows, D.cflag, (const uint8_t *)D.hflag, (const int2 *)D.shub_chunk, g->n_schunks,
                       g->n_schunks_lds, D.rlist, D.slist, D.hlist, D.ictr);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? RS_OK : hip_fail(e, "incremental marks launch");
}

rs_status launch_incremental_marks(rs_graph *g) {
    return g->d.off64 ? incremental_marks_t<long long>(g) : incremental_marks_t<int32_t>(g);
}

// ============================================================ readers
__global__ void k_gather_scores(const double *R, const int32_t *new2old, const DevCounters *ctr,
                                const unsigned long long *gwmax, const int32_t *vgraph, long long n, int raw,
                                double *out) {
    const double wmax = bitsd(ctr->wmax_bits);
    for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (long long)gridDim.x * blockDim.x)
        out[new2old[v]] = raw ? R[v] * (gwmax ? bitsd(gwmax[vgraph[v]]) : wmax) : R[v];
}

rs_status launch_gather_scores(rs_graph *g, double *d_out, int raw) {
    const int grid = grid_for(g->d.n, 256, 8192);
    hipLaunchKernelGGL(k_gather_scores, dim3(grid), dim3(256), 0, g->stream, g->d.R, g->d.new2old, g->d.ctr,
                       g->n_graphs > 0 ? g->d.gwmax : nullptr, g->d.vgraph, (long long)g->d.n, raw, d_out);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? RS_OK : hip_fail(e, "gather launch");
}

rs_status launch_zero_u64(rs_graph *g, unsigned long long *p, int count) {
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, g->stream, p, count);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? RS_OK : hip_fail(e, "zero launch");
}

// ============================================================ reachable communities
// For the absolute AWCC of the robustness experiments (Section VII-B): the
// connected components of the current graph by hooking and pointer jumping
// (labels only decrease along parent links, so no cycle can form), then, for
// each source, the communities of the other members of its component.
__global__ __launch_bounds__(kBlock) void k_cc_init(int32_t *comp, long long n) {
    for (long long v = (long long)blockIdx.x * kBlock + threadIdx.x; v < n; v += (long long)gridDim.x * kBlock)
        comp[v] = (int32_t)v;
}

// Hook the root of the larger label under the smaller one across every live
// edge; comp[] holds roots here (the jump kernel ran before).
template <typename OffT>
__global__ __launch_bounds__(kBlock) void k_cc_hook(const OffT *off, const int32_t *deg, const int32_t *col,
                                                    int32_t *comp, long long n, unsigned int *changed) {
    for (long long v = (long long)blockIdx.x * kBlock + threadIdx.x; v < n; v += (long long)gridDim.x * kBlock) {
        const long long rb = (long long)off[v];
        const int d = deg[v];
        bool hooked = false;
        for (int j = 0; j < d; ++j) {
            const int32_t x = col[rb + j];
            if (x < 0) continue;  // (rows are compacted after removals; defensive)
            const int32_t cu = comp[x], cv = comp[v];
            if (cu < cv) {
                atomicMin(&comp[cv], cu);
                hooked = true;
            }
        }
        if (hooked) *changed = 1u;
    }
}

// Point every vertex at its root.
__global__ __launch_bounds__(kBlock) void k_cc_jump(int32_t *comp, long long n) {
    for (long long v = (long long)blockIdx.x * kBlock + threadIdx.x; v < n; v += (long long)gridDim.x * kBlock) {
        int32_t c = comp[v];
        while (comp[c] != c) c = comp[c];
        comp[v] = c;
    }
}

// bits[i][c] = 1 when some vertex other than source i lies in source i's
// component and belongs to community c.
__global__ __launch_bounds__(kBlock) void k_reach_bits(const int32_t *comp, const int32_t *lab, long long n,
                                                       const int32_t *src, int ns, int words, unsigned int *bits) {
    __shared__ int32_t s_c[kMaxReachSources], s_v[kMaxReachSources];
    for (int i = threadIdx.x; i < ns; i += kBlock) {
        s_v[i] = src[i];
        s_c[i] = comp[src[i]];
    }
    __syncthreads();
    for (long long v = (long long)blockIdx.x * kBlock + threadIdx.x; v < n; v += (long long)gridDim.x * kBlock) {
        const int32_t c = comp[v];
        const int32_t l = lab[v];
        const unsigned int bit = 1u << (l & 31);
        for (int i = 0; i < ns; ++i)
            if (s_c[i] == c && s_v[i] != (int32_t)v) {
                unsigned int *w = &bits[(long long)i * words + (l >> 5)];
                if (!(__hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & bit))
                    atomicOr(w, bit);  // most members find their community's bit already set
            }
    }
}

__global__ void k_zero_u32(unsigned int *p, long long count) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (long long)gridDim.x * blockDim.x)
        p[i] = 0u;
}

template <typename OffT>
static rs_status components_t(rs_graph *g, int32_t *comp, unsigned int *d_changed, unsigned int *h_changed) {
    DeviceGraph &D = g->d;
    const int grid = grid_for(D.n, kBlock, 8192);
    hipLaunchKernelGGL(k_cc_init, dim3(grid), dim3(kBlock), 0, g->stream, comp, (long long)D.n);
    // rounds go in groups of four between host checks; the flag tells
    // whether the group's last round hooked anything (rounds after
    // convergence change nothing)
    for (int it = 0; it < 512; it += 4) {
        for (int q = 0; q < 4; ++q) {
            hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, g->stream, d_changed, 1ll);
            hipLaunchKernelGGL(k_cc_hook<OffT>, dim3(grid), dim3(kBlock), 0, g->stream, (const OffT *)D.off, D.deg,
                               D.col, comp, (long long)D.n, d_changed);
            hipLaunchKernelGGL(k_cc_jump, dim3(grid), dim3(kBlock), 0, g->stream, comp, (long long)D.n);
        }
        hipError_t e = hipMemcpyAsync(h_changed, d_changed, sizeof(unsigned int), hipMemcpyDeviceToHost, g->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
        if (e != hipSuccess) return hip_fail(e, "components");
        if (*h_changed == 0u) return RS_OK;
    }
    return fail(RS_ERR_STATE, "components did not converge");
}

rs_status launch_reach(rs_graph *g, const int32_t *d_src, int ns, int32_t *comp, unsigned int *bits, int words,
                       unsigned int *d_changed, unsigned int *h_changed) {
    DeviceGraph &D = g->d;
    rs_status st = D.off64 ? components_t<long long>(g, comp, d_changed, h_changed)
                           : components_t<int32_t>(g, comp, d_changed, h_changed);
    if (st != RS_OK) return st;
    const int grid = grid_for(D.n, kBlock, 8192);
    hipLaunchKernelGGL(k_zero_u32, dim3(grid_for((long long)ns * words, kBlock, 1024)), dim3(kBlock), 0, g->stream,
                       bits, (long long)ns * words);
    hipLaunchKernelGGL(k_reach_bits, dim3(grid), dim3(kBlock), 0, g->stream, comp, D.lab, (long long)D.n, d_src, ns,
                       words, bits);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? RS_OK : hip_fail(e, "reach launch");
}

// ------------------------------------------------------------ static scratch
// Device memory of rs_reachable_communities_static, the entry point for
// callers that cannot allocate: one array per device (it lives as long as
// the process), shared by every call on that device.  Host code never passes
// the array's name to a kernel -- that is a host-side stand-in, not a device
// address -- but the per-device address taken once with
// hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices] = {};

rs_status static_scratch(int device, void **out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return fail(RS_ERR_ARG, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e == hipSuccess && cur != device) e = hipSetDevice(device);
        void *p = nullptr;
        if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur >= 0 && cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return RS_OK;
}

// counts[i] = the bits set in source i's community bitmap (one wavefront per
// source).
__global__ __launch_bounds__(kBlock) void k_reach_counts(const unsigned int *bits, int ns, int words,
                                                         long long *counts) {
    const int i = (int)blockIdx.x * (kBlock / 64) + (int)(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= ns) return;
    long long c = 0;
    for (int w = lane; w < words; w += 64) c += __popc(bits[(long long)i * words + w]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
    if (lane == 0) counts[i] = c;
}

rs_status launch_reach_counts(rs_graph *g, const unsigned int *bits, int ns, int words, long long *d_counts) {
    hipLaunchKernelGGL(k_reach_counts, dim3((ns + kBlock / 64 - 1) / (kBlock / 64)), dim3(kBlock), 0, g->stream,
                       bits, ns, words, d_counts);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? RS_OK : hip_fail(e, "reach counts launch");
}

}  // namespace rs
