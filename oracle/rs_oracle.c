/*
 * rs_oracle.c -- plain CPU oracle for the robust-spanner (RS) scoring pass.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the GPU library is checked against.  Only the tests, the
 * smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product path never does.  It shares no code, header or helper with the HIP
 * library.
 *
 * What it computes (paper: "A Parallel Algorithm for Finding Robust Spanners
 * in Large Social Networks", Sections II-IV):
 *   - G undirected simple graph, C(u) one non-overlapping community per vertex
 *     (Section II).  A border vertex has a neighbour in another community.
 *   - L(u,v): frequencies of the communities of N(v), excluding C(u)
 *     (Eq. cont).  H(L) = -sum p log2 p with p = f / sum(f) (Eq. entropy; the
 *     log base is 2, fixed by the worked weight example of Section VI-B).
 *   - w_v(u) = H(L(u,v)) * |L(u,v)| (Eq. weight); by Lemma 1 it depends only
 *     on v and C(u), so it is stored per (v, community).
 *   - R(u) = 1/(d(u)(d(u)-1)) * sum over ordered (w in N(u), v in N(w)) with
 *     the triad indicator of Eq. RSI of cbrt(w_v(u) w_w(v) w_w(u)), each term
 *     divided by w_max, the largest weight of E_b (Algorithm 1, Steps 2-3).
 *   - Top-K by (R descending, vertex id ascending) (Algorithm 1, Step 4).
 *
 * Readings taken where the paper is silent or inconsistent (each is listed in
 * the design notes of the repository):
 *   A3  |L| counts the distinct communities of N(v) other than the reference
 *       one (Eq. weight), also when the reference community is absent from
 *       N(v); ALG2_LITERAL switches to Algorithm 2's uniform L_all - 1.
 *   A4  0 log 0 = 0; an empty L has H = 0 and weight 0.
 *   A5  w_max = max over border v of w_v(c), c in {C(v)} U {communities of
 *       N(v)}, and 0 if there is none (then every R is 0).
 *   A7  a closed triangle u-w-v with C(u) = C(v) != C(w) counts once, as a
 *       type-II triad.
 *   A8  ordered pairs (w, v): a type-I triangle counts twice at u.
 *   A9  v != u.
 *   A10 both C(w) != C(u) and C(w) != C(v) are required.
 *   A11 R(u) = 0 when d(u) < 2.
 *   A12 d(u) is the degree in G.
 *   A14 ties in top-K are broken by the smaller vertex id.
 *   A15 fp64 everywhere, libm log2 and cbrt, integer counts in int64.
 *
 * Built with: gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared -lm
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define RSO_OK 0
#define RSO_ERR_ARG 1
#define RSO_ERR_GRAPH 2
#define RSO_ERR_NOMEM 4
#define RSO_ERR_INTERNAL 7

#define RSO_ALG2_LITERAL 1u

/* ---------------------------------------------------------------- O0 ---- */
/* A simple undirected graph (Section II): offsets start at 0 and never
 * decrease, ids in range, each row strictly ascending (no duplicates), no
 * self-loops, every (u,v) has its (v,u), labels non-negative. */
static int has_edge(const int64_t *off, const int32_t *col, int64_t u, int32_t v)
{
    int64_t lo = off[u], hi = off[u + 1];
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (col[mid] < v)
            lo = mid + 1;
        else if (col[mid] > v)
            hi = mid;
        else
            return 1;
    }
    return 0;
}

int rso_validate(int64_t n, const int64_t *off, const int32_t *col, const int32_t *lab)
{
    if (n < 0 || !off)
        return RSO_ERR_ARG;
    if (off[0] != 0)
        return RSO_ERR_GRAPH;
    for (int64_t u = 0; u < n; ++u)
        if (off[u + 1] < off[u])
            return RSO_ERR_GRAPH;
    for (int64_t u = 0; u < n; ++u) {
        if (lab[u] < 0)
            return RSO_ERR_GRAPH;
        for (int64_t e = off[u]; e < off[u + 1]; ++e) {
            int32_t v = col[e];
            if (v < 0 || v >= n || v == u)
                return RSO_ERR_GRAPH;
            if (e > off[u] && col[e - 1] >= v)
                return RSO_ERR_GRAPH;
            if (!has_edge(off, col, v, (int32_t)u))
                return RSO_ERR_GRAPH;
        }
    }
    return RSO_OK;
}

/* ------------------------------------------------------------ O4 (Eq) ---- */
/* Weight of a neighbourhood toward a reference community (Eq. entropy and
 * Eq. weight): L = {(c, f) : c != ref, f > 0}; Y = sum f;
 * H = -sum (f/Y) log2(f/Y) summed directly; w = H * |L|. */
double rso_weight(int64_t k, const int32_t *comms, const int64_t *counts, int32_t ref,
                  unsigned flags)
{
    double Y = 0.0;
    int64_t L = 0, all = 0;
    for (int64_t i = 0; i < k; ++i) {
        if (counts[i] <= 0)
            continue;
        ++all;
        if (comms[i] == ref)
            continue;
        Y += (double)counts[i];
        ++L;
    }
    if (L == 0)
        return 0.0;
    double H = 0.0;
    for (int64_t i = 0; i < k; ++i) {
        if (counts[i] <= 0 || comms[i] == ref)
            continue;
        double p = (double)counts[i] / Y;
        H -= p * log2(p);
    }
    if (flags & RSO_ALG2_LITERAL)
        return H * (double)(all - 1);
    return H * (double)L;
}

/* One weighted triad of Eq. RSI: the cube root of the product of its three
 * weights, w_v(u) * w_w(v) * w_w(u). */
double rso_triad_term(double w_vu, double w_wv, double w_wu)
{
    return cbrt(w_vu * w_wv * w_wu);
}

/* Eq. RSI's reduction over the weighted triads of one vertex of degree d,
 * with Algorithm 1's division of every term by w_max (A11: 0 when d < 2). */
double rso_rsi_from_terms(int64_t d, int64_t nterms, const double *w_vu, const double *w_wv,
                          const double *w_wu, double omega_max)
{
    if (d < 2 || !(omega_max > 0.0))
        return 0.0;
    double r = 0.0;
    for (int64_t i = 0; i < nterms; ++i)
        r += rso_triad_term(w_vu[i], w_wv[i], w_wu[i]) / omega_max;
    return r / (double)(d * (d - 1));
}

/* --------------------------------------------------------- O3 rows ---- */
typedef struct {
    int64_t n;
    const int64_t *off;
    const int32_t *col;
    const int32_t *lab;
    /* rows of (community, count, weight) sorted by community, stored at off[v] */
    int32_t *hc;
    int64_t *hf;
    double *hw;
    int32_t *ell;
    double *w_own;
    unsigned flags;
    int err;
} oracle_t;

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* f_v(c) for every community c of N(v): sort the neighbour labels and count
 * runs (Eq. cont with no exclusion; L(u,v) is formed per reference below). */
static void build_row(oracle_t *o, int64_t v, int32_t *tmp)
{
    int64_t b = o->off[v], d = o->off[v + 1] - b;
    for (int64_t i = 0; i < d; ++i)
        tmp[i] = o->lab[o->col[b + i]];
    qsort(tmp, (size_t)d, sizeof(int32_t), cmp_i32);
    int64_t k = 0;
    for (int64_t i = 0; i < d; ++i) {
        if (k > 0 && o->hc[b + k - 1] == tmp[i]) {
            o->hf[b + k - 1] += 1;
        } else {
            o->hc[b + k] = tmp[i];
            o->hf[b + k] = 1;
            ++k;
        }
    }
    o->ell[v] = (int32_t)k;
}

/* w_v(c) for every c in K_v = {C(v)} U {communities of N(v)}. */
static void row_weights(oracle_t *o, int64_t v)
{
    int64_t b = o->off[v];
    int64_t k = o->ell[v];
    for (int64_t i = 0; i < k; ++i)
        o->hw[b + i] = rso_weight(k, o->hc + b, o->hf + b, o->hc[b + i], o->flags);
    o->w_own[v] = rso_weight(k, o->hc + b, o->hf + b, o->lab[v], o->flags);
}

/* w_x(c), Lemma 1 storage: own community from w_own, others from x's row. */
static double lookup(oracle_t *o, int64_t x, int32_t c)
{
    if (c == o->lab[x])
        return o->w_own[x];
    int64_t lo = o->off[x], hi = o->off[x] + o->ell[x];
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (o->hc[mid] < c)
            lo = mid + 1;
        else if (o->hc[mid] > c)
            hi = mid;
        else
            return o->hw[mid];
    }
    o->err = 1; /* every weight read by Eq. RSI lies in K_x */
    return NAN;
}

/* ----------------------------------------------------- O6 indicator ---- */
/* The triad indicator of Eq. RSI for the ordered pair (w, v) at u, with
 * w in N(u) and v in N(w):
 *   0  not counted
 *   1  type-I: closed triad over three distinct communities
 *   2  type-II, open: (u,v) not an edge, C(v) = C(u) (augmented edge)
 *   3  type-II, closed (reading A7)
 * Conditions: v != u (A9); C(w) != C(u) and C(w) != C(v) (A10). */
static int classify(oracle_t *o, int64_t u, int64_t w, int64_t v)
{
    const int32_t *lab = o->lab;
    if (v == u || w == u || v == w)
        return 0;
    if (lab[w] == lab[u] || lab[w] == lab[v])
        return 0;
    int closed = has_edge(o->off, o->col, u, (int32_t)v);
    if (lab[v] == lab[u])
        return closed ? 3 : 2;
    return closed ? 1 : 0;
}

/* ------------------------------------------------------------- API ---- */
static int prepare(oracle_t *o, int64_t n, const int64_t *off, const int32_t *col,
                   const int32_t *lab, unsigned flags, int nthreads)
{
    memset(o, 0, sizeof(*o));
    o->n = n;
    o->off = off;
    o->col = col;
    o->lab = lab;
    o->flags = flags;
    int64_t nnz = off[n];
    size_t cap = (size_t)(nnz > 0 ? nnz : 1);
    o->hc = (int32_t *)malloc(cap * sizeof(int32_t));
    o->hf = (int64_t *)malloc(cap * sizeof(int64_t));
    o->hw = (double *)malloc(cap * sizeof(double));
    o->ell = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    o->w_own = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    if (!o->hc || !o->hf || !o->hw || !o->ell || !o->w_own)
        return RSO_ERR_NOMEM;
    int64_t dmax = 0;
    for (int64_t v = 0; v < n; ++v)
        if (off[v + 1] - off[v] > dmax)
            dmax = off[v + 1] - off[v];
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    int fail = 0;
#pragma omp parallel
    {
        int32_t *tmp = (int32_t *)malloc((size_t)(dmax > 0 ? dmax : 1) * sizeof(int32_t));
        if (!tmp) {
#pragma omp atomic write
            fail = 1;
        } else {
#pragma omp for schedule(dynamic, 256)
            for (int64_t v = 0; v < n; ++v) {
                build_row(o, v, tmp);
                row_weights(o, v);
            }
        }
        free(tmp);
    }
    return fail ? RSO_ERR_NOMEM : RSO_OK;
}

static void release(oracle_t *o)
{
    free(o->hc);
    free(o->hf);
    free(o->hw);
    free(o->ell);
    free(o->w_own);
}

static int is_border(oracle_t *o, int64_t v)
{
    for (int64_t e = o->off[v]; e < o->off[v + 1]; ++e)
        if (o->lab[o->col[e]] != o->lab[v])
            return 1;
    return 0;
}

/* O5: w_max over E_b (reading A5). */
static double omega_max_of(oracle_t *o)
{
    double m = 0.0;
    for (int64_t v = 0; v < o->n; ++v) {
        if (!is_border(o, v))
            continue;
        if (o->w_own[v] > m)
            m = o->w_own[v];
        for (int64_t i = 0; i < o->ell[v]; ++i)
            if (o->hw[o->off[v] + i] > m)
                m = o->hw[o->off[v] + i];
    }
    return m;
}

/*
 * Full pass.  subset == NULL scores every vertex; otherwise only the listed
 * vertices get R / raw / tI / tII (arrays are still indexed by vertex id).
 * Optional outputs may be NULL.  hist_* receive the rows compacted in vertex
 * order (hist_off[n+1] is filled first; hist_comm/cnt/w need off[n] room).
 */
int rso_score(int64_t n, const int64_t *off, const int32_t *col, const int32_t *lab,
              const int64_t *subset, int64_t n_subset, unsigned flags, int nthreads,
              double *R, double *raw, uint8_t *border, int32_t *ell, int32_t *dprime,
              int64_t *tI, int64_t *tII, int64_t *tII_closed, double *w_own,
              int64_t *hist_off, int32_t *hist_comm, int64_t *hist_cnt, double *hist_w,
              double *omega_max_out, int64_t *n_border_out, int64_t *m_inter_out)
{
    if (n < 0 || !off || (n > 0 && (!col || !lab)))
        return RSO_ERR_ARG;
    oracle_t o;
    int rc = prepare(&o, n, off, col, lab, flags, nthreads);
    if (rc != RSO_OK) {
        release(&o);
        return rc;
    }
    double omax = omega_max_of(&o);
    int64_t nb = 0, mx2 = 0;
    for (int64_t v = 0; v < n; ++v) {
        int64_t fo = 0;
        for (int64_t e = off[v]; e < off[v + 1]; ++e)
            if (lab[col[e]] == lab[v])
                ++fo;
        int64_t dp = (off[v + 1] - off[v]) - fo;
        if (border)
            border[v] = dp > 0;
        if (dprime)
            dprime[v] = (int32_t)dp;
        if (ell)
            ell[v] = o.ell[v];
        if (w_own)
            w_own[v] = o.w_own[v];
        nb += dp > 0;
        mx2 += dp;
    }
    if (hist_off) {
        hist_off[0] = 0;
        for (int64_t v = 0; v < n; ++v)
            hist_off[v + 1] = hist_off[v] + o.ell[v];
        for (int64_t v = 0; v < n; ++v)
            for (int64_t i = 0; i < o.ell[v]; ++i) {
                if (hist_comm)
                    hist_comm[hist_off[v] + i] = o.hc[off[v] + i];
                if (hist_cnt)
                    hist_cnt[hist_off[v] + i] = o.hf[off[v] + i];
                if (hist_w)
                    hist_w[hist_off[v] + i] = o.hw[off[v] + i];
            }
    }
    int64_t cnt = subset ? n_subset : n;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t s = 0; s < cnt; ++s) {
        int64_t u = subset ? subset[s] : s;
        if (u < 0 || u >= n)
            continue;
        double sum_norm = 0.0, sum_raw = 0.0;
        int64_t c1 = 0, c2 = 0, c2c = 0;
        for (int64_t e = off[u]; e < off[u + 1]; ++e) {
            int64_t w = col[e];
            if (lab[w] == lab[u])
                continue;
            for (int64_t f = off[w]; f < off[w + 1]; ++f) {
                int64_t v = col[f];
                int kind = classify(&o, u, w, v);
                if (kind == 0)
                    continue;
                if (kind == 1)
                    ++c1;
                else
                    ++c2;
                if (kind == 3)
                    ++c2c;
                double t = rso_triad_term(lookup(&o, v, lab[u]), lookup(&o, w, lab[v]),
                                          lookup(&o, w, lab[u]));
                sum_raw += t;
                if (omax > 0.0)
                    sum_norm += t / omax;
            }
        }
        int64_t d = off[u + 1] - off[u];
        double dd = (double)(d * (d - 1));
        if (R)
            R[u] = (d >= 2 && omax > 0.0) ? sum_norm / dd : 0.0;
        if (raw)
            raw[u] = (d >= 2) ? sum_raw / dd : 0.0;
        if (tI)
            tI[u] = c1;
        if (tII)
            tII[u] = c2;
        if (tII_closed)
            tII_closed[u] = c2c;
    }
    if (omega_max_out)
        *omega_max_out = omax;
    if (n_border_out)
        *n_border_out = nb;
    if (m_inter_out)
        *m_inter_out = mx2 / 2;
    rc = o.err ? RSO_ERR_INTERNAL : RSO_OK;
    release(&o);
    return rc;
}

/* Every triad counted at u: (w, v, kind) with kind as in classify().
 * Returns the number of triads (only the first cap are written). */
int64_t rso_triads(int64_t n, const int64_t *off, const int32_t *col, const int32_t *lab,
                   int64_t u, int64_t cap, int64_t *out_w, int64_t *out_v, int32_t *out_kind)
{
    if (u < 0 || u >= n)
        return -1;
    oracle_t o;
    memset(&o, 0, sizeof(o));
    o.n = n;
    o.off = off;
    o.col = col;
    o.lab = lab;
    int64_t k = 0;
    for (int64_t e = off[u]; e < off[u + 1]; ++e) {
        int64_t w = col[e];
        for (int64_t f = off[w]; f < off[w + 1]; ++f) {
            int64_t v = col[f];
            int kind = classify(&o, u, w, v);
            if (!kind)
                continue;
            if (k < cap) {
                out_w[k] = w;
                out_v[k] = v;
                out_kind[k] = kind;
            }
            ++k;
        }
    }
    return k;
}

/* ----------------------------------------------------------- O8 top-K ---- */
static const double *g_sort_key;
static int cmp_rank(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    double rx = g_sort_key[x], ry = g_sort_key[y];
    if (rx > ry)
        return -1;
    if (rx < ry)
        return 1;
    return (x > y) - (x < y);
}

/* K highest scores, ties by smaller id; removed vertices (alive[v] == 0)
 * are skipped.  Returns min(K, number of live vertices) in *count. */
int rso_topk(int64_t n, const double *R, const uint8_t *alive, int64_t K, int32_t *ids,
             double *scores, int64_t *count)
{
    if (n < 0 || K < 0 || !count)
        return RSO_ERR_ARG;
    int64_t *idx = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!idx)
        return RSO_ERR_NOMEM;
    int64_t m = 0;
    for (int64_t v = 0; v < n; ++v)
        if (!alive || alive[v])
            idx[m++] = v;
    g_sort_key = R;
    qsort(idx, (size_t)m, sizeof(int64_t), cmp_rank);
    int64_t k = K < m ? K : m;
    for (int64_t i = 0; i < k; ++i) {
        ids[i] = (int32_t)idx[i];
        scores[i] = R[idx[i]];
    }
    *count = k;
    free(idx);
    return RSO_OK;
}
