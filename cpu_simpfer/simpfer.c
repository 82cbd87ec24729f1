/*
 * Simpfer on the CPU, as the paper designs it: the pre-processing of
 * Algorithm 1, the block-wise online query of Algorithm 3 with its linear
 * scan (Algorithm 2), and OpenMP over the blocks (Sections 4.3 and 5.6).  It
 * is a comparison baseline (the paper's design on the host), shares no code
 * with the GPU library or with the oracle, and is never called by the
 * library.
 *
 * Arithmetic: every inner product is taken in double precision, summed in
 * coordinate order, on the float32 inputs.  The tests of Lemma 1, Lemma 3
 * and Corollary 2 compare such values (the stored lower bounds are inner
 * products of real items), so with the strict "no" tests below the answers
 * are exact.  The tests that use Cauchy-Schwarz (Lemma 2, Lemma 3 and
 * Corollary 1) multiply computed norms, whose product may fall an ulp or so
 * below the computed inner product it bounds; those bounds are raised by
 * the factor CS_SLACK so that they stay upper bounds.
 *
 * Readings where the algorithms are silent or would be wrong with ties:
 *  - ties go to q: u is a member iff fewer than k items p have
 *    u.p > u.q, so every "no" test is strict (Lemmas 1 and 3, Corollary 2);
 *  - the linear scan starts with tau = -infinity (a threshold of 0 would
 *    ignore items with 0 >= u.p > u.q), and a scan that reaches the end of
 *    P answers yes;
 *  - the last, partial block is kept, and a block's lower bounds start at
 *    +infinity;
 *  - P' is the first lb_items items in norm order (default 2 k_max), the
 *    block size b defaults to ceil(log2 n), and equal norms keep the input
 *    order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* |f - |u||p|| rounding: norms and inner products carry relative errors of
 * about d * 2^-53 each; 2^-40 covers d up to 2^10 with room to spare. */
#define CS_SLACK (1.0 + 0x1p-40)

typedef struct {
    int64_t n, m;
    int32_t d, kmax, lb_items, b;
    int64_t nblocks;
    float *Qs;        /* [n][d] users in descending norm order */
    float *Ps;        /* [m][d] items in descending norm order */
    int32_t *qid;     /* original id of sorted user i */
    double *nu;       /* |u_i| */
    double *np;       /* |p_j| */
    double *L;        /* [n][kmax] L_i^j (descending), -inf beyond |P'| */
    double *LB;       /* [nblocks][kmax] block minima (Equation (1)) */
} cs_index;

typedef struct {
    int64_t blocks, blocks_pruned, users, lemma1_no, lemma2_yes, scans, scan_items, results;
} cs_stats;

static double cs_dot(const float *x, const float *y, int32_t d)
{
    double s = 0.0;
    for (int32_t i = 0; i < d; ++i)
        s += (double)x[i] * (double)y[i];
    return s;
}

static const double *g_key;
static int cs_cmp(const void *a, const void *b)
{
    int32_t i = *(const int32_t *)a, j = *(const int32_t *)b;
    if (g_key[i] > g_key[j]) return -1;
    if (g_key[i] < g_key[j]) return 1;
    return (i > j) - (i < j);
}

/* Sorted copy of X (descending norm, ties by input order), norms, order. */
static void cs_sort(const float *X, int64_t rows, int32_t d, float *Xs, double *nrm, int32_t *ord)
{
    double *sq = (double *)malloc(sizeof(double) * (size_t)(rows > 0 ? rows : 1));
    for (int64_t r = 0; r < rows; ++r) {
        sq[r] = cs_dot(X + r * d, X + r * d, d);
        ord[r] = (int32_t)r;
    }
    g_key = sq;
    qsort(ord, (size_t)rows, sizeof(int32_t), cs_cmp);
    g_key = NULL;
    for (int64_t r = 0; r < rows; ++r) {
        memcpy(Xs + r * d, X + (int64_t)ord[r] * d, sizeof(float) * (size_t)d);
        nrm[r] = sqrt(sq[ord[r]]);
    }
    free(sq);
}

/* Lower-bound arrays over P' and block minima for the current kmax. */
static void cs_bounds(cs_index *x)
{
    const int64_t pp = x->lb_items < x->m ? x->lb_items : x->m;
    free(x->L);
    free(x->LB);
    x->L = (double *)malloc(sizeof(double) * (size_t)(x->n * x->kmax + 1));
    x->nblocks = (x->n + x->b - 1) / x->b;
    x->LB = (double *)malloc(sizeof(double) * (size_t)(x->nblocks * x->kmax + 1));
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < x->n; ++i) {
        /* R = the kmax items of P' with the largest u_i.p, kept descending */
        double *top = x->L + i * x->kmax;
        int32_t len = 0;
        for (int64_t t = 0; t < pp; ++t) {
            const double v = cs_dot(x->Qs + i * x->d, x->Ps + t * x->d, x->d);
            if (len == x->kmax && !(v > top[len - 1]))
                continue;
            int32_t j = len < x->kmax ? len++ : len - 1;
            while (j > 0 && top[j - 1] < v) {
                top[j] = top[j - 1];
                --j;
            }
            top[j] = v;
        }
        for (int32_t j = len; j < x->kmax; ++j)
            top[j] = -INFINITY;
    }
    for (int64_t B = 0; B < x->nblocks; ++B)
        for (int32_t j = 0; j < x->kmax; ++j) {
            double lo = INFINITY;
            for (int64_t i = B * x->b; i < (B + 1) * x->b && i < x->n; ++i)
                if (x->L[i * x->kmax + j] < lo)
                    lo = x->L[i * x->kmax + j];
            x->LB[B * x->kmax + j] = lo;
        }
}

/* Algorithm 1.  lb_items <= 0: 2 kmax; b <= 0: ceil(log2 n). */
cs_index *cs_build(const float *Q, int64_t n, const float *P, int64_t m, int32_t d,
                   int32_t kmax, int32_t lb_items, int32_t b)
{
    if (n < 0 || m < 0 || d < 1 || kmax < 1)
        return NULL;
    cs_index *x = (cs_index *)calloc(1, sizeof(cs_index));
    x->n = n;
    x->m = m;
    x->d = d;
    x->kmax = kmax;
    x->lb_items = lb_items > 0 ? lb_items : 2 * kmax;
    if (b <= 0) {
        b = 1;
        while (((int64_t)1 << b) < n)
            ++b;
    }
    x->b = b;
    x->Qs = (float *)malloc(sizeof(float) * (size_t)(n * d + 1));
    x->Ps = (float *)malloc(sizeof(float) * (size_t)(m * d + 1));
    x->qid = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
    x->nu = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    x->np = (double *)malloc(sizeof(double) * (size_t)(m + 1));
    int32_t *pid = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m + 1));
    cs_sort(Q, n, d, x->Qs, x->nu, x->qid);
    cs_sort(P, m, d, x->Ps, x->np, pid);
    free(pid);
    cs_bounds(x);
    return x;
}

/* k > kmax: the paper rebuilds the lower-bound arrays (Section 4.1). */
void cs_rebuild(cs_index *x, int32_t kmax)
{
    x->kmax = kmax;
    if (x->lb_items < kmax)
        x->lb_items = kmax;
    cs_bounds(x);
}

void cs_free(cs_index *x)
{
    if (!x)
        return;
    free(x->Qs);
    free(x->Ps);
    free(x->qid);
    free(x->nu);
    free(x->np);
    free(x->L);
    free(x->LB);
    free(x);
}

/* Algorithm 2 for sorted user i: 1 = yes, 0 = no. */
static int cs_linear_scan(const cs_index *x, int64_t i, const float *q, double uq, int32_t k,
                          double *I, int64_t *items)
{
    (void)q;
    const float *u = x->Qs + i * x->d;
    const double nu = x->nu[i] * CS_SLACK;
    /* I: the largest of {u.q} and the inner products seen, descending;
     * tau = its k-th entry once it holds k + 1 (-inf before) */
    int32_t len = 1;
    I[0] = uq;
    double tau = -INFINITY;
    for (int64_t j = 0; j < x->m; ++j) {
        if (uq >= nu * x->np[j])           /* Corollary 1 */
            return 1;
        const double g = cs_dot(u, x->Ps + j * x->d, x->d);
        ++*items;
        if (g > tau) {
            int32_t t = len++;
            while (t > 0 && I[t - 1] < g) {
                I[t] = I[t - 1];
                --t;
            }
            I[t] = g;
            if (len > k) {
                len = k;                   /* drop the (k+1)-th */
                tau = I[k - 1];
            }
            if (tau > uq)                  /* Corollary 2 */
                return 0;
        }
    }
    return 1;                              /* fewer than k items beat q */
}

static int cs_cmp_i32(const void *a, const void *b)
{
    int32_t i = *(const int32_t *)a, j = *(const int32_t *)b;
    return (i > j) - (i < j);
}

/* Algorithm 3.  ids receives the members' original ids, ascending; returns
 * their number, or -1 when k < 1 or kmax < k <= m (call cs_rebuild first).
 * k > m: fewer than k items exist, every user is a member. */
int64_t cs_query(const cs_index *x, const float *q, int32_t k, int32_t *ids, cs_stats *st)
{
    memset(st, 0, sizeof(*st));
    if (k < 1 || (k > x->kmax && k <= x->m))
        return -1;
    if (k > x->m) {
        for (int64_t i = 0; i < x->n; ++i)
            ids[i] = (int32_t)i;
        st->results = x->n;
        return x->n;
    }
    if (x->n == 0)
        return 0;
    const double nq = sqrt(cs_dot(q, q, x->d)) * CS_SLACK;
    const double pk = x->np[k - 1] * CS_SLACK;  /* |p_k| of Lemma 2 (k <= m here) */
    int64_t count = 0;
    cs_stats tot = {0};
#pragma omp parallel
    {
        cs_stats s = {0};
        double *I = (double *)malloc(sizeof(double) * (size_t)(k + 2));
#pragma omp for schedule(dynamic, 4)
        for (int64_t B = 0; B < x->nblocks; ++B) {
            const int64_t first = B * x->b;
            ++s.blocks;
            if (!(x->nu[first] * nq >= x->LB[B * x->kmax + (k - 1)])) {   /* Lemma 3 (strict) */
                ++s.blocks_pruned;
                continue;
            }
            for (int64_t i = first; i < first + x->b && i < x->n; ++i) {
                ++s.users;
                const double g = cs_dot(x->Qs + i * x->d, q, x->d);
                if (g < x->L[i * x->kmax + (k - 1)]) {                    /* Lemma 1 (strict) */
                    ++s.lemma1_no;
                    continue;
                }
                int yes;
                if (g >= x->nu[i] * pk) {                                  /* Lemma 2 */
                    ++s.lemma2_yes;
                    yes = 1;
                } else {
                    ++s.scans;
                    yes = cs_linear_scan(x, i, q, g, k, I, &s.scan_items);
                }
                if (yes) {
                    int64_t at;
#pragma omp atomic capture
                    at = count++;
                    ids[at] = x->qid[i];
                }
            }
        }
        free(I);
#pragma omp critical
        {
            tot.blocks += s.blocks;
            tot.blocks_pruned += s.blocks_pruned;
            tot.users += s.users;
            tot.lemma1_no += s.lemma1_no;
            tot.lemma2_yes += s.lemma2_yes;
            tot.scans += s.scans;
            tot.scan_items += s.scan_items;
        }
    }
    qsort(ids, (size_t)count, sizeof(int32_t), cs_cmp_i32);
    tot.results = count;
    *st = tot;
    return count;
}

int32_t cs_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void cs_set_threads(int32_t t)
{
#ifdef _OPENMP
    if (t > 0)
        omp_set_num_threads(t);
#else
    (void)t;
#endif
}
