/*
 * Reverse k-MIPS CPU oracle.  TEST INFRASTRUCTURE ONLY: nothing on the
 * product path may link, load or call this file; only the test-suite, the
 * smoke check and the benchmark's CPU-baseline leg do.
 *
 * Plain, slow and obviously correct.  Every floating-point value is computed
 * in IEEE double precision from the float32 inputs widened to double.
 *
 * The inner product used everywhere is
 *     f(x, y) = sum_{i=0}^{d-1} x_i * y_i,
 * accumulated in double, sequentially in i = 0 .. d-1.  Each float32*float32
 * product is exact in double (48 significant bits <= 53), so the value does
 * not depend on whether the compiler contracts the multiply-add; only the
 * summation order matters, and that order is fixed here.
 *
 * Problem (Definition 2 of the paper, Section 2): user u belongs to the
 * reverse k-MIPS result of query q iff q is among the k best items of u over
 * P u {q}.  Ties go to q: u is a member iff fewer than k items p of P have
 * f(p, u) > f(q, u).  A duplicate of q inside P therefore never counts
 * against q (the paper allows q in P, Section 2 and Example 1).
 *
 * OpenMP is used only to run independent users on separate threads; it does
 * not change any arithmetic.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* Inner product f(x, y): double accumulation in index order (see header). */
double ork_dot(const float *x, const float *y, int32_t d)
{
    double s = 0.0;
    for (int32_t i = 0; i < d; ++i)
        s += (double)x[i] * (double)y[i];
    return s;
}

/* Definition 2, literally: count the items that beat q for each user.
 * The count stops as soon as it reaches k, because membership only asks
 * whether the count is below k.  member[u] = 1 for members, else 0.
 * Returns the number of members. */
int64_t ork_brute(const float *Q, int64_t n, const float *P, int64_t m,
                  int32_t d, const float *q, int32_t k, uint8_t *member)
{
    int64_t total = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : total)
    for (int64_t u = 0; u < n; ++u) {
        const float *uu = Q + u * (int64_t)d;
        double fq = ork_dot(q, uu, d);
        int64_t beats = 0;
        for (int64_t p = 0; p < m && beats < k; ++p)
            if (ork_dot(P + p * (int64_t)d, uu, d) > fq)
                ++beats;
        member[u] = (uint8_t)(beats < k);
        total += member[u];
    }
    return total;
}

/* Insert v into the descending array top[0..len) of capacity cap, keeping the
 * cap largest values.  Returns the new length. */
static int32_t top_insert(double *top, int32_t len, int32_t cap, double v)
{
    if (len == cap) {
        if (!(v > top[cap - 1]))
            return len;
        len = cap - 1; /* drop the smallest */
    }
    int32_t j = len;
    while (j > 0 && top[j - 1] < v) {
        top[j] = top[j - 1];
        --j;
    }
    top[j] = v;
    return len + 1;
}

/* theta[u*kmax + j] = the (j+1)-th largest f(p, u) over all of P (with
 * multiplicity), descending; -inf where j >= m.  This is the exact value the
 * lower-bound array of Definition 4 approximates from below. */
void ork_theta(const float *Q, int64_t n, const float *P, int64_t m, int32_t d,
               int32_t kmax, double *theta)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t u = 0; u < n; ++u) {
        double *top = theta + u * (int64_t)kmax;
        int32_t len = 0;
        const float *uu = Q + u * (int64_t)d;
        for (int64_t p = 0; p < m; ++p)
            len = top_insert(top, len, kmax, ork_dot(P + p * (int64_t)d, uu, d));
        for (int32_t j = len; j < kmax; ++j)
            top[j] = -INFINITY;
    }
}

/* Membership from the exact table: the number of items beating q is below k
 * iff the k-th largest value is <= f(q, u) (order-statistic identity).  When
 * k > m no k items exist and every user is a member; then theta holds -inf. */
int64_t ork_theta_query(const double *theta, int32_t kmax, const float *Q,
                        int64_t n, int32_t d, const float *q, int32_t k,
                        uint8_t *member)
{
    int64_t total = 0;
#pragma omp parallel for schedule(static) reduction(+ : total)
    for (int64_t u = 0; u < n; ++u) {
        double fq = ork_dot(q, Q + u * (int64_t)d, d);
        member[u] = (uint8_t)(theta[u * (int64_t)kmax + (k - 1)] <= fq);
        total += member[u];
    }
    return total;
}

/* f for a list of (row of A, row of B) pairs. */
void ork_pair_dots(const float *A, const float *B, int32_t d, const int64_t *ia,
                   const int64_t *ib, int64_t npairs, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < npairs; ++t)
        out[t] = ork_dot(A + ia[t] * (int64_t)d, B + ib[t] * (int64_t)d, d);
}

/* ---- Pre-processing, Algorithm 1 (Section 4.1) ------------------------- */

/* Squared norms sum_i x_i^2 in double, index order.  Sorting by the squared
 * norm orders vectors exactly as sorting by the norm does. */
void ork_sqnorms(const float *X, int64_t n, int32_t d, double *s2)
{
    for (int64_t r = 0; r < n; ++r)
        s2[r] = ork_dot(X + r * (int64_t)d, X + r * (int64_t)d, d);
}

static const double *g_sort_key;
static int cmp_desc(const void *a, const void *b)
{
    int32_t i = *(const int32_t *)a, j = *(const int32_t *)b;
    double ki = g_sort_key[i], kj = g_sort_key[j];
    if (ki > kj) return -1;
    if (ki < kj) return 1;
    return (i > j) - (i < j); /* equal keys keep input order */
}

/* perm[r] = index of the r-th vector in descending key order; equal keys in
 * ascending index order (a deterministic, stable order). */
void ork_sort_desc(const double *key, int64_t n, int32_t *perm)
{
    for (int64_t r = 0; r < n; ++r)
        perm[r] = (int32_t)r;
    g_sort_key = key;
    qsort(perm, (size_t)n, sizeof(int32_t), cmp_desc);
    g_sort_key = NULL;
}

/* Lower-bound arrays (Definition 4): P' is the first lb_items items of P in
 * descending norm order; for the user in sorted position i,
 *     L[j*n + i] = the (j+1)-th largest f(p, u_i) over p in P'
 * and -inf where j >= |P'|.  Users are addressed in sorted order via permQ,
 * items via permP. */
void ork_lower_bounds(const float *Q, int64_t n, const float *P, int64_t m,
                      int32_t d, const int32_t *permQ, const int32_t *permP,
                      int32_t kmax, int64_t lb_items, double *L)
{
    if (lb_items > m)
        lb_items = m;
#pragma omp parallel
    {
        double *top = (double *)malloc(sizeof(double) * (size_t)kmax);
#pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < n; ++i) {
            const float *uu = Q + (int64_t)permQ[i] * d;
            int32_t len = 0;
            for (int64_t t = 0; t < lb_items; ++t)
                len = top_insert(top, len, kmax,
                                 ork_dot(P + (int64_t)permP[t] * d, uu, d));
            for (int32_t j = 0; j < kmax; ++j)
                L[(int64_t)j * n + i] = j < len ? top[j] : -INFINITY;
        }
        free(top);
    }
}

/* Blocks (Definition 5, Equation (1)): consecutive runs of b sorted users,
 * the last one possibly shorter; LB[j*nB + B] = min over the block of
 * L[j*n + i].  Returns the number of blocks. */
int64_t ork_block_min(const double *L, int64_t n, int32_t kmax, int32_t b,
                      double *LB)
{
    int64_t nB = (n + b - 1) / b;
    for (int32_t j = 0; j < kmax; ++j)
        for (int64_t B = 0; B < nB; ++B) {
            double lo = INFINITY;
            for (int64_t i = B * b; i < n && i < (B + 1) * b; ++i)
                if (L[(int64_t)j * n + i] < lo)
                    lo = L[(int64_t)j * n + i];
            LB[(int64_t)j * nB + B] = lo;
        }
    return nB;
}

int32_t ork_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void ork_set_threads(int32_t t)
{
#ifdef _OPENMP
    if (t > 0)
        omp_set_num_threads(t);
#else
    (void)t;
#endif
}
