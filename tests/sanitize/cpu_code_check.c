/* The oracle and the host CPU Simpfer under AddressSanitizer and
 * UndefinedBehaviorSanitizer, on small seeded inputs (integer-valued vectors,
 * so ties are frequent; a zero user; k from 1 to beyond m; empty sets).  The
 * brute form, the table form and CPU Simpfer must agree on every set. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int64_t ork_brute(const float *Q, int64_t n, const float *P, int64_t m, int32_t d,
                  const float *q, int32_t k, uint8_t *member);
void ork_theta(const float *Q, int64_t n, const float *P, int64_t m, int32_t d, int32_t kmax,
               double *theta);
int64_t ork_theta_query(const double *theta, int32_t kmax, const float *Q, int64_t n, int32_t d,
                        const float *q, int32_t k, uint8_t *member);
void ork_sqnorms(const float *X, int64_t n, int32_t d, double *s2);
void ork_sort_desc(const double *key, int64_t n, int32_t *perm);
void ork_lower_bounds(const float *Q, int64_t n, const float *P, int64_t m, int32_t d,
                      const int32_t *permQ, const int32_t *permP, int32_t kmax, int64_t lb_items,
                      double *L);
int64_t ork_block_min(const double *L, int64_t n, int32_t kmax, int32_t b, double *LB);

typedef struct {
    int64_t blocks, blocks_pruned, users, lemma1_no, lemma2_yes, scans, scan_items, results;
} cs_stats;
void *cs_build(const float *Q, int64_t n, const float *P, int64_t m, int32_t d, int32_t kmax,
               int32_t lb_items, int32_t b);
void cs_rebuild(void *x, int32_t kmax);
void cs_free(void *x);
int64_t cs_query(const void *x, const float *q, int32_t k, int32_t *ids, cs_stats *st);

static uint64_t rng = 88172645463325252ull;
static int next_int(int lo, int hi)
{
    rng ^= rng << 13;
    rng ^= rng >> 7;
    rng ^= rng << 17;
    return lo + (int)(rng % (uint64_t)(hi - lo + 1));
}

static int run(int64_t n, int64_t m, int32_t d, int32_t kmax, int32_t lb, int32_t b)
{
    float *Q = malloc(sizeof(float) * (size_t)(n * d + 1));
    float *P = malloc(sizeof(float) * (size_t)(m * d + 1));
    for (int64_t i = 0; i < n * d; ++i) Q[i] = (float)next_int(-3, 3);
    for (int64_t i = 0; i < m * d; ++i) P[i] = (float)next_int(-3, 3);
    if (n > 2) memset(Q + 2 * d, 0, sizeof(float) * (size_t)d); /* a zero user */
    int bad = 0;
    double *th = malloc(sizeof(double) * (size_t)(n * kmax + 1));
    ork_theta(Q, n, P, m, d, kmax, th);
    double *s2 = malloc(sizeof(double) * (size_t)(n + m + 1));
    int32_t *pq = malloc(sizeof(int32_t) * (size_t)(n + 1)), *pp = malloc(sizeof(int32_t) * (size_t)(m + 1));
    ork_sqnorms(Q, n, d, s2);
    ork_sort_desc(s2, n, pq);
    ork_sqnorms(P, m, d, s2);
    ork_sort_desc(s2, m, pp);
    double *L = malloc(sizeof(double) * (size_t)(n * kmax + 1));
    ork_lower_bounds(Q, n, P, m, d, pq, pp, kmax, lb, L);
    double *LB = malloc(sizeof(double) * (size_t)(((n + b - 1) / b) * kmax + 1));
    if (n) ork_block_min(L, n, kmax, b, LB);
    void *cs = cs_build(Q, n, P, m, d, kmax, lb, b);
    uint8_t *mb = malloc((size_t)n + 1), *mt = malloc((size_t)n + 1);
    int32_t *ids = malloc(sizeof(int32_t) * (size_t)(n + 1));
    float *q = malloc(sizeof(float) * (size_t)d);
    for (int t = 0; t < 12; ++t) {
        if (m > 0 && t % 2 == 0) memcpy(q, P + (int64_t)next_int(0, (int)m - 1) * d, sizeof(float) * (size_t)d);
        else for (int32_t c = 0; c < d; ++c) q[c] = (float)next_int(-3, 3);
        for (int32_t k = 1; k <= kmax + 2; ++k) {
            memset(mb, 0, (size_t)n + 1);
            const int64_t cb = ork_brute(Q, n, P, m, d, q, k, mb);
            if (k <= kmax) {
                memset(mt, 0, (size_t)n + 1);
                const int64_t ct = ork_theta_query(th, kmax, Q, n, d, q, k, mt);
                if (ct != cb || memcmp(mb, mt, (size_t)n)) ++bad;
            }
            cs_stats st;
            if (k > kmax && k <= m) cs_rebuild(cs, k);
            const int64_t cc = cs_query(cs, q, k, ids, &st);
            int64_t j = 0;
            for (int64_t u = 0; u < n; ++u)
                if (mb[u]) {
                    if (j >= cc || ids[j] != u) ++bad;
                    ++j;
                }
            if (j != cc) ++bad;
        }
    }
    cs_free(cs);
    free(Q); free(P); free(th); free(s2); free(pq); free(pp); free(L); free(LB);
    free(mb); free(mt); free(ids); free(q);
    if (bad) fprintf(stderr, "n=%lld m=%lld d=%d kmax=%d lb=%d b=%d: %d mismatches\n", (long long)n,
                     (long long)m, d, kmax, lb, b, bad);
    return bad;
}

int main(void)
{
    int bad = 0;
    bad += run(300, 80, 3, 6, 8, 8);
    bad += run(257, 65, 4, 10, 0, 16);
    bad += run(64, 5, 2, 4, 3, 1);      /* k beyond m */
    bad += run(1, 1, 1, 1, 1, 1);
    bad += run(0, 10, 3, 2, 2, 4);      /* no users */
    bad += run(20, 0, 3, 2, 2, 4);      /* no items: everyone */
    if (bad) return 1;
    printf("oracle and cpu simpfer ok\n");
    return 0;
}
