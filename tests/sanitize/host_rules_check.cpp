// Host-rule checks under AddressSanitizer and UndefinedBehaviorSanitizer:
// argument validation, error bounds and workspace sizing over a grid of
// shapes from the empty index to the largest sizes the library accepts.
// Every layout must stay inside its array, aligned and without overlap, and
// no size computation may overflow (the sanitizer aborts on signed overflow).
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <vector>

#include "host_rules.h"

using namespace rk;

static int failures = 0;
#define CHECK(c)                                                          \
  do {                                                                    \
    if (!(c)) {                                                           \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      ++failures;                                                         \
    }                                                                     \
  } while (0)

static rk_build_opts defaults() {
  rk_build_opts o;
  std::memset(&o, 0, sizeof(o));
  return o;
}

int main() {
  // option and size validation
  rk_build_opts o = defaults();
  CHECK(opts_error(o) == nullptr);
  for (int bs : {0, 16, 32, 64}) { o = defaults(); o.block_size = bs; CHECK(opts_error(o) == nullptr); }
  for (int bs : {1, 8, 48, 128, -64}) { o = defaults(); o.block_size = bs; CHECK(opts_error(o) != nullptr); }
  const double bad_margins[] = {-1e-9, 0.5, 1.0, std::numeric_limits<double>::infinity(),
                                std::numeric_limits<double>::quiet_NaN()};
  for (double mr : bad_margins) { o = defaults(); o.margin_rel = mr; CHECK(opts_error(o) != nullptr); }
  o = defaults(); o.precision = 7; CHECK(opts_error(o) != nullptr);
  o = defaults(); o.lb_items = -1; CHECK(opts_error(o) != nullptr);
  o = defaults(); o.pair_cap = -1; CHECK(opts_error(o) != nullptr);
  o = defaults(); o.device = -1; CHECK(opts_error(o) != nullptr);
  CHECK(sizes_error(0, 0, 1, 1) == nullptr);
  CHECK(sizes_error(INT32_MAX - 64, INT32_MAX - 64, 512, 128) == nullptr);
  CHECK(sizes_error(INT32_MAX - 63, 1, 8, 1) != nullptr);
  CHECK(sizes_error(-1, 1, 8, 1) != nullptr);
  CHECK(sizes_error(1, 1, 513, 1) != nullptr);
  CHECK(sizes_error(1, 1, 0, 1) != nullptr);
  CHECK(sizes_error(1, 1, 8, 129) != nullptr);
  CHECK(sizes_error(1, 1, 8, 0) != nullptr);
  const float vals[] = {0.f, -3.f, 1e30f, std::numeric_limits<float>::infinity(),
                        std::numeric_limits<float>::quiet_NaN(), 1099511627776.0f, 1.0e12f};
  CHECK(values_ok(vals, 2));
  CHECK(!values_ok(vals, 3));
  CHECK(!values_ok(vals + 3, 1) && !values_ok(vals + 4, 1) && !values_ok(vals + 5, 1));
  CHECK(values_ok(vals + 6, 1));
  CHECK(values_ok(nullptr, 0));

  // error bounds: positive, increasing in d, bf16 looser than float32
  for (int d = 1; d <= kMaxD; ++d) {
    CHECK(eps_fp32(d) > 0 && eps_fp32(d) < 1e-4);
    CHECK(eps_bf16(d) > eps_fp32(d) && eps_bf16(d) < 1e-2);
    if (d > 1) CHECK(eps_fp32(d) > eps_fp32(d - 1));
  }

  // query-tile parts of the batched filter: none for catalogs with at
  // least as many blocks as slots; about two workgroups per slot otherwise,
  // at most kQSplitMax parts of at least four tiles
  CHECK(bfilter_qsplit(1563, 63, 0) == 1);
  CHECK(bfilter_qsplit(1563, 63, 1024) == 1);
  CHECK(bfilter_qsplit(782, 64, 1024) == 3);
  CHECK(bfilter_qsplit(782, 8, 1024) == 2);
  CHECK(bfilter_qsplit(782, 7, 1024) == 1);
  CHECK(bfilter_qsplit(32, 64, 1024) == kQSplitMax);
  for (int64_t nb : {1, 2, 100, 1000, 1563, 5000, 8191, 100000})
    for (int64_t nt : {1, 4, 8, 16, 63, 64})
      for (int64_t sl : {1, 512, 1024, 2048}) {
        const int q = bfilter_qsplit(nb, nt, sl);
        CHECK(q >= 1 && q <= kQSplitMax);
        CHECK(q == 1 || nt / q >= 4);
        if (nb >= sl) CHECK(q == 1);
      }

  // workspace sizing over a grid of shapes
  const int64_t ns[] = {0, 1, 63, 64, 65, 2000, 100000, 540000, 1000000, 2000000, 7000000,
                        (int64_t)INT32_MAX - 64};
  const int32_t ds[] = {1, 3, 50, 64, 100, 200, 255, 512};
  const int32_t kms[] = {1, 25, 50, 128};
  const int64_t nqs[] = {0, 1, 63, 4096, 100000};
  int64_t layouts = 0;
  for (int64_t n : ns)
    for (int32_t d : ds)
      for (int32_t km : kms)
        for (int exact = 0; exact < 2; ++exact)
          for (int bf = 0; bf < 2; ++bf) {
            BatchShape x;
            x.n = n;
            x.n_pad = round_up(n, TILE);
            x.nB = (int32_t)(x.n_pad / TILE);
            x.d = d;
            x.d16 = (int32_t)round_up(d, 16);
            x.kmax = km;
            x.exact = exact;
            x.bf16 = bf;
            for (int64_t nq : nqs) {
              const int32_t c = batch_chunk(x, nq);
              CHECK(c >= 1 && c <= kBatchChunkMax);
              CHECK(c <= std::max<int64_t>(nq, 1));
              const BatchSizes z = batch_sizes(x, c);
              CHECK(z.pc >= 1 && z.bytes > 0);
              CHECK(z.pc <= INT32_MAX);  // the pair list is indexed with int32 capacities
              if (!exact) CHECK(z.chunk_cap >= 1 && z.chunk_cap <= INT32_MAX / kPairChunk);
              if (!exact) continue;
              const size_t bytes = size_t(64) << 20;
              const int32_t cn = noalloc_chunk(x, nq, bytes);
              if (cn == 0) {
                CHECK(n > 7000000);  // 64-query chunks fit up to about 7.5 million users
                continue;
              }
              CHECK(cn >= 1 && cn <= c);
              const ScratchLayout L = scratch_layout(x, cn, bytes);
              ++layouts;
              CHECK(L.end <= bytes && L.fixed <= L.end && L.pc >= 1);
              const size_t starts[] = {L.bits, L.counts, L.qn, L.perm, L.qt, L.qn_s, L.k_s, L.kofs_s,
                                       L.tsum, L.all, L.npairs, L.ks, L.pair_u, L.pair_j, L.pair_s};
              for (size_t v : starts) CHECK(v % 256 == 0 && v < L.end);
              for (size_t i = 1; i < sizeof(starts) / sizeof(starts[0]); ++i)
                CHECK(starts[i] > starts[i - 1]);  // in order, so regions cannot overlap
              const int64_t W = bitmap_words(n);
              CHECK(L.counts >= L.bits + (size_t)cn * (size_t)W * 4);
              CHECK(L.end >= L.pair_s + (size_t)L.pc * 4);
              if (bf) CHECK(L.qb > L.qt && L.qn_s >= L.qb + (size_t)round_up(cn, TILE) * x.d16 * 2);
            }
          }
  CHECK(layouts > 100);

  // index footprint: defined for every accepted size, -1 for bad ones
  for (int64_t n : ns)
    for (int32_t d : ds)
      for (int bs : {0, 16, 32}) {
        rk_build_opts f = defaults();
        f.block_size = bs;
        f.precision = RK_BF16;
        CHECK(index_footprint(n, n / 10, d, 128, f) > 0);
      }
  CHECK(index_footprint(-1, 1, 1, 1, defaults()) == -1);

  for (int64_t nq : {1, 2, 3, 1024, 1025, 1 << 20}) {
    const int b = size_bucket(nq);
    CHECK(b >= 0 && b < kSizeBuckets);
    if (b < kSizeBuckets - 1) CHECK((int64_t(1) << b) >= nq);
  }
  if (failures) {
    std::fprintf(stderr, "%d checks failed\n", failures);
    return 1;
  }
  std::printf("host rules ok (%lld workspace layouts)\n", (long long)layouts);
  return 0;
}
