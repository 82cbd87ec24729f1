// Host-side rules of the library that involve no device: argument checks,
// the error bounds of the certified comparisons, and the sizing of the
// batched path's workspace (chunks of queries, pair slots, the layout of the
// static workspace of the entry point that allocates nothing) and of an
// index.  Plain C++ (no HIP): the runtime uses it, and a host build with
// address and undefined-behaviour sanitizers exercises it on the CPU.
#pragma once
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <cstddef>

#include "rkmips.h"

namespace rk {

constexpr int TILE = 64;              // users per tile == items per tile == wave size
constexpr int kBatchChunkMax = 4096;  // queries per chunk (single-workgroup sort in LDS)
constexpr int kPairChunk = 256;       // slots per pair chunk (bounded table)
constexpr int kUserPairs = 8;         // flagged-pair slots per user in the scan's long pass
constexpr int kExactRun = 64;         // exact table: pair slots a filter wave reserves at a time
constexpr int32_t kMaxD = 512;
constexpr int32_t kVerifyTilesMaxD = 256;  // widest rows of the one-query tiled scan (prefetch registers)
constexpr int32_t kMaxKmax = 128;
constexpr int64_t kBitmapBudget = 512ll << 20;  // bytes of per-query result bits per chunk
// Undecided-pair slots per chunk of queries.  Exact table: only the pairs
// within rounding of theta_k (rechecks); bounded table: every survivor of the
// filter goes to the scan, and a query chunk is sized for a quarter of the
// users surviving per query.  Larger chunks cost the scan less per query
// (the per-chunk passes and hand-offs): 2^29 slots (8 GB of pair list) take
// 1M users x 100k items, P' = 50, from six chunks to two (129 -> 104 ms per
// 3,000 queries) and 500k x 50k, P' = 100, from four to one (673 -> 183 ms).
constexpr int64_t kPairBudgetExact = 1ll << 24;
constexpr int64_t kPairBudget = 1ll << 29;
// Bounded table: batches of at least this many queries run the scan's first
// pass (the item prefix of every user) before the filter, whose bounds it
// tightens; smaller ones leave it to the blocks that have pairs.
constexpr int64_t kPrescanMin = 256;

// Scan list length per user: k_max + 2 rounded up to a multiple of 4.
constexpr int bscan_list_len(int kmax) { return (kmax + 2 + 3) / 4 * 4; }

inline int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

// Words of a batched result bitmap row: one bit per user, rows 16-byte aligned.
inline int64_t bitmap_words(int64_t n) { return round_up(std::max<int64_t>((n + 31) / 32, 1), 4); }

inline double gamma_(double k, double u) { return k * u / (1.0 - k * u); }

// Rigorous relative bounds |approx u.x - f(x,u)| <= eps * |u| |x|: float32
// accumulation of d exact or once-rounded products in any order, plus the
// float64 rounding of f itself, plus slack for evaluating the certified tests
// in float32.
inline double eps_fp32(int d) {
  return gamma_(d + 2, 0x1p-24) + gamma_(d, 0x1p-53) + 16 * 0x1p-24;
}
inline double eps_bf16(int d) {
  const double r = (1 + 0x1p-8) * (1 + 0x1p-8) * (1 + gamma_(d + 2, 0x1p-24)) - 1;
  return r + gamma_(d, 0x1p-53) + 16 * 0x1p-24;
}

// Largest batch that runs one query at a time when the caller may use the
// index's one-query workspace: a batched launch costs about the same for 1
// to ~64 queries (every block's prologue), a one-query launch about a fifth
// to a sixth of it (measured, exact tables: 50k users / d = 50, 0.06 vs 0.02
// ms; 500k / d = 100, 0.24 vs 0.06 ms; 1M / d = 100, 0.50 vs 0.12 ms; 2M /
// d = 200, 2.1 vs 0.38 ms per query).
inline int64_t small_batch_max(int64_t nB) { return std::max<int64_t>(2, nB / 4096); }

// Query-tile parts per user block in the batched filter (exact table).  A
// catalog with fewer blocks than the device has workgroup slots (resident
// workgroups per CU x CUs) leaves CUs idle or thinly occupied: each block's
// query tiles are then split into parts, one workgroup each (each with its
// own prologue: the block's rows, bounds and Lemma 3 masks over its tiles),
// for about two workgroups per slot, with at least four tiles a part.
// Measured per 4,096 queries: 50k users (782 blocks on 1,024 slots) in 3
// parts, float32 347 -> 310 us, bf16 242 -> 230 us.  100k users (1,563
// blocks) stay whole: 3 parts gained 3% in float32 but lost 7% in bf16, 5
// and 8 parts lost 5-29% in both (the prologues cost more than the partial
// last round, whose workgroups run faster at the lower occupancy).
constexpr int kQSplitMax = 8;
inline int bfilter_qsplit(int64_t nB, int64_t nT, int64_t slots) {
  if (slots <= 0 || nB <= 0 || nB >= slots) return 1;
  const int64_t want = (2 * slots + nB - 1) / nB;
  return (int)std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(want, nT / 4), kQSplitMax));
}

// nullptr when the options are valid, else the reason.
inline const char* opts_error(const rk_build_opts& o) {
  if (o.precision != RK_FP32 && o.precision != RK_BF16) return "precision must be RK_FP32 or RK_BF16";
  if (o.lb_items < 0) return "lb_items must be >= 0";
  if (o.block_size != 0 && o.block_size != 16 && o.block_size != 32 && o.block_size != TILE)
    return "block_size must be 0, 16, 32 or 64";
  if (!(o.margin_rel >= 0.0) || !std::isfinite(o.margin_rel) || o.margin_rel >= 0.5)
    return "margin_rel must be finite, >= 0 and < 0.5";
  if (o.cand_cap < 0) return "cand_cap must be >= 0";
  if (o.pair_cap < 0) return "pair_cap must be >= 0";
  if (o.handoff_tiles < 0) return "handoff_tiles must be >= 0";
  if (o.device < 0) return "device must be >= 0";
  return nullptr;
}

inline const char* sizes_error(int64_t n, int64_t m, int32_t d, int32_t k_max) {
  if (n < 0 || m < 0) return "n and m must be >= 0";
  if (n > INT32_MAX - 64 || m > INT32_MAX - 64) return "n and m must fit int32 ids";
  if (d < 1 || d > kMaxD) return "d must be in [1, 512]";
  if (k_max < 1 || k_max > kMaxKmax) return "k_max must be in [1, 128]";
  return nullptr;
}

// Every value finite and below 2^40 in magnitude (products and sums of such
// values stay far from float32 overflow).
inline bool values_ok(const float* x, int64_t count) {
  for (int64_t i = 0; i < count; ++i)
    if (!(std::fabs(x[i]) < 1099511627776.0f)) return false;
  return true;
}

// What the batched path's sizing needs to know of an index.
struct BatchShape {
  int64_t n = 0, n_pad = 0;
  int32_t nB = 0, d = 1, d16 = 16, kmax = 1;
  bool exact = true, bf16 = false;
  int64_t pair_cap_opt = 0;  // rk_build_opts.pair_cap (0 = default)
};

// Sizes of the batched path's workspace for chunks of `chunk` queries.
struct BatchSizes {
  int64_t pc = 0;         // pair slots
  int64_t chunk_cap = 0;  // pair chunks (bounded table)
  int64_t maxc = 0;       // chunk-list capacity per block (bounded table)
  int64_t bytes = 0;      // device bytes of the whole workspace
};

inline BatchSizes batch_sizes(const BatchShape& x, int32_t chunk) {
  BatchSizes z;
  const int64_t cp = round_up(chunk, TILE), W = bitmap_words(x.n);
  int64_t pc = std::min<int64_t>((int64_t)chunk * std::max<int64_t>(x.n_pad, 1),
                                 x.exact ? kPairBudgetExact : kPairBudget);
  // exact table: each of a block's four filter waves may leave up to
  // kExactRun - 1 slots of its last reserved run unused (bounded so that very
  // large catalogs keep a modest list)
  if (x.exact) pc += std::min<int64_t>(4 * (int64_t)x.nB * kExactRun, 3 * kPairBudgetExact);
  if (x.pair_cap_opt > 0) pc = x.pair_cap_opt;
  if (!x.exact) {
    // Chunks of kPairChunk slots: every chunk is full but the one each of a
    // block's four filter waves is filling, so pc pairs need at most
    // pc / kPairChunk + 4 nB chunks (an explicit pair_cap is taken as is).
    z.chunk_cap = x.pair_cap_opt > 0 ? pc / kPairChunk
                                     : (pc + kPairChunk - 1) / kPairChunk + 4 * (int64_t)x.nB;
    z.chunk_cap = std::min<int64_t>(z.chunk_cap, INT32_MAX / kPairChunk);
    pc = std::max<int64_t>(pc, z.chunk_cap * kPairChunk);
    z.maxc = TILE * cp / kPairChunk + 4;
  }
  z.pc = pc;
  const int64_t d2 = x.d + (x.d & 1);
  int64_t b = chunk * 4 * 2 + cp * d2 * 4 + (x.bf16 ? cp * x.d16 * 2 : 0) + cp * 12 + cp / TILE * 32 +
              chunk * W * 4 + chunk * 8 + chunk + 8 + pc * 12 + chunk * 4;
  if (!x.exact)
    b += std::max<int64_t>(pc, 1) * 4 + std::max<int64_t>(z.chunk_cap, 1) * 4 + 4 +
         std::max<int64_t>(x.nB, 1) * 4 * (1 + z.maxc) +
         std::max<int64_t>(x.n_pad, 1) * (8 * (int64_t)bscan_list_len(x.kmax) + 4) + 4 +
         std::max<int64_t>(x.nB, 1) * 4 + std::max<int64_t>(x.n_pad, 1) * (20 + 12 * kUserPairs) + 4;
  z.bytes = b;
  return z;
}

// Queries per chunk of the batched path for a batch of nq queries.  With a
// bounded table every survivor of the filter takes a pair slot; the chunk is
// sized so that up to a quarter of all (user, query) pairs fit the slots (a
// larger share would spill into the filter's in-kernel float64 fallback).
inline int32_t batch_chunk(const BatchShape& x, int64_t nq) {
  const int64_t W = bitmap_words(x.n);
  int64_t c = std::min<int64_t>({nq, (int64_t)kBatchChunkMax, kBitmapBudget / (W * 4)});
  if (!x.exact && x.pair_cap_opt == 0)
    c = std::min<int64_t>(c, std::max<int64_t>(TILE, kPairBudget / std::max<int64_t>(x.n_pad / 4, 1)));
  return (int32_t)std::max<int64_t>(1, c);
}

// Byte offsets of the exact-table batch workspace inside one static array
// (the entry point that allocates nothing): every region 256-byte aligned,
// pair slots last with what is left (at most the regular budget; pairs
// beyond them are decided in float64 by the filter).
struct ScratchLayout {
  size_t bits = 0, counts = 0, qn = 0, perm = 0, qt = 0, qb = 0, qn_s = 0, k_s = 0, kofs_s = 0,
         tsum = 0, all = 0, npairs = 0, ks = 0, pair_u = 0, pair_j = 0, pair_s = 0;
  size_t fixed = 0;  // bytes before the pair slots
  size_t end = 0;    // bytes of the whole layout
  int64_t pc = 0;    // pair slots
};

inline ScratchLayout scratch_layout(const BatchShape& x, int32_t chunk, size_t bytes) {
  ScratchLayout L;
  const int64_t cp = round_up(chunk, TILE), W = bitmap_words(x.n);
  size_t off = 0;
  auto take = [&](size_t& at, int64_t count, size_t elem) {
    off = (size_t)round_up((int64_t)off, 256);
    at = off;
    off += (size_t)std::max<int64_t>(count, 1) * elem;
  };
  take(L.bits, (int64_t)chunk * std::max<int64_t>(W, 1), 4);
  take(L.counts, chunk, 8);
  take(L.qn, chunk, 4);
  take(L.perm, chunk, 4);
  take(L.qt, cp * (x.d + (x.d & 1)), 4);
  if (x.bf16) take(L.qb, cp * x.d16, 2);
  take(L.qn_s, cp, 4);
  take(L.k_s, cp, 4);
  take(L.kofs_s, cp, 4);
  take(L.tsum, cp / TILE * 8, 4);
  take(L.all, chunk, 1);
  take(L.npairs, 1, 8);
  take(L.ks, chunk, 4);
  L.fixed = off;
  const size_t left = bytes > L.fixed + 4 * 256 ? bytes - L.fixed - 4 * 256 : 0;
  L.pc = std::min<int64_t>(batch_sizes(x, chunk).pc, (int64_t)(left / 12));
  take(L.pair_u, L.pc, 4);
  take(L.pair_j, L.pc, 4);
  take(L.pair_s, L.pc, 4);
  L.end = off;
  return L;
}

// The largest chunk (the regular one, halved as often as needed, at least
// 64 queries) whose layout fits `bytes` with room for 64 Ki pair slots; 0
// when even 64 queries do not fit.
inline int32_t noalloc_chunk(const BatchShape& x, int64_t nq, size_t bytes) {
  int32_t chunk = batch_chunk(x, nq);
  for (;;) {
    const ScratchLayout L = scratch_layout(x, chunk, bytes);
    const int64_t want_pairs = std::min<int64_t>(batch_sizes(x, chunk).pc, 1 << 16);
    if (L.fixed + 4 * 256 + (size_t)want_pairs * 12 <= bytes) return chunk;
    if (chunk <= TILE) return 0;
    chunk = std::max<int32_t>(TILE, chunk / 2);
  }
}

// Device bytes of an index (rk_index_footprint).
inline int64_t index_footprint(int64_t n, int64_t m, int32_t d, int32_t k_max, const rk_build_opts& o) {
  if (n < 0 || m < 0 || d < 1 || k_max < 1) return -1;
  const int64_t np = round_up(n, TILE), mp = round_up(m, TILE);
  const int64_t nB = np / (o.block_size == 16 || o.block_size == 32 ? o.block_size : TILE);
  const int64_t d16 = round_up(d, 16);
  int64_t b = 0;
  b += n * 8 + m * 8 + n * 4 + m * 4;                 // squared norms, permutations
  b += np * d * 4 + np * 4 + mp * d * 4 + mp * 4 + m * d * 4 + n * d * 4;  // tiled copies, norms, rows
  if (o.precision == RK_BF16) b += (np + mp) * d16 * 2;
  b += (int64_t)k_max * np * 12 + (int64_t)k_max * nB * 4 + nB * 4;  // L64, L32, LB, bnorm
  b += ((n + 31) / 32) * 4 + np * 12 + 4 * 4 + 4 + 16 * 8 + d * 4 + std::max<int64_t>(n, 1) * 4 + 8;
  return b;
}

// Serving: launch-time estimates per batch-size bucket (ceil(log2(nq)), 0..15).
constexpr int kSizeBuckets = 16;
inline int size_bucket(int64_t nq) {
  int b = 0;
  while (b < kSizeBuckets - 1 && (int64_t(1) << b) < nq) ++b;
  return b;
}

}  // namespace rk
