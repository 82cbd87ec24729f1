// Batched online query: many queries of mixed k in one pass over the users.
//
// Algorithm 3 is run for every (user, query) pair of a batch, but organised
// for the device: one workgroup owns one block of 64 norm-sorted users
// (Definition 5) and walks every 64-query tile of the batch.  The block's
// users are read from HBM once; query tiles stay in L2.  Queries are sorted
// by descending norm first, so a tile whose every query is pruned for the
// block by Lemma 3 is skipped as a whole.  Scores u.q come from MFMA tiles
// (32x32 blocks, float32 or bfloat16 inputs with float32 accumulation); the
// certified Lemma 1 / Lemma 2 / exact-table tests run in the epilogue.
// Pairs that remain undecided go to a pair list: the linear scan of
// Algorithm 2 (bounded-table mode) or the float64 recheck.  Results are
// per-query bitmaps over original user ids, turned into CSR rows at the end.
#include "batch_device.h"
#include <atomic>
#include <climits>

namespace rk {

__device__ __forceinline__ unsigned long long lanemask_lt_b() {
  const int lane = threadIdx.x & 63;
  return lane ? (~0ull >> (64 - lane)) : 0ull;
}

// ---------------------------------------------------------------------------
// Per query of the chunk: |q| rounded up (one wave per query).
__global__ void k_bnorms(const float* __restrict__ qs, int32_t nq, int32_t d,
                         float* __restrict__ qn, unsigned long long* __restrict__ npairs) {
  const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (j == 0 && lane == 0) *npairs = 0;
  if (j >= nq) return;
  const float* q = qs + j * d;
  double s = 0.0;
  for (int c = lane; c < d; c += 64) s = fma((double)q[c], (double)q[c], s);
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if (lane == 0) qn[j] = f32_up(sqrt(s) * (1.0 + (double)(d + 4) * 0x1p-53));
}

// Sort of the chunk's queries by k ascending, then |q| descending in buckets
// of 1/16 octave below the chunk's largest norm (64 buckets per k), so that a
// 64-query tile usually has one k and queries of similar norm: the Lemma 3
// test then prunes whole tiles and the epilogue reads one lower bound per
// user.  Counting sort in one workgroup (histogram, scan, scatter); the order
// inside a bucket is the atomics' order, which no result depends on (every
// decision is per (user, query)).
constexpr int kSortBuckets = 64;

__global__ void __launch_bounds__(1024) k_bsort(const float* __restrict__ qn,
                                                const int32_t* __restrict__ ks, int32_t nq,
                                                int32_t kmax, int32_t* __restrict__ perm) {
  extern __shared__ int hist[];  // (kmax + 1) * kSortBuckets bins
  __shared__ uint32_t top_bits;
  __shared__ int wsum[16];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int nbins = (kmax + 1) * kSortBuckets;
  if (t == 0) top_bits = 0u;
  for (int i = t; i < nbins; i += 1024) hist[i] = 0;
  __syncthreads();
  uint32_t mx = 0u;  // norms are >= 0: larger float bits = larger norm
  for (int p = t; p < nq; p += 1024) mx = max(mx, __float_as_uint(qn[p]));
  for (int off = 32; off > 0; off >>= 1) mx = max(mx, (uint32_t)__shfl_xor((int)mx, off));
  if (lane == 0) atomicMax(&top_bits, mx);
  __syncthreads();
  const uint32_t top = top_bits;
  int key[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int p = t + 1024 * e;
    key[e] = -1;
    if (p < nq) {
      const int k = min(max(ks[p], 0), kmax);
      const uint32_t bk = min((top - __float_as_uint(qn[p])) >> 19, (uint32_t)(kSortBuckets - 1));
      key[e] = k * kSortBuckets + (int)bk;
      atomicAdd(&hist[key[e]], 1);
    }
  }
  __syncthreads();
  // exclusive scan of the bins: thread t owns bins [t*per, (t+1)*per)
  const int per = (nbins + 1023) / 1024;
  const int b0 = min(t * per, nbins), b1 = min(b0 + per, nbins);
  int local = 0;
  for (int i = b0; i < b1; ++i) local += hist[i];
  int incl = local;
  for (int off = 1; off < 64; off <<= 1) {
    const int v = __shfl_up(incl, off);
    if (lane >= off) incl += v;
  }
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  int run = incl - local;
  for (int w = 0; w < wave; ++w) run += wsum[w];
  for (int i = b0; i < b1; ++i) {
    const int cnt = hist[i];
    hist[i] = run;
    run += cnt;
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < 4; ++e)
    if (key[e] >= 0) perm[atomicAdd(&hist[key[e]], 1)] = t + 1024 * e;
}

// Query tiles in sorted order: fp32 [T][d][64] and (bf16 mode) [T][G][64][8],
// plus sorted norms and k.  Padding queries are zero with k = 0.
// A query with k > m has every user as a member: it gets k = 0 here (no
// filter work) and is marked in `all` for the assembly.
__global__ void k_btile(const float* __restrict__ qs, const int32_t* __restrict__ ks,
                        const float* __restrict__ qn, const int32_t* __restrict__ perm,
                        int32_t nq, int32_t nq_pad, int32_t d, int32_t d16, int64_t m,
                        float* __restrict__ qt, uint16_t* __restrict__ qb,
                        float* __restrict__ qn_s, int32_t* __restrict__ k_s,
                        int32_t* __restrict__ kofs_s, uint8_t* __restrict__ all) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.y + threadIdx.y;
  if (r >= nq_pad) return;
  const bool valid = r < nq;
  const int64_t src = valid ? perm[r] : 0;
  const int d2 = d + (d & 1);  // fp32 query tiles have an even number of rows
  for (int c = threadIdx.x; c < d2; c += blockDim.x)
    qt[tix(r, c, d2)] = (valid && c < d) ? qs[src * d + c] : 0.0f;
  if (qb) {
    const int64_t tile = r / TILE, lane = r % TILE;
    for (int c = threadIdx.x; c < d16; c += blockDim.x) {
      const float v = (valid && c < d) ? qs[src * d + c] : 0.0f;
      qb[((tile * (d16 / 8) + c / 8) * TILE + lane) * 8 + (c % 8)] = bf16_bits(v);
    }
  }
  if (threadIdx.x == 0) {
    const int32_t k = valid ? ks[src] : 0;
    qn_s[r] = valid ? qn[src] : 0.0f;
    k_s[r] = k > m ? 0 : k;
    kofs_s[r] = (k > m || k < 1 ? 0 : k - 1) * TILE;
    if (valid) all[src] = k > m ? 1 : 0;
  }
}

// Per tile of sorted queries and per query half (rows 32 h .. 32 h + 31): the
// largest norm (float bits), the smallest and largest k row, and the first
// row of the largest k when the half holds at most two k's (0 for one k; -1
// for more).  Rows are sorted by k, so with two k's every live row from that
// row on has the larger one (rows of k > m or padding, which hold row 0,
// come last and are never live).  One wave per tile.
__global__ void k_btsum(const float* __restrict__ qn_s, const int32_t* __restrict__ kofs_s,
                        int32_t* __restrict__ tsum) {
  const int64_t T = blockIdx.x;
  const int lane = threadIdx.x & 63, h = lane >> 5;
  const float n = qn_s[T * TILE + lane];
  const int k = kofs_s[T * TILE + lane];
  float nmax = n;
  int kmin = k, kmx = k;
  for (int off = 16; off > 0; off >>= 1) {  // within each half of the wave
    nmax = fmaxf(nmax, __shfl_xor(nmax, off));
    kmin = min(kmin, __shfl_xor(kmin, off));
    kmx = max(kmx, __shfl_xor(kmx, off));
  }
  const uint32_t other = (uint32_t)(__ballot(k != kmin && k != kmx) >> (32 * h));
  const uint32_t hi = (uint32_t)(__ballot(k == kmx) >> (32 * h));
  const int code = kmin == kmx ? 0 : (other ? -1 : __ffs((int)hi) - 1);
  if ((lane & 31) < 4) {
    const int v[4] = {__float_as_int(nmax), kmin, kmx, code};
    tsum[T * 8 + 4 * h + (lane & 31)] = v[lane & 31];
  }
}

// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// The batched filter.  Workgroup = 4 waves = one user block B (64 users).
// It first evaluates Lemma 3 for every query of the chunk against the block
// (one bit per query, a 64-bit mask per 64-query tile, kept in LDS) and then
// walks only the tiles that have a live query.  All four waves work on the
// same query tile, staged in LDS: wave w computes the 32x32 quarter (user
// half w&1, query half w>>1) with MFMA, so a lane holds one user and 16
// queries.  While a tile is processed the next live tile is being fetched:
// small bf16 tiles (d <= 64) straight into a second LDS buffer
// (global_load_lds, one barrier per tile), other tiles into registers,
// written to LDS between two barriers.  The epilogue
// is the certified Lemma 1 test only; every pair it cannot reject is
// appended to the pair list, decided afterwards by the recheck or the scan.
constexpr int PF_VEC = 16;  // prefetch registers per thread: 16 x 16 bytes (64 KiB tiles)

__device__ __forceinline__ int next_live(const unsigned long long* masks, int from, int nT) {
  int T = from;
  while (T < nT && masks[T] == 0ull) ++T;
  return T;
}

// Prefetch of query tile T (tile_vecs 16-byte vectors, thread t takes
// t, t+256, ...) and its metadata into registers, and their store to LDS.
// A tile of NV >= 4 vectors per thread has more than NV / 2 of them (the
// launch picks the smallest NV that holds it), so the low half needs no bound
// check.
template <int NV>
__device__ __forceinline__ constexpr bool lo_half(int v) { return NV >= 4 && v < NV / 2; }

template <int NV>
__device__ __forceinline__ void stage_tile(const u32x4* __restrict__ qsrc, const BatchView& bv,
                                           int T, int tile_vecs, int t, u32x4 (&pf)[NV],
                                           float& pf_n, int32_t& pf_k) {
  const u32x4* src = qsrc + (int64_t)T * tile_vecs;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const int i = v * 256 + t;
    if (lo_half<NV>(v) || i < tile_vecs) pf[v] = src[i];
  }
  if (t < TILE) pf_n = bv.qn_s[(int64_t)T * TILE + t];
  else if (t < 2 * TILE) pf_k = bv.kofs_s[(int64_t)T * TILE + t - TILE];
  else if (t < 2 * TILE + 8) pf_k = bv.tsum[(int64_t)T * 8 + t - 2 * TILE];
}

template <int NV>
__device__ __forceinline__ void commit_tile(unsigned char* qbuf, float* meta_n, int32_t* meta_k,
                                            int tile_vecs, int t, const u32x4 (&pf)[NV],
                                            float pf_n, int32_t pf_k) {
  u32x4* dst = (u32x4*)qbuf;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const int i = v * 256 + t;
    if (lo_half<NV>(v) || i < tile_vecs) dst[i] = pf[v];
  }
  if (t < TILE) meta_n[t] = pf_n;
  else if (t < 2 * TILE + 8) meta_k[t - TILE] = pf_k;  // k rows, then the 8 summary words
}

typedef __attribute__((address_space(3))) void lds_void_t;

// Query tile T and its metadata straight from global memory into LDS
// (global_load_lds: lane l of a wave writes 16 bytes at the wave's LDS base +
// 16 l, so one instruction moves 1 KiB): wave w moves the 1 KiB chunks w,
// w+4, ...; waves 0 and 1 move the 64 norms and k rows.  The data is there
// once the issuing wave has waited for its vector memory operations.
__device__ __forceinline__ void issue_tile(const unsigned char* __restrict__ qsrc, const BatchView& bv,
                                           int T, int tile_bytes, int lane, int wave,
                                           unsigned char* qdst, float* mn_dst, int32_t* mk_dst) {
  const unsigned char* src = qsrc + (int64_t)T * tile_bytes;
  for (int c = wave; c * 1024 < tile_bytes; c += 4) {
    if (c * 1024 + lane * 16 < tile_bytes)
      __builtin_amdgcn_global_load_lds((const void*)(src + c * 1024 + lane * 16),
                                       (lds_void_t*)(qdst + c * 1024), 16, 0, 0);
  }
  if (wave == 0)
    __builtin_amdgcn_global_load_lds((const void*)(bv.qn_s + (int64_t)T * TILE + lane),
                                     (lds_void_t*)mn_dst, 4, 0, 0);
  else if (wave == 1)
    __builtin_amdgcn_global_load_lds((const void*)(bv.kofs_s + (int64_t)T * TILE + lane),
                                     (lds_void_t*)mk_dst, 4, 0, 0);
  else if (wave == 2 && lane < 8)
    __builtin_amdgcn_global_load_lds((const void*)(bv.tsum + (int64_t)T * 8 + lane),
                                     (lds_void_t*)(mk_dst + TILE), 4, 0, 0);
}

// Inclusive prefix sum over the 64 lanes of a wave in registers (DPP): the
// shifts by 1, 2, 4 and 8 lanes scan each row of 16 lanes (a lane with no
// source lane adds 0), then the last lane of row 0 (of row 2) is added to row 1
// (row 3), and that of row 1 to rows 2 and 3.
__device__ __forceinline__ int wave_incl_scan(int x) {
  x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xF, 0xF, false);  // row_shr:1
  x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xF, 0xF, false);  // row_shr:2
  x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xF, 0xF, false);  // row_shr:4
  x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xF, 0xF, false);  // row_shr:8
  x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xA, 0xF, false);  // row_bcast:15 -> rows 1, 3
  x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xC, 0xF, false);  // row_bcast:31 -> rows 2, 3
  return x;
}

// Occupancy: float32 tiles of d <= 64 (NV <= 4) run 4 waves per SIMD
// (within 128 registers, no spill); wider tiles keep their prefetch
// registers and 2-3 waves.
template <bool BF16, int NV>
__global__ void __launch_bounds__(256, (!BF16 && NV <= 4) ? 4 : 2) k_bfilter(DevIndex ix, BatchView bv) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int d = ix.d;
  // the workgroup's user block, and its part of the chunk's query tiles
  // [T0, nT) (a catalog with few blocks splits each block's tiles)
  const int64_t B = blockIdx.x % ix.nB;
  const int part = (int)(blockIdx.x / ix.nB);
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int half = lane >> 5, col = lane & 31;
  const int uh = wave & 1, qhalf = wave >> 1;
  const int G = ix.d16 / 8;
  const int d2 = d + (d & 1);  // fp32 tiles carry an even number of rows
  const int tile_bytes = BF16 ? G * TILE * 16 : d2 * TILE * 4;
  const int tile_vecs = tile_bytes / 16;
  const int T0 = (int)((int64_t)part * (bv.nq_pad / TILE) / bv.qsplit);
  const int nT = (int)((int64_t)(part + 1) * (bv.nq_pad / TILE) / bv.qsplit);
  unsigned char* p = lds_raw;
  unsigned char* ubuf = p;
  p += (tile_bytes + 15) / 16 * 16;
  // query tile buffers: small bf16 tiles two, alternating (filled straight
  // from global memory while the other is used); otherwise one, filled from
  // prefetch registers (a second float32 buffer would cost a workgroup per
  // CU; and as the compiler waits for the direct loads before the next LDS
  // read, larger tiles lose the overlap: 42-66% slower at d = 100-200)
  constexpr bool LDSD = BF16 && NV <= 2;
  unsigned char* qbuf2[2];
  qbuf2[0] = p;
  p += (tile_bytes + 15) / 16 * 16;
  qbuf2[1] = p;
  if (LDSD) p += (tile_bytes + 15) / 16 * 16;
  float* meta_n2 = (float*)p;    // [2][64] norms of the tile's queries
  p += 2 * TILE * 4;
  int32_t* meta_k2 = (int32_t*)p;  // [2][72] their k's rows in the (k, user) tables, and
                                   // the tile's two half summaries (k_btsum)
  p += 2 * (TILE + 8) * 4;
  // Lemma 3 blocks of bsize users: nsb per 64-user tile, a live-query mask
  // per (block, query tile), and with nsb > 1 their union (the tile walk)
  constexpr int MT = kBatchChunkMax / TILE;
  const int nsb = TILE / ix.bsize;
  unsigned long long* masks = (unsigned long long*)p;  // [nsb][MT] (+ [MT] union)
  unsigned long long* walk = masks + (nsb > 1 ? nsb * MT : 0);
  p += (nsb > 1 ? nsb + 1 : 1) * MT * 8;
  float* Ll = (float*)p;
  p += ix.kmax * TILE * 4;
  float* LBl = (float*)p;  // [nsb][kmax]
  p += ix.kmax * nsb * 4;
  p += ix.kmax * 4;
  float* Yl = (float*)p;  // [kmax][64] "yes" thresholds per (k, user)

  // user tile, lower-bound rows and block minima of this block
  if (BF16) {
    const u32x4* src = (const u32x4*)(ix.Qb + B * (int64_t)G * TILE * 8);
    u32x4* dst = (u32x4*)ubuf;
    for (int i = t; i < tile_vecs; i += 256) dst[i] = src[i];
  } else {
    const u32x4* src = (const u32x4*)(ix.Qt + B * (int64_t)d * TILE);
    u32x4* dst = (u32x4*)ubuf;
    for (int i = t; i < d * TILE / 4; i += 256) dst[i] = src[i];
    if (d & 1) ((float*)ubuf)[d * TILE + (t & 63)] = 0.f;  // zero pad row
  }
  // lower bounds L_k(u); after the call's first pass over the item prefix
  // (bounded table) also each user's k-th largest product over it less the
  // bound on any product's error, and the block minima of the larger
  // (Definition 4 and Equation 1 over the longer prefix)
  const int K = bscan_list_len(ix.kmax);
  const float e0 = ix.eps_rel32 * ix.normP[0];
  for (int i = t; i < ix.kmax * TILE; i += 256) {
    const int kk = i / TILE;
    const int64_t uu = B * TILE + (i % TILE);
    float L = ix.L32[(int64_t)kk * ix.n_pad + uu];
    if (bv.lists)
      L = fmaxf(L, f32_down((double)bv.gl_v[uu * K + kk] - (double)(e0 * ix.normQ[uu] + ix.eps_abs)));
    Ll[i] = L;
  }
  for (int i = t; i < ix.kmax * nsb; i += 256)
    LBl[i] = ix.LB[(int64_t)(i % ix.kmax) * ix.nSB + B * nsb + i / ix.kmax];
  if (bv.lists) {
    __syncthreads();
    for (int i = t; i < ix.kmax * nsb; i += 256) {
      const int kk = i % ix.kmax, sb = i / ix.kmax;
      float mn = INFINITY;
      for (int c = sb * ix.bsize; c < (sb + 1) * ix.bsize; ++c) mn = fminf(mn, Ll[kk * TILE + c]);
      LBl[i] = fmaxf(LBl[i], mn);
    }
  }
  // yes threshold of (k, user): exact table -> the float above L (>= theta_k);
  // bounded table -> Lemma 2's bound cs_inflate |u|^ |p_k|^
  for (int i = t; i < ix.kmax * TILE; i += 256) {
    const int kk = i / TILE;
    const float L = ix.L32[(int64_t)kk * ix.n_pad + B * TILE + (i % TILE)];
    Yl[i] = ix.exact ? f32_next_up(L)
                     : (ix.cs_inflate * ix.normQ[B * TILE + (i % TILE)]) *
                           (kk < ix.m ? ix.normP[kk] : INFINITY);
  }
  __syncthreads();

  // Lemma 3 for every query of the chunk and every block b of the tile:
  // query j lives iff cs_inflate * |u_first(b)| * |q_j| >= L^k(b).
  uint32_t c_vis = 0, c_pr = 0;  // per-lane counts (< 2^16 after the wave sum)
  for (int sb = 0; sb < nsb; ++sb) {
    const float csb = ix.cs_inflate * ix.bnorm[B * nsb + sb];
    const float* lbs = LBl + sb * ix.kmax;
    for (int base = T0 * TILE; base < nT * TILE; base += 256) {
      const int j = base + t;
      int kq = 0;
      float nqq = 0.f;
      if (j < nT * TILE) {
        kq = bv.k_s[j];
        nqq = bv.qn_s[j];
      }
      const bool live = kq > 0 && !(ix.use_blocks && csb * nqq < lbs[kq > 0 ? kq - 1 : 0]);
      const unsigned long long m = __ballot(live);
      if (lane == 0 && base + wave * TILE < nT * TILE) masks[sb * MT + (base + wave * TILE) / TILE] = m;
      c_vis += kq > 0;
      c_pr += kq > 0 && !live;
    }
  }
  if (nsb > 1) {
    __syncthreads();
    for (int Tw = T0 + t; Tw < nT; Tw += 256) {
      unsigned long long u = 0ull;
      for (int sb = 0; sb < nsb; ++sb) u |= masks[sb * MT + Tw];
      walk[Tw] = u;
    }
  }
  __syncthreads();

  const int64_t u = B * TILE + uh * 32 + col;  // this lane's user
  const bool valid = u < ix.n;
  const float a_u = ix.eps_rel * ix.normQ[u];
  const int32_t orig_u = valid ? ix.permQ[u] : 0;
  uint32_t c_users = 0, c_rest = 0, c_yes = 0;

  const unsigned char* qsrc = BF16 ? (const unsigned char*)bv.qb : (const unsigned char*)bv.qt;
  // float32: prefetch registers for the next tile (tile bytes + 512 bytes of metadata)
  u32x4 pf[LDSD ? 1 : NV];
  float pf_n = 0.f;
  int32_t pf_k = 0;

  // bounded table: this wave's current pair chunk and its fill
  int ccur = -1, cfill_w = kPairChunk;
  // exact table: this wave's current run of reserved pair slots
  // [erun0, erun0 + erun), of which efill are used
  int64_t erun0 = 0;
  int erun = 0, efill = 0;

  int T = next_live(walk, T0, nT), slot = 0;
  int Tn = next_live(walk, T + 1, nT);
  if constexpr (LDSD) {
    if (T < nT) issue_tile(qsrc, bv, T, tile_bytes, lane, wave, qbuf2[0], meta_n2, meta_k2);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  } else {
    if (T < nT) {
      stage_tile((const u32x4*)qsrc, bv, T, tile_vecs, t, pf, pf_n, pf_k);
      commit_tile(qbuf2[0], meta_n2, meta_k2, tile_vecs, t, pf, pf_n, pf_k);
    }
    __syncthreads();
    if (Tn < nT) stage_tile((const u32x4*)qsrc, bv, Tn, tile_vecs, t, pf, pf_n, pf_k);
  }

  while (T < nT) {
    // small bf16 tiles: the next live tile streams into the other buffer
    // (read last in the previous step, which every wave has finished) while
    // this one is used
    if (LDSD && Tn < nT)
      issue_tile(qsrc, bv, Tn, tile_bytes, lane, wave, qbuf2[slot ^ 1], meta_n2 + (slot ^ 1) * TILE,
                 meta_k2 + (slot ^ 1) * (TILE + 8));
    // (offset from one base, not an array of pointers: the reads stay LDS reads)
    const unsigned char* qbuf = qbuf2[0] + (LDSD ? slot * (int)(qbuf2[1] - qbuf2[0]) : 0);
    const float* meta_n = meta_n2 + slot * TILE;
    const int32_t* meta_k = meta_k2 + slot * (TILE + 8);
    const unsigned long long mask = walk[T];
    // this wave's query half may have no live query at all
    const uint32_t hmask = (uint32_t)(mask >> (qhalf * 32));
    if (hmask != 0u) {
    // ---- scores of the quarter: S[query][user], 32 x 32, one accumulator
    // (a second one alternating over the k-steps measured 1-4% slower).  The
    // first product takes a zero accumulator operand, which clears none.
    const f32x16 zero = {};
    f32x16 acc;
    if (!BF16) {
      const float* qf = (const float*)qbuf + qhalf * 32 + col + half * TILE;
      const float* uf = (const float*)ubuf + uh * 32 + col + half * TILE;
      const int nsteps = d2 / 2;
      int ks = 1;
      if constexpr (NV >= 8) {
        // d > 64 (more than 32 steps): the operands of the next four steps
        // are read before the current four multiply, so that the reads'
        // latency hides behind the products.  The read of the group after
        // the last full one is clamped to that group (read twice, used once),
        // which keeps every read inside the tile and the code free of
        // branches between the reads and their products.
        const int last = nsteps - 4;  // first step of the last full group
        float a0[4], b0[4], a1[4], b1[4];
        const float x0 = qf[0], y0 = uf[0];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          a0[i] = qf[(2 * (1 + i)) * TILE];
          b0[i] = uf[(2 * (1 + i)) * TILE];
        }
        __builtin_amdgcn_sched_barrier(0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(x0, y0, zero, 0, 0, 0);
        for (;;) {
          int kn = min(ks + 4, last);
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            a1[i] = qf[(2 * (kn + i)) * TILE];
            b1[i] = uf[(2 * (kn + i)) * TILE];
          }
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int i = 0; i < 4; ++i) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a0[i], b0[i], acc, 0, 0, 0);
          ks += 4;
          if (ks > last) break;
          kn = min(ks + 4, last);
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            a0[i] = qf[(2 * (kn + i)) * TILE];
            b0[i] = uf[(2 * (kn + i)) * TILE];
          }
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int i = 0; i < 4; ++i) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a1[i], b1[i], acc, 0, 0, 0);
          ks += 4;
          if (ks > last) break;
        }
      } else {
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(qf[0], uf[0], zero, 0, 0, 0);
        for (; ks + 4 <= nsteps; ks += 4) {
          float a[4], b[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            a[i] = qf[(2 * (ks + i)) * TILE];
            b[i] = uf[(2 * (ks + i)) * TILE];
          }
#pragma unroll
          for (int i = 0; i < 4; ++i) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i], b[i], acc, 0, 0, 0);
        }
      }
      for (; ks < nsteps; ++ks)
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(qf[2 * ks * TILE], uf[2 * ks * TILE], acc, 0, 0, 0);
    } else {
      const bf16x8* qv = (const bf16x8*)qbuf + qhalf * 32 + col + half * TILE;
      const bf16x8* uv = (const bf16x8*)ubuf + uh * 32 + col + half * TILE;
      const int nsteps = G / 2;
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(qv[0], uv[0], zero, 0, 0, 0);
      int ks = 1;
      for (; ks + 2 <= nsteps; ks += 2) {
        const bf16x8 a0 = qv[2 * ks * TILE], b0 = uv[2 * ks * TILE];
        const bf16x8 a1 = qv[(2 * ks + 2) * TILE], b1 = uv[(2 * ks + 2) * TILE];
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b0, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b1, acc, 0, 0, 0);
      }
      if (ks < nsteps)
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(qv[2 * ks * TILE], uv[2 * ks * TILE], acc, 0, 0, 0);
    }

    // ---- conservative Lemma 1 pass with the tile half's summary (k_btsum):
    // the largest query norm's margin and one or two lower bounds per user,
    // two vector operations per pair.  It rejects only what the exact test
    // below rejects; the exact tests run only for a wave with a pair it does
    // not reject (or that counts statistics).  Used for tiles of d = 65-128
    // (NV = 4 in bf16, 8 in float32), where it measured 5% faster in both
    // precisions at d = 100; at d = 50 its registers cost the bf16 filter a
    // wave per SIMD (6-7% slower in both precisions), and at d = 200 with k ~
    // U{1..50} too many tile halves hold several k's (2-9% slower).
    constexpr bool FASTL1 = BF16 ? NV == 4 : NV == 8;
    bool flag = true;
    if constexpr (FASTL1) {
      const int4 sm = *(const int4*)(meta_k + TILE + 4 * qhalf);
      const int uc = uh * 32 + col;
      const float e = fmaf(a_u, __int_as_float(sm.x), ix.eps_abs);
      const float Lhi = Ll[sm.z + uc];
      if (sm.w == 0) {
        // rounding is monotone, so every acc[r] + e < Lhi iff the largest does
        float mx = acc[0];
#pragma unroll
        for (int r = 1; r < 16; ++r) mx = fmaxf(mx, acc[r]);
        flag = !(mx + e < Lhi);
      } else if (sm.w > 0) {
        const float Llo = Ll[sm.y + uc];
        bool fl = false;
#pragma unroll
        for (int r = 0; r < 16; ++r)
          fl |= !(acc[r] + e < ((r / 4) * 8 + half * 4 + (r % 4) >= sm.w ? Lhi : Llo));
        flag = fl;
      }
      flag = flag && valid;
    }
    if (!FASTL1 || bv.ctr || __ballot(flag)) {
      // ---- certified tests.  Lemma 1: "no" iff s + e < L.  "Yes" iff
      // s - e >= Y, with Y the float above L (exact table: f >= theta_k) or
      // the Cauchy-Schwarz bound of the k-th item (Lemma 2), both per (k,
      // user) in LDS.  e = eps|u||q| + eps_abs; both tests round relative to
      // |u||q|, which the slack inside eps covers.
      // the lane's rows are qhalf*32 + g*8 + half*4 + i  (r = 4g + i)
      // the rows live for this lane's own block (blocks of fewer than 64 users)
      const uint32_t hm = (nsb > 1 ? (uint32_t)(masks[((uh * 32 + col) / ix.bsize) * MT + T] >> (qhalf * 32))
                                   : hmask) >> (half * 4);
      const uint32_t cells = (hm & 0xFu) | ((hm >> 4) & 0xF0u) | ((hm >> 8) & 0xF00u) |
                             ((hm >> 12) & 0xF000u);
      const int ucol = uh * 32 + col;
      uint32_t rest = 0;
  #pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int rb = quarter_row(qhalf, half, g * 4);
        const float4 n4 = *(const float4*)(meta_n + rb);
        const int4 k4 = *(const int4*)(meta_k + rb);
        const float nqs[4] = {n4.x, n4.y, n4.z, n4.w};
        const int kks[4] = {k4.x, k4.y, k4.z, k4.w};
  #pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int r = g * 4 + i;
          const float ev = fmaf(a_u, nqs[i], ix.eps_abs);
          const float L = Ll[kks[i] + ucol];
          rest |= (uint32_t)!(acc[r] + ev < L) << r;
        }
      }
      rest &= valid ? cells : 0u;
      uint32_t yes = 0;
      if (__ballot(rest != 0u)) {  // some pair Lemma 1 did not reject: the "yes" test
        // small float32 tiles: the rows' norms and k's are read again here
        // instead of held in registers since the Lemma 1 test (an opaque row
        // offset keeps the compiler from reusing those loads), so that the
        // 4-wave register budget needs no spill: a spilled address reloaded
        // before the products waited for the next tile's loads (5% faster).
        // Larger tiles keep them (1-2% faster).
        int rq = quarter_row(qhalf, half, 0);
        if constexpr (!BF16 && NV <= 4) asm volatile("" : "+v"(rq));
  #pragma unroll
        for (int g = 0; g < 4; ++g) {
          const int rb = rq + g * 8;
          const float4 n4 = *(const float4*)(meta_n + rb);
          const int4 k4 = *(const int4*)(meta_k + rb);
          const float nqs[4] = {n4.x, n4.y, n4.z, n4.w};
          const int kks[4] = {k4.x, k4.y, k4.z, k4.w};
  #pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int r = g * 4 + i;
            const float ev = fmaf(a_u, nqs[i], ix.eps_abs);
            const float Y = Yl[kks[i] + ucol];
            yes |= (uint32_t)(acc[r] - ev >= Y) << r;
          }
        }
        yes &= rest;
      }
      const uint32_t und = rest & ~yes;
      if (bv.ctr) {
        c_users += valid ? __popc(cells) : 0;
        c_rest += __popc(rest);
        c_yes += __popc(yes);
      }
      // ---- certified members: result bits and counts.  The wave goes over
      // the rows that hold any result (a lane's row r is row
      // (r/4)*8 + half*4 + r%4 of the quarter; lane l < 32 loads the
      // caller-order index of row l once), with one count update per row and
      // wave half instead of one per result, which the row's lanes would all
      // make to one address.  Same-box A/B: 50k users x 10k items, 312 ->
      // 270 us per 4,096 queries; 100k x 20k in bf16, 277 -> 216 us per
      // 4,000; 500k x 50k at d = 200 in bf16 (fewer results per row) 2%
      // slower.
      if (__ballot(yes != 0u)) {
        const int32_t jrow = bv.perm[(int64_t)T * TILE + qhalf * 32 + (lane & 31)];
        uint32_t any = yes;
        for (int off = 32; off > 0; off >>= 1) any |= __shfl_xor(any, off);
        while (any) {
          const int r = __ffs(any) - 1;
          any &= any - 1;
          const unsigned long long b = __ballot((yes >> r) & 1u);
          const int32_t jo = __shfl(jrow, (r / 4) * 8 + half * 4 + (r % 4));
          if ((yes >> r) & 1u) atomicOr(&bv.bits[(int64_t)jo * bv.W + (orig_u >> 5)], 1u << (orig_u & 31));
          const uint32_t c = __popc(half ? (uint32_t)(b >> 32) : (uint32_t)b);
          if (col == 0 && c) atomicAdd(&bv.counts[jo], (unsigned long long)c);
        }
      }
      // ---- undecided pairs: appended (one atomic per wave).  Exact table:
      // one flat list.  Bounded table: the wave fills chunks of its own, each
      // registered in the block's chunk list, so that the scan finds the
      // block's pairs together.
      if (__ballot(und != 0u)) {
        const int cnt = __popc(und);
        const int incl = wave_incl_scan(cnt);
        uint32_t ovf = 0;  // pairs beyond the list's capacity
        if (ix.exact) {
          // slots come from the wave's run of reserved slots, and a new run
          // only when it is used up: the returning atomic's wait covers every
          // load in flight, the next tile's prefetch included (vector memory
          // returns in order), so one per tile with such pairs cost the bf16
          // filter 11-21%
          const int total = __builtin_amdgcn_readlane(incl, 63);
          const int avail = erun - efill;
          int need = 0;
          int64_t nb = 0;
          if (total > avail) {
            need = (total - avail + kExactRun - 1) / kExactRun * kExactRun;
            unsigned long long got = 0;
            if (lane == 0) got = atomicAdd(bv.npairs, (unsigned long long)need);
            const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)got, 0);
            const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(got >> 32), 0);
            nb = (int64_t)(((uint64_t)hi << 32) | lo);
          }
          int p = incl - cnt;
  #pragma unroll
          for (int r = 0; r < 16; ++r) {
            if ((und >> r) & 1u) {
              const int64_t pos = p < avail ? erun0 + efill + p : nb + (p - avail);
              ++p;
              if (pos < bv.pair_cap) {
                bv.pair_u[pos] = (int32_t)u;
                bv.pair_j[pos] = (int32_t)((int64_t)T * TILE + quarter_row(qhalf, half, r));
                bv.pair_s[pos] = acc[r];
              } else {
                ovf |= 1u << r;
              }
            }
          }
          if (need > 0) {
            erun0 = nb;
            erun = need;
            efill = total - avail;
          } else {
            efill += total;
          }
        } else {
          const int total = __builtin_amdgcn_readlane(incl, 63);
          const int avail = kPairChunk - cfill_w;  // free slots of the current chunk
          const int need = total > avail ? (total - avail + kPairChunk - 1) / kPairChunk : 0;
          int nb = 0;
          if (need > 0) {
            if (lane == 0) nb = atomicAdd(bv.nchunks, need);
            nb = __builtin_amdgcn_readlane(nb, 0);
            if (lane < need && nb + lane < bv.chunk_cap) {
              bv.cfill[nb + lane] = kPairChunk;  // the last one is corrected at the end
              const int at = atomicAdd(&bv.bcnt[B], 1);
              bv.bchunks[B * bv.maxc + at] = nb + lane;
            }
          }
          int p = incl - cnt;  // this lane's first pair within the wave's append
  #pragma unroll
          for (int r = 0; r < 16; ++r) {
            if ((und >> r) & 1u) {
              int c, slot;
              if (p < avail) {
                c = ccur;
                slot = cfill_w + p;
              } else {
                c = nb + (p - avail) / kPairChunk;
                slot = (p - avail) % kPairChunk;
              }
              if (c < bv.chunk_cap) {
                const int64_t pos = (int64_t)c * kPairChunk + slot;
                bv.pair_u[pos] = (int32_t)u;
                bv.pair_j[pos] = (int32_t)((int64_t)T * TILE + quarter_row(qhalf, half, r));
                bv.pair_s[pos] = acc[r];
              } else {
                ovf |= 1u << r;
              }
              ++p;
            }
          }
          if (need > 0) {
            ccur = nb + need - 1;
            cfill_w = total - avail - (need - 1) * kPairChunk;
          } else {
            cfill_w += total;
          }
        }
        while (ovf) {  // rare: decide in float64 here
          const int r = __ffs(ovf) - 1;
          ovf &= ovf - 1;
          const int32_t jj = (int32_t)((int64_t)T * TILE + quarter_row(qhalf, half, r));
          if (decide_f64(ix, bv, u, jj)) {
            const int32_t jo = bv.perm[jj];
            atomicOr(&bv.bits[(int64_t)jo * bv.W + (orig_u >> 5)], 1u << (orig_u & 31));
            atomicAdd(&bv.counts[jo], 1ull);
          }
          // this path's loads are all complete here: without the explicit
          // wait the compiler's analysis keeps them pending around the tile
          // loop and waits for every load before the next tile's products,
          // the prefetched tile's included
          __builtin_amdgcn_s_waitcnt(0);
        }
      }
    }  // exact tests

    }  // hmask

    // ---- next tile: small bf16 tiles landed in the other buffer; others
    // from the prefetch registers into the one buffer
    if constexpr (LDSD) {
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      T = Tn;
      Tn = next_live(walk, T + 1, nT);
      slot ^= 1;
    } else {
      __syncthreads();
      if (Tn < nT) commit_tile(qbuf2[0], meta_n2, meta_k2, tile_vecs, t, pf, pf_n, pf_k);
      T = Tn;
      Tn = next_live(walk, T + 1, nT);
      __syncthreads();
      if (Tn < nT) stage_tile((const u32x4*)qsrc, bv, Tn, tile_vecs, t, pf, pf_n, pf_k);
    }
  }
  if (!ix.exact && lane == 0 && ccur >= 0 && ccur < bv.chunk_cap) bv.cfill[ccur] = cfill_w;
  // exact table: the unused end of the wave's last run holds no pair
  if (ix.exact)
    for (int i = efill + lane; i < erun; i += 64)
      if (erun0 + i < bv.pair_cap) bv.pair_u[erun0 + i] = -1;

  if (bv.ctr) {
    for (int off = 32; off > 0; off >>= 1) {
      c_users += __shfl_xor(c_users, off);
      c_rest += __shfl_xor(c_rest, off);
      c_yes += __shfl_xor(c_yes, off);
      c_vis += __shfl_xor(c_vis, off);
      c_pr += __shfl_xor(c_pr, off);
    }
    if (lane == 0) {
      atomicAdd(&bv.ctr[C_BLOCKS], (unsigned long long)c_vis);
      atomicAdd(&bv.ctr[C_PRUNED], (unsigned long long)c_pr);
      atomicAdd(&bv.ctr[C_USERS], (unsigned long long)c_users);
      atomicAdd(&bv.ctr[C_L1NO], (unsigned long long)(c_users - c_rest));
      atomicAdd(&bv.ctr[ix.exact ? C_TYES : C_L2YES], (unsigned long long)c_yes);
      atomicAdd(&bv.ctr[ix.exact ? C_RCHK : C_SURV], (unsigned long long)(c_rest - c_yes));
    }
  }
}

// ---------------------------------------------------------------------------
// Undecided pairs of the exact table: float64 f(q,u) against theta_k, one
// lane per pair.  (The bounded table's pairs go to the grouped linear scan,
// scan_kernels.hip.)  Most slots of the list are unused ends of the filter
// waves' reserved runs, so a wave reads 64 slots at a time and queues the
// used ones in LDS, deciding 64 pairs with all lanes whenever it holds that
// many (and the rest at its end): one lane per slot left most lanes idle
// through the float64 products.  1M x 100k: bf16 (214k pairs) 216 -> 163
// us, float32 (34k pairs) 81 -> 70 us; 500k x 50k at d = 200 in bf16 4%
// slower.
__device__ __forceinline__ bool decide_exact_pair(const DevIndex& ix, const BatchView& bv, int64_t t) {
  const int64_t r = bv.pair_u[t];
  const int64_t jj = bv.pair_j[t];
  const int32_t jo = bv.perm[jj];
  const float* x = bv.qs + (int64_t)jo * ix.d;
  const float* y = ix.Qrow + r * ix.d;
  // rows of 16-byte aligned float4s take a quarter of the load instructions
  const double fq = ((ix.d & 3) == 0 && (((uintptr_t)x | (uintptr_t)y) & 15) == 0)
                        ? dot64_rows4((const float4*)x, (const float4*)y, ix.d / 4)
                        : dot64_rows(x, y, ix.d);
  const int k = bv.k_s[jj];
  if (fq >= ix.L64[(int64_t)(k - 1) * ix.n_pad + r]) {
    set_pair_result(bv, ix, r, jo);
    return true;
  }
  return false;
}

__global__ void __launch_bounds__(256) k_brecheck_exact(DevIndex ix, BatchView bv) {
  __shared__ int32_t queue[4][2 * TILE];  // per wave: slots of used pairs, at most 127
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int32_t* q = queue[wave];
  const int64_t np = (int64_t)min(*bv.npairs, (unsigned long long)bv.pair_cap);
  const int64_t nw = (int64_t)gridDim.x * 4;
  unsigned long long yes_count = 0;
  int qn = 0;  // queued slots (wave-uniform)
  for (int64_t base = ((int64_t)blockIdx.x * 4 + wave) * TILE; base < np; base += nw * TILE) {
    const int64_t t = base + lane;
    const bool used = t < np && bv.pair_u[t] >= 0;
    const unsigned long long m = __ballot(used);
    if (used) q[qn + __popcll(m & lanemask_lt_b())] = (int32_t)t;
    qn += __popcll(m);
    __builtin_amdgcn_wave_barrier();
    if (qn >= TILE) {
      yes_count += decide_exact_pair(ix, bv, q[lane]);
      const int rest = qn - TILE;
      const int32_t v = lane < rest ? q[TILE + lane] : 0;
      __builtin_amdgcn_wave_barrier();
      if (lane < rest) q[lane] = v;
      qn = rest;
      __builtin_amdgcn_wave_barrier();
    }
  }
  if (lane < qn) yes_count += decide_exact_pair(ix, bv, q[lane]);
  if (bv.ctr && yes_count) atomicAdd(&bv.ctr[C_TYES], yes_count);
}

// ---------------------------------------------------------------------------
// CSR assembly.  Offsets: one workgroup scans the chunk's counts (original
// chunk order) starting from *base.  Ids: one wave per query turns its
// bitmap row into ascending ids, then clears the row and the count.
__global__ void __launch_bounds__(1024) k_boffsets(const unsigned long long* __restrict__ counts,
                                                const uint8_t* __restrict__ all, int64_t n,
                                                int32_t nq, const int64_t* __restrict__ base,
                                                int64_t* __restrict__ offs) {
  __shared__ int64_t part[1024];
  const int t = threadIdx.x;
  const int i0 = (int)((int64_t)nq * t / 1024), i1 = (int)((int64_t)nq * (t + 1) / 1024);
  int64_t c = 0;
  for (int i = i0; i < i1; ++i) c += all[i] ? n : (int64_t)counts[i];
  part[t] = c;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    int64_t v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int64_t run = *base + part[t] - c;
  for (int i = i0; i < i1; ++i) {
    run += all[i] ? n : (int64_t)counts[i];
    offs[i + 1] = run;  // offs[0] is *base, written by the previous chunk
  }
}

__global__ void __launch_bounds__(256) k_bassemble(BatchView bv, int32_t nq,
                                                   const int64_t* __restrict__ offs,
                                                   int32_t* __restrict__ ids, int64_t cap) {
  // One wave per query, one pass over its bitmap row (W words, a multiple of
  // 4) in rounds of G groups of 64 vectors, all loaded at once: lane L holds
  // vector 64 g + L of each group, so with the groups in order and the lanes
  // in order within a group the ids come out ascending.  Words that held
  // bits are cleared.
  const int lane = threadIdx.x & 63;
  const int32_t j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= nq) return;
  u32x4* row = (u32x4*)(bv.bits + (int64_t)j * bv.W);
  const int64_t nv = bv.W / 4;
  constexpr int G = 16, GS = 4;
  u32x4 xs[G];
  auto load = [&](int64_t v00) {
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int64_t v = v00 + 64 * g + lane;
      xs[g] = u32x4{0u, 0u, 0u, 0u};
      if (v < nv) xs[g] = row[v];
    }
  };
  load(0);  // in flight with the query's flag and offset
  const int64_t start = offs[j];
  if (bv.all[j]) {  // k > m: every user, ascending
    for (int64_t i = lane; i < bv.n && start + i < cap; i += 64) ids[start + i] = (int32_t)i;
    if (lane == 0 && bv.ctr) atomicAdd(&bv.ctr[C_RES], (unsigned long long)bv.n);
    return;
  }
  int64_t pos = start;
  for (int64_t v00 = 0; v00 < nv; v00 += 64 * G) {
    if (v00 > 0) load(v00);
#pragma unroll
    for (int g0 = 0; g0 < G; g0 += GS) {  // scans of GS groups at a time
    int cnt[GS], incl[GS];
#pragma unroll
    for (int h = 0; h < GS; ++h) {
      const u32x4 x = xs[g0 + h];
      cnt[h] = __popc(x[0]) + __popc(x[1]) + __popc(x[2]) + __popc(x[3]);
      incl[h] = wave_incl_scan(cnt[h]);
    }
#pragma unroll
    for (int h = 0; h < GS; ++h) {
      const int g = g0 + h;
      const int tot = __builtin_amdgcn_readlane(incl[h], 63);
      if (tot == 0) continue;
      if (cnt[h]) {
        const int64_t v = v00 + 64 * g + lane;
        row[v] = u32x4{0u, 0u, 0u, 0u};
        int64_t p = pos + incl[h] - cnt[h];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          uint32_t bits = xs[g][q];
          while (bits) {
            const int b = __ffs(bits) - 1;
            bits &= bits - 1;
            if ((uint64_t)p < (uint64_t)cap) ids[p] = (int32_t)((4 * v + q) * 32 + b);
            ++p;
          }
        }
      }
      pos += tot;
    }
    }
  }
  if (lane == 0) {
    if (bv.ctr) atomicAdd(&bv.ctr[C_RES], (unsigned long long)(pos - start));
    bv.counts[j] = 0ull;
  }
}

// p[0..n) = v: clears flags, counters and carried state in stream order.
__global__ void k_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

void launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
  if (n <= 0) return;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
}

// Bounded table: empty chunk lists before the filter.
__global__ void k_bclear(int32_t* __restrict__ bcnt, int32_t nB, int32_t* __restrict__ nchunks,
                         int32_t* __restrict__ sg_block, int32_t* __restrict__ sg_count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nB) {
    bcnt[i] = 0;
    sg_block[i] = 0;
  }
  if (i == 0) {
    *nchunks = 0;
    sg_count[0] = 0;
    sg_count[1] = 0;
  }
}

// ---------------------------------------------------------------------------
void launch_bprep(const DevIndex& ix, const BatchView& bv, const int32_t* ks_dev, int32_t nq,
                  hipStream_t s) {
  hipLaunchKernelGGL(k_bnorms, dim3((nq + 3) / 4), dim3(256), 0, s, bv.qs, nq, ix.d, bv.qn,
                     bv.npairs);
  if (!ix.exact && ix.nB > 0)
    hipLaunchKernelGGL(k_bclear, dim3((ix.nB + 255) / 256), dim3(256), 0, s, bv.bcnt, ix.nB,
                       bv.nchunks, bv.sg_block, bv.sg_count);
  hipLaunchKernelGGL(k_bsort, dim3(1), dim3(1024), (size_t)(ix.kmax + 1) * kSortBuckets * 4, s,
                     bv.qn, ks_dev, nq, ix.kmax, bv.perm);
  dim3 blk(64, 4);
  hipLaunchKernelGGL(k_btile, dim3((bv.nq_pad + 3) / 4), blk, 0, s, bv.qs, ks_dev, bv.qn,
                     bv.perm, nq, bv.nq_pad, ix.d, ix.d16, ix.m, bv.qt, ix.bf16 ? bv.qb : nullptr,
                     bv.qn_s, bv.k_s, bv.kofs_s, bv.all);
  hipLaunchKernelGGL(k_btsum, dim3(bv.nq_pad / TILE), dim3(64), 0, s, bv.qn_s, bv.kofs_s, bv.tsum);
}

size_t bfilter_lds_bytes(const DevIndex& ix) {
  const size_t tile = ix.bf16 ? (size_t)(ix.d16 / 8) * TILE * 16 : (size_t)(ix.d + (ix.d & 1)) * TILE * 4;
  const bool ldsd = ix.bf16 && (tile / 16 + 255) / 256 <= 2;  // the kernel's direct-load case (NV <= 2)
  const size_t nsb = TILE / ix.bsize;
  return (ldsd ? 3 : 2) * ((tile + 15) / 16 * 16) + 4 * TILE * 4 + 2 * 8 * 4 +
         (nsb > 1 ? nsb + 1 : 1) * (kBatchChunkMax / TILE) * 8 + 2 * (size_t)ix.kmax * TILE * 4 +
         (size_t)ix.kmax * 4 * (nsb + 1);
}

// Largest query tile the filter's prefetch registers hold.
size_t bfilter_max_tile_bytes() { return (size_t)PF_VEC * 256 * 16; }

// Workgroup slots of the device for a kernel and its dynamic LDS (resident
// workgroups per CU x CUs), cached per device for the last LDS size asked;
// 0 if the runtime cannot tell.
constexpr int kSlotDevices = 64;
static int64_t device_slots(const void* f, size_t lds, std::atomic<uint64_t>* cache) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kSlotDevices) return 0;
  const uint64_t key = (uint64_t)lds << 24;
  const uint64_t c = cache[dev].load(std::memory_order_relaxed);
  if (c != 0 && (c & ~0xFFFFFFull) == key) return (int64_t)(c & 0xFFFFFFull);
  int occ = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, f, 256, lds) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  const int64_t slots = std::min<int64_t>((int64_t)occ * cus, 0xFFFFFF);
  cache[dev].store(key | (uint64_t)slots, std::memory_order_relaxed);
  return slots;
}

template <bool BF16, int NV>
static void bfilter_nv(const DevIndex& ix, const BatchView& bv0, size_t lds, hipStream_t s) {
  static std::atomic<uint64_t> slots_cache[kSlotDevices];
  const void* f = (const void*)k_bfilter<BF16, NV>;
  if (lds > 65536) (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  BatchView bv = bv0;
  // exact table: split the query tiles of a catalog with few blocks (the
  // bounded table keeps one workgroup per block: its pair chunks are listed
  // per block by the block's own waves)
  bv.qsplit = ix.exact ? bfilter_qsplit(ix.nB, bv.nq_pad / TILE, device_slots(f, lds, slots_cache)) : 1;
  hipLaunchKernelGGL((k_bfilter<BF16, NV>), dim3((unsigned)(ix.nB * bv.qsplit)), dim3(256), lds, s, ix,
                     bv);
}

template <bool BF16>
static void bfilter_prec(const DevIndex& ix, const BatchView& bv, size_t lds, hipStream_t s) {
  const size_t tile = BF16 ? (size_t)(ix.d16 / 8) * TILE * 16 : (size_t)(ix.d + (ix.d & 1)) * TILE * 4;
  const size_t per_thread = (tile / 16 + 255) / 256;  // 16-byte vectors per thread
  if (per_thread <= 2) bfilter_nv<BF16, 2>(ix, bv, lds, s);
  else if (per_thread <= 4) bfilter_nv<BF16, 4>(ix, bv, lds, s);
  else if (per_thread <= 8) bfilter_nv<BF16, 8>(ix, bv, lds, s);
  else bfilter_nv<BF16, 16>(ix, bv, lds, s);
}

void launch_bfilter(const DevIndex& ix, const BatchView& bv, hipStream_t s) {
  if (ix.nB == 0) return;
  const size_t lds = bfilter_lds_bytes(ix);
  if (ix.bf16) bfilter_prec<true>(ix, bv, lds, s);
  else bfilter_prec<false>(ix, bv, lds, s);
}

void launch_bpairs(const DevIndex& ix, const BatchView& bv, hipStream_t s) {
  if (ix.nB == 0) return;
  if (ix.exact) {
    // grid-stride over the used part of the list (the reserved runs leave
    // unused slots, marked -1, between the pairs)
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((bv.pair_cap + 255) / 256, 2048));
    hipLaunchKernelGGL(k_brecheck_exact, dim3((unsigned)blocks), dim3(256), 0, s, ix, bv);
    return;
  }
  launch_bscan(ix, bv, s);
}

void launch_bassemble(const BatchView& bv, int32_t nq, const int64_t* base, int64_t* offs,
                      int32_t* ids, int64_t cap, hipStream_t s) {
  hipLaunchKernelGGL(k_boffsets, dim3(1), dim3(1024), 0, s, bv.counts, bv.all, bv.n, nq, base, offs);
  hipLaunchKernelGGL(k_bassemble, dim3((nq + 3) / 4), dim3(256), 0, s, bv, nq, offs, ids, cap);
}

}  // namespace rk
