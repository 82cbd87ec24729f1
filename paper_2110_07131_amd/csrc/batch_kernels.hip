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
#include "rk_batch.h"

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

namespace rk {

__device__ __forceinline__ unsigned long long lanemask_lt_b() {
  const int lane = threadIdx.x & 63;
  return lane ? (~0ull >> (64 - lane)) : 0ull;
}

// ---------------------------------------------------------------------------
// Per query of the chunk: |q| rounded up (one wave per query).
__global__ void k_bnorms(const float* __restrict__ qs, int32_t nq, int32_t d,
                         float* __restrict__ qn, int32_t* __restrict__ npairs) {
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

// Single workgroup bitonic sort of the chunk's queries by descending norm
// (ties by index); writes the sorted order perm[0..nq).
__global__ void __launch_bounds__(1024) k_bsort(const float* __restrict__ qn, int32_t nq,
                                                int32_t* __restrict__ perm) {
  __shared__ float key[kBatchChunkMax];
  __shared__ int32_t idx[kBatchChunkMax];
  int P2 = 1;
  while (P2 < nq) P2 <<= 1;
  for (int i = threadIdx.x; i < P2; i += blockDim.x) {
    key[i] = i < nq ? qn[i] : -INFINITY;
    idx[i] = i < nq ? i : INT32_MAX;
  }
  __syncthreads();
  for (int size = 2; size <= P2; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < P2; i += blockDim.x) {
        const int pj = i ^ stride;
        if (pj > i) {
          const bool desc = (i & size) == 0;
          // "a before b" in the final order: larger key, then smaller index
          const bool i_first = key[i] > key[pj] || (key[i] == key[pj] && idx[i] < idx[pj]);
          if (desc != i_first) {
            float tk = key[i]; key[i] = key[pj]; key[pj] = tk;
            int32_t ti = idx[i]; idx[i] = idx[pj]; idx[pj] = ti;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < nq; i += blockDim.x) perm[i] = idx[i];
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
                        uint8_t* __restrict__ all) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.y + threadIdx.y;
  if (r >= nq_pad) return;
  const bool valid = r < nq;
  const int64_t src = valid ? perm[r] : 0;
  for (int c = threadIdx.x; c < d; c += blockDim.x) qt[tix(r, c, d)] = valid ? qs[src * d + c] : 0.0f;
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
    if (valid) all[src] = k > m ? 1 : 0;
  }
}

// ---------------------------------------------------------------------------
// Exact float64 decision of one (user, query) pair, used by a lane whose
// undecided pair does not fit the pair list: with an exact table f(q,u)
// against theta_k; otherwise the float64 linear scan (Algorithm 2).
__device__ bool decide_f64(const DevIndex& ix, const BatchView& bv, int64_t r, int32_t jj) {
  const int32_t jo = bv.perm[jj];
  const int k = bv.k_s[jj];
  const float* q = bv.qs + (int64_t)jo * ix.d;
  const float* u = ix.Qt + (r / TILE) * (int64_t)ix.d * TILE + (r % TILE);
  double fq = 0.0;
  for (int c = 0; c < ix.d; ++c) fq = fma((double)q[c], (double)u[(int64_t)c * TILE], fq);
  if (ix.exact) return fq >= ix.L64[(int64_t)(k - 1) * ix.n_pad + r];
  const double csu = (double)ix.cs_inflate * (double)ix.normQ[r] * (1.0 + 0x1p-50);
  int beats = 0;
  for (int64_t j = 0; j < ix.m && beats < k; ++j) {
    if (csu * (double)ix.normP[j] <= fq) break;
    const float* p = ix.Prow + j * ix.d;
    double fp = 0.0;
    for (int c = 0; c < ix.d; ++c) fp = fma((double)p[c], (double)u[(int64_t)c * TILE], fp);
    beats += fp > fq;
  }
  return beats < k;
}

// ---------------------------------------------------------------------------
// The batched filter.  Workgroup = 4 waves = one user block B; wave w takes
// query tiles w, w+4, ...  Per tile: Lemma 3 for each of its 64 queries
// (lane = query) gives a 64-bit mask of the queries that keep the block;
// an all-zero mask skips the tile.  Otherwise the 64x64 score tile S[query][user]
// is formed by four 32x32 MFMA blocks (A = queries, B = users), so a lane
// holds two users (its column in both user halves) and 16 queries per half.
template <bool BF16>
__global__ void __launch_bounds__(256) k_bfilter(DevIndex ix, BatchView bv) {
  extern __shared__ float lds[];
  const int d = ix.d;
  const int64_t B = blockIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int half = lane >> 5, col = lane & 31;
  // LDS: user tile (fp32 [d][64] or bf16 [G][64][8]), L32 rows [kmax][64],
  // LB column [kmax], |p_k| [kmax]
  const int G = ix.d16 / 8;
  const size_t ubytes = BF16 ? (size_t)G * TILE * 8 * 2 : (size_t)d * TILE * 4;
  float* uA = lds;
  uint16_t* uB = (uint16_t*)lds;
  float* Ll = (float*)((char*)lds + ubytes);
  float* LBl = Ll + ix.kmax * TILE;
  float* npk = LBl + ix.kmax;
  if (BF16) {
    const uint4* src = (const uint4*)(ix.Qb + B * (int64_t)G * TILE * 8);
    uint4* dst = (uint4*)uB;
    for (int i = threadIdx.x; i < G * TILE; i += blockDim.x) dst[i] = src[i];
  } else {
    const float* src = ix.Qt + B * (int64_t)d * TILE;
    for (int i = threadIdx.x; i < d * TILE; i += blockDim.x) uA[i] = src[i];
  }
  for (int i = threadIdx.x; i < ix.kmax * TILE; i += blockDim.x)
    Ll[i] = ix.L32[(int64_t)(i / TILE) * ix.n_pad + B * TILE + (i % TILE)];
  for (int i = threadIdx.x; i < ix.kmax; i += blockDim.x) {
    LBl[i] = ix.LB[(int64_t)i * ix.nB + B];
    npk[i] = i < ix.m ? ix.normP[i] : 0.0f;
  }
  __syncthreads();

  const float bn = ix.bnorm[B];
  const float csb = ix.cs_inflate * bn;
  // the lane's two users
  const int64_t u0 = B * TILE + col, u1 = u0 + 32;
  const bool v0 = u0 < ix.n, v1 = u1 < ix.n;
  const float nu0 = ix.normQ[u0], nu1 = ix.normQ[u1];
  const float a0 = ix.eps_rel * nu0, a1 = ix.eps_rel * nu1;
  const float c0 = ix.cs_inflate * nu0, c1 = ix.cs_inflate * nu1;
  const int32_t o0 = v0 ? ix.permQ[u0] : 0, o1 = v1 ? ix.permQ[u1] : 0;
  const int nT = bv.nq_pad / TILE;
  unsigned long long c_vis = 0, c_pr = 0, c_users = 0, c_no1 = 0, c_yes2 = 0, c_yesT = 0, c_und = 0;

  for (int T = wave; T < nT; T += 4) {
    // Lemma 3 for query T*64 + lane
    const int64_t jq = (int64_t)T * TILE + lane;
    const int kq = bv.k_s[jq];
    const float nqq = bv.qn_s[jq];
    const bool live = kq > 0 && !(csb * nqq < LBl[kq > 0 ? kq - 1 : 0]);
    const unsigned long long mask = __ballot(live);
    c_vis += __popcll(__ballot(kq > 0));
    c_pr += __popcll(__ballot(kq > 0 && !live));
    if (!mask) continue;

    f32x16 acc00 = {}, acc01 = {}, acc10 = {}, acc11 = {};  // [query half][user half]
    if (!BF16) {
      const float* qt = bv.qt + (int64_t)T * d * TILE;
      for (int ks = 0; ks < (d + 1) / 2; ++ks) {
        const int c = 2 * ks + half;
        float qa0 = 0.f, qa1 = 0.f, ub0 = 0.f, ub1 = 0.f;
        if (c < d) {
          qa0 = qt[c * TILE + col];
          qa1 = qt[c * TILE + 32 + col];
          ub0 = uA[c * TILE + col];
          ub1 = uA[c * TILE + 32 + col];
        }
        acc00 = __builtin_amdgcn_mfma_f32_32x32x2f32(qa0, ub0, acc00, 0, 0, 0);
        acc01 = __builtin_amdgcn_mfma_f32_32x32x2f32(qa0, ub1, acc01, 0, 0, 0);
        acc10 = __builtin_amdgcn_mfma_f32_32x32x2f32(qa1, ub0, acc10, 0, 0, 0);
        acc11 = __builtin_amdgcn_mfma_f32_32x32x2f32(qa1, ub1, acc11, 0, 0, 0);
      }
    } else {
      const uint4* qb = (const uint4*)(bv.qb + (int64_t)T * G * TILE * 8);
      const uint4* ub = (const uint4*)uB;
      for (int ks = 0; ks < G / 2; ++ks) {
        const int g = 2 * ks + half;
        const uint4 x0 = qb[g * TILE + col], x1 = qb[g * TILE + 32 + col];
        const uint4 y0 = ub[g * TILE + col], y1 = ub[g * TILE + 32 + col];
        bf16x8 qa0, qa1, ub0, ub1;
        __builtin_memcpy(&qa0, &x0, 16);
        __builtin_memcpy(&qa1, &x1, 16);
        __builtin_memcpy(&ub0, &y0, 16);
        __builtin_memcpy(&ub1, &y1, 16);
        acc00 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(qa0, ub0, acc00, 0, 0, 0);
        acc01 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(qa0, ub1, acc01, 0, 0, 0);
        acc10 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(qa1, ub0, acc10, 0, 0, 0);
        acc11 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(qa1, ub1, acc11, 0, 0, 0);
      }
    }

    // Epilogue: lane holds queries (r/4)*8 + half*4 + r%4 (+32 for the second
    // query half) against users col and 32 + col.
#pragma unroll
    for (int qh = 0; qh < 2; ++qh) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = qh * 32 + (r / 4) * 8 + half * 4 + (r % 4);
        const bool cell = (mask >> row) & 1ull;
        const int64_t jj = (int64_t)T * TILE + row;  // sorted query position
        const int kk = cell ? bv.k_s[jj] : 1;
        const float nqj = cell ? bv.qn_s[jj] : 0.f;
        const float Lk0 = Ll[(kk - 1) * TILE + col], Lk1 = Ll[(kk - 1) * TILE + 32 + col];
        const float s0 = qh ? acc10[r] : acc00[r];
        const float s1 = qh ? acc11[r] : acc01[r];
        const float e0 = fmaf(a0, nqj, ix.eps_abs), e1 = fmaf(a1, nqj, ix.eps_abs);
        const bool x0 = cell && v0, x1 = cell && v1;
        const bool no0 = x0 && (s0 + e0 < Lk0), no1 = x1 && (s1 + e1 < Lk1);
        const bool rest0 = x0 && !no0, rest1 = x1 && !no1;
        if (bv.ctr) {
          c_users += (unsigned)x0 + (unsigned)x1;
          c_no1 += (unsigned)no0 + (unsigned)no1;
        }
        if (__ballot(rest0 || rest1) == 0ull) continue;
        const float pk = npk[kk - 1];
        const bool y20 = rest0 && (s0 - e0 >= c0 * pk);
        const bool y21 = rest1 && (s1 - e1 >= c1 * pk);
        const bool yT0 = rest0 && !y20 && ix.exact && (s0 - e0 >= f32_next_up(Lk0));
        const bool yT1 = rest1 && !y21 && ix.exact && (s1 - e1 >= f32_next_up(Lk1));
        const bool un0 = rest0 && !y20 && !yT0, un1 = rest1 && !y21 && !yT1;
        const int32_t jo = (y20 || yT0 || y21 || yT1 || un0 || un1) ? bv.perm[jj] : 0;  // chunk-local query id
        if (y20 || yT0) {
          atomicOr(&bv.bits[(int64_t)jo * bv.W + (o0 >> 5)], 1u << (o0 & 31));
          atomicAdd(&bv.counts[jo], 1ull);
        }
        if (y21 || yT1) {
          atomicOr(&bv.bits[(int64_t)jo * bv.W + (o1 >> 5)], 1u << (o1 & 31));
          atomicAdd(&bv.counts[jo], 1ull);
        }
        // undecided pairs: wave-aggregated appends
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const bool un = h ? un1 : un0;
          const unsigned long long um = __ballot(un);
          if (!um) continue;
          const int leader = __ffsll((long long)um) - 1;
          int base = 0;
          if (lane == leader) base = atomicAdd(bv.npairs, (int)__popcll(um));
          base = __shfl(base, leader);
          if (un) {
            const int pos = base + __popcll(um & lanemask_lt_b());
            const int64_t uu = h ? u1 : u0;
            if (pos < bv.pair_cap) {
              bv.pair_u[pos] = (int32_t)uu;
              bv.pair_j[pos] = (int32_t)jj;
              bv.pair_s[pos] = h ? s1 : s0;
            } else if (decide_f64(ix, bv, uu, (int32_t)jj)) {
              const int32_t oo = h ? o1 : o0;
              atomicOr(&bv.bits[(int64_t)jo * bv.W + (oo >> 5)], 1u << (oo & 31));
              atomicAdd(&bv.counts[jo], 1ull);
            }
          }
        }
        if (bv.ctr) {
          c_yes2 += (unsigned)y20 + (unsigned)y21;
          c_yesT += (unsigned)yT0 + (unsigned)yT1;
          c_und += (unsigned)un0 + (unsigned)un1;
        }
      }
    }
  }
  if (bv.ctr) {
    // per-lane partial counts -> one atomic per counter per wave
    for (int off = 32; off > 0; off >>= 1) {
      c_users += __shfl_xor(c_users, off);
      c_no1 += __shfl_xor(c_no1, off);
      c_yes2 += __shfl_xor(c_yes2, off);
      c_yesT += __shfl_xor(c_yesT, off);
      c_und += __shfl_xor(c_und, off);
    }
    if (lane == 0) {
      atomicAdd(&bv.ctr[C_BLOCKS], c_vis);
      atomicAdd(&bv.ctr[C_PRUNED], c_pr);
      atomicAdd(&bv.ctr[C_USERS], c_users);
      atomicAdd(&bv.ctr[C_L1NO], c_no1);
      atomicAdd(&bv.ctr[C_L2YES], c_yes2);
      atomicAdd(&bv.ctr[C_TYES], c_yesT);
      atomicAdd(&bv.ctr[ix.exact ? C_RCHK : C_SURV], c_und);
    }
  }
}

// ---------------------------------------------------------------------------
// Undecided pairs.  Exact table: float64 f(q,u) against theta_k (one thread
// per pair).  Bounded table: the linear scan of Algorithm 2, one wave per
// pair, lane = item (Corollaries 1 and 2 with certified margins); a pair the
// scan cannot certify is decided by the float64 scan in the same wave.
__device__ __forceinline__ void set_pair_result(const BatchView& bv, const DevIndex& ix,
                                                int64_t r, int32_t jo) {
  const int32_t orig = ix.permQ[r];
  atomicOr(&bv.bits[(int64_t)jo * bv.W + (orig >> 5)], 1u << (orig & 31));
  atomicAdd(&bv.counts[jo], 1ull);
}

__global__ void __launch_bounds__(256) k_brecheck_exact(DevIndex ix, BatchView bv) {
  const int np = min(*bv.npairs, bv.pair_cap);
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < np;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = bv.pair_u[t];
    const int32_t jj = bv.pair_j[t];
    const int32_t jo = bv.perm[jj];
    const float* q = bv.qs + (int64_t)jo * ix.d;
    const float* u = ix.Qt + (r / TILE) * (int64_t)ix.d * TILE + (r % TILE);
    double fq = 0.0;
    for (int c = 0; c < ix.d; ++c) fq = fma((double)q[c], (double)u[(int64_t)c * TILE], fq);
    const int k = bv.k_s[jj];
    if (fq >= ix.L64[(int64_t)(k - 1) * ix.n_pad + r]) set_pair_result(bv, ix, r, jo);
  }
}

template <bool BF16>
__global__ void __launch_bounds__(256) k_bverify(DevIndex ix, BatchView bv) {
  const int lane = threadIdx.x & 63;
  const int np = min(*bv.npairs, bv.pair_cap);
  const int64_t nwaves = (int64_t)gridDim.x * 4;
  for (int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); w < np; w += nwaves) {
    const int64_t r = bv.pair_u[w];
    const int32_t jj = bv.pair_j[w];
    const float s = bv.pair_s[w];
    const int k = bv.k_s[jj];
    const float nq = bv.qn_s[jj];
    const float nu = ix.normQ[r];
    const float euq = margin(ix, nu, nq);
    const float sl = s - euq;
    int64_t lo = 0, hi = ix.m;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if ((ix.cs_inflate * nu) * ix.normP[mid] <= sl) hi = mid;
      else lo = mid + 1;
    }
    const int64_t stop = lo;
    int beats = 0, unsure = 0;
    const int64_t ub = r / TILE, ul = r % TILE;
    for (int64_t t0 = 0; t0 < stop && beats < k; t0 += TILE) {
      const int64_t j = t0 + lane;
      const bool inb = j < stop;
      float g;
      if (!BF16) {
        const float* u = ix.Qt + ub * (int64_t)ix.d * TILE + ul;
        const float* p = ix.Pt + (t0 / TILE) * (int64_t)ix.d * TILE + lane;
        float x0 = 0.f, x1 = 0.f;
        int c = 0;
        for (; c + 2 <= ix.d; c += 2) {
          x0 = fmaf(u[c * TILE], p[c * TILE], x0);
          x1 = fmaf(u[(c + 1) * TILE], p[(c + 1) * TILE], x1);
        }
        if (c < ix.d) x0 = fmaf(u[c * TILE], p[c * TILE], x0);
        g = x0 + x1;
      } else {
        const int G = ix.d16 / 8;
        const uint4* u = (const uint4*)(ix.Qb + (ub * G * TILE + ul) * 8);
        const uint4* p = (const uint4*)(ix.Pb + ((t0 / TILE) * G * TILE + lane) * 8);
        float x0 = 0.f, x1 = 0.f;
        for (int gg = 0; gg < G; ++gg) {
          const uint4 wu = u[gg * TILE], wp = p[gg * TILE];
          const uint32_t xu[4] = {wu.x, wu.y, wu.z, wu.w}, xp[4] = {wp.x, wp.y, wp.z, wp.w};
#pragma unroll
          for (int h = 0; h < 4; ++h) {
            x0 = fmaf(bf16_to_f32((uint16_t)(xu[h] & 0xFFFFu)), bf16_to_f32((uint16_t)(xp[h] & 0xFFFFu)), x0);
            x1 = fmaf(bf16_to_f32((uint16_t)(xu[h] >> 16)), bf16_to_f32((uint16_t)(xp[h] >> 16)), x1);
          }
        }
        g = x0 + x1;
      }
      const float np_ = inb ? ix.normP[j] : 0.f;
      const float tol = margin(ix, nu, np_) + euq;
      const float diff = g - s;
      const bool beat = inb && (diff > tol);
      const bool unc = inb && !beat && !(diff <= -tol);
      beats += __popcll(__ballot(beat));
      unsure += __popcll(__ballot(unc));
    }
    const int32_t jo = bv.perm[jj];
    if (beats >= k) continue;
    if (beats + unsure < k) {
      if (lane == 0) set_pair_result(bv, ix, r, jo);
      continue;
    }
    // float64 scan in this wave: lane = item, counts up to k
    const float* q = bv.qs + (int64_t)jo * ix.d;
    const float* u = ix.Qt + ub * (int64_t)ix.d * TILE + ul;
    double fq = 0.0;
    for (int c = 0; c < ix.d; ++c) fq = fma((double)q[c], (double)u[(int64_t)c * TILE], fq);
    const double csu = (double)ix.cs_inflate * (double)nu * (1.0 + 0x1p-50);
    int b64 = 0;
    for (int64_t t0 = 0; t0 < ix.m && b64 < k; t0 += TILE) {
      const int64_t j = t0 + lane;
      bool beat = false;
      if (j < ix.m && csu * (double)ix.normP[j] > fq) {
        const float* p = ix.Prow + j * ix.d;
        double fp = 0.0;
        for (int c = 0; c < ix.d; ++c) fp = fma((double)p[c], (double)u[(int64_t)c * TILE], fp);
        beat = fp > fq;
      }
      b64 += __popcll(__ballot(beat));
      // items are norm-sorted: once a whole tile is past the bound, stop
      if (__ballot(j < ix.m && csu * (double)ix.normP[j] > fq) == 0ull) break;
    }
    if (bv.ctr && lane == 0) atomicAdd(&bv.ctr[C_RCHK], 1ull);
    if (b64 < k && lane == 0) set_pair_result(bv, ix, r, jo);
  }
}

// ---------------------------------------------------------------------------
// CSR assembly.  Offsets: one workgroup scans the chunk's counts (original
// chunk order) starting from *base.  Ids: one workgroup per query turns its
// bitmap row into ascending ids, then clears the row and the count.
__global__ void __launch_bounds__(1024) k_bscan(const unsigned long long* __restrict__ counts,
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

__global__ void __launch_bounds__(256) k_bassemble(BatchView bv, const int64_t* __restrict__ offs,
                                                   int32_t* __restrict__ ids, int64_t cap) {
  __shared__ int64_t part[256];
  const int32_t j = blockIdx.x;
  uint32_t* row = bv.bits + (int64_t)j * bv.W;
  const int t = threadIdx.x;
  if (bv.all[j]) {  // k > m: every user, ascending
    const int64_t b0 = offs[j];
    for (int64_t i = t; i < bv.n && b0 + i < cap; i += blockDim.x) ids[b0 + i] = (int32_t)i;
    if (t == 0 && bv.ctr) atomicAdd(&bv.ctr[C_RES], (unsigned long long)bv.n);
    return;
  }
  const int64_t w0 = bv.W * t / 256, w1 = bv.W * (t + 1) / 256;
  int64_t c = 0;
  for (int64_t w = w0; w < w1; ++w) c += __popc(row[w]);
  part[t] = c;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    int64_t v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int64_t pos = offs[j] + part[t] - c;
  for (int64_t w = w0; w < w1; ++w) {
    uint32_t bits = row[w];
    if (!bits) continue;
    row[w] = 0u;
    while (bits) {
      const int b = __ffs(bits) - 1;
      bits &= bits - 1;
      if (pos < cap) ids[pos] = (int32_t)(w * 32 + b);
      ++pos;
    }
  }
  if (t == 0) {
    if (bv.ctr) atomicAdd(&bv.ctr[C_RES], (unsigned long long)part[255]);
    bv.counts[j] = 0ull;
  }
}

// ---------------------------------------------------------------------------
void launch_bprep(const DevIndex& ix, const BatchView& bv, const int32_t* ks_dev, int32_t nq,
                  hipStream_t s) {
  hipLaunchKernelGGL(k_bnorms, dim3((nq + 3) / 4), dim3(256), 0, s, bv.qs, nq, ix.d, bv.qn,
                     bv.npairs);
  hipLaunchKernelGGL(k_bsort, dim3(1), dim3(1024), 0, s, bv.qn, nq, bv.perm);
  dim3 blk(64, 4);
  hipLaunchKernelGGL(k_btile, dim3((bv.nq_pad + 3) / 4), blk, 0, s, bv.qs, ks_dev, bv.qn,
                     bv.perm, nq, bv.nq_pad, ix.d, ix.d16, ix.m, bv.qt, ix.bf16 ? bv.qb : nullptr,
                     bv.qn_s, bv.k_s, bv.all);
}

size_t bfilter_lds_bytes(const DevIndex& ix) {
  const size_t ubytes = ix.bf16 ? (size_t)(ix.d16 / 8) * TILE * 16 : (size_t)ix.d * TILE * 4;
  return ubytes + (size_t)ix.kmax * TILE * 4 + (size_t)ix.kmax * 8;
}

void launch_bfilter(const DevIndex& ix, const BatchView& bv, hipStream_t s) {
  if (ix.nB == 0) return;
  const size_t lds = bfilter_lds_bytes(ix);
  if (lds > 65536) {
    (void)hipFuncSetAttribute((const void*)k_bfilter<true>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    (void)hipFuncSetAttribute((const void*)k_bfilter<false>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  }
  if (ix.bf16) hipLaunchKernelGGL(k_bfilter<true>, dim3(ix.nB), dim3(256), lds, s, ix, bv);
  else hipLaunchKernelGGL(k_bfilter<false>, dim3(ix.nB), dim3(256), lds, s, ix, bv);
}

void launch_bpairs(const DevIndex& ix, const BatchView& bv, hipStream_t s) {
  if (ix.nB == 0) return;
  if (ix.exact) {
    hipLaunchKernelGGL(k_brecheck_exact, dim3(256), dim3(256), 0, s, ix, bv);
  } else if (ix.bf16) {
    hipLaunchKernelGGL(k_bverify<true>, dim3(2048), dim3(256), 0, s, ix, bv);
  } else {
    hipLaunchKernelGGL(k_bverify<false>, dim3(2048), dim3(256), 0, s, ix, bv);
  }
}

void launch_bassemble(const BatchView& bv, int32_t nq, const int64_t* base, int64_t* offs,
                      int32_t* ids, int64_t cap, hipStream_t s) {
  hipLaunchKernelGGL(k_bscan, dim3(1), dim3(1024), 0, s, bv.counts, bv.all, bv.n, nq, base, offs);
  hipLaunchKernelGGL(k_bassemble, dim3(nq), dim3(256), 0, s, bv, offs, ids, cap);
}

}  // namespace rk
