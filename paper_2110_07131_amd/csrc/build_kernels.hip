// Index build kernels: pre-processing of Simpfer (Algorithm 1, Section 4.1).
//
//  norms        squared norms in float64 (index order) for the norm sort
//  tile         gather rows into norm-sorted tiled layouts, norms rounded up
//  lb_exact     lower-bound arrays over a short prefix P' of the sorted items,
//               every inner product in float64 in the oracle's order
//  lb_candidates / lb_refine / lb_overflow
//               the same arrays over a long prefix (up to all of P): an MFMA
//               pass keeps each user's items that can reach its k_max-th
//               value, and only those are recomputed in float64
//  lb_merge / gather_bounds
//               catalog updates: new items merged into the exact table; the
//               rows of old and new users gathered into the grown norm order
//  blocks       block minima L^j(B) (Equation (1)) and first-user norms
#include "rk_kernels.h"

typedef float f32x16 __attribute__((ext_vector_type(16)));

namespace rk {

// ---------------------------------------------------------------------------
__global__ void k_check_inputs(const float* __restrict__ X, int64_t count, int32_t* flag) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  bool bad = false;
  for (; i < count; i += stride) {
    float v = X[i];
    // non-finite or |v| >= 2^40 (keeps every float32 product and norm finite)
    bad |= !(fabsf(v) < 1099511627776.0f);
  }
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

void launch_check_inputs(const float* X, int64_t count, int32_t* flag, hipStream_t s) {
  if (count <= 0) return;
  int64_t blocks = (count + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_check_inputs, dim3((unsigned)blocks), dim3(256), 0, s, X, count, flag);
}

// ---------------------------------------------------------------------------
// Squared norm of every row, summed in float64 in index order.
__global__ void k_sqnorms(const float* __restrict__ X, int64_t rows, int32_t d,
                          double* __restrict__ s2) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  const float* x = X + r * d;
  double s = 0.0;
  for (int c = 0; c < d; ++c) s = fma((double)x[c], (double)x[c], s);
  s2[r] = s;
}

void launch_sqnorms(const float* X, int64_t rows, int32_t d, double* s2, hipStream_t s) {
  if (rows <= 0) return;
  hipLaunchKernelGGL(k_sqnorms, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, s, X, rows,
                     d, s2);
}

// ---------------------------------------------------------------------------
// Sorted position r takes original row perm[r].  Writes the tiled fp32 copy,
// optionally the tiled bf16 copy and a sorted row-major copy, and the norm
// rounded up: the true Euclidean norm of the float32 row is at most
// sqrt(s2 * (1 + gamma_d)) with s2 the float64 sum; the factor below also
// covers the square root's and the product's own rounding.
__global__ void k_tile_rows(const float* __restrict__ X, const int32_t* __restrict__ perm,
                            const double* __restrict__ s2, int64_t rows, int64_t rows_pad,
                            int32_t d, int32_t d16, float* __restrict__ Xt,
                            float* __restrict__ norm_up, uint16_t* __restrict__ Xb,
                            float* __restrict__ Xrow) {
  int64_t r = (int64_t)blockIdx.x * blockDim.y + threadIdx.y;
  if (r >= rows_pad) return;
  const bool valid = r < rows;
  const int64_t src = valid ? perm[r] : 0;
  for (int c = threadIdx.x; c < d; c += blockDim.x) {
    float v = valid ? X[src * d + c] : 0.0f;
    Xt[tix(r, c, d)] = v;
    if (Xrow && valid) Xrow[r * d + c] = v;
  }
  if (Xb) {
    const int64_t tile = r / TILE, lane = r % TILE;
    for (int c = threadIdx.x; c < d16; c += blockDim.x) {
      float v = (valid && c < d) ? X[src * d + c] : 0.0f;
      Xb[((tile * (d16 / 8) + c / 8) * TILE + lane) * 8 + (c % 8)] = bf16_bits(v);
    }
  }
  if (threadIdx.x == 0) {
    float nu = 0.0f;
    if (valid) {
      const double g = (double)(d + 4) * 0x1p-53;
      nu = f32_up(sqrt(s2[src]) * (1.0 + g));
    }
    norm_up[r] = nu;
  }
}

void launch_tile_rows(const float* X, const int32_t* perm, const double* s2, int64_t rows,
                      int64_t rows_pad, int32_t d, int32_t d16, float* Xt, float* norm_up,
                      uint16_t* Xb, float* Xrow, hipStream_t s) {
  if (rows_pad <= 0) return;
  dim3 blk(64, 4);
  hipLaunchKernelGGL(k_tile_rows, dim3((unsigned)((rows_pad + 3) / 4)), blk, 0, s, X, perm, s2,
                     rows, rows_pad, d, d16, Xt, norm_up, Xb, Xrow);
}

// ---------------------------------------------------------------------------
// Descending register top-K: inserting v keeps the K largest values seen.
template <int K>
__device__ __forceinline__ void topk_insert(double (&top)[K], double v) {
#pragma unroll
  for (int j = 0; j < K; ++j) {
    double hi = fmax(top[j], v);
    v = fmin(top[j], v);
    top[j] = hi;
  }
}

// Exact float64 inner product of sorted user r (tiled layout) with a
// contiguous row x, summed in index order.
__device__ __forceinline__ double dot64_user_row(const float* __restrict__ Qt, int64_t r,
                                                 int d, const float* __restrict__ x) {
  double s = 0.0;
  const float* u = Qt + (r / TILE) * (int64_t)d * TILE + (r % TILE);
  for (int c = 0; c < d; ++c) s = fma((double)u[(int64_t)c * TILE], (double)x[c], s);
  return s;
}

// Lower-bound arrays over the first S sorted items (Algorithm 1, building
// L_i): one lane per user, float64 inner products (same order as the
// oracle), register top-K.  In seed mode only the k_max-th value is kept.
template <int K>
__global__ void __launch_bounds__(64) k_lb_exact(DevIndex ix, int64_t S, double* __restrict__ L64,
                                                 float* __restrict__ L32, float* __restrict__ t0) {
  const int64_t r = (int64_t)blockIdx.x * TILE + threadIdx.x;
  const bool valid = r < ix.n;
  double top[K];
#pragma unroll
  for (int j = 0; j < K; ++j) top[j] = -INFINITY;
  if (valid) {
    const int d = ix.d;
    const float* u = ix.Qt + (r / TILE) * (int64_t)d * TILE + (r % TILE);
    int64_t t = 0;
    for (; t + 4 <= S; t += 4) {
      const float* p = ix.Prow + t * d;
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
      for (int c = 0; c < d; ++c) {
        double uc = (double)u[(int64_t)c * TILE];
        a0 = fma((double)p[c], uc, a0);
        a1 = fma((double)p[d + c], uc, a1);
        a2 = fma((double)p[2 * d + c], uc, a2);
        a3 = fma((double)p[3 * d + c], uc, a3);
      }
      if (a0 > top[K - 1]) topk_insert<K>(top, a0);
      if (a1 > top[K - 1]) topk_insert<K>(top, a1);
      if (a2 > top[K - 1]) topk_insert<K>(top, a2);
      if (a3 > top[K - 1]) topk_insert<K>(top, a3);
    }
    for (; t < S; ++t) {
      double a = dot64_user_row(ix.Qt, r, d, ix.Prow + t * d);
      if (a > top[K - 1]) topk_insert<K>(top, a);
    }
  }
  if (r >= ix.n_pad) return;
  if (t0) {
    if (valid) {
      double v = -INFINITY;
#pragma unroll
      for (int j = 0; j < K; ++j)
        if (j == ix.kmax - 1) v = top[j];
      t0[r] = f32_down(v);
    }
    return;
  }
#pragma unroll
  for (int j = 0; j < K; ++j) {
    if (j < ix.kmax) {
      double v = valid ? top[j] : INFINITY;
      L64[(int64_t)j * ix.n_pad + r] = v;
      L32[(int64_t)j * ix.n_pad + r] = valid ? f32_down(v) : INFINITY;
    }
  }
}

template <int K>
static void lb_exact_k(const DevIndex& ix, int64_t S, double* L64, float* L32, float* t0,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_lb_exact<K>, dim3((unsigned)(ix.n_pad / TILE)), dim3(64), 0, s, ix, S,
                     L64, L32, t0);
}

void launch_lb_exact(const DevIndex& ix, int64_t S, double* L64, float* L32, float* t0,
                     hipStream_t s) {
  if (ix.n_pad == 0) return;
  if (ix.kmax <= 8) lb_exact_k<8>(ix, S, L64, L32, t0, s);
  else if (ix.kmax <= 16) lb_exact_k<16>(ix, S, L64, L32, t0, s);
  else if (ix.kmax <= 32) lb_exact_k<32>(ix, S, L64, L32, t0, s);
  else if (ix.kmax <= 64) lb_exact_k<64>(ix, S, L64, L32, t0, s);
  else lb_exact_k<128>(ix, S, L64, L32, t0, s);
}

// ---------------------------------------------------------------------------
// Candidate pass (FP32 MFMA).  One workgroup = one block of 64 users; its 4
// waves take item tiles round-robin.  Per item tile a wave forms the 64x64
// score tile with v_mfma_f32_32x32x2f32: A = 32 items x 2 coords, B = 2
// coords x 32 users, so each lane's 16 accumulators hold one user and 16
// items.  An item is a candidate of a user when its score plus the bulk
// error margin reaches the user's seed value t0 (a true lower bound of the
// k_max-th largest inner product), so the candidates contain every item of
// the exact top-k_max.
__global__ void __launch_bounds__(256) k_lb_candidates(DevIndex ix, int64_t S_end,
                                                       const float* __restrict__ t0,
                                                       int32_t cap, int32_t* __restrict__ cand,
                                                       int32_t* __restrict__ ccount) {
  extern __shared__ float lds[];  // [d][64] user tile, then 64 counters
  const int d = ix.d;
  const int64_t B = blockIdx.x;
  float* uA = lds;
  int32_t* cnt = (int32_t*)(lds + (size_t)d * TILE);
  const float* src = ix.Qt + B * (int64_t)d * TILE;
  for (int i = threadIdx.x; i < d * TILE; i += blockDim.x) uA[i] = src[i];
  if (threadIdx.x < TILE) cnt[threadIdx.x] = 0;
  __syncthreads();

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int half = lane >> 5, col = lane & 31;
  int64_t u0 = B * TILE + col, u1 = u0 + 32;
  const bool v0 = u0 < ix.n, v1 = u1 < ix.n;
  const float nu0 = ix.normQ[u0], nu1 = ix.normQ[u1];
  const float th0 = v0 ? t0[u0] : INFINITY, th1 = v1 ? t0[u1] : INFINITY;
  const int64_t nT = (S_end + TILE - 1) / TILE;
  const int ksteps = (d + 1) / 2;

  for (int64_t T = wave; T < nT; T += 4) {
    f32x16 acc00 = {}, acc01 = {}, acc10 = {}, acc11 = {};  // [item half][user half]
    const float* pt = ix.Pt + T * (int64_t)d * TILE;
    for (int ks = 0; ks < ksteps; ++ks) {
      const int c = 2 * ks + half;
      float a0 = 0.f, a1 = 0.f, b0 = 0.f, b1 = 0.f;
      if (c < d) {
        a0 = pt[c * TILE + col];
        a1 = pt[c * TILE + 32 + col];
        b0 = uA[c * TILE + col];
        b1 = uA[c * TILE + 32 + col];
      }
      acc00 = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b0, acc00, 0, 0, 0);
      acc01 = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b1, acc01, 0, 0, 0);
      acc10 = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b0, acc10, 0, 0, 0);
      acc11 = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b1, acc11, 0, 0, 0);
    }
    // lane holds rows (items) (r/4)*8 + half*4 + r%4 of its column (user)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = (r / 4) * 8 + half * 4 + (r % 4);
#pragma unroll
      for (int ih = 0; ih < 2; ++ih) {
        const int64_t j = T * TILE + ih * 32 + row;
        if (j < S_end) {
          const float np = ix.normP[j];
          const float s0 = ih ? acc10[r] : acc00[r];
          const float s1 = ih ? acc11[r] : acc01[r];
          if (s0 + margin(ix, nu0, np) >= th0) {
            int pos = atomicAdd(&cnt[col], 1);
            if (pos < cap) cand[u0 * cap + pos] = (int32_t)j;
          }
          if (s1 + margin(ix, nu1, np) >= th1) {
            int pos = atomicAdd(&cnt[32 + col], 1);
            if (pos < cap) cand[u1 * cap + pos] = (int32_t)j;
          }
        }
      }
    }
  }
  __syncthreads();
  if (threadIdx.x < TILE) {
    int64_t u = B * TILE + threadIdx.x;
    if (u < ix.n) ccount[u] = cnt[threadIdx.x];
  }
}

void launch_lb_candidates(const DevIndex& ix, int64_t S_end, const float* t0, int32_t cap,
                          int32_t* cand, int32_t* ccount, hipStream_t s) {
  if (ix.nB == 0) return;
  size_t lds = (size_t)ix.d * TILE * sizeof(float) + TILE * sizeof(int32_t);
  if (lds > 65536)
    (void)hipFuncSetAttribute((const void*)k_lb_candidates,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(k_lb_candidates, dim3(ix.nB), dim3(256), lds, s, ix, S_end, t0, cap, cand,
                     ccount);
}

// ---------------------------------------------------------------------------
// Refine: each user's candidates in float64 (oracle order), top-k_max kept.
template <int K>
__global__ void __launch_bounds__(64) k_lb_refine(DevIndex ix, int32_t cap,
                                                  const int32_t* __restrict__ cand,
                                                  const int32_t* __restrict__ ccount,
                                                  double* __restrict__ L64,
                                                  float* __restrict__ L32,
                                                  int32_t* __restrict__ ovf_list,
                                                  int32_t* __restrict__ n_ovf) {
  const int64_t r = (int64_t)blockIdx.x * TILE + threadIdx.x;
  if (r >= ix.n_pad) return;
  const bool valid = r < ix.n;
  double top[K];
#pragma unroll
  for (int j = 0; j < K; ++j) top[j] = -INFINITY;
  if (valid) {
    const int cnt = ccount[r];
    if (cnt > cap) {
      ovf_list[atomicAdd(n_ovf, 1)] = (int32_t)r;
      return;  // filled in by the overflow kernel
    }
    for (int t = 0; t < cnt; ++t) {
      const int64_t j = cand[r * cap + t];
      double a = dot64_user_row(ix.Qt, r, ix.d, ix.Prow + j * ix.d);
      if (a > top[K - 1]) topk_insert<K>(top, a);
    }
  }
#pragma unroll
  for (int j = 0; j < K; ++j) {
    if (j < ix.kmax) {
      double v = valid ? top[j] : INFINITY;
      L64[(int64_t)j * ix.n_pad + r] = v;
      L32[(int64_t)j * ix.n_pad + r] = valid ? f32_down(v) : INFINITY;
    }
  }
}

template <int K>
static void lb_refine_k(const DevIndex& ix, int32_t cap, const int32_t* cand,
                        const int32_t* ccount, double* L64, float* L32, int32_t* ovf_list,
                        int32_t* n_ovf, hipStream_t s) {
  hipLaunchKernelGGL(k_lb_refine<K>, dim3((unsigned)(ix.n_pad / TILE)), dim3(64), 0, s, ix, cap,
                     cand, ccount, L64, L32, ovf_list, n_ovf);
}

void launch_lb_refine(const DevIndex& ix, int32_t cap, const int32_t* cand,
                      const int32_t* ccount, double* L64, float* L32, int32_t* ovf_list,
                      int32_t* n_ovf, hipStream_t s) {
  if (ix.n_pad == 0) return;
  if (ix.kmax <= 8) lb_refine_k<8>(ix, cap, cand, ccount, L64, L32, ovf_list, n_ovf, s);
  else if (ix.kmax <= 16) lb_refine_k<16>(ix, cap, cand, ccount, L64, L32, ovf_list, n_ovf, s);
  else if (ix.kmax <= 32) lb_refine_k<32>(ix, cap, cand, ccount, L64, L32, ovf_list, n_ovf, s);
  else if (ix.kmax <= 64) lb_refine_k<64>(ix, cap, cand, ccount, L64, L32, ovf_list, n_ovf, s);
  else lb_refine_k<128>(ix, cap, cand, ccount, L64, L32, ovf_list, n_ovf, s);
}

// ---------------------------------------------------------------------------
// Users whose candidate list overflowed: one wave per user scans all items
// [0, S_end) in float64 (lane j takes items j, j+64, ...), then the 64
// per-lane top-K lists are merged by K rounds of a wave-wide maximum.
template <int K>
__global__ void __launch_bounds__(64) k_lb_overflow(DevIndex ix, int64_t S_end,
                                                    const int32_t* __restrict__ ovf_list,
                                                    double* __restrict__ L64,
                                                    float* __restrict__ L32) {
  const int64_t r = ovf_list[blockIdx.x];
  const int lane = threadIdx.x;
  double top[K];
#pragma unroll
  for (int j = 0; j < K; ++j) top[j] = -INFINITY;
  for (int64_t t = lane; t < S_end; t += TILE) {
    double a = dot64_user_row(ix.Qt, r, ix.d, ix.Prow + t * ix.d);
    if (a > top[K - 1]) topk_insert<K>(top, a);
  }
  for (int j = 0; j < ix.kmax && j < K; ++j) {
    // wave maximum of the lane heads; the lowest lane holding it pops
    double best = top[0];
    for (int off = 32; off > 0; off >>= 1) best = fmax(best, __shfl_xor(best, off));
    unsigned long long owners = __ballot(top[0] == best);
    int owner = __ffsll((long long)owners) - 1;
    if (lane == owner) {
#pragma unroll
      for (int i = 0; i < K - 1; ++i) top[i] = top[i + 1];
      top[K - 1] = -INFINITY;
    }
    if (lane == 0) {
      L64[(int64_t)j * ix.n_pad + r] = best;
      L32[(int64_t)j * ix.n_pad + r] = f32_down(best);
    }
  }
}

void launch_lb_overflow(const DevIndex& ix, int64_t S_end, const int32_t* ovf_list,
                        int32_t n_ovf, double* L64, float* L32, hipStream_t s) {
  if (n_ovf <= 0) return;
  dim3 g((unsigned)n_ovf);
  if (ix.kmax <= 8) hipLaunchKernelGGL(k_lb_overflow<8>, g, dim3(64), 0, s, ix, S_end, ovf_list, L64, L32);
  else if (ix.kmax <= 16) hipLaunchKernelGGL(k_lb_overflow<16>, g, dim3(64), 0, s, ix, S_end, ovf_list, L64, L32);
  else if (ix.kmax <= 32) hipLaunchKernelGGL(k_lb_overflow<32>, g, dim3(64), 0, s, ix, S_end, ovf_list, L64, L32);
  else if (ix.kmax <= 64) hipLaunchKernelGGL(k_lb_overflow<64>, g, dim3(64), 0, s, ix, S_end, ovf_list, L64, L32);
  else hipLaunchKernelGGL(k_lb_overflow<128>, g, dim3(64), 0, s, ix, S_end, ovf_list, L64, L32);
}

// ---------------------------------------------------------------------------
// Catalog updates.  New items: the exact table's k_max largest values of
// each user take the new items' float64 products in (the top-k_max multiset
// over the grown catalog, so the table stays exact and equals a fresh
// build's).  One lane per sorted user; Pnew holds the m_new new rows.
template <int K>
__global__ void __launch_bounds__(64) k_lb_merge(DevIndex ix, const float* __restrict__ Pnew,
                                                 int64_t m_new, double* __restrict__ L64,
                                                 float* __restrict__ L32) {
  const int64_t r = (int64_t)blockIdx.x * TILE + threadIdx.x;
  if (r >= ix.n) return;
  double top[K];
#pragma unroll
  for (int j = 0; j < K; ++j) top[j] = j < ix.kmax ? L64[(int64_t)j * ix.n_pad + r] : -INFINITY;
  for (int64_t t = 0; t < m_new; ++t) {
    const double a = dot64_user_row(ix.Qt, r, ix.d, Pnew + t * ix.d);
    if (a > top[K - 1]) topk_insert<K>(top, a);
  }
#pragma unroll
  for (int j = 0; j < K; ++j) {
    if (j < ix.kmax) {
      L64[(int64_t)j * ix.n_pad + r] = top[j];
      L32[(int64_t)j * ix.n_pad + r] = f32_down(top[j]);
    }
  }
}

template <int K>
static void lb_merge_k(const DevIndex& ix, const float* Pnew, int64_t m_new, double* L64, float* L32,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_lb_merge<K>, dim3((unsigned)(ix.n_pad / TILE)), dim3(64), 0, s, ix, Pnew, m_new,
                     L64, L32);
}

void launch_lb_merge(const DevIndex& ix, const float* Pnew, int64_t m_new, double* L64, float* L32,
                     hipStream_t s) {
  if (ix.n_pad == 0 || m_new == 0) return;
  if (ix.kmax <= 8) lb_merge_k<8>(ix, Pnew, m_new, L64, L32, s);
  else if (ix.kmax <= 16) lb_merge_k<16>(ix, Pnew, m_new, L64, L32, s);
  else if (ix.kmax <= 32) lb_merge_k<32>(ix, Pnew, m_new, L64, L32, s);
  else if (ix.kmax <= 64) lb_merge_k<64>(ix, Pnew, m_new, L64, L32, s);
  else lb_merge_k<128>(ix, Pnew, m_new, L64, L32, s);
}

// New users: the lower-bound rows of the grown user set in its norm order,
// gathered from the old index's rows (src >= 0: old sorted position) and
// the new users' rows (src < 0: new user -1 - src); padding rows +inf.
__global__ void k_gather_bounds(int32_t kmax, int64_t n, int64_t n_pad, const int64_t* __restrict__ src,
                                const double* __restrict__ L64a, const float* __restrict__ L32a,
                                int64_t na_pad, const double* __restrict__ L64b,
                                const float* __restrict__ L32b, int64_t nb_pad, double* __restrict__ L64,
                                float* __restrict__ L32) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_pad) return;
  const int64_t sr = r < n ? src[r] : 0;
  for (int j = 0; j < kmax; ++j) {
    double v = INFINITY;
    float v32 = INFINITY;
    if (r < n) {
      if (sr >= 0) {
        v = L64a[(int64_t)j * na_pad + sr];
        v32 = L32a[(int64_t)j * na_pad + sr];
      } else {
        v = L64b[(int64_t)j * nb_pad + (-1 - sr)];
        v32 = L32b[(int64_t)j * nb_pad + (-1 - sr)];
      }
    }
    L64[(int64_t)j * n_pad + r] = v;
    L32[(int64_t)j * n_pad + r] = v32;
  }
}

void launch_gather_bounds(int32_t kmax, int64_t n, int64_t n_pad, const int64_t* src,
                          const double* L64a, const float* L32a, int64_t na_pad, const double* L64b,
                          const float* L32b, int64_t nb_pad, double* L64, float* L32, hipStream_t s) {
  if (n_pad <= 0) return;
  hipLaunchKernelGGL(k_gather_bounds, dim3((unsigned)((n_pad + 255) / 256)), dim3(256), 0, s, kmax, n,
                     n_pad, src, L64a, L32a, na_pad, L64b, L32b, nb_pad, L64, L32);
}

// ---------------------------------------------------------------------------
// Blocks (Definition 5, Equation (1)) of bsize users: LB[j][b] = min of
// L32[j][.] over the real users of block b (+inf when it has none);
// bnorm[b] = norm of its first (largest-norm) user.
__global__ void k_blocks(DevIndex ix, float* __restrict__ LB, float* __restrict__ bnorm) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)ix.kmax * ix.nSB;
  if (t >= total) return;
  const int64_t j = t / ix.nSB, b = t % ix.nSB;
  float lo = INFINITY;
  for (int64_t r = b * ix.bsize; r < (b + 1) * ix.bsize && r < ix.n; ++r)
    lo = fminf(lo, ix.L32[j * ix.n_pad + r]);
  LB[j * ix.nSB + b] = lo;
  if (j == 0) bnorm[b] = ix.normQ[b * ix.bsize];
}

void launch_blocks(const DevIndex& ix, float* LB, float* bnorm, hipStream_t s) {
  const int64_t total = (int64_t)ix.kmax * ix.nSB;
  if (total == 0) return;
  hipLaunchKernelGGL(k_blocks, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, ix, LB,
                     bnorm);
}

}  // namespace rk
