// Device helpers shared by the batched filter and the bounded table's scan.
#pragma once
#include "rk_batch.h"

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

namespace rk {

// Exact float64 decision of one (user, query) pair, used by a lane whose
// undecided pair does not fit the pair list: with an exact table f(q,u)
// against theta_k; otherwise the float64 linear scan (Algorithm 2).
__device__ __forceinline__ bool decide_f64(const DevIndex& ix, const BatchView& bv, int64_t r,
                                           int32_t jj) {
  const int32_t jo = bv.perm[jj];
  const int k = bv.k_s[jj];
  const float* u = ix.Qrow + r * ix.d;
  const double fq = dot64_rows(bv.qs + (int64_t)jo * ix.d, u, ix.d);
  if (ix.exact) return fq >= ix.L64[(int64_t)(k - 1) * ix.n_pad + r];
  const double csu = (double)ix.cs_inflate * (double)ix.normQ[r] * (1.0 + 0x1p-50);
  int beats = 0;
  for (int64_t j = 0; j < ix.m && beats < k; ++j) {
    if (csu * (double)ix.normP[j] <= fq) break;
    beats += dot64_rows(ix.Prow + j * ix.d, u, ix.d) > fq;
  }
  return beats < k;
}

// Row of the 32x32 MFMA output (v_mfma_f32_32x32x*) that accumulator entry r
// of a lane in half `half` of the wave holds, in the quarter starting at
// row 32 * qhalf.
__device__ __forceinline__ int quarter_row(int qhalf, int half, int r) {
  return qhalf * 32 + (r / 4) * 8 + half * 4 + (r % 4);
}

// A pair decided yes: the user's bit in the query's result row and the
// query's result count.
__device__ __forceinline__ void set_pair_result(const BatchView& bv, const DevIndex& ix,
                                                int64_t r, int32_t jo) {
  const int32_t orig = ix.permQ[r];
  atomicOr(&bv.bits[(int64_t)jo * bv.W + (orig >> 5)], 1u << (orig & 31));
  atomicAdd(&bv.counts[jo], 1ull);
}

}  // namespace rk
