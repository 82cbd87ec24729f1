// Host launch wrappers of the HIP kernels (each defined next to its kernel).
#pragma once
#include "rk_common.h"

namespace rk {

// ---- index build (Algorithm 1) -------------------------------------------
void launch_check_inputs(const float* X, int64_t count, int32_t* flag, hipStream_t s);
void launch_sqnorms(const float* X, int64_t rows, int32_t d, double* s2, hipStream_t s);
void launch_tile_rows(const float* X, const int32_t* perm, const double* s2, int64_t rows,
                      int64_t rows_pad, int32_t d, int32_t d16, float* Xt, float* norm_up,
                      uint16_t* Xb, float* Xrow, hipStream_t s);
// Exact float64 top-k_max over the first S sorted items.  Writes L64/L32
// (when t0 == nullptr) or the k_max-th value rounded down into t0 (seed).
void launch_lb_exact(const DevIndex& ix, int64_t S, double* L64, float* L32, float* t0,
                     hipStream_t s);
// MFMA pass over items [0, S_end): candidates of each user (item indices).
void launch_lb_candidates(const DevIndex& ix, int64_t S_end, const float* t0, int32_t cap,
                          int32_t* cand, int32_t* ccount, hipStream_t s);
void launch_lb_refine(const DevIndex& ix, int32_t cap, const int32_t* cand,
                      const int32_t* ccount, double* L64, float* L32, int32_t* ovf_list,
                      int32_t* n_ovf, hipStream_t s);
void launch_lb_overflow(const DevIndex& ix, int64_t S_end, const int32_t* ovf_list,
                        int32_t n_ovf, double* L64, float* L32, hipStream_t s);
void launch_blocks(const DevIndex& ix, float* LB, float* bnorm, hipStream_t s);
// Catalog updates: m_new new items (rows Pnew) merged into the exact table
// of every user; the rows of a grown user set gathered from two tables
// (src[r] >= 0: row of the first, else row -1 - src[r] of the second).
void launch_lb_merge(const DevIndex& ix, const float* Pnew, int64_t m_new, double* L64, float* L32,
                     hipStream_t s);
void launch_gather_bounds(int32_t kmax, int64_t n, int64_t n_pad, const int64_t* src,
                          const double* L64a, const float* L32a, int64_t na_pad, const double* L64b,
                          const float* L32b, int64_t nb_pad, double* L64, float* L32, hipStream_t s);

// ---- online query (Algorithms 2 and 3) -----------------------------------
void launch_filter(const DevIndex& ix, const float* q, int32_t k, const QueryWS& ws,
                   hipStream_t s);
void launch_verify(const DevIndex& ix, const float* q, int32_t k, const QueryWS& ws,
                   hipStream_t s);
void launch_recheck(const DevIndex& ix, const float* q, int32_t k, const QueryWS& ws,
                    hipStream_t s);
// Ids to ids[base...] (base may be nullptr = 0); *out = base + count.
void launch_finalize(const DevIndex& ix, const QueryWS& ws, int32_t* ids, int64_t cap,
                     const int64_t* base, int64_t* out, hipStream_t s);
void launch_fill_all(int64_t n, int32_t* ids, int64_t cap, const int64_t* base, int64_t* out,
                     hipStream_t s);
void launch_set_i64(int64_t* p, int64_t v, hipStream_t s);

}  // namespace rk
