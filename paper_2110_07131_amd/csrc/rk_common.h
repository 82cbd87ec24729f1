// Shared definitions of the reverse k-MIPS HIP library (gfx950, wave64).
//
// Device layouts (users and items both sorted by descending norm, Algorithm 1):
//   tiled fp32   X_t[tile][c][64]            element (row r, coord c) at
//                (r/64)*D*64 + c*64 + r%64, D = d.  One tile of 64 rows is one
//                user block (Definition 5) = one wavefront; a fixed coordinate
//                of 64 consecutive rows is one coalesced 256-byte segment.
//   tiled bf16   X_b[tile][g][64][8]         groups of 8 coordinates, 16 bytes
//                per (row, group), D padded with zeros to a multiple of 16.
//   row-major    P_row[j][c]                 sorted items (float64 rechecks).
//   bound tables L32/L64[j][r]               j-th lower bound of sorted user r;
//                a fixed j over consecutive users is contiguous.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "host_rules.h"
#include "rkmips.h"

namespace rk {

__host__ __device__ inline int64_t tix(int64_t r, int c, int d) {
  return (r / TILE) * (int64_t)d * TILE + (int64_t)c * TILE + (r % TILE);
}

// float32 rounded toward -inf / +inf from a double (exact directed rounding).
__host__ __device__ inline float f32_down(double x) {
  float f = (float)x;
  if ((double)f > x) f = nextafterf(f, -INFINITY);
  return f;
}
__host__ __device__ inline float f32_up(double x) {
  float f = (float)x;
  if ((double)f < x) f = nextafterf(f, INFINITY);
  return f;
}
// Smallest float strictly above x (x finite or -inf).
__host__ __device__ inline float f32_next_up(float x) { return nextafterf(x, INFINITY); }

// float32 -> bfloat16 bits, round to nearest even (finite inputs).
__host__ __device__ inline uint16_t bf16_bits(float x) {
  uint32_t b;
  memcpy(&b, &x, 4);
  b += 0x7FFFu + ((b >> 16) & 1u);
  return (uint16_t)(b >> 16);
}
__host__ __device__ inline float bf16_to_f32(uint16_t h) {
  uint32_t b = (uint32_t)h << 16;
  float f;
  memcpy(&f, &b, 4);
  return f;
}
__host__ __device__ inline float bf16_round(float x) { return bf16_to_f32(bf16_bits(x)); }

// Read-only view of a device-resident index, passed to kernels by value.
struct DevIndex {
  int64_t n, m;          // users, items
  int64_t n_pad, m_pad;  // rounded up to TILE
  int32_t d, d16;        // dimension; bf16 padded dimension (multiple of 16)
  int32_t kmax, nB, mB;  // k_max; user tiles of 64; item tiles
  int32_t bsize, nSB;    // users per Lemma 3 block (16, 32 or 64); such blocks (n_pad / bsize)
  int32_t use_blocks;    // 0: Lemma 3 is not applied (every block evaluated)
  int32_t lb_items;      // |P'|
  int32_t exact;         // 1 if L holds the exact k_max largest values over P
  int32_t bf16;          // 1 if the bulk products use the bf16 copies
  const float* Qt;       // tiled fp32 users
  const float* Qrow;     // [n][d] sorted users, row-major (float64 rechecks)
  const uint16_t* Qb;    // tiled bf16 users (bf16 mode)
  const float* normQ;    // [n_pad] norm rounded up (0 for padding)
  const int32_t* permQ;  // [n] original id of sorted user
  const float* Pt;       // tiled fp32 items
  const uint16_t* Pb;    // tiled bf16 items (bf16 mode)
  const float* Prow;     // [m][d] sorted items, row-major
  const float* normP;    // [m_pad] norm rounded up (0 for padding)
  const float* L32;      // [kmax][n_pad] lower bounds rounded down
  const double* L64;     // [kmax][n_pad] lower bounds, exact
  const float* LB;       // [kmax][nSB] block minima of L32
  const float* bnorm;    // [nSB] norm of the first user of each block
  // Certified-comparison constants (see margin()):
  float eps_rel;         // relative bound on |approx u.x - f(x,u)| / (|u||x|)
  float eps_abs;         // absolute slack (underflow)
  float cs_inflate;      // 1 + gamma64_d + slack: f(p,u) <= cs_inflate*|u|^*|p|^
  float eps_rel32;       // eps_rel of float32 products (the verification pass)
  int32_t handoff_tiles; // batched scan: hand over only with more tiles than this left
  int32_t verify_tiles;  // one query: from this many survivors on, the tiled linear scan
};

// f(x, y) in float64, index order, from two contiguous float32 rows: the
// inner product of the definition (each product is exact in double; the
// loads are batched ahead of the sequential accumulation).
__device__ __forceinline__ double dot64_rows(const float* __restrict__ x,
                                             const float* __restrict__ y, int d) {
  double s = 0.0;
  int c0 = 0;
  for (; c0 + 8 <= d; c0 += 8) {
    float xv[8], yv[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      xv[i] = x[c0 + i];
      yv[i] = y[c0 + i];
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) s = fma((double)xv[i], (double)yv[i], s);
  }
  for (; c0 < d; ++c0) s = fma((double)x[c0], (double)y[c0], s);
  return s;
}

// The same from rows of d4 float4s (16-byte aligned, d = 4 d4): the same
// products summed in the same order, a quarter of the load instructions.
__device__ __forceinline__ double dot64_rows4(const float4* __restrict__ x,
                                              const float4* __restrict__ y, int d4) {
  double s = 0.0;
  int c0 = 0;
  for (; c0 + 8 <= d4; c0 += 8) {
    float4 xv[8], yv[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      xv[i] = x[c0 + i];
      yv[i] = y[c0 + i];
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      s = fma((double)xv[i].x, (double)yv[i].x, s);
      s = fma((double)xv[i].y, (double)yv[i].y, s);
      s = fma((double)xv[i].z, (double)yv[i].z, s);
      s = fma((double)xv[i].w, (double)yv[i].w, s);
    }
  }
  for (; c0 < d4; ++c0) {
    const float4 a = x[c0], b = y[c0];
    s = fma((double)a.x, (double)b.x, s);
    s = fma((double)a.y, (double)b.y, s);
    s = fma((double)a.z, (double)b.z, s);
    s = fma((double)a.w, (double)b.w, s);
  }
  return s;
}

// |approx - f| <= margin(|u|^, |x|^) for every bulk inner product.
__device__ __forceinline__ float margin(const DevIndex& ix, float nu, float nx) {
  return ix.eps_rel * (nu * nx) + ix.eps_abs;
}

// Per-query device workspace.
struct QueryWS {
  uint32_t* rbits;          // [ceil(n/32)] result bits by original id; all
                            // zero between queries (finalize clears them)
  int32_t* surv_idx;        // [n] survivors for the linear scan (sorted idx)
  float* surv_s;            // [n] their approximate u.q
  int32_t* rchk_idx;        // [n] users for float64 recomputation
  int32_t* cnt;             // [4]: survivors, rechecks, -, -  (reset by finalize)
  float* qnorm;             // [1] |q| rounded up (written by the filter)
  unsigned long long* ctr;  // [16] statistics counters or nullptr
  uint8_t* trace_cls;       // [n] by original id, or nullptr
  float* trace_s;           // [n] by original id, or nullptr
};

// Counter slots (statistics).
enum Ctr {
  C_BLOCKS = 0, C_PRUNED, C_USERS, C_L1NO, C_L2YES, C_TYES, C_SURV, C_SCAN,
  C_RCHK, C_RES, C_LONG, C_F64SCAN, C_HANDOFF, C_SQUART, C_SVALU, C_NCTR
};
static_assert(C_NCTR <= 16, "the counter array holds 16 slots");

}  // namespace rk
