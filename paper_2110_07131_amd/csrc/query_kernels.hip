// Online query kernels: Simpfer (Algorithm 3) with its linear scan
// (Algorithm 2), Sections 4.2-4.3.
//
//  filter    one wavefront per user block: Lemma 3 on the block, then u.q for
//            its 64 users (lane = user, coalesced tiled reads) and the O(1)
//            tests of Lemmas 1 and 2 (and, with an exact table, the k-th
//            value itself); ballot/popcount compaction of the undecided users
//  verify    linear scan of the norm-sorted items for each survivor
//            (Corollaries 1 and 2), one wavefront per survivor, lane = item;
//            with many survivors, 64 survivors per workgroup over shared
//            MFMA item tiles
//  recheck   float64 recomputation (oracle order) for users whose decision
//            the bulk precision cannot certify
//  finalize  result bits (by original id) -> ascending ids
//
// Every "no" and "yes" is certified: a comparison of bulk-precision values is
// used only when it holds with the error margin of both sides (rk_common.h,
// margin()); otherwise the user moves on to the next, always sound, step.
#include "rk_kernels.h"
#include "batch_device.h"

namespace rk {

__device__ __forceinline__ unsigned long long lanemask_lt() {
  const int lane = threadIdx.x & 63;
  return lane ? (~0ull >> (64 - lane)) : 0ull;
}

// Wave-aggregated append: each lane with `pred` gets a distinct slot.
__device__ __forceinline__ int wave_append(bool pred, int32_t* counter) {
  const unsigned long long mask = __ballot(pred);
  if (!mask) return -1;
  const int leader = __ffsll((long long)mask) - 1;
  int base = 0;
  if ((threadIdx.x & 63) == leader) base = atomicAdd(counter, __popcll(mask));
  base = __shfl(base, leader);
  return pred ? base + __popcll(mask & lanemask_lt()) : -1;
}

__device__ __forceinline__ void ctr_add(const QueryWS& ws, int slot, unsigned long long v) {
  if (ws.ctr && v) atomicAdd(&ws.ctr[slot], v);
}

// |q| rounded up, from every lane's share of q (any summation order: the
// float64 sum has relative error <= gamma_d; the factor covers it, the
// square root and the final product).
__device__ float wave_qnorm_up(const float* __restrict__ q, int d) {
  const int lane = threadIdx.x & 63;
  double s = 0.0;
  for (int c = lane; c < d; c += 64) s = fma((double)q[c], (double)q[c], s);
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  return f32_up(sqrt(s) * (1.0 + (double)(d + 4) * 0x1p-53));
}

__device__ __forceinline__ void set_result(const QueryWS& ws, const DevIndex& ix, int64_t r) {
  const int32_t orig = ix.permQ[r];
  atomicOr(&ws.rbits[orig >> 5], 1u << (orig & 31));
}

__device__ __forceinline__ void trace(const QueryWS& ws, const DevIndex& ix, int64_t r, int cls,
                                      float s) {
  if (ws.trace_cls) {
    const int32_t orig = ix.permQ[r];
    ws.trace_cls[orig] = (uint8_t)cls;
    if (ws.trace_s && !isnan(s)) ws.trace_s[orig] = s;
  }
}

// ---------------------------------------------------------------------------
// Bulk u.q of the lane's user in block B (coalesced tiled reads).
template <bool BF16>
__device__ __forceinline__ float block_dot(const DevIndex& ix, int64_t B, const float* __restrict__ q) {
  const int lane = threadIdx.x & 63;
  if (!BF16) {
    const float* u = ix.Qt + B * (int64_t)ix.d * TILE + lane;
    float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
    int c = 0;
    for (; c + 4 <= ix.d; c += 4) {
      a0 = fmaf(u[(c + 0) * TILE], q[c + 0], a0);
      a1 = fmaf(u[(c + 1) * TILE], q[c + 1], a1);
      a2 = fmaf(u[(c + 2) * TILE], q[c + 2], a2);
      a3 = fmaf(u[(c + 3) * TILE], q[c + 3], a3);
    }
    for (; c < ix.d; ++c) a0 = fmaf(u[c * TILE], q[c], a0);
    return (a0 + a1) + (a2 + a3);
  } else {
    const int G = ix.d16 / 8;
    const uint4* u = (const uint4*)(ix.Qb + (B * G * TILE + lane) * 8);
    float a0 = 0.f, a1 = 0.f;
    for (int g = 0; g < G; ++g) {
      const uint4 w = u[g * TILE];
      const uint32_t ws_[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        const int c = g * 8 + 2 * h;
        const float ql = c < ix.d ? bf16_round(q[c]) : 0.f;
        const float qh = c + 1 < ix.d ? bf16_round(q[c + 1]) : 0.f;
        a0 = fmaf(bf16_to_f32((uint16_t)(ws_[h] & 0xFFFFu)), ql, a0);
        a1 = fmaf(bf16_to_f32((uint16_t)(ws_[h] >> 16)), qh, a1);
      }
    }
    return a0 + a1;
  }
}

// ---------------------------------------------------------------------------
// Algorithm 3 for one query.  Wave w of the grid takes block B = w.
template <bool BF16>
__global__ void __launch_bounds__(256) k_filter(DevIndex ix, const float* __restrict__ q,
                                                int32_t k, QueryWS ws) {
  const int lane = threadIdx.x & 63;
  const int64_t B = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (B >= ix.nB) return;
  const float nq = wave_qnorm_up(q, ix.d);
  if (B == 0 && lane == 0) *ws.qnorm = nq;

  // Lemma 3: every u of a block has f(q,u) <= cs_inflate*|u_first||q|;
  // prune when that is strictly below the block's k-th lower bound.  The
  // wave's 64 users hold 64 / bsize blocks; it returns when all are pruned.
  const int64_t sb = B * (TILE / ix.bsize) + lane / ix.bsize;
  const float lbk = ix.LB[(int64_t)(k - 1) * ix.nSB + sb];
  const bool pruned = ix.use_blocks && (ix.cs_inflate * ix.bnorm[sb]) * nq < lbk;
  const unsigned long long pm = __ballot(pruned);
  if (lane == 0) {
    ctr_add(ws, C_BLOCKS, TILE / ix.bsize);
    ctr_add(ws, C_PRUNED, __popcll(pm) / ix.bsize);
  }
  if (pm == ~0ull) return;

  const int64_t r = B * TILE + lane;
  const bool valid = r < ix.n && !pruned;
  const float s = block_dot<BF16>(ix, B, q);
  const float nu = ix.normQ[r];
  const float e = margin(ix, nu, nq);
  const float L = ix.L32[(int64_t)(k - 1) * ix.n_pad + r];
  const float csk = (ix.cs_inflate * nu) * ix.normP[k - 1];

  // Lemma 1 (strict): k items have f >= L > f(q,u).
  const bool no1 = valid && (s + e < L);
  // Lemma 2: the items from the k-th on cannot beat q.
  const bool yes2 = valid && !no1 && (s - e >= csk);
  // Exact table: f(q,u) >= theta_k  <=>  member.
  const bool yesT = valid && ix.exact && !no1 && !yes2 && (s - e >= f32_next_up(L));
  const bool undecided = valid && !no1 && !yes2 && !yesT;

  if (yes2 || yesT) set_result(ws, ix, r);
  if (ws.trace_cls && valid)
    trace(ws, ix, r, no1 ? RK_C_LEMMA1_NO : (yes2 ? RK_C_LEMMA2_YES : (yesT ? RK_C_TABLE_YES : 255)), s);

  if (ix.exact) {
    // undecided users sit inside the margin of theta_k: float64 recheck
    const int pos = wave_append(undecided, &ws.cnt[1]);
    if (undecided) ws.rchk_idx[pos] = (int32_t)r;
  } else {
    const int pos = wave_append(undecided, &ws.cnt[0]);
    if (undecided) {
      ws.surv_idx[pos] = (int32_t)r;
      ws.surv_s[pos] = s;
    }
  }
  if (ws.ctr) {  // ballots taken by the whole wave, counters added by one lane
    const int c_users = __popcll(__ballot(valid));
    const int c_no1 = __popcll(__ballot(no1));
    const int c_yes2 = __popcll(__ballot(yes2));
    const int c_yesT = __popcll(__ballot(yesT));
    const int c_und = __popcll(__ballot(undecided));
    if (lane == 0) {
      ctr_add(ws, C_USERS, c_users);
      ctr_add(ws, C_L1NO, c_no1);
      ctr_add(ws, C_L2YES, c_yes2);
      ctr_add(ws, C_TYES, c_yesT);
      ctr_add(ws, ix.exact ? C_RCHK : C_SURV, c_und);
    }
  }
}

void launch_filter(const DevIndex& ix, const float* q, int32_t k, const QueryWS& ws,
                   hipStream_t s) {
  if (ix.nB == 0) return;
  dim3 g((unsigned)((ix.nB + 3) / 4));
  if (ix.bf16) hipLaunchKernelGGL(k_filter<true>, g, dim3(256), 0, s, ix, q, k, ws);
  else hipLaunchKernelGGL(k_filter<false>, g, dim3(256), 0, s, ix, q, k, ws);
}

// ---------------------------------------------------------------------------
// Algorithm 2 (Linear-scan) for every survivor; one wave per survivor, lane
// = item of the current 64-item tile.  Counts the items certified to beat q
// (Corollary 2: k of them decide "no") and stops at the first item whose
// Cauchy-Schwarz bound cannot exceed u.q (Corollary 1: nothing after it can
// beat q).  Items whose comparison is inside the margin are compared in
// float64 right there (f(p,u) against f(q,u), both in the definition's
// order; the item equal to q of a query taken from P is one of them), so
// every item's verdict is exact: "no" once k items beat q, "yes" at the
// Corollary 1 limit.
template <bool BF16>
__global__ void __launch_bounds__(256) k_verify(DevIndex ix, const float* __restrict__ q,
                                                int32_t k, QueryWS ws) {
  const int lane = threadIdx.x & 63;
  // float32: the survivor's user row, per wave, read as broadcasts (d <= 512)
  __shared__ __align__(16) float urow_s[4][BF16 ? 4 : 512];
  float* uw = urow_s[threadIdx.x >> 6];
  const int nsurv = ws.cnt[0];
  if (nsurv >= ix.verify_tiles) return;  // k_verify_tiles takes them
  const int64_t nwaves = (int64_t)gridDim.x * 4;
  const float nq = *ws.qnorm;
  for (int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); w < nsurv; w += nwaves) {
    const int64_t r = ws.surv_idx[w];
    const float s = ws.surv_s[w];
    const float nu = ix.normQ[r];
    const float euq = margin(ix, nu, nq);
    const float sl = s - euq;  // certified lower end of f(q,u)
    // stop index: first item j with cs_inflate*|u||p_j| <= sl (binary search
    // on the non-increasing item norms)
    int64_t lo = 0, hi = ix.m;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if ((ix.cs_inflate * nu) * ix.normP[mid] <= sl) hi = mid;
      else lo = mid + 1;
    }
    const int64_t stop = lo;
    int beats = 0;
    bool used64 = false;
    double fq = 0.0;
    const float* urow = ix.Qrow + r * ix.d;
    int64_t scanned = 0;
    const int64_t ub = r / TILE, ul = r % TILE;
    if (!BF16) {
      for (int c = lane; c < ix.d; c += 64) uw[c] = urow[c];
      __builtin_amdgcn_wave_barrier();
    }
    for (int64_t t0 = 0; t0 < stop && beats < k; t0 += TILE) {
      const int64_t j = t0 + lane;
      const bool inb = j < stop;
      float g = 0.f;
      if (!BF16) {
        // sixteen coordinates of item loads in flight (coalesced rows of the
        // item tile), the user's coordinates from LDS
        const float* p = ix.Pt + (t0 / TILE) * (int64_t)ix.d * TILE + lane;
        float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
        int c = 0;
        for (; c + 16 <= ix.d; c += 16) {
          float pv[16];
#pragma unroll
          for (int i = 0; i < 16; ++i) pv[i] = p[(c + i) * TILE];
#pragma unroll
          for (int i = 0; i < 16; i += 4) {
            const float4 u4 = *(const float4*)(uw + c + i);
            a0 = fmaf(u4.x, pv[i], a0);
            a1 = fmaf(u4.y, pv[i + 1], a1);
            a2 = fmaf(u4.z, pv[i + 2], a2);
            a3 = fmaf(u4.w, pv[i + 3], a3);
          }
        }
        for (; c < ix.d; ++c) a0 = fmaf(uw[c], p[c * TILE], a0);
        g = (a0 + a1) + (a2 + a3);
      } else {
        const int G = ix.d16 / 8;
        const uint4* u = (const uint4*)(ix.Qb + (ub * G * TILE + ul) * 8);
        const uint4* p = (const uint4*)(ix.Pb + ((t0 / TILE) * G * TILE + lane) * 8);
        float a0 = 0.f, a1 = 0.f;
        for (int gg = 0; gg < G; ++gg) {
          const uint4 wu = u[gg * TILE], wp = p[gg * TILE];
          const uint32_t xu[4] = {wu.x, wu.y, wu.z, wu.w}, xp[4] = {wp.x, wp.y, wp.z, wp.w};
#pragma unroll
          for (int h = 0; h < 4; ++h) {
            a0 = fmaf(bf16_to_f32((uint16_t)(xu[h] & 0xFFFFu)), bf16_to_f32((uint16_t)(xp[h] & 0xFFFFu)), a0);
            a1 = fmaf(bf16_to_f32((uint16_t)(xu[h] >> 16)), bf16_to_f32((uint16_t)(xp[h] >> 16)), a1);
          }
        }
        g = a0 + a1;
      }
      const float np = inb ? ix.normP[j] : 0.f;
      const float tol = margin(ix, nu, np) + euq;
      const float diff = g - s;
      const bool beat = inb && (diff > tol);
      const bool unc = inb && !beat && !(diff <= -tol);
      beats += __popcll(__ballot(beat));
      if (__ballot(unc)) {  // inside the margin: float64 for these items only
        if (!used64) fq = dot64_rows(q, urow, ix.d);
        used64 = true;
        const bool b64 = unc && dot64_rows(ix.Prow + j * ix.d, urow, ix.d) > fq;
        beats += __popcll(__ballot(b64));
      }
      scanned += (stop - t0 < TILE) ? (stop - t0) : TILE;
    }
    const bool yes = beats < k;
    if (!BF16) __builtin_amdgcn_wave_barrier();  // uw is rewritten for the next survivor
    if (yes && lane == 0) set_result(ws, ix, r);
    if (lane == 0) {
      trace(ws, ix, r,
            used64 ? (yes ? RK_C_RECHECK_YES : RK_C_RECHECK_NO) : (yes ? RK_C_SCAN_YES : RK_C_SCAN_NO),
            NAN);
      ctr_add(ws, C_SCAN, (unsigned long long)scanned);
      if (used64) ctr_add(ws, C_RCHK, 1);
    }
  }
}

// The same scan for many survivors at once.  A workgroup takes a chunk of up
// to 512 survivors and scans the norm-sorted item tiles for all of them in
// rounds: each round, groups of 64 of the chunk's survivors still scanning
// keep their rows in LDS and walk the round's item tiles together (64x64
// float32 MFMA products; wave w: survivors of half w&1, items of half w>>1),
// so each tile is read once per group instead of once per survivor; after
// the round the survivors that stopped leave and the rest are regrouped,
// all at the same item position.  Rounds grow from 4 to 64 tiles.  Each
// (survivor, item) gets the one-wave scan's certified test (beat if
// u.p - u.q exceeds both margins, float64 inside them); a survivor stops at
// its Corollary 1 limit or once k items beat q, tested after each tile as
// above.  Runs when the filter left at least ix.verify_tiles survivors (the
// one-wave scan then returns at once).
constexpr int kVtChunk = 512;    // survivors regrouped within a workgroup
constexpr int kVtGrid = 1024;    // workgroups of the tiled scan
constexpr int kVtChunks = 256;   // chunks the survivors are split into (while at most 512 each)
constexpr int kVtRound0 = 4;     // item tiles of the first round
constexpr int kVtRoundMax = 64;  // ... and of the longest

template <int NV>
__global__ void __launch_bounds__(256) k_verify_tiles(DevIndex ix, const float* __restrict__ q,
                                                      int32_t k, QueryWS ws) {
  const int nsurv = ws.cnt[0];
  if (nsurv < ix.verify_tiles) return;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int half = lane >> 5, col = lane & 31, uh = wave & 1, ih = wave >> 1;
  const int d = ix.d, d2 = d + (d & 1);
  float* ubuf = (float*)lds_raw;   // [d2][64] the current group's survivors (columns)
  float* pbuf = ubuf + d2 * TILE;  // [d2][64] the current item tile
  // the chunk's survivors: sorted user index, u.q, |u|, its margin, limit,
  // beats so far, float64 used
  __shared__ int32_t r_c[kVtChunk], stop_c[kVtChunk], beats_c[kVtChunk], f64_c[kVtChunk];
  __shared__ float s_c[kVtChunk], nu_c[kVtChunk], euq_c[kVtChunk];
  __shared__ int32_t act_l[2][kVtChunk];  // survivors still scanning (chunk positions), ping-pong
  __shared__ int32_t gm[TILE];            // chunk position of each column of the group
  __shared__ int32_t act_n[2];
  __shared__ float np_s[TILE];
  const float nq = *ws.qnorm;
  // chunks of 64..512 survivors, about one per CU (measured against one per
  // workgroup of the grid, and 512 always, on 48k- and 480k-survivor queries)
  const int per = min(kVtChunk / TILE, max(1, (nsurv + TILE * kVtChunks - 1) / (TILE * kVtChunks)));
  const int CH = per * TILE;
  const int nchunks = (nsurv + CH - 1) / CH;
  const int nv = d * (TILE / 4);  // 16-byte vectors of an item tile
  const int u = uh * 32 + col;    // the lane's column
  unsigned long long c_scan = 0, c_f64 = 0;
  u32x4 pf[NV];
  auto load_tile = [&](int64_t I) {
    const u32x4* src = (const u32x4*)(ix.Pt + I * d * TILE);
#pragma unroll
    for (int v = 0; v < NV; ++v)
      if (v * 256 + t < nv) pf[v] = src[v * 256 + t];
  };
  for (int ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
    const int cnt = min(CH, nsurv - ch * CH);
    if (t == 0) act_n[0] = 0;
    __syncthreads();
    for (int i = t; i < cnt; i += 256) {
      const int32_t r = ws.surv_idx[(int64_t)ch * CH + i];
      const float sv = ws.surv_s[(int64_t)ch * CH + i];
      const float nu = ix.normQ[r];
      const float euq = margin(ix, nu, nq);
      const float sl = sv - euq;  // certified lower end of f(q,u)
      int64_t lo = 0, hi = ix.m;  // Corollary 1 limit, as in the one-wave scan
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((ix.cs_inflate * nu) * ix.normP[mid] <= sl) hi = mid;
        else lo = mid + 1;
      }
      r_c[i] = r;
      s_c[i] = sv;
      nu_c[i] = nu;
      euq_c[i] = euq;
      stop_c[i] = (int32_t)lo;
      beats_c[i] = 0;
      f64_c[i] = 0;
      if (lo > 0) act_l[0][atomicAdd(&act_n[0], 1)] = i;
    }
    __syncthreads();
    int64_t P = 0;  // item tile every scanning survivor of the chunk has reached
    int len = kVtRound0, cur = 0;
    while (act_n[cur] > 0 && P < ix.mB) {
      const int na = act_n[cur];
      const int64_t P1 = min(P + (int64_t)len, ix.mB);
      for (int g0 = 0; g0 < na; g0 += TILE) {
        const int ng = min(TILE, na - g0);
        if (t < TILE) gm[t] = t < ng ? act_l[cur][g0 + t] : -1;
        __syncthreads();
        for (int i = t; i < d * TILE; i += 256) {
          const int c = i & (TILE - 1);
          ubuf[i] = c < ng ? ix.Qrow[(int64_t)r_c[gm[c]] * d + (i >> 6)] : 0.f;
        }
        if (d & 1) {
          if (t < TILE) ubuf[d * TILE + t] = 0.f;
          else if (t < 2 * TILE) pbuf[d * TILE + t - TILE] = 0.f;
        }
        const int mine = u < ng ? gm[u] : -1;
        load_tile(P);
        for (int64_t I = P; I < P1; ++I) {
          __syncthreads();  // the counts of tile I - 1 are in; pbuf is free
          // every wave reads the same settled state, so all leave together
          const int gl = lane < ng ? gm[lane] : -1;
          if (!__ballot(gl >= 0 && beats_c[gl] < k && I * TILE < stop_c[gl])) break;
          const bool act = mine >= 0 && beats_c[mine] < k && I * TILE < stop_c[mine];
          {
            u32x4* dst = (u32x4*)pbuf;
#pragma unroll
            for (int v = 0; v < NV; ++v)
              if (v * 256 + t < nv) dst[v * 256 + t] = pf[v];
          }
          if (t < TILE) np_s[t] = I * TILE + t < ix.m ? ix.normP[I * TILE + t] : 0.f;
          if (I + 1 < P1) load_tile(I + 1);
          __syncthreads();  // pbuf holds tile I
          if (!__ballot(act)) continue;
          f32x16 acc = {};
          const float* pa = pbuf + ih * 32 + col + half * TILE;
          const float* ua = ubuf + uh * 32 + col + half * TILE;
          for (int ks = 0; ks < d2 / 2; ++ks)
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(pa[2 * ks * TILE], ua[2 * ks * TILE], acc, 0, 0, 0);
          if (!act) continue;
          const int stop = stop_c[mine];
          const float sv = s_c[mine], nu = nu_c[mine], euq = euq_c[mine];
          int beats = 0;
          unsigned unc = 0;  // rows inside the margins
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const int row = quarter_row(ih, half, r);
            // the float32 product's own margin plus u.q's (bulk precision)
            const float tol = (ix.eps_rel32 * (nu * np_s[row]) + ix.eps_abs) + euq;
            const float diff = acc[r] - sv;
            const bool in = I * TILE + row < stop;
            beats += in && diff > tol;
            unc |= (unsigned)(in && !(diff > tol) && !(diff <= -tol)) << r;
          }
          if (unc) {  // float64 for these items only
            const float* urow = ix.Qrow + (int64_t)r_c[mine] * d;
            const double fq = dot64_rows(q, urow, d);
            for (; unc; unc &= unc - 1) {
              const int64_t j = I * TILE + quarter_row(ih, half, __ffs(unc) - 1);
              beats += dot64_rows(ix.Prow + j * d, urow, d) > fq;
            }
            f64_c[mine] = 1;
          }
          if (beats) atomicAdd(&beats_c[mine], beats);
          if (ih == 0 && half == 0) c_scan += (unsigned long long)min((int64_t)TILE, (int64_t)stop - I * TILE);
        }
        __syncthreads();  // the group's counts are in; gm and ubuf are free
      }
      // the survivors still scanning at P1, regrouped for the next round
      if (t == 0) act_n[cur ^ 1] = 0;
      __syncthreads();
      for (int i = t; i < na; i += 256) {
        const int c = act_l[cur][i];
        if (beats_c[c] < k && P1 * TILE < stop_c[c]) act_l[cur ^ 1][atomicAdd(&act_n[cur ^ 1], 1)] = c;
      }
      __syncthreads();
      cur ^= 1;
      P = P1;
      len = min(2 * len, kVtRoundMax);
    }
    for (int i = t; i < cnt; i += 256) {
      const bool yes = beats_c[i] < k;
      const int64_t r = r_c[i];
      if (yes) set_result(ws, ix, r);
      trace(ws, ix, r,
            f64_c[i] ? (yes ? RK_C_RECHECK_YES : RK_C_RECHECK_NO) : (yes ? RK_C_SCAN_YES : RK_C_SCAN_NO),
            NAN);
      c_f64 += (unsigned long long)f64_c[i];
    }
    __syncthreads();  // the chunk's state is read before the next chunk writes it
  }
  if (ws.ctr) {
    for (int off = 32; off > 0; off >>= 1) {
      c_scan += __shfl_xor(c_scan, off);
      c_f64 += __shfl_xor(c_f64, off);
    }
    if (lane == 0) {
      ctr_add(ws, C_SCAN, c_scan);
      ctr_add(ws, C_RCHK, c_f64);
    }
  }
}

template <int NV>
static void verify_tiles_nv(const DevIndex& ix, const float* q, int32_t k, const QueryWS& ws,
                            hipStream_t s) {
  const size_t lds = 2 * (size_t)(ix.d + (ix.d & 1)) * TILE * sizeof(float);
  if (lds > 65536)
    (void)hipFuncSetAttribute((const void*)k_verify_tiles<NV>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(k_verify_tiles<NV>, dim3(kVtGrid), dim3(256), lds, s, ix, q, k, ws);
}

void launch_verify(const DevIndex& ix, const float* q, int32_t k, const QueryWS& ws,
                   hipStream_t s) {
  if (ix.nB == 0 || ix.exact) return;
  dim3 g(512);
  if (ix.bf16) hipLaunchKernelGGL(k_verify<true>, g, dim3(256), 0, s, ix, q, k, ws);
  else hipLaunchKernelGGL(k_verify<false>, g, dim3(256), 0, s, ix, q, k, ws);
  // the survivor count is known on the device only: both scans are queued,
  // and the one not meant for it returns at once
  if (ix.verify_tiles == INT32_MAX) return;
  const int per_thread = (ix.d * (TILE / 4) + 255) / 256;  // 16-byte vectors of an item tile
  if (per_thread <= 2) verify_tiles_nv<2>(ix, q, k, ws, s);
  else if (per_thread <= 4) verify_tiles_nv<4>(ix, q, k, ws, s);
  else if (per_thread <= 8) verify_tiles_nv<8>(ix, q, k, ws, s);
  else verify_tiles_nv<16>(ix, q, k, ws, s);
}

// ---------------------------------------------------------------------------
// Float64 recomputation, one thread per user: f(q,u) in the oracle's order.
// With an exact table the decision is f(q,u) >= theta_k(u).  Otherwise the
// linear scan of Algorithm 2 runs entirely in float64: count items with
// f(p,u) > f(q,u) up to k, stopping at the first item whose Cauchy-Schwarz
// bound cannot exceed f(q,u).
__global__ void __launch_bounds__(256) k_recheck(DevIndex ix, const float* __restrict__ q,
                                                 int32_t k, QueryWS ws) {
  const int n = ws.cnt[1];
  const double cs = (double)ix.cs_inflate;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = ws.rchk_idx[t];
    const float* u = ix.Qrow + r * ix.d;
    const double fq = dot64_rows(q, u, ix.d);
    bool yes;
    if (ix.exact) {
      yes = fq >= ix.L64[(int64_t)(k - 1) * ix.n_pad + r];
    } else {
      const double nu = (double)ix.normQ[r];
      int beats = 0;
      for (int64_t j = 0; j < ix.m && beats < k; ++j) {
        if (cs * nu * (double)ix.normP[j] * (1.0 + 0x1p-50) <= fq) break;
        beats += dot64_rows(ix.Prow + j * ix.d, u, ix.d) > fq;
      }
      yes = beats < k;
    }
    if (yes) set_result(ws, ix, r);
    trace(ws, ix, r, yes ? RK_C_RECHECK_YES : RK_C_RECHECK_NO, NAN);
  }
}

void launch_recheck(const DevIndex& ix, const float* q, int32_t k, const QueryWS& ws,
                    hipStream_t s) {
  if (ix.nB == 0) return;
  hipLaunchKernelGGL(k_recheck, dim3(64), dim3(256), 0, s, ix, q, k, ws);
}

// ---------------------------------------------------------------------------
// Result assembly: one workgroup turns the result bits (original-id order)
// into ascending ids, clears the bits and the per-query counters.  With
// `base` (batch form) the ids go to ids[*base ...] and *out = *base + count
// (the next CSR offset); otherwise to ids[0 ...] and *out = count.  Ids at
// positions >= cap are dropped; *out is always exact.
__global__ void __launch_bounds__(1024) k_finalize(int64_t n, QueryWS ws, int32_t* __restrict__ ids,
                                                   int64_t cap, const int64_t* __restrict__ base,
                                                   int64_t* __restrict__ out,
                                                   unsigned long long* ctr) {
  __shared__ int64_t part[1024];
  const int64_t W = (n + 31) / 32;
  const int t = threadIdx.x;
  const int64_t w0 = W * t / 1024, w1 = W * (t + 1) / 1024;
  int64_t c = 0;
  for (int64_t w = w0; w < w1; ++w) c += __popc(ws.rbits[w]);
  part[t] = c;
  __syncthreads();
  // inclusive scan (Hillis-Steele) over 1024 partial counts
  for (int off = 1; off < 1024; off <<= 1) {
    int64_t v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  const int64_t b0 = base ? *base : 0;
  int64_t pos = b0 + part[t] - c;
  for (int64_t w = w0; w < w1; ++w) {
    uint32_t bits = ws.rbits[w];
    if (!bits) continue;
    ws.rbits[w] = 0u;
    while (bits) {
      const int b = __ffs(bits) - 1;
      bits &= bits - 1;
      if (pos < cap) ids[pos] = (int32_t)(w * 32 + b);
      ++pos;
    }
  }
  if (t == 1023) {
    *out = b0 + part[1023];
    ws.cnt[0] = 0;
    ws.cnt[1] = 0;
    if (ctr) atomicAdd(&ctr[C_RES], (unsigned long long)part[1023]);
  }
}

void launch_finalize(const DevIndex& ix, const QueryWS& ws, int32_t* ids, int64_t cap,
                     const int64_t* base, int64_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), 0, s, ix.n, ws, ids, cap, base, out, ws.ctr);
}

// k > m: every user is a member (same output convention as k_finalize).
__global__ void k_fill_all(int64_t n, int32_t* ids, int64_t cap, const int64_t* base,
                           int64_t* out) {
  const int64_t b0 = base ? *base : 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n && b0 + i < cap;
       i += (int64_t)gridDim.x * blockDim.x)
    ids[b0 + i] = (int32_t)i;
  if (blockIdx.x == 0 && threadIdx.x == 0) *out = b0 + n;
}

void launch_fill_all(int64_t n, int32_t* ids, int64_t cap, const int64_t* base, int64_t* out,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_fill_all, dim3(256), dim3(256), 0, s, n, ids, cap, base, out);
}

__global__ void k_set_i64(int64_t* p, int64_t v) { *p = v; }

void launch_set_i64(int64_t* p, int64_t v, hipStream_t s) {
  hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(1), 0, s, p, v);
}

}  // namespace rk
