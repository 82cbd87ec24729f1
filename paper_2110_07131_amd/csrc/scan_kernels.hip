// The bounded table's undecided pairs: the grouped linear scan (Algorithm 2
// with Corollaries 1 and 2) of every pair of a user block at once, group
// passes of the users handed over from several blocks, and the decisions of
// their pairs.
#include "batch_device.h"
#include <climits>

namespace rk {

// ---------------------------------------------------------------------------
// Grouped linear scan (bounded table): Algorithm 2 for every undecided pair of
// one user block at once.  u.p does not depend on q, so the scan's products
// are computed once per (user, item) of the block, in 64x64 float32 MFMA tiles
// over the items in norm order, and each pair reads them through an order
// statistic: within a prefix of the items at least k items beat q iff the
// k-th largest u.p of the prefix exceeds f(q,u) (Corollary 2), and once the
// prefix reaches the pair's Corollary 1 limit (the first item with
// cs|u||p| <= a lower bound of f(q,u); no later item can beat q) fewer than k
// beats in it mean "yes".  Each user keeps the k_max largest approximate
// products of the items scanned so far (LDS).  With e = eps|u||p_0| + eps_abs
// bounding the error of every product of the prefix and [lo, hi] = s -+ e_q
// bounding f(q,u):
//   no   iff  top_k - e > hi;   yes iff  top_k + e <= lo   (top_k = -inf when
//   the prefix has fewer than k items); otherwise the float64 scan decides.
// Short pass: the first kShortTiles item tiles, then every pair is read once;
// most pairs end here.  The others are flagged; the scan then continues, for
// the users that have such pairs only, until each of their pairs is either
// decided no (k list entries certainly above it: Algorithm 2's early exit)
// or covered to its limit, and the flagged pairs are decided at the end.
// The last users of a block still scanning with a long way to go are handed
// to group passes that continue 64 such users from any blocks at once.  The
// lists and their coverage carry over to the next query chunk of the call.
constexpr int kShortTiles = 4;
// ... and when it runs for every block ahead of the filter, whose bounds it
// tightens (4, 8, 12 and 16 tiles measured 86, 83, 80 and 80 ms per step on
// 1M users x 100k items, P' = 50; 4.9, 4.4, 4.3 and 4.3 ms on 100k x 20k)
constexpr int kPrescanTiles = 12;
// pass 1 stages a block's chunk ids and fills (at most 64 x 4096 / 256 + 4
// each) in the candidate region
static_assert(2 * (TILE * kBatchChunkMax / kPairChunk + 4) <= TILE * TILE,
              "the chunk lists of a block fit the candidate region");
// ALIAS mode: floats of the item-tile region (the tile, or the candidates,
// their rows and the pair slots, whichever is larger)
__host__ __device__ constexpr int bscan_tile_region(int d2) {
  return d2 * TILE > TILE * TILE + TILE * TILE / 4 + 3 * TILE * kUserPairs
             ? d2 * TILE
             : TILE * TILE + TILE * TILE / 4 + 3 * TILE * kUserPairs;
}
constexpr int kFlagCap = 1024;  // flagged pairs listed in LDS per block
constexpr int kHandoff = 24;    // at most this many users of a block still scanning: hand them over
constexpr int kGroupHandoff = 16;  // the same for a group pass (but the last)
constexpr int kGroupLevels = 2;    // group passes (thresholds and depth measured on 1M users x 100k items)
// ... and only with more than ix.handoff_tiles item tiles left (512 unless
// the index options say otherwise: shorter tails cost less where they are
// than the extra passes)


template <int NV>
__device__ __forceinline__ void load_item_tile(const DevIndex& ix, int64_t I, int t,
                                               u32x4 (&pf)[NV]) {
  const u32x4* src = (const u32x4*)(ix.Pt + I * (int64_t)ix.d * TILE);
  const int nv = ix.d * (TILE / 4);
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const int i = v * 256 + t;
    if (i < nv) pf[v] = src[i];
  }
}

template <int NV>
__device__ __forceinline__ void store_item_tile(float* pbuf, int d, int t, const u32x4 (&pf)[NV]) {
  u32x4* dst = (u32x4*)pbuf;
  const int nv = d * (TILE / 4);
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const int i = v * 256 + t;
    if (i < nv) dst[i] = pf[v];
  }
}

// f(q,u) approximated in float32, sequential over the coordinates (query row
// in caller order, user column of the block tile in LDS).
__device__ __forceinline__ float dot32_col(const float* __restrict__ q, const float* ucol, int d) {
  float acc = 0.f;
  for (int c = 0; c < d; ++c) acc = fmaf(q[c], ucol[c * TILE], acc);
  return acc;
}

// Order-preserving map between the bits of a float and an int, its own
// inverse: for non-NaN floats a < b iff fkey(bits a) < fkey(bits b).
__device__ __forceinline__ int fkey(int b) { return b >= 0 ? b : b ^ 0x7fffffff; }

// An undecided pair, decided exactly from the user's list of the k_max
// largest products of the prefix (values and item ids): entries certainly
// above f(q,u) count, entries within the error band are compared in float64
// (usually the one item equal to q), and the items outside the list are below
// its last entry, certainly not above f(q,u) unless that entry is itself in
// the band, when the float64 scan decides.  The prefix must reach the pair's
// Corollary 1 limit; when it does not (short_prefix), the float64 scan
// decides directly.
__device__ __forceinline__ bool resolve_pair(const DevIndex& ix, const BatchView& bv, int64_t u,
                                          int32_t jj, int k, float lo, float hi, float nu,
                                          const float* tk, const int32_t* ti, int K,
                                          bool short_prefix, unsigned long long& full_scans) {
  if (short_prefix) {
    ++full_scans;
    return decide_f64(ix, bv, u, jj);
  }
  const float* urow = ix.Qrow + u * ix.d;
  const float* qrow = bv.qs + (int64_t)bv.perm[jj] * ix.d;
  double fq = 0.0;
  bool have_fq = false;
  int beats = 0;
  for (int p = 0; p < K; ++p) {
    const int32_t id = ti[p];
    if (id < 0) return true;  // the prefix has no further item
    const float v = tk[p];
    const float ei = ix.eps_rel32 * (nu * ix.normP[id]) + ix.eps_abs;
    if (v - ei > hi) {
      ++beats;
    } else if (!(v + ei <= lo)) {
      if (!have_fq) {
        fq = dot64_rows(qrow, urow, ix.d);
        have_fq = true;
      }
      beats += dot64_rows(ix.Prow + (int64_t)id * ix.d, urow, ix.d) > fq;
    }
    if (beats >= k) return false;
  }
  const float eK = ix.eps_rel32 * (nu * ix.normP[0]) + ix.eps_abs;
  if (tk[K - 1] + eK <= lo) return true;
  ++full_scans;
  return decide_f64(ix, bv, u, jj);
}

// Four lanes of a quad exchange a value (lane ^ 1, lane ^ 2).
__device__ __forceinline__ int quad_xor1(int v) { return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false); }
__device__ __forceinline__ int quad_xor2(int v) { return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false); }

// (value, position) minimum over the four lanes of a quad; ties go to the
// smaller position, so all four lanes agree.
__device__ __forceinline__ void quad_min(float& v, int& p) {
  float ov = __int_as_float(quad_xor1(__float_as_int(v)));
  int op = quad_xor1(p);
  if (ov < v || (ov == v && op < p)) v = ov, p = op;
  ov = __int_as_float(quad_xor2(__float_as_int(v)));
  op = quad_xor2(p);
  if (ov < v || (ov == v && op < p)) v = ov, p = op;
}

__device__ __forceinline__ int quad_sum(int v) {
  v += quad_xor1(v);
  return v + quad_xor2(v);
}

// GROUP = false: workgroup B = user block B, all passes; users still scanning
// when at most kHandoff of the block are, are handed over.  GROUP = true:
// workgroup B = the handed-over users 64B .. 64B+63 of the current list
// (from any blocks), the long pass only, continued from their lists; it
// hands over its last kGroupHandoff users in turn, but in the last group
// pass.  Their pairs are decided by k_bdecide.
template <int NV, bool GROUP, bool ALIAS>
__global__ void __launch_bounds__(256) k_bscan(DevIndex ix, BatchView bv) {
  const int64_t B = blockIdx.x;
  int nch = 0, nusers = TILE;
  const int32_t* glist = bv.sg_sorted;  // group's input: the current list ordered by depth
  int32_t* hlist = bv.sg_users + (int64_t)(GROUP ? (bv.sg_level & 1) ^ 1 : 0) * ix.n_pad;  // handed over
  int32_t* hcount = bv.sg_count + (GROUP ? (bv.sg_level & 1) ^ 1 : 0);
  if (GROUP) {
    const int cnt = bv.sg_count[bv.sg_level & 1];
    if (B * TILE >= cnt) return;
    nusers = (int)min((int64_t)TILE, cnt - B * TILE);
  } else {
    // (the first pass of a call over every block: no pairs yet)
    nch = bv.prescan ? 0 : min(bv.bcnt[B], bv.maxc);
    if (nch == 0 && !bv.prescan) return;
  }
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int half = lane >> 5, col = lane & 31;
  const int uh = wave & 1, ih = wave >> 1;
  // list upkeep: the four lanes of quad uo serve user uo; lane sub holds the
  // list entries j = 4i + sub
  const int uo = t >> 2, sub = t & 3;
  // K >= k_max + 2 list entries (a multiple of 4): the entry after the k-th
  // is usually not the item equal to q, so an undecided pair rarely needs
  // the float64 scan
  const int d = ix.d, d2 = d + (d & 1), K = bscan_list_len(ix.kmax), K4 = K / 4;
  // ALIAS (65 <= d <= 128, and wider tiles whose separate buffers would not
  // fit): the candidates, their rows and the pair slots share the item
  // tile's region (written after a barrier once every wave has read the
  // tile), and there is no list of flagged pairs, so that two workgroups fit
  // a CU up to d ~ 110.
  float* ubuf = (float*)lds_raw;        // [d2][64] users of the block
  float* pbuf = ubuf + d2 * TILE;       // [d2][64] current item tile
  float* pend = pbuf + (ALIAS ? bscan_tile_region(d2) : d2 * TILE);
  float* cand = ALIAS ? pbuf : pend;    // [64][64] candidates of the tile per user
  float* topk = ALIAS ? pend : cand + TILE * TILE;  // [64][K] list values (sorted after each pass)
  int32_t* topi = (int32_t*)(topk + TILE * K);  // [64][K] their item ids (-1: none)
  float* thr = (float*)(topi + TILE * K);       // [64] smallest list value
  int* ccnt = (int*)(thr + TILE);       // [64] candidates per user
  int* open = ccnt + TILE;              // [64] 1 while a flagged pair of the user needs items
  int* Cov = open + TILE;               // [64] items covered by the user's list
  // [64][64] candidate rows within the tile
  uint8_t* crow = ALIAS ? (uint8_t*)(pbuf + TILE * TILE) : (uint8_t*)(Cov + TILE);
  __shared__ int nflag, more_w[4];
  constexpr int flist_cap = ALIAS ? 0 : kFlagCap;
  __shared__ int32_t flist[ALIAS ? 1 : kFlagCap];  // slots of the flagged pairs
  // Long pass, per user: kUserPairs slots of flagged pairs (largest k,
  // smallest lower and largest upper bound of f(q,u), as ordered integer
  // keys); the last slot holds the extremes over the user's remaining pairs,
  // which settle when it does.  A slot settles once the list has k entries
  // certainly above its upper bound (its pairs are no: Alg. 2's early exit)
  // or the scan reaches its Corollary 1 limit (cs|u||p_i| <= its lower
  // bound); a user stops when all its slots have.  Also the user's error
  // bound of a product.
  __shared__ int npu[TILE];
  __shared__ int slots_st[ALIAS ? 1 : 3 * TILE * kUserPairs];
  int* pk_s = ALIAS ? (int*)(pbuf + TILE * TILE + TILE * TILE / 4) : slots_st;
  int* plo_s = pk_s + TILE * kUserPairs;
  int* phi_s = plo_s + TILE * kUserPairs;
  __shared__ float eu[TILE];
  __shared__ float nu_s[TILE];  // |u| of the block's users (pass 1)
  const int32_t* clist = bv.bchunks + B * bv.maxc;
  // sorted index of the user of column c (c < nusers)
  auto urow = [&](int c) -> int64_t { return GROUP ? (int64_t)glist[B * TILE + c] : B * TILE + c; };

  {
    if (GROUP) {  // gather the users' rows into columns
      for (int i = t; i < d * TILE; i += 256) {
        const int c = i & (TILE - 1);
        ubuf[i] = c < nusers ? ix.Qrow[urow(c) * d + (i >> 6)] : 0.f;
      }
    } else {
      const u32x4* src = (const u32x4*)(ix.Qt + B * (int64_t)d * TILE);
      u32x4* dst = (u32x4*)ubuf;
      for (int i = t; i < d * TILE / 4; i += 256) dst[i] = src[i];
    }
    if (d & 1) {
      if (t < TILE) ubuf[d * TILE + t] = 0.f;
      else if (t < 2 * TILE) pbuf[d * TILE + t - TILE] = 0.f;
    }
    // lists carried from the previous chunks of this call or handed over (or empty)
    for (int i = t; i < TILE * K; i += 256) {
      const int c = i / K;
      const bool have = GROUP ? c < nusers : bv.carry_in && bv.gdone[B * TILE + c] > 0;
      const int64_t at = have ? urow(c) * K + (i - c * K) : 0;
      topk[i] = have ? bv.gl_v[at] : -INFINITY;
      topi[i] = have ? bv.gl_i[at] : -1;
    }
    if (t < TILE) {
      // padding columns of a group count as fully scanned
      Cov[t] = GROUP ? (t < nusers ? bv.gdone[urow(t)] : (int)ix.m) : bv.carry_in ? bv.gdone[B * TILE + t] : 0;
      ccnt[t] = 0;
      open[t] = 0;
      npu[t] = 0;
    }
    if (t == 0) nflag = 0;
  }
  const int nshort = (int)min((int64_t)(bv.prescan ? kPrescanTiles : kShortTiles), (int64_t)ix.mB);
  unsigned long long c_scan = 0, c_l2 = 0, c_f64 = 0, c_long = 0, c_full = 0, c_quart = 0, c_valu = 0;
  // Quad uo: its lane's smallest entry (lmn at lmp) and the list's (gmn at
  // gpos).  The lists are sorted (or empty) here and after every pass, the
  // minimum last.
  float lmn, gmn;
  int lmp, gpos;
  auto list_reset = [&]() {
    lmp = K - 4 + sub;
    lmn = topk[uo * K + lmp];
    gpos = K - 1;
    gmn = topk[uo * K + K - 1];
  };
  bool handoff = false;  // the last users handed over to a group pass
  int nopen0 = TILE;     // users still scanning when the long pass starts
  // Long pass, quad uo: its user's slots still open (bit p); per slot k,
  // bounds and the number of list entries v with v - e > hi, kept as entries
  // are replaced; hmin is the smallest upper bound of an open slot (a product
  // below it changes no count).
  unsigned rem = 0;
  float eut = 0.f, csut = 0.f, hmin = INFINITY;
  int pk[kUserPairs], cnt[kUserPairs];
  float plo[kUserPairs], ph[kUserPairs];
  // nlim: the first tile end at which an open slot of the user reaches its
  // Corollary 1 limit; between such tile ends a slot settles only when the
  // list changes (its count), so the tile loop tests the slots only then.
  int nlim = INT_MAX;
  // first tile end j*64 (< m) with cs|u||p_j*64| <= lo, else the end of the
  // catalog (mB*64 >= m): the test settle makes there, by bisection over
  // the non-increasing norms
  auto limit_pos = [&](float lo) -> int {
    int a = 1, b = (int)ix.mB;
    while (a < b) {
      const int mid = (a + b) >> 1;
      if (csut * ix.normP[(int64_t)mid * TILE] <= lo) b = mid;
      else a = mid + 1;
    }
    return a * TILE;
  };
  // the quad's lanes split the open slots, then agree on the minimum
  auto update_nlim = [&]() {
    int l = INT_MAX;
    for (int p = sub; p < kUserPairs; p += 4)
      if ((rem >> p) & 1u) l = min(l, limit_pos(plo[p]));
    l = min(l, quad_xor1(l));
    nlim = min(l, quad_xor2(l));
  };
  // settles the slots decided no, or covered to their limit at item pos
  // (npos = |p_pos|)
  auto settle = [&](int pos, float npos) {
    const bool end = pos >= ix.m;
    float h = INFINITY;
#pragma unroll
    for (int p = 0; p < kUserPairs; ++p) {
      if (cnt[p] >= pk[p] || end || csut * npos <= plo[p]) rem &= ~(1u << p);
      if ((rem >> p) & 1u) h = fminf(h, ph[p]);
    }
    hmin = h;
  };

  // Item tiles from I0 (to I1, or until no user of the block has an open
  // pair): MFMA quarter (user half uh, item half ih) for the active users;
  // products above the user's list minimum become candidates; the user's
  // quad then puts each candidate in place of the list's minimum.  The next
  // tile is prefetched into registers.
  u32x4 pf[NV];
  // the next tile into pbuf (ALIAS: also its zero row for odd d, which the
  // candidates overwrote)
  auto store_tile = [&]() {
    store_item_tile(pbuf, d, t, pf);
    if (ALIAS && (d & 1) && t < TILE) pbuf[d * TILE + t] = 0.f;
  };
  auto scan_tiles = [&](int I0, int I1, bool all_users) {
    if (I0 >= I1) return;
    load_item_tile(ix, I0, t, pf);
    __syncthreads();
    store_tile();
    if (I0 + 1 < I1) load_item_tile(ix, I0 + 1, t, pf);
    for (int I = I0; I < I1; ++I) {
      __syncthreads();  // pbuf holds tile I; candidate lists are empty
      if (!all_users && !(more_w[0] | more_w[1] | more_w[2] | more_w[3])) break;
      // (a group hands over only if it started with more than twice as many)
      if (!all_users && (!GROUP || (!bv.sg_last && nopen0 > 2 * kGroupHandoff)) &&
          ix.mB - I > ix.handoff_tiles &&
          __popcll(__ballot(open[lane] != 0)) <= (GROUP ? kGroupHandoff : kHandoff)) {
        handoff = true;
        break;
      }
      const int64_t pos = (int64_t)(I + 1) * TILE;  // items covered after this tile
      const float npos = !all_users && pos < ix.m ? ix.normP[pos] : 0.f;
      const int ul = uh * 32 + col;
      // users whose list already covers the tile skip it
      const bool act = (all_users || open[ul]) && I * TILE >= Cov[ul];
      // Long pass with at most 8 active users (the block's last ones): wave w
      // computes the products of the w-th and (w+4)-th active user over the
      // tile on the vector ALU, one item per lane, instead of MFMA quarters.
      unsigned long long am = 0;
      if (!all_users) am = __ballot(open[lane] && I * TILE >= Cov[lane]);
      const bool sparse = !all_users && __popcll(am) <= 8;
      const int64_t left = ix.m - (int64_t)I * TILE;  // items of this tile that exist
      int u0 = -1, u1 = -1;
      float va = 0.f, vb = 0.f;
      f32x16 acc = {};
      bool dense = false;
      if (sparse) {
        unsigned long long mk = am;
        for (int i = 0; i < wave; ++i) mk &= mk - 1;
        u0 = mk ? __ffsll(mk) - 1 : -1;
        for (int i = 0; i < 4 && mk; ++i) mk &= mk - 1;
        u1 = mk ? __ffsll(mk) - 1 : -1;
        const float* pc = pbuf + lane;
        if (u0 >= 0 && u1 < 0) {
          float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
          const float* x0 = ubuf + u0;
          int k = 0;
          for (; k + 4 <= d; k += 4) {
            a0 = fmaf(pc[k * TILE], x0[k * TILE], a0);
            a1 = fmaf(pc[(k + 1) * TILE], x0[(k + 1) * TILE], a1);
            a2 = fmaf(pc[(k + 2) * TILE], x0[(k + 2) * TILE], a2);
            a3 = fmaf(pc[(k + 3) * TILE], x0[(k + 3) * TILE], a3);
          }
          for (; k < d; ++k) a0 = fmaf(pc[k * TILE], x0[k * TILE], a0);
          va = (a0 + a1) + (a2 + a3);
        } else if (u1 >= 0) {
          float a0 = 0.f, a1 = 0.f, b0 = 0.f, b1 = 0.f;
          const float* x0 = ubuf + u0;
          const float* x1 = ubuf + u1;
          int k = 0;
          for (; k + 2 <= d; k += 2) {
            const float p0 = pc[k * TILE], p1 = pc[(k + 1) * TILE];
            a0 = fmaf(p0, x0[k * TILE], a0);
            b0 = fmaf(p0, x1[k * TILE], b0);
            a1 = fmaf(p1, x0[(k + 1) * TILE], a1);
            b1 = fmaf(p1, x1[(k + 1) * TILE], b1);
          }
          if (k < d) {
            a0 = fmaf(pc[k * TILE], x0[k * TILE], a0);
            b0 = fmaf(pc[k * TILE], x1[k * TILE], b0);
          }
          va = a0 + a1;
          vb = b0 + b1;
        }
      } else if (__ballot(act)) {
        dense = true;
        f32x16 acc2 = {};
        const float* pf_ = pbuf + ih * 32 + col + half * TILE;
        const float* uf = ubuf + uh * 32 + col + half * TILE;
        const int nsteps = d2 / 2;
        int ks = 0;
        for (; ks + 4 <= nsteps; ks += 4) {
          float a[4], b[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            a[i] = pf_[(2 * (ks + i)) * TILE];
            b[i] = uf[(2 * (ks + i)) * TILE];
          }
          acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[0], b[0], acc, 0, 0, 0);
          acc2 = __builtin_amdgcn_mfma_f32_32x32x2f32(a[1], b[1], acc2, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[2], b[2], acc, 0, 0, 0);
          acc2 = __builtin_amdgcn_mfma_f32_32x32x2f32(a[3], b[3], acc2, 0, 0, 0);
        }
        for (; ks < nsteps; ++ks)
          acc = __builtin_amdgcn_mfma_f32_32x32x2f32(pf_[2 * ks * TILE], uf[2 * ks * TILE], acc, 0, 0, 0);
        acc += acc2;
      }
      if (bv.ctr && lane == 0) {
        c_quart += dense;
        c_valu += sparse && wave == 0;
      }
      if (ALIAS) __syncthreads();  // every wave has read the tile: its region takes the candidates
      // products above the user's list minimum become candidates
      if (sparse) {
        if (u0 >= 0 && lane < left && va > thr[u0]) {
          const int at = atomicAdd(&ccnt[u0], 1);
          cand[u0 * TILE + at] = va;
          crow[u0 * TILE + at] = (uint8_t)lane;
        }
        if (u1 >= 0 && lane < left && vb > thr[u1]) {
          const int at = atomicAdd(&ccnt[u1], 1);
          cand[u1 * TILE + at] = vb;
          crow[u1 * TILE + at] = (uint8_t)lane;
        }
      } else if (dense && act) {
        const float th = thr[ul];
        // most tiles of the long pass have no product above the list minimum
        float mx = acc[0];
#pragma unroll
        for (int r = 1; r < 16; ++r) mx = fmaxf(mx, acc[r]);
        if (left < TILE || mx > th) {
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const int row = quarter_row(ih, half, r);
            if (row < left && acc[r] > th) {
              const int at = atomicAdd(&ccnt[ul], 1);
              cand[ul * TILE + at] = acc[r];
              crow[ul * TILE + at] = (uint8_t)row;
            }
          }
        }
      }
      __syncthreads();  // candidates complete; pbuf free (unless ALIAS: it holds them)
      if (!ALIAS && I + 1 < I1) {
        store_tile();
        if (I + 2 < I1) load_item_tile(ix, I + 2, t, pf);
      }
      {
        const bool was_act = (all_users || open[uo]) && I * TILE >= Cov[uo];
        const int c = ccnt[uo];
        float* tk = topk + uo * K;
        int32_t* ti = topi + uo * K;
        for (int i = 0; i < c; ++i) {
          const float v = cand[uo * TILE + i];
          if (v > gmn) {
            if (!all_users && v - eut > hmin) {
#pragma unroll
              for (int p = 0; p < kUserPairs; ++p)
                cnt[p] += (int)(v - eut > ph[p]) - (int)(gmn - eut > ph[p]);
            }
            if ((gpos & 3) == sub) {  // the lane holding the minimum replaces it
              tk[gpos] = v;
              ti[gpos] = I * TILE + crow[uo * TILE + i];
              lmn = INFINITY;
              for (int e = 0; e < K4; ++e) {
                const float x = tk[4 * e + sub];
                if (x < lmn) lmn = x, lmp = 4 * e + sub;
              }
            }
            float a = lmn;
            int pa = lmp;
            quad_min(a, pa);
            gmn = a;
            gpos = pa;
          }
        }
        if (was_act && !all_users && rem && (c > 0 || pos >= nlim)) {
          settle((int)pos, npos);
          update_nlim();
        }
        if (sub == 0) {
          if (c > 0) {
            thr[uo] = gmn;
            ccnt[uo] = 0;
          }
          if (was_act) {
            Cov[uo] = (int)pos;  // the list covers the items [0, (I+1)*64)
            if (!all_users && !rem) open[uo] = 0;  // every pair settled: the user stops
            if (bv.ctr) c_scan += (unsigned long long)min((int64_t)TILE, ix.m - (int64_t)I * TILE);
          }
        }
        if (!all_users) {
          const unsigned long long still = __ballot(rem != 0u);
          if (lane == 0) more_w[wave] = still != 0ull;
        }
      }
      if (ALIAS) {
        __syncthreads();  // candidates consumed: the region takes the next tile
        if (I + 1 < I1) {
          store_tile();
          if (I + 2 < I1) load_item_tile(ix, I + 2, t, pf);
        }
      }
    }
    __syncthreads();
    // Sort every list in descending order (value, then item id); S lanes per
    // list (S a power of two >= K), 64 / S lists per wave at once.
    if (K <= TILE) {
      const int S = K <= 4 ? 4 : K <= 8 ? 8 : K <= 16 ? 16 : K <= 32 ? 32 : 64;
      const int per = TILE / S, g = lane / S, j = lane % S;
      for (int u0 = wave * per; u0 < TILE; u0 += 4 * per) {
        const int uu = u0 + g;
        float v = j < K ? topk[uu * K + j] : -INFINITY;
        int32_t id = j < K ? topi[uu * K + j] : INT32_MAX;
        for (int size = 2; size <= S; size <<= 1) {
          for (int stride = size >> 1; stride > 0; stride >>= 1) {
            const float ov = __shfl_xor(v, stride);
            const int32_t oid = __shfl_xor(id, stride);
            const bool keep_max = ((j & stride) == 0) == ((j & size) == 0);
            const bool other_greater = ov > v || (ov == v && oid < id);
            const bool other_less = ov < v || (ov == v && oid > id);
            if (keep_max ? other_greater : other_less) {
              v = ov;
              id = oid;
            }
          }
        }
        if (j < K) {
          topk[uu * K + j] = v;
          topi[uu * K + j] = id == INT32_MAX ? -1 : id;
        }
      }
    } else if (t < TILE) {
      float* tk = topk + t * K;
      int32_t* ti = topi + t * K;
      for (int i = 1; i < K; ++i) {
        const float v = tk[i];
        const int32_t id = ti[i];
        int p = i;
        while (p > 0 && (tk[p - 1] < v || (tk[p - 1] == v && ti[p - 1] > id))) {
          tk[p] = tk[p - 1];
          ti[p] = ti[p - 1];
          --p;
        }
        tk[p] = v;
        ti[p] = id;
      }
    }
    __syncthreads();
    list_reset();
  };

  __syncthreads();
  list_reset();
  if (sub == 0) thr[uo] = gmn;  // read after the next barrier
  const float e0 = ix.eps_rel32 * ix.normP[0];  // times |u|, plus eps_abs: any product's bound
  if (!GROUP) scan_tiles(0, nshort, true);
  // pair slots (after the short pass: in ALIAS mode they share the tile region)
  for (int i = t; i < TILE * kUserPairs; i += 256) {
    pk_s[i] = 0;
    plo_s[i] = INT_MAX;
    phi_s[i] = INT_MIN;
  }
  __syncthreads();

  // f(q,u) in [lo, hi]: float32 bounds (recomputed from the float32 rows in
  // bf16 mode, where the filter's product is a bf16 one).
  auto pair_bounds = [&](int64_t slot, int ul, int32_t jj, float nu, float& lo, float& hi) {
    float s = bv.pair_s[slot];
    if (ix.bf16) s = dot32_col(bv.qs + (int64_t)bv.perm[jj] * d, ubuf + ul, d);
    const float es = ix.eps_rel32 * (nu * bv.qn_s[jj]) + ix.eps_abs;
    lo = s - es;
    hi = s + es;
  };

  // Pass 1: every pair of the block, PG chunks at a time.  The chunk ids and
  // fills are staged in LDS (the candidate region, free until the long
  // pass), as are the users' norms; the next group's pairs are loaded while
  // the current group's query data are gathered and its pairs classified.
  // Classes: 0 no, 1 yes, 2 long (flagged), 3 resolve.
  constexpr int PG = 4;
  int32_t* cid_s = (int32_t*)cand;     // [maxc] chunk ids of the block
  int32_t* cfl_s = cid_s + bv.maxc;    // [maxc] their fills
  if (!GROUP) {
    for (int i = t; i < nch; i += 256) {
      const int32_t c = clist[i];
      cid_s[i] = c;
      cfl_s[i] = bv.cfill[c];
    }
    if (t < TILE) nu_s[t] = ix.normQ[B * TILE + t];
    __syncthreads();
  }
  int64_t slot[PG];
  bool ok[PG];
  int32_t uv[PG], jv[PG];
  float sv[PG];
  auto load_group = [&](int cg) {
#pragma unroll
    for (int g = 0; g < PG; ++g) {
      ok[g] = cg + g < nch && t < cfl_s[cg + g];
      slot[g] = ok[g] ? (int64_t)cid_s[cg + g] * kPairChunk + t : 0;
    }
#pragma unroll
    for (int g = 0; g < PG; ++g) {
      uv[g] = ok[g] ? bv.pair_u[slot[g]] : (int32_t)(B * TILE);
      jv[g] = ok[g] ? bv.pair_j[slot[g]] : 0;
      sv[g] = ok[g] ? bv.pair_s[slot[g]] : 0.f;
    }
  };
  if (!GROUP && nch > 0) load_group(0);
  for (int cg = 0; cg < (GROUP ? 0 : nch); cg += PG) {
    // this group's query data first, then the next group's pairs, so that
    // waiting for the first leaves the second in flight
    int kv[PG];
    float nqv[PG];
#pragma unroll
    for (int g = 0; g < PG; ++g) {
      kv[g] = ok[g] ? bv.k_s[jv[g]] : 1;
      nqv[g] = ok[g] ? bv.qn_s[jv[g]] : 0.f;
    }
    int64_t slot_c[PG];
    bool ok_c[PG];
    int32_t uv_c[PG], jv_c[PG];
    float sv_c[PG];
#pragma unroll
    for (int g = 0; g < PG; ++g) {
      slot_c[g] = slot[g];
      ok_c[g] = ok[g];
      uv_c[g] = uv[g];
      jv_c[g] = jv[g];
      sv_c[g] = sv[g];
    }
    __builtin_amdgcn_sched_barrier(0);
    if (cg + PG < nch) load_group(cg + PG);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int g = 0; g < PG; ++g) {
      if (!ok_c[g]) continue;
      const int64_t u = uv_c[g];
      const int ul = (int)(u - B * TILE);
      const int32_t jj = jv_c[g];
      const int k = kv[g];
      const float nu = nu_s[ul];
      const float e = e0 * nu + ix.eps_abs;
      const float kth = topk[ul * K + k - 1];
      int cls;
      float lo = 0.f, hi = 0.f;
      const float eb = ix.eps_rel * (nu * nqv[g]) + ix.eps_abs;  // bulk-precision bound
      if (kth - e > sv_c[g] + eb) {
        cls = 0;
      } else {
        // f(q,u) in [lo, hi]: float32 bounds (recomputed from the float32
        // rows in bf16 mode, where the filter's product is a bf16 one)
        float sf = sv_c[g];
        if (ix.bf16) sf = dot32_col(bv.qs + (int64_t)bv.perm[jj] * d, ubuf + ul, d);
        const float es = ix.eps_rel32 * (nu * nqv[g]) + ix.eps_abs;
        lo = sf - es;
        hi = sf + es;
        const float csu = ix.cs_inflate * nu;
        if (kth - e > hi) {
          cls = 0;
        } else if (lo >= csu * ix.normP[k - 1]) {
          cls = 1;  // Lemma 2
          ++c_l2;
        } else if (Cov[ul] >= ix.m || csu * ix.normP[Cov[ul]] <= lo) {
          cls = (kth + e <= lo) ? 1 : 3;
        } else {
          cls = 2;
          const int at = ul * kUserPairs + min(atomicAdd(&npu[ul], 1), kUserPairs - 1);
          atomicMax(&pk_s[at], k);
          atomicMin(&plo_s[at], fkey(__float_as_int(lo)));
          atomicMax(&phi_s[at], fkey(__float_as_int(hi)));
        }
      }
      bv.pair_st[slot_c[g]] = cls == 2;
      if (cls == 2) {
        const int at = atomicAdd(&nflag, 1);
        if (at < flist_cap) flist[at] = (int32_t)slot_c[g];
        ++c_long;
      }
      bool yes = cls == 1;
      if (cls == 3) {
        yes = resolve_pair(ix, bv, u, jj, k, lo, hi, nu, topk + ul * K, topi + ul * K, K, false,
                           c_full);
        ++c_f64;
      }
      if (yes) set_pair_result(bv, ix, u, bv.perm[jj]);
    }
  }
  __syncthreads();

  // Long pass: flagged pairs, their users' scan continued until each of
  // their pairs has settled.
  auto decide_flagged = [&](int64_t slot) {
    const int64_t u = bv.pair_u[slot];
    const int ul = (int)(u - B * TILE);
    if (open[ul] == 2) {  // handed over: k_bdecide decides it
      bv.pair_st[slot] = 2;
      return;
    }
    const int32_t jj = bv.pair_j[slot];
    const int k = bv.k_s[jj];
    const float nu = ix.normQ[u];
    const float e = eu[ul];
    const float kth = topk[ul * K + k - 1];
    float lo, hi;
    pair_bounds(slot, ul, jj, nu, lo, hi);
    const float csu = ix.cs_inflate * nu;
    // the scan stopped before this pair's limit: not expected, as a user
    // stops only when each of its pairs is decided no or covered to its
    // limit; float64 then decides
    const bool short_prefix = Cov[ul] < ix.m && csu * ix.normP[Cov[ul]] > lo;
    bool yes;
    if (kth - e > hi) {
      yes = false;
    } else if (!short_prefix && kth + e <= lo) {
      yes = true;
    } else {
      yes = resolve_pair(ix, bv, u, jj, k, lo, hi, nu, topk + ul * K, topi + ul * K, K,
                         short_prefix, c_full);
      ++c_f64;
    }
    if (yes) set_pair_result(bv, ix, u, bv.perm[jj]);
  };
  const int nfl = GROUP ? 1 : nflag;
  if (nfl > 0) {
    {
      const bool real = !GROUP || uo < nusers;
      const float nuo = real ? ix.normQ[urow(uo)] : 0.f;
      eut = e0 * nuo + ix.eps_abs;
      csut = ix.cs_inflate * nuo;
      if (!GROUP && t < TILE) eu[t] = e0 * ix.normQ[B * TILE + t] + ix.eps_abs;
      const int np = !real ? 0 : GROUP ? bv.st_np[urow(uo)] : npu[uo];
      const int64_t so = real ? urow(uo) * kUserPairs : 0;
#pragma unroll
      for (int p = 0; p < kUserPairs; ++p) {
        const bool have = p < np;
        if (GROUP) {
          pk[p] = have ? bv.st_pk[so + p] : INT_MAX;
          plo[p] = have ? bv.st_plo[so + p] : INFINITY;
          ph[p] = have ? bv.st_ph[so + p] : INFINITY;
        } else {
          pk[p] = have ? pk_s[uo * kUserPairs + p] : INT_MAX;
          plo[p] = have ? __int_as_float(fkey(plo_s[uo * kUserPairs + p])) : INFINITY;
          ph[p] = have ? __int_as_float(fkey(phi_s[uo * kUserPairs + p])) : INFINITY;
        }
        rem |= (unsigned)have << p;
        cnt[p] = 0;
      }
      if (rem) {
        for (int i = 0; i < K4; ++i) {
          const float a = topk[uo * K + 4 * i + sub] - eut;
#pragma unroll
          for (int p = 0; p < kUserPairs; ++p) cnt[p] += a > ph[p];
        }
#pragma unroll
        for (int p = 0; p < kUserPairs; ++p) cnt[p] = quad_sum(cnt[p]);
        // users whose lists already settle every flagged pair stop here
        const int cv = Cov[uo];
        settle(cv, cv < ix.m ? ix.normP[cv] : 0.f);
        update_nlim();
      }
      if (sub == 0) open[uo] = rem != 0u;
      const unsigned long long still = __ballot(rem != 0u);
      if (lane == 0) more_w[wave] = still != 0ull;
    }
    __syncthreads();
    // tiles from the smallest coverage of a user with an open pair
    int tmin = INT_MAX, nopen = 0;
    for (int i = 0; i < TILE; ++i)
      if (open[i]) tmin = min(tmin, Cov[i]), ++nopen;
    nopen0 = nopen;
    if (!GROUP && nopen <= kHandoff && ix.mB - tmin / TILE > ix.handoff_tiles) handoff = nopen > 0;
    else if (tmin < INT_MAX) scan_tiles(tmin / TILE, (int)ix.mB, false);
    if (handoff) {
      // users still scanning: a place in the next group pass, and from a
      // block their pair slots (their sorted lists and coverage are stored
      // below)
      if (sub == 0 && open[uo]) {
        const int64_t u = urow(uo);
        hlist[atomicAdd(hcount, 1)] = (int32_t)u;
        if (bv.ctr) atomicAdd(&bv.ctr[C_HANDOFF], 1ull);
        // depth key: the tile of the first item past the Corollary 1 limit
        // of the user's deepest open pair (smallest lower bound), so that a
        // group pass takes users of similar depth together
        float lmin = INFINITY;
        for (int p = 0; p < kUserPairs; ++p)
          if ((rem >> p) & 1u) lmin = fminf(lmin, plo[p]);
        int a = Cov[uo], b2 = (int)ix.m;
        while (a < b2) {
          const int mid = (a + b2) >> 1;
          if (csut * ix.normP[mid] <= lmin) b2 = mid;
          else a = mid + 1;
        }
        bv.sg_key[u] = a / TILE;
        if (!GROUP) {
          const int np = min(npu[uo], kUserPairs);
          bv.st_np[u] = np;
          for (int p = 0; p < kUserPairs; ++p) {
            if (p < np) {
              bv.st_pk[u * kUserPairs + p] = pk[p];
              bv.st_plo[u * kUserPairs + p] = plo[p];
              bv.st_ph[u * kUserPairs + p] = ph[p];
            }
          }
          open[uo] = 2;
        }
      }
      if (!GROUP && t == 0) bv.sg_block[B] = 1;
    }
    __syncthreads();
    if (GROUP) {
      // the lists (sorted), their coverage
      for (int i = t; i < TILE * K; i += 256) {
        const int c = i / K;
        if (c < nusers) {
          bv.gl_v[urow(c) * K + (i - c * K)] = topk[i];
          bv.gl_i[urow(c) * K + (i - c * K)] = topi[i];
        }
      }
      if (t < nusers) bv.gdone[urow(t)] = Cov[t];
    } else if (nfl <= flist_cap) {
      for (int i = t; i < nfl; i += 256) decide_flagged(flist[i]);
    } else {  // more than the list holds: find them by their flags
      for (int ci = 0; ci < nch; ++ci) {
        const int32_t c = clist[ci];
        if (t >= bv.cfill[c]) continue;
        const int64_t slot = (int64_t)c * kPairChunk + t;
        if (bv.pair_st[slot]) decide_flagged(slot);
      }
    }
  }

  // the lists (sorted) and what they cover, for the call's next chunks and
  // the users handed over
  if (!GROUP && (bv.carry_out || handoff)) {
    __syncthreads();
    const int64_t g0 = B * TILE * (int64_t)K;
    for (int i = t; i < TILE * K; i += 256) {
      if (bv.carry_out || open[i / K] == 2) {
        bv.gl_v[g0 + i] = topk[i];
        bv.gl_i[g0 + i] = topi[i];
      }
    }
    if (t < TILE && (bv.carry_out || open[t] == 2)) bv.gdone[B * TILE + t] = Cov[t];
  }

  if (bv.ctr) {
    for (int off = 32; off > 0; off >>= 1) {
      c_l2 += __shfl_xor(c_l2, off);
      c_f64 += __shfl_xor(c_f64, off);
      c_scan += __shfl_xor(c_scan, off);
      c_long += __shfl_xor(c_long, off);
      c_full += __shfl_xor(c_full, off);
      c_quart += __shfl_xor(c_quart, off);
      c_valu += __shfl_xor(c_valu, off);
    }
    if (lane == 0) {
      if (c_quart) atomicAdd(&bv.ctr[C_SQUART], c_quart);
      if (c_valu) atomicAdd(&bv.ctr[C_SVALU], c_valu);
      if (c_long) atomicAdd(&bv.ctr[C_LONG], c_long);
      if (c_full) atomicAdd(&bv.ctr[C_F64SCAN], c_full);
      if (c_l2) atomicAdd(&bv.ctr[C_L2YES], c_l2);
      if (c_f64) atomicAdd(&bv.ctr[C_RCHK], c_f64);
      if (c_scan) atomicAdd(&bv.ctr[C_SCAN], c_scan);
    }
  }
}

// The list of handed-over users ordered by their depth key (64 buckets over
// the item tiles; order within a bucket arbitrary): one workgroup, counting
// sort.
__global__ void __launch_bounds__(1024) k_bsgsort(const int32_t* __restrict__ in,
                                                  const int32_t* __restrict__ count,
                                                  const int32_t* __restrict__ key,
                                                  int32_t* __restrict__ out, int32_t mB) {
  __shared__ int hist[64];
  const int t = threadIdx.x;
  const int n = *count;
  if (t < 64) hist[t] = 0;
  __syncthreads();
  const int64_t span = (int64_t)mB + 1;
  auto bucket = [&](int32_t u) { return (int)min((int64_t)63, (int64_t)key[u] * 64 / span); };
  for (int i = t; i < n; i += 1024) atomicAdd(&hist[bucket(in[i])], 1);
  __syncthreads();
  if (t == 0) {
    int acc = 0;
    for (int b = 0; b < 64; ++b) {
      const int c = hist[b];
      hist[b] = acc;
      acc += c;
    }
  }
  __syncthreads();
  for (int i = t; i < n; i += 1024) {
    const int32_t u = in[i];
    out[atomicAdd(&hist[bucket(u)], 1)] = u;
  }
}

// The flagged pairs of the users a block handed over, decided from their
// final lists (global), as in the block's own long pass.
__global__ void __launch_bounds__(256) k_bdecide(DevIndex ix, BatchView bv) {
  const int64_t B = blockIdx.x;
  if (!bv.sg_block[B]) return;
  const int t = threadIdx.x, lane = t & 63;
  const int nch = min(bv.bcnt[B], bv.maxc);
  const int K = bscan_list_len(ix.kmax);
  const float e0 = ix.eps_rel32 * ix.normP[0];
  const int32_t* clist = bv.bchunks + B * bv.maxc;
  unsigned long long c_f64 = 0, c_full = 0;
  for (int ci = 0; ci < nch; ++ci) {
    const int32_t c = clist[ci];
    if (t >= bv.cfill[c]) continue;
    const int64_t slot = (int64_t)c * kPairChunk + t;
    if (bv.pair_st[slot] != 2) continue;
    const int64_t u = bv.pair_u[slot];
    const int32_t jj = bv.pair_j[slot];
    const int k = bv.k_s[jj];
    const float nu = ix.normQ[u];
    const float e = e0 * nu + ix.eps_abs;
    const float* tk = bv.gl_v + u * K;
    const int32_t* ti = bv.gl_i + u * K;
    const float kth = tk[k - 1];
    float s = bv.pair_s[slot];
    if (ix.bf16)  // the user's column of the block tile, as the scan reads it
      s = dot32_col(bv.qs + (int64_t)bv.perm[jj] * ix.d, ix.Qt + B * (int64_t)ix.d * TILE + (u - B * TILE), ix.d);
    const float es = ix.eps_rel32 * (nu * bv.qn_s[jj]) + ix.eps_abs;
    const float lo = s - es, hi = s + es;
    const float csu = ix.cs_inflate * nu;
    const int cov = bv.gdone[u];
    const bool short_prefix = cov < ix.m && csu * ix.normP[cov] > lo;
    bool yes;
    if (kth - e > hi) {
      yes = false;
    } else if (!short_prefix && kth + e <= lo) {
      yes = true;
    } else {
      yes = resolve_pair(ix, bv, u, jj, k, lo, hi, nu, tk, ti, K, short_prefix, c_full);
      ++c_f64;
    }
    if (yes) set_pair_result(bv, ix, u, bv.perm[jj]);
  }
  if (bv.ctr) {
    for (int off = 32; off > 0; off >>= 1) {
      c_f64 += __shfl_xor(c_f64, off);
      c_full += __shfl_xor(c_full, off);
    }
    if (lane == 0) {
      if (c_full) atomicAdd(&bv.ctr[C_F64SCAN], c_full);
      if (c_f64) atomicAdd(&bv.ctr[C_RCHK], c_f64);
    }
  }
}

// ---------------------------------------------------------------------------
void launch_bscan_reset(const DevIndex& ix, const BatchView& bv, hipStream_t s) {
  if (ix.exact || ix.n_pad == 0) return;
  launch_fill_i32(bv.gdone, ix.n_pad, 0, s);
}

static size_t bscan_lds_mode(const DevIndex& ix, bool alias) {
  const size_t d2 = (size_t)(ix.d + (ix.d & 1));
  if (alias)
    return (d2 * TILE + bscan_tile_region((int)d2) + 2 * (size_t)TILE * bscan_list_len(ix.kmax) +
            4 * TILE) * 4;
  return (2 * d2 * TILE + TILE * TILE + 2 * (size_t)TILE * bscan_list_len(ix.kmax) + 4 * TILE) * 4 +
         TILE * TILE;
}

static size_t bscan_static_mode(bool alias) {
  hipFuncAttributes a{};
  const void* f = alias ? (const void*)k_bscan<16, false, true> : (const void*)k_bscan<2, false, false>;
  if (hipFuncGetAttributes(&a, f) != hipSuccess) return 16384;
  return a.sharedSizeBytes;
}

constexpr size_t kBscanMaxLds = 160 * 1024;

// The shared tile region: tiles of 65..128 coordinates (two workgroups per
// CU), and wider ones whose separate buffers would not fit.
static bool bscan_alias(const DevIndex& ix) {
  const int per_thread = (ix.d * (TILE / 4) + 255) / 256;  // the kernel's NV
  if (per_thread <= 4) return false;
  if (per_thread <= 8) return true;
  return bscan_lds_mode(ix, false) + bscan_static_mode(false) > kBscanMaxLds;
}

size_t bscan_lds_bytes(const DevIndex& ix) { return bscan_lds_mode(ix, bscan_alias(ix)); }

bool bscan_fits(const DevIndex& ix) {
  const bool alias = bscan_alias(ix);
  return bscan_lds_mode(ix, alias) + bscan_static_mode(alias) <= kBscanMaxLds;
}

template <int NV, bool ALIAS>
static void bscan_nv(const DevIndex& ix, const BatchView& bv, hipStream_t s) {
  const size_t lds = bscan_lds_mode(ix, ALIAS);
  if (lds > 65536) {
    (void)hipFuncSetAttribute((const void*)k_bscan<NV, false, ALIAS>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    (void)hipFuncSetAttribute((const void*)k_bscan<NV, true, ALIAS>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  }
  hipLaunchKernelGGL((k_bscan<NV, false, ALIAS>), dim3(ix.nB), dim3(256), lds, s, ix, bv);
  // the handed-over users, 64 per workgroup (at most nB groups; the rest
  // exit), in passes over alternating lists
  for (int lev = 0; lev < kGroupLevels; ++lev) {
    BatchView g = bv;
    g.sg_level = lev;
    g.sg_last = lev == kGroupLevels - 1;
    // the list this pass hands over to starts empty (the first is cleared with the chunk)
    if (lev > 0 && !g.sg_last) launch_fill_i32(g.sg_count + ((lev & 1) ^ 1), 1, 0, s);
    hipLaunchKernelGGL(k_bsgsort, dim3(1), dim3(1024), 0, s, g.sg_users + (int64_t)(lev & 1) * ix.n_pad,
                       g.sg_count + (lev & 1), g.sg_key, g.sg_sorted, ix.mB);
    hipLaunchKernelGGL((k_bscan<NV, true, ALIAS>), dim3(ix.nB), dim3(256), lds, s, ix, g);
  }
  hipLaunchKernelGGL(k_bdecide, dim3(ix.nB), dim3(256), 0, s, ix, bv);
}

void launch_bprescan(const DevIndex& ix, const BatchView& bv, hipStream_t s) {
  if (ix.nB == 0) return;
  BatchView p = bv;
  p.prescan = 1;
  p.carry_in = 0;
  p.carry_out = 1;  // store every block's lists
  const size_t lds = bscan_lds_bytes(ix);
  const int per_thread = (ix.d * (TILE / 4) + 255) / 256;
  const bool alias = bscan_alias(ix);
  auto go = [&](const void* f) {
    if (lds > 65536) (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  };
  if (per_thread <= 2) {
    go((const void*)k_bscan<2, false, false>);
    hipLaunchKernelGGL((k_bscan<2, false, false>), dim3(ix.nB), dim3(256), lds, s, ix, p);
  } else if (per_thread <= 4) {
    go((const void*)k_bscan<4, false, false>);
    hipLaunchKernelGGL((k_bscan<4, false, false>), dim3(ix.nB), dim3(256), lds, s, ix, p);
  } else if (per_thread <= 8) {
    go((const void*)k_bscan<8, false, true>);
    hipLaunchKernelGGL((k_bscan<8, false, true>), dim3(ix.nB), dim3(256), lds, s, ix, p);
  } else if (alias) {
    go((const void*)k_bscan<16, false, true>);
    hipLaunchKernelGGL((k_bscan<16, false, true>), dim3(ix.nB), dim3(256), lds, s, ix, p);
  } else {
    go((const void*)k_bscan<16, false, false>);
    hipLaunchKernelGGL((k_bscan<16, false, false>), dim3(ix.nB), dim3(256), lds, s, ix, p);
  }
}

void launch_bscan(const DevIndex& ix, const BatchView& bv, hipStream_t s) {
  const int per_thread = (ix.d * (TILE / 4) + 255) / 256;  // 16-byte vectors of an item tile
  if (per_thread <= 2) bscan_nv<2, false>(ix, bv, s);
  else if (per_thread <= 4) bscan_nv<4, false>(ix, bv, s);
  else if (per_thread <= 8) bscan_nv<8, true>(ix, bv, s);
  else if (bscan_alias(ix)) bscan_nv<16, true>(ix, bv, s);
  else bscan_nv<16, false>(ix, bv, s);
}

}  // namespace rk
