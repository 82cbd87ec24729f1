// Host runtime and C ABI (include/rkmips.h).  Owns every device buffer of an
// index, validates arguments before any device work, sequences the build
// (Algorithm 1) and query (Algorithms 2-3) kernels on the index's stream.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <mutex>
#include <numeric>
#include <string>
#include <thread>
#include <type_traits>
#include <vector>

#include "rk_batch.h"
#include "rk_kernels.h"

using namespace rk;

namespace {

thread_local std::string g_err;

rk_status fail(rk_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

#define HIPTRY(expr)                                                                  \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(e_ == hipErrorOutOfMemory ? RK_E_NOMEM : RK_E_DEVICE,               \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                 \
  } while (0)

constexpr int64_t kSeedItems = 1024;  // exact float64 prefix that seeds the full build

// Device workspace of the batched path for chunks of up to qcap queries
// (grown on demand).  An index owns one for its own calls; every serving slot
// owns another, so that batches over one index can be in flight on several
// streams at once.
struct BatchWS {
  int32_t qcap = 0;       // queries per chunk it is sized for
  int64_t pair_cap = 0;
  float *qn = nullptr, *qt = nullptr, *qn_s = nullptr, *pair_s = nullptr;
  uint16_t* qb = nullptr;
  unsigned long long* npairs = nullptr;
  int32_t *perm = nullptr, *k_s = nullptr, *kofs_s = nullptr, *tsum = nullptr, *pair_u = nullptr,
          *pair_j = nullptr, *ks_dev = nullptr;
  // bounded table: chunked pair slots, per-block chunk lists
  int32_t *pair_st = nullptr, *cfill = nullptr, *nchunks = nullptr, *bcnt = nullptr,
          *bchunks = nullptr, *gl_i = nullptr, *gdone = nullptr;
  float* gl_v = nullptr;
  // users handed to the grouped pass and their pair slots
  int32_t *sg_count = nullptr, *sg_users = nullptr, *sg_block = nullptr, *st_np = nullptr,
          *st_pk = nullptr, *sg_key = nullptr, *sg_sorted = nullptr;
  float *st_plo = nullptr, *st_ph = nullptr;
  int32_t chunk_cap = 0, maxc = 0;
  uint32_t* bits = nullptr;
  unsigned long long* counts = nullptr;
  uint8_t* all = nullptr;
  int32_t* ks_pinned = nullptr;   // host staging of k values
  int64_t ks_pinned_cap = 0;
  hipEvent_t ks_done = nullptr;   // the last copy out of ks_pinned
  std::vector<void*> dev;         // owned device buffers
  int64_t bytes = 0;              // their size

  template <typename T>
  hipError_t alloc(T** p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void**)p, count * sizeof(T));
    if (e == hipSuccess) {
      dev.push_back((void*)*p);
      bytes += (int64_t)(count * sizeof(T));
    }
    return e;
  }
  // Frees the device buffers (the pinned staging and its event stay).
  void release() {
    for (void* q : dev) (void)hipFree(q);
    int32_t* kp = ks_pinned;
    const int64_t kc = ks_pinned_cap;
    hipEvent_t ke = ks_done;
    *this = BatchWS();
    ks_pinned = kp;
    ks_pinned_cap = kc;
    ks_done = ke;
  }
  void destroy() {
    release();
    if (ks_pinned) (void)hipHostFree(ks_pinned);
    if (ks_done) (void)hipEventDestroy(ks_done);
    ks_pinned = nullptr;
    ks_pinned_cap = 0;
    ks_done = nullptr;
  }
};

}  // namespace

struct rk_index {
  int device = 0;
  hipStream_t stream = nullptr;
  rk_build_opts opts{};
  DevIndex ix{};
  double eps32 = 0;  // float32 bound (build candidate pass)
  std::vector<std::pair<void*, size_t>> dbufs;  // owned device buffers and sizes
  std::vector<void*> hbufs;
  size_t footprint = 0;
  // owned device arrays
  float *Qt = nullptr, *Qrow = nullptr, *normQ = nullptr, *Pt = nullptr, *Prow = nullptr, *normP = nullptr;
  uint16_t *Qb = nullptr, *Pb = nullptr;
  int32_t *permQ = nullptr, *permP = nullptr;
  double *s2Q = nullptr, *s2P = nullptr, *L64 = nullptr;
  float *L32 = nullptr, *LB = nullptr, *bnorm = nullptr;
  // query workspace
  QueryWS ws{};
  float* q_dev = nullptr;
  int32_t* ids_dev = nullptr;
  int64_t* count_dev = nullptr;
  unsigned long long* ctr_dev = nullptr;
  bool counting = false;
  // optional per-kernel event timing (kernel class, start, end)
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_used;
  size_t ev_next = 0;
  // pinned host staging (ids/count are mapped: the finalize kernel writes them)
  float* q_host = nullptr;
  int32_t* ids_host = nullptr;
  int64_t* count_host = nullptr;
  int32_t* ids_host_dev = nullptr;
  int64_t* count_host_dev = nullptr;
  // batched-query workspace of the index's own calls (grown on demand)
  BatchWS bw;
  // build statistics
  double build_ms = 0;
  int64_t cand_total = 0, cand_ovf = 0, rebuilds = 0, updates = 0;
  std::atomic<int64_t> queries{0};
  std::atomic<int32_t> served{0};  // servers holding the index as a catalog

  ~rk_index() {
    if (device >= 0) (void)hipSetDevice(device);
    if (stream) (void)hipStreamSynchronize(stream);
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    bw.destroy();
    for (auto& b : dbufs) (void)hipFree(b.first);
    for (void* p : hbufs) (void)hipHostFree(p);
    if (stream) (void)hipStreamDestroy(stream);
  }

  template <typename T>
  hipError_t dalloc(T** p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void**)p, count * sizeof(T));
    if (e == hipSuccess) {
      dbufs.push_back({(void*)*p, count * sizeof(T)});
      footprint += count * sizeof(T);
    }
    return e;
  }
  void dfree(void* p) {
    for (auto it = dbufs.begin(); it != dbufs.end(); ++it)
      if (it->first == p) {
        footprint -= it->second;
        (void)hipFree(p);
        dbufs.erase(it);
        return;
      }
  }
  void hfree(void* p) {
    for (auto it = hbufs.begin(); it != hbufs.end(); ++it)
      if (*it == p) {
        (void)hipHostFree(p);
        hbufs.erase(it);
        return;
      }
  }
};

namespace {

rk_status check_opts(const rk_build_opts& o) {
  const char* e = opts_error(o);
  return e ? fail(RK_E_INVAL, e) : RK_OK;
}

rk_status check_sizes(int64_t n, int64_t m, int32_t d, int32_t k_max) {
  const char* e = sizes_error(n, m, d, k_max);
  return e ? fail(RK_E_INVAL, e) : RK_OK;
}

bool host_values_ok(const float* x, int64_t count) { return values_ok(x, count); }

// Build the lower-bound arrays and blocks for the index's current k_max from
// the sorted device copies (Algorithm 1, lower-bound arrays and blocks).
// Lower-bound arrays L64/L32 ([k_max][x.n_pad]) of the users of x over the
// first x.lb_items sorted items (Algorithm 1): x is the index itself, or a
// view of it whose users are a catalog update's new users.
rk_status compute_bounds(rk_index* h, const DevIndex& ix, double* L64, float* L32) {
  hipStream_t s = h->stream;
  const int64_t lb = ix.lb_items;
  if (ix.n_pad > 0) {
    if (lb <= kSeedItems) {
      launch_lb_exact(ix, lb, L64, L32, nullptr, s);
      HIPTRY(hipGetLastError());
    } else {
      // Long prefix: exact seed over the first kSeedItems items, one MFMA pass
      // over [0, lb) keeping candidates, float64 refine of the candidates.
      DevIndex bx = ix;
      bx.eps_rel = (float)h->eps32;  // the candidate pass runs in float32
      const int32_t cap = h->opts.cand_cap > 0 ? h->opts.cand_cap : std::max(128, 2 * ix.kmax + 64);
      float* t0 = nullptr;
      int32_t *cand = nullptr, *ccount = nullptr, *ovf = nullptr, *novf = nullptr;
      HIPTRY(hipMalloc(&t0, ix.n_pad * sizeof(float)));
      std::vector<void*> tmp{t0};
      auto cleanup = [&]() { for (void* p : tmp) (void)hipFree(p); };
      hipError_t e = hipMalloc(&cand, (size_t)ix.n_pad * cap * sizeof(int32_t));
      if (e == hipSuccess) { tmp.push_back(cand); e = hipMalloc(&ccount, ix.n_pad * sizeof(int32_t)); }
      if (e == hipSuccess) { tmp.push_back(ccount); e = hipMalloc(&ovf, ix.n_pad * sizeof(int32_t)); }
      if (e == hipSuccess) { tmp.push_back(ovf); e = hipMalloc(&novf, sizeof(int32_t)); }
      if (e == hipSuccess) { tmp.push_back(novf); e = hipMemsetAsync(novf, 0, sizeof(int32_t), s); }
      if (e != hipSuccess) { cleanup(); HIPTRY(e); }
      launch_lb_exact(bx, kSeedItems, nullptr, nullptr, t0, s);
      launch_lb_candidates(bx, lb, t0, cap, cand, ccount, s);
      launch_lb_refine(bx, cap, cand, ccount, L64, L32, ovf, novf, s);
      int32_t n_ovf = 0;
      e = hipGetLastError();
      if (e == hipSuccess) e = hipMemcpyAsync(&n_ovf, novf, sizeof(int32_t), hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e == hipSuccess && n_ovf > 0) {
        launch_lb_overflow(bx, lb, ovf, n_ovf, L64, L32, s);
        e = hipGetLastError();
      }
      std::vector<int32_t> cc(ix.n);
      if (e == hipSuccess && ix.n > 0)
        e = hipMemcpyAsync(cc.data(), ccount, ix.n * sizeof(int32_t), hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      cleanup();
      HIPTRY(e);
      for (int32_t c : cc) h->cand_total += std::min(c, cap);
      h->cand_ovf += n_ovf;
    }
  }
  HIPTRY(hipStreamSynchronize(s));
  return RK_OK;
}

// Block minima and first-user norms of the index's current table.
rk_status build_blocks(rk_index* h) {
  DevIndex& ix = h->ix;
  HIPTRY(h->dalloc(&h->LB, (size_t)ix.kmax * ix.nSB));
  HIPTRY(h->dalloc(&h->bnorm, (size_t)ix.nSB));
  ix.LB = h->LB;
  ix.bnorm = h->bnorm;
  if (ix.n_pad > 0) {
    launch_blocks(ix, h->LB, h->bnorm, h->stream);
    HIPTRY(hipGetLastError());
  }
  HIPTRY(hipStreamSynchronize(h->stream));
  return RK_OK;
}

rk_status build_bounds(rk_index* h) {
  DevIndex& ix = h->ix;
  HIPTRY(h->dalloc(&h->L64, (size_t)ix.kmax * ix.n_pad));
  HIPTRY(h->dalloc(&h->L32, (size_t)ix.kmax * ix.n_pad));
  ix.L64 = h->L64;
  ix.L32 = h->L32;
  h->cand_total = 0;
  h->cand_ovf = 0;
  rk_status st = compute_bounds(h, ix, h->L64, h->L32);
  if (st != RK_OK) return st;
  return build_blocks(h);
}

std::vector<int32_t> sort_desc(const std::vector<double>& key) {
  std::vector<int32_t> perm(key.size());
  std::iota(perm.begin(), perm.end(), 0);
  std::sort(perm.begin(), perm.end(), [&](int32_t a, int32_t b) {
    if (key[a] != key[b]) return key[a] > key[b];
    return a < b;
  });
  return perm;
}

// One side of the index (users or items) from rows in original order on the
// device: squared norms, the descending norm order (stable by original
// index) and the sorted copies with upward-rounded norms (Algorithm 1's
// first step).  Sets the side's sizes and pointers; perm_out receives the
// order (sorted position -> original index).
rk_status build_side(rk_index* h, const float* Xd, int64_t rows, bool users,
                     std::vector<int32_t>* perm_out) {
  DevIndex& ix = h->ix;
  hipStream_t s = h->stream;
  const int32_t d = ix.d;
  const int64_t pad = round_up(rows, TILE);
  double*& s2 = users ? h->s2Q : h->s2P;
  int32_t*& perm = users ? h->permQ : h->permP;
  float*& Xt = users ? h->Qt : h->Pt;
  float*& norm = users ? h->normQ : h->normP;
  float*& Xrow = users ? h->Qrow : h->Prow;
  uint16_t*& Xb = users ? h->Qb : h->Pb;
  HIPTRY(h->dalloc(&s2, (size_t)rows));
  launch_sqnorms(Xd, rows, d, s2, s);
  HIPTRY(hipGetLastError());
  std::vector<double> key(rows);
  if (rows) HIPTRY(hipMemcpyAsync(key.data(), s2, rows * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPTRY(hipStreamSynchronize(s));
  std::vector<int32_t> pr = sort_desc(key);
  HIPTRY(h->dalloc(&perm, (size_t)rows));
  if (rows) HIPTRY(hipMemcpyAsync(perm, pr.data(), rows * sizeof(int32_t), hipMemcpyHostToDevice, s));
  HIPTRY(h->dalloc(&Xt, (size_t)pad * d));
  HIPTRY(h->dalloc(&norm, (size_t)pad));
  HIPTRY(h->dalloc(&Xrow, (size_t)rows * d));
  if (ix.bf16) HIPTRY(h->dalloc(&Xb, (size_t)pad * ix.d16));
  launch_tile_rows(Xd, perm, s2, rows, pad, d, ix.d16, Xt, norm, ix.bf16 ? Xb : nullptr, Xrow, s);
  HIPTRY(hipGetLastError());
  HIPTRY(hipStreamSynchronize(s));
  if (users) {
    ix.n = rows;
    ix.n_pad = pad;
    ix.nB = (int32_t)(pad / TILE);
    ix.nSB = (int32_t)(pad / ix.bsize);
    ix.Qt = h->Qt; ix.Qrow = h->Qrow; ix.Qb = h->Qb; ix.normQ = h->normQ; ix.permQ = h->permQ;
  } else {
    ix.m = rows;
    ix.m_pad = pad;
    ix.mB = (int32_t)(pad / TILE);
    ix.Pt = h->Pt; ix.Pb = h->Pb; ix.Prow = h->Prow; ix.normP = h->normP;
  }
  if (perm_out) *perm_out = std::move(pr);
  return RK_OK;
}

void free_side(rk_index* h, bool users) {
  if (users) {
    for (void* p : {(void*)h->s2Q, (void*)h->permQ, (void*)h->Qt, (void*)h->normQ, (void*)h->Qrow, (void*)h->Qb})
      if (p) h->dfree(p);
    h->s2Q = nullptr; h->permQ = nullptr; h->Qt = nullptr; h->normQ = nullptr; h->Qrow = nullptr; h->Qb = nullptr;
  } else {
    for (void* p : {(void*)h->s2P, (void*)h->permP, (void*)h->Pt, (void*)h->normP, (void*)h->Prow, (void*)h->Pb})
      if (p) h->dfree(p);
    h->s2P = nullptr; h->permP = nullptr; h->Pt = nullptr; h->normP = nullptr; h->Prow = nullptr; h->Pb = nullptr;
  }
}

// The one-query workspace and staging sized by the number of users.
rk_status alloc_user_ws(rk_index* h) {
  const int64_t n = h->ix.n, W = (n + 31) / 32;
  hipStream_t s = h->stream;
  HIPTRY(h->dalloc(&h->ws.rbits, (size_t)std::max<int64_t>(W, 1)));
  HIPTRY(h->dalloc(&h->ws.surv_idx, (size_t)h->ix.n_pad));
  HIPTRY(h->dalloc(&h->ws.surv_s, (size_t)h->ix.n_pad));
  HIPTRY(h->dalloc(&h->ws.rchk_idx, (size_t)h->ix.n_pad));
  HIPTRY(h->dalloc(&h->ids_dev, (size_t)std::max<int64_t>(n, 1)));
  HIPTRY(hipMemsetAsync(h->ws.rbits, 0, std::max<int64_t>(W, 1) * sizeof(uint32_t), s));
  HIPTRY(hipHostMalloc((void**)&h->ids_host, std::max<int64_t>(n, 1) * sizeof(int32_t), hipHostMallocMapped));
  h->hbufs.push_back(h->ids_host);
  HIPTRY(hipHostGetDevicePointer((void**)&h->ids_host_dev, h->ids_host, 0));
  HIPTRY(hipStreamSynchronize(s));
  return RK_OK;
}

void free_user_ws(rk_index* h) {
  for (void* p : {(void*)h->ws.rbits, (void*)h->ws.surv_idx, (void*)h->ws.surv_s, (void*)h->ws.rchk_idx,
                  (void*)h->ids_dev})
    if (p) h->dfree(p);
  if (h->ids_host) h->hfree(h->ids_host);
  h->ws.rbits = nullptr; h->ws.surv_idx = nullptr; h->ws.surv_s = nullptr; h->ws.rchk_idx = nullptr;
  h->ids_dev = nullptr; h->ids_host = nullptr; h->ids_host_dev = nullptr;
}

// Rows of one side in original order, on the host (from the sorted copy and
// its order).
rk_status side_rows_host(rk_index* h, bool users, std::vector<float>& out) {
  const int64_t rows = users ? h->ix.n : h->ix.m;
  const int32_t d = h->ix.d;
  std::vector<float> sorted((size_t)rows * d);
  std::vector<int32_t> perm(rows);
  hipStream_t s = h->stream;
  if (rows) {
    HIPTRY(hipMemcpyAsync(sorted.data(), users ? h->Qrow : h->Prow, (size_t)rows * d * sizeof(float),
                          hipMemcpyDeviceToHost, s));
    HIPTRY(hipMemcpyAsync(perm.data(), users ? h->permQ : h->permP, rows * sizeof(int32_t),
                          hipMemcpyDeviceToHost, s));
  }
  HIPTRY(hipStreamSynchronize(s));
  out.resize((size_t)rows * d);
  for (int64_t i = 0; i < rows; ++i)
    std::memcpy(&out[(size_t)perm[i] * d], &sorted[(size_t)i * d], d * sizeof(float));
  return RK_OK;
}

rk_status build_impl(const float* Q, int64_t n, const float* P, int64_t m, int32_t d,
                     int32_t k_max, const rk_build_opts* opts_in, bool on_device, rk_index** out) {
  if (!out) return fail(RK_E_INVAL, "out is NULL");
  *out = nullptr;
  rk_build_opts o;
  rk_build_opts_default(&o);
  if (opts_in) o = *opts_in;
  rk_status st;
  if ((st = check_sizes(n, m, d, k_max)) != RK_OK) return st;
  if ((st = check_opts(o)) != RK_OK) return st;
  if ((n > 0 && !Q) || (m > 0 && !P)) return fail(RK_E_INVAL, "Q or P is NULL");
  if (!on_device) {
    if (!host_values_ok(Q, n * d) || !host_values_ok(P, m * d))
      return fail(RK_E_INVAL, "input has a non-finite value or |x| >= 2^40");
  }
  int ndev = 0;
  HIPTRY(hipGetDeviceCount(&ndev));
  if (o.device >= ndev) return fail(RK_E_INVAL, "device ordinal out of range");
  auto t_start = std::chrono::steady_clock::now();

  rk_index* h = new rk_index();
  h->device = o.device;
  h->opts = o;
  auto bail = [&](rk_status s) { delete h; return s; };
#define BTRY(expr)                                         \
  do {                                                     \
    hipError_t be_ = (expr);                               \
    if (be_ != hipSuccess) {                               \
      rk_status s_ = fail(be_ == hipErrorOutOfMemory ? RK_E_NOMEM : RK_E_DEVICE, \
                          std::string(#expr) + ": " + hipGetErrorString(be_));   \
      return bail(s_);                                     \
    }                                                      \
  } while (0)
  BTRY(hipSetDevice(o.device));
  BTRY(hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking));
  hipStream_t s = h->stream;

  DevIndex& ix = h->ix;
  ix.n = n;
  ix.m = m;
  ix.n_pad = round_up(n, TILE);
  ix.m_pad = round_up(m, TILE);
  ix.d = d;
  ix.d16 = (int32_t)round_up(d, 16);
  ix.kmax = k_max;
  ix.nB = (int32_t)(ix.n_pad / TILE);
  ix.mB = (int32_t)(ix.m_pad / TILE);
  ix.bsize = o.block_size ? o.block_size : TILE;
  ix.nSB = (int32_t)(ix.n_pad / ix.bsize);
  ix.use_blocks = o.no_blocks ? 0 : 1;
  const int64_t lb = (o.lb_items == 0 || o.lb_items >= m) ? m : o.lb_items;
  ix.lb_items = (int32_t)lb;
  ix.exact = (lb == m) ? 1 : 0;
  ix.bf16 = o.precision == RK_BF16 ? 1 : 0;
  h->eps32 = std::max(eps_fp32(d), o.margin_rel);
  const double eps = std::max(ix.bf16 ? eps_bf16(d) : eps_fp32(d), o.margin_rel);
  ix.eps_rel = f32_up(eps);
  ix.eps_rel32 = f32_up(h->eps32);
  ix.handoff_tiles = h->opts.handoff_tiles > 0 ? h->opts.handoff_tiles : 512;
  ix.verify_tiles = h->opts.verify_tiles < 0 || d > kVerifyTilesMaxD ? INT32_MAX
                    : h->opts.verify_tiles > 0 ? h->opts.verify_tiles : 2048;
  ix.eps_abs = std::ldexp((double)(d + 2), -124);
  ix.cs_inflate = f32_up(1.0 + gamma_(d, 0x1p-53) + 8 * 0x1p-24);

  // Raw inputs on the device (temporary when given host pointers).
  const float *Qd = Q, *Pd = P;
  float *Qtmp = nullptr, *Ptmp = nullptr;
  int32_t* flag = nullptr;
  std::vector<void*> tmp;
  auto free_tmp = [&]() { for (void* p : tmp) (void)hipFree(p); tmp.clear(); };
#define TTRY(expr)                                         \
  do {                                                     \
    hipError_t e_ = (expr);                                \
    if (e_ != hipSuccess) { free_tmp();  BTRY(e_); }       \
  } while (0)
  if (!on_device) {
    if (n > 0) { TTRY(hipMalloc(&Qtmp, n * d * sizeof(float))); tmp.push_back(Qtmp); }
    if (m > 0) { TTRY(hipMalloc(&Ptmp, m * d * sizeof(float))); tmp.push_back(Ptmp); }
    if (n > 0) TTRY(hipMemcpyAsync(Qtmp, Q, n * d * sizeof(float), hipMemcpyHostToDevice, s));
    if (m > 0) TTRY(hipMemcpyAsync(Ptmp, P, m * d * sizeof(float), hipMemcpyHostToDevice, s));
    Qd = Qtmp;
    Pd = Ptmp;
  } else {
    TTRY(hipMalloc(&flag, sizeof(int32_t)));
    tmp.push_back(flag);
    TTRY(hipMemsetAsync(flag, 0, sizeof(int32_t), s));
    launch_check_inputs(Qd, n * d, flag, s);
    launch_check_inputs(Pd, m * d, flag, s);
    int32_t bad = 0;
    TTRY(hipMemcpyAsync(&bad, flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    TTRY(hipStreamSynchronize(s));
    if (bad) { free_tmp(); return bail(fail(RK_E_INVAL, "input has a non-finite value or |x| >= 2^40")); }
  }

  // Step 1: squared norms, descending norm sort (stable by original index),
  // sorted tiled copies and upward-rounded norms.
  if ((st = build_side(h, Qd, n, true, nullptr)) != RK_OK || (st = build_side(h, Pd, m, false, nullptr)) != RK_OK) {
    free_tmp();
    return bail(st);
  }
  free_tmp();

  // Steps 2-3: lower-bound arrays and blocks.
  if ((st = build_bounds(h)) != RK_OK) return bail(st);

  // Query workspace.
  if ((st = alloc_user_ws(h)) != RK_OK) return bail(st);
  BTRY(h->dalloc(&h->ws.cnt, 4));
  BTRY(h->dalloc(&h->ws.qnorm, 1));
  BTRY(h->dalloc(&h->ctr_dev, 16));
  BTRY(h->dalloc(&h->q_dev, (size_t)d));
  BTRY(h->dalloc(&h->count_dev, 1));
  BTRY(hipMemsetAsync(h->ws.cnt, 0, 4 * sizeof(int32_t), s));
  BTRY(hipMemsetAsync(h->ctr_dev, 0, 16 * sizeof(unsigned long long), s));
  h->ws.ctr = nullptr;
  BTRY(hipHostMalloc((void**)&h->q_host, d * sizeof(float), hipHostMallocDefault));
  h->hbufs.push_back(h->q_host);
  BTRY(hipHostMalloc((void**)&h->count_host, sizeof(int64_t), hipHostMallocMapped));
  h->hbufs.push_back(h->count_host);
  BTRY(hipHostGetDevicePointer((void**)&h->count_host_dev, h->count_host, 0));
  BTRY(hipStreamSynchronize(s));
  h->build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
  *out = h;
  return RK_OK;
#undef TTRY
#undef BTRY
}

// Enqueue one query (device q) on stream s; ids/count are device-visible.
// Kernel classes of the per-kernel event timing.
enum KClass {
  K_FILTER = 0, K_VERIFY, K_RECHECK, K_FINALIZE, K_FILL,
  K_BPREP, K_BFILTER, K_BPAIRS, K_BASSEMBLE, K_NCLASS
};

// Records an event before a launch when timing is on; returns the pool slot.
struct Timer {
  rk_index* h;
  hipStream_t s;
  int cls;
  hipEvent_t e0 = nullptr;
  Timer(rk_index* h_, hipStream_t s_, int c, bool on = true) : h(h_), s(s_), cls(c) {
    if (!on || !h->timing || h->ev_next + 2 > h->ev_pool.size()) return;
    e0 = h->ev_pool[h->ev_next++];
    (void)hipEventRecord(e0, s);
  }
  ~Timer() {
    if (!e0) return;
    hipEvent_t e1 = h->ev_pool[h->ev_next++];
    (void)hipEventRecord(e1, s);
    h->ev_used.push_back({cls, {e0, e1}});
  }
};

// Ids go to ids[*base ...] when base is given (batch CSR), else ids[0 ...];
// *out receives base + count.
rk_status enqueue_query(rk_index* h, const float* q_dev, int32_t k, int32_t* ids, int64_t cap,
                        const int64_t* base, int64_t* out, hipStream_t s, uint8_t* tcls,
                        float* ts) {
  const DevIndex& ix = h->ix;
  if (k > ix.m || ix.n == 0) {
    Timer t(h, s, K_FILL);
    launch_fill_all(k > ix.m ? ix.n : 0, ids, cap, base, out, s);
    HIPTRY(hipGetLastError());
    h->queries++;
    return RK_OK;
  }
  QueryWS ws = h->ws;
  ws.ctr = h->counting ? h->ctr_dev : nullptr;
  ws.trace_cls = tcls;
  ws.trace_s = ts;
  { Timer t(h, s, K_FILTER); launch_filter(ix, q_dev, k, ws, s); }
  if (!ix.exact) { Timer t(h, s, K_VERIFY); launch_verify(ix, q_dev, k, ws, s); }
  { Timer t(h, s, K_RECHECK); launch_recheck(ix, q_dev, k, ws, s); }
  { Timer t(h, s, K_FINALIZE); launch_finalize(ix, ws, ids, cap, base, out, s); }
  HIPTRY(hipGetLastError());
  h->queries++;
  return RK_OK;
}

rk_status check_k(rk_index* h, int32_t k) {
  if (k < 1) return fail(RK_E_INVAL, "k must be >= 1");
  if (k > h->ix.kmax && k <= h->ix.m) {
    if (!h->opts.auto_rebuild) return fail(RK_E_KMAX, "k > k_max (build with a larger k_max or set auto_rebuild)");
    rk_status st = rk_index_rebuild(h, k);
    if (st != RK_OK) return st;
  }
  return RK_OK;
}

rk_status check_batch_ks(rk_index* h, const int32_t* ks, int64_t nq) {
  int32_t need = 0;
  for (int64_t i = 0; i < nq; ++i) {
    if (ks[i] < 1) return fail(RK_E_INVAL, "k must be >= 1");
    if (ks[i] > h->ix.kmax && ks[i] <= h->ix.m) need = std::max(need, ks[i]);
  }
  if (need) {
    if (!h->opts.auto_rebuild) return fail(RK_E_KMAX, "k > k_max (build with a larger k_max or set auto_rebuild)");
    return rk_index_rebuild(h, need);
  }
  return RK_OK;
}

constexpr size_t kMaxLds = 160 * 1024;

BatchShape shape_of(const rk_index* h) {
  BatchShape x;
  x.n = h->ix.n;
  x.n_pad = h->ix.n_pad;
  x.nB = h->ix.nB;
  x.d = h->ix.d;
  x.d16 = h->ix.d16;
  x.kmax = h->ix.kmax;
  x.exact = h->ix.exact != 0;
  x.bf16 = h->ix.bf16 != 0;
  x.pair_cap_opt = h->opts.pair_cap;
  return x;
}

BatchSizes batch_sizes(const rk_index* h, int32_t chunk) { return batch_sizes(shape_of(h), chunk); }

int32_t batch_chunk(const rk_index* h, int64_t nq) { return batch_chunk(shape_of(h), nq); }

rk_status ensure_batch_ws(rk_index* h, BatchWS& b, int32_t chunk, hipStream_t s) {
  if (b.qcap >= chunk) return RK_OK;
  // earlier calls may still use the buffers, on this stream or another
  HIPTRY(hipDeviceSynchronize());
  b.release();
  const DevIndex& ix = h->ix;
  const BatchSizes z = batch_sizes(h, chunk);
  const int64_t cp = round_up(chunk, TILE), W = bitmap_words(ix.n);
  const int64_t pc = z.pc;
  HIPTRY(b.alloc(&b.qn, chunk));
  HIPTRY(b.alloc(&b.perm, chunk));
  HIPTRY(b.alloc(&b.qt, cp * (ix.d + (ix.d & 1))));
  if (ix.bf16) HIPTRY(b.alloc(&b.qb, cp * ix.d16));
  HIPTRY(b.alloc(&b.qn_s, cp));
  HIPTRY(b.alloc(&b.k_s, cp));
  HIPTRY(b.alloc(&b.kofs_s, cp));
  HIPTRY(b.alloc(&b.tsum, cp / TILE * 8));
  HIPTRY(b.alloc(&b.bits, (size_t)chunk * std::max<int64_t>(W, 1)));
  HIPTRY(b.alloc(&b.counts, chunk));
  HIPTRY(b.alloc(&b.all, chunk));
  HIPTRY(b.alloc(&b.npairs, 1));
  HIPTRY(b.alloc(&b.pair_u, pc));
  HIPTRY(b.alloc(&b.pair_j, pc));
  HIPTRY(b.alloc(&b.pair_s, pc));
  HIPTRY(b.alloc(&b.ks_dev, chunk));
  if (!ix.exact) {
    b.chunk_cap = (int32_t)z.chunk_cap;
    b.maxc = (int32_t)z.maxc;
    HIPTRY(b.alloc(&b.pair_st, std::max<int64_t>(pc, 1)));
    HIPTRY(b.alloc(&b.cfill, std::max<int64_t>(b.chunk_cap, 1)));
    HIPTRY(b.alloc(&b.nchunks, 1));
    HIPTRY(b.alloc(&b.bcnt, std::max<int64_t>(ix.nB, 1)));
    HIPTRY(b.alloc(&b.bchunks, (int64_t)std::max<int64_t>(ix.nB, 1) * b.maxc));
    const int64_t nl = std::max<int64_t>(ix.n_pad, 1) * bscan_list_len(ix.kmax);
    HIPTRY(b.alloc(&b.gl_v, nl));
    HIPTRY(b.alloc(&b.gl_i, nl));
    HIPTRY(b.alloc(&b.gdone, std::max<int64_t>(ix.n_pad, 1)));
    const int64_t np1 = std::max<int64_t>(ix.n_pad, 1);
    HIPTRY(b.alloc(&b.sg_count, 2));
    HIPTRY(b.alloc(&b.sg_users, 2 * np1));
    HIPTRY(b.alloc(&b.sg_block, std::max<int64_t>(ix.nB, 1)));
    HIPTRY(b.alloc(&b.st_np, np1));
    HIPTRY(b.alloc(&b.st_pk, np1 * kUserPairs));
    HIPTRY(b.alloc(&b.st_plo, np1 * kUserPairs));
    HIPTRY(b.alloc(&b.st_ph, np1 * kUserPairs));
    HIPTRY(b.alloc(&b.sg_key, np1));
    HIPTRY(b.alloc(&b.sg_sorted, np1));
  }
  HIPTRY(hipMemsetAsync(b.bits, 0, (size_t)chunk * std::max<int64_t>(W, 1) * 4, s));
  HIPTRY(hipMemsetAsync(b.counts, 0, (size_t)chunk * 8, s));
  HIPTRY(hipStreamSynchronize(s));
  b.qcap = chunk;
  b.pair_cap = pc;
  return RK_OK;
}

// Stage k values in pinned memory (guarded by an event so a previous copy
// out of it has finished) and copy them to the device.
rk_status stage_ks(BatchWS& b, const int32_t* ks, int64_t nq, int32_t* dst, hipStream_t s) {
  if (!b.ks_done) HIPTRY(hipEventCreateWithFlags(&b.ks_done, hipEventDisableTiming));
  HIPTRY(hipEventSynchronize(b.ks_done));
  if (b.ks_pinned_cap < nq) {
    if (b.ks_pinned) (void)hipHostFree(b.ks_pinned);
    b.ks_pinned = nullptr;
    b.ks_pinned_cap = 0;
    HIPTRY(hipHostMalloc((void**)&b.ks_pinned, nq * sizeof(int32_t), hipHostMallocDefault));
    b.ks_pinned_cap = nq;
  }
  std::memcpy(b.ks_pinned, ks, nq * sizeof(int32_t));
  HIPTRY(hipMemcpyAsync(dst, b.ks_pinned, nq * sizeof(int32_t), hipMemcpyHostToDevice, s));
  HIPTRY(hipEventRecord(b.ks_done, s));
  return RK_OK;
}

// The batch path cannot run this index's tiles (too wide for the filter's or
// the scan's LDS): batch calls go one query at a time through the index's
// single-query workspace.
bool batch_one_at_a_time(const DevIndex& ix) {
  const size_t tile_bytes = ix.bf16 ? (size_t)ix.d16 * TILE * 2 : (size_t)(ix.d + (ix.d & 1)) * TILE * 4;
  return bfilter_lds_bytes(ix) > kMaxLds || tile_bytes > bfilter_max_tile_bytes() ||
         (!ix.exact && !bscan_fits(ix));
}

// Enqueues a batch on stream s with workspace b (per-kernel event timing
// only when `timed`, for the index's own calls).  small_direct: the caller
// is the index's only user, so a batch of at most small_batch_max(nB)
// queries may run one query at a time on the index's one-query workspace
// (faster than the batched kernels' per-block cost for so few queries).  chunk > 0: queries per
// chunk, for a workspace already laid out for it (no growth); direct_ks: the
// k values go to the device straight from the caller's memory instead of
// through the workspace's pinned staging.
rk_status batch_enqueue(rk_index* h, BatchWS& b, const float* qs_dev, int64_t nq,
                        const int32_t* ks, int64_t* offs, int32_t* ids, int64_t cap,
                        hipStream_t s, bool timed, int32_t chunk_fixed = 0,
                        bool direct_ks = false, bool small_direct = false) {
  const DevIndex& ix = h->ix;
  launch_set_i64(offs, 0, s);
  HIPTRY(hipGetLastError());
  if (nq == 0) return RK_OK;
  if (batch_one_at_a_time(ix) || (small_direct && nq <= small_batch_max(ix.nB))) {
    // too wide for the block-resident batched filter, or too few queries to
    // pay for its per-block cost: one query at a time
    for (int64_t i = 0; i < nq; ++i) {
      rk_status st = enqueue_query(h, qs_dev + i * ix.d, ks[i], ids, cap, offs + i, offs + i + 1,
                                   s, nullptr, nullptr);
      if (st != RK_OK) return st;
    }
    return RK_OK;
  }
  const int64_t W = bitmap_words(ix.n);
  const int32_t chunk = chunk_fixed > 0 ? chunk_fixed : batch_chunk(h, nq);
  // bounded table, large batches: the scan's first pass for every block
  // first, so that the filter's Lemma 1 and 3 tests use the tighter bounds
  // of the longer prefix and leave far fewer pairs
  const bool prescan = !ix.exact && nq >= kPrescanMin;
  rk_status st = RK_OK;
  if (chunk_fixed <= 0 && (st = ensure_batch_ws(h, b, chunk, s)) != RK_OK) return st;
  for (int64_t c0 = 0; c0 < nq; c0 += chunk) {
    const int32_t nc = (int32_t)std::min<int64_t>(chunk, nq - c0);
    if (direct_ks) {
      HIPTRY(hipMemcpyAsync(b.ks_dev, ks + c0, nc * sizeof(int32_t), hipMemcpyHostToDevice, s));
    } else if ((st = stage_ks(b, ks + c0, nc, b.ks_dev, s)) != RK_OK) {
      return st;
    }
    BatchView bv{};
    bv.qs = qs_dev + c0 * ix.d;
    bv.qn = b.qn; bv.perm = b.perm; bv.qt = b.qt; bv.qb = b.qb;
    bv.qn_s = b.qn_s; bv.k_s = b.k_s; bv.kofs_s = b.kofs_s; bv.tsum = b.tsum;
    bv.nq_pad = (int32_t)round_up(nc, TILE);
    bv.bits = b.bits; bv.W = W; bv.counts = b.counts; bv.all = b.all; bv.n = ix.n;
    bv.npairs = b.npairs; bv.pair_cap = (int32_t)b.pair_cap;
    bv.pair_u = b.pair_u; bv.pair_j = b.pair_j; bv.pair_s = b.pair_s;
    bv.pair_st = b.pair_st; bv.cfill = b.cfill; bv.nchunks = b.nchunks;
    bv.chunk_cap = b.chunk_cap; bv.maxc = b.maxc; bv.bcnt = b.bcnt; bv.bchunks = b.bchunks;
    bv.gl_v = b.gl_v; bv.gl_i = b.gl_i; bv.gdone = b.gdone;
    bv.sg_count = b.sg_count; bv.sg_users = b.sg_users; bv.sg_block = b.sg_block;
    bv.st_np = b.st_np; bv.st_pk = b.st_pk; bv.st_plo = b.st_plo; bv.st_ph = b.st_ph;
    bv.sg_key = b.sg_key; bv.sg_sorted = b.sg_sorted;
    bv.carry_in = c0 > 0 || prescan;
    bv.carry_out = c0 + nc < nq;
    bv.lists = prescan;
    if (c0 == 0 && prescan) {
      Timer t(h, s, K_BPAIRS, timed);
      launch_bprescan(ix, bv, s);  // every user's list over the item prefix, before any pair
    } else if (c0 == 0 && bv.carry_out) {
      launch_bscan_reset(ix, bv, s);  // the scan state is per call
    }
    bv.ctr = h->counting ? h->ctr_dev : nullptr;
    { Timer t(h, s, K_BPREP, timed); launch_bprep(ix, bv, b.ks_dev, nc, s); }
    { Timer t(h, s, K_BFILTER, timed); launch_bfilter(ix, bv, s); }
    { Timer t(h, s, K_BPAIRS, timed); launch_bpairs(ix, bv, s); }
    { Timer t(h, s, K_BASSEMBLE, timed); launch_bassemble(bv, nc, offs + c0, offs + c0, ids, cap, s); }
    HIPTRY(hipGetLastError());
    h->queries += nc;
  }
  return RK_OK;
}

}  // namespace

// ===========================================================================
// Workspace for callers that cannot allocate
// (rk_reverse_kmips_batch_dev_noalloc): one static device array per GPU,
// shared by every such call on that GPU and kept until the process ends.
constexpr size_t kScratchBytes = size_t(64) << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kScratchDevices] = {};

// Device address of the current device's scratch array, looked up once per
// device (in host code `scratch` names a host-side stand-in, not this address).
rk_status scratch_for(int device, unsigned char** out) {
  if (device < 0 || device >= kScratchDevices) return fail(RK_E_INVAL, "device ordinal too large");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(RK_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[device] = (unsigned char*)p;
  }
  *out = g_scratch_ptr[device];
  return RK_OK;
}

// Points the workspace b at the layout of chunks of `chunk` queries inside
// the static array at base.
void carve_ws(const rk_index* h, BatchWS& b, int32_t chunk, unsigned char* base, size_t bytes) {
  const ScratchLayout L = scratch_layout(shape_of(h), chunk, bytes);
  b = BatchWS();
  b.bits = (uint32_t*)(base + L.bits);
  b.counts = (unsigned long long*)(base + L.counts);
  b.qn = (float*)(base + L.qn);
  b.perm = (int32_t*)(base + L.perm);
  b.qt = (float*)(base + L.qt);
  b.qb = h->ix.bf16 ? (uint16_t*)(base + L.qb) : nullptr;
  b.qn_s = (float*)(base + L.qn_s);
  b.k_s = (int32_t*)(base + L.k_s);
  b.kofs_s = (int32_t*)(base + L.kofs_s);
  b.tsum = (int32_t*)(base + L.tsum);
  b.all = (uint8_t*)(base + L.all);
  b.npairs = (unsigned long long*)(base + L.npairs);
  b.ks_dev = (int32_t*)(base + L.ks);
  b.pair_u = (int32_t*)(base + L.pair_u);
  b.pair_j = (int32_t*)(base + L.pair_j);
  b.pair_s = (float*)(base + L.pair_s);
  b.pair_cap = L.pc;
  b.qcap = chunk;
}

}  // namespace

// ===========================================================================
// Serving: continuous batching over resident catalogs (rk_server_*).
//
// Every catalog has `slots` launch slots.  A slot owns a HIP stream, a
// batch workspace sized for max_batch queries, query/offset/id buffers and a
// thread.  A free slot takes whatever the catalog has queued (up to
// max_batch), launches it on its stream and waits for it; requests that
// arrive meanwhile are taken by the next free slot, so their work runs on
// the device while the earlier launch is still there.  Device memory is
// reserved per slot when the catalog is admitted, so requests never allocate
// workspace; only the id buffers of a slot grow, within the budget.
namespace {

struct ServerReq {
  int32_t k = 0;
  int64_t tag = 0;
  double t_submit = 0;
  std::vector<float> q;
};

struct ServerDone {
  rk_completion c{};
  std::vector<int32_t> ids;
};

struct ServerSlot {
  BatchWS ws;
  hipStream_t stream = nullptr;
  float* q_dev = nullptr;
  int64_t* offs_dev = nullptr;
  int32_t* ids_dev = nullptr;
  int64_t ids_cap = 0;
  float* q_pin = nullptr;
  int64_t* offs_pin = nullptr;
  int32_t* ids_pin = nullptr;
  std::thread worker;
};

struct ServerCatalog {
  rk_index* idx = nullptr;
  int32_t d = 0;
  std::deque<ServerReq> queue;
  std::vector<ServerSlot*> slots;
  int32_t running = 0;          // slots with a launch in flight
  std::vector<std::pair<double, int64_t>> starts;  // start and size of each running launch
  int64_t bytes = 0;            // device bytes charged to the budget
  double est_ms[kSizeBuckets];  // moving average of launch time by batch size (< 0: none yet)
  std::condition_variable cv;   // requests queued, a launch ended, or the server stops
  ServerCatalog() { for (double& e : est_ms) e = -1.0; }
  // Estimated time of a launch of nq queries: the smallest bucket at or
  // above nq's with a measurement (< 0 when there is none).
  double estimate(int64_t nq) const {
    for (int b = size_bucket(nq); b < kSizeBuckets; ++b)
      if (est_ms[b] >= 0) return est_ms[b];
    return -1.0;
  }
};

double ms_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

void free_slot_buffers(ServerSlot* c) {
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  c->ws.destroy();
  if (c->q_dev) (void)hipFree(c->q_dev);
  if (c->offs_dev) (void)hipFree(c->offs_dev);
  if (c->ids_dev) (void)hipFree(c->ids_dev);
  if (c->q_pin) (void)hipHostFree(c->q_pin);
  if (c->offs_pin) (void)hipHostFree(c->offs_pin);
  if (c->ids_pin) (void)hipHostFree(c->ids_pin);
  if (c->stream) (void)hipStreamDestroy(c->stream);
  c->q_dev = nullptr;
  c->offs_dev = nullptr;
  c->ids_dev = nullptr;
  c->q_pin = nullptr;
  c->offs_pin = nullptr;
  c->ids_pin = nullptr;
  c->stream = nullptr;
}

hipError_t alloc_ids(ServerSlot* c, int64_t cap) {
  if (c->ids_dev) (void)hipFree(c->ids_dev);
  if (c->ids_pin) (void)hipHostFree(c->ids_pin);
  c->ids_dev = nullptr;
  c->ids_pin = nullptr;
  c->ids_cap = 0;
  hipError_t e = hipMalloc((void**)&c->ids_dev, cap * sizeof(int32_t));
  if (e == hipSuccess) e = hipHostMalloc((void**)&c->ids_pin, cap * sizeof(int32_t), hipHostMallocDefault);
  if (e == hipSuccess) c->ids_cap = cap;
  return e;
}

}  // namespace

struct rk_server {
  rk_server_opts opts{};
  std::chrono::steady_clock::time_point t0;
  std::vector<ServerCatalog*> cats;
  std::mutex mu;
  std::condition_variable cv_done;
  std::deque<ServerDone> done;
  int64_t inflight = 0;
  int64_t used = 0;
  int64_t budget = 0;
  bool stop = false;

  // Grows slot c's id buffers to hold `want` ids if the budget allows.
  bool grow_ids(ServerCatalog* cat, ServerSlot* c, int64_t want) {
    const int64_t cap = want + want / 4 + 1024;
    const int64_t extra = (cap - c->ids_cap) * (int64_t)sizeof(int32_t);
    {
      std::lock_guard<std::mutex> lk(mu);
      if (used + extra > budget) return false;
      used += extra;
      cat->bytes += extra;
    }
    const int64_t old = c->ids_cap;
    if (alloc_ids(c, cap) == hipSuccess) return true;
    // the old buffers are gone too: take back what they held, try them again
    std::lock_guard<std::mutex> lk(mu);
    used -= extra;
    cat->bytes -= extra;
    if (alloc_ids(c, old) != hipSuccess) {
      used -= old * (int64_t)sizeof(int32_t);
      cat->bytes -= old * (int64_t)sizeof(int32_t);
    }
    return false;
  }

  void finish(int32_t ci, const std::vector<ServerReq>& batch, int64_t lo, int64_t hi,
              rk_status st, const ServerSlot* c) {
    const double t_done = ms_since(t0);
    std::lock_guard<std::mutex> lk(mu);
    for (int64_t i = lo; i < hi; ++i) {
      ServerDone dn;
      dn.c.tag = batch[i].tag;
      dn.c.catalog = ci;
      dn.c.status = st;
      dn.c.submit_ms = batch[i].t_submit;
      dn.c.done_ms = t_done;
      if (st == RK_OK) {
        const int64_t a = c->offs_pin[i - lo], b = c->offs_pin[i - lo + 1];
        dn.c.count = b - a;
        dn.ids.assign(c->ids_pin + a, c->ids_pin + b);
      }
      done.push_back(std::move(dn));
    }
    inflight -= hi - lo;
    cv_done.notify_all();
  }

  // Runs requests [lo, hi) of a batch on slot c and hands their results over.
  // A launch whose ids do not fit the slot's buffers grows them within the
  // budget and runs again; when the budget does not allow it, the range is
  // run in halves (a single request that cannot fit fails with RK_E_NOMEM).
  void run_range(int32_t ci, ServerCatalog* cat, ServerSlot* c, const std::vector<ServerReq>& batch,
                 int64_t lo, int64_t hi) {
    const int64_t nq = hi - lo;
    const int d = cat->d;
    std::vector<int32_t> ks(nq);
    for (int64_t i = 0; i < nq; ++i) {
      std::memcpy(c->q_pin + i * d, batch[lo + i].q.data(), d * sizeof(float));
      ks[i] = batch[lo + i].k;
    }
    rk_status st = RK_OK;
    int64_t total = 0;
    hipError_t e = hipMemcpyAsync(c->q_dev, c->q_pin, nq * d * sizeof(float), hipMemcpyHostToDevice, c->stream);
    for (int attempt = 0; attempt < 2 && e == hipSuccess; ++attempt) {
      // with one slot the catalog's index has no other user: small batches
      // may take the one-query path
      st = batch_enqueue(cat->idx, c->ws, c->q_dev, nq, ks.data(), c->offs_dev, c->ids_dev, c->ids_cap,
                         c->stream, false, 0, false, cat->slots.size() == 1);
      if (st != RK_OK) break;
      e = hipMemcpyAsync(c->offs_pin, c->offs_dev, (nq + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, c->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
      if (e != hipSuccess) break;
      total = c->offs_pin[nq];
      if (total <= c->ids_cap) break;
      if (attempt == 1 || !grow_ids(cat, c, total)) {
        if (nq == 1) {
          st = fail(RK_E_NOMEM, "serving: a result does not fit the device budget");
          break;
        }
        const int64_t mid = lo + nq / 2;
        run_range(ci, cat, c, batch, lo, mid);
        run_range(ci, cat, c, batch, mid, hi);
        return;
      }
    }
    if (e == hipSuccess && st == RK_OK && total > 0) {
      e = hipMemcpyAsync(c->ids_pin, c->ids_dev, total * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    }
    if (st == RK_OK && e != hipSuccess) st = e == hipErrorOutOfMemory ? RK_E_NOMEM : RK_E_DEVICE;
    finish(ci, batch, lo, hi, st, c);
  }

  // Thread of one slot of catalog ci.  With no launch of the catalog on the
  // device it takes the queued requests at once.  While other slots'
  // launches run, it joins in only when the first of them to end is
  // expected to run at least twice as long again as the queued requests
  // take on their own (measured launch times by batch size; before a
  // launch of that size has been measured: when it has run twice as long):
  // a request arriving early in a long launch then finishes long before
  // it, while a launch that ends soon is waited for rather than slowed down
  // by splitting the device.
  void loop(int32_t ci, ServerCatalog* cat, ServerSlot* c) {
    (void)hipSetDevice(opts.device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      cat->cv.wait(lk, [&] { return stop || !cat->queue.empty(); });
      if (cat->queue.empty()) {
        if (stop) break;
        continue;
      }
      if (opts.max_wait_us > 0) {
        const double deadline = cat->queue.front().t_submit + opts.max_wait_us / 1000.0;
        while (!stop && (int64_t)cat->queue.size() < opts.max_batch) {
          const double left = deadline - ms_since(t0);
          if (left <= 0) break;
          cat->cv.wait_for(lk, std::chrono::duration<double, std::milli>(left));
        }
        if (cat->queue.empty()) continue;  // another slot took them
      }
      if (cat->running > 0 && !stop) {
        const int64_t want = std::min<int64_t>((int64_t)cat->queue.size(), opts.max_batch);
        const double tb = cat->estimate(want);
        if (tb < 0) {                       // no estimate yet: wait for the launch to end
          cat->cv.wait(lk);
          continue;
        }
        const double now = ms_since(t0);
        double left = INFINITY, elapsed = 0;
        bool known = true;
        for (const auto& r : cat->starts) {
          const double er = cat->estimate(r.second);
          known = known && er >= 0;
          left = std::min(left, er - (now - r.first));
          elapsed = std::max(elapsed, now - r.first);
        }
        if (known && left < 2 * tb) {       // ends soon: wait for it
          cat->cv.wait(lk);
          continue;
        }
        if (!known && elapsed < 2 * tb) {
          cat->cv.wait_for(lk, std::chrono::duration<double, std::milli>(2 * tb - elapsed));
          continue;
        }
      }
      const int64_t nb = std::min<int64_t>((int64_t)cat->queue.size(), opts.max_batch);
      std::vector<ServerReq> batch;
      batch.reserve(nb);
      for (int64_t i = 0; i < nb; ++i) {
        batch.push_back(std::move(cat->queue.front()));
        cat->queue.pop_front();
      }
      ++cat->running;
      const double started = ms_since(t0);
      cat->starts.emplace_back(started, nb);
      lk.unlock();
      run_range(ci, cat, c, batch, 0, nb);
      lk.lock();
      const double took = ms_since(t0) - started;
      cat->starts.erase(std::find(cat->starts.begin(), cat->starts.end(), std::make_pair(started, nb)));
      --cat->running;
      double& e = cat->est_ms[size_bucket(nb)];
      e = e < 0 ? took : 0.7 * e + 0.3 * took;
      cat->cv.notify_all();  // slots waiting for this launch re-decide
    }
  }

  ~rk_server() {
    {
      std::lock_guard<std::mutex> lk(mu);
      stop = true;
    }
    for (ServerCatalog* cat : cats) cat->cv.notify_all();
    for (ServerCatalog* cat : cats)
      for (ServerSlot* c : cat->slots)
        if (c->worker.joinable()) c->worker.join();
    (void)hipSetDevice(opts.device);
    for (ServerCatalog* cat : cats) {
      for (ServerSlot* c : cat->slots) {
        free_slot_buffers(c);
        delete c;
      }
      cat->idx->served--;
      delete cat;
    }
  }
};

// ===========================================================================
extern "C" {

void rk_build_opts_default(rk_build_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precision = RK_FP32;
  o->lb_items = 0;
  o->block_size = 0;
  o->device = 0;
  o->margin_rel = 0.0;
  o->cand_cap = 0;
  o->auto_rebuild = 0;
}

const char* rk_last_error(void) { return g_err.c_str(); }

rk_status rk_build_index(const float* Q, int64_t n, const float* P, int64_t m, int32_t d,
                         int32_t k_max, const rk_build_opts* opts, rk_index** out) {
  return build_impl(Q, n, P, m, d, k_max, opts, false, out);
}

rk_status rk_build_index_dev(const float* Q, int64_t n, const float* P, int64_t m, int32_t d,
                             int32_t k_max, const rk_build_opts* opts, rk_index** out) {
  return build_impl(Q, n, P, m, d, k_max, opts, true, out);
}

void rk_index_free(rk_index* idx) { delete idx; }

rk_status rk_index_rebuild(rk_index* h, int32_t k_max) {
  if (!h) return fail(RK_E_INVAL, "index is NULL");
  if (h->served > 0) return fail(RK_E_INVAL, "the index is a catalog of a server (free the server first)");
  if (k_max < 1 || k_max > kMaxKmax) return fail(RK_E_INVAL, "k_max must be in [1, 128]");
  HIPTRY(hipSetDevice(h->device));
  auto t0 = std::chrono::steady_clock::now();
  HIPTRY(hipStreamSynchronize(h->stream));
  for (void* p : {(void*)h->L64, (void*)h->L32, (void*)h->LB, (void*)h->bnorm}) h->dfree(p);
  h->ix.kmax = k_max;
  rk_status st = build_bounds(h);
  if (st != RK_OK) return st;
  h->rebuilds++;
  h->build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return RK_OK;
}

rk_status rk_index_add_items(rk_index* h, const float* P, int64_t m_new) {
  if (!h) return fail(RK_E_INVAL, "index is NULL");
  if (h->served > 0) return fail(RK_E_INVAL, "the index is a catalog of a server (free the server first)");
  if (m_new < 0 || (m_new > 0 && !P)) return fail(RK_E_INVAL, "P is NULL or m_new < 0");
  if (m_new == 0) return RK_OK;
  DevIndex& ix = h->ix;
  rk_status st = check_sizes(ix.n, ix.m + m_new, ix.d, ix.kmax);
  if (st != RK_OK) return st;
  if (!host_values_ok(P, m_new * ix.d)) return fail(RK_E_INVAL, "input has a non-finite value or |x| >= 2^40");
  HIPTRY(hipSetDevice(h->device));
  auto t0 = std::chrono::steady_clock::now();
  HIPTRY(hipDeviceSynchronize());
  const int64_t m_old = ix.m, m_all = m_old + m_new;
  const int32_t d = ix.d;
  std::vector<float> rows;
  if ((st = side_rows_host(h, false, rows)) != RK_OK) return st;
  rows.resize((size_t)m_all * d);
  std::memcpy(&rows[(size_t)m_old * d], P, (size_t)m_new * d * sizeof(float));
  float* Pall = nullptr;
  HIPTRY(hipMalloc(&Pall, (size_t)m_all * d * sizeof(float)));
  hipError_t e = hipMemcpyAsync(Pall, rows.data(), (size_t)m_all * d * sizeof(float), hipMemcpyHostToDevice,
                                h->stream);
  if (e != hipSuccess) { (void)hipFree(Pall); HIPTRY(e); }
  free_side(h, false);
  st = build_side(h, Pall, m_all, false, nullptr);
  if (st == RK_OK && ix.exact) {
    // the exact table stays exact: each user's k_max largest values take
    // the new items' products in
    launch_lb_merge(ix, Pall + m_old * d, m_new, h->L64, h->L32, h->stream);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) { (void)hipFree(Pall); HIPTRY(e); }
    ix.lb_items = (int32_t)m_all;
    h->dfree(h->LB);
    h->dfree(h->bnorm);
    st = build_blocks(h);
  }
  // (a bounded table keeps its rows: the k-th largest value over the first
  // lb_items items of the old order only grows with more items, so they
  // stay lower bounds, and the linear scan covers the grown catalog)
  (void)hipFree(Pall);
  if (st != RK_OK) return st;
  h->updates++;
  h->build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return RK_OK;
}

rk_status rk_index_add_users(rk_index* h, const float* Q, int64_t n_new) {
  if (!h) return fail(RK_E_INVAL, "index is NULL");
  if (h->served > 0) return fail(RK_E_INVAL, "the index is a catalog of a server (free the server first)");
  if (n_new < 0 || (n_new > 0 && !Q)) return fail(RK_E_INVAL, "Q is NULL or n_new < 0");
  if (n_new == 0) return RK_OK;
  DevIndex& ix = h->ix;
  rk_status st = check_sizes(ix.n + n_new, ix.m, ix.d, ix.kmax);
  if (st != RK_OK) return st;
  if (!host_values_ok(Q, n_new * ix.d)) return fail(RK_E_INVAL, "input has a non-finite value or |x| >= 2^40");
  HIPTRY(hipSetDevice(h->device));
  auto t0 = std::chrono::steady_clock::now();
  HIPTRY(hipDeviceSynchronize());
  hipStream_t s = h->stream;
  const int64_t n_old = ix.n, n_all = n_old + n_new;
  const int64_t old_pad = ix.n_pad, new_pad = round_up(n_new, TILE);
  const int32_t d = ix.d, K = ix.kmax;
  std::vector<void*> tmp;
  auto cleanup = [&]() { for (void* p : tmp) (void)hipFree(p); tmp.clear(); };
#define UTRY(expr)                                       \
  do {                                                   \
    hipError_t ue_ = (expr);                             \
    if (ue_ != hipSuccess) { cleanup(); HIPTRY(ue_); }   \
  } while (0)
  auto talloc = [&](void** p, size_t bytes) {
    hipError_t e = hipMalloc(p, std::max<size_t>(bytes, 1));
    if (e == hipSuccess) tmp.push_back(*p);
    return e;
  };
  // 1. the new users' lower-bound rows, from a view of the index whose users
  // are the new ones (in their given order)
  float *Qn = nullptr, *Qtn = nullptr, *normn = nullptr, *rown = nullptr, *L32n = nullptr;
  double *s2n = nullptr, *L64n = nullptr;
  int32_t* idn = nullptr;
  uint16_t* Qbn = nullptr;
  UTRY(talloc((void**)&Qn, (size_t)n_new * d * sizeof(float)));
  UTRY(talloc((void**)&s2n, (size_t)n_new * sizeof(double)));
  UTRY(talloc((void**)&idn, (size_t)n_new * sizeof(int32_t)));
  UTRY(talloc((void**)&Qtn, (size_t)new_pad * d * sizeof(float)));
  UTRY(talloc((void**)&normn, (size_t)new_pad * sizeof(float)));
  UTRY(talloc((void**)&rown, (size_t)n_new * d * sizeof(float)));
  if (ix.bf16) UTRY(talloc((void**)&Qbn, (size_t)new_pad * ix.d16 * sizeof(uint16_t)));
  UTRY(talloc((void**)&L64n, (size_t)K * new_pad * sizeof(double)));
  UTRY(talloc((void**)&L32n, (size_t)K * new_pad * sizeof(float)));
  std::vector<int32_t> iden(n_new);
  std::iota(iden.begin(), iden.end(), 0);
  UTRY(hipMemcpyAsync(Qn, Q, (size_t)n_new * d * sizeof(float), hipMemcpyHostToDevice, s));
  UTRY(hipMemcpyAsync(idn, iden.data(), n_new * sizeof(int32_t), hipMemcpyHostToDevice, s));
  launch_sqnorms(Qn, n_new, d, s2n, s);
  launch_tile_rows(Qn, idn, s2n, n_new, new_pad, d, ix.d16, Qtn, normn, Qbn, rown, s);
  UTRY(hipGetLastError());
  DevIndex tx = ix;
  tx.n = n_new;
  tx.n_pad = new_pad;
  tx.nB = (int32_t)(new_pad / TILE);
  tx.nSB = (int32_t)(new_pad / ix.bsize);
  tx.Qt = Qtn; tx.normQ = normn; tx.Qb = Qbn; tx.Qrow = rown; tx.permQ = idn;
  st = compute_bounds(h, tx, L64n, L32n);
  if (st != RK_OK) { cleanup(); return st; }
  // 2. the grown user side in its norm order
  std::vector<float> rows;
  std::vector<int32_t> perm_old(n_old);
  if (n_old) UTRY(hipMemcpyAsync(perm_old.data(), h->permQ, n_old * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  if ((st = side_rows_host(h, true, rows)) != RK_OK) { cleanup(); return st; }
  rows.resize((size_t)n_all * d);
  std::memcpy(&rows[(size_t)n_old * d], Q, (size_t)n_new * d * sizeof(float));
  float* Qall = nullptr;
  UTRY(talloc((void**)&Qall, (size_t)n_all * d * sizeof(float)));
  UTRY(hipMemcpyAsync(Qall, rows.data(), (size_t)n_all * d * sizeof(float), hipMemcpyHostToDevice, s));
  free_side(h, true);
  std::vector<int32_t> perm_all;
  if ((st = build_side(h, Qall, n_all, true, &perm_all)) != RK_OK) { cleanup(); return st; }
  // 3. rows of the table gathered into that order: old users from their old
  // sorted position, new users from step 1
  std::vector<int64_t> pos_old(n_old), src(n_all);
  for (int64_t i = 0; i < n_old; ++i) pos_old[perm_old[i]] = i;
  for (int64_t i = 0; i < n_all; ++i) {
    const int64_t o = perm_all[i];
    src[i] = o < n_old ? pos_old[o] : -1 - (o - n_old);
  }
  int64_t* srcd = nullptr;
  UTRY(talloc((void**)&srcd, (size_t)n_all * sizeof(int64_t)));
  UTRY(hipMemcpyAsync(srcd, src.data(), n_all * sizeof(int64_t), hipMemcpyHostToDevice, s));
  double* L64o = h->L64;
  float* L32o = h->L32;
  h->L64 = nullptr;
  h->L32 = nullptr;
  UTRY(h->dalloc(&h->L64, (size_t)K * ix.n_pad));
  UTRY(h->dalloc(&h->L32, (size_t)K * ix.n_pad));
  launch_gather_bounds(K, n_all, ix.n_pad, srcd, L64o, L32o, old_pad, L64n, L32n, new_pad, h->L64, h->L32, s);
  UTRY(hipGetLastError());
  UTRY(hipStreamSynchronize(s));
  ix.L64 = h->L64;
  ix.L32 = h->L32;
  h->dfree(L64o);
  h->dfree(L32o);
  cleanup();
#undef UTRY
  // 4. blocks over the grown order, and the workspaces sized by users
  h->dfree(h->LB);
  h->dfree(h->bnorm);
  if ((st = build_blocks(h)) != RK_OK) return st;
  free_user_ws(h);
  if ((st = alloc_user_ws(h)) != RK_OK) return st;
  h->bw.release();
  h->updates++;
  h->build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return RK_OK;
}

rk_status rk_reverse_kmips(rk_index* h, const float* q, int32_t k, int32_t* ids, int64_t cap,
                           int64_t* count) {
  if (!h || !q || !count || (cap > 0 && !ids) || cap < 0) return fail(RK_E_INVAL, "NULL argument or cap < 0");
  rk_status st = check_k(h, k);
  if (st != RK_OK) return st;
  if (!host_values_ok(q, h->ix.d)) return fail(RK_E_INVAL, "q has a non-finite value or |x| >= 2^40");
  HIPTRY(hipSetDevice(h->device));
  std::memcpy(h->q_host, q, h->ix.d * sizeof(float));
  HIPTRY(hipMemcpyAsync(h->q_dev, h->q_host, h->ix.d * sizeof(float), hipMemcpyHostToDevice, h->stream));
  st = enqueue_query(h, h->q_dev, k, h->ids_host_dev, std::max<int64_t>(h->ix.n, 1), nullptr,
                     h->count_host_dev, h->stream, nullptr, nullptr);
  if (st != RK_OK) return st;
  HIPTRY(hipStreamSynchronize(h->stream));
  const int64_t c = *(volatile int64_t*)h->count_host;
  *count = c;
  std::memcpy(ids, h->ids_host, std::min(c, cap) * sizeof(int32_t));
  if (c > cap) return fail(RK_E_TRUNC, "result larger than cap");
  return RK_OK;
}

rk_status rk_reverse_kmips_dev(rk_index* h, const float* q_dev, int32_t k, int32_t* ids_dev,
                               int64_t cap, int64_t* count_dev, void* stream) {
  if (!h || !q_dev || !count_dev || (cap > 0 && !ids_dev) || cap < 0) return fail(RK_E_INVAL, "NULL argument or cap < 0");
  rk_status st = check_k(h, k);
  if (st != RK_OK) return st;
  HIPTRY(hipSetDevice(h->device));
  hipStream_t s = stream ? (hipStream_t)stream : h->stream;
  return enqueue_query(h, q_dev, k, ids_dev, cap, nullptr, count_dev, s, nullptr, nullptr);
}

rk_status rk_reverse_kmips_trace(rk_index* h, const float* q, int32_t k, uint8_t* cls, float* shat) {
  if (!h || !q || !cls) return fail(RK_E_INVAL, "NULL argument");
  rk_status st = check_k(h, k);
  if (st != RK_OK) return st;
  if (!host_values_ok(q, h->ix.d)) return fail(RK_E_INVAL, "q has a non-finite value or |x| >= 2^40");
  HIPTRY(hipSetDevice(h->device));
  const int64_t n = h->ix.n;
  uint8_t* tcls = nullptr;
  float* ts = nullptr;
  HIPTRY(hipMalloc(&tcls, std::max<int64_t>(n, 1)));
  hipError_t e = hipMalloc(&ts, std::max<int64_t>(n, 1) * sizeof(float));
  if (e != hipSuccess) { (void)hipFree(tcls); HIPTRY(e); }
  auto done = [&](rk_status s_) { (void)hipFree(tcls); (void)hipFree(ts); return s_; };
  hipStream_t s = h->stream;
  if ((e = hipMemsetAsync(tcls, RK_C_BLOCK_NO, std::max<int64_t>(n, 1), s)) != hipSuccess ||
      (e = hipMemsetAsync(ts, 0xFF, std::max<int64_t>(n, 1) * sizeof(float), s)) != hipSuccess ||
      (e = hipMemcpyAsync(h->q_dev, q, h->ix.d * sizeof(float), hipMemcpyHostToDevice, s)) != hipSuccess)
    return done(fail(RK_E_DEVICE, hipGetErrorString(e)));
  if (k > h->ix.m) {
    std::memset(cls, RK_C_LEMMA2_YES, n);
    if (shat) for (int64_t i = 0; i < n; ++i) shat[i] = NAN;
    return done(RK_OK);
  }
  st = enqueue_query(h, h->q_dev, k, h->ids_dev, n, nullptr, h->count_dev, s, tcls, ts);
  if (st != RK_OK) return done(st);
  if ((e = hipMemcpyAsync(cls, tcls, n, hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (shat && (e = hipMemcpyAsync(shat, ts, n * sizeof(float), hipMemcpyDeviceToHost, s)) != hipSuccess) ||
      (e = hipStreamSynchronize(s)) != hipSuccess)
    return done(fail(RK_E_DEVICE, hipGetErrorString(e)));
  return done(RK_OK);
}

rk_status rk_reverse_kmips_batch_dev(rk_index* h, const float* qs_dev, int64_t nq,
                                     const int32_t* ks, int64_t* offsets_dev, int32_t* ids_dev,
                                     int64_t cap, void* stream) {
  if (!h || nq < 0 || (nq > 0 && (!qs_dev || !ks)) || !offsets_dev || cap < 0 || (cap > 0 && !ids_dev))
    return fail(RK_E_INVAL, "NULL argument or negative size");
  if (nq > INT32_MAX) return fail(RK_E_INVAL, "nq too large");
  rk_status st = check_batch_ks(h, ks, nq);
  if (st != RK_OK) return st;
  HIPTRY(hipSetDevice(h->device));
  hipStream_t s = stream ? (hipStream_t)stream : h->stream;
  return batch_enqueue(h, h->bw, qs_dev, nq, ks, offsets_dev, ids_dev, cap, s, true, 0, false, true);
}

rk_status rk_reverse_kmips_batch_dev_noalloc(rk_index* h, const float* qs_dev, int64_t nq,
                                             const int32_t* ks, int64_t* offsets_dev,
                                             int32_t* ids_dev, int64_t cap, void* stream) {
  if (!h || nq < 0 || (nq > 0 && (!qs_dev || !ks)) || !offsets_dev || cap < 0 || (cap > 0 && !ids_dev))
    return fail(RK_E_INVAL, "NULL argument or negative size");
  if (nq > INT32_MAX) return fail(RK_E_INVAL, "nq too large");
  const DevIndex& ix = h->ix;
  if (!ix.exact) return fail(RK_E_INVAL, "noalloc batch: needs an exact lower-bound table (lb_items 0 or m)");
  if (batch_one_at_a_time(ix)) return fail(RK_E_INVAL, "noalloc batch: tiles too wide for the batched kernels");
  for (int64_t i = 0; i < nq; ++i) {
    if (ks[i] < 1) return fail(RK_E_INVAL, "k must be >= 1");
    if (ks[i] > ix.kmax && ks[i] <= ix.m)
      return fail(RK_E_KMAX, "noalloc batch: k > k_max (a rebuild would allocate)");
  }
  HIPTRY(hipSetDevice(h->device));
  hipStream_t s = stream ? (hipStream_t)stream : h->stream;
  unsigned char* base = nullptr;
  rk_status st = scratch_for(h->device, &base);
  if (st != RK_OK) return st;
  if (nq == 0 || ix.n == 0) {  // every row is empty
    launch_fill_i32((int32_t*)offsets_dev, 2 * (nq + 1), 0, s);
    HIPTRY(hipGetLastError());
    return RK_OK;
  }
  // the largest chunk (a power-of-two fraction of the regular one, at least
  // 64 queries) whose workspace fits with room for 64 Ki pair slots
  const int32_t chunk = noalloc_chunk(shape_of(h), nq, kScratchBytes);
  if (chunk == 0)
    return fail(RK_E_INVAL, "noalloc batch: " + std::to_string(ix.n) + " users need more than the " +
                                std::to_string(kScratchBytes >> 20) + " MiB static workspace");
  BatchWS b;
  carve_ws(h, b, chunk, base, kScratchBytes);
  // the array keeps the last call's contents: result bits and counts must
  // start at zero (the assembly clears them again after each chunk)
  const int64_t W = bitmap_words(ix.n);
  launch_fill_i32((int32_t*)b.bits, (int64_t)chunk * std::max<int64_t>(W, 1), 0, s);
  launch_fill_i32((int32_t*)b.counts, 2 * (int64_t)chunk, 0, s);
  HIPTRY(hipGetLastError());
  return batch_enqueue(h, b, qs_dev, nq, ks, offsets_dev, ids_dev, cap, s, false, chunk, true);
}

rk_status rk_reverse_kmips_batch(rk_index* h, const float* qs, int64_t nq, const int32_t* ks,
                                 int64_t* offsets, int32_t* ids, int64_t cap) {
  if (!h || nq < 0 || (nq > 0 && (!qs || !ks)) || !offsets || cap < 0 || (cap > 0 && !ids))
    return fail(RK_E_INVAL, "NULL argument or negative size");
  rk_status st = check_batch_ks(h, ks, nq);
  if (st != RK_OK) return st;
  if (!host_values_ok(qs, nq * h->ix.d)) return fail(RK_E_INVAL, "a query has a non-finite value or |x| >= 2^40");
  HIPTRY(hipSetDevice(h->device));
  hipStream_t s = h->stream;
  float* qd = nullptr;
  int64_t* od = nullptr;
  int32_t* idd = nullptr;
  const int64_t dcap = std::max<int64_t>(cap, 1);
  std::vector<void*> tmp;
  auto done = [&](rk_status r) { (void)hipStreamSynchronize(s); for (void* p : tmp) (void)hipFree(p); return r; };
  hipError_t e = hipMalloc(&qd, std::max<int64_t>(nq * h->ix.d, 1) * sizeof(float));
  if (e == hipSuccess) { tmp.push_back(qd); e = hipMalloc(&od, (nq + 1) * sizeof(int64_t)); }
  if (e == hipSuccess) { tmp.push_back(od); e = hipMalloc(&idd, dcap * sizeof(int32_t)); }
  if (e == hipSuccess) { tmp.push_back(idd); if (nq) e = hipMemcpyAsync(qd, qs, nq * h->ix.d * sizeof(float), hipMemcpyHostToDevice, s); }
  if (e != hipSuccess) return done(fail(e == hipErrorOutOfMemory ? RK_E_NOMEM : RK_E_DEVICE, hipGetErrorString(e)));
  st = rk_reverse_kmips_batch_dev(h, qd, nq, ks, od, idd, cap, s);
  if (st != RK_OK) return done(st);
  if ((e = hipMemcpyAsync(offsets, od, (nq + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (e = hipStreamSynchronize(s)) != hipSuccess)
    return done(fail(RK_E_DEVICE, hipGetErrorString(e)));
  const int64_t total = offsets[nq];
  const int64_t ncopy = std::min(total, cap);
  if (ncopy > 0 && (e = hipMemcpyAsync(ids, idd, ncopy * sizeof(int32_t), hipMemcpyDeviceToHost, s)) != hipSuccess)
    return done(fail(RK_E_DEVICE, hipGetErrorString(e)));
  st = done(RK_OK);
  if (total > cap) return fail(RK_E_TRUNC, "results larger than cap");
  return st;
}

rk_status rk_index_set_timing(rk_index* h, int32_t max_launches) {
  if (!h || max_launches < 0) return fail(RK_E_INVAL, "index is NULL or max_launches < 0");
  HIPTRY(hipSetDevice(h->device));
  HIPTRY(hipStreamSynchronize(h->stream));
  h->ev_used.clear();
  h->ev_next = 0;
  const size_t want = (size_t)max_launches * 2;
  while (h->ev_pool.size() < want) {
    hipEvent_t e;
    HIPTRY(hipEventCreate(&e));
    h->ev_pool.push_back(e);
  }
  h->timing = max_launches > 0;
  return RK_OK;
}

rk_status rk_index_kernel_times(rk_index* h, double* ms, int64_t* launches, int32_t nclass) {
  if (!h || !ms || !launches || nclass < 1) return fail(RK_E_INVAL, "NULL argument");
  for (int i = 0; i < nclass; ++i) { ms[i] = 0; launches[i] = 0; }
  HIPTRY(hipSetDevice(h->device));
  for (auto& u : h->ev_used) {
    HIPTRY(hipEventSynchronize(u.second.second));
    float t = 0;
    HIPTRY(hipEventElapsedTime(&t, u.second.first, u.second.second));
    if (u.first < nclass) { ms[u.first] += t; launches[u.first] += 1; }
  }
  h->ev_used.clear();
  h->ev_next = 0;
  return RK_OK;
}

rk_status rk_index_set_counting(rk_index* h, int32_t on) {
  if (!h) return fail(RK_E_INVAL, "index is NULL");
  h->counting = on != 0;
  return RK_OK;
}

rk_status rk_index_reset_counters(rk_index* h) {
  if (!h) return fail(RK_E_INVAL, "index is NULL");
  HIPTRY(hipSetDevice(h->device));
  HIPTRY(hipMemsetAsync(h->ctr_dev, 0, 16 * sizeof(unsigned long long), h->stream));
  HIPTRY(hipStreamSynchronize(h->stream));
  h->queries = 0;
  return RK_OK;
}

rk_status rk_index_stats(const rk_index* hc, rk_stats* o) {
  if (!hc || !o) return fail(RK_E_INVAL, "NULL argument");
  rk_index* h = const_cast<rk_index*>(hc);
  std::memset(o, 0, sizeof(*o));
  const DevIndex& ix = h->ix;
  o->n = ix.n; o->m = ix.m; o->d = ix.d; o->k_max = ix.kmax; o->lb_items = ix.lb_items;
  o->block_size = ix.bsize; o->n_blocks = ix.nSB; o->precision = ix.bf16 ? RK_BF16 : RK_FP32;
  o->footprint_bytes = (int64_t)h->footprint + h->bw.bytes;
  o->build_ms = h->build_ms;
  o->build_cand_total = h->cand_total;
  o->build_cand_overflow_users = h->cand_ovf;
  o->rebuilds = h->rebuilds;
  o->updates = h->updates;
  o->queries = h->queries;
  unsigned long long c[16] = {};
  HIPTRY(hipSetDevice(h->device));
  HIPTRY(hipMemcpyAsync(c, h->ctr_dev, sizeof(c), hipMemcpyDeviceToHost, h->stream));
  HIPTRY(hipStreamSynchronize(h->stream));
  o->blocks_visited = c[C_BLOCKS]; o->blocks_pruned = c[C_PRUNED]; o->users_evaluated = c[C_USERS];
  o->lemma1_no = c[C_L1NO]; o->lemma2_yes = c[C_L2YES]; o->table_yes = c[C_TYES];
  o->survivors = c[C_SURV]; o->scan_items = c[C_SCAN]; o->rechecks = c[C_RCHK]; o->results = c[C_RES];
  o->scan_long = c[C_LONG]; o->scan_full_f64 = c[C_F64SCAN]; o->scan_handoff = c[C_HANDOFF];
  o->scan_quarters = c[C_SQUART]; o->scan_valu_tiles = c[C_SVALU];
  return RK_OK;
}

rk_status rk_index_export(const rk_index* hc, int32_t field, void* dst, int64_t bytes) {
  if (!hc || !dst) return fail(RK_E_INVAL, "NULL argument");
  rk_index* h = const_cast<rk_index*>(hc);
  const DevIndex& ix = h->ix;
  const void* src = nullptr;
  int64_t need = 0, rows = 0, width = 0, pitch = 0;  // 2-D copies drop padding
  switch (field) {
    case RK_F_PERM_Q: src = h->permQ; need = ix.n * 4; break;
    case RK_F_PERM_P: src = h->permP; need = ix.m * 4; break;
    case RK_F_SQNORM_Q: src = h->s2Q; need = ix.n * 8; break;
    case RK_F_SQNORM_P: src = h->s2P; need = ix.m * 8; break;
    case RK_F_NORM_Q: src = h->normQ; need = ix.n * 4; break;
    case RK_F_NORM_P: src = h->normP; need = ix.m * 4; break;
    case RK_F_L64: src = h->L64; rows = ix.kmax; width = ix.n * 8; pitch = ix.n_pad * 8; break;
    case RK_F_L32: src = h->L32; rows = ix.kmax; width = ix.n * 4; pitch = ix.n_pad * 4; break;
    case RK_F_LB: src = h->LB; need = (int64_t)ix.kmax * ix.nSB * 4; break;
    case RK_F_BNORM: src = h->bnorm; need = (int64_t)ix.nSB * 4; break;
    default: return fail(RK_E_INVAL, "unknown field");
  }
  if (rows) need = rows * width;
  if (bytes != need) return fail(RK_E_INVAL, "size mismatch for field");
  if (need == 0) return RK_OK;
  HIPTRY(hipSetDevice(h->device));
  if (rows) {
    HIPTRY(hipMemcpy2DAsync(dst, width, src, pitch, width, rows, hipMemcpyDeviceToHost, h->stream));
  } else {
    HIPTRY(hipMemcpyAsync(dst, src, need, hipMemcpyDeviceToHost, h->stream));
  }
  HIPTRY(hipStreamSynchronize(h->stream));
  return RK_OK;
}

int64_t rk_index_footprint(int64_t n, int64_t m, int32_t d, int32_t k_max, const rk_build_opts* opts) {
  rk_build_opts o;
  rk_build_opts_default(&o);
  if (opts) o = *opts;
  return index_footprint(n, m, d, k_max, o);
}

void rk_server_opts_default(rk_server_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->max_batch = 1024;
  o->slots = 1;
  o->max_queue = 1 << 16;
}

rk_status rk_server_create(const rk_server_opts* opts, rk_server** out) {
  if (!out) return fail(RK_E_INVAL, "out is NULL");
  *out = nullptr;
  rk_server_opts o;
  rk_server_opts_default(&o);
  if (opts) o = *opts;
  if (o.max_batch == 0) o.max_batch = 1024;
  if (o.slots == 0) o.slots = 1;
  if (o.max_queue == 0) o.max_queue = 1 << 16;
  if (o.max_batch < 0 || o.max_wait_us < 0 || o.hbm_budget < 0 || o.slots < 0 || o.max_queue < 0)
    return fail(RK_E_INVAL, "max_batch, max_wait_us, slots, max_queue and hbm_budget must be >= 0");
  if (o.slots > 16) return fail(RK_E_INVAL, "slots must be at most 16");
  int ndev = 0;
  HIPTRY(hipGetDeviceCount(&ndev));
  if (o.device < 0 || o.device >= ndev) return fail(RK_E_INVAL, "no such device");
  HIPTRY(hipSetDevice(o.device));
  int64_t budget = o.hbm_budget;
  if (budget == 0) {
    size_t fr = 0, tot = 0;
    HIPTRY(hipMemGetInfo(&fr, &tot));
    budget = (int64_t)(0.9 * (double)fr);
  }
  rk_server* s = new rk_server();
  s->opts = o;
  s->budget = budget;
  s->t0 = std::chrono::steady_clock::now();
  *out = s;
  return RK_OK;
}

rk_status rk_server_add_catalog(rk_server* s, rk_index* h, int32_t* catalog) {
  if (!s || !h || !catalog) return fail(RK_E_INVAL, "NULL argument");
  if (h->device != s->opts.device) return fail(RK_E_INVAL, "the index is on another device");
  {
    std::lock_guard<std::mutex> lk(s->mu);
    for (const ServerCatalog* c : s->cats)
      if (c->idx == h) return fail(RK_E_INVAL, "the index is already a catalog of this server");
  }
  HIPTRY(hipSetDevice(s->opts.device));
  const int64_t B = s->opts.max_batch, d = h->ix.d;
  const int32_t chunk = batch_chunk(h, B);
  // an index whose batches go one query at a time shares its single-query
  // workspace between launches: one slot
  const int32_t nslots = batch_one_at_a_time(h->ix) ? 1 : s->opts.slots;
  const int64_t ws = batch_sizes(h, chunk).bytes;
  const int64_t ids0 = B * 64;
  const int64_t bufs = B * d * 4 + (B + 1) * 8 + ids0 * 4;
  const int64_t need = (int64_t)h->footprint + h->bw.bytes + nslots * (ws + bufs);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->used + need > s->budget)
      return fail(RK_E_NOMEM, "admission: the catalog needs " + std::to_string(need) + " device bytes (" +
                                  std::to_string(nslots) + " slots), " +
                                  std::to_string(s->budget - s->used) + " of the budget are left");
    s->used += need;
  }
  auto cat = new ServerCatalog();
  cat->idx = h;
  cat->d = (int32_t)d;
  cat->bytes = need;
  auto undo = [&](rk_status st) {
    for (ServerSlot* c : cat->slots) {
      free_slot_buffers(c);
      delete c;
    }
    delete cat;
    std::lock_guard<std::mutex> lk(s->mu);
    s->used -= need;
    return st;
  };
  for (int32_t i = 0; i < nslots; ++i) {
    auto c = new ServerSlot();
    cat->slots.push_back(c);
    hipError_t e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMalloc((void**)&c->q_dev, std::max<int64_t>(B * d, 1) * sizeof(float));
    if (e == hipSuccess) e = hipMalloc((void**)&c->offs_dev, (B + 1) * sizeof(int64_t));
    if (e == hipSuccess) e = hipHostMalloc((void**)&c->q_pin, std::max<int64_t>(B * d, 1) * sizeof(float), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&c->offs_pin, (B + 1) * sizeof(int64_t), hipHostMallocDefault);
    if (e == hipSuccess) e = alloc_ids(c, ids0);
    if (e != hipSuccess)
      return undo(fail(e == hipErrorOutOfMemory ? RK_E_NOMEM : RK_E_DEVICE, hipGetErrorString(e)));
    rk_status st = ensure_batch_ws(h, c->ws, chunk, c->stream);
    if (st != RK_OK) return undo(st);
  }
  std::lock_guard<std::mutex> lk(s->mu);
  const int32_t ci = (int32_t)s->cats.size();
  *catalog = ci;
  s->cats.push_back(cat);
  h->served++;
  for (ServerSlot* c : cat->slots) c->worker = std::thread([s, ci, cat, c] { s->loop(ci, cat, c); });
  return RK_OK;
}

rk_status rk_server_submit(rk_server* s, int32_t catalog, const float* q, int32_t k, int64_t tag) {
  if (!s || !q) return fail(RK_E_INVAL, "NULL argument");
  ServerReq r;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (catalog < 0 || catalog >= (int32_t)s->cats.size()) return fail(RK_E_INVAL, "no such catalog");
    const rk_index* h = s->cats[catalog]->idx;
    if (k < 1) return fail(RK_E_INVAL, "k must be >= 1");
    if (k > h->ix.kmax) return fail(RK_E_KMAX, "k > k_max of the catalog");
    r.q.assign(q, q + h->ix.d);
  }
  if (!host_values_ok(r.q.data(), (int64_t)r.q.size()))
    return fail(RK_E_INVAL, "the query has a non-finite value or |x| >= 2^40");
  r.k = k;
  r.tag = tag;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    ServerCatalog* cat = s->cats[catalog];
    if ((int64_t)cat->queue.size() >= s->opts.max_queue)
      return fail(RK_E_BUSY, "the catalog's queue is full (max_queue)");
    r.t_submit = ms_since(s->t0);
    cat->queue.push_back(std::move(r));
    ++s->inflight;
    cat->cv.notify_one();
  }
  return RK_OK;
}

rk_status rk_server_submit_many(rk_server* s, int64_t n, const int32_t* catalog,
                                const float* const* q, const int32_t* k, const int64_t* tag,
                                const double* arrival_ms) {
  if (!s || n < 0 || (n > 0 && (!catalog || !q || !k || !tag)))
    return fail(RK_E_INVAL, "NULL argument or negative size");
  std::vector<ServerReq> rs(n);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    for (int64_t i = 0; i < n; ++i) {
      if (catalog[i] < 0 || catalog[i] >= (int32_t)s->cats.size() || !q[i])
        return fail(RK_E_INVAL, "request " + std::to_string(i) + ": no such catalog or NULL query");
      const rk_index* h = s->cats[catalog[i]]->idx;
      if (k[i] < 1) return fail(RK_E_INVAL, "request " + std::to_string(i) + ": k must be >= 1");
      if (k[i] > h->ix.kmax) return fail(RK_E_KMAX, "request " + std::to_string(i) + ": k > k_max");
      rs[i].q.assign(q[i], q[i] + h->ix.d);
    }
  }
  for (int64_t i = 0; i < n; ++i) {
    if (!host_values_ok(rs[i].q.data(), (int64_t)rs[i].q.size()))
      return fail(RK_E_INVAL, "request " + std::to_string(i) + ": a non-finite value or |x| >= 2^40");
    rs[i].k = k[i];
    rs[i].tag = tag[i];
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    std::vector<int64_t> add(s->cats.size(), 0);
    for (int64_t i = 0; i < n; ++i) ++add[catalog[i]];
    for (size_t c = 0; c < s->cats.size(); ++c)
      if ((int64_t)s->cats[c]->queue.size() + add[c] > s->opts.max_queue)
        return fail(RK_E_BUSY, "catalog " + std::to_string(c) + ": the queue has no room for " +
                                   std::to_string(add[c]) + " more requests (max_queue)");
    const double now = ms_since(s->t0);
    for (int64_t i = 0; i < n; ++i) {
      rs[i].t_submit = arrival_ms ? std::min(arrival_ms[i], now) : now;
      s->cats[catalog[i]]->queue.push_back(std::move(rs[i]));
    }
    s->inflight += n;
    for (size_t c = 0; c < s->cats.size(); ++c)
      if (add[c]) s->cats[c]->cv.notify_all();
  }
  return RK_OK;
}

rk_status rk_server_catalog_state(rk_server* s, int32_t catalog, int64_t* queued, int32_t* running) {
  if (!s || !queued || !running) return fail(RK_E_INVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  if (catalog < 0 || catalog >= (int32_t)s->cats.size()) return fail(RK_E_INVAL, "no such catalog");
  *queued = (int64_t)s->cats[catalog]->queue.size();
  *running = s->cats[catalog]->running;
  return RK_OK;
}

double rk_server_now_ms(rk_server* s) { return s ? ms_since(s->t0) : -1.0; }

int64_t rk_server_poll(rk_server* s, rk_completion* out, int64_t max_out, int32_t* ids,
                       int64_t ids_cap, int32_t wait_us) {
  if (!s || max_out < 0 || ids_cap < 0 || (max_out > 0 && !out) || (ids_cap > 0 && !ids)) {
    fail(RK_E_INVAL, "NULL argument or negative size");
    return -1;
  }
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->done.empty() && wait_us > 0)
    s->cv_done.wait_for(lk, std::chrono::microseconds(wait_us), [&] { return !s->done.empty(); });
  int64_t n = 0, used = 0;
  while (n < max_out && !s->done.empty()) {
    ServerDone& dn = s->done.front();
    const int64_t sz = (int64_t)dn.ids.size();
    if (used + sz > ids_cap) {
      if (n == 0) {
        fail(RK_E_TRUNC, "the next finished request has " + std::to_string(sz) + " ids");
        return -1;
      }
      break;
    }
    if (sz) std::memcpy(ids + used, dn.ids.data(), sz * sizeof(int32_t));
    out[n] = dn.c;
    out[n].ids_offset = used;
    used += sz;
    s->done.pop_front();
    ++n;
  }
  return n;
}

int64_t rk_server_inflight(rk_server* s) {
  if (!s) return -1;
  std::lock_guard<std::mutex> lk(s->mu);
  return s->inflight;
}

int64_t rk_server_used_bytes(rk_server* s) {
  if (!s) return -1;
  std::lock_guard<std::mutex> lk(s->mu);
  return s->used;
}

void rk_server_free(rk_server* s) { delete s; }

}  // extern "C"
