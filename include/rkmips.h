/*
 * rkmips.h: C ABI of the MI355X (gfx950) exact reverse k-MIPS library.
 *
 * Method: Simpfer (Amagata & Hara, "Reverse Maximum Inner Product Search",
 * RecSys 2021).  Given users Q (n x d), items P (m x d), a query item q and k,
 * the reverse k-MIPS result is every user u for which q is among the k best
 * items of u over P u {q} (Definition 2, Section 2).  Ties go to q: u is a
 * member iff fewer than k items p in P have f(p,u) > f(q,u).
 *
 * Exactness contract.  f(x,y) is the inner product of the float32 inputs
 * accumulated in double precision in index order (i = 0..d-1).  Every result
 * set returned by this library equals the set defined with that f, whatever
 * precision the bulk arithmetic runs in: decisions taken in float32 or
 * bfloat16 are taken only when a rigorous error bound certifies them, and
 * every other user is decided by a float64 recomputation of f on the device.
 *
 * Conventions for every entry point:
 *  - All matrices are row-major, float32, contiguous; row r of Q is user r.
 *  - Result ids are original row indices of Q, int32, strictly ascending.
 *  - Host pointers are borrowed for the duration of the call only.  "_dev"
 *    entry points take device pointers (HIP device memory of the index's
 *    device) and a hipStream_t passed as void* (NULL = the index's own
 *    stream); they enqueue work and return without waiting unless stated.
 *  - On any error nothing is written to outputs except where stated, no
 *    partial index is left behind, and rk_last_error() returns a message.
 *  - An rk_index is used by one host thread at a time.
 */
#ifndef RKMIPS_H
#define RKMIPS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rk_index rk_index;

typedef enum {
    RK_OK = 0,
    RK_E_INVAL = 1,  /* null pointer, n < 0, m < 0, d < 1, k < 1, k_max < 1,
                        non-finite input or |x_i| >= 2^40, bad option */
    RK_E_KMAX = 2,   /* k > k_max of the index and auto_rebuild is off */
    RK_E_NOMEM = 3,  /* device allocation failed; nothing was created */
    RK_E_TRUNC = 4,  /* output capacity too small; counts hold true sizes */
    RK_E_DEVICE = 5, /* HIP runtime error; see rk_last_error() */
    RK_E_BUSY = 6    /* serving: the catalog's request queue is full */
} rk_status;

typedef enum {
    RK_FP32 = 0,     /* bulk inner products in float32 (VALU or FP32 MFMA) */
    RK_BF16 = 1      /* bulk inner products from bfloat16 copies of Q, P and q
                        with float32 accumulation (BF16 MFMA); users inside
                        the bf16 error margin are recomputed in float64 */
} rk_precision;

/* Options of rk_build_index.  Call rk_build_opts_default() first. */
typedef struct {
    int32_t precision;    /* rk_precision */
    int32_t lb_items;     /* |P'|, the number of largest-norm items the
                             lower-bound arrays are taken over (Definition 4,
                             Algorithm 1).  0 = all of P: the arrays then hold
                             each user's exact k_max largest inner products
                             and every decision is a single certified compare.
                             k_max..m = the paper's P' prefix (its experiments
                             use O(k_max)); values above m are clamped to m. */
    int32_t block_size;   /* users per block of the Lemma 3 filter
                             (Definition 5, Equation (1)): 0 -> 64 (one block
                             = one 64-lane wavefront), 16 or 32 (the kernels
                             still work in 64-user tiles; a tile is skipped
                             when all its blocks are pruned, and the pairs of
                             pruned blocks inside a live tile are not tested) */
    int32_t device;       /* HIP device ordinal */
    double margin_rel;    /* extra relative margin: the certified tests use
                             max(margin_rel, rigorous bound) * |u||q| */
    int32_t cand_cap;     /* 0 = default.  Per-user capacity of the candidate
                             list in the full-table build; users that overflow
                             it are recomputed exactly over all of P (a test
                             hook for that path) */
    int32_t auto_rebuild; /* nonzero: a query with k > k_max first rebuilds
                             the lower-bound arrays with k_max = k (the
                             paper's rule for k > k_max, Section 4.1) */
    int32_t pair_cap;     /* 0 = default.  Capacity of the batched path's list
                             of undecided (user, query) pairs per chunk; pairs
                             beyond it are decided in float64 inside the
                             filter kernel (a test hook for that path) */
    int32_t handoff_tiles; /* 0 = default (512).  Bounded table, batched scan:
                             the last users of a block (or group) still
                             scanning are handed to a group pass of users from
                             several blocks only with more than this many
                             64-item tiles left (a tuning and test hook) */
    int32_t no_blocks;    /* nonzero: no Lemma 3 filter (every block is
                             evaluated: the paper's "Simpfer without blocks",
                             Section 5.2); results are unchanged */
    int32_t verify_tiles; /* 0 = default (2048).  Bounded table, one query:
                             from this many survivors on, the linear scans
                             (Algorithm 2) run 64 survivors per workgroup
                             over shared float32 MFMA item tiles instead of
                             one wave per survivor; < 0: never.  d > 256
                             always uses one wave per survivor.  Results
                             are unchanged (a tuning and test hook) */
    int32_t reserved[2];
} rk_build_opts;

/* Counters and sizes of an index.  Query counters accumulate over every
 * query since the build or the last rk_index_reset_counters(). */
typedef struct {
    int64_t n, m;
    int32_t d, k_max, lb_items, block_size, n_blocks, precision;
    int64_t footprint_bytes;   /* device bytes owned by the index */
    double build_ms;           /* wall time of the last (re)build */
    int64_t build_cand_total;  /* candidates refined in float64 (full table) */
    int64_t build_cand_overflow_users;
    int64_t rebuilds;
    int64_t queries;
    int64_t blocks_visited;    /* (block, query) pairs tested with Lemma 3
                                  (block = block_size users) */
    int64_t blocks_pruned;     /* ... and pruned by it */
    int64_t users_evaluated;   /* u.q computed (users of unpruned blocks) */
    int64_t lemma1_no;         /* certified no by Lemma 1 */
    int64_t lemma2_yes;        /* certified yes by Lemma 2 */
    int64_t table_yes;         /* certified yes by the exact k-th value */
    int64_t survivors;         /* users sent to the linear scan */
    int64_t scan_items;        /* item inner products computed in scans */
    int64_t rechecks;          /* users decided by float64 recomputation */
    int64_t results;           /* total result-set sizes */
    int64_t scan_long;         /* batched scan: pairs whose Corollary 1 limit lies
                                  beyond the short pass (decided by the long pass) */
    int64_t scan_full_f64;     /* pairs decided by the full float64 scan */
    int64_t scan_handoff;      /* batched scan: users handed from their block (or
                                  group) to a group pass of users from several blocks */
    int64_t scan_quarters;     /* batched scan: 32-user x 32-item MFMA products
                                  computed (scan_items / (1024 scan_quarters) is
                                  the share of them that was needed) */
    int64_t scan_valu_tiles;   /* batched scan: item tiles of at most 8 users
                                  computed on the vector ALU */
    int64_t updates;           /* catalog updates (rk_index_add_items/_users) */
    int64_t reserved[2];
} rk_stats;

/* Index fields readable with rk_index_export (sorted = descending norm). */
typedef enum {
    RK_F_PERM_Q = 0,   /* int32 [n]: original user id of sorted position i */
    RK_F_PERM_P = 1,   /* int32 [m]: original item id of sorted position j */
    RK_F_SQNORM_Q = 2, /* double [n], original order: sum x_i^2 (index order) */
    RK_F_SQNORM_P = 3, /* double [m], original order */
    RK_F_NORM_Q = 4,   /* float [n], sorted: norm rounded upward */
    RK_F_NORM_P = 5,   /* float [m], sorted: norm rounded upward */
    RK_F_L64 = 6,      /* double [k_max][n], sorted users: L_i^j exactly */
    RK_F_L32 = 7,      /* float [k_max][n]: L_i^j rounded downward */
    RK_F_LB = 8,       /* float [k_max][n_blocks]: block minima L^j(B) */
    RK_F_BNORM = 9     /* float [n_blocks]: first (largest) norm of a block */
} rk_field;

/* Per-user decision classes written by rk_reverse_kmips_trace. */
typedef enum {
    RK_C_BLOCK_NO = 0,   /* block pruned by Lemma 3 */
    RK_C_LEMMA1_NO = 1,  /* certified no by Lemma 1 */
    RK_C_LEMMA2_YES = 2, /* certified yes by Lemma 2 */
    RK_C_TABLE_YES = 3,  /* certified yes by the exact k-th value */
    RK_C_SCAN_NO = 4,    /* linear scan: k items certified to beat q */
    RK_C_SCAN_YES = 5,   /* linear scan: certified fewer than k */
    RK_C_RECHECK_NO = 6, /* float64 recomputation: no */
    RK_C_RECHECK_YES = 7 /* float64 recomputation: yes */
} rk_class;

void rk_build_opts_default(rk_build_opts *opts);

/* Offline pre-processing, Algorithm 1 (Section 4.1): norms, descending norm
 * sort of Q and P, lower-bound arrays over P' (Definition 4), blocks with
 * their minima (Definition 5, Equation (1)).  Copies Q and P to the device;
 * the index owns every device buffer until rk_index_free.  n = 0 and m = 0
 * are allowed.  opts may be NULL (defaults).  Synchronous. */
rk_status rk_build_index(const float *Q, int64_t n, const float *P, int64_t m,
                         int32_t d, int32_t k_max, const rk_build_opts *opts,
                         rk_index **out);

/* Same, from device pointers (not retained).  Synchronous. */
rk_status rk_build_index_dev(const float *Q_dev, int64_t n, const float *P_dev,
                             int64_t m, int32_t d, int32_t k_max,
                             const rk_build_opts *opts, rk_index **out);

/* One query, Algorithm 3 with Algorithm 2 (Sections 4.2-4.3).  q: host,
 * d floats.  Writes min(count, cap) ascending ids and *count = true size;
 * returns RK_E_TRUNC when count > cap.  k > m returns every user.
 * Synchronous. */
rk_status rk_reverse_kmips(rk_index *idx, const float *q, int32_t k,
                           int32_t *ids, int64_t cap, int64_t *count);

/* One query on device buffers: q_dev (d floats), ids_dev (cap ints),
 * count_dev (one int64, receives the true size; ids beyond cap are dropped).
 * Enqueued on stream; returns without waiting. */
rk_status rk_reverse_kmips_dev(rk_index *idx, const float *q_dev, int32_t k,
                               int32_t *ids_dev, int64_t cap,
                               int64_t *count_dev, void *stream);

/* A batch of nq queries of mixed k.  qs: host [nq][d]; ks: host [nq].
 * Result in CSR form: offsets[nq+1] (host, offsets[0] = 0) and ids (host,
 * cap ints).  Returns RK_E_TRUNC when offsets[nq] > cap (offsets are still
 * complete).  Synchronous. */
rk_status rk_reverse_kmips_batch(rk_index *idx, const float *qs, int64_t nq,
                                 const int32_t *ks, int64_t *offsets,
                                 int32_t *ids, int64_t cap);

/* Batch on device buffers: qs_dev [nq][d], ks_host [nq] (host: validated
 * before anything is enqueued), offsets_dev (nq+1 int64), ids_dev (cap
 * int32; ids beyond cap are dropped while offsets stay exact).  Enqueued on
 * stream; returns without waiting. */
rk_status rk_reverse_kmips_batch_dev(rk_index *idx, const float *qs_dev,
                                     int64_t nq, const int32_t *ks_host,
                                     int64_t *offsets_dev, int32_t *ids_dev,
                                     int64_t cap, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the batch
 * of rk_reverse_kmips_batch_dev, same arguments and results, with no
 * allocation of any kind.  Its workspace (result bitmaps, query tiles,
 * pair slots) is one static 64 MiB device array per GPU, held until the
 * process ends and shared by every call of this function on that GPU: calls
 * that overlap on one GPU (other streams or threads) race and must not be
 * made.  The array keeps the last call's contents; each call clears what
 * must start at zero.  Chunks of queries are sized to fit the array (at
 * least 64 queries per chunk: RK_E_INVAL for an index whose 64-query chunk
 * needs more, i.e. beyond about 7.5 million users).  Exact lower-bound
 * tables only (lb_items 0 or m; RK_E_INVAL otherwise, and for tiles too
 * wide for the batched kernels).  k > k_max (and k <= m) is RK_E_KMAX even
 * with auto_rebuild, since a rebuild allocates.  ks_host is copied to the
 * device with a stream-ordered copy from the caller's memory: keep it
 * unchanged until the stream has passed this call. */
rk_status rk_reverse_kmips_batch_dev_noalloc(rk_index *idx, const float *qs_dev,
                                             int64_t nq, const int32_t *ks_host,
                                             int64_t *offsets_dev, int32_t *ids_dev,
                                             int64_t cap, void *stream);

/* One query with per-user decision classes (rk_class, one byte per user,
 * indexed by original id; users never evaluated keep RK_C_BLOCK_NO) and
 * optionally the bulk-precision u.q (float per original id; NaN where not
 * computed).  shat may be NULL.  Host buffers.  Synchronous. */
rk_status rk_reverse_kmips_trace(rk_index *idx, const float *q, int32_t k,
                                 uint8_t *cls, float *shat);

/* Per-kernel event timing for profiling: with max_launches > 0 every
 * kernel the index launches afterwards is bracketed by two HIP events on the
 * stream it runs on (up to max_launches launches; later ones untimed).
 * rk_index_kernel_times waits for them and returns, per kernel class
 * (0 filter, 1 verify, 2 recheck, 3 finalize, 4 fill-all, 5 batch
 * preparation, 6 batch filter, 7 batch pair decisions, 8 batch assembly),
 * the summed milliseconds and launch counts, then clears the record.
 * 0 turns timing off. */
rk_status rk_index_set_timing(rk_index *idx, int32_t max_launches);
rk_status rk_index_kernel_times(rk_index *idx, double *ms, int64_t *launches,
                                int32_t nclass);

/* Counters are off by default (they cost atomics on the query path). */
rk_status rk_index_set_counting(rk_index *idx, int32_t on);
rk_status rk_index_stats(const rk_index *idx, rk_stats *out);
rk_status rk_index_reset_counters(rk_index *idx);

/* Copy one index field (rk_field) into host memory of `bytes` bytes; the
 * size must match the field exactly. */
rk_status rk_index_export(const rk_index *idx, int32_t field, void *dst,
                          int64_t bytes);

/* Rebuild the lower-bound arrays and blocks with a new k_max from the
 * device-resident sorted copies (Section 4.1, k > k_max).  Synchronous. */
rk_status rk_index_rebuild(rk_index *idx, int32_t k_max);

/* Catalog updates (Section 4.1: the bounds stay valid as the item set grows;
 * new users need their own rows and new blocks).  Synchronous; the index
 * must not be in use (no call in flight on it, and not a catalog of a
 * server: RK_E_INVAL).  Original ids continue the existing ones: new items
 * get ids m, m+1, ...; new users n, n+1, ....
 *
 * rk_index_add_items: P holds m_new items (host, [m_new][d]).  The items are
 * re-sorted by norm.  An exact table (lb_items = m) takes the new items'
 * float64 products into every user's k_max largest values and stays exact
 * (identical to building from scratch on the grown catalog); a bounded
 * table keeps its rows, which remain lower bounds of the grown catalog's
 * k-th largest values (the k-th largest over a subset of the items), and
 * the linear scan of Algorithm 2 covers the new items.
 *
 * rk_index_add_users: Q holds n_new users (host, [n_new][d]).  Their lower-
 * bound rows are computed as in the build (over the same item prefix), the
 * users re-sorted by norm with the existing ones, and the blocks of
 * Definition 5 rebuilt over the grown order: the index equals one built
 * from scratch on the grown user set.
 *
 * Errors: RK_E_INVAL (NULL pointer with a positive count, negative count,
 * non-finite values, a grown size beyond the library's limits, the index
 * held by a server); RK_E_NOMEM / RK_E_DEVICE leave the index unusable (free
 * it). */
rk_status rk_index_add_items(rk_index *idx, const float *P, int64_t m_new);
rk_status rk_index_add_users(rk_index *idx, const float *Q, int64_t n_new);

/* Device bytes an index with these sizes and options would own. */
int64_t rk_index_footprint(int64_t n, int64_t m, int32_t d, int32_t k_max,
                           const rk_build_opts *opts);

void rk_index_free(rk_index *idx);

/* Message of the last error on the calling thread ("" if none). */
const char *rk_last_error(void);

/* ------------------------------------------------------------------------
 * Serving: the online phase (Algorithm 3; Theorem 2 bounds its cost per
 * query) under a stream of single-query requests over several resident
 * catalogs, with continuous batching.  Every catalog has `slots` launch
 * slots; a slot owns a HIP stream, a batch workspace for max_batch queries,
 * query/result buffers and a thread.  A free slot takes whatever the
 * catalog has queued (up to max_batch) and runs it through the batched path
 * of the catalog's index; requests that arrive while that launch is on the
 * device are taken by the next free slot, so their work overlaps on the
 * device with the earlier launch (a small late request can finish before a
 * large earlier batch).  While launches of the catalog are on the device, a
 * free slot joins in only when the first of them to end is expected to run
 * at least twice as long again as the queued requests take alone (moving
 * averages of launch time per batch size), so a launch that ends soon is
 * waited for rather than slowed down by splitting the device.  Results come
 * back to the host per request.  Catalogs run concurrently.
 *
 * Every slot's stream is one of catalogs x slots streams of the process.
 * HIP spreads streams over GPU_MAX_HW_QUEUES hardware queues (4 unless the
 * environment sets it), and the launches of streams that share a queue run
 * in order: a small catalog's launch then waits behind a large catalog's.
 * With one slot per catalog and the default 4 queues, three catalogs
 * (50k, 500k and 2M users) measured p50 0.9-1.3 ms and p99 9-19 ms over
 * all requests; with 8 queues the small catalog's p50 fell to 0.2 ms but
 * the large catalog's p99 rose to 12-36 ms, and with two slots per catalog
 * the catalog whose stream shared a queue with the large catalog's waited
 * behind its launches (p50 2-12 ms).  GPU_MAX_HW_QUEUES is read at the
 * process's first HIP call.
 *
 * Admission by device-memory footprint: a catalog is admitted when its
 * index's bytes plus, per slot, the batch workspace and buffers for
 * max_batch queries fit in what is left of hbm_budget, else RK_E_NOMEM.  A
 * request is admitted when its catalog's queue holds fewer than max_queue
 * requests, else RK_E_BUSY; it needs no device memory of its own beyond its
 * slot's, except when its batch's ids outgrow the slot's id buffer: the
 * buffer grows within the budget, and when the budget does not allow it
 * the batch runs in halves (a single result that cannot fit completes with
 * status RK_E_NOMEM).
 *
 * A catalog's index is borrowed: it must outlive the server, and nothing
 * else may query it while the server runs.  Requests for different catalogs
 * never share a launch, and a request's result set does not depend on what
 * it was batched with.  All functions are thread-safe.
 * ---------------------------------------------------------------------- */
typedef struct rk_server rk_server;

typedef struct {
    int32_t device;       /* HIP device of the catalogs */
    int32_t max_batch;    /* 0 -> 1024: queries per launch (per catalog) */
    int32_t max_wait_us;  /* 0: launch as soon as the device is free;
                             > 0: a batch smaller than max_batch may wait up
                             to this long after its oldest request arrived */
    int32_t slots;        /* 0 -> 1: launches in flight per catalog (1..16); an
                             index whose batches run one query at a time
                             (tiles too wide for the batched kernels) gets 1.
                             More than one pays where a catalog's launches
                             run for tens of milliseconds (a late request
                             overlaps them); with several catalogs their
                             extra streams share hardware queues (see above) */
    int64_t hbm_budget;   /* 0 -> 90% of the device memory free at creation */
    int64_t max_queue;    /* 0 -> 65536: queued requests per catalog */
    int64_t reserved[5];
} rk_server_opts;

typedef struct {
    int64_t tag;          /* the caller's tag from rk_server_submit */
    int32_t catalog;
    int32_t status;       /* rk_status of the query */
    int64_t count;        /* result size (ascending original user ids) */
    int64_t ids_offset;   /* first id in the buffer passed to rk_server_poll */
    double submit_ms;     /* server clock, ms since rk_server_create */
    double done_ms;       /* result on the host */
} rk_completion;

void rk_server_opts_default(rk_server_opts *o);
rk_status rk_server_create(const rk_server_opts *opts, rk_server **out);

/* Admit a built index as a catalog; *catalog receives its number (0, 1, ...).
 * The index's batch workspace for max_batch queries is allocated here. */
rk_status rk_server_add_catalog(rk_server *s, rk_index *idx, int32_t *catalog);

/* Queue one query (host vector of the catalog's d floats, copied) at k.
 * RK_E_INVAL: bad catalog, k < 1 or a non-finite value; RK_E_KMAX: k >
 * k_max (no rebuild while serving); RK_E_BUSY: the catalog's queue already
 * holds max_queue requests (nothing is queued; retry later). */
rk_status rk_server_submit(rk_server *s, int32_t catalog, const float *q, int32_t k,
                           int64_t tag);

/* Queue n queries at once, with the checks of rk_server_submit (all or
 * nothing; RK_E_BUSY when some catalog's queue has no room for its share).  q[i] points to the d floats of query i's catalog.  arrival_ms
 * (or NULL: now) is each request's arrival on the server clock, the time its
 * latency counts from: an open-loop load generator that submits late passes
 * the scheduled times (later than now counts as now). */
rk_status rk_server_submit_many(rk_server *s, int64_t n, const int32_t *catalog,
                                const float *const *q, const int32_t *k, const int64_t *tag,
                                const double *arrival_ms);

/* The server clock: ms since rk_server_create. */
double rk_server_now_ms(rk_server *s);

/* Move up to max_out finished requests out of the server, oldest first:
 * their records to out[], their ids one after another into ids[0..ids_cap).
 * Waits up to wait_us microseconds for a first one when none is finished.
 * Returns the number of records written (0 if none finished), or -1 when
 * the next finished request alone has more ids than ids_cap (it stays in
 * the server; the message gives its size). */
int64_t rk_server_poll(rk_server *s, rk_completion *out, int64_t max_out, int32_t *ids,
                       int64_t ids_cap, int32_t wait_us);

/* Requests submitted and not yet finished. */
int64_t rk_server_inflight(rk_server *s);

/* A catalog's queued requests (not yet taken by a slot) and its slots with
 * a launch in flight. */
rk_status rk_server_catalog_state(rk_server *s, int32_t catalog, int64_t *queued,
                                  int32_t *running);

/* Device bytes held by the admitted catalogs (indices, workspaces, buffers). */
int64_t rk_server_used_bytes(rk_server *s);

/* Finish the queued requests, stop the slots, release the server's own
 * buffers (not the indices).  Unpolled results are dropped. */
void rk_server_free(rk_server *s);

#ifdef __cplusplus
}
#endif
#endif /* RKMIPS_H */
