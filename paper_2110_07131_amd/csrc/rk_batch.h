// Batched query path: device workspace view and launch wrappers.
#pragma once
#include "rk_common.h"

namespace rk {


struct BatchView {
  const float* qs;              // chunk queries [nq][d], caller order
  float* qn;                    // [nq] |q| rounded up, caller order
  int32_t* perm;                // [nq] sorted position -> caller-order index
  float* qt;                    // sorted query tiles, fp32 [T][d][64]
  uint16_t* qb;                 // sorted query tiles, bf16 [T][G][64][8]
  float* qn_s;                  // [nq_pad] sorted norms
  int32_t* k_s;                 // [nq_pad] sorted k (0 = padding or no work)
  int32_t* kofs_s;              // [nq_pad] 64 (max(k,1) - 1): the k's row of the filter's (k, user) tables
  int32_t* tsum;                // [nq_pad / 64][2][4] per tile and query half: largest norm (bits),
                                // smallest and largest k row, first row of the largest k (-1: > 2 k's)
  int32_t nq_pad;
  int32_t qsplit;               // filter: query-tile parts per user block (one workgroup each;
                                // set by launch_bfilter)
  uint32_t* bits;               // [nq][W] result bits by original user id
  int64_t W;                    // words per bitmap row
  unsigned long long* counts;   // [nq] result sizes, caller order
  uint8_t* all;                 // [nq] 1 if k > m (every user is a member)
  int64_t n;                    // users
  unsigned long long* npairs;   // exact table: pair slots reserved (may exceed cap;
                                // 64-bit: a chunk can reserve more than 2^31)
  int32_t pair_cap;
  int32_t* pair_u;              // sorted user index
  int32_t* pair_j;              // sorted query position
  float* pair_s;                // bulk-precision u.q
  // Bounded table only: the pair slots are grouped in chunks of kPairChunk;
  // every chunk holds pairs of one user block, listed per block.
  int32_t* pair_st;             // 1 = left for the scan's long pass
  int32_t* cfill;               // [chunk_cap] used slots per chunk
  int32_t* nchunks;             // chunks handed out (may exceed chunk_cap)
  int32_t chunk_cap;
  int32_t maxc;                 // list capacity per block
  int32_t* bcnt;                // [nB] chunks of the filter's pairs per block
  int32_t* bchunks;             // [nB][maxc] their ids
  // Per-user scan state carried across the chunks of one batch call: the
  // largest approximate products of the items [0, gdone[u]) (descending,
  // with item ids), bscan_list_len(k_max) entries per user.
  float* gl_v;
  int32_t* gl_i;
  int32_t* gdone;               // [n_pad] items covered (a multiple of 64); 0 at a call's start
  int32_t carry_in;             // 1: the lists hold the previous chunks' state
  int32_t carry_out;            // 1: later chunks follow (store the lists)
  int32_t prescan;              // 1: the scan's first pass over the item prefix for every
                                // user block, before the call's first chunk (no pairs)
  int32_t lists;                // 1: the filter tightens the lower bounds with the lists
  // Users still scanning when at most a few of their block are, handed to
  // passes that scan them in groups of 64 from several blocks (a group pass
  // hands its own last users to the next): the users of two alternating
  // lists, a flag per block that handed any over, and each user's pair slots
  // (count, k, lower and upper bound of f(q,u)); their lists and covered
  // lengths are in gl_v, gl_i and gdone.
  int32_t* sg_count;            // [2] users in each list
  int32_t* sg_users;            // [2][n_pad] their sorted indices
  int32_t sg_level;             // group pass: reads list sg_level & 1, hands over to the other
  int32_t sg_last;              // group pass: 1 = the last, scans to the end
  int32_t* sg_block;            // [nB]
  int32_t* sg_key;              // [n_pad] item tile of the deepest Corollary 1 limit of a handed user's open pairs
  int32_t* sg_sorted;           // [n_pad] the current list ordered by that key (the group pass reads it)
  int32_t* st_np;               // [n_pad]
  int32_t* st_pk;               // [n_pad][kUserPairs]
  float* st_plo;                // [n_pad][kUserPairs]
  float* st_ph;                 // [n_pad][kUserPairs]
  unsigned long long* ctr;      // statistics or nullptr
};

void launch_bprep(const DevIndex& ix, const BatchView& bv, const int32_t* ks_dev, int32_t nq,
                  hipStream_t s);
size_t bfilter_lds_bytes(const DevIndex& ix);
size_t bfilter_max_tile_bytes();
void launch_bfilter(const DevIndex& ix, const BatchView& bv, hipStream_t s);
void launch_bpairs(const DevIndex& ix, const BatchView& bv, hipStream_t s);
// Bounded table: the grouped linear scan of the chunk's pairs (scan_kernels.hip).
void launch_bscan(const DevIndex& ix, const BatchView& bv, hipStream_t s);
// Bounded table: the scan's first pass (the first kShortTiles item tiles)
// for every user block, leaving each user's list in gl_v/gl_i/gdone.
void launch_bprescan(const DevIndex& ix, const BatchView& bv, hipStream_t s);
// Dynamic LDS of the grouped linear scan (bounded table).
size_t bscan_lds_bytes(const DevIndex& ix);
// whether the scan's workgroup (dynamic and static LDS) fits a CU
bool bscan_fits(const DevIndex& ix);
// p[0..n) = v (a fill kernel: stream-ordered, and capturable in a graph).
void launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
// Bounded table: the carried scan state starts empty for a batch call.
void launch_bscan_reset(const DevIndex& ix, const BatchView& bv, hipStream_t s);
// offs[0] must hold the chunk's first offset; writes offs[1..nq] and ids.
void launch_bassemble(const BatchView& bv, int32_t nq, const int64_t* base, int64_t* offs,
                      int32_t* ids, int64_t cap, hipStream_t s);

}  // namespace rk
