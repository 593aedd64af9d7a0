// Launchers of the join kernels (join.hip).
#pragma once

#include "apss_internal.h"

namespace apss {

struct JoinArgs {
  // corpus index
  const int64_t* rp;      // [n+1] row offsets of the rank-space rows
  const RComp* rc;        // [nnz] components, densest dimension first
  const RowStat* rs;      // [n]
  const int64_t* off;     // [m+1] list offsets by rank
  const Post* post;       // [P]   list entries, vector ids ascending within a list
  const uint32_t* post4;  // [P]   the same entries packed: id mod 2^16 | half weight (rounded up) << 16
  const uint32_t* hoff;   // [(nb+1) * H] first entry of list r at or after block b
  int32_t H;              // ranks with block offsets
  int64_t nb;             // corpus blocks
  int64_t n;              // corpus vectors
  // queries (rank space, densest dimension first)
  const int64_t* qrp;     // [nq+1]
  const RComp* qrc;       // [qnnz]
  const float* qmw;       // [nq] maxweight(q)
  const float* qt;        // [nq] per-query threshold, or NULL
  float t;                // threshold when qt is NULL
  int64_t nq;
  int32_t triangle;       // 1: self-join, query q only meets corpus rows y < q
  uint32_t* cur_pos;      // [qnnz] list cursors of tiles too large to stage in LDS
  uint32_t* cur_ny;       // [qnnz] vector id at each such cursor
  int64_t ntiles;
  // output
  uint64_t* out_key;      // [cap] (i << bj) | j
  float* out_sim;         // [cap]
  int64_t cap;
  int32_t bj;
  unsigned long long* counters;  // [C_NUM]
};

// Compiled tile variants of the join kernel.
int join_num_variants();
int join_variant_geometry(int variant, int* queries_per_tile, int* block_rows);
hipError_t launch_join(const JoinArgs& a, int variant, hipStream_t s);
hipError_t launch_unpack_pairs(const uint64_t* keys, const float* sim, int64_t cnt, int bj, uint32_t* oi,
                               uint32_t* oj, float* os, hipStream_t s);

}  // namespace apss
