// Launchers of the join kernels (join.hip).
#pragma once

#include "apss_internal.h"

namespace apss {

// zero entries after the last list of the packed list array: a list chunk's
// lanes past its end stay inside the allocation
constexpr int64_t kPost4Pad = 64;

struct JoinArgs {
  // corpus index
  const int64_t* rp;      // [n+1] row offsets of the rank-space rows
  const RComp* rc;        // [nnz] components, densest dimension first
  const RowStat* rs;      // [n]
  float pnrm_max;         // max over rows of rs[y].pnrm
  const uint8_t* pn8;     // [n] rs[y].pnrm as a byte code (kPn8None: no bound; else pnrm <= code / 254)
  const int64_t* off;     // [m+1] list offsets by rank
  const Post* post;       // [P+2] list entries, vector ids ascending within a list; 2 padding entries
  const uint32_t* post4;  // [P+kPost4Pad] the same entries packed: id mod 2^16 | weight in 2^-15 units (rounded up) << 16
  uint32_t post4_bytes;   // size of post4 in bytes (< 2^32)
  const uint32_t* hoff;   // [(nb+1) * H] first entry of list r at or after block b
  int32_t H;              // ranks with block offsets
  int64_t nb;             // corpus blocks
  int64_t n;              // corpus vectors
  // queries (rank space, densest dimension first)
  const int64_t* qrp;     // [nq+1]
  const RComp* qrc;       // [qnnz]
  const float* qmw;       // [nq] maxweight(q)
  const RowStat* qrs;     // [nq] or NULL: when every corpus row's unindexed part is exactly its
                          // components of rank < some head size, qrs[q].pnrm bounds the norm of
                          // q's own head part (used in the L2 bound); NULL means 1
  const float* qt;        // [nq] per-query threshold, or NULL
  float t;                // threshold when qt is NULL
  int64_t nq;
  int32_t triangle;       // 1: self-join, query q only meets corpus rows y < q
  int64_t ntiles;
  const int64_t* tstart;  // [ntiles+1] first query of each tile (tiles hold <= QT queries)
  // work items (group of rg consecutive corpus ranges of K blocks each,
  // query tile), queued per XCD
  const uint32_t* toff;   // [(nR+1) * m_tail] first entry of sparse list H + rt at or after range R
  int32_t m_tail;         // m - H
  int32_t K;              // blocks per range
  int32_t rg;             // ranges per item (>= 1)
  int32_t nR;             // corpus ranges
  int64_t nrx;            // group slots per XCD queue
  const int64_t* qcum;    // [8 * (nrx+1)] cumulative item counts of queue x's groups x, x+8, ...
  unsigned int* qctr;     // [8] next item of each queue (zero at launch)
  uint32_t* wg_cur;       // per-workgroup cursors of tiles too large to stage in LDS
  int64_t wg_cur_stride;  // 2 * largest tile's component count
  // local pruning (Lemma 1): parts > 1 splits every (range, tile) item into
  // parts items, item part r scoring the indexed ranks [part_lo[r],
  // part_lo[r + 1]) against the local threshold; survivors are decided on
  // their exact full score, so a pair can be emitted by several parts
  int32_t parts;          // 1: off
  const int32_t* part_lo; // [parts + 1] rank bounds (device), or NULL when parts == 1
  // remscore: qadm[q] = position of query q's first component that admits
  // new candidates (components before it, the densest ones, only add to
  // candidates admitted by a later one); NULL: off
  const int32_t* qadm;
  // output
  uint64_t* out_key;      // [cap] (i << bj) | j
  float* out_sim;         // [cap]
  int64_t cap;
  int32_t bj;
  unsigned long long* counters;  // [C_NUM]
};

// True when every device buffer the join kernel dereferences is present.
inline bool join_args_complete(const JoinArgs& a) {
  return a.rp && a.rc && a.rs && a.pn8 && a.off && a.post && a.post4 && a.hoff && a.qrp && a.qrc && a.qmw && a.toff && a.tstart &&
         a.qcum && a.qctr && a.wg_cur && a.out_key && a.out_sim && a.counters;
}

// Compiled tile variants of the join kernel.
int join_num_variants();
int join_variant_geometry(int variant, int* queries_per_tile, int* block_rows);
// Components of one tile that the variant stages in LDS.
int join_variant_staging(int variant);
hipError_t launch_join(const JoinArgs& a, int variant, int grid, hipStream_t s);
// Workgroups of a variant (with or without the remscore rule) that fit on the device at once.
int join_resident_groups(int variant, bool remscore = false);
// qadm[q] = position of the first component of query row q (rank space,
// densest first) at which sum_{i <= k} q_i * maxweight_{r_i}(V) reaches its
// threshold (qt[q], or t when qt is NULL); the row length if it never does.
hipError_t launch_admit_pos(const int64_t* qrp, const RComp* qrc, const float* mw_r, const float* qt, float t,
                            int64_t nq, int32_t* qadm, hipStream_t s);
hipError_t launch_range_offsets(const int64_t* off, const Post* post, int32_t H, int64_t m, int64_t nR,
                                int64_t range_rows, uint32_t* toff, hipStream_t s);
hipError_t launch_max_tile_nnz(const int64_t* qrp, int64_t nq, int qt, unsigned long long* out, hipStream_t s);
hipError_t launch_unpack_pairs(const uint64_t* keys, const float* sim, int64_t cnt, int bj, uint32_t* oi,
                               uint32_t* oj, float* os, hipStream_t s);

}  // namespace apss
