// Launchers of the index builder kernels (index_build.hip).
#pragma once

#include "apss_internal.h"

namespace apss {

enum ErrBits : uint32_t {
  ERR_ROWPTR = 1u,   // row_ptr not monotone or not spanning [0, nnz]
  ERR_DIM = 2u,      // dimension id outside [0, m)
  ERR_WEIGHT = 4u,   // weight not finite or not > 0
  ERR_NORM = 8u,     // |norm - 1| above tolerance
  ERR_DUP = 16u,     // repeated dimension inside a row
};

hipError_t launch_check_rowptr(const int64_t* rp, int64_t n, int64_t nnz, uint32_t* err, unsigned long long* bad,
                               hipStream_t s);
hipError_t launch_validate_rows(const int64_t* rp, const int32_t* col, const float* val, int64_t n, int64_t m,
                                double tol, uint32_t* err, unsigned long long* bad, hipStream_t s);
hipError_t launch_count_dims(const int32_t* col, const float* val, int64_t nnz, uint32_t* cnt, uint32_t* mwbits,
                             hipStream_t s);
hipError_t launch_dim_keys(const uint32_t* cnt, int64_t m, int64_t n, int dbits, uint64_t* keys, uint64_t* vals,
                           hipStream_t s);
hipError_t launch_rank_from_sorted(const uint64_t* vals, int64_t m, const uint32_t* cnt, const uint32_t* mwbits,
                                   int32_t* rank, int32_t* inv, float* mw_r, uint32_t* cnt_r, hipStream_t s);
hipError_t launch_row_keys(const int64_t* rp, const int32_t* col, const float* val, const int32_t* rank, int64_t n,
                           int rbits, uint64_t* keys, uint32_t* vals, hipStream_t s);
hipError_t launch_unpack_rows(const uint64_t* keys, const uint32_t* vals, int64_t nnz, int rbits, RComp* rc,
                              uint32_t* err, hipStream_t s);
// head >= 0: the unindexed part of every row is its components of rank < head (t and l2 unused;
// head = 0 indexes every component); head < 0: the running-bound cutoff at t
hipError_t launch_cutoff(const int64_t* rp, const RComp* rc, const float* mw_r, int64_t n, float t, int l2,
                         int32_t head, RowStat* rs, float* xmw, int64_t* nidx, hipStream_t s);
hipError_t launch_emit_indexed(const int64_t* rp, const RComp* rc, const RowStat* rs, const int64_t* ibase, int64_t n,
                               uint64_t* keys, uint64_t* vals, hipStream_t s);
hipError_t launch_count_ranks(const uint64_t* keys, int64_t P, int64_t* cnt, hipStream_t s);
hipError_t launch_unpack_post(const uint64_t* vals, int64_t P, Post* post, hipStream_t s);
// *out = max over rows of rs[r].pnrm as float bits (atomicMax; *out zeroed before)
hipError_t launch_max_pnrm(const RowStat* rs, int64_t n, uint32_t* out, uint8_t* pn8, hipStream_t s);
hipError_t launch_pack_post4(const Post* post, int64_t P, uint32_t* post4, hipStream_t s);
hipError_t launch_block_offsets(const int64_t* off, const Post* post, int32_t H, int64_t nb, int32_t CB,
                                uint32_t* hoff, hipStream_t s);
hipError_t launch_query_keys(const int64_t* rp, const int32_t* col, const float* val, const int32_t* rank, int64_t nq,
                             int64_t m, int rbits, double tol, uint64_t* keys, uint32_t* vals, float* qmw,
                             uint32_t* err, unsigned long long* bad, hipStream_t s);

}  // namespace apss
