// Index builder kernels (partial indexing, Section 3.2.2).
//
//  k_check_rowptr / k_validate_rows   input checks of Section 2.1
//  k_count_dims                       non-zero count and maxweight_d(V) per dimension
//  k_dim_keys / k_rank_from_sorted    density order: decreasing count, ties by id
//  k_row_keys / k_unpack_rows         every row's components re-ordered densest first
//  k_cutoff                           running bound b = sum x[d] maxweight_d(V) in double;
//                                     the leading components with b < t are x' (or, for
//                                     the head-cut index of the screened join, the
//                                     components of rank < head)
//  k_count_indexed / k_emit_indexed   inverted lists of the indexed parts, by vector id
//  k_block_offsets                    where each dense list enters each corpus block
#include "apss_internal.h"
#include "index_build.h"

namespace apss {

namespace {

__global__ void k_check_rowptr(const int64_t* __restrict__ rp, int64_t n, int64_t nnz, uint32_t* __restrict__ err,
                               unsigned long long* __restrict__ bad_row) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r <= n; r += (int64_t)gridDim.x * blockDim.x) {
    bool bad = false;
    if (r == 0 && rp[0] != 0) bad = true;
    if (r == n && rp[n] != nnz) bad = true;
    if (r < n && rp[r + 1] < rp[r]) bad = true;
    if (bad) {
      atomicOr(err, ERR_ROWPTR);
      atomicMin(bad_row, (unsigned long long)r);
    }
  }
}

// One thread per row: dimension range, positive finite weights, unit norm.
__global__ void k_validate_rows(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                const float* __restrict__ val, int64_t n, int64_t m, double norm_tol,
                                uint32_t* __restrict__ err, unsigned long long* __restrict__ bad_row) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a = rp[r], b = rp[r + 1];
    uint32_t e = 0;
    double ss = 0.0;
    for (int64_t k = a; k < b; ++k) {
      const int32_t d = col[k];
      const float w = val[k];
      if (d < 0 || (int64_t)d >= m) e |= ERR_DIM;
      if (!(w > 0.0f) || !isfinite(w)) e |= ERR_WEIGHT;
      ss += (double)w * (double)w;
    }
    if (b > a && !(fabs(sqrt(ss) - 1.0) <= norm_tol)) e |= ERR_NORM;
    if (e) {
      atomicOr(err, e);
      atomicMin(bad_row, (unsigned long long)r);
    }
  }
}

__global__ void k_count_dims(const int32_t* __restrict__ col, const float* __restrict__ val, int64_t nnz,
                             uint32_t* __restrict__ cnt, uint32_t* __restrict__ mwbits) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nnz; k += (int64_t)gridDim.x * blockDim.x) {
    const int32_t d = col[k];
    atomicAdd(&cnt[d], 1u);
    // weights are positive floats, whose bit patterns order like the values
    atomicMax(&mwbits[d], __float_as_uint(val[k]));
  }
}

__global__ void k_dim_keys(const uint32_t* __restrict__ cnt, int64_t m, int64_t n, int dbits, uint64_t* __restrict__ keys,
                           uint64_t* __restrict__ vals) {
  for (int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; d < m; d += (int64_t)gridDim.x * blockDim.x) {
    keys[d] = ((uint64_t)(n - (int64_t)cnt[d]) << dbits) | (uint64_t)d;
    vals[d] = (uint64_t)d;
  }
}

__global__ void k_rank_from_sorted(const uint64_t* __restrict__ vals, int64_t m, const uint32_t* __restrict__ cnt,
                                   const uint32_t* __restrict__ mwbits, int32_t* __restrict__ rank,
                                   int32_t* __restrict__ inv, float* __restrict__ mw_by_rank,
                                   uint32_t* __restrict__ cnt_by_rank) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < m; r += (int64_t)gridDim.x * blockDim.x) {
    const int32_t d = (int32_t)vals[r];
    rank[d] = (int32_t)r;
    inv[r] = d;
    mw_by_rank[r] = __uint_as_float(mwbits[d]);
    cnt_by_rank[r] = cnt[d];
  }
}

// One thread per row: keys (row, rank) for every component, values = weight bits.
__global__ void k_row_keys(const int64_t* __restrict__ rp, const int32_t* __restrict__ col, const float* __restrict__ val,
                           const int32_t* __restrict__ rank, int64_t n, int rbits, uint64_t* __restrict__ keys,
                           uint32_t* __restrict__ vals) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
    for (int64_t k = rp[r]; k < rp[r + 1]; ++k) {
      keys[k] = ((uint64_t)r << rbits) | (uint64_t)rank[col[k]];
      vals[k] = __float_as_uint(val[k]);
    }
  }
}

__global__ void k_unpack_rows(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ vals, int64_t nnz,
                              int rbits, RComp* __restrict__ rc, uint32_t* __restrict__ err) {
  const uint64_t rmask = (1ull << rbits) - 1;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nnz; k += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t key = keys[k];
    RComp c;
    c.r = (int32_t)(key & rmask);
    c.w = __uint_as_float(vals[k]);
    rc[k] = c;
    if (k > 0 && keys[k - 1] == key) atomicOr(err, ERR_DUP);
  }
}

// Partial indexing cutoff, one thread per row, in double in the order of the
// components (densest dimension first).  A component is indexed as soon as
// the running bound including it reaches t; with l2 the unindexed part also
// ends once its own squared norm reaches t^2 (exact for float t).
__global__ void k_cutoff(const int64_t* __restrict__ rp, const RComp* __restrict__ rc, const float* __restrict__ mw_r,
                         int64_t n, float t, int l2, int32_t head, RowStat* __restrict__ rs, float* __restrict__ xmw,
                         int64_t* __restrict__ nidx) {
  const double td = (double)t;
  const double t2 = td * td;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a = rp[r];
    const int32_t len = (int32_t)(rp[r + 1] - a);
    double b = 0.0, sq = 0.0, sqp = 0.0;
    int32_t cut = len;
    float pm = 0.0f, xm = 0.0f;
    for (int32_t k = 0; k < len; ++k) {
      const RComp c = rc[a + k];
      const double w = (double)c.w;
      bool stop;
      if (head >= 0) {
        // head cut: the unindexed part is the head (with head = 0 it is
        // empty and every component is indexed)
        stop = c.r >= head;
        sq += w * w;
      } else {
        b += w * (double)mw_r[c.r];
        sq += w * w;
        stop = b >= td || (l2 && sq >= t2);
      }
      if (stop) {
        cut = k;
        break;
      }
      sqp = sq;
      pm = fmaxf(pm, c.w);
    }
    for (int32_t k = 0; k < len; ++k) xm = fmaxf(xm, rc[a + k].w);
    RowStat s;
    s.cut = cut;
    s.len = len;
    s.pmw = pm;
    // ||x'||_2 rounded up, with a relative nudge covering the double sqrt's rounding
    s.pnrm = sqp > 0.0 ? __double2float_ru(sqrt(sqp) * (1.0 + 0x1p-50)) : 0.0f;
    rs[r] = s;
    xmw[r] = xm;
    nidx[r] = (int64_t)(len - cut);
  }
}

// Largest unindexed-part norm over the rows (norms are >= 0, so their bit
// patterns order like the values), and each row's norm as a one-byte upper
// bound: the smallest k with pnrm <= k / 254 (in double), or kPn8None.
__global__ void k_max_pnrm(const RowStat* __restrict__ rs, int64_t n, uint32_t* __restrict__ out,
                           uint8_t* __restrict__ pn8) {
  uint32_t m = 0u;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
    const float p = rs[r].pnrm;
    m = max(m, __float_as_uint(p));
    const double k = ceil((double)p * 254.0);
    pn8[r] = k <= 254.0 ? (uint8_t)k : kPn8None;
  }
  if (m) atomicMax(out, m);
}

// Indexed components in row-major order -> (key = rank, value = y << 32 | weight bits).
__global__ void k_emit_indexed(const int64_t* __restrict__ rp, const RComp* __restrict__ rc,
                               const RowStat* __restrict__ rs, const int64_t* __restrict__ ibase, int64_t n,
                               uint64_t* __restrict__ keys, uint64_t* __restrict__ vals) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a = rp[r], b = rp[r + 1];
    int64_t o = ibase[r];
    for (int64_t k = a + rs[r].cut; k < b; ++k, ++o) {
      const RComp c = rc[k];
      keys[o] = (uint64_t)(uint32_t)c.r;
      vals[o] = ((uint64_t)(uint32_t)r << 32) | (uint64_t)__float_as_uint(c.w);
    }
  }
}

__global__ void k_count_ranks(const uint64_t* __restrict__ keys, int64_t P, int64_t* __restrict__ cnt) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < P; k += (int64_t)gridDim.x * blockDim.x)
    atomicAdd((unsigned long long*)&cnt[keys[k]], 1ull);
}

__global__ void k_unpack_post(const uint64_t* __restrict__ vals, int64_t P, Post* __restrict__ post) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < P; k += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t v = vals[k];
    Post p;
    p.y = (uint32_t)(v >> 32);
    p.w = __uint_as_float((uint32_t)v);
    post[k] = p;
  }
}

// Packed copy of the list entries for streaming: low 16 bits = vector id mod
// 2^16 (its offset inside any power-of-two block), high 16 bits = the weight
// in units of 2^-15 rounded up (w * 2^15 is exact in float, so the ceiling is
// the smallest such unit count not below w).
__global__ void k_pack_post4(const Post* __restrict__ post, int64_t P, uint32_t* __restrict__ post4) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < P; k += (int64_t)gridDim.x * blockDim.x) {
    const Post p = post[k];
    uint32_t w15 = (uint32_t)ceilf(p.w * 32768.0f);
    if (w15 > 0xFFFFu) w15 = 0xFFFFu;
    post4[k] = (p.y & 0xFFFFu) | (w15 << 16);
  }
}

// hoff[b * H + r] = first position in list r whose vector id is >= b * CB.
__global__ void k_block_offsets(const int64_t* __restrict__ off, const Post* __restrict__ post, int32_t H, int64_t nb,
                                int32_t CB, uint32_t* __restrict__ hoff) {
  const int64_t total = (nb + 1) * (int64_t)H;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = e / H;
    const int32_t r = (int32_t)(e - b * H);
    int64_t lo = off[r], hi = off[r + 1];
    const uint64_t y0 = (uint64_t)b * (uint64_t)CB;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if ((uint64_t)post[mid].y < y0) lo = mid + 1;
      else hi = mid;
    }
    hoff[e] = (uint32_t)lo;
  }
}

// Query rows: dimension ids -> ranks (keys (row, rank)), with input checks.
// One wave per row: lanes over its components (coalesced), then the row's
// squared norm, maxweight and error flags reduced across the wave in a
// fixed order.
__global__ void k_query_keys(const int64_t* __restrict__ rp, const int32_t* __restrict__ col, const float* __restrict__ val,
                             const int32_t* __restrict__ rank, int64_t nq, int64_t m, int rbits, double norm_tol,
                             uint64_t* __restrict__ keys, uint32_t* __restrict__ vals, float* __restrict__ qmw,
                             uint32_t* __restrict__ err, unsigned long long* __restrict__ bad_row) {
  const int lane = (int)(threadIdx.x & 63u);
  const int64_t wpb = (int64_t)(blockDim.x >> 6);
  for (int64_t r = (int64_t)blockIdx.x * wpb + (int64_t)(threadIdx.x >> 6); r < nq; r += (int64_t)gridDim.x * wpb) {
    const int64_t a = rp[r], b = rp[r + 1];
    uint32_t e = 0;
    double ss = 0.0;
    float mx = 0.0f;
    for (int64_t k = a + lane; k < b; k += 64) {
      const int32_t d = col[k];
      const float w = val[k];
      if (d < 0 || (int64_t)d >= m) {
        e |= ERR_DIM;
        keys[k] = ((uint64_t)r << rbits);
      } else {
        keys[k] = ((uint64_t)r << rbits) | (uint64_t)rank[d];
      }
      if (!(w > 0.0f) || !isfinite(w)) e |= ERR_WEIGHT;
      ss += (double)w * (double)w;
      mx = fmaxf(mx, w);
      vals[k] = __float_as_uint(w);
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      ss += __shfl_xor(ss, o, 64);
      mx = fmaxf(mx, __shfl_xor(mx, o, 64));
      e |= __shfl_xor(e, o, 64);
    }
    if (lane == 0) {
      if (b > a && !(fabs(sqrt(ss) - 1.0) <= norm_tol)) e |= ERR_NORM;
      qmw[r] = mx;
      if (e) {
        atomicOr(err, e);
        atomicMin(bad_row, (unsigned long long)r);
      }
    }
  }
}

unsigned grid(int64_t n, int threads = 256) {
  int64_t g = (n + threads - 1) / threads;
  if (g > 32768) g = 32768;
  if (g < 1) g = 1;
  return (unsigned)g;
}

}  // namespace

#define LAUNCH(k, n, ...)                                                 \
  do {                                                                    \
    hipLaunchKernelGGL(k, dim3(grid(n)), dim3(256), 0, s, __VA_ARGS__);   \
    hipError_t e_ = hipGetLastError();                                    \
    if (e_ != hipSuccess) return e_;                                      \
  } while (0)

hipError_t launch_check_rowptr(const int64_t* rp, int64_t n, int64_t nnz, uint32_t* err, unsigned long long* bad,
                               hipStream_t s) {
  LAUNCH(k_check_rowptr, n + 1, rp, n, nnz, err, bad);
  return hipSuccess;
}

hipError_t launch_validate_rows(const int64_t* rp, const int32_t* col, const float* val, int64_t n, int64_t m,
                                double tol, uint32_t* err, unsigned long long* bad, hipStream_t s) {
  LAUNCH(k_validate_rows, n, rp, col, val, n, m, tol, err, bad);
  return hipSuccess;
}

hipError_t launch_count_dims(const int32_t* col, const float* val, int64_t nnz, uint32_t* cnt, uint32_t* mwbits,
                             hipStream_t s) {
  LAUNCH(k_count_dims, nnz, col, val, nnz, cnt, mwbits);
  return hipSuccess;
}

hipError_t launch_dim_keys(const uint32_t* cnt, int64_t m, int64_t n, int dbits, uint64_t* keys, uint64_t* vals,
                           hipStream_t s) {
  LAUNCH(k_dim_keys, m, cnt, m, n, dbits, keys, vals);
  return hipSuccess;
}

hipError_t launch_rank_from_sorted(const uint64_t* vals, int64_t m, const uint32_t* cnt, const uint32_t* mwbits,
                                   int32_t* rank, int32_t* inv, float* mw_r, uint32_t* cnt_r, hipStream_t s) {
  LAUNCH(k_rank_from_sorted, m, vals, m, cnt, mwbits, rank, inv, mw_r, cnt_r);
  return hipSuccess;
}

hipError_t launch_row_keys(const int64_t* rp, const int32_t* col, const float* val, const int32_t* rank, int64_t n,
                           int rbits, uint64_t* keys, uint32_t* vals, hipStream_t s) {
  LAUNCH(k_row_keys, n, rp, col, val, rank, n, rbits, keys, vals);
  return hipSuccess;
}

hipError_t launch_unpack_rows(const uint64_t* keys, const uint32_t* vals, int64_t nnz, int rbits, RComp* rc,
                              uint32_t* err, hipStream_t s) {
  LAUNCH(k_unpack_rows, nnz, keys, vals, nnz, rbits, rc, err);
  return hipSuccess;
}

hipError_t launch_cutoff(const int64_t* rp, const RComp* rc, const float* mw_r, int64_t n, float t, int l2,
                         int32_t head, RowStat* rs, float* xmw, int64_t* nidx, hipStream_t s) {
  LAUNCH(k_cutoff, n, rp, rc, mw_r, n, t, l2, head, rs, xmw, nidx);
  return hipSuccess;
}

hipError_t launch_emit_indexed(const int64_t* rp, const RComp* rc, const RowStat* rs, const int64_t* ibase, int64_t n,
                               uint64_t* keys, uint64_t* vals, hipStream_t s) {
  LAUNCH(k_emit_indexed, n, rp, rc, rs, ibase, n, keys, vals);
  return hipSuccess;
}

hipError_t launch_count_ranks(const uint64_t* keys, int64_t P, int64_t* cnt, hipStream_t s) {
  LAUNCH(k_count_ranks, P, keys, P, cnt);
  return hipSuccess;
}

hipError_t launch_unpack_post(const uint64_t* vals, int64_t P, Post* post, hipStream_t s) {
  LAUNCH(k_unpack_post, P, vals, P, post);
  return hipSuccess;
}

hipError_t launch_max_pnrm(const RowStat* rs, int64_t n, uint32_t* out, uint8_t* pn8, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  LAUNCH(k_max_pnrm, n, rs, n, out, pn8);
  return hipSuccess;
}

hipError_t launch_pack_post4(const Post* post, int64_t P, uint32_t* post4, hipStream_t s) {
  LAUNCH(k_pack_post4, P, post, P, post4);
  return hipSuccess;
}

hipError_t launch_block_offsets(const int64_t* off, const Post* post, int32_t H, int64_t nb, int32_t CB,
                                uint32_t* hoff, hipStream_t s) {
  LAUNCH(k_block_offsets, (nb + 1) * (int64_t)H, off, post, H, nb, CB, hoff);
  return hipSuccess;
}

hipError_t launch_query_keys(const int64_t* rp, const int32_t* col, const float* val, const int32_t* rank, int64_t nq,
                             int64_t m, int rbits, double tol, uint64_t* keys, uint32_t* vals, float* qmw,
                             uint32_t* err, unsigned long long* bad, hipStream_t s) {
  if (nq <= 0) return hipSuccess;
  const int64_t blocks = (nq + 3) / 4;  // 4 waves of 64 lanes per block, one row per wave
  hipLaunchKernelGGL(k_query_keys, dim3((unsigned)(blocks < 32768 ? blocks : 32768)), dim3(256), 0, s, rp, col, val, rank,
                     nq, m, rbits, tol, keys, vals, qmw, err, bad);
  return hipGetLastError();
}

}  // namespace apss
