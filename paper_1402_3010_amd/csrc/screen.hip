// Head screen of the screened self-join.
//
// Partial indexing (Section 3.2.2) leaves the densest dimensions out of
// the inverted lists, and the paper notes that this splits the work into a
// dense and a sparse phase, the dense one suited to brute force.  The
// screened join makes that split explicit with a fixed head: the `head`
// densest dimensions.  A pair (x, y) has sim = H + T, H over the head and T
// over the tail.
//
//  * Pairs with T > 0 share a tail dimension; the sparse pass (the join
//    kernel over an index whose unindexed part of every row is its head)
//    finds and decides all of them.
//  * Pairs with T = 0 have sim = H <= ||x_h|| ||y_h||, so both rows have
//    head norm >= t.  Those rows are gathered (sorted by decreasing head
//    norm), their head parts packed as a dense bf16 block, and H~ is formed
//    for every pair of them whose norm product reaches t by bf16 MFMA with
//    float accumulation.  A pair is a candidate when
//    H~ >= t - kScreenMargin ||x_h|| ||y_h|| - kScreenEps, which no pair with
//    H >= t can miss; candidates that share no tail dimension are rescored
//    exactly and decided like every other pair.
//
// The two sets are disjoint and their union is every pair with sim >= t.
#include "apss_internal.h"
#include "rescore.h"
#include "screen.h"

namespace apss {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

#define LAUNCH1D(kern, nthreads, ...)                                                       \
  do {                                                                                      \
    const int64_t nt__ = (nthreads);                                                        \
    if (nt__ > 0) {                                                                         \
      int64_t g__ = (nt__ + 255) / 256;                                                     \
      if (g__ > 65536) g__ = 65536;                                                         \
      hipLaunchKernelGGL(kern, dim3((unsigned)g__), dim3(256), 0, s, __VA_ARGS__);          \
      const hipError_t e__ = hipGetLastError();                                             \
      if (e__ != hipSuccess) return e__;                                                    \
    }                                                                                       \
  } while (0)

__global__ void k_screen_select(const RowStat* __restrict__ rs, int64_t n, float t, uint64_t* __restrict__ keys,
                                unsigned long long* __restrict__ count) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
    const float nh = rs[r].pnrm;
    if (nh >= t) {
      const unsigned long long k = atomicAdd(count, 1ull);
      keys[k] = ((uint64_t)(0xFFFFFFFFu - __float_as_uint(nh)) << 32) | (uint64_t)r;
    }
  }
}

__global__ void k_screen_unpack(const uint64_t* __restrict__ keys, int64_t S, int64_t Sp, int32_t* __restrict__ sid,
                                float* __restrict__ nh) {
  for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < Sp; a += (int64_t)gridDim.x * blockDim.x) {
    if (a < S) {
      const uint64_t k = keys[a];
      sid[a] = (int32_t)(uint32_t)k;
      nh[a] = __uint_as_float(0xFFFFFFFFu - (uint32_t)(k >> 32));
    } else {
      sid[a] = -1;
      nh[a] = 0.0f;
    }
  }
}

// float -> bf16 bits, round to nearest even (weights are finite and positive)
__device__ __forceinline__ uint16_t bf16_rne(float f) {
  const uint32_t u = __float_as_uint(f);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// Packed head block, tile-major: row a, head rank k sits in the panel of
// (row tile a / 128, K step k / 32), each panel 128 rows x 32 bf16 stored
// contiguously (8 KB), so every operand load of the screen kernel reads a
// contiguous stream.
__device__ __forceinline__ int64_t panel_index(int64_t a, int32_t k, int32_t nks) {
  return ((((a >> 7) * nks + (k >> 5)) << 12) | ((a & 127) << 5)) | (k & 31);
}

__global__ void k_screen_pack(const int64_t* __restrict__ rp, const RComp* __restrict__ rc,
                              const int32_t* __restrict__ sid, int64_t S, int32_t head, int32_t ld,
                              uint16_t* __restrict__ X) {
  const int32_t nks = ld >> 5;
  for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < S; a += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = sid[a];
    const int64_t b = rp[r], e = rp[r + 1];
    // rank-space rows are in rank order: the head is a prefix
    for (int64_t k = b; k < e; ++k) {
      const RComp c = rc[k];
      if (c.r >= head) break;
      X[panel_index(a, c.r, nks)] = bf16_rne(c.w);
    }
  }
}

// One workgroup (4 waves) per output tile of 128 x 256 packed rows (row
// tile I against the two row tiles 2J, 2J + 1); wave w owns the 64 x 128
// part (w / 2, w % 2) as 2 x 4 MFMA blocks of 32 x 32
// (v_mfma_f32_32x32x16_bf16, float accumulation), so that every operand
// fragment read from LDS feeds two or four MFMAs.  Lane l of a 32 x 32 x 16
// MFMA holds operand row (l % 32), k = 8 (l / 32) .. + 7; result element r of
// lane l is row 8 (r / 4) + 4 (l / 32) + r % 4, column l % 32.
//
// K advances in steps of 32 through two LDS buffers.  Each buffer row is 32
// bf16 = four 16-byte chunks; chunk c of row r is stored at position
// c ^ ((r >> 2) & 3), so the 16 rows read by 16 lanes of one 128-bit LDS
// read hit 16 different bank groups.  Global loads run two steps ahead in
// two register sets (the loop is unrolled by two so the sets stay static).
constexpr int kStepK = 32;

__device__ __forceinline__ int swz(int row, int c) { return row * 4 + (c ^ ((row >> 2) & 3)); }

template <bool DUMP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_screen_mfma(ScreenArgs a, int64_t chunk) {
  __shared__ u32x4 As[2][kScreenTile * 4];
  __shared__ u32x4 Bs[2][kScreenTileB * 4];
  // the workgroups of one XCD (round-robin over blockIdx) take one
  // contiguous chunk of the tile list, which is ordered in blocks
  const int64_t ti = (int64_t)(blockIdx.x & 7u) * chunk + (int64_t)(blockIdx.x >> 3);
  if (ti >= a.ntiles) return;
  const int I = a.tiles[2 * ti], J = a.tiles[2 * ti + 1];
  const int64_t a0 = (int64_t)I * kScreenTile, b0 = (int64_t)J * kScreenTileB;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = (wave >> 1) * 64, wc = (wave & 1) * 128;
  const int nks = a.ld / kStepK;

  // this thread's chunks of each operand per step: rows tid / 4 + 64 h of
  // the step's contiguous 8 KB panels (one panel of the first operand's row
  // tile, two of the second's), chunk tid % 4
  const int lrow = tid >> 2, lc = tid & 3;
  const uint16_t* pa0 = a.X + (((int64_t)I * nks) << 12) + lrow * 32 + lc * 8;
  const uint16_t* pa1 = pa0 + 64 * 32;
  const uint16_t* pb0 = a.X + (((int64_t)(2 * J) * nks) << 12) + lrow * 32 + lc * 8;
  const uint16_t* pb1 = pb0 + 64 * 32;
  const uint16_t* pb2 = a.X + (((int64_t)(2 * J + 1) * nks) << 12) + lrow * 32 + lc * 8;
  const uint16_t* pb3 = pb2 + 64 * 32;
  const int s0 = swz(lrow, lc), s1 = swz(lrow + 64, lc), s2 = swz(lrow + 128, lc), s3 = swz(lrow + 192, lc);

  u32x4 r0[6], r1[6];
  auto ldg = [&](int ks, u32x4 (&r)[6]) {
    const int64_t o = (int64_t)ks << 12;
    r[0] = *reinterpret_cast<const u32x4*>(pa0 + o);
    r[1] = *reinterpret_cast<const u32x4*>(pa1 + o);
    r[2] = *reinterpret_cast<const u32x4*>(pb0 + o);
    r[3] = *reinterpret_cast<const u32x4*>(pb1 + o);
    r[4] = *reinterpret_cast<const u32x4*>(pb2 + o);
    r[5] = *reinterpret_cast<const u32x4*>(pb3 + o);
  };
  auto sts = [&](int buf, const u32x4 (&r)[6]) {
    As[buf][s0] = r[0];
    As[buf][s1] = r[1];
    Bs[buf][s0] = r[2];
    Bs[buf][s1] = r[3];
    Bs[buf][s2] = r[4];
    Bs[buf][s3] = r[5];
  };

  floatx16 acc[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

  const int frow = lane & 31, fh = lane >> 5;
  auto compute = [&](int buf) {
#pragma unroll
    for (int kk = 0; kk < kStepK / 16; ++kk) {
      bf16x8 fa[2], fb[4];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const u32x4 v = As[buf][swz(wr + 32 * i + frow, 2 * kk + fh)];
        fa[i] = __builtin_bit_cast(bf16x8, v);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const u32x4 v = Bs[buf][swz(wc + 32 * j + frow, 2 * kk + fh)];
        fb[j] = __builtin_bit_cast(bf16x8, v);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[i], fb[j], acc[i][j], 0, 0, 0);
    }
  };

  // prologue: step 0 in LDS, step 1 in flight (ld is a multiple of 64, so
  // the number of steps is even and at least 2).  The loads are issued
  // unconditionally (past the end they re-read the last panel) so that no
  // branch merge forces an early wait on them.
  ldg(0, r0);
  ldg(1, r1);
  sts(0, r0);
  __syncthreads();
  const int last = nks - 1;
  for (int ks = 0; ks < nks; ks += 2) {
    // even step ks: r1 holds step ks + 1, r0 is free
    ldg(ks + 2 < last ? ks + 2 : last, r0);
    compute(0);
    sts(1, r1);
    __syncthreads();
    // odd step ks + 1: r0 holds step ks + 2, r1 is free
    ldg(ks + 3 < last ? ks + 3 : last, r1);
    compute(1);
    sts(0, r0);
    __syncthreads();
  }

  if constexpr (DUMP) {
    // the accumulators themselves, for a check of the error bound
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t b = b0 + wc + 32 * j + (lane & 31);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int64_t ar = a0 + wr + 32 * i + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
          a.dump[ar * a.dump_ld + b] = acc[i][j][r];
        }
    }
    return;
  }

  // epilogue: threshold test and compaction by wave ballot
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int64_t b = b0 + wc + 32 * j + (lane & 31);
    const float nb = a.nh[b];
    const int32_t ib = a.sid[b];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t ar = a0 + wr + 32 * i + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const float na = a.nh[ar];
        const float p = na * nb;
        // the upper triangle only: a tile reaching the diagonal also holds
        // pairs (b, a) of earlier rows, and rows pair with themselves
        const bool want = ar < b && p * (1.0f + 0x1p-20f) >= a.t &&
                          acc[i][j][r] >= a.t - kScreenMargin * p - kScreenEps;
        const uint64_t m = __ballot(want);
        if (m) {
          unsigned long long base = 0;
          if (lane == 0) base = atomicAdd(a.count, (unsigned long long)__popcll(m));
          base = __shfl(base, 0);
          if (want) {
            const unsigned long long k = base + (unsigned long long)__popcll(m & lt);
            if ((int64_t)k < a.cap) {
              const uint32_t ia = (uint32_t)a.sid[ar];
              const uint32_t lo = ia < (uint32_t)ib ? ia : (uint32_t)ib;
              const uint32_t hi = ia < (uint32_t)ib ? (uint32_t)ib : ia;
              a.out[k] = ((uint64_t)lo << a.bj) | (uint64_t)hi;
            }
          }
        }
      }
    }
  }
}

// q's weight in rank r by binary search of its rank-ordered row (0 if absent)
__device__ __forceinline__ float row_lookup(const RComp* __restrict__ q, int qlen, int32_t r) {
  int lo = 0, hi = qlen;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (q[mid].r < r) lo = mid + 1;
    else hi = mid;
  }
  return (lo < qlen && q[lo].r == r) ? q[lo].w : 0.0f;
}

__global__ __launch_bounds__(256) void k_screen_verify(const uint64_t* __restrict__ cand, int64_t nc, int bj,
                                                       const int64_t* __restrict__ rp, const RComp* __restrict__ rc,
                                                       int32_t head, float t, uint64_t* __restrict__ out_key,
                                                       float* __restrict__ out_sim, int64_t cap,
                                                       unsigned long long* __restrict__ counters) {
  const int lane = threadIdx.x & 63;
  const int64_t wv = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const uint64_t jmask = (1ull << bj) - 1ull;
  WaveEmit em;
  for (int64_t p = wv; p < nc; p += nw) {
    const uint64_t key = cand[p];
    const int64_t i = (int64_t)(key >> bj), j = (int64_t)(key & jmask);
    // y = the smaller id, q = the larger: the orientation of the join kernel
    const int64_t ys = rp[i], qs = rp[j];
    const int ylen = (int)(rp[i + 1] - ys), qlen = (int)(rp[j + 1] - qs);
    const RComp* yrow = rc + ys;
    const RComp* qrow = rc + qs;
    auto look = [&](int32_t r) { return row_lookup(qrow, qlen, r); };
    bool tail = false;
    for (int k = lane; k < ylen; k += 64) {
      const RComp c = yrow[k];
      if (c.r >= head && look(c.r) != 0.0f) tail = true;
    }
    if (__ballot(tail)) continue;  // shares a tail dimension: decided by the sparse pass
    const float s32 = wave_dot2(yrow, ylen, lane, look);
    float sim;
    bool banded;
    const bool keep = wave_decide(yrow, ylen, lane, look, s32, t, &sim, &banded);
    if (banded && lane == 0) atomicAdd(&counters[C_BAND], 1ull);
    if (keep) {
      em.add(lane, key, sim);
      if (em.n == 64) em.flush(lane, counters, out_key, out_sim, cap);
    }
  }
  em.flush(lane, counters, out_key, out_sim, cap);
}

}  // namespace

hipError_t launch_screen_select(const RowStat* rs, int64_t n, float t, uint64_t* keys, unsigned long long* count,
                                hipStream_t s) {
  LAUNCH1D(k_screen_select, n, rs, n, t, keys, count);
  return hipSuccess;
}

hipError_t launch_screen_unpack(const uint64_t* keys, int64_t S, int64_t Sp, int32_t* sid, float* nh, hipStream_t s) {
  LAUNCH1D(k_screen_unpack, Sp, keys, S, Sp, sid, nh);
  return hipSuccess;
}

hipError_t launch_screen_pack(const int64_t* rp, const RComp* rc, const int32_t* sid, int64_t S, int32_t head,
                              int32_t ld, uint16_t* X, hipStream_t s) {
  LAUNCH1D(k_screen_pack, S, rp, rc, sid, S, head, ld, X);
  return hipSuccess;
}

hipError_t launch_screen_mfma(const ScreenArgs& a, hipStream_t s) {
  if (a.ntiles <= 0) return hipSuccess;
  if (!a.X || !a.tiles || a.ld <= 0 || a.ld % kScreenK) return hipErrorInvalidValue;
  if (!a.dump && (!a.nh || !a.sid || !a.out || !a.count)) return hipErrorInvalidValue;
  const int64_t chunk = (a.ntiles + 7) / 8;
  const int64_t grid = 8 * chunk;
  if (grid > 0x7FFFFFFF) return hipErrorInvalidValue;
  if (a.dump)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_screen_mfma<true>), dim3((unsigned)grid), dim3(256), 0, s, a, chunk);
  else
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_screen_mfma<false>), dim3((unsigned)grid), dim3(256), 0, s, a, chunk);
  return hipGetLastError();
}

hipError_t launch_screen_verify(const uint64_t* cand, int64_t nc, int bj, const int64_t* rp, const RComp* rc,
                                int32_t head, float t, uint64_t* out_key, float* out_sim, int64_t cap,
                                unsigned long long* counters, hipStream_t s) {
  if (nc <= 0) return hipSuccess;
  if (!cand || !rp || !rc || !out_key || !out_sim || !counters) return hipErrorInvalidValue;
  int64_t g = (nc + 3) / 4;  // 4 waves per workgroup, one pair per wave
  if (g > 8192) g = 8192;
  hipLaunchKernelGGL(k_screen_verify, dim3((unsigned)g), dim3(256), 0, s, cand, nc, bj, rp, rc, head, t, out_key,
                     out_sim, cap, counters);
  return hipGetLastError();
}

}  // namespace apss
