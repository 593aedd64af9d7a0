// Candidate generation, pruning, verification and rescoring (the hot path).
//
// Find-Matches (Algorithm 2) for a tile of QT query vectors at once, swept
// over the corpus in blocks of CB consecutive vector ids (the vector-range
// blocking of the paper's horizontal distribution, Section 5.2, applied
// inside one GPU).  For one (tile, block):
//
//  1. accumulate: for every component (d, q_d) of every query in the tile,
//     the entries (y, y_d) of the inverted list I_d with y in the block are
//     added into A_q[y] += q_d * y_d.  The lists hold only the indexed parts
//     of the corpus vectors (partial indexing, Section 3.2.2).  The score
//     array A is dense over the block (the all-pairs-0-array choice,
//     Section 4) and lives in LDS as unsigned fixed point (2^-30 units,
//     products rounded up), so sums are exact integers and independent of
//     the order of the LDS atomics.
//     Dense lists (rank < H) are located with per-(block, rank) offsets and
//     streamed coalesced by whole waves with a load-balanced split over all
//     segments of the tile; sparse lists keep per-component cursors that
//     advance monotonically as the tile sweeps the blocks.
//  2. filter each candidate (A > 0): size bound |y| maxweight(q) >= t,
//     max-weight bound A + min(|y'|,|q|) maxweight(q) maxweight(y') >= t
//     (the upperbound test of all-pairs-2), and the L2 bound
//     A + ||q_u|| ||y'|| >= t (Cauchy-Schwarz; q_u is q restricted to the
//     dimensions that can be unindexed, so ||q_u|| <= 1, and it is q's head
//     part when every row's unindexed part is its head); all with a small slack.
//  3. verify survivors: s = A + dot(q, y') (one wave per survivor when few,
//     else one lane per survivor); survivors of an item's blocks share one
//     queue and are verified together.
//  4. rescore verified pairs over the full rows in float with compensated
//     products and sums (Ogita, Rump and Oishi 2005, Dot2) in a fixed
//     lane-strided order and a fixed butterfly, so the result depends only on
//     (q, y); if it lies within kBand of t the pair is decided by a double
//     rescore.  One wave per pair; each kept pair takes its output slot from
//     a global atomic counter.
#include "apss_internal.h"
#include "join.h"
#include "rescore.h"

#include <type_traits>

namespace apss {

namespace {

// q_d * y_d in 2^-30 units, rounded up: an upper bound of the exact
// product.  The float product p is rounded to nearest; the fused multiply-add
// gives its exact residual a*b - p, and when that is positive p is replaced
// by the next float above it, which is at least a*b.  Scaling by 2^30 is
// exact (p <= 1), so the ceiling bounds a*b * 2^30 from above.  Both weights
// are positive, so a product that underflows still counts one unit.
__device__ __forceinline__ uint32_t fixp(float a, float b) {
  const float p = __fmul_rn(a, b);
  const float e = __builtin_fmaf(a, b, -p);
  const float pu = e > 0.0f ? __uint_as_float(__float_as_uint(p) + 1u) : p;
  const uint32_t v = (uint32_t)ceilf(pu * kFix);
  return v > 0u ? v : 1u;
}

// Query weight in units of 2^-15, rounded up.  A packed list entry holds the
// corpus weight in the same units (bits 16..31, rounded up) and the vector id
// modulo 2^16 (bits 0..15), so the product of the two 15-bit counts is an
// upper bound of q_d * y_d in units of 2^-30, computed by one 24-bit multiply.
__device__ __forceinline__ uint32_t q15(float w) {
  const uint32_t v = (uint32_t)ceilf(w * 32768.0f);
  return v > 0xFFFFu ? 0xFFFFu : v;
}
__device__ __forceinline__ uint32_t packed_product(uint32_t q, uint32_t e) { return __umul24(q, e >> 16); }

// Upper bound of a row's unindexed-part norm from its byte code.  Rounding
// of the product and sum it enters stays far inside the 4,096 accumulator
// units (4e-6 of a score) by which the filters' byte tests are loosened.
__device__ __forceinline__ float pn8_bound(uint8_t k) { return k == kPn8None ? 3.0e38f : (float)k * (1.0f / 254.0f); }

// (p & mask) | base in one instruction (the compiler turns the OR of
// disjoint bits back into an add and spends three instructions on it)
__device__ __forceinline__ uint32_t and_or(uint32_t p, uint32_t mask, uint32_t base) {
  uint32_t d;
  asm("v_and_or_b32 %0, %1, %2, %3" : "=v"(d) : "v"(p), "s"(mask), "v"(base));
  return d;
}

// Buffer descriptor of a device array (gfx9 resource word 3); loads through it
// take a scalar base offset and are bounds-checked by the hardware.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, (int)bytes, 0x00020000);
}

// segments at least this long are streamed by a whole wave
constexpr int kLongSeg = 32;

// list cursor of a staged component whose list has no entry in the work item's range
constexpr uint32_t kDead = 0xFFFFFFFFu;

// Values known to be equal across the wave, moved to scalar registers so that
// loops and branches on them stay scalar.
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ int64_t uni64(int64_t x) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)x);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)x >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// One dense-list segment of a (tile, block): list positions [pos, pos + len)
// feed query slot qi with the query weight q (units of 2^-15).  lenq = len | qi << 16.
struct Seg {
  uint32_t pos;
  uint32_t lenq;
  uint32_t q;
};

template <int QT_, int CB_, int NT_, int RD_, int SQ_, int QB_, int U_, int UL_, int WPE_>
struct Cfg {
  static constexpr int QT = QT_;  // queries per tile
  static constexpr int CB = CB_;  // corpus rows per block (accumulator width)
  static constexpr int NT = NT_;  // threads per workgroup
  static constexpr int RD = RD_;  // ranks with a dense per-query lookup table
  static constexpr int SQ = SQ_;  // survivor queue capacity
  static constexpr int QB = QB_;  // tile components staged in LDS
  static constexpr int U = U_;    // list loads in flight per lane, short segments
  static constexpr int UL = UL_;  // list loads in flight per lane, long segments
  static constexpr int WPE = WPE_;  // waves per SIMD the register budget must allow
};

template <class C, bool REM>
struct Smem {
  // the per-tile fields first: at small offsets, so that reads of them at
  // fixed addresses share one base register (the address offset a
  // local-memory instruction carries is 16 bits)
  int64_t qoff[C::QT + 1];
  float qmw[C::QT];
  float qpn[C::QT];  // bound on the query's part in the corpus rows' unindexed dimensions
  float qt[C::QT];
  float4 qb[C::QT];  // filter bounds of each query, times 2^30: threshold - slack, max weight, length * max weight, qpn
  float2 rtest;      // the tile's lowest qb.x (less 4,096 units) and highest qb.w: a row test that every slot's L2 bound implies
  int32_t qlen[C::QT];
  int32_t qhead[C::QT];
  int32_t wsum[C::NT / 64];
  uint2 wsum2[C::NT / 64];  // per-wave totals of the block path's segment allocation
  int32_t nshort;  // staged segments of a hashed item, stored from the back of seg[]
  int32_t qcount;
  int32_t ovf;
  int32_t vtot;    // list entries of the tile in the item's range (staged tiles)
  int32_t slot;    // range slot of the current item in its queue
  int64_t item;
  unsigned long long cnt[C_NUM];
  uint32_t acc[C::QT * C::CB];
  // remscore: one admission bit per accumulator slot -- bit (y - block
  // start) * QT + query slot on the block path, bit h (hash slot) on the
  // hashed path; cleared after each filter pass
  uint32_t adm[REM ? C::QT * C::CB / 32 : 1];
  float qd[C::QT * C::RD];
  Seg seg[C::QB];
  int32_t segpre[C::QB + 1];
  // the short stream's tables
  struct ShortTables {
    uint8_t flag[C::NT / 64][C::U][64];  // segment-start flags: one row per wave and chunk of a batch
    uint16_t first[C::QB * (kLongSeg - 1) / 64 + 2];  // segment holding each 64-entry chunk's first entry
    uint8_t sink[64];  // flag writes of lanes that have none (never read)
  };
  // survivor queue entries: the configured capacity less the tables' room
  static constexpr int SQE = C::SQ - (int)((sizeof(ShortTables) + 15) / 16);
  uint4 sq[SQE];  // x = slot << 16 | y - dbase, y = fixed-point score (0 = dropped), z unused, w = cut | len << 16
  ShortTables ss;
  // per-lane targets of the segment placement's stores that have nothing to
  // place (never read)
  Seg seg_sink[64];
  int32_t pre_sink[64];
  uint16_t first_sink[64];
  RComp qrow[C::QB];     // staged components of the tile
  uint2 cur[C::QB];      // list cursor of each staged component: {position, vector id at it}
  uint8_t cqi[C::QB];    // query slot of each staged component; bit 7: it admits new candidates (remscore)
};

// Orders the LDS accesses of one wave around an exchange between its lanes
// (LDS executes a wave's accesses in order; this keeps the compiler from
// moving or forwarding them).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// min of two non-negative finite floats (weights are validated positive):
// their bit patterns order like the values, so one integer min does it
__device__ __forceinline__ float min_nonneg(float x, float y) {
  return __uint_as_float(min(__float_as_uint(x), __float_as_uint(y)));
}

// REM: the remscore rule -- a candidate counts only once a component that
// admits new candidates has reached it (admission bits beside the scores).
template <class C, bool REM>
__global__ __launch_bounds__(C::NT) __attribute__((amdgpu_waves_per_eu(C::WPE))) void k_join(JoinArgs a) {
  constexpr int QT = C::QT, CB = C::CB, NT = C::NT, RD = C::RD, SQ = Smem<C, REM>::SQE, QB = C::QB, U = C::U,
                UL = C::UL;
  constexpr int NW = NT / 64;
  constexpr int KMAX = QB / NT;  // staged components per thread
  constexpr int YPT = CB / NT;   // corpus rows per thread in the filter
  // with the register budget of two waves per SIMD, the list offsets of an
  // item's next range are loaded while the current range is processed
  constexpr bool PF = C::WPE <= 2;
  static_assert(KMAX >= 1 && QB % NT == 0 && CB % NT == 0, "tile geometry");
  static_assert(CB <= 65536 && QT <= 256, "survivor packing");
  static_assert(SQ >= 128, "survivor queue");
  // the short stream's chunk table covers a hashed item's entries (at most
  // 3/4 of the table size) and its per-batch tags fit a byte
  static_assert((QT * CB / 2) * 3 / 4 / 64 + 1 <= QB * (kLongSeg - 1) / 64 + 2, "chunk table");
  static_assert((QB * (kLongSeg - 1) / NW + 64) / (64 * U) + 2 < 255, "stream tags");
  __shared__ Smem<C, REM> sm;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = uni(tid >> 6);
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

  unsigned long long c_visit = 0, c_tail = 0, c_cand = 0, c_surv = 0, c_ver = 0, c_band = 0;
  if (tid < C_NUM) sm.cnt[tid] = 0;
  const __amdgpu_buffer_rsrc_t prs = make_rsrc(a.post4, a.post4_bytes);
  // the accumulators start at zero and every item leaves them at zero
  for (int e = tid; e < QT * CB; e += NT) sm.acc[e] = 0u;
  constexpr int ADMW = QT * CB / 32;  // admission words (remscore)
  if constexpr (REM)
    for (int e = tid; e < ADMW; e += NT) sm.adm[e] = 0u;
  // every filter pass leaves the admission bits at zero
  auto clear_adm = [&]() {
    if constexpr (REM)
      for (int e = tid; e < ADMW; e += NT) sm.adm[e] = 0u;
  };
  // admission bit of (row offset in the block, query slot) on the block path
  auto admit_row = [&](uint32_t yl, int qi) {
    const uint32_t b = yl * (uint32_t)QT + (uint32_t)qi;
    atomicOr(&sm.adm[b >> 5], 1u << (b & 31u));
  };

  // Persistent loop over work items (group of rg consecutive corpus ranges,
  // query tile T).  The queue of XCD x holds the groups x, x + 8, ... in
  // order, so the workgroups resident on one XCD share a few ranges of lists
  // in its L2; an XCD whose queue is empty takes items from the others.
  // An item stages its tile once and then visits its ranges in turn.
  const int xcd = (int)(blockIdx.x & 7u);
  for (int qx = 0; qx < 8; ++qx) {
    const int x = (xcd + qx) & 7;
    const int64_t* cum = a.qcum + (int64_t)x * (a.nrx + 1);
    const int64_t total = cum[a.nrx];
    __syncthreads();
    if (tid == 0) sm.item = (int64_t)atomicAdd(&a.qctr[x], 1u);
    for (;;) {
      __syncthreads();
      const int64_t it = uni64(sm.item);
      if (it >= total) break;
      // the next item's index is fetched now and published at the end of
      // this item, so the atomic's latency overlaps the work
      uint32_t next_item = 0;
      if (tid == 0) next_item = atomicAdd(&a.qctr[x], 1u);
      // range slot j with cum[j] <= it < cum[j + 1]: wave 0 compares 64
      // slots per load round (cum is non-decreasing, cum[0] = 0)
      if (wave == 0) {
        int j = 0;
        for (int c0 = 0; c0 < (int)a.nrx; c0 += 64) {
          const int jj = c0 + lane;
          const uint64_t m = __ballot(jj < (int)a.nrx && cum[jj] <= it);
          if (m) j = c0 + 63 - (int)__builtin_clzll(m);
          if (m != ~0ull) break;
        }
        if (lane == 0) sm.slot = j;
      }
      __syncthreads();
      const int lo_j = uni(sm.slot);
      const int64_t grp = (int64_t)x + 8 * (int64_t)lo_j;  // range group
      int64_t u = it - cum[lo_j];
      // local pruning: consecutive items of a (range, tile) score its parts
      int32_t plo = 0, phi = 0x7FFFFFFF;
      if (a.parts > 1) {
        const int64_t pr = u % a.parts;
        u /= a.parts;
        plo = a.part_lo[pr];
        phi = a.part_lo[pr + 1];
      }
      const int64_t tile = a.ntiles - 1 - u;
  const int64_t q0 = a.tstart[tile];
  const int qn = (int)(a.tstart[tile + 1] - q0);

  if (tid <= qn) sm.qoff[tid] = a.qrp[q0 + tid];
  if (tid < QT) {
    sm.qmw[tid] = tid < qn ? a.qmw[q0 + tid] : 0.0f;
    sm.qpn[tid] = (tid < qn && a.qrs) ? a.qrs[q0 + tid].pnrm : 1.0f;
    sm.qt[tid] = (tid < qn && a.qt) ? a.qt[q0 + tid] : a.t;
  }
  if (tid == 0) {
    sm.nshort = 0;
    sm.qcount = 0;
    sm.ovf = 0;
    sm.vtot = 0;
  }
  if (tid < QT) sm.qhead[tid] = 0;  // staged tiles count their dense-table components
  for (int e = tid; e < QT * RD; e += NT) sm.qd[e] = 0.0f;
  __syncthreads();
  const int64_t qbase = uni64(sm.qoff[0]);
  const int64_t tile_nnz = uni64(sm.qoff[qn]) - qbase;
  const bool staged = tile_nnz <= QB;
  // first component of each query with rank >= RD (searched in global
  // memory only for tiles too large to stage)
  auto find_head = [&](const RComp* row, int len) {
    int lo = 0, hi = len;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (row[mid].r < RD) lo = mid + 1;
      else hi = mid;
    }
    return lo;
  };
  if (tid < qn) {
    const int64_t r0 = sm.qoff[tid], r1 = sm.qoff[tid + 1];
    sm.qlen[tid] = (int32_t)(r1 - r0);
    if (!staged) sm.qhead[tid] = find_head(a.qrc + r0, (int)(r1 - r0));
  }
  if (tid < QT) {
    // slots past qn never hold a score, so their bounds are never used
    // min(cut, len) * maxweight == min(cut * maxweight, len * maxweight) in
    // float: rounding is monotone, so the per-row part needs one product
    // The bounds are kept in accumulator units (2^30 per unit of score):
    // scaling by a power of two commutes with float rounding, so comparing
    // the raw accumulator with them decides exactly as in score units.
    const int ql = tid < qn ? (int)(sm.qoff[tid + 1] - sm.qoff[tid]) : 0;
    // With local pruning over p parts (a power of two) every bound is
    // divided by p: the size test is unchanged, and the score tests become
    // A_r + U/p >= (t - slack)/p, the local test of Lemma 1 with the bound U
    // of the unindexed part shared evenly by the parts.
    const float fx = a.parts > 1 ? kFix / (float)a.parts : kFix;
    sm.qb[tid] = make_float4((sm.qt[tid] - kSlack) * fx, sm.qmw[tid] * fx, (float)ql * sm.qmw[tid] * fx,
                             sm.qpn[tid] * fx);
  }
  // query slot of tile component k: the last qi with qoff[qi] <= k
  auto find_slot = [&](int64_t k) {
    int qi = 0;
#pragma unroll
    for (int step = QT / 2; step >= 1; step >>= 1)
      if (qi + step < qn && sm.qoff[qi + step] <= k) qi += step;
    return qi;
  };
  int64_t last_b = -1;
  if (qn > 0 && a.n > 0) last_b = a.triangle ? (q0 + qn - 1) / CB : (a.nb - 1);
  uint32_t* const gcur = a.wg_cur + (int64_t)blockIdx.x * a.wg_cur_stride;  // cursors of unstaged tiles
  // the item's ranges: those of its group that hold rows the tile meets
  // (the first always does: items exist only for such tiles)
  const int64_t R0 = grp * a.rg;
  int64_t R1 = R0 + a.rg - 1;
  if (R1 > a.nR - 1) R1 = a.nR - 1;
  if (last_b >= 0 && last_b / a.K < R1) R1 = last_b / a.K;
  if (R1 < R0) R1 = R0;

  // stage the tile once: its components, their query slots and admission
  // flags, and the dense lookup table (each thread later reads back only the
  // components it wrote, so no barrier is needed before the ranges)
  if (staged && last_b >= R0 * a.K) {
#pragma unroll
    for (int j = 0; j < KMAX; ++j) {
      const int k = j * NT + tid;
      if (k < tile_nnz) {
        const RComp c = a.qrc[qbase + k];
        const int qi = find_slot(qbase + k);
        bool admits = true;  // remscore: the component admits new candidates
        if constexpr (REM) admits = qbase + k - sm.qoff[qi] >= (int64_t)a.qadm[q0 + qi];
        if (c.r < RD) {
          // rows are in rank order: a query's components of rank < RD come
          // first, and their count is the position of its first other one
          sm.qd[qi * RD + c.r] = c.w;
          atomicAdd(&sm.qhead[qi], 1);
        }
        sm.qrow[k] = c;
        sm.cqi[k] = (uint8_t)(qi | (admits ? 0x80 : 0));
      }
    }
  }

  uint32_t pc[KMAX], pn[KMAX];  // (PF) the next range's first and end offsets of this thread's components
#pragma unroll
  for (int j = 0; j < KMAX; ++j) pc[j] = pn[j] = 0u;
  for (int64_t R = R0; R <= R1; ++R) {
  if (R > R0) {
    // the previous range is done with the per-range fields
    __syncthreads();
    if (tid == 0) {
      sm.nshort = 0;
      sm.vtot = 0;
    }
    __syncthreads();
  }
  const int64_t b_begin = R * a.K;
  const int64_t b_end = (b_begin + a.K) < (last_b + 1) ? (b_begin + a.K) : (last_b + 1);

  // place every list cursor at the range's first block (block offsets for
  // dense lists, range offsets for sparse ones), and fetch that block's
  // segment ends of the dense lists
  uint32_t hn[KMAX];
#pragma unroll
  for (int j = 0; j < KMAX; ++j) hn[j] = 0;
  int32_t vmine = 0;  // this thread's share of the range's list entries
  if (b_begin < b_end && staged) {
    // A staged tile has at most QB = KMAX * NT components: every list-offset
    // load is issued first, then the LDS writes, so the loads' latencies
    // overlap instead of adding up per component.  Live segments take their
    // places by one atomic per wave.
    RComp cc[KMAX];
    int cq[KMAX];
    bool cadm[KMAX];
#pragma unroll
    for (int j = 0; j < KMAX; ++j) {
      const int k = j * NT + tid;  // < QB: the LDS reads stay in bounds
      const int c8 = sm.cqi[k];
      cc[j] = k < tile_nnz ? sm.qrow[k] : RComp{0x7FFFFFFF, 0.0f};
      cq[j] = c8 & 0x7F;
      cadm[j] = (c8 >> 7) != 0;
    }
    uint32_t p0[KMAX], p1[KMAX];
#pragma unroll
    for (int j = 0; j < KMAX; ++j) {
      const int k = j * NT + tid;
      const int32_t r = cc[j].r;
      p0[j] = 0u;
      p1[j] = 0u;
      if (k < tile_nnz) {
        // dense lists by block offsets, sparse ones by range offsets
        const bool dense = r < a.H;
        if (PF && R > R0) {
          p0[j] = pc[j];
          p1[j] = pn[j];
        } else {
          const uint32_t* t0 =
              dense ? a.hoff + b_begin * (int64_t)a.H + r : a.toff + R * (int64_t)a.m_tail + (r - a.H);
          const uint32_t* t1 =
              dense ? a.hoff + b_end * (int64_t)a.H + r : a.toff + (R + 1) * (int64_t)a.m_tail + (r - a.H);
          p0[j] = *t0;
          p1[j] = *t1;
        }
        // the next block's segment end of a dense list (b_begin + 1 <= nb);
        // with PF loaded by the block path when a range takes it
        if (!PF) hn[j] = dense ? a.hoff[(b_begin + 1) * (int64_t)a.H + r] : 0u;
      }
    }
#pragma unroll
    for (int j = 0; j < KMAX; ++j) {
      const int k = j * NT + tid;
      const bool valid = k < tile_nnz;
      const RComp c = cc[j];
      const int qi = cq[j];
      const bool admits = valid && cadm[j];
      // no list entry in the corpus range, or a rank outside the item's part
      const bool dead = !valid || p1[j] == p0[j] || c.r < plo || c.r >= phi;
      vmine += dead ? 0 : (int32_t)(p1[j] - p0[j]);
      if (valid) {
        // the block path loads the first entry's vector id of a sparse list
        // once the range is known to take that path
        sm.cur[k] = make_uint2(dead ? kDead : p0[j], 0u);
      }
      if (!PF && dead) hn[j] = 0u;
      // the component's entries in the whole range, for a hashed item
      // (whose segments are all short enough for the 16-bit length)
      const uint64_t m = __ballot(!dead);
      int base = 0;
      if (lane == 0 && m) base = atomicAdd(&sm.nshort, (int)__popcll(m));
      base = __shfl(base, 0);
      if (!dead) {
        Seg sg;
        sg.pos = p0[j];
        sg.lenq = ((p1[j] - p0[j]) & 0xFFFFu) | ((uint32_t)qi << 16);
        // bit 31 (remscore): the component admits; the 24-bit product ignores it
        sg.q = q15(c.w) | (REM && admits ? 0x80000000u : 0u);
        sm.seg[QB - 1 - (base + (int)__popcll(m & lt))] = sg;
      }
    }
    if constexpr (PF) {
      // the next range starts where this one ends; its ends are loaded now
      // and waited for only when that range is staged
      if (R < R1) {
        const int64_t nend = ((R + 2) * a.K) < (last_b + 1) ? ((R + 2) * a.K) : (last_b + 1);
#pragma unroll
        for (int j = 0; j < KMAX; ++j) {
          const int k = j * NT + tid;
          const int32_t r = cc[j].r;
          pc[j] = p1[j];
          if (k < tile_nnz)
            pn[j] = r < a.H ? a.hoff[nend * (int64_t)a.H + r] : a.toff[(R + 2) * (int64_t)a.m_tail + (r - a.H)];
        }
      }
    }
  } else if (b_begin < b_end) {
    // tiles too large to stage: list cursors in the workgroup's global space
    for (int64_t k = tid; k < tile_nnz; k += NT) {
      const RComp c = a.qrc[qbase + k];
      const int qi = find_slot(qbase + k);
      if (c.r < RD) sm.qd[qi * RD + c.r] = c.w;
      uint32_t p0, p1, ny = 0;
      if (c.r < a.H) {
        p0 = a.hoff[b_begin * (int64_t)a.H + c.r];
        p1 = a.hoff[b_end * (int64_t)a.H + c.r];
      } else {
        p0 = a.toff[R * (int64_t)a.m_tail + (c.r - a.H)];
        p1 = a.toff[(R + 1) * (int64_t)a.m_tail + (c.r - a.H)];
        ny = (int64_t)p0 < a.off[c.r + 1] ? a.post[p0].y : 0xFFFFFFFFu;
      }
      // no list entry in the item's corpus range, or a rank outside the item's part
      const bool dead = p1 == p0 || c.r < plo || c.r >= phi;
      if (dead) p1 = p0;
      vmine += (int32_t)(p1 - p0);
      gcur[2 * k] = dead ? kDead : p0;
      gcur[2 * k + 1] = ny;
    }
  }
  // one atomic per wave for the item's entry count
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) vmine += __shfl_xor(vmine, o, 64);
  if (lane == 0 && vmine) atomicAdd(&sm.vtot, vmine);
  __syncthreads();
  if (wave == 0) {
    // a slot's L2 bound A + qb.w * pnrm >= qb.x implies the row test
    // amax + rtest.y * pnrm >= rtest.x for the row's largest score amax
    // (float sums and products are monotone; the 4,096 units, 4e-6 of a
    // score, cover a fused multiply-add on one side only).  Read by the
    // filters, after barriers to come.
    float tmin = 3.0e38f, wmax = 0.0f;
    if (lane < qn) {
      tmin = sm.qb[lane].x;
      wmax = sm.qb[lane].w;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      tmin = fminf(tmin, __shfl_xor(tmin, o, 64));
      wmax = fmaxf(wmax, __shfl_xor(wmax, o, 64));
    }
    if (lane == 0) sm.rtest = make_float2(tmin - 4096.0f, wmax);
  }

  // q[r] for the query in slot qi (0 if absent)
  auto qlookup = [&](int qi, int32_t r) -> float {
    if (r < RD) return sm.qd[qi * RD + r];
    const RComp* row = staged ? (sm.qrow + (sm.qoff[qi] - qbase)) : (a.qrc + sm.qoff[qi]);
    int lo = sm.qhead[qi], hi = sm.qlen[qi];
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (row[mid].r < r) lo = mid + 1;
      else hi = mid;
    }
    return (lo < sm.qlen[qi] && row[lo].r == r) ? row[lo].w : 0.0f;
  };


  // Exclusive prefix sums of the lengths of sseg[0..ns) into sm.segpre (KMAX
  // consecutive segments per thread), and for every 64-entry chunk of the
  // concatenated segments the segment that holds its first entry.  Ends
  // with the writes pending: the caller synchronises.
  auto scan_short = [&](const Seg* sseg, int ns) {
    int loc[KMAX], len[KMAX];
    int run = 0;
#pragma unroll
    for (int j = 0; j < KMAX; ++j) {
      const int e = tid * KMAX + j;
      loc[j] = run;
      len[j] = e < ns ? (int)(sseg[e].lenq & 0xFFFFu) : 0;
      run += len[j];
    }
    int incl = run;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int u = __shfl_up(incl, o, 64);
      if (lane >= o) incl += u;
    }
    if (lane == 63) sm.wsum[wave] = incl;
    __syncthreads();
    int woff = 0;
    for (int w = 0; w < wave; ++w) woff += sm.wsum[w];
    const int excl = woff + incl - run;
#pragma unroll
    for (int j = 0; j < KMAX; ++j) {
      const int e = tid * KMAX + j;
      if (e < ns) {
        const int s0 = excl + loc[j];
        sm.segpre[e] = s0;
        for (int c = (s0 + 63) & ~63; c < s0 + len[j]; c += 64) sm.ss.first[c >> 6] = (uint16_t)e;
      }
    }
    if (tid == NT - 1) sm.segpre[ns] = woff + incl;
  };

  // Every entry of the short segments sseg[0..ns) (exclusive prefix sums of
  // their lengths in sm.segpre, L entries in all, chunk table from
  // scan_short): wave w takes a contiguous slice of whole 64-entry chunks, U
  // chunks per batch (lane l, entry c + l), U loads in flight per lane.  The
  // segment of each entry: the chunk table gives the segment sa holding the
  // chunk's first entry; lane j takes the start of segment sa + 1 + j and
  // flags it in the chunk's LDS row; every lane counts the flags at or before
  // its own entry (one ballot).  Segments are never empty, so at most 63 of
  // them start inside a chunk.  A flag holds the batch's tag, so older flags
  // need no clearing.  The chunks of a batch are independent, so their LDS
  // round trips overlap.  add(qi, packed entry, query weight, live) is
  // called by every lane; live is false for lanes past the wave's slice,
  // whose segment, slot and (bounds-checked) load are still valid.
  auto stream_short = [&](const Seg* sseg, int ns, int L, auto&& add) {
    const int per = (((L + NW - 1) / NW) + 63) & ~63;
    const int vbeg = wave * per;
    const int vend = (vbeg + per) < L ? (vbeg + per) : L;
    if (vbeg >= vend) return;
#pragma unroll
    for (int u = 0; u < U; ++u) sm.ss.flag[wave][u][lane] = 0;
    uint32_t tag = 0u;
    for (int base = vbeg; base < vend; base += 64 * U) {
      ++tag;
      int sa[U], rel[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int c = base + u * 64;
        sa[u] = c < vend ? (int)sm.ss.first[c >> 6] : 0;
        const int sj = sa[u] + 1 + lane;
        // (read at sj clamped to ns, where the total is, so without a branch)
        const int d = sm.segpre[sj < ns ? sj : ns] - c;
        rel[u] = (c < vend && sj < ns) ? d : 0x7FFFFFFF;  // >= 1: segment sa holds entry c
      }
      // every lane stores: a lane whose segment does not start in the chunk
      // writes to the sink instead of branching around the store
#pragma unroll
      for (int u = 0; u < U; ++u)
        *((uint32_t)rel[u] < 64u ? &sm.ss.flag[wave][u][rel[u]] : &sm.ss.sink[lane]) = (uint8_t)tag;
      wave_lds_sync();
      uint32_t pos[U], qwb[U];
      int qs[U];
      bool lv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int c = base + u * 64;
        const bool f = sm.ss.flag[wave][u][lane] == (uint8_t)tag;
        const uint64_t fm = __ballot(f);
        const int k = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(fm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)fm, 0u)) +
                      (f ? 1 : 0);
        const int sg = sa[u] + k;
        const Seg S = sseg[sg];
        const int v = c + lane;
        pos[u] = S.pos + (uint32_t)(v - sm.segpre[sg]);
        qwb[u] = S.q;
        // lanes past the slice keep a valid segment (sg < ns) and slot
        qs[u] = (int)(S.lenq >> 16);
        lv[u] = v < vend;
      }
      wave_lds_sync();
      uint32_t pv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) pv[u] = __builtin_amdgcn_raw_buffer_load_b32(prs, (int)(pos[u] * 4u), 0, 0);
#pragma unroll
      for (int u = 0; u < U; ++u)
        add(qs[u], pv[u], qwb[u], lv[u]);
    }
  };

  // ------------------------------------------------------------ verify, rescore
  // survivors in sm.sq name rows by their offset from dbase
  int64_t dbase = 0;
  auto drain = [&]() {
    const int ns = uni(sm.qcount < SQ ? sm.qcount : SQ);
    // verify s = A + dot(q, y'); y' is the first cut components of the row,
    // densest dimension first.  Few survivors: one wave per survivor, lanes
    // over y' (short latency chain); many: one lane per survivor.  With
    // local pruning A is one part's score only: every survivor goes to the
    // rescore, which decides on the full dot product.
    if (a.parts > 1) {
      if (tid == 0) c_ver += (unsigned long long)ns;
    } else if (ns <= 4 * NW) {
      for (int e = wave; e < ns; e += NW) {
        const uint4 it = sm.sq[e];
        const int qi = (int)(it.x >> 16);
        uint32_t cut = it.w & 0xFFFFu;
        if ((it.w >> 16) == 0xFFFFu) cut = (uint32_t)a.rs[dbase + (it.x & 0xFFFFu)].cut;
        const uint32_t ys = (uint32_t)a.rp[dbase + (it.x & 0xFFFFu)];  // row offsets fit 32 bits (nnz < 2^32)
        float part = 0.0f;
        for (uint32_t k = (uint32_t)lane; k < cut; k += 64) {
          const RComp c = a.rc[ys + k];
          part += qlookup(qi, c.r) * c.w;
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) part += __shfl_xor(part, o, 64);
        const float sc = (float)it.y * kInvFix + part;
        if (lane == 0) {
          if (sc >= sm.qt[qi] - kSlack) ++c_ver;
          else sm.sq[e].y = 0u;
        }
      }
    } else
    for (int e = tid; e < ns; e += NT) {
      const uint4 it = sm.sq[e];
      const int qi = (int)(it.x >> 16);
      uint32_t cut = it.w & 0xFFFFu;
      if ((it.w >> 16) == 0xFFFFu) cut = (uint32_t)a.rs[dbase + (it.x & 0xFFFFu)].cut;
      const uint32_t ys = (uint32_t)a.rp[dbase + (it.x & 0xFFFFu)];
      float sc = (float)it.y * kInvFix;
      for (uint32_t k0 = 0; k0 < cut; k0 += 4) {
        RComp c[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) c[u] = a.rc[ys + (k0 + u < cut ? k0 + u : cut - 1)];
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (k0 + u < cut) sc += qlookup(qi, c[u].r) * c[u].w;
      }
      if (sc >= sm.qt[qi] - kSlack) ++c_ver;
      else sm.sq[e].y = 0u;
    }
    __syncthreads();
    // rescore: one wave per verified pair; each wave's kept pairs are
    // written together
    for (int base = wave * 64; base < ns; base += NT) {
      const int e = base + lane;
      uint64_t fm = __ballot(e < ns && sm.sq[e < ns ? e : 0].y != 0u);
      WaveEmit em;
      while (fm) {
        const int l = __ffsll((unsigned long long)fm) - 1;
        fm &= fm - 1;
        const uint4 it = sm.sq[base + l];
        const int qi = (int)(it.x >> 16);
        const int64_t y = dbase + (int64_t)(it.x & 0xFFFFu);
        const int64_t ys = a.rp[y];
        int ylen = (int)(it.w >> 16);
        if (ylen == 0xFFFF) ylen = (int)(a.rp[y + 1] - a.rp[y]);
        const RComp* yrow = a.rc + ys;
        auto look = [&](int32_t r) { return qlookup(qi, r); };
        const float s32 = wave_dot2(yrow, ylen, lane, look);
        float sim;
        bool banded;
        const bool keep = wave_decide(yrow, ylen, lane, look, s32, sm.qt[qi], &sim, &banded);
        if (banded && lane == 0) ++c_band;
        if (keep) {
          const uint64_t qid = (uint64_t)(q0 + qi);
          em.add(lane, a.triangle ? (((uint64_t)y << a.bj) | qid) : ((qid << a.bj) | (uint64_t)y), sim);
        }
      }
      em.flush(lane, a.counters, a.out_key, a.out_sim, a.cap);
    }
    __syncthreads();
    if (tid == 0) {
      sm.qcount = 0;
      sm.ovf = 0;
    }
    __syncthreads();
  };


  // ------------------------------------------------------------ sparse items
  // An item whose lists hold at most 3 HS / 4 entries in the whole range is
  // accumulated at once into an open-addressing hash table in LDS (keys and
  // fixed-point scores in the two halves of the accumulator array, key 0 =
  // free), and only the touched slots are filtered.  The table never fills,
  // so every probe sequence ends.  Other items sweep the range block by block.
  constexpr int HS = QT * CB / 2;
  constexpr int HBITS = (HS == 8192) ? 13 : (HS == 4096) ? 12 : (HS == 2048) ? 11 : 10;
  static_assert((1 << HBITS) == HS, "hash table size");
  const bool hashed = staged && b_begin < b_end && (int64_t)a.K * CB <= 65536 && uni(sm.vtot) <= HS - HS / 4;
  if (hashed) {
    uint32_t* const hval = sm.acc;
    uint32_t* const hkey = sm.acc + HS;
    const int64_t rbeg = b_begin * CB;
    // the live segments written at staging, contiguous at the back of seg[]
    const int ns = uni(sm.nshort);
    Seg* const sseg = sm.seg + (QB - ns);
    scan_short(sseg, ns);
    __syncthreads();
    const int L = uni(sm.segpre[ns]);
    if (tid == 0) c_visit += (unsigned long long)L;
    // every entry of every segment, split evenly over the waves
    stream_short(sseg, ns, L, [&](int qi, uint32_t p, uint32_t qw, bool live) {
      if (!live) return;
      const uint32_t key = (((uint32_t)qi << 16) | ((p - (uint32_t)rbeg) & 0xFFFFu)) + 1u;
      // double hashing: a second multiplicative hash gives an odd step, so
      // the probe sequence visits every slot of the power-of-two table (which
      // is never full) and keys that collide once part at the next probe
      uint32_t h = (key * 0x9E3779B1u) >> (32 - HBITS);
      const uint32_t step = ((key * 0x85EBCA77u) >> (32 - HBITS)) | 1u;
      for (;;) {
        const uint32_t old = atomicCAS(&hkey[h], 0u, key);
        if (old == 0u || old == key) {
          atomicAdd(&hval[h], packed_product(qw, p));
          if constexpr (REM)
            if (qw >> 31) atomicOr(&sm.adm[h >> 5], 1u << (h & 31u));
          break;
        }
        h = (h + step) & (uint32_t)(HS - 1);
      }
    });
    __syncthreads();
    // filter the touched slots; survivors that do not fit the queue stay
    // in the table for the next pass
    dbase = rbeg;
    for (;;) {
      if constexpr (QT >= 16) {
        // 16-query tiles: G slots per thread at a time, their row-statistics
        // loads issued together (unconditionally, row 0 for empty slots)
        // before any is used.  (8-query tiles keep one slot at a time: the
        // grouped form costs registers their block path needs.)
        constexpr int G = (HS / NT) < 4 ? (HS / NT) : 4;
        static_assert(G >= 1 && (HS / NT) % G == 0, "hash filter groups");
#pragma unroll 1
        for (int h0 = 0; h0 < HS; h0 += G * NT) {
          uint32_t kk[G], hv[G];
          int64_t yv[G];
          bool ok[G], pre[G];
          float qw[G], qx[G];
          uint8_t k8[G];
          RowStat stg[G];
#pragma unroll
          for (int g = 0; g < G; ++g) {
            const int h = h0 + g * NT + tid;
            kk[g] = hkey[h];
            hv[g] = hval[h];
            const int qi = (int)((kk[g] - 1u) >> 16);
            yv[g] = rbeg + (int64_t)((kk[g] - 1u) & 0xFFFFu);
            ok[g] = kk[g] != 0u && yv[g] < a.n && !(a.triangle && yv[g] >= q0 + qi);
            if constexpr (REM) ok[g] = ok[g] && ((sm.adm[h >> 5] >> (h & 31)) & 1u);
            // the L2 bound with the largest unindexed-part norm of any row,
            // then with the row's own norm as a byte: a candidate that fails
            // either cannot survive and needs no row statistics
            const float4 qbq = sm.qb[ok[g] ? qi : 0];
            qw[g] = qbq.w;
            qx[g] = qbq.x - 4096.0f;
            pre[g] = ok[g] && (float)hv[g] + qbq.w * a.pnrm_max >= qx[g];
            k8[g] = a.pn8[pre[g] ? yv[g] : 0];
          }
          bool need = false;
#pragma unroll
          for (int g = 0; g < G; ++g) {
            pre[g] = pre[g] && (float)hv[g] + qw[g] * pn8_bound(k8[g]) >= qx[g];
            need = need || pre[g];
            stg[g] = RowStat{0, 0, 0.0f, 0.0f};
          }
          // row statistics only where a lane of the wave still needs them
          if (__ballot(need)) {
#pragma unroll
            for (int g = 0; g < G; ++g) stg[g] = a.rs[pre[g] ? yv[g] : 0];
          }
#pragma unroll
          for (int g = 0; g < G; ++g) {
            const int h = h0 + g * NT + tid;
            bool want = false, retry = false;
            const int qi = (int)((kk[g] - 1u) >> 16);
            const int yl = (int)((kk[g] - 1u) & 0xFFFFu);
            const uint32_t av = hv[g];
            uint32_t packed = 0u;
            if (pre[g]) {
              const RowStat st = stg[g];
              const int ylen = st.len;
              packed = (uint32_t)(st.cut < 0xFFFF ? st.cut : 0xFFFF) | ((uint32_t)(ylen < 0xFFFF ? ylen : 0xFFFF) << 16);
              const float A = (float)av;  // accumulator units, as the bounds
              const float4 qb = sm.qb[qi];
              const float thr = qb.x, qm = qb.y;
              want = ((float)ylen * qm >= thr) && (A + min_nonneg((float)st.cut * qm, qb.z) * st.pmw >= thr) &&
                     (A + qb.w * st.pnrm >= thr);
            }
            if (ok[g]) ++c_cand;
            const uint64_t wm = __ballot(want);
            if (wm) {
              int qb = 0;
              if (lane == 0) qb = atomicAdd(&sm.qcount, (int)__popcll(wm));
              qb = __shfl(qb, 0);
              if (want) {
                const int slot = qb + (int)__popcll(wm & lt);
                if (slot < SQ) {
                  sm.sq[slot] = make_uint4(((uint32_t)qi << 16) | (uint32_t)yl, av, 0u, packed);
                  ++c_surv;
                } else {
                  retry = true;
                  --c_cand;
                  sm.ovf = 1;
                }
              }
            }
            if (kk[g] && !retry) {
              hkey[h] = 0u;
              hval[h] = 0u;
              }
          }
        }
      } else {
#pragma unroll 1
        for (int h0 = 0; h0 < HS; h0 += NT) {
          const int h = h0 + tid;
          const uint32_t kk = hkey[h];
          bool want = false, retry = false;
          int qi = 0, yl = 0;
          uint32_t av = 0u, packed = 0u;
          if (kk) {
            qi = (int)((kk - 1u) >> 16);
            yl = (int)((kk - 1u) & 0xFFFFu);
            const int64_t y = rbeg + yl;
            av = hval[h];
            bool adm_ok = true;
            if constexpr (REM) adm_ok = (sm.adm[h >> 5] >> (h & 31)) & 1u;
            if (adm_ok && y < a.n && !(a.triangle && y >= q0 + qi)) {
              const float4 qb = sm.qb[qi];
              const float A = (float)av;  // accumulator units, as the bounds
              // the L2 bound with the largest unindexed-part norm of any row
              // first, then with the row's own norm as a byte
              if (A + qb.w * a.pnrm_max >= qb.x - 4096.0f && A + qb.w * pn8_bound(a.pn8[y]) >= qb.x - 4096.0f) {
                const RowStat st = a.rs[y];
                const int ylen = st.len;
                packed = (uint32_t)(st.cut < 0xFFFF ? st.cut : 0xFFFF) | ((uint32_t)(ylen < 0xFFFF ? ylen : 0xFFFF) << 16);
                const float thr = qb.x, qm = qb.y;
                want = ((float)ylen * qm >= thr) && (A + min_nonneg((float)st.cut * qm, qb.z) * st.pmw >= thr) &&
                       (A + qb.w * st.pnrm >= thr);
              }
              ++c_cand;
            }
          }
          const uint64_t wm = __ballot(want);
          if (wm) {
            int qb = 0;
            if (lane == 0) qb = atomicAdd(&sm.qcount, (int)__popcll(wm));
            qb = __shfl(qb, 0);
            if (want) {
              const int slot = qb + (int)__popcll(wm & lt);
              if (slot < SQ) {
                sm.sq[slot] = make_uint4(((uint32_t)qi << 16) | (uint32_t)yl, av, 0u, packed);
                ++c_surv;
              } else {
                retry = true;
                --c_cand;
                sm.ovf = 1;
              }
            }
          }
          if (kk && !retry) {
            hkey[h] = 0u;
            hval[h] = 0u;
          }
        }
      }
      __syncthreads();
      const int o = uni(sm.ovf);
      const int qc = uni(sm.qcount);
      __syncthreads();
      if (qc > 0) drain();
      if (!o) {
        clear_adm();
        break;
      }
    }
  }

  if (!hashed && b_begin < b_end) {
    // the block path builds its own segments, and walks the sparse lists
    // from the vector id of their first entry in the range
    if (staged) {
      for (int64_t k = tid; k < tile_nnz; k += NT) {
        const uint2 cu = sm.cur[k];
        if (cu.x != kDead && sm.qrow[k].r >= a.H) sm.cur[k] = make_uint2(cu.x, a.post[cu.x].y);
      }
      if constexpr (PF) {
        // the next block's segment ends of the live dense lists
#pragma unroll
        for (int j = 0; j < KMAX; ++j) {
          const int k = j * NT + tid;
          const int32_t r = sm.qrow[k].r;
          hn[j] = (k < tile_nnz && sm.cur[k].x != kDead && r < a.H) ? a.hoff[(b_begin + 1) * (int64_t)a.H + r] : 0u;
        }
      }
    }
    __syncthreads();
  }
  // Survivors of several blocks share the queue (their rows named from the
  // item's first row) when the item's rows fit the 16-bit offset; the queue
  // is drained when half full, on overflow and after the item's last block.
  const bool defer = (int64_t)a.K * CB <= 65536;
  for (int64_t b = (hashed ? b_end : b_begin); b < b_end; ++b) {
    const int64_t blk0 = b * CB;
    dbase = defer ? b_begin * CB : blk0;
    const uint32_t yoff = (uint32_t)(blk0 - dbase);  // queue offset of the block's first row
    const int64_t blk1 = (blk0 + CB) < a.n ? (blk0 + CB) : a.n;
    const uint32_t* hend = a.hoff + (b + 1) * (int64_t)a.H;   // end of each dense list's block segment
    const uint32_t* hnext = a.hoff + (b + 2) * (int64_t)a.H;  // same for the next block (b < last_b)

    // per-row data of the filter's first rows; the loads overlap the accumulation
    RowStat stN;
    auto load_rows = [&](int yi) {
      const int64_t y = blk0 + yi * NT + tid;
      stN = a.rs[y < blk1 ? y : blk0];
    };
    load_rows(0);

    // ------------------------------------------------------------ accumulate
    for (int64_t cb = 0; cb < tile_nnz; cb += QB) {
      // pass 1: every component's segment of a dense list is known from the
      // block offsets; sparse lists with an entry in this block get their
      // first two entries loaded (no waiting here)
      bool thit[KMAX];
      Seg sgj[KMAX];  // this thread's segment of each component, placed after the allocation scan
      int sk[KMAX];   // its kind: 0 none, 1 short, 2 long
      Post t0[KMAX];
      uint32_t t1y[KMAX];
      uint32_t hq[KMAX];  // byte offset of the next block's segment end in hnext (out of range: none)
      uint32_t tpos[KMAX], tend[KMAX];
      float tw[KMAX];
      int tqi[KMAX];
      bool tadm[KMAX];  // remscore: the sparse list's component admits new candidates
      // (one copy of the loop per tile kind; the staged one has no
      // conditional loads, whose results later code would wait for)
      auto pass1 = [&](auto kind) {
        constexpr bool ST = decltype(kind)::value;
#pragma unroll
        for (int j = 0; j < KMAX; ++j) {
          const int64_t k = cb + (int64_t)j * NT + tid;
          bool has_seg = false;
          Seg sg = {0u, 0u, 0u};
          thit[j] = false;
          hq[j] = 0xFFFFFFFFu;
          if constexpr (ST) {
            // without branches around loads: k < QB, so the LDS reads stay
            // in bounds, and a component that is not a sparse hit loads the
            // lists' first entry instead of its own
            const RComp c = sm.qrow[k];
            const int cq8 = sm.cqi[k];
            const int qi = cq8 & 0x7F;
            const bool admits = REM && (cq8 >> 7);
            const uint2 cu = sm.cur[k];
            const uint32_t pos = cu.x, ny = cu.y;
            const bool live = k < tile_nnz && pos != kDead;
            const bool dense = c.r < a.H;
            const uint32_t e = hn[j];
            if (live && dense) hq[j] = (uint32_t)c.r * 4u;  // prefetched below for the next block
            has_seg = live && dense && e > pos;
            sg.pos = pos;
            sg.lenq = (e - pos) | ((uint32_t)qi << 16);
            sg.q = q15(c.w) | (admits ? 0x80000000u : 0u);
            if (has_seg) sm.cur[k] = make_uint2(e, 0u);
            const bool hit = live && !dense && (int64_t)ny < blk1;
            thit[j] = hit;
            tpos[j] = pos;
            tw[j] = c.w;
            tqi[j] = qi;
            tadm[j] = admits;
            const uint32_t pp = hit ? pos : 0u;
            tend[j] = (uint32_t)a.off[hit ? c.r + 1 : 0];
            t0[j] = a.post[pp];
            t1y[j] = a.post[pp + 1].y;  // the list array carries one padding entry
          } else if (k < tile_nnz) {
            const RComp c = a.qrc[qbase + k];
            const int qi = find_slot(qbase + k);
            bool admits = false;
            if constexpr (REM) admits = qbase + k - sm.qoff[qi] >= (int64_t)a.qadm[q0 + qi];
            const uint32_t pos = gcur[2 * k], ny = gcur[2 * k + 1];
            if (pos == kDead) {
              // no entry of this list in the item's range
            } else if (c.r < a.H) {
              const uint32_t e = hend[c.r];
              if (e > pos) {
                has_seg = true;
                sg.pos = pos;
                sg.lenq = (e - pos) | ((uint32_t)qi << 16);
                sg.q = q15(c.w) | (admits ? 0x80000000u : 0u);
                gcur[2 * k] = e;
              }
            } else if ((int64_t)ny < blk1) {
              thit[j] = true;
              tpos[j] = pos;
              tw[j] = c.w;
              tqi[j] = qi;
              tadm[j] = admits;
              tend[j] = (uint32_t)a.off[c.r + 1];
              t0[j] = a.post[pos];
              t1y[j] = a.post[pos + 1].y;
            }
          }
          sgj[j] = sg;
          sk[j] = !has_seg ? 0 : ((sg.lenq & 0xFFFFu) >= (uint32_t)kLongSeg ? 2 : 1);
        }
      };
      if (staged) pass1(std::integral_constant<bool, true>{});
      else pass1(std::integral_constant<bool, false>{});
      // the dense lists' segment ends of the next block, for staged tiles:
      // unconditional buffer loads (a component with none reads out of
      // range, which returns 0), so nothing waits on them before that block
      if (staged) {
        const __amdgpu_buffer_rsrc_t hrs = make_rsrc(hnext, b + 1 < b_end ? (uint32_t)a.H * 4u : 0u);
#pragma unroll
        for (int j = 0; j < KMAX; ++j) hn[j] = __builtin_amdgcn_raw_buffer_load_b32(hrs, (int)hq[j], 0, 0);
      }
      // Allocation: an exclusive scan over the threads of (long segments,
      // short segments, short entries) places long segments at the front of
      // seg[] (one wave each) and short ones, in thread order, at the back
      // (split evenly over all lanes), with their entry prefix sums and the
      // chunk table of the short stream.
      int nl, ns, L;
      Seg* sseg;
      {
        uint32_t cnt = 0u, len = 0u;  // long << 16 | short, short entries
#pragma unroll
        for (int j = 0; j < KMAX; ++j) {
          cnt += sk[j] == 2 ? 0x10000u : (sk[j] == 1 ? 1u : 0u);
          len += sk[j] == 1 ? (sgj[j].lenq & 0xFFFFu) : 0u;
        }
        uint32_t icnt = cnt, ilen = len;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
          const uint32_t uc = __shfl_up(icnt, o, 64);
          const uint32_t ul = __shfl_up(ilen, o, 64);
          if (lane >= o) {
            icnt += uc;
            ilen += ul;
          }
        }
        if (lane == 63) sm.wsum2[wave] = make_uint2(icnt, ilen);
        __syncthreads();
        // totals of the earlier waves, then of all waves (uniform loops:
        // no per-wave predicates to keep in registers)
        uint32_t wc = 0u, wl = 0u;
        for (int w = 0; w < wave; ++w) {
          const uint2 v = sm.wsum2[w];
          wc += v.x;
          wl += v.y;
        }
        uint32_t tc = wc, tl = wl;
        for (int w = wave; w < NW; ++w) {
          const uint2 v = sm.wsum2[w];
          tc += v.x;
          tl += v.y;
        }
        nl = (int)(tc >> 16);
        ns = (int)(tc & 0xFFFFu);
        L = (int)tl;
        sseg = sm.seg + (QB - ns);
        const uint32_t ec = wc + icnt - cnt;
        int lb = (int)(ec >> 16), sb = (int)(ec & 0xFFFFu), lp = (int)(wl + ilen - len);
        // without branches: every component stores its segment, prefix sum
        // and chunk-table entry, to a sink slot when it has none.  A short
        // segment holds fewer than 64 entries, so at most one chunk starts
        // inside it.
#pragma unroll
        for (int j = 0; j < KMAX; ++j) {
          const bool isl = sk[j] == 2, iss = sk[j] == 1;
          const int sl = iss ? (int)(sgj[j].lenq & 0xFFFFu) : 0;
          *(isl ? &sm.seg[lb] : (iss ? &sseg[sb] : &sm.seg_sink[lane])) = sgj[j];
          *(iss ? &sm.segpre[sb] : &sm.pre_sink[lane]) = lp;
          const int c = (lp + 63) & ~63;
          *((iss && c < lp + sl) ? &sm.ss.first[c >> 6] : &sm.first_sink[lane]) = (uint16_t)sb;
          lb += isl ? 1 : 0;
          sb += iss ? 1 : 0;
          lp += sl;
        }
        if (tid == 0) sm.segpre[ns] = L;
      }
      __syncthreads();
      if (tid == 0) c_visit += (unsigned long long)L;
      // pass 2: sparse lists, usually one entry per block (after the
      // allocation, whose barrier covers the first entries' loads; the
      // accumulation commutes with the streams, so no barrier follows)
#pragma unroll
      for (int j = 0; j < KMAX; ++j) {
        if (thit[j]) {
          const int64_t k = cb + (int64_t)j * NT + tid;
          uint32_t pos = tpos[j];
          const uint32_t end = tend[j];
          const int ab = tqi[j] * CB - (int)blk0;
          atomicAdd(&sm.acc[ab + (int)t0[j].y], fixp(tw[j], t0[j].w));
          if constexpr (REM)
            if (tadm[j]) admit_row((uint32_t)(t0[j].y - (uint32_t)blk0), tqi[j]);
          ++c_tail;
          ++pos;
          uint32_t ny = pos < end ? t1y[j] : 0xFFFFFFFFu;
          while ((int64_t)ny < blk1) {
            const Post p = a.post[pos];
            atomicAdd(&sm.acc[ab + (int)p.y], fixp(tw[j], p.w));
            if constexpr (REM)
              if (tadm[j]) admit_row((uint32_t)(p.y - (uint32_t)blk0), tqi[j]);
            ++c_tail;
            ++pos;
            ny = pos < end ? a.post[pos].y : 0xFFFFFFFFu;
          }
          if (staged) {
            sm.cur[k] = make_uint2(pos, ny);
          } else {
            gcur[2 * k] = pos;
            gcur[2 * k + 1] = ny;
          }
        }
      }
      // short segments: each wave takes a contiguous range of their visits;
      // every lane keeps U list loads in flight
      stream_short(sseg, ns, L, [&](int qi, uint32_t p, uint32_t qw, bool live) {
        // a lane past the slice adds zero to a slot of its row (no branch)
        atomicAdd(&sm.acc[qi * CB + (int)(p & (CB - 1))], live ? packed_product(qw, p) : 0u);
        if constexpr (REM)
          if (live && (qw >> 31)) admit_row(p & (uint32_t)(CB - 1), qi);
      });
      // long segments: wave w takes segments w, w + NW, ... in chunks of 64
      // entries (one per lane).  Lane i holds the descriptor of the wave's
      // segment i (64 at a time), which the walk reads with readlane: the
      // bookkeeping stays in scalar registers and needs no LDS access.  Two
      // batches of UL chunks alternate: the next batch's loads are issued
      // before the current batch is accumulated, so loads stay in flight.
      {
        const int nwl = nl > wave ? (nl - wave + NW - 1) / NW : 0;  // this wave's segments
        uint32_t dpos = 0u, dab = 0u, dq = 0u;  // lane i: segment j0 + i (byte offset, acc row, weight)
        int dlen = 0;
        auto load_desc = [&](int j0) {
          dlen = 0;
          if (j0 + lane < nwl) {
            const Seg S = sm.seg[wave + (j0 + lane) * NW];
            dpos = S.pos * 4u;
            dlen = (int)(S.lenq & 0xFFFFu);
            dab = (S.lenq >> 16) * (uint32_t)CB;
            dq = S.q;
            c_visit += (unsigned long long)dlen;
          }
        };
        int j = 0;     // segment being handed out
        int left = 0;  // its entries not yet handed out (<= 0: the wave is done)
        uint32_t soff = 0u, sab = 0u, sq = 0u;
        auto take = [&]() {  // j < nwl
          if ((j & 63) == 0) load_desc(j);
          const int l = j & 63;
          soff = (uint32_t)__builtin_amdgcn_readlane((int)dpos, l);
          left = __builtin_amdgcn_readlane(dlen, l);
          sab = (uint32_t)__builtin_amdgcn_readlane((int)dab, l);
          sq = (uint32_t)__builtin_amdgcn_readlane((int)dq, l);
        };
        if (nwl > 0) take();
        // next UL chunks (uniform values); chunks past the end have no entries
        auto gather = [&](uint32_t (&coff)[UL], uint32_t (&cq)[UL], int (&ccnt)[UL], uint32_t (&cab)[UL]) {
#pragma unroll
          for (int u = 0; u < UL; ++u) {
            ccnt[u] = left < 64 ? left : 64;
            coff[u] = left > 0 ? soff : 0u;
            cab[u] = sab;
            cq[u] = sq;
            soff += 256u;
            left -= 64;
            if (left <= 0 && j + 1 < nwl) {
              ++j;
              take();
            }
          }
        };
        // one buffer load per chunk: scalar base, lane offset; lanes past the
        // chunk read other entries, or the zero padding after the last list
        auto issue = [&](uint32_t (&p)[UL], const uint32_t (&coff)[UL]) {
#pragma unroll
          for (int u = 0; u < UL; ++u) p[u] = __builtin_amdgcn_raw_buffer_load_b32(prs, lane * 4, (int)coff[u], 0);
        };
        // lanes past the chunk add zero to a slot of the same accumulator row
        auto consume = [&](const uint32_t (&p)[UL], const uint32_t (&cq)[UL], const int (&ccnt)[UL],
                           const uint32_t (&cab)[UL]) {
#pragma unroll
          for (int u = 0; u < UL; ++u) {
            const uint32_t w = lane < ccnt[u] ? packed_product(cq[u], p[u]) : 0u;
            atomicAdd(&sm.acc[and_or(p[u], (uint32_t)(CB - 1), cab[u])], w);
            if constexpr (REM)
              if ((cq[u] >> 31) && lane < ccnt[u]) admit_row(p[u] & (uint32_t)(CB - 1), (int)(cab[u] / CB));
          }
        };
        uint32_t aoff[UL], aq[UL], pa[UL], boff[UL], bq[UL], pb[UL], aab[UL], bab[UL];
        int acnt[UL], bcnt[UL];
        gather(aoff, aq, acnt, aab);
        issue(pa, aoff);
        // (the scheduling barriers keep each batch's loads ahead of the
        // other batch's accumulation)
        for (;;) {
          if (acnt[0] <= 0) break;
          gather(boff, bq, bcnt, bab);
          issue(pb, boff);
          __builtin_amdgcn_sched_barrier(0);
          consume(pa, aq, acnt, aab);
          if (bcnt[0] <= 0) break;
          gather(aoff, aq, acnt, aab);
          issue(pa, aoff);
          __builtin_amdgcn_sched_barrier(0);
          consume(pb, bq, bcnt, bab);
        }
      }
      __syncthreads();
    }

    // A full block (every row inside the corpus and, in a self-join, before
    // the tile's first query) pairs every row with every slot: its copy of
    // the row loop has no per-slot limit to apply.
    const bool full_block = blk1 == blk0 + CB && (!a.triangle || blk0 + CB <= q0);
    auto filter_rows = [&](auto full_t) {
      constexpr bool FULL = decltype(full_t)::value;
#pragma unroll 1
      for (int yi = 0; yi < YPT; ++yi) {
        const RowStat st = stN;
        const int ylen = st.len;
        if (yi + 1 < YPT) load_rows(yi + 1);
        const int yl = yi * NT + tid;
        const int64_t y = blk0 + yl;
        // query slots qi >= qlo pair with this row: the triangle keeps the
        // pairs whose corpus row precedes the query
        int qlo = 0;
        if constexpr (!FULL) {
          if (y >= blk1) {
            qlo = QT;
          } else if (a.triangle) {
            const int64_t d = y - q0 + 1;
            qlo = d <= 0 ? 0 : (d >= QT ? QT : (int)d);
          }
        }
        const uint32_t packed = (uint32_t)(st.cut < 0xFFFF ? st.cut : 0xFFFF) |
                                ((uint32_t)(ylen < 0xFFFF ? ylen : 0xFFFF) << 16);
        const float ylf = (float)ylen, cutf = (float)st.cut;
        // slots beyond qn were never written and hold zeros
        uint32_t av[QT];
#pragma unroll
        for (int qi = 0; qi < QT; ++qi) av[qi] = sm.acc[qi * CB + yl];
        uint32_t abits = ~0u;  // remscore: slots whose candidate was admitted
        if constexpr (REM) {
          const uint32_t b = (uint32_t)yl * (uint32_t)QT;
          abits = sm.adm[b >> 5] >> (b & 31u);
        }
        // the candidates (live slots), and the row's largest score
        uint32_t lbits = 0u, amax = 0u;
#pragma unroll
        for (int qi = 0; qi < QT; ++qi) {
          bool live = FULL ? (av[qi] != 0u) : ((av[qi] != 0u) & (qi >= qlo));
          if constexpr (REM) live = live & (((abits >> qi) & 1u) != 0u);
          lbits |= live ? (1u << qi) : 0u;
          amax = max(amax, av[qi]);
        }
        uint32_t ncand = (uint32_t)__popc(lbits);
        // the bounds of all slots, without branches, unless no row of the
        // wave passes the row test (the usual case: survivors are rare);
        // the survivors are then queued slot by slot
        uint32_t wbits = 0u;
        const float2 rt = sm.rtest;
        if (__ballot((float)amax + rt.y * st.pnrm >= rt.x)) {
#pragma unroll
          for (int qi = 0; qi < QT; ++qi) {
            const float4 qb = sm.qb[qi];
            const bool live = (lbits >> qi) & 1u;
            const float A = (float)av[qi];  // accumulator units, as the bounds
            const bool want = live & (ylf * qb.y >= qb.x) & (A + min_nonneg(cutf * qb.y, qb.z) * st.pmw >= qb.x) &
                              (A + qb.w * st.pnrm >= qb.x);
            wbits |= want ? (1u << qi) : 0u;
          }
        }
        uint32_t keep = 0u;  // queue full: these slots stay for the next pass
        if (__ballot(wbits != 0u)) {
#pragma unroll
          for (int qi = 0; qi < QT; ++qi) {
            const bool want = (wbits >> qi) & 1u;
            const uint64_t wm = __ballot(want);
            if (wm) {
              int qb = 0;
              if (lane == 0) qb = atomicAdd(&sm.qcount, (int)__popcll(wm));
              qb = __shfl(qb, 0);
              if (want) {
                const int slot = qb + (int)__popcll(wm & lt);
                if (slot < SQ) {
                  sm.sq[slot] = make_uint4(((uint32_t)qi << 16) | (yoff + (uint32_t)yl), av[qi], 0u, packed);
                  ++c_surv;
                } else {
                  keep |= 1u << qi;
                  --ncand;
                  sm.ovf = 1;
                }
              }
            }
          }
        }
#pragma unroll
        for (int qi = 0; qi < QT; ++qi) sm.acc[qi * CB + yl] = ((keep >> qi) & 1u) ? av[qi] : 0u;
        c_cand += ncand;
      }
    };
    for (bool first = true;; first = false) {
      if (!first) load_rows(0);
      if (full_block) filter_rows(std::integral_constant<bool, true>{});
      else filter_rows(std::integral_constant<bool, false>{});
      __syncthreads();
      const int o = uni(sm.ovf);
      const int qc = uni(sm.qcount);
      __syncthreads();
      if (qc > 0 && (o || !defer || b + 1 == b_end || qc >= SQ / 2)) drain();
      if (!o) {
        clear_adm();
        break;
      }
    }
  }

  }  // ranges of the item
      if (tid == 0) sm.item = (int64_t)next_item;
    }  // items of queue x
  }    // queues

  // ------------------------------------------------------------ counters
  __syncthreads();
  atomicAdd(&sm.cnt[C_VISITS], c_visit);
  atomicAdd(&sm.cnt[C_TAILVISITS], c_tail);
  atomicAdd(&sm.cnt[C_CANDIDATES], c_cand);
  atomicAdd(&sm.cnt[C_SURVIVORS], c_surv);
  atomicAdd(&sm.cnt[C_VERIFIED], c_ver);
  atomicAdd(&sm.cnt[C_BAND], c_band);
  __syncthreads();
  if (tid < C_NUM && tid != C_MATCHES && sm.cnt[tid]) atomicAdd(&a.counters[tid], sm.cnt[tid]);
}

// toff[R * (m - H) + (r - H)] = first position in sparse list r whose vector
// id is >= R * range_rows.
__global__ void k_range_offsets(const int64_t* __restrict__ off, const Post* __restrict__ post, int32_t H, int64_t m,
                                int64_t nR, int64_t range_rows, uint32_t* __restrict__ toff) {
  const int64_t mt = m - H;
  const int64_t total = (nR + 1) * mt;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t R = e / mt;
    const int64_t r = H + (e - R * mt);
    int64_t lo = off[r], hi = off[r + 1];
    const uint64_t y0 = (uint64_t)R * (uint64_t)range_rows;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if ((uint64_t)post[mid].y < y0) lo = mid + 1;
      else hi = mid;
    }
    toff[e] = (uint32_t)lo;
  }
}

// Remscore (all-pairs-2, Section 3.2.2): a query's components are processed
// rarest first and admit new candidates while the remaining bound -- the sum
// of q_i * maxweight_i(V) over the components not yet processed, the current
// one included -- is at least t.  In rank space (densest first) that bound
// is the prefix sum up to the component, so the admitting components are
// those from the first position where the prefix sum reaches t onward.  The
// sum is taken in double over exact float products; the comparison is made
// against t less 1e-9, which only admits earlier.
__global__ void k_admit_pos(const int64_t* __restrict__ qrp, const RComp* __restrict__ qrc,
                            const float* __restrict__ mw_r, const float* __restrict__ qt, float t, int64_t nq,
                            int32_t* __restrict__ qadm) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nq; q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a0 = qrp[q], a1 = qrp[q + 1];
    const double tq = (double)(qt ? qt[q] : t) - 1e-9;
    double b = 0.0;
    int32_t pos = (int32_t)(a1 - a0);
    for (int64_t k = a0; k < a1; ++k) {
      const RComp c = qrc[k];
      b += (double)c.w * (double)mw_r[c.r];
      if (b >= tq) {
        pos = (int32_t)(k - a0);
        break;
      }
    }
    qadm[q] = pos;
  }
}

__global__ void k_max_tile_nnz(const int64_t* __restrict__ qrp, int64_t nq, int qt, unsigned long long* __restrict__ out) {
  const int64_t nt = (nq + qt - 1) / qt;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nt; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = (t + 1) * qt < nq ? (t + 1) * qt : nq;
    atomicMax(out, (unsigned long long)(qrp[e] - qrp[t * qt]));
  }
}

__global__ void k_unpack_pairs(const uint64_t* __restrict__ keys, const float* __restrict__ sim, int64_t cnt, int bj,
                               uint32_t* __restrict__ oi, uint32_t* __restrict__ oj, float* __restrict__ os) {
  const uint64_t jm = (1ull << bj) - 1;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < cnt; k += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t key = keys[k];
    oi[k] = (uint32_t)(key >> bj);
    oj[k] = (uint32_t)(key & jm);
    os[k] = sim[k];
  }
}

unsigned grid(int64_t n, int threads = 256) {
  int64_t g = (n + threads - 1) / threads;
  if (g > 32768) g = 32768;
  if (g < 1) g = 1;
  return (unsigned)g;
}

}  // namespace

hipError_t launch_unpack_pairs(const uint64_t* keys, const float* sim, int64_t cnt, int bj, uint32_t* oi, uint32_t* oj,
                               float* os, hipStream_t s) {
  if (cnt <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_unpack_pairs, dim3(grid(cnt)), dim3(256), 0, s, keys, sim, cnt, bj, oi, oj, os);
  return hipGetLastError();
}

// (queries per tile, corpus rows per block, threads, dense lookup ranks,
//  survivor queue, staged components, loads in flight for short / long
//  segments, waves per SIMD)
using V0 = Cfg<8, 2048, 512, 512, 1024, 1024, 8, 8, 2>;
using V1 = Cfg<8, 1024, 512, 128, 512, 1024, 4, 4, 4>;
using V2 = Cfg<16, 1024, 512, 256, 1024, 1536, 8, 8, 2>;
using V3 = Cfg<4, 2048, 256, 256, 512, 1024, 8, 8, 2>;

int join_num_variants() { return 4; }

int join_variant_staging(int v) {
  switch (v) {
    case 0: return V0::QB;
    case 1: return V1::QB;
    case 2: return V2::QB;
    case 3: return V3::QB;
    default: return 0;
  }
}

int join_variant_geometry(int v, int* qt, int* cb) {
  switch (v) {
    case 0: *qt = V0::QT; *cb = V0::CB; return 0;
    case 1: *qt = V1::QT; *cb = V1::CB; return 0;
    case 2: *qt = V2::QT; *cb = V2::CB; return 0;
    case 3: *qt = V3::QT; *cb = V3::CB; return 0;
    default: return -1;
  }
}

template <class C>
hipError_t launch_variant(const JoinArgs& a, int grid, hipStream_t s) {
  if (a.qadm)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_join<C, true>), dim3((unsigned)grid), dim3(C::NT), 0, s, a);
  else
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_join<C, false>), dim3((unsigned)grid), dim3(C::NT), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_join(const JoinArgs& a, int variant, int grid, hipStream_t s) {
  // variant 3 is withdrawn (see variant_available in the host library)
  if (variant == 3) return hipErrorInvalidValue;
  if (a.ntiles <= 0 || grid <= 0) return hipSuccess;
  switch (variant) {
    case 0: return launch_variant<V0>(a, grid, s);
    case 1: return launch_variant<V1>(a, grid, s);
    case 2: return launch_variant<V2>(a, grid, s);
    case 3: return launch_variant<V3>(a, grid, s);
    default: return hipErrorInvalidValue;
  }
}

template <class C>
int resident(int cus, bool rem) {
  int per_cu = 0;
  const void* f = rem ? reinterpret_cast<const void*>(&k_join<C, true>) : reinterpret_cast<const void*>(&k_join<C, false>);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, C::NT, 0) != hipSuccess || per_cu < 1) per_cu = 1;
  return per_cu * cus;
}

int join_resident_groups(int variant, bool remscore) {
  int dev = 0, cus = 0;
  (void)hipGetDevice(&dev);
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 1;
  switch (variant) {
    case 0: return resident<V0>(cus, remscore);
    case 1: return resident<V1>(cus, remscore);
    case 2: return resident<V2>(cus, remscore);
    case 3: return resident<V3>(cus, remscore);
    default: return cus;
  }
}

hipError_t launch_range_offsets(const int64_t* off, const Post* post, int32_t H, int64_t m, int64_t nR,
                                int64_t range_rows, uint32_t* toff, hipStream_t s) {
  const int64_t total = (nR + 1) * (m - H);
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_range_offsets, dim3(grid(total)), dim3(256), 0, s, off, post, H, m, nR, range_rows, toff);
  return hipGetLastError();
}

hipError_t launch_admit_pos(const int64_t* qrp, const RComp* qrc, const float* mw_r, const float* qt, float t,
                            int64_t nq, int32_t* qadm, hipStream_t s) {
  if (nq <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_admit_pos, dim3(grid(nq)), dim3(256), 0, s, qrp, qrc, mw_r, qt, t, nq, qadm);
  return hipGetLastError();
}

hipError_t launch_max_tile_nnz(const int64_t* qrp, int64_t nq, int qt, unsigned long long* out, hipStream_t s) {
  const int64_t nt = (nq + qt - 1) / qt;
  if (nt <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_max_tile_nnz, dim3(grid(nt)), dim3(256), 0, s, qrp, nq, qt, out);
  return hipGetLastError();
}

}  // namespace apss
