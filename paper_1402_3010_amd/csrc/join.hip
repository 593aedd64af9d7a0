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
//     (the upperbound test of all-pairs-2), and the L2 bound A + ||y'|| >= t
//     (Cauchy-Schwarz, ||q|| = 1); all with a small slack.
//  3. verify survivors: s = A + dot(q, y') (one lane per survivor).
//  4. rescore verified pairs over the full rows in float with compensated
//     products and sums (Ogita, Rump and Oishi 2005, Dot2) in a fixed
//     lane-strided order and a fixed butterfly, so the result depends only on
//     (q, y); if it lies within kBand of t the pair is decided by a double
//     rescore.  Emitted pairs are compacted per wave (ballot + prefix).
#include "apss_internal.h"
#include "join.h"

namespace apss {

namespace {

__device__ __forceinline__ uint32_t fixp(float a, float b) { return __float2uint_ru(__fmul_rn(a, b) * kFix); }

__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
  s = __fadd_rn(a, b);
  const float z = __fsub_rn(s, a);
  e = __fadd_rn(__fsub_rn(a, __fsub_rn(s, z)), __fsub_rn(b, z));
}

template <int QT, int CB, int NT, int RD, int SQ, int QB>
struct Smem {
  uint32_t acc[QT * CB];
  float qd[QT * RD];
  int4 seg[NT];  // x = first list position, y = length, z = query weight bits, w = query slot
  int32_t segpre[NT + 1];
  uint2 sq[SQ];  // x = slot * CB + local y, y = fixed-point score (0 = dropped)
  RComp qrow[QB];
  int64_t qoff[QT + 1];
  float qmw[QT];
  float qt[QT];
  int32_t qlen[QT];
  int32_t qhead[QT];
  int32_t wsum[NT / 64];
  int32_t nseg;
  int32_t qcount;
  int32_t ovf;
  int32_t staged;
  unsigned long long cnt[C_NUM];
};

template <int QT, int CB, int NT, int RD, int SQ, int QB>
__global__ __launch_bounds__(NT) void k_join(JoinArgs a) {
  constexpr int NW = NT / 64;
  using S = Smem<QT, CB, NT, RD, SQ, QB>;
  __shared__ S sm;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

  const int64_t tile = a.ntiles - 1 - (int64_t)blockIdx.x;  // heaviest tiles first
  const int64_t q0 = tile * QT;
  const int qn = (int)((a.nq - q0) < QT ? (a.nq - q0) : QT);

  if (tid <= qn) sm.qoff[tid] = a.qrp[q0 + tid];
  if (tid < QT) {
    sm.qmw[tid] = tid < qn ? a.qmw[q0 + tid] : 0.0f;
    sm.qt[tid] = (tid < qn && a.qt) ? a.qt[q0 + tid] : a.t;
  }
  if (tid < C_NUM) sm.cnt[tid] = 0;
  if (tid == 0) {
    sm.nseg = 0;
    sm.qcount = 0;
    sm.ovf = 0;
  }
  for (int e = tid; e < QT * RD; e += NT) sm.qd[e] = 0.0f;
  for (int e = tid; e < QT * CB; e += NT) sm.acc[e] = 0u;
  __syncthreads();
  const int64_t qbase = sm.qoff[0];
  const int64_t tile_nnz = sm.qoff[qn] - qbase;
  const bool staged = tile_nnz <= QB;
  if (tid < qn) {
    const int64_t r0 = sm.qoff[tid], r1 = sm.qoff[tid + 1];
    sm.qlen[tid] = (int32_t)(r1 - r0);
    int64_t lo = r0, hi = r1;  // first component with rank >= RD
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (a.qrc[mid].r < RD) lo = mid + 1;
      else hi = mid;
    }
    sm.qhead[tid] = (int32_t)(lo - r0);
  }
  auto find_slot = [&](int64_t k) {
    int qi = 0;
    while (qi + 1 < qn && sm.qoff[qi + 1] <= k) ++qi;
    return qi;
  };
  for (int64_t k = tid; k < tile_nnz; k += NT) {
    const RComp c = a.qrc[qbase + k];
    if (staged) sm.qrow[k] = c;
    if (c.r < RD) sm.qd[find_slot(qbase + k) * RD + c.r] = c.w;
  }
  __syncthreads();

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

  unsigned long long c_visit = 0, c_tail = 0, c_cand = 0, c_surv = 0, c_ver = 0, c_band = 0;

  int64_t last_b = -1;
  if (qn > 0 && a.n > 0) last_b = a.triangle ? (q0 + qn - 1) / CB : (a.nb - 1);

  for (int64_t b = 0; b <= last_b; ++b) {
    const int64_t blk0 = b * CB;
    const int64_t blk1 = (blk0 + CB) < a.n ? (blk0 + CB) : a.n;
    const uint32_t* hb = a.hoff + b * (int64_t)a.H;

    // ------------------------------------------------------------ accumulate
    for (int64_t cb = 0; cb < tile_nnz; cb += NT) {
      const int64_t k = cb + tid;
      bool has_seg = false;
      int4 sg = make_int4(0, 0, 0, 0);
      if (k < tile_nnz) {
        const int64_t kk = qbase + k;
        const RComp c = staged ? sm.qrow[k] : a.qrc[kk];
        const int qi = find_slot(kk);
        if (c.r < a.H) {
          const uint32_t s0 = hb[c.r], s1 = hb[a.H + c.r];
          if (s1 > s0) {
            has_seg = true;
            sg = make_int4((int)s0, (int)(s1 - s0), __float_as_int(c.w), qi);
          }
        } else {
          uint2 cu = a.cur[kk];
          if ((int64_t)cu.y < blk1) {
            uint32_t pos = cu.x;
            const uint32_t end = (uint32_t)a.off[c.r + 1];
            uint32_t ny = cu.y;
            do {
              const float pw = a.post[pos].w;
              atomicAdd(&sm.acc[qi * CB + (int)(ny - (uint32_t)blk0)], fixp(c.w, pw));
              ++c_tail;
              ++pos;
              ny = pos < end ? a.post[pos].y : 0xFFFFFFFFu;
            } while ((int64_t)ny < blk1);
            a.cur[kk] = make_uint2(pos, ny);
          }
        }
      }
      const uint64_t m = __ballot(has_seg);
      int sbase = 0;
      if (lane == 0 && m) sbase = atomicAdd(&sm.nseg, (int)__popcll(m));
      sbase = __shfl(sbase, 0);
      if (has_seg) sm.seg[sbase + (int)__popcll(m & lt)] = sg;
      __syncthreads();
      const int ns = sm.nseg;
      // exclusive scan of segment lengths
      {
        const int len = tid < ns ? sm.seg[tid].y : 0;
        int incl = len;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
          const int u = __shfl_up(incl, o, 64);
          if (lane >= o) incl += u;
        }
        if (lane == 63) sm.wsum[wave] = incl;
        __syncthreads();
        int woff = 0;
        for (int w = 0; w < wave; ++w) woff += sm.wsum[w];
        if (tid < ns) sm.segpre[tid] = woff + incl - len;
        if (tid == NT - 1) sm.segpre[ns] = woff + incl;
      }
      __syncthreads();
      if (tid == 0) sm.nseg = 0;
      const int L = sm.segpre[ns];
      if (tid == 0) c_visit += (unsigned long long)L;
      {
        const int per = (((L + NW - 1) / NW) + 63) & ~63;
        const int vbeg = wave * per;
        const int vend = (vbeg + per) < L ? (vbeg + per) : L;
        if (vbeg < vend) {
          int lo = 0, hi = ns - 1;  // last segment starting at or before vbeg
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (sm.segpre[mid] <= vbeg) lo = mid;
            else hi = mid - 1;
          }
          int s = lo, cs = -1, pre = 0;
          int4 S = make_int4(0, 0, 0, 0);
          for (int base = vbeg; base < vend; base += 64) {
            const int v = base + lane;
            if (v < vend) {
              while (sm.segpre[s + 1] <= v) ++s;
              if (s != cs) {
                S = sm.seg[s];
                pre = sm.segpre[s];
                cs = s;
              }
              const Post p = a.post[(uint32_t)S.x + (uint32_t)(v - pre)];
              atomicAdd(&sm.acc[S.w * CB + (int)(p.y - (uint32_t)blk0)], fixp(__int_as_float(S.z), p.w));
            }
          }
        }
      }
      __syncthreads();
    }

    // ------------------------------------------------------------ filter, verify, rescore
    auto drain = [&]() {
      const int ns = sm.qcount < SQ ? sm.qcount : SQ;
      // verify: one lane per survivor, s = A + dot(q, y')
      for (int e = tid; e < ns; e += NT) {
        const uint2 it = sm.sq[e];
        const int qi = (int)(it.x / CB);
        const int64_t y = blk0 + (int64_t)(it.x % CB);
        const int64_t ys = a.rp[y];
        const int cut = a.rs[y].cut;
        float s = (float)it.y * kInvFix;
        for (int k = 0; k < cut; ++k) {
          const RComp c = a.rc[ys + k];
          s += qlookup(qi, c.r) * c.w;
        }
        if (s >= sm.qt[qi] - kSlack) ++c_ver;
        else sm.sq[e].y = 0u;
      }
      __syncthreads();
      // rescore: one wave per verified pair
      for (int base = wave * 64; base < ns; base += NT) {
        const int e = base + lane;
        uint64_t fm = __ballot(e < ns && sm.sq[e < ns ? e : 0].y != 0u);
        while (fm) {
          const int l = __ffsll((unsigned long long)fm) - 1;
          fm &= fm - 1;
          const uint2 it = sm.sq[base + l];
          const int qi = (int)(it.x / CB);
          const int64_t y = blk0 + (int64_t)(it.x % CB);
          const int64_t ys = a.rp[y];
          const int ylen = (int)(a.rp[y + 1] - ys);
          float hi = 0.0f, lo = 0.0f;
          for (int k = lane; k < ylen; k += 64) {
            const RComp c = a.rc[ys + k];
            const float qv = qlookup(qi, c.r);
            const float p = __fmul_rn(qv, c.w);
            const float ep = __fmaf_rn(qv, c.w, -p);
            float s2, es;
            two_sum(hi, p, s2, es);
            hi = s2;
            lo = __fadd_rn(lo, __fadd_rn(es, ep));
          }
#pragma unroll
          for (int o = 32; o >= 1; o >>= 1) {
            const float h2 = __shfl_xor(hi, o, 64);
            const float l2 = __shfl_xor(lo, o, 64);
            float s2, e2;
            two_sum(hi, h2, s2, e2);
            hi = s2;
            lo = __fadd_rn(__fadd_rn(lo, l2), e2);
          }
          const float s32 = __fadd_rn(hi, lo);
          const float tq = sm.qt[qi];
          bool keep;
          float sim;
          if (fabsf(s32 - tq) <= kBand) {
            double d = 0.0;
            for (int k = lane; k < ylen; k += 64) {
              const RComp c = a.rc[ys + k];
              d += (double)qlookup(qi, c.r) * (double)c.w;
            }
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) d += __shfl_xor(d, o, 64);
            keep = d >= (double)tq;
            sim = (float)d;
            if (lane == 0) ++c_band;
          } else {
            keep = s32 >= tq;
            sim = s32;
          }
          if (keep && lane == 0) {
            const uint64_t qid = (uint64_t)(q0 + qi);
            const uint64_t key = a.triangle ? (((uint64_t)y << a.bj) | qid) : ((qid << a.bj) | (uint64_t)y);
            const unsigned long long idx = atomicAdd(&a.counters[C_MATCHES], 1ull);
            if ((int64_t)idx < a.cap) {
              a.out_key[idx] = key;
              a.out_sim[idx] = sim;
            }
          }
        }
      }
      __syncthreads();
      if (tid == 0) {
        sm.qcount = 0;
        sm.ovf = 0;
      }
      __syncthreads();
    };

    for (int yb = 0; yb < CB; yb += NT) {
      const int yl = yb + tid;
      const int64_t y = blk0 + yl;
      const bool yv = y < blk1;
      RowStat st = {0, 0.0f, 0.0f, 0.0f};
      int ylen = 0;
      if (yv) {
        st = a.rs[y];
        ylen = (int)(a.rp[y + 1] - a.rp[y]);
      }
      for (;;) {
        for (int qi = 0; qi < qn; ++qi) {
          const int e = qi * CB + yl;
          const uint32_t av = sm.acc[e];
          bool want = false;
          if (av) {
            if (!yv || (a.triangle && y >= q0 + qi)) {
              sm.acc[e] = 0u;
            } else {
              const float A = (float)av * kInvFix;
              const float thr = sm.qt[qi] - kSlack;
              const float qm = sm.qmw[qi];
              const float mn = (float)(st.cut < sm.qlen[qi] ? st.cut : sm.qlen[qi]);
              const bool ok = ((float)ylen * qm >= thr) && (A + mn * qm * st.pmw >= thr) && (A + st.pnrm >= thr);
              if (ok) {
                want = true;
              } else {
                sm.acc[e] = 0u;
                ++c_cand;
              }
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
                sm.sq[slot] = make_uint2((uint32_t)(qi * CB + yl), av);
                sm.acc[e] = 0u;
                ++c_cand;
                ++c_surv;
              } else {
                sm.ovf = 1;
              }
            }
          }
        }
        __syncthreads();
        const int o = sm.ovf;
        const int qc = sm.qcount;
        __syncthreads();
        if (o || qc >= SQ / 2 || (yb + NT >= CB && qc > 0)) drain();
        if (!o) break;
      }
    }
  }

  // ------------------------------------------------------------ counters
  atomicAdd(&sm.cnt[C_VISITS], c_visit);
  atomicAdd(&sm.cnt[C_TAILVISITS], c_tail);
  atomicAdd(&sm.cnt[C_CANDIDATES], c_cand);
  atomicAdd(&sm.cnt[C_SURVIVORS], c_surv);
  atomicAdd(&sm.cnt[C_VERIFIED], c_ver);
  atomicAdd(&sm.cnt[C_BAND], c_band);
  __syncthreads();
  if (tid < C_NUM && tid != C_MATCHES && sm.cnt[tid]) atomicAdd(&a.counters[tid], sm.cnt[tid]);
}

// Tail cursors: first entry of each sparse list a query component reads.
__global__ void k_init_cursors(const RComp* __restrict__ qrc, int64_t qnnz, const int64_t* __restrict__ off,
                               const Post* __restrict__ post, int32_t H, uint2* __restrict__ cur) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < qnnz; k += (int64_t)gridDim.x * blockDim.x) {
    const int32_t r = qrc[k].r;
    if (r < H) continue;
    const int64_t p0 = off[r], p1 = off[r + 1];
    cur[k] = make_uint2((uint32_t)p0, p0 < p1 ? post[p0].y : 0xFFFFFFFFu);
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

hipError_t launch_init_cursors(const RComp* qrc, int64_t qnnz, const int64_t* off, const Post* post, int32_t H,
                               uint2* cur, hipStream_t s) {
  if (qnnz <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_init_cursors, dim3(grid(qnnz)), dim3(256), 0, s, qrc, qnnz, off, post, H, cur);
  return hipGetLastError();
}

hipError_t launch_unpack_pairs(const uint64_t* keys, const float* sim, int64_t cnt, int bj, uint32_t* oi, uint32_t* oj,
                               float* os, hipStream_t s) {
  if (cnt <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_unpack_pairs, dim3(grid(cnt)), dim3(256), 0, s, keys, sim, cnt, bj, oi, oj, os);
  return hipGetLastError();
}

// Tile and block geometry of the compiled variant.
constexpr int kQT = 8;
constexpr int kCB = 2048;
constexpr int kNT = 512;
constexpr int kRD = 512;
constexpr int kSQ = 2048;
constexpr int kQB = 2048;

int join_tile_queries() { return kQT; }
int join_block_rows() { return kCB; }

hipError_t launch_join(const JoinArgs& a, hipStream_t s) {
  if (a.ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(HIP_KERNEL_NAME(k_join<kQT, kCB, kNT, kRD, kSQ, kQB>), dim3((unsigned)a.ntiles), dim3(kNT), 0, s,
                     a);
  return hipGetLastError();
}

}  // namespace apss
