// Final score of a verified pair, shared by every kernel that reports
// pairs, so that a pair's reported similarity does not depend on the path
// that found it.
//
// One wavefront scores one pair (y, q): lane l takes the components
// l, l + 64, ... of row y (rank order) and looks up q's weight in the same
// dimension.  Products and sums are compensated (error-free product by FMA,
// TwoSum; the Dot2 scheme of Ogita, Rump and Oishi 2005) and the 64 lane
// results are combined by a fixed xor butterfly, so the value is a function
// of the two rows only.  Its error is below (ceil(k/64) + 7) 2^-24 for k
// components, well inside the 1e-5 band in which the caller decides by the
// double-precision sum instead.
#pragma once

#include "apss_internal.h"

namespace apss {

__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
  s = __fadd_rn(a, b);
  const float z = __fsub_rn(s, a);
  e = __fadd_rn(__fsub_rn(a, __fsub_rn(s, z)), __fsub_rn(b, z));
}

// Compensated float dot product of row y (ylen components) with the query
// whose weight in rank r is look(r) (0 when absent).  Same value on every lane.
template <class Lookup>
__device__ __forceinline__ float wave_dot2(const RComp* __restrict__ y, int ylen, int lane, Lookup look) {
  float hi = 0.0f, lo = 0.0f;
  for (int k = lane; k < ylen; k += 64) {
    const RComp c = y[k];
    const float qv = look(c.r);
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
  return __fadd_rn(hi, lo);
}

// The same dot product in double (products of floats are exact in double).
template <class Lookup>
__device__ __forceinline__ double wave_dot64(const RComp* __restrict__ y, int ylen, int lane, Lookup look) {
  double d = 0.0;
  for (int k = lane; k < ylen; k += 64) {
    const RComp c = y[k];
    d += (double)look(c.r) * (double)c.w;
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) d += __shfl_xor(d, o, 64);
  return d;
}

// Decision and reported value for a pair with float score s32 and threshold
// tq: outside the band the float score decides; inside it the double sum.
// Returns true to keep; *sim receives the value to report.  Wave-uniform.
template <class Lookup>
__device__ __forceinline__ bool wave_decide(const RComp* __restrict__ y, int ylen, int lane, Lookup look, float s32,
                                            float tq, float* sim, bool* banded) {
  if (fabsf(s32 - tq) <= kBand) {
    const double d = wave_dot64(y, ylen, lane, look);
    *sim = (float)d;
    *banded = true;
    return d >= (double)tq;
  }
  *sim = s32;
  *banded = false;
  return s32 >= tq;
}

// Pair compaction of one wavefront: the wave's kept pairs wait in its lanes
// (the k-th in lane k) and are written at consecutive output positions
// reserved by one counter atomic per flush, at most 64 pairs at a time.
// add() and flush() are called by every lane of the wave with the same
// arguments (the decisions above are wave-uniform).  The counter still
// counts pairs past the capacity, whose writes are dropped.
struct WaveEmit {
  uint64_t key = 0;
  float sim = 0.0f;
  int n = 0;  // pairs held; wave-uniform, at most 64
  __device__ __forceinline__ void add(int lane, uint64_t k, float s) {
    if (lane == n) {
      key = k;
      sim = s;
    }
    ++n;
  }
  __device__ __forceinline__ void flush(int lane, unsigned long long* counters, uint64_t* __restrict__ out_key,
                                        float* __restrict__ out_sim, int64_t cap) {
    if (n == 0) return;
    unsigned long long b = 0;
    if (lane == 0) b = atomicAdd(&counters[C_MATCHES], (unsigned long long)n);
    b = (unsigned long long)__shfl((long long)b, 0, 64);
    const int64_t k = (int64_t)b + lane;
    if (lane < n && k < cap) {
      out_key[k] = key;
      out_sim[k] = sim;
    }
    n = 0;
  }
};

}  // namespace apss
