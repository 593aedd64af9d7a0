// Internal declarations of the apss library (gfx950).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

namespace apss {

// One component of a vector in rank space: the dimension's position in the
// density order (0 = densest) and the weight.
struct RComp {
  int32_t r;
  float w;
};

// One inverted-list entry: vector id and weight.
struct Post {
  uint32_t y;
  float w;
};

// Per-vector data used by the bounds of Section 3.2.2:
//   cut  = |x'|, the number of unindexed leading components;
//   len  = |x|, the number of components;
//   pmw  = maxweight(x');
//   pnrm = ||x'||_2 rounded up to float.
struct RowStat {
  int32_t cut;
  int32_t len;
  float pmw;
  float pnrm;
};

// One-byte upper bound of a row's unindexed-part norm: code k < 255 means
// pnrm <= k / 254; kPn8None means no bound.
constexpr uint8_t kPn8None = 255;

// Counters written by the join kernels (uint64 slots).
enum Counter {
  C_VISITS = 0,
  C_CANDIDATES,
  C_SURVIVORS,
  C_VERIFIED,
  C_BAND,
  C_MATCHES,   // pairs emitted (may exceed the output capacity)
  C_TAILVISITS,
  C_NUM = 8
};

// Fixed-point scale of the accumulators: scores are sums of products in
// (0, 1] and never exceed 1 + O(k 2^-30) by Cauchy-Schwarz, so 2^30 units
// fit an unsigned 32-bit word.
constexpr float kFix = 1073741824.0f;
constexpr float kInvFix = 1.0f / 1073741824.0f;

// Decision band of the float rescore (a pair whose float score is within
// this distance of t is rescored in double).
constexpr float kBand = 1e-5f;
// Slack of the pruning tests evaluated on accumulated float / fixed-point
// partial scores; well above their worst-case rounding error.
constexpr float kSlack = 1e-4f;

// ---------------------------------------------------------------- errors
std::string& last_error();
void set_error(const char* fmt, ...);

#define APSS_HIP(call)                                                                          \
  do {                                                                                          \
    hipError_t e_ = (call);                                                                     \
    if (e_ != hipSuccess) {                                                                     \
      ::apss::set_error("%s:%d %s: %s", __FILE__, __LINE__, #call, hipGetErrorString(e_));       \
      return APSS_EDEVICE;                                                                      \
    }                                                                                           \
  } while (0)

// ---------------------------------------------------------------- primitives
// Exclusive scan of int64 values in place (n entries); returns the total.
// tmp must hold scan_tmp_elems(n) int64.
int64_t scan_tmp_elems(int64_t n);
hipError_t exclusive_scan_i64(int64_t* data, int64_t n, int64_t* tmp, int64_t* total_dev, hipStream_t s);

// Stable sort of (key, value) pairs by key; keys must be below 2^key_bits.
// LSD radix passes over 8-bit digits, or for up to 8,192 pairs with at most
// 51 key bits one workgroup in LDS.  Sorted result ends in keys/vals;
// ktmp/vtmp are equal-sized scratch.
// hist must hold radix_hist_elems(n) int64.
int64_t radix_hist_elems(int64_t n);
int64_t radix_scan_tmp_elems(int64_t n);
hipError_t radix_sort_u64(uint64_t* keys, uint64_t* vals, uint64_t* ktmp, uint64_t* vtmp, int64_t n,
                          int key_bits, int64_t* hist, int64_t* scan_tmp, hipStream_t s);
hipError_t radix_sort_u64_u32(uint64_t* keys, uint32_t* vals, uint64_t* ktmp, uint32_t* vtmp, int64_t n,
                              int key_bits, int64_t* hist, int64_t* scan_tmp, hipStream_t s);
// Independent stable sorts of the segments [seg[b], seg[b + 1]), b < nseg,
// each of at most kSortSegment pairs (keys below 2^51), one workgroup each.
constexpr int64_t kSortSegment = 8192;
hipError_t segment_sort_u64_u32(uint64_t* keys, uint32_t* vals, const int64_t* seg, int64_t nseg, hipStream_t s);

// Keep the first of each run of equal keys of a sorted (key, value) array,
// in place: the distinct pairs end in keys/vals[0, *total_dev).  flags holds
// n int64, scan_tmp scan_tmp_elems(n), ktmp/vtmp n entries.
hipError_t unique_sorted_u64_u32(uint64_t* keys, uint32_t* vals, int64_t n, int64_t* flags, int64_t* scan_tmp,
                                 int64_t* total_dev, uint64_t* ktmp, uint32_t* vtmp, hipStream_t s);

// Fill helpers (graph-safe kernels rather than memset nodes).
hipError_t fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);
hipError_t fill_u64(uint64_t* p, uint64_t v, int64_t n, hipStream_t s);

inline int ceil_log2(uint64_t x) {
  int b = 0;
  while ((1ull << b) < x) ++b;
  return b;
}

}  // namespace apss
