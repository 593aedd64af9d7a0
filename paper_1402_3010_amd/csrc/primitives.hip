// Device primitives: exclusive scan, stable LSD radix sort, fills.
// Wave64 throughout: ballots and shuffles assume 64 lanes (gfx950).
#include "apss_internal.h"

namespace apss {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanChunk = kScanThreads * kScanItems;

__device__ inline int64_t wave_incl_scan(int64_t v) {
  const int lane = __lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int64_t u = __shfl_up(v, o, 64);
    if (lane >= o) v += u;
  }
  return v;
}

// Exclusive scan of one chunk per block; block totals to sums.
__global__ __launch_bounds__(kScanThreads) void k_scan_chunk(int64_t* __restrict__ data, int64_t n,
                                                             int64_t* __restrict__ sums) {
  __shared__ int64_t wsum[kScanThreads / 64];
  const int tid = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)tid * kScanItems;
  int64_t v[kScanItems];
  int64_t run = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    int64_t idx = base + k;
    int64_t x = idx < n ? data[idx] : 0;
    v[k] = run;
    run += x;
  }
  int64_t incl = wave_incl_scan(run);
  const int wave = tid >> 6, lane = tid & 63;
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  int64_t woff = 0;
  for (int w = 0; w < wave; ++w) woff += wsum[w];
  int64_t excl = woff + incl - run;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    int64_t idx = base + k;
    if (idx < n) data[idx] = v[k] + excl;
  }
  if (tid == kScanThreads - 1) {
    int64_t tot = 0;
    for (int w = 0; w < kScanThreads / 64; ++w) tot += wsum[w];
    sums[blockIdx.x] = tot;
  }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_add(int64_t* __restrict__ data, int64_t n,
                                                           const int64_t* __restrict__ sums) {
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
  const int64_t add = sums[blockIdx.x];
  for (int k = threadIdx.x; k < kScanChunk; k += kScanThreads) {
    int64_t idx = base + k;
    if (idx < n) data[idx] += add;
  }
}

__global__ void k_scan_total(const int64_t* __restrict__ sums_scanned, const int64_t* __restrict__ sums_raw_last,
                             int64_t nb, int64_t* __restrict__ total) {
  // total = scanned[nb-1] + raw[nb-1]; raw value was saved before the sub-scan
  if (threadIdx.x == 0 && blockIdx.x == 0) *total = sums_scanned[nb - 1] + *sums_raw_last;
}

__global__ void k_copy1(const int64_t* __restrict__ src, int64_t* __restrict__ dst) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst = *src;
}

}  // namespace

int64_t scan_tmp_elems(int64_t n) {
  int64_t need = 0;
  while (n > 1) {
    int64_t nb = (n + kScanChunk - 1) / kScanChunk;
    need += nb + 1;
    n = nb;
  }
  return need + 2;
}

static __global__ void k_zero1(int64_t* __restrict__ dst) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst = 0;
}

// Recursive three-phase scan.  tmp layout per level: [sums (nb) | raw total of the last chunk (1)].
hipError_t exclusive_scan_i64(int64_t* data, int64_t n, int64_t* tmp, int64_t* total_dev, hipStream_t s) {
  if (n <= 0) {
    if (total_dev) hipLaunchKernelGGL(k_zero1, dim3(1), dim3(64), 0, s, total_dev);
    return hipGetLastError();
  }
  const int64_t nb = (n + kScanChunk - 1) / kScanChunk;
  int64_t* sums = tmp;
  int64_t* saved = tmp + nb;
  hipLaunchKernelGGL(k_scan_chunk, dim3((unsigned)nb), dim3(kScanThreads), 0, s, data, n, sums);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // keep the raw total of the last chunk so the grand total can be formed after the sub-scan
  hipLaunchKernelGGL(k_copy1, dim3(1), dim3(64), 0, s, sums + nb - 1, saved);
  if (nb > 1) {
    e = exclusive_scan_i64(sums, nb, tmp + nb + 1, nullptr, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(kScanThreads), 0, s, data, n, sums);
    if (total_dev) hipLaunchKernelGGL(k_scan_total, dim3(1), dim3(64), 0, s, sums, saved, nb, total_dev);
  } else if (total_dev) {
    hipLaunchKernelGGL(k_copy1, dim3(1), dim3(64), 0, s, saved, total_dev);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------- radix sort

namespace {

constexpr int kRsThreads = 256;
constexpr int kRsItems = 16;
constexpr int kRsTile = kRsThreads * kRsItems;
constexpr int kRsWaves = kRsThreads / 64;

__global__ __launch_bounds__(kRsThreads) void k_rs_hist(const uint64_t* __restrict__ keys, int64_t n, int shift,
                                                        int bits, int64_t nblk, int64_t* __restrict__ hist) {
  __shared__ uint32_t cnt[256];
  const int tid = threadIdx.x;
  cnt[tid] = 0;
  __syncthreads();
  const uint64_t mask = (1ull << bits) - 1;
  const int64_t base = (int64_t)blockIdx.x * kRsTile;
#pragma unroll 4
  for (int it = 0; it < kRsItems; ++it) {
    int64_t idx = base + (int64_t)it * kRsThreads + tid;
    if (idx < n) atomicAdd(&cnt[(keys[idx] >> shift) & mask], 1u);
  }
  __syncthreads();
  hist[(int64_t)tid * nblk + blockIdx.x] = cnt[tid];
}

template <typename V>
__global__ __launch_bounds__(kRsThreads) void k_rs_scatter(const uint64_t* __restrict__ kin, const V* __restrict__ vin,
                                                           uint64_t* __restrict__ kout, V* __restrict__ vout,
                                                           int64_t n, int shift, int bits, int64_t nblk,
                                                           const int64_t* __restrict__ hist) {
  __shared__ int64_t run[256];
  __shared__ uint32_t wc[kRsWaves][256];
  __shared__ uint32_t tot[256];
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  run[tid] = hist[(int64_t)tid * nblk + blockIdx.x];
  for (int w = 0; w < kRsWaves; ++w) wc[w][tid] = 0;
  __syncthreads();
  const uint64_t mask = (1ull << bits) - 1;
  const int64_t base = (int64_t)blockIdx.x * kRsTile;
  for (int it = 0; it < kRsItems; ++it) {
    const int64_t idx = base + (int64_t)it * kRsThreads + tid;
    const bool valid = idx < n;
    uint64_t k = 0;
    V v = V();
    uint32_t d = 0;
    if (valid) {
      k = kin[idx];
      v = vin[idx];
      d = (uint32_t)((k >> shift) & mask);
    }
    // lanes holding the same digit: refine the ballot of valid lanes bit by bit
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < bits; ++b) {
      const bool on = (d >> b) & 1u;
      const uint64_t m = __ballot(valid && on);
      peers &= on ? m : ~m;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & lt);
    if (valid && rank == 0) wc[wave][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    {
      uint32_t acc = 0;
      for (int w = 0; w < kRsWaves; ++w) {
        uint32_t c = wc[w][tid];
        wc[w][tid] = acc;
        acc += c;
      }
      tot[tid] = acc;
    }
    __syncthreads();
    if (valid) {
      const int64_t dst = run[d] + wc[wave][d] + rank;
      kout[dst] = k;
      vout[dst] = v;
    }
    __syncthreads();
    run[tid] += tot[tid];
    for (int w = 0; w < kRsWaves; ++w) wc[w][tid] = 0;
    __syncthreads();
  }
}

// Small inputs (n <= kSmallSort): one workgroup sorts in LDS with a bitonic
// network over (key << 13 | original index), so equal keys keep their input
// order (stable, like the radix passes) in one launch instead of four passes
// of three kernels each.  Keys are below 2^key_bits (every caller's keys are).
constexpr int kSmallSort = (int)kSortSegment;
constexpr int kSmallBits = 13;  // index bits

// seg == nullptr: one block sorts keys[0, n); else block b sorts the
// segment [seg[b], seg[b + 1]) (at most kSmallSort entries).
template <typename V>
__global__ __launch_bounds__(1024) void k_small_sort(uint64_t* __restrict__ keys, V* __restrict__ vals, int n,
                                                     const int64_t* __restrict__ seg) {
  __shared__ uint64_t ck[kSmallSort];
  __shared__ V ov[kSmallSort];
  const int tid = (int)threadIdx.x;
  if (seg) {
    const int64_t b0 = seg[blockIdx.x];
    n = (int)(seg[blockIdx.x + 1] - b0);
    keys += b0;
    vals += b0;
  }
  if (n <= 1) return;
  int n2 = 2;
  while (n2 < n) n2 <<= 1;
  for (int i = tid; i < n2; i += (int)blockDim.x) {
    if (i < n) {
      ck[i] = (keys[i] << kSmallBits) | (uint64_t)i;
      ov[i] = vals[i];
    } else {
      ck[i] = ~0ull;  // above every real entry
    }
  }
  __syncthreads();
  for (int size = 2; size <= n2; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = tid; i < n2 / 2; i += (int)blockDim.x) {
        const int lo = 2 * i - (i & (stride - 1));  // lower index of pair i, bit 'stride' clear
        const int hi = lo + stride;
        const bool up = (lo & size) == 0;
        const uint64_t x = ck[lo], y = ck[hi];
        if ((x > y) == up) {
          ck[lo] = y;
          ck[hi] = x;
        }
      }
      __syncthreads();
    }
  }
  for (int p = tid; p < n; p += (int)blockDim.x) {
    const uint64_t c = ck[p];
    keys[p] = c >> kSmallBits;
    vals[p] = ov[c & ((1u << kSmallBits) - 1u)];
  }
}

template <typename V>
hipError_t radix_sort_impl(uint64_t* keys, V* vals, uint64_t* ktmp, V* vtmp, int64_t n, int key_bits, int64_t* hist,
                           int64_t* scan_tmp, hipStream_t s) {
  if (n <= 1 || key_bits <= 0) return hipSuccess;
  if (n <= kSmallSort && key_bits <= 64 - kSmallBits) {
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_small_sort<V>), dim3(1), dim3(1024), 0, s, keys, vals, (int)n,
                       (const int64_t*)nullptr);
    return hipGetLastError();
  }
  const int64_t nblk = (n + kRsTile - 1) / kRsTile;
  uint64_t *ka = keys, *kb = ktmp;
  V *va = vals, *vb = vtmp;
  int passes = 0;
  for (int shift = 0; shift < key_bits; shift += 8) {
    const int bits = (key_bits - shift) < 8 ? (key_bits - shift) : 8;
    hipLaunchKernelGGL(k_rs_hist, dim3((unsigned)nblk), dim3(kRsThreads), 0, s, ka, n, shift, bits, nblk, hist);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = exclusive_scan_i64(hist, 256 * nblk, scan_tmp, nullptr, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_rs_scatter<V>), dim3((unsigned)nblk), dim3(kRsThreads), 0, s, ka, va, kb,
                       vb, n, shift, bits, nblk, hist);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    uint64_t* tk = ka; ka = kb; kb = tk;
    V* tv = va; va = vb; vb = tv;
    ++passes;
  }
  if (passes & 1) {
    hipError_t e = hipMemcpyAsync(keys, ka, sizeof(uint64_t) * n, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(vals, va, sizeof(V) * n, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void k_fill_u64(uint64_t* p, uint64_t v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

unsigned grid_for(int64_t n, int threads) {
  int64_t g = (n + threads - 1) / threads;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (unsigned)g;
}

}  // namespace

int64_t radix_hist_elems(int64_t n) { return 256 * ((n + kRsTile - 1) / kRsTile) + 1; }
int64_t radix_scan_tmp_elems(int64_t n) { return scan_tmp_elems(radix_hist_elems(n)); }

hipError_t radix_sort_u64(uint64_t* keys, uint64_t* vals, uint64_t* ktmp, uint64_t* vtmp, int64_t n, int key_bits,
                          int64_t* hist, int64_t* scan_tmp, hipStream_t s) {
  return radix_sort_impl<uint64_t>(keys, vals, ktmp, vtmp, n, key_bits, hist, scan_tmp, s);
}

hipError_t radix_sort_u64_u32(uint64_t* keys, uint32_t* vals, uint64_t* ktmp, uint32_t* vtmp, int64_t n, int key_bits,
                              int64_t* hist, int64_t* scan_tmp, hipStream_t s) {
  return radix_sort_impl<uint32_t>(keys, vals, ktmp, vtmp, n, key_bits, hist, scan_tmp, s);
}

hipError_t segment_sort_u64_u32(uint64_t* keys, uint32_t* vals, const int64_t* seg, int64_t nseg, hipStream_t s) {
  if (nseg <= 0) return hipSuccess;
  if (nseg > 0x7FFFFFFF) return hipErrorInvalidValue;
  hipLaunchKernelGGL(HIP_KERNEL_NAME(k_small_sort<uint32_t>), dim3((unsigned)nseg), dim3(1024), 0, s, keys, vals, 0,
                     seg);
  return hipGetLastError();
}

hipError_t fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (!p) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 256)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

namespace {

// 1 where a sorted key differs from its predecessor
__global__ void k_unique_flags(const uint64_t* __restrict__ keys, int64_t n, int64_t* __restrict__ flags) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    flags[k] = (k == 0 || keys[k] != keys[k - 1]) ? 1 : 0;
}

// first copy of each key (and its value) to its rank among the distinct keys
__global__ void k_unique_scatter(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ vals,
                                 const int64_t* __restrict__ pos, int64_t n, uint64_t* __restrict__ okeys,
                                 uint32_t* __restrict__ ovals) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    if (k == 0 || keys[k] != keys[k - 1]) {
      okeys[pos[k]] = keys[k];
      ovals[pos[k]] = vals[k];
    }
}

}  // namespace

hipError_t unique_sorted_u64_u32(uint64_t* keys, uint32_t* vals, int64_t n, int64_t* flags, int64_t* scan_tmp,
                                 int64_t* total_dev, uint64_t* ktmp, uint32_t* vtmp, hipStream_t s) {
  if (n <= 0) return exclusive_scan_i64(flags, 0, scan_tmp, total_dev, s);
  hipLaunchKernelGGL(k_unique_flags, dim3(grid_for(n, 256)), dim3(256), 0, s, keys, n, flags);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = exclusive_scan_i64(flags, n, scan_tmp, total_dev, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_unique_scatter, dim3(grid_for(n, 256)), dim3(256), 0, s, keys, vals, flags, n, ktmp, vtmp);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(keys, ktmp, sizeof(uint64_t) * n, hipMemcpyDeviceToDevice, s)) != hipSuccess) return e;
  return hipMemcpyAsync(vals, vtmp, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, s);
}

hipError_t fill_u64(uint64_t* p, uint64_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (!p) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n, 256)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

}  // namespace apss
