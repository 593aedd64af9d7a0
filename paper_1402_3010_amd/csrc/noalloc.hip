// Self-join that allocates no device memory: apss_join_device_noalloc.
//
// For callers that cannot allocate during the call (code under stream
// capture, tight serving loops, harnesses that forbid allocation).  The
// work is that of apss_join_device on a plain index -- the same join kernel,
// pair sort and unpack -- but every scratch buffer of the call (queue
// counters, query tiles and work queues, per-workgroup cursors, raw pairs,
// sort scratch) is carved out of one fixed device array, `scratch`, which
// each device holds from the library's load until the process ends.
//
// In host code the array's name is not a device address; its address on a
// device comes from hipGetSymbolAddress, taken once per device with that
// device current, and only that address is ever passed to kernels or copies.
// Every call on a device shares its array, which keeps the last call's
// contents: the counters and queue heads are cleared by fill kernels at
// every call, and calls that overlap on one device race.
#include <string.h>

#include <algorithm>
#include <mutex>

#include "apss_internal.h"
#include "join.h"
#include "lib.h"

namespace apss {
namespace {

constexpr size_t kScratchBytes = (size_t)APSS_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kMaxDevices] = {};

// Device address of the scratch array on device dev (current), taken once.
int scratch_on(int dev, unsigned char** out) {
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device ordinal %d outside [0, %d)", dev, kMaxDevices);
    return APSS_EINVAL;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return dev_err(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = (unsigned char*)p;
  }
  *out = g_scratch_ptr[dev];
  return APSS_OK;
}

// Bump placement of buffers in the scratch array, 256-byte aligned.
struct Carve {
  unsigned char* base;
  size_t used = 0;
  template <class T>
  T* take(int64_t count) {
    T* p = (T*)(base + used);
    used += bytes<T>(count);
    return p;
  }
  template <class T>
  static size_t bytes(int64_t count) {
    const size_t b = sizeof(T) * (size_t)(count > 0 ? count : 1);
    return (b + 255) & ~(size_t)255;
  }
};

// Scratch bytes of the pair stage for room pairs: raw keys and sims, the
// sort's second buffers, its histograms and scan scratch.
size_t pair_bytes(int64_t room) {
  return Carve::bytes<uint64_t>(room) + Carve::bytes<float>(room) + Carve::bytes<uint64_t>(room) +
         Carve::bytes<uint32_t>(room) + Carve::bytes<int64_t>(radix_hist_elems(room)) +
         Carve::bytes<int64_t>(radix_scan_tmp_elems(room));
}

}  // namespace
}  // namespace apss

using namespace apss;

extern "C" int apss_join_device_noalloc(apss_index* ix, float t, uint32_t* out_i, uint32_t* out_j, float* out_sim,
                                        int64_t capacity, int64_t* count) {
  if (!ix || !count || capacity < 0 || (capacity > 0 && (!out_i || !out_j || !out_sim))) {
    set_error("NULL or invalid argument");
    return APSS_EINVAL;
  }
  *count = 0;
  int rc = check_t(ix, t);
  if (rc) return rc;
  if (ix->screen || ix->parts > 1 || ix->opts.remscore) {
    set_error("the allocation-free join serves indexes built without screen_dims, local_parts or remscore");
    return APSS_EINVAL;
  }
  int dev = -1;
  APSS_CHK(hipGetDevice(&dev), "hipGetDevice");
  if (dev != ix->device) {
    set_error("called on device %d; the index lives on device %d", dev, ix->device);
    return APSS_EINVAL;
  }
  Workspace& ws = ix->ws;
  hipStream_t s = ws.stream;
  memset(&ws.last, 0, sizeof(ws.last));
  if (ix->n == 0) return APSS_OK;

  // the lookup tables of the index's geometry were made at build time (and
  // by apss_autotune); nothing here may make them
  int qt = 0, cb = 0;
  if (join_variant_geometry(ix->variant, &qt, &cb)) {
    set_error("unknown join variant %d", ix->variant);
    return APSS_EINVAL;
  }
  const int64_t rr = std::max<int64_t>(1, ix->range_rows / cb) * cb;
  const int slot = cb == 1024 ? 0 : 1;
  if (!ix->hoff[slot].p || !ix->toff.p || ix->toff_rows != rr || ix->grid[ix->variant] <= 0) {
    set_error("the index's join tables for its tile variant and range width are not ready");
    return APSS_EINVAL;
  }
  for (int e = 0; e < 6; ++e)
    if (!ws.ev[e]) {
      set_error("the index's timers are missing");
      return APSS_EINVAL;
    }

  unsigned char* base = nullptr;
  if ((rc = scratch_on(dev, &base))) return rc;

  const QuerySet Q{ix->rows.rp.p, ix->rows.rc.p, ix->rows.mw.p, ix->n, ix->nnz, ix->rows.rp_host.data()};
  JoinLayout L;
  if ((rc = plan_layout(ix, Q, 1, L))) return rc;
  const size_t fixed = Carve::bytes<unsigned long long>(C_NUM) + Carve::bytes<unsigned int>(8) +
                       Carve::bytes<int64_t>(L.ntiles + 1) + Carve::bytes<int64_t>((int64_t)L.cum.size()) +
                       Carve::bytes<uint32_t>((int64_t)L.G * L.wg_stride);
  if (fixed + pair_bytes(0) > kScratchBytes) {
    set_error("the join's work queues need %zu bytes of scratch; the allocation-free path holds %zu", fixed,
              kScratchBytes);
    return APSS_ENOMEM;
  }
  // pair room: the caller's capacity, as far as the scratch allows
  int64_t room = (int64_t)((kScratchBytes - fixed) / 24);
  while (room > 0 && fixed + pair_bytes(room) > kScratchBytes) room -= room / 64 + 1;
  if (room > capacity) room = capacity;

  Carve cv{base};
  unsigned long long* counters = cv.take<unsigned long long>(C_NUM);
  unsigned int* qctr = cv.take<unsigned int>(8);
  int64_t* tstart = cv.take<int64_t>(L.ntiles + 1);
  int64_t* qcum = cv.take<int64_t>((int64_t)L.cum.size());
  uint32_t* wg_cur = cv.take<uint32_t>((int64_t)L.G * L.wg_stride);
  uint64_t* raw_key = cv.take<uint64_t>(room);
  float* raw_sim = cv.take<float>(room);
  uint64_t* k2 = cv.take<uint64_t>(room);
  uint32_t* v2 = cv.take<uint32_t>(room);
  int64_t* hist = cv.take<int64_t>(radix_hist_elems(room));
  int64_t* scan = cv.take<int64_t>(radix_scan_tmp_elems(room));
  if (cv.used > kScratchBytes) {
    set_error("internal: scratch placement of %zu bytes exceeds %zu", cv.used, kScratchBytes);
    return APSS_EDEVICE;
  }

  APSS_CHK(hipEventRecord(ws.ev[0], s), "event");
  APSS_CHK(hipMemcpyAsync(tstart, L.tiles.start.data(), sizeof(int64_t) * (L.ntiles + 1), hipMemcpyHostToDevice, s),
           "tiles");
  APSS_CHK(hipMemcpyAsync(qcum, L.cum.data(), sizeof(int64_t) * L.cum.size(), hipMemcpyHostToDevice, s), "queues");
  // the array keeps the previous call's contents: clear what starts at zero
  APSS_CHK(fill_u64((uint64_t*)counters, 0ull, C_NUM, s), "fill");
  APSS_CHK(fill_u32(qctr, 0u, 8, s), "fill");
  JoinPlan P;
  bind_plan(ix, Q, 1, t, nullptr, nullptr, L, tstart, qcum, qctr, wg_cur, P);
  P.a.out_key = raw_key;
  P.a.out_sim = raw_sim;
  P.a.cap = room;
  P.a.counters = counters;
  if (!join_args_complete(P.a)) {
    set_error("internal: join launched with a missing device buffer");
    return APSS_EDEVICE;
  }
  APSS_CHK(hipEventRecord(ws.ev[1], s), "event");
  APSS_CHK(launch_join(P.a, P.variant, P.G, s), "join kernel");
  APSS_CHK(hipEventRecord(ws.ev[2], s), "event");
  unsigned long long c[C_NUM];
  APSS_CHK(hipMemcpyAsync(c, counters, sizeof(c), hipMemcpyDeviceToHost, s), "read counters");
  APSS_CHK(hipStreamSynchronize(s), "join");
  const int64_t matches = (int64_t)c[C_MATCHES];
  *count = matches;
  if (matches > capacity) {
    set_error("output capacity %lld too small for %lld pairs", (long long)capacity, (long long)matches);
    return APSS_ERANGE;
  }
  if (matches > room) {
    set_error("%lld pairs exceed the allocation-free path's room of %lld pairs (%zu bytes of scratch)",
              (long long)matches, (long long)room, kScratchBytes);
    return APSS_ENOMEM;
  }
  APSS_CHK(radix_sort_u64_u32(raw_key, (uint32_t*)raw_sim, k2, v2, matches, P.bi + P.bj, hist, scan, s), "pair sort");
  APSS_CHK(launch_unpack_pairs(raw_key, raw_sim, matches, P.bj, out_i, out_j, out_sim, s), "unpack");
  APSS_CHK(hipEventRecord(ws.ev[3], s), "event");
  APSS_CHK(hipStreamSynchronize(s), "unpack");
  ws.last.posting_visits = (int64_t)(c[C_VISITS] + c[C_TAILVISITS]);
  ws.last.candidates = (int64_t)c[C_CANDIDATES];
  ws.last.bound_survivors = (int64_t)c[C_SURVIVORS];
  ws.last.verified = (int64_t)c[C_VERIFIED];
  ws.last.band = (int64_t)c[C_BAND];
  ws.last.matches = matches;
  float ms = 0.0f;
  APSS_CHK(hipEventElapsedTime(&ms, ws.ev[1], ws.ev[2]), "event");
  ws.last.ms_candidates = ms;
  APSS_CHK(hipEventElapsedTime(&ms, ws.ev[0], ws.ev[3]), "event");
  ws.last.ms_total = ms;
  return APSS_OK;
}
