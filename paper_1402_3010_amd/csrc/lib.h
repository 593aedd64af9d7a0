// Host-side internals of the apss library shared by the C ABI (capi.cpp)
// and the serving loop (server.cpp).  Not part of the ABI.
#pragma once

#include <stdint.h>

#include <mutex>
#include <string>
#include <vector>

#include "../../include/apss.h"
#include "apss_internal.h"
#include "join.h"

namespace apss {

// Owned device allocation.
template <typename T>
struct DBuf {
  T* p = nullptr;
  int64_t n = 0;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  ~DBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  hipError_t alloc(int64_t count) {
    release();
    if (count <= 0) count = 1;
    hipError_t e = hipMalloc((void**)&p, sizeof(T) * (size_t)count);
    if (e != hipSuccess) {
      p = nullptr;
      return e;
    }
    n = count;
    return hipSuccess;
  }
  // grow without preserving contents
  hipError_t reserve(int64_t count) {
    if (count <= n && p) return hipSuccess;
    return alloc(count);
  }
  int64_t bytes() const { return p ? n * (int64_t)sizeof(T) : 0; }
};

// Rank-space rows of a query set (the corpus itself for the self-join).
struct RankRows {
  int64_t n = 0, nnz = 0;
  DBuf<int64_t> rp;
  DBuf<RComp> rc;
  DBuf<float> mw;
  std::vector<int64_t> rp_host;  // host copy of rp (tile formation)
};

// Sort scratch sized for the largest sort done so far.
// Page-locked host buffer that only grows (copies from and to it run
// asynchronously by DMA).
template <class T>
struct PinnedBuf {
  T* p = nullptr;
  size_t n = 0;
  bool reserve(size_t k) {
    if (k <= n) return true;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    n = 0;
    if (hipHostMalloc((void**)&p, (k > 0 ? k : 1) * sizeof(T), hipHostMallocDefault) != hipSuccess) {
      p = nullptr;
      return false;
    }
    n = k;
    return true;
  }
  ~PinnedBuf() {
    if (p) (void)hipHostFree(p);
  }
};

struct SortScratch {
  DBuf<uint64_t> k1, k2, v64a, v64b;
  DBuf<uint32_t> v32a, v32b;
  DBuf<int64_t> hist, scan;
  DBuf<int64_t> seg;             // segment bounds of a segmented row sort
  std::vector<int64_t> seg_host;  // their host copy (kept until the copy is done)
  int64_t bytes() const {
    return k1.bytes() + k2.bytes() + v64a.bytes() + v64b.bytes() + v32a.bytes() + v32b.bytes() + hist.bytes() +
           scan.bytes() + seg.bytes();
  }
};

// A captured launch sequence of a self-join (fills, join kernel, counter
// read-back, pair sort, unpack into the caller's buffers), replayed while
// the threshold, the outputs and every buffer it names stay the same.
struct JoinGraph {
  hipGraphExec_t exec = nullptr;
  float t = 0.0f;
  const void* out[3] = {nullptr, nullptr, nullptr};
  int64_t capacity = 0;
  int64_t count = 0;
  std::vector<const void*> baked;     // device buffers the graph uses
  unsigned long long* hctr = nullptr;  // pinned copy of the counters
  void reset() {
    if (exec) (void)hipGraphExecDestroy(exec);
    exec = nullptr;
  }
  ~JoinGraph() {
    reset();
    if (hctr) (void)hipHostFree(hctr);
  }
};

// Everything one join or query call needs besides the index: its stream,
// scratch, raw output and timing.  The index has one for apss_join and
// apss_query; every slot of a server has its own, so calls on different
// workspaces may run at the same time.
struct Workspace {
  hipStream_t stream = nullptr;
  SortScratch ss;
  DBuf<int64_t> tstart, qcum;
  DBuf<unsigned int> qctr;
  DBuf<uint32_t> wg_cur;
  DBuf<unsigned long long> counters;
  DBuf<int64_t> uniq_total;  // distinct pairs after a join with local pruning
  DBuf<int32_t> qadm;        // remscore: first admitting component of each query
  DBuf<uint64_t> raw_key;
  DBuf<float> raw_sim;
  DBuf<float> qt;
  // query CSR copied from the host (kept between calls)
  DBuf<int32_t> q_col;
  DBuf<float> q_val;
  DBuf<uint32_t> err;
  DBuf<unsigned long long> bad;
  // head screen of the screened join
  DBuf<uint64_t> s_keys, s_cand;
  DBuf<unsigned long long> s_cnt;
  DBuf<int32_t> s_sid, s_tiles;
  DBuf<float> s_nh;
  DBuf<uint16_t> s_X;
  JoinGraph graph;
  PinnedBuf<uint32_t> host_out;  // staging of result pairs copied to the host
  apss_stats last;
  int64_t regrows = 0;  // joins rerun because the pair buffer was too small
  hipEvent_t ev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  ~Workspace() {
    for (int e = 0; e < 6; ++e)
      if (ev[e]) (void)hipEventDestroy(ev[e]);
  }
  int64_t bytes() const {
    return ss.bytes() + tstart.bytes() + qcum.bytes() + qctr.bytes() + wg_cur.bytes() + counters.bytes() +
           raw_key.bytes() + raw_sim.bytes() + qt.bytes() + uniq_total.bytes() + qadm.bytes() + q_col.bytes() + q_val.bytes() + s_keys.bytes() + s_cand.bytes() + s_sid.bytes() +
           s_tiles.bytes() + s_nh.bytes() + s_X.bytes();
  }
};

}  // namespace apss

struct apss_index {
  int device = 0;
  apss_opts opts;
  int64_t n = 0, m = 0, nnz = 0, P = 0;
  float t_build = 0.0f;
  int32_t H = 0;
  float pnrm_max = 0.0f;    // largest unindexed-part norm over the rows (RowStat.pnrm)
  int variant = 1;          // tile variant of the join kernel
  int64_t range_rows = 0;   // corpus rows per work-item range
  int32_t range_group = 1;  // ranges per work item
  int32_t head_cut = 0;     // > 0: the unindexed part of every row is its components of rank < head_cut
  apss_index* screen = nullptr;  // head-cut index over the same rows (screened join), owned
  apss::RankRows rows;  // corpus rows in rank space (densest dimension first)
  apss::DBuf<apss::RowStat> rs;
  apss::DBuf<int32_t> rank, inv;
  apss::DBuf<float> mw_r;  // maxweight by rank
  apss::DBuf<int64_t> off;
  apss::DBuf<apss::Post> post;
  apss::DBuf<uint32_t> post4;  // packed copy of post for streaming
  apss::DBuf<uint8_t> pn8;     // [n] RowStat.pnrm as a byte code (kPn8None or an upper bound in 1/254 steps)
  // local pruning: rank bounds of the parts (parts + 1 entries)
  int32_t parts = 1;
  apss::DBuf<int32_t> part_lo;
  std::vector<int32_t> part_lo_host;
  // lazily built tables (guarded by prep_mu)
  std::mutex prep_mu;
  apss::DBuf<uint32_t> hoff[2];  // per-block offsets of the dense lists (block width 1024, 2048)
  int64_t hoff_nb[2] = {0, 0};
  apss::DBuf<uint32_t> toff;  // per-range offsets of the sparse lists
  int64_t toff_rows = 0, toff_nR = 0;
  int grid[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  apss::Workspace ws;  // for apss_join / apss_query
};

namespace apss {

struct QuerySet {
  const int64_t* rp;  // device
  const RComp* rc;
  const float* mw;
  int64_t n, nnz;
  const int64_t* rp_host;  // host copy of rp
};

// Query tiles of a join: first query of each tile (ntiles + 1 entries) and
// the largest tile's component count.
struct Tiles {
  std::vector<int64_t> start;
  int64_t max_nnz = 0;
};

// Host side of one join kernel launch: geometry, query tiles and the
// cumulative item counts of the 8 per-XCD work queues.
struct JoinLayout {
  int variant = 0, QT = 0, CB = 0, slot = 0, K = 0, G = 0, parts = 1, rg = 1;
  int64_t nb = 0, nR = 0, nrx = 0, ntiles = 0, wg_stride = 0;
  Tiles tiles;
  std::vector<int64_t> cum;  // 8 * (nrx + 1)
};

// A join kernel launch with every argument but its outputs and counters.
struct JoinPlan {
  JoinArgs a{};
  int variant = 0;
  int G = 0;
  int bi = 0, bj = 0;
};

// Layout of a join of Q against the index (the index's tables for its tile
// variant and range width must have been made ready by prepare()).
int plan_layout(apss_index* ix, const QuerySet& Q, int triangle, JoinLayout& L);
// Kernel arguments of that layout with the given device copies of its tiles
// (L.ntiles + 1 entries) and queues (L.cum), 8 queue counters and
// L.G * L.wg_stride cursor words.
void bind_plan(apss_index* ix, const QuerySet& Q, int triangle, float t, const float* qt_dev, const RowStat* qrs,
               const JoinLayout& L, const int64_t* tstart_dev, const int64_t* qcum_dev, unsigned int* qctr_dev,
               uint32_t* wg_cur_dev, JoinPlan& P);

std::string& last_error();  // per calling thread
void set_error(const char* fmt, ...);
int dev_err(hipError_t e, const char* what);
int check_t(const apss_index* ix, float t);
// Make the lookup tables of a tile variant and range width ready (built on
// stream s, finished before return); safe to call from several threads.
// Rebuilding the range table for another width while a join runs is not.
int prepare(apss_index* ix, hipStream_t s, int variant, int64_t range_rows);
// most corpus ranges one work item of the join visits
constexpr int kMaxRangeGroup = 64;
int64_t default_range_rows(int variant);
// Query rows -> rank space on ws's stream (validates; t_per_row is host memory or NULL).
int stage_queries(apss_index* ix, Workspace& ws, int64_t nq, const int64_t* q_row_ptr, const int32_t* q_col,
                  const float* q_val, int on_device, const float* t_per_row, float t, RankRows& rows);
// Run the join kernels; sorted raw pairs in ws.raw_key / ws.raw_sim; count in
// *count.  cap_hint: pair capacity to start with (grown and rerun on overflow).
int run_join(apss_index* ix, Workspace& ws, const QuerySet& Q, int triangle, float t, const float* qt_dev,
             int64_t cap_hint, int64_t* count);
// Tile variants that may be launched.  Variant 3 (4 queries x 2048 rows,
// 256 threads) faulted on the GPU (memory aperture violation) in two tuning
// runs on the 500k-vector workloads, intermittently and without an
// identified cause, so it is refused everywhere until that is found.
inline bool variant_available(int variant) { return variant != 3; }
inline bool screen_variant_ok(int variant) { return variant_available(variant); }
// Screened self-join of an index built with screen_dims > 0 (ix->screen set).
int run_screen_join(apss_index* ix, Workspace& ws, float t, int64_t cap_hint, int64_t* count);
// Unpack the sorted raw pairs into device arrays / library-owned host arrays.
// finish_device waits for the unpack unless wait is false (then the caller
// synchronises the stream and calls record_total).
int finish_device(Workspace& ws, int64_t cnt, int bj, uint32_t* out_i, uint32_t* out_j, float* out_sim,
                  int64_t capacity, int64_t* count, bool wait = true);
int record_total(Workspace& ws);
int finish_host(Workspace& ws, int64_t cnt, int bj, apss_pairs* out);

}  // namespace apss

#define APSS_CHK(expr, what)                               \
  do {                                                     \
    hipError_t e__ = (expr);                               \
    if (e__ != hipSuccess) return ::apss::dev_err(e__, what); \
  } while (0)
