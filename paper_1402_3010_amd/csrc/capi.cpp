// C ABI of the apss library: index construction, self-join, external
// queries.  Host code only orchestrates device work; every step of the
// join runs in the kernels of index_build.hip, join.hip and primitives.hip.
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "../../include/apss.h"
#include "apss_internal.h"
#include "index_build.h"
#include "join.h"

namespace apss {

std::string& last_error() {
  static thread_local std::string s;
  return s;
}

void set_error(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  last_error() = buf;
}

namespace {

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
};

int dev_err(hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
    set_error("%s: out of device memory", what);
    (void)hipGetLastError();
    return APSS_ENOMEM;
  }
  set_error("%s: %s", what, hipGetErrorString(e));
  return APSS_EDEVICE;
}

#define CHK(expr, what)                         \
  do {                                          \
    hipError_t e__ = (expr);                    \
    if (e__ != hipSuccess) return dev_err(e__, what); \
  } while (0)

// Rank-space rows of a query set (the corpus itself for the self-join).
struct RankRows {
  int64_t n = 0, nnz = 0;
  DBuf<int64_t> rp;
  DBuf<RComp> rc;
  DBuf<float> mw;
};

// Sort scratch sized for the largest sort done so far.
struct SortScratch {
  DBuf<uint64_t> k1, k2, v64a, v64b;
  DBuf<uint32_t> v32a, v32b;
  DBuf<int64_t> hist, scan;
};

const char* err_bits_text(uint32_t e) {
  if (e & ERR_ROWPTR) return "row_ptr must start at 0, be non-decreasing and end at nnz";
  if (e & ERR_DIM) return "dimension id outside [0, m)";
  if (e & ERR_WEIGHT) return "weights must be finite and > 0";
  if (e & ERR_NORM) return "non-empty rows must have unit L2 norm (|norm - 1| <= 1e-5)";
  if (e & ERR_DUP) return "repeated dimension id inside a row";
  return "invalid input";
}

}  // namespace
}  // namespace apss

using namespace apss;

struct apss_index {
  int device = 0;
  hipStream_t stream = nullptr;
  apss_opts opts;
  int64_t n = 0, m = 0, nnz = 0, P = 0;
  float t_build = 0.0f;
  int32_t H = 0;
  RankRows rows;          // corpus rows in rank space (densest dimension first)
  DBuf<RowStat> rs;
  DBuf<int32_t> rank, inv;
  DBuf<float> mw_r;       // maxweight by rank
  DBuf<int64_t> off;
  DBuf<Post> post;
  DBuf<uint32_t> post4;   // packed copy of post for streaming
  // per-block list offsets for each block width in use (index 0: 1024 rows, 1: 2048 rows)
  DBuf<uint32_t> hoff[2];
  int64_t hoff_nb[2] = {0, 0};
  int variant = 0;
  // range offsets of the sparse lists for one range width (rows)
  DBuf<uint32_t> toff;
  int64_t toff_rows = 0, toff_nR = 0;
  std::vector<int64_t> rp_host;  // host copy of the corpus row offsets
  // join workspace
  DBuf<int64_t> tstart;
  DBuf<uint32_t> wg_cur;
  DBuf<int64_t> qcum;
  DBuf<unsigned int> qctr;
  DBuf<unsigned long long> scalar;
  int grid[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  DBuf<uint64_t> raw_key;
  DBuf<float> raw_sim;
  DBuf<unsigned long long> counters;
  SortScratch ss;
  apss_stats last;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
};

namespace {

// Sort (row, rank) keys with float payload into rank-space rows; checks for duplicates.
int sort_rows(apss_index* ix, uint64_t* keys, uint32_t* vals, int64_t nnz, int key_bits, int rbits, RComp* rc_out,
              uint32_t* err_dev) {
  hipStream_t s = ix->stream;
  SortScratch& ss = ix->ss;
  CHK(ss.k2.reserve(nnz), "sort scratch");
  CHK(ss.v32b.reserve(nnz), "sort scratch");
  CHK(ss.hist.reserve(radix_hist_elems(nnz)), "sort scratch");
  CHK(ss.scan.reserve(radix_scan_tmp_elems(nnz)), "sort scratch");
  CHK(radix_sort_u64_u32(keys, vals, ss.k2.p, ss.v32b.p, nnz, key_bits, ss.hist.p, ss.scan.p, s), "row sort");
  CHK(launch_unpack_rows(keys, vals, nnz, rbits, rc_out, err_dev, s), "row unpack");
  return APSS_OK;
}

int check_err(apss_index* ix, uint32_t* err_dev, unsigned long long* bad_dev, const char* what) {
  uint32_t err = 0;
  unsigned long long bad = ~0ull;
  CHK(hipMemcpyAsync(&err, err_dev, sizeof(err), hipMemcpyDeviceToHost, ix->stream), what);
  if (bad_dev) CHK(hipMemcpyAsync(&bad, bad_dev, sizeof(bad), hipMemcpyDeviceToHost, ix->stream), what);
  CHK(hipStreamSynchronize(ix->stream), what);
  if (err) {
    if (bad != ~0ull) set_error("%s: %s (row %llu)", what, err_bits_text(err), bad);
    else set_error("%s: %s", what, err_bits_text(err));
    return APSS_EINVAL;
  }
  return APSS_OK;
}

// Device copies of a CSR given on host or device.
struct CsrDev {
  DBuf<int64_t> rp;
  DBuf<int32_t> col;
  DBuf<float> val;
  const int64_t* prp = nullptr;
  const int32_t* pcol = nullptr;
  const float* pval = nullptr;
};

int stage_csr(apss_index* ix, int64_t n, const int64_t* row_ptr, const int32_t* col, const float* val, int on_device,
              int64_t* nnz_out, CsrDev& d) {
  hipStream_t s = ix->stream;
  int64_t nnz = 0;
  if (on_device) {
    CHK(hipMemcpyAsync(&nnz, row_ptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, s), "read nnz");
    CHK(hipStreamSynchronize(s), "read nnz");
    d.prp = row_ptr;
    d.pcol = col;
    d.pval = val;
  } else {
    nnz = row_ptr[n];
    if (row_ptr[0] != 0 || nnz < 0) {
      set_error("row_ptr must start at 0 and end at nnz >= 0");
      return APSS_EINVAL;
    }
    for (int64_t r = 0; r < n; ++r)
      if (row_ptr[r + 1] < row_ptr[r]) {
        set_error("row_ptr must be non-decreasing (row %lld)", (long long)r);
        return APSS_EINVAL;
      }
    CHK(d.rp.alloc(n + 1), "alloc csr");
    CHK(d.col.alloc(nnz), "alloc csr");
    CHK(d.val.alloc(nnz), "alloc csr");
    CHK(hipMemcpyAsync(d.rp.p, row_ptr, sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, s), "copy csr");
    if (nnz) {
      CHK(hipMemcpyAsync(d.col.p, col, sizeof(int32_t) * nnz, hipMemcpyHostToDevice, s), "copy csr");
      CHK(hipMemcpyAsync(d.val.p, val, sizeof(float) * nnz, hipMemcpyHostToDevice, s), "copy csr");
    }
    d.prp = d.rp.p;
    d.pcol = d.col.p;
    d.pval = d.val.p;
  }
  if (nnz < 0 || nnz >= (1ll << 32)) {
    set_error("nnz must be in [0, 2^32)");
    return APSS_EINVAL;
  }
  *nnz_out = nnz;
  return APSS_OK;
}

int hoff_slot(int cb) { return cb == 1024 ? 0 : 1; }

// Per-(block, rank) list offsets for the block width of a tile variant.
int ensure_hoff(apss_index* ix, int variant) {
  int qt = 0, cb = 0;
  if (join_variant_geometry(variant, &qt, &cb)) {
    set_error("unknown join variant %d", variant);
    return APSS_EINVAL;
  }
  const int slot = hoff_slot(cb);
  if (ix->hoff[slot].p) return APSS_OK;
  const int64_t nb = (ix->n + cb - 1) / cb;
  CHK(ix->hoff[slot].alloc((nb + 1) * (int64_t)ix->H), "alloc block offsets");
  CHK(launch_block_offsets(ix->off.p, ix->post.p, ix->H, nb, cb, ix->hoff[slot].p, ix->stream), "block offsets");
  ix->hoff_nb[slot] = nb;
  return APSS_OK;
}

int build_impl(apss_index* ix, const int64_t* row_ptr, const int32_t* col, const float* val, int on_device) {
  hipStream_t s = ix->stream;
  const int64_t n = ix->n, m = ix->m;
  CsrDev in;
  int64_t nnz = 0;
  int rc = stage_csr(ix, n, row_ptr, col, val, on_device, &nnz, in);
  if (rc) return rc;
  ix->nnz = nnz;

  DBuf<uint32_t> err;
  DBuf<unsigned long long> bad;
  CHK(err.alloc(1), "alloc");
  CHK(bad.alloc(1), "alloc");
  CHK(fill_u32(err.p, 0u, 1, s), "fill");
  CHK(fill_u64((uint64_t*)bad.p, ~0ull, 1, s), "fill");
  CHK(launch_check_rowptr(in.prp, n, nnz, err.p, bad.p, s), "check row_ptr");
  if ((rc = check_err(ix, err.p, bad.p, "build_index"))) return rc;
  CHK(launch_validate_rows(in.prp, in.pcol, in.pval, n, m, 1e-5, err.p, bad.p, s), "validate");
  if ((rc = check_err(ix, err.p, bad.p, "build_index"))) return rc;

  // density order and maxweight_d(V)
  DBuf<uint32_t> cnt, mwbits, cnt_r;
  CHK(cnt.alloc(m), "alloc");
  CHK(mwbits.alloc(m), "alloc");
  CHK(cnt_r.alloc(m), "alloc");
  CHK(fill_u32(cnt.p, 0u, m, s), "fill");
  CHK(fill_u32(mwbits.p, 0u, m, s), "fill");
  CHK(launch_count_dims(in.pcol, in.pval, nnz, cnt.p, mwbits.p, s), "count dims");
  const int dbits = ceil_log2((uint64_t)m);
  const int cbits = ceil_log2((uint64_t)n + 1);
  SortScratch& ss = ix->ss;
  const int64_t big = std::max<int64_t>(nnz, m);
  CHK(ss.k1.reserve(big), "alloc sort");
  CHK(ss.v64a.reserve(m), "alloc sort");
  CHK(ss.k2.reserve(big), "alloc sort");
  CHK(ss.v64b.reserve(m), "alloc sort");
  CHK(ss.hist.reserve(radix_hist_elems(big)), "alloc sort");
  CHK(ss.scan.reserve(radix_scan_tmp_elems(big)), "alloc sort");
  CHK(launch_dim_keys(cnt.p, m, n, dbits, ss.k1.p, ss.v64a.p, s), "dim keys");
  CHK(radix_sort_u64(ss.k1.p, ss.v64a.p, ss.k2.p, ss.v64b.p, m, dbits + cbits, ss.hist.p, ss.scan.p, s), "dim sort");
  CHK(ix->rank.alloc(m), "alloc");
  CHK(ix->inv.alloc(m), "alloc");
  CHK(ix->mw_r.alloc(m), "alloc");
  CHK(launch_rank_from_sorted(ss.v64a.p, m, cnt.p, mwbits.p, ix->rank.p, ix->inv.p, ix->mw_r.p, cnt_r.p, s),
      "ranks");

  // rows in rank space, densest dimension first
  const int rbits = dbits;
  const int nbits = ceil_log2((uint64_t)std::max<int64_t>(n, 1));
  CHK(ss.v32a.reserve(nnz), "alloc");
  CHK(launch_row_keys(in.prp, in.pcol, in.pval, ix->rank.p, n, rbits, ss.k1.p, ss.v32a.p, s), "row keys");
  ix->rows.n = n;
  ix->rows.nnz = nnz;
  CHK(ix->rows.rp.alloc(n + 1), "alloc");
  CHK(hipMemcpyAsync(ix->rows.rp.p, in.prp, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToDevice, s), "copy");
  ix->rp_host.resize((size_t)n + 1);
  CHK(hipMemcpyAsync(ix->rp_host.data(), in.prp, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost, s), "copy");
  CHK(ix->rows.rc.alloc(nnz), "alloc");
  if ((rc = sort_rows(ix, ss.k1.p, ss.v32a.p, nnz, nbits + rbits, rbits, ix->rows.rc.p, err.p))) return rc;
  if ((rc = check_err(ix, err.p, nullptr, "build_index"))) return rc;

  // cutoff of the unindexed part
  CHK(ix->rs.alloc(n), "alloc");
  CHK(ix->rows.mw.alloc(n), "alloc");
  DBuf<int64_t> nidx, scan_tmp, total;
  CHK(nidx.alloc(n + 1), "alloc");
  CHK(scan_tmp.alloc(scan_tmp_elems(n + 1)), "alloc");
  CHK(total.alloc(1), "alloc");
  CHK(launch_cutoff(ix->rows.rp.p, ix->rows.rc.p, ix->mw_r.p, n, ix->t_build, ix->opts.query_safe ? 1 : 0, ix->rs.p,
                    ix->rows.mw.p, nidx.p, s),
      "cutoff");
  CHK(exclusive_scan_i64(nidx.p, n, scan_tmp.p, total.p, s), "scan");
  int64_t P = 0;
  CHK(hipMemcpyAsync(&P, total.p, sizeof(int64_t), hipMemcpyDeviceToHost, s), "read P");
  CHK(hipStreamSynchronize(s), "read P");
  ix->P = P;
  if (4 * (P + 1) >= (1ll << 32)) {
    set_error("index too large: %lld postings (the packed lists must stay below 4 GiB)", (long long)P);
    return APSS_EINVAL;
  }

  // inverted lists of the indexed parts: stable sort by rank keeps vector ids ascending
  CHK(ss.k1.reserve(P), "alloc");
  CHK(ss.k2.reserve(P), "alloc");
  CHK(ss.v64a.reserve(P), "alloc");
  CHK(ss.v64b.reserve(P), "alloc");
  CHK(ss.hist.reserve(radix_hist_elems(P)), "alloc");
  CHK(ss.scan.reserve(radix_scan_tmp_elems(P)), "alloc");
  CHK(launch_emit_indexed(ix->rows.rp.p, ix->rows.rc.p, ix->rs.p, nidx.p, n, ss.k1.p, ss.v64a.p, s), "emit");
  CHK(radix_sort_u64(ss.k1.p, ss.v64a.p, ss.k2.p, ss.v64b.p, P, rbits, ss.hist.p, ss.scan.p, s), "list sort");
  CHK(ix->off.alloc(m + 1), "alloc");
  CHK(fill_u64((uint64_t*)ix->off.p, 0ull, m + 1, s), "fill");
  CHK(launch_count_ranks(ss.k1.p, P, ix->off.p, s), "count");
  DBuf<int64_t> scan2;
  CHK(scan2.alloc(scan_tmp_elems(m + 1)), "alloc");
  CHK(exclusive_scan_i64(ix->off.p, m + 1, scan2.p, nullptr, s), "scan");
  // one padding entry after the last list lets the join read position p + 1 for any p < P
  CHK(ix->post.alloc(P + 1), "alloc");
  CHK(fill_u64((uint64_t*)ix->post.p + P, ~0ull, 1, s), "fill");
  CHK(launch_unpack_post(ss.v64a.p, P, ix->post.p, s), "post");
  CHK(ix->post4.alloc(P + 1), "alloc");
  CHK(launch_pack_post4(ix->post.p, P, ix->post4.p, s), "post4");

  // per-block offsets of the dense lists, for the default tile variant
  int32_t H = ix->opts.head_dims > 0 ? ix->opts.head_dims : 32768;
  if (H > m) H = (int32_t)m;
  ix->H = H;
  if ((rc = ensure_hoff(ix, ix->variant))) return rc;
  CHK(hipStreamSynchronize(s), "build_index");
  // sort scratch is re-grown on demand by the joins
  ss.k1.release();
  ss.k2.release();
  ss.v64a.release();
  ss.v64b.release();
  ss.v32a.release();
  ss.v32b.release();
  return APSS_OK;
}

struct QuerySet {
  const int64_t* rp;       // device
  const RComp* rc;
  const float* mw;
  int64_t n, nnz;
  const int64_t* rp_host;  // host copy of rp
};

// Query tiles: consecutive queries, at most QT of them and, unless a single
// query is larger, at most QB components, so that a tile fits the LDS staging.
struct Tiles {
  std::vector<int64_t> start;  // ntiles + 1 entries
  int64_t max_nnz = 0;
};

Tiles make_tiles(const int64_t* rp, int64_t n, int QT, int QB) {
  Tiles T;
  T.start.push_back(0);
  int64_t nnz = 0;
  for (int64_t q = 0; q < n; ++q) {
    const int64_t len = rp[q + 1] - rp[q];
    const int64_t cur = T.start.back();
    if (q > cur && (q - cur == QT || nnz + len > QB)) {
      T.max_nnz = std::max(T.max_nnz, nnz);
      T.start.push_back(q);
      nnz = 0;
    }
    nnz += len;
  }
  T.max_nnz = std::max(T.max_nnz, nnz);
  T.start.push_back(n);
  return T;
}

// Run the join kernels; raw (unsorted) pairs in ix->raw_key / raw_sim, count in *count.
int run_join(apss_index* ix, const QuerySet& Q, int triangle, float t, const float* qt_dev, int64_t* count) {
  hipStream_t s = ix->stream;
  memset(&ix->last, 0, sizeof(ix->last));
  *count = 0;
  for (int e = 0; e < 4; ++e)
    if (!ix->ev[e]) CHK(hipEventCreate(&ix->ev[e]), "event");
  CHK(hipEventRecord(ix->ev[0], s), "event");
  if (Q.n == 0 || ix->n == 0) return APSS_OK;
  const int variant = ix->variant;
  int QT = 0, CB = 0;
  if (join_variant_geometry(variant, &QT, &CB)) {
    set_error("unknown join variant %d", variant);
    return APSS_EINVAL;
  }
  int rc0 = ensure_hoff(ix, variant);
  if (rc0) return rc0;
  const int slot = hoff_slot(CB);
  const int64_t nb = ix->hoff_nb[slot];
  // work items: ranges of K blocks x query tiles
  int K = std::max(1, 8192 / CB);
  if (const char* ev = getenv("APSS_RANGE_ROWS")) {
    const int rr = atoi(ev);
    if (rr >= CB) K = rr / CB;
  }
  const int64_t nR = (nb + K - 1) / K;
  const int64_t range_rows = (int64_t)K * CB;
  if (!ix->toff.p || ix->toff_rows != range_rows) {
    CHK(ix->toff.alloc((nR + 1) * std::max<int64_t>(ix->m - ix->H, 1)), "alloc range offsets");
    CHK(launch_range_offsets(ix->off.p, ix->post.p, ix->H, ix->m, nR, range_rows, ix->toff.p, s), "range offsets");
    ix->toff_rows = range_rows;
    ix->toff_nR = nR;
  }
  const Tiles tiles = make_tiles(Q.rp_host, Q.n, QT, join_variant_staging(variant));
  const int64_t ntiles = (int64_t)tiles.start.size() - 1;
  CHK(ix->tstart.reserve(ntiles + 1), "alloc tiles");
  CHK(hipMemcpyAsync(ix->tstart.p, tiles.start.data(), sizeof(int64_t) * (ntiles + 1), hipMemcpyHostToDevice, s),
      "tiles");
  const int64_t nrx = (nR + 7) / 8;
  std::vector<int64_t> cum((size_t)(8 * (nrx + 1)), 0);
  for (int x = 0; x < 8; ++x) {
    int64_t c = 0;
    for (int64_t j = 0; j <= nrx; ++j) {
      cum[(size_t)(x * (nrx + 1) + j)] = c;
      const int64_t R = x + 8 * j;
      if (j < nrx && R < nR) {
        // first tile whose last query reaches the range (self-join triangle)
        const int64_t tmin =
            triangle ? (int64_t)(std::upper_bound(tiles.start.begin() + 1, tiles.start.end(), R * range_rows) -
                                 (tiles.start.begin() + 1))
                     : 0;
        c += ntiles - tmin;
      }
    }
  }
  CHK(ix->qcum.reserve((int64_t)cum.size()), "alloc queues");
  CHK(hipMemcpyAsync(ix->qcum.p, cum.data(), sizeof(int64_t) * cum.size(), hipMemcpyHostToDevice, s), "queues");
  CHK(ix->qctr.reserve(8), "alloc queues");
  CHK(ix->counters.reserve(C_NUM), "alloc counters");
  if (!ix->grid[variant]) ix->grid[variant] = join_resident_groups(variant);
  const int G = ix->grid[variant];
  // per-workgroup cursor space for tiles too large to stage in LDS
  const int64_t wg_stride = 2 * std::max<int64_t>(tiles.max_nnz, 1);
  CHK(ix->wg_cur.reserve((int64_t)G * wg_stride), "alloc cursors");
  if (!ix->raw_key.p) {
    const int64_t cap0 = std::max<int64_t>(1 << 20, 16 * std::max(ix->n, Q.n));
    CHK(ix->raw_key.alloc(cap0), "alloc pairs");
    CHK(ix->raw_sim.alloc(cap0), "alloc pairs");
  }
  const int bj = ceil_log2((uint64_t)(triangle ? ix->n : ix->n));
  const int bi = ceil_log2((uint64_t)(triangle ? ix->n : Q.n));
  for (int attempt = 0; attempt < 2; ++attempt) {
    CHK(hipEventRecord(ix->ev[0], s), "event");
    CHK(fill_u64((uint64_t*)ix->counters.p, 0ull, C_NUM, s), "fill");
    CHK(fill_u32(ix->qctr.p, 0u, 8, s), "fill");
    JoinArgs a;
    a.rp = ix->rows.rp.p;
    a.rc = ix->rows.rc.p;
    a.rs = ix->rs.p;
    a.off = ix->off.p;
    a.post = ix->post.p;
    a.post4 = ix->post4.p;
    a.post4_bytes = (uint32_t)(4 * (ix->P + 1));
    a.hoff = ix->hoff[slot].p;
    a.H = ix->H;
    a.nb = nb;
    a.n = ix->n;
    a.qrp = Q.rp;
    a.qrc = Q.rc;
    a.qmw = Q.mw;
    a.qt = qt_dev;
    a.t = t;
    a.nq = Q.n;
    a.triangle = triangle;
    a.ntiles = ntiles;
    a.tstart = ix->tstart.p;
    a.toff = ix->toff.p;
    a.m_tail = (int32_t)(ix->m - ix->H);
    a.K = K;
    a.nrx = nrx;
    a.qcum = ix->qcum.p;
    a.qctr = ix->qctr.p;
    a.wg_cur = ix->wg_cur.p;
    a.wg_cur_stride = wg_stride;
    a.out_key = ix->raw_key.p;
    a.out_sim = ix->raw_sim.p;
    a.cap = ix->raw_key.n;
    a.bj = bj;
    a.counters = ix->counters.p;
    CHK(hipEventRecord(ix->ev[1], s), "event");
    if (!join_args_complete(a)) {
      set_error("internal: join launched with a missing device buffer");
      return APSS_EDEVICE;
    }
    CHK(launch_join(a, variant, G, s), "join kernel");
    CHK(hipEventRecord(ix->ev[2], s), "event");
    unsigned long long c[C_NUM];
    CHK(hipMemcpyAsync(c, ix->counters.p, sizeof(c), hipMemcpyDeviceToHost, s), "read counters");
    CHK(hipStreamSynchronize(s), "join");
    const int64_t matches = (int64_t)c[C_MATCHES];
    if (matches > ix->raw_key.n) {
      const int64_t cap = matches + matches / 8 + 1024;
      CHK(ix->raw_key.alloc(cap), "alloc pairs");
      CHK(ix->raw_sim.alloc(cap), "alloc pairs");
      continue;  // rerun with room for every pair
    }
    ix->last.posting_visits = (int64_t)(c[C_VISITS] + c[C_TAILVISITS]);
    ix->last.candidates = (int64_t)c[C_CANDIDATES];
    ix->last.bound_survivors = (int64_t)c[C_SURVIVORS];
    ix->last.verified = (int64_t)c[C_VERIFIED];
    ix->last.band = (int64_t)c[C_BAND];
    ix->last.matches = matches;
    float ms = 0.0f;
    CHK(hipEventElapsedTime(&ms, ix->ev[1], ix->ev[2]), "event");
    ix->last.ms_candidates = ms;
    // sort by key
    SortScratch& ss = ix->ss;
    CHK(ss.k2.reserve(matches), "alloc sort");
    CHK(ss.v32b.reserve(matches), "alloc sort");
    CHK(ss.hist.reserve(radix_hist_elems(matches)), "alloc sort");
    CHK(ss.scan.reserve(radix_scan_tmp_elems(matches)), "alloc sort");
    CHK(radix_sort_u64_u32(ix->raw_key.p, (uint32_t*)ix->raw_sim.p, ss.k2.p, ss.v32b.p, matches, bi + bj, ss.hist.p,
                           ss.scan.p, s),
        "pair sort");
    *count = matches;
    return APSS_OK;
  }
  set_error("pair buffer kept overflowing");
  return APSS_ENOMEM;
}

int check_t(const apss_index* ix, float t) {
  if (!(t > 0.0f && t <= 1.0f)) {
    set_error("threshold %g outside (0, 1]", (double)t);
    return APSS_ETHRESH;
  }
  if (t < ix->t_build) {
    set_error("threshold %g below the index build threshold %g", (double)t, (double)ix->t_build);
    return APSS_ETHRESH;
  }
  return APSS_OK;
}

int finish_device(apss_index* ix, int64_t cnt, int bj, uint32_t* out_i, uint32_t* out_j, float* out_sim,
                  int64_t capacity, int64_t* count) {
  *count = cnt;
  if (cnt > capacity) {
    set_error("output capacity %lld too small for %lld pairs", (long long)capacity, (long long)cnt);
    return APSS_ERANGE;
  }
  CHK(launch_unpack_pairs(ix->raw_key.p, ix->raw_sim.p, cnt, bj, out_i, out_j, out_sim, ix->stream), "unpack");
  CHK(hipEventRecord(ix->ev[3], ix->stream), "event");
  CHK(hipStreamSynchronize(ix->stream), "unpack");
  float ms = 0.0f;
  CHK(hipEventElapsedTime(&ms, ix->ev[0], ix->ev[3]), "event");
  ix->last.ms_total = ms;
  return APSS_OK;
}

int finish_host(apss_index* ix, int64_t cnt, int bj, apss_pairs* out) {
  out->count = 0;
  out->i = out->j = nullptr;
  out->sim = nullptr;
  DBuf<uint32_t> di, dj;
  DBuf<float> ds;
  CHK(di.alloc(cnt), "alloc");
  CHK(dj.alloc(cnt), "alloc");
  CHK(ds.alloc(cnt), "alloc");
  int64_t c2 = 0;
  int rc = finish_device(ix, cnt, bj, di.p, dj.p, ds.p, cnt, &c2);
  if (rc) return rc;
  const size_t nb = (size_t)(cnt > 0 ? cnt : 1);
  out->i = (uint32_t*)malloc(nb * sizeof(uint32_t));
  out->j = (uint32_t*)malloc(nb * sizeof(uint32_t));
  out->sim = (float*)malloc(nb * sizeof(float));
  if (!out->i || !out->j || !out->sim) {
    free(out->i);
    free(out->j);
    free(out->sim);
    out->i = out->j = nullptr;
    out->sim = nullptr;
    set_error("host allocation failed");
    return APSS_ENOMEM;
  }
  if (cnt) {
    CHK(hipMemcpyAsync(out->i, di.p, sizeof(uint32_t) * cnt, hipMemcpyDeviceToHost, ix->stream), "copy out");
    CHK(hipMemcpyAsync(out->j, dj.p, sizeof(uint32_t) * cnt, hipMemcpyDeviceToHost, ix->stream), "copy out");
    CHK(hipMemcpyAsync(out->sim, ds.p, sizeof(float) * cnt, hipMemcpyDeviceToHost, ix->stream), "copy out");
  }
  CHK(hipStreamSynchronize(ix->stream), "copy out");
  out->count = cnt;
  return APSS_OK;
}

// Query rows -> rank space (validated), per-row thresholds on device.
struct QueryStage {
  RankRows rows;
  DBuf<float> qt;
  std::vector<int64_t> rp_host;
};

int stage_queries(apss_index* ix, int64_t nq, const int64_t* q_row_ptr, const int32_t* q_col, const float* q_val,
                  int on_device, const float* t_per_row, float t, QueryStage& qs) {
  hipStream_t s = ix->stream;
  if (!ix->opts.query_safe) {
    set_error("index was built with query_safe = 0; external queries need the L2 cutoff clause");
    return APSS_EINVAL;
  }
  if (t_per_row) {
    for (int64_t q = 0; q < nq; ++q) {
      int rc = check_t(ix, t_per_row[q]);
      if (rc) return rc;
    }
  } else {
    int rc = check_t(ix, t);
    if (rc) return rc;
  }
  CsrDev in;
  int64_t nnz = 0;
  int rc = stage_csr(ix, nq, q_row_ptr, q_col, q_val, on_device, &nnz, in);
  if (rc) return rc;
  DBuf<uint32_t> err;
  DBuf<unsigned long long> bad;
  CHK(err.alloc(1), "alloc");
  CHK(bad.alloc(1), "alloc");
  CHK(fill_u32(err.p, 0u, 1, s), "fill");
  CHK(fill_u64((uint64_t*)bad.p, ~0ull, 1, s), "fill");
  CHK(launch_check_rowptr(in.prp, nq, nnz, err.p, bad.p, s), "check row_ptr");
  if ((rc = check_err(ix, err.p, bad.p, "query"))) return rc;
  qs.rows.n = nq;
  qs.rows.nnz = nnz;
  CHK(qs.rows.rp.alloc(nq + 1), "alloc");
  CHK(hipMemcpyAsync(qs.rows.rp.p, in.prp, sizeof(int64_t) * (nq + 1), hipMemcpyDeviceToDevice, s), "copy");
  qs.rp_host.resize((size_t)nq + 1);
  CHK(hipMemcpyAsync(qs.rp_host.data(), in.prp, sizeof(int64_t) * (nq + 1), hipMemcpyDeviceToHost, s), "copy");
  CHK(qs.rows.rc.alloc(nnz), "alloc");
  CHK(qs.rows.mw.alloc(nq), "alloc");
  SortScratch& ss = ix->ss;
  CHK(ss.k1.reserve(nnz), "alloc");
  CHK(ss.v32a.reserve(nnz), "alloc");
  const int rbits = ceil_log2((uint64_t)ix->m);
  const int nbits = ceil_log2((uint64_t)std::max<int64_t>(nq, 1));
  CHK(launch_query_keys(in.prp, in.pcol, in.pval, ix->rank.p, nq, ix->m, rbits, 1e-5, ss.k1.p, ss.v32a.p,
                        qs.rows.mw.p, err.p, bad.p, s),
      "query keys");
  if ((rc = check_err(ix, err.p, bad.p, "query"))) return rc;
  if ((rc = sort_rows(ix, ss.k1.p, ss.v32a.p, nnz, nbits + rbits, rbits, qs.rows.rc.p, err.p))) return rc;
  if ((rc = check_err(ix, err.p, nullptr, "query"))) return rc;
  if (t_per_row) {
    CHK(qs.qt.alloc(nq), "alloc");
    CHK(hipMemcpyAsync(qs.qt.p, t_per_row, sizeof(float) * nq, hipMemcpyHostToDevice, s), "copy thresholds");
  }
  return APSS_OK;
}

}  // namespace

extern "C" {

void apss_default_opts(apss_opts* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->struct_size = (int32_t)sizeof(apss_opts);
  o->stream = nullptr;
  o->query_safe = 1;
  o->variant = -1;
  o->head_dims = 0;
}

int apss_build_index(int64_t n, int64_t m, const int64_t* row_ptr, const int32_t* col, const float* val, int on_device,
                     float t_build, const apss_opts* opts, apss_index** out) {
  if (!out || !row_ptr || (!col && n > 0) || (!val && n > 0)) {
    set_error("NULL argument");
    return APSS_EINVAL;
  }
  *out = nullptr;
  if (n < 0 || n >= (1ll << 31) || m <= 0 || m >= (1ll << 31)) {
    set_error("need 0 <= n < 2^31 and 0 < m < 2^31");
    return APSS_EINVAL;
  }
  if (!(t_build > 0.0f && t_build <= 1.0f)) {
    set_error("t_build %g outside (0, 1]", (double)t_build);
    return APSS_ETHRESH;
  }
  apss_opts o;
  apss_default_opts(&o);
  if (opts) {
    if (opts->struct_size != (int32_t)sizeof(apss_opts)) {
      set_error("apss_opts.struct_size mismatch (use apss_default_opts)");
      return APSS_EINVAL;
    }
    o = *opts;
  }
  if (o.variant < -1 || o.variant >= join_num_variants()) {
    set_error("variant %d outside [-1, %d)", o.variant, join_num_variants());
    return APSS_EINVAL;
  }
  apss_index* ix = new (std::nothrow) apss_index();
  if (!ix) {
    set_error("host allocation failed");
    return APSS_ENOMEM;
  }
  ix->opts = o;
  ix->stream = (hipStream_t)o.stream;
  ix->n = n;
  ix->m = m;
  ix->t_build = t_build;
  ix->variant = o.variant >= 0 ? o.variant : 1;
  if (const char* ev = getenv("APSS_VARIANT")) {
    const int v = atoi(ev);
    if (v >= 0 && v < join_num_variants()) ix->variant = v;
  }
  (void)hipGetDevice(&ix->device);
  int rc = build_impl(ix, row_ptr, col, val, on_device);
  if (rc) {
    (void)hipStreamSynchronize(ix->stream);
    apss_index_free(ix);
    return rc;
  }
  *out = ix;
  return APSS_OK;
}

void apss_index_free(apss_index* idx) {
  if (!idx) return;
  (void)hipStreamSynchronize(idx->stream);
  for (int e = 0; e < 4; ++e)
    if (idx->ev[e]) (void)hipEventDestroy(idx->ev[e]);
  delete idx;
}

int apss_join_device(apss_index* ix, float t, uint32_t* out_i, uint32_t* out_j, float* out_sim, int64_t capacity,
                     int64_t* count) {
  if (!ix || !count || (capacity > 0 && (!out_i || !out_j || !out_sim))) {
    set_error("NULL argument");
    return APSS_EINVAL;
  }
  int rc = check_t(ix, t);
  if (rc) return rc;
  QuerySet Q{ix->rows.rp.p, ix->rows.rc.p, ix->rows.mw.p, ix->n, ix->nnz, ix->rp_host.data()};
  int64_t cnt = 0;
  if ((rc = run_join(ix, Q, 1, t, nullptr, &cnt))) return rc;
  return finish_device(ix, cnt, ceil_log2((uint64_t)ix->n), out_i, out_j, out_sim, capacity, count);
}

int apss_join(apss_index* ix, float t, apss_pairs* out) {
  if (!ix || !out) {
    set_error("NULL argument");
    return APSS_EINVAL;
  }
  out->count = 0;
  out->i = out->j = nullptr;
  out->sim = nullptr;
  int rc = check_t(ix, t);
  if (rc) return rc;
  QuerySet Q{ix->rows.rp.p, ix->rows.rc.p, ix->rows.mw.p, ix->n, ix->nnz, ix->rp_host.data()};
  int64_t cnt = 0;
  if ((rc = run_join(ix, Q, 1, t, nullptr, &cnt))) return rc;
  return finish_host(ix, cnt, ceil_log2((uint64_t)ix->n), out);
}

int apss_query_device(apss_index* ix, int64_t nq, const int64_t* q_row_ptr, const int32_t* q_col, const float* q_val,
                      int on_device, const float* t_per_row, float t, uint32_t* out_i, uint32_t* out_j,
                      float* out_sim, int64_t capacity, int64_t* count) {
  if (!ix || !count || !q_row_ptr || nq < 0 || nq >= (1ll << 31) ||
      (capacity > 0 && (!out_i || !out_j || !out_sim))) {
    set_error("NULL or invalid argument");
    return APSS_EINVAL;
  }
  QueryStage qs;
  int rc = stage_queries(ix, nq, q_row_ptr, q_col, q_val, on_device, t_per_row, t, qs);
  if (rc) return rc;
  QuerySet Q{qs.rows.rp.p, qs.rows.rc.p, qs.rows.mw.p, nq, qs.rows.nnz, qs.rp_host.data()};
  int64_t cnt = 0;
  if ((rc = run_join(ix, Q, 0, t, t_per_row ? qs.qt.p : nullptr, &cnt))) return rc;
  return finish_device(ix, cnt, ceil_log2((uint64_t)ix->n), out_i, out_j, out_sim, capacity, count);
}

int apss_query(apss_index* ix, int64_t nq, const int64_t* q_row_ptr, const int32_t* q_col, const float* q_val,
               int on_device, const float* t_per_row, float t, apss_pairs* out) {
  if (!ix || !out || !q_row_ptr || nq < 0 || nq >= (1ll << 31)) {
    set_error("NULL or invalid argument");
    return APSS_EINVAL;
  }
  out->count = 0;
  out->i = out->j = nullptr;
  out->sim = nullptr;
  QueryStage qs;
  int rc = stage_queries(ix, nq, q_row_ptr, q_col, q_val, on_device, t_per_row, t, qs);
  if (rc) return rc;
  QuerySet Q{qs.rows.rp.p, qs.rows.rc.p, qs.rows.mw.p, nq, qs.rows.nnz, qs.rp_host.data()};
  int64_t cnt = 0;
  if ((rc = run_join(ix, Q, 0, t, t_per_row ? qs.qt.p : nullptr, &cnt))) return rc;
  return finish_host(ix, cnt, ceil_log2((uint64_t)ix->n), out);
}

void apss_pairs_free(apss_pairs* p) {
  if (!p) return;
  free(p->i);
  free(p->j);
  free(p->sim);
  p->i = p->j = nullptr;
  p->sim = nullptr;
  p->count = 0;
}

int apss_last_stats(const apss_index* ix, apss_stats* out) {
  if (!ix || !out) {
    set_error("NULL argument");
    return APSS_EINVAL;
  }
  *out = ix->last;
  return APSS_OK;
}

int apss_index_export(const apss_index* ix, int32_t* rank, float* maxweight, int32_t* cut) {
  if (!ix) {
    set_error("NULL argument");
    return APSS_EINVAL;
  }
  hipStream_t s = ix->stream;
  if (rank) CHK(hipMemcpyAsync(rank, ix->rank.p, sizeof(int32_t) * ix->m, hipMemcpyDeviceToHost, s), "export");
  std::vector<float> mwr;
  std::vector<int32_t> inv;
  if (maxweight) {
    mwr.resize((size_t)ix->m);
    inv.resize((size_t)ix->m);
    CHK(hipMemcpyAsync(mwr.data(), ix->mw_r.p, sizeof(float) * ix->m, hipMemcpyDeviceToHost, s), "export");
    CHK(hipMemcpyAsync(inv.data(), ix->inv.p, sizeof(int32_t) * ix->m, hipMemcpyDeviceToHost, s), "export");
  }
  std::vector<RowStat> st;
  if (cut && ix->n) {
    st.resize((size_t)ix->n);
    CHK(hipMemcpyAsync(st.data(), ix->rs.p, sizeof(RowStat) * ix->n, hipMemcpyDeviceToHost, s), "export");
  }
  CHK(hipStreamSynchronize(s), "export");
  if (maxweight)
    for (int64_t r = 0; r < ix->m; ++r) maxweight[inv[(size_t)r]] = mwr[(size_t)r];
  if (cut)
    for (int64_t i = 0; i < ix->n; ++i) cut[i] = st[(size_t)i].cut;
  return APSS_OK;
}

int apss_index_sizes(const apss_index* ix, int64_t* n, int64_t* m, int64_t* nnz, int64_t* postings) {
  if (!ix) {
    set_error("NULL argument");
    return APSS_EINVAL;
  }
  if (n) *n = ix->n;
  if (m) *m = ix->m;
  if (nnz) *nnz = ix->nnz;
  if (postings) *postings = ix->P;
  return APSS_OK;
}

const char* apss_strerror(int code) {
  switch (code) {
    case APSS_OK: return "ok";
    case APSS_EINVAL: return "invalid argument";
    case APSS_ETHRESH: return "threshold out of range";
    case APSS_ENOMEM: return "out of memory";
    case APSS_EDEVICE: return "device error";
    case APSS_ERANGE: return "output buffer too small";
    case APSS_EBUSY: return "busy";
    case APSS_PENDING: return "pending";
    default: return "unknown error";
  }
}

const char* apss_last_error(void) { return last_error().c_str(); }

}  // extern "C"
