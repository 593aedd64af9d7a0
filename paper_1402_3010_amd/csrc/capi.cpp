// C ABI of the apss library: index construction, self-join, external
// queries.  Host code only orchestrates device work; every step of the
// join runs in the kernels of index_build.hip, join.hip and primitives.hip.
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <new>
#include <string>
#include <vector>

#include "../../include/apss.h"
#include "apss_internal.h"
#include "index_build.h"
#include "join.h"
#include "lib.h"
#include "screen.h"

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

int dev_err(hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
    set_error("%s: out of device memory", what);
    (void)hipGetLastError();
    return APSS_ENOMEM;
  }
  set_error("%s: %s", what, hipGetErrorString(e));
  return APSS_EDEVICE;
}

namespace {

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

#define CHK APSS_CHK

namespace {

// Sort (row, rank) keys with float payload into rank-space rows; checks for duplicates.
// Rows are contiguous in row-major order, so with the row index in the key's
// high bits sorting groups of whole rows independently sorts the whole
// array: given the host row offsets, rows are grouped into segments of at
// most kSortSegment entries, one workgroup each (one launch); otherwise, or
// when a row is longer, radix passes over the whole array.
int sort_rows(Workspace& ws, uint64_t* keys, uint32_t* vals, int64_t nnz, int key_bits, int rbits, RComp* rc_out,
              uint32_t* err_dev, const int64_t* rp_host = nullptr, int64_t nrows = 0) {
  hipStream_t s = ws.stream;
  SortScratch& ss = ws.ss;
  if (rp_host && nnz > kSortSegment && key_bits <= 51) {
    std::vector<int64_t>& seg = ss.seg_host;
    seg.clear();
    seg.push_back(0);
    bool fits = true;
    for (int64_t r = 0; r < nrows && fits; ++r) {
      const int64_t e = rp_host[r + 1];
      if (e - rp_host[r] > kSortSegment) fits = false;
      else if (e - seg.back() > kSortSegment) seg.push_back(rp_host[r]);
    }
    if (fits) {
      if (seg.back() != nnz) seg.push_back(nnz);
      const int64_t nseg = (int64_t)seg.size() - 1;
      CHK(ss.seg.reserve(nseg + 1), "sort scratch");
      CHK(hipMemcpyAsync(ss.seg.p, seg.data(), sizeof(int64_t) * (nseg + 1), hipMemcpyHostToDevice, s), "row sort");
      CHK(segment_sort_u64_u32(keys, vals, ss.seg.p, nseg, s), "row sort");
      CHK(launch_unpack_rows(keys, vals, nnz, rbits, rc_out, err_dev, s), "row unpack");
      return APSS_OK;
    }
  }
  CHK(ss.k2.reserve(nnz), "sort scratch");
  CHK(ss.v32b.reserve(nnz), "sort scratch");
  CHK(ss.hist.reserve(radix_hist_elems(nnz)), "sort scratch");
  CHK(ss.scan.reserve(radix_scan_tmp_elems(nnz)), "sort scratch");
  CHK(radix_sort_u64_u32(keys, vals, ss.k2.p, ss.v32b.p, nnz, key_bits, ss.hist.p, ss.scan.p, s), "row sort");
  CHK(launch_unpack_rows(keys, vals, nnz, rbits, rc_out, err_dev, s), "row unpack");
  return APSS_OK;
}

int check_err(hipStream_t s, uint32_t* err_dev, unsigned long long* bad_dev, const char* what) {
  uint32_t err = 0;
  unsigned long long bad = ~0ull;
  CHK(hipMemcpyAsync(&err, err_dev, sizeof(err), hipMemcpyDeviceToHost, s), what);
  if (bad_dev) CHK(hipMemcpyAsync(&bad, bad_dev, sizeof(bad), hipMemcpyDeviceToHost, s), what);
  CHK(hipStreamSynchronize(s), what);
  if (err) {
    if (bad != ~0ull) set_error("%s: %s (row %llu)", what, err_bits_text(err), bad);
    else set_error("%s: %s", what, err_bits_text(err));
    return APSS_EINVAL;
  }
  return APSS_OK;
}

// Cleared error flag and first-bad-row slot of a workspace.
int reset_err(Workspace& ws) {
  CHK(ws.err.reserve(1), "alloc");
  CHK(ws.bad.reserve(1), "alloc");
  CHK(fill_u32(ws.err.p, 0u, 1, ws.stream), "fill");
  CHK(fill_u64((uint64_t*)ws.bad.p, ~0ull, 1, ws.stream), "fill");
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

int stage_csr(hipStream_t s, int64_t n, const int64_t* row_ptr, const int32_t* col, const float* val, int on_device,
              int64_t* nnz_out, CsrDev& d) {
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

int build_lists(apss_index* ix);

int build_impl(apss_index* ix, const int64_t* row_ptr, const int32_t* col, const float* val, int on_device) {
  Workspace& ws = ix->ws;
  hipStream_t s = ws.stream;
  const int64_t n = ix->n, m = ix->m;
  CsrDev in;
  int64_t nnz = 0;
  int rc = stage_csr(s, n, row_ptr, col, val, on_device, &nnz, in);
  if (rc) return rc;
  ix->nnz = nnz;

  if ((rc = reset_err(ws))) return rc;
  uint32_t* err = ws.err.p;
  unsigned long long* bad = ws.bad.p;
  CHK(launch_check_rowptr(in.prp, n, nnz, err, bad, s), "check row_ptr");
  if ((rc = check_err(s, err, bad, "build_index"))) return rc;
  CHK(launch_validate_rows(in.prp, in.pcol, in.pval, n, m, 1e-5, err, bad, s), "validate");
  if ((rc = check_err(s, err, bad, "build_index"))) return rc;

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
  SortScratch& ss = ws.ss;
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
  ix->rows.rp_host.resize((size_t)n + 1);
  CHK(hipMemcpyAsync(ix->rows.rp_host.data(), in.prp, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost, s), "copy");
  CHK(ix->rows.rc.alloc(nnz), "alloc");
  if ((rc = sort_rows(ws, ss.k1.p, ss.v32a.p, nnz, nbits + rbits, rbits, ix->rows.rc.p, err))) return rc;
  if ((rc = check_err(s, err, nullptr, "build_index"))) return rc;
  return build_lists(ix);
}

// From the rank-space rows on: cutoff of every row, the inverted lists of
// the indexed parts and the lookup tables of the join.
int build_lists(apss_index* ix) {
  Workspace& ws = ix->ws;
  hipStream_t s = ws.stream;
  SortScratch& ss = ws.ss;
  const int64_t n = ix->n, m = ix->m;
  const int rbits = ceil_log2((uint64_t)m);
  int rc = APSS_OK;

  // cutoff of the unindexed part
  CHK(ix->rs.alloc(n), "alloc");
  CHK(ix->rows.mw.alloc(n), "alloc");
  DBuf<int64_t> nidx, scan_tmp, total;
  CHK(nidx.alloc(n + 1), "alloc");
  CHK(scan_tmp.alloc(scan_tmp_elems(n + 1)), "alloc");
  CHK(total.alloc(1), "alloc");
  // head >= 0: the unindexed part of every row is its components of rank
  // below head (the screened join's head cut, or nothing at all for the
  // all-pairs-0-array index); -1: the paper's cutoff
  const int32_t head = ix->opts.index_all ? 0 : (ix->head_cut > 0 ? ix->head_cut : -1);
  CHK(launch_cutoff(ix->rows.rp.p, ix->rows.rc.p, ix->mw_r.p, n, ix->t_build, ix->opts.query_safe ? 1 : 0, head,
                    ix->rs.p, ix->rows.mw.p, nidx.p, s),
      "cutoff");
  CHK(exclusive_scan_i64(nidx.p, n, scan_tmp.p, total.p, s), "scan");
  // the largest unindexed-part norm and each row's as a byte: the hashed
  // filter's tests before it reads a row's statistics
  DBuf<uint32_t> pmax;
  CHK(pmax.alloc(1), "alloc");
  CHK(ix->pn8.alloc(std::max<int64_t>(n, 1)), "alloc");
  CHK(fill_u32(pmax.p, 0u, 1, s), "fill");
  CHK(launch_max_pnrm(ix->rs.p, n, pmax.p, ix->pn8.p, s), "max norm");
  int64_t P = 0;
  uint32_t pmax_bits = 0u;
  CHK(hipMemcpyAsync(&P, total.p, sizeof(int64_t), hipMemcpyDeviceToHost, s), "read P");
  CHK(hipMemcpyAsync(&pmax_bits, pmax.p, sizeof(uint32_t), hipMemcpyDeviceToHost, s), "read max norm");
  CHK(hipStreamSynchronize(s), "read P");
  ix->P = P;
  memcpy(&ix->pnrm_max, &pmax_bits, sizeof(float));
  if (4 * (P + kPost4Pad) >= (1ll << 32)) {
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
  // two padding entries after the last list let the join read positions p
  // and p + 1 for any p <= P (p = 0 too when there are no lists)
  CHK(ix->post.alloc(P + 2), "alloc");
  CHK(fill_u64((uint64_t*)ix->post.p + P, ~0ull, 2, s), "fill");
  CHK(launch_unpack_post(ss.v64a.p, P, ix->post.p, s), "post");
  // the join's list loads put a chunk's base in the scalar offset, which the
  // hardware range check does not cover: 64 zero entries after the last list
  // keep a chunk's lanes past its end inside the allocation
  CHK(ix->post4.alloc(P + kPost4Pad), "alloc");
  CHK(fill_u32(ix->post4.p + P, 0u, kPost4Pad, s), "fill");
  CHK(launch_pack_post4(ix->post.p, P, ix->post4.p, s), "post4");

  // local pruning: split the indexed ranks into parts of about equal
  // postings; ranks are in decreasing density, so the first parts hold the
  // few heaviest lists and the last ones the long tail
  ix->parts = ix->opts.local_parts > 1 ? ix->opts.local_parts : 1;
  if (ix->parts > 1) {
    std::vector<int64_t> off_h((size_t)m + 1);
    CHK(hipMemcpyAsync(off_h.data(), ix->off.p, sizeof(int64_t) * (m + 1), hipMemcpyDeviceToHost, s), "read lists");
    CHK(hipStreamSynchronize(s), "read lists");
    ix->part_lo_host.assign((size_t)ix->parts + 1, 0);
    for (int r = 1; r < ix->parts; ++r) {
      const int64_t target = (P * r + ix->parts - 1) / ix->parts;
      const int64_t k = std::lower_bound(off_h.begin(), off_h.end(), target) - off_h.begin();
      ix->part_lo_host[(size_t)r] = (int32_t)std::max<int64_t>(ix->part_lo_host[(size_t)r - 1], std::min<int64_t>(k, m));
    }
    ix->part_lo_host[(size_t)ix->parts] = (int32_t)m;
    CHK(ix->part_lo.alloc(ix->parts + 1), "alloc");
    CHK(hipMemcpyAsync(ix->part_lo.p, ix->part_lo_host.data(), sizeof(int32_t) * (ix->parts + 1),
                       hipMemcpyHostToDevice, s),
        "parts");
  }

  // per-block offsets of the dense lists, for the default tile variant
  int32_t H = ix->opts.head_dims > 0 ? ix->opts.head_dims : 32768;
  if (H > m) H = (int32_t)m;
  ix->H = H;
  if ((rc = prepare(ix, s, ix->variant, ix->range_rows))) return rc;
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

template <typename T>
int copy_buf(DBuf<T>& dst, const DBuf<T>& src, int64_t count, hipStream_t s) {
  CHK(dst.alloc(count), "alloc");
  if (count > 0) CHK(hipMemcpyAsync(dst.p, src.p, sizeof(T) * count, hipMemcpyDeviceToDevice, s), "copy");
  return APSS_OK;
}

// The head-cut index of the screened join: the same rank-space rows, with
// every row's unindexed part set to its components of rank < head.
int build_screen(apss_index* ix, int32_t head) {
  apss_index* sx = new (std::nothrow) apss_index();
  if (!sx) {
    set_error("host allocation failed");
    return APSS_ENOMEM;
  }
  ix->screen = sx;
  hipStream_t s = ix->ws.stream;
  sx->device = ix->device;
  sx->opts = ix->opts;
  sx->opts.screen_dims = 0;
  sx->ws.stream = s;
  sx->n = ix->n;
  sx->m = ix->m;
  sx->nnz = ix->nnz;
  sx->t_build = ix->t_build;
  sx->variant = ix->variant;
  sx->range_rows = ix->range_rows;
  sx->range_group = ix->range_group;
  sx->head_cut = head;
  sx->rows.n = ix->rows.n;
  sx->rows.nnz = ix->rows.nnz;
  sx->rows.rp_host = ix->rows.rp_host;
  int rc;
  if ((rc = copy_buf(sx->rows.rp, ix->rows.rp, ix->n + 1, s))) return rc;
  if ((rc = copy_buf(sx->rows.rc, ix->rows.rc, ix->nnz, s))) return rc;
  if ((rc = copy_buf(sx->mw_r, ix->mw_r, ix->m, s))) return rc;
  CHK(sx->rows.mw.alloc(ix->n), "alloc");
  return build_lists(sx);
}

// Query tiles: consecutive queries, at most QT of them and, unless a single
// query is larger, at most QB components, so that a tile fits the LDS staging.
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

}  // namespace

namespace apss {

int64_t default_range_rows(int variant) {
  int qt = 0, cb = 1024;
  (void)join_variant_geometry(variant, &qt, &cb);
  // 16,384 rows: the measured best for the self-join and for query batches
  // on corpora of 0.5-2M vectors (the autotuner refines it per workload)
  return (int64_t)std::max(1, 16384 / cb) * cb;
}

int prepare(apss_index* ix, hipStream_t s, int variant, int64_t range_rows) {
  int qt = 0, cb = 0;
  if (join_variant_geometry(variant, &qt, &cb)) {
    set_error("unknown join variant %d", variant);
    return APSS_EINVAL;
  }
  const int64_t K = std::max<int64_t>(1, range_rows / cb);
  range_rows = K * cb;
  std::lock_guard<std::mutex> lock(ix->prep_mu);
  bool built = false;
  const int slot = hoff_slot(cb);
  if (!ix->hoff[slot].p) {
    const int64_t nb = (ix->n + cb - 1) / cb;
    CHK(ix->hoff[slot].alloc((nb + 1) * (int64_t)ix->H), "alloc block offsets");
    CHK(launch_block_offsets(ix->off.p, ix->post.p, ix->H, nb, cb, ix->hoff[slot].p, s), "block offsets");
    ix->hoff_nb[slot] = nb;
    built = true;
  }
  if (!ix->toff.p || ix->toff_rows != range_rows) {
    const int64_t nb = (ix->n + cb - 1) / cb;
    const int64_t nR = (nb + K - 1) / K;
    CHK(ix->toff.alloc((nR + 1) * std::max<int64_t>(ix->m - ix->H, 1)), "alloc range offsets");
    CHK(launch_range_offsets(ix->off.p, ix->post.p, ix->H, ix->m, nR, range_rows, ix->toff.p, s), "range offsets");
    ix->toff_rows = range_rows;
    ix->toff_nR = nR;
    built = true;
  }
  if (!ix->grid[variant]) ix->grid[variant] = join_resident_groups(variant, ix->opts.remscore != 0);
  // other streams read the tables as soon as the lock is released
  if (built) CHK(hipStreamSynchronize(s), "prepare");
  return APSS_OK;
}

int plan_layout(apss_index* ix, const QuerySet& Q, int triangle, JoinLayout& L) {
  const int variant = ix->variant;
  if (join_variant_geometry(variant, &L.QT, &L.CB)) {
    set_error("unknown join variant %d", variant);
    return APSS_EINVAL;
  }
  L.variant = variant;
  L.slot = hoff_slot(L.CB);
  L.nb = ix->hoff_nb[L.slot];
  // work items: ranges of K blocks x query tiles
  const int64_t range_rows = ix->toff_rows;
  L.K = (int)(range_rows / L.CB);
  L.nR = ix->toff_nR;
  L.rg = std::max(1, std::min<int>(ix->range_group, kMaxRangeGroup));
  L.tiles = make_tiles(Q.rp_host, Q.n, L.QT, join_variant_staging(variant));
  L.ntiles = (int64_t)L.tiles.start.size() - 1;
  const int64_t ngroups = (L.nR + L.rg - 1) / L.rg;
  L.nrx = (ngroups + 7) / 8;
  L.parts = ix->parts;
  L.cum.assign((size_t)(8 * (L.nrx + 1)), 0);
  for (int x = 0; x < 8; ++x) {
    int64_t c = 0;
    for (int64_t j = 0; j <= L.nrx; ++j) {
      L.cum[(size_t)(x * (L.nrx + 1) + j)] = c;
      const int64_t g = x + 8 * j;
      const int64_t R = g * L.rg;  // the group's first range
      if (j < L.nrx && g < ngroups) {
        // first tile whose last query reaches the group's first range (self-join triangle)
        const int64_t tmin =
            triangle ? (int64_t)(std::upper_bound(L.tiles.start.begin() + 1, L.tiles.start.end(), R * range_rows) -
                                 (L.tiles.start.begin() + 1))
                     : 0;
        c += (L.ntiles - tmin) * L.parts;
      }
    }
  }
  // no more workgroups than work items: a small batch leaves the rest of
  // the device to work running beside it (another serving slot)
  int64_t items = 0;
  for (int x = 0; x < 8; ++x) items += L.cum[(size_t)(x * (L.nrx + 1) + L.nrx)];
  L.G = (int)std::max<int64_t>(1, std::min<int64_t>(ix->grid[variant], items));
  // per-workgroup cursor space for tiles too large to stage in LDS
  L.wg_stride = 2 * std::max<int64_t>(L.tiles.max_nnz, 1);
  return APSS_OK;
}

void bind_plan(apss_index* ix, const QuerySet& Q, int triangle, float t, const float* qt_dev, const RowStat* qrs,
               const JoinLayout& L, const int64_t* tstart_dev, const int64_t* qcum_dev, unsigned int* qctr_dev,
               uint32_t* wg_cur_dev, JoinPlan& P) {
  JoinArgs& a = P.a;
  a = JoinArgs{};
  a.rp = ix->rows.rp.p;
  a.rc = ix->rows.rc.p;
  a.rs = ix->rs.p;
  a.pnrm_max = ix->pnrm_max;
  a.pn8 = ix->pn8.p;
  a.off = ix->off.p;
  a.post = ix->post.p;
  a.post4 = ix->post4.p;
  a.post4_bytes = (uint32_t)(4 * (ix->P + kPost4Pad));
  a.hoff = ix->hoff[L.slot].p;
  a.H = ix->H;
  a.nb = L.nb;
  a.n = ix->n;
  a.qrp = Q.rp;
  a.qrc = Q.rc;
  a.qmw = Q.mw;
  a.qrs = qrs;
  a.qt = qt_dev;
  a.t = t;
  a.nq = Q.n;
  a.triangle = triangle;
  a.ntiles = L.ntiles;
  a.tstart = tstart_dev;
  a.toff = ix->toff.p;
  a.m_tail = (int32_t)(ix->m - ix->H);
  a.K = L.K;
  a.rg = L.rg;
  a.nR = (int32_t)L.nR;
  a.nrx = L.nrx;
  a.qcum = qcum_dev;
  a.qctr = qctr_dev;
  a.wg_cur = wg_cur_dev;
  a.wg_cur_stride = L.wg_stride;
  a.parts = L.parts;
  a.part_lo = L.parts > 1 ? ix->part_lo.p : nullptr;
  a.qadm = nullptr;
  P.variant = L.variant;
  P.G = L.G;
  P.bj = ceil_log2((uint64_t)ix->n);
  P.bi = ceil_log2((uint64_t)(triangle ? ix->n : Q.n));
  a.bj = P.bj;
}

int plan_join(apss_index* ix, Workspace& ws, const QuerySet& Q, int triangle, float t, const float* qt_dev,
              const RowStat* qrs, JoinPlan& P) {
  hipStream_t s = ws.stream;
  int rc0 = prepare(ix, s, ix->variant, ix->range_rows);
  if (rc0) return rc0;
  JoinLayout L;
  if ((rc0 = plan_layout(ix, Q, triangle, L))) return rc0;
  CHK(ws.tstart.reserve(L.ntiles + 1), "alloc tiles");
  CHK(hipMemcpyAsync(ws.tstart.p, L.tiles.start.data(), sizeof(int64_t) * (L.ntiles + 1), hipMemcpyHostToDevice, s),
      "tiles");
  CHK(ws.qcum.reserve((int64_t)L.cum.size()), "alloc queues");
  CHK(hipMemcpyAsync(ws.qcum.p, L.cum.data(), sizeof(int64_t) * L.cum.size(), hipMemcpyHostToDevice, s), "queues");
  CHK(ws.qctr.reserve(8), "alloc queues");
  CHK(ws.counters.reserve(C_NUM), "alloc counters");
  CHK(ws.wg_cur.reserve((int64_t)L.G * L.wg_stride), "alloc cursors");
  bind_plan(ix, Q, triangle, t, qt_dev, qrs, L, ws.tstart.p, ws.qcum.p, ws.qctr.p, ws.wg_cur.p, P);
  return APSS_OK;
}

// Launch a planned join writing pairs into ws.raw_key / raw_sim through ws.counters.
int launch_planned(Workspace& ws, JoinPlan& P) {
  JoinArgs& a = P.a;
  a.out_key = ws.raw_key.p;
  a.out_sim = ws.raw_sim.p;
  a.cap = ws.raw_key.n;
  a.counters = ws.counters.p;
  a.qctr = ws.qctr.p;
  CHK(fill_u32(ws.qctr.p, 0u, 8, ws.stream), "fill");
  if (!join_args_complete(a)) {
    set_error("internal: join launched with a missing device buffer");
    return APSS_EDEVICE;
  }
  CHK(launch_join(a, P.variant, P.G, ws.stream), "join kernel");
  return APSS_OK;
}

int ensure_pair_capacity(Workspace& ws, int64_t cap) {
  if (ws.raw_key.p && ws.raw_key.n >= cap) return APSS_OK;
  cap = std::max<int64_t>(cap, 1 << 16);
  CHK(ws.raw_key.alloc(cap), "alloc pairs");
  CHK(ws.raw_sim.alloc(cap), "alloc pairs");
  return APSS_OK;
}

int sort_pairs(Workspace& ws, int64_t matches, int key_bits) {
  SortScratch& ss = ws.ss;
  // 1.5x: after the sort this scratch holds the unpacked (i, j, sim) arrays
  // of finish_host, so that call never reallocates it under queued work
  CHK(ss.k2.reserve(matches + matches / 2 + 1), "alloc sort");
  CHK(ss.v32b.reserve(matches), "alloc sort");
  CHK(ss.hist.reserve(radix_hist_elems(matches)), "alloc sort");
  CHK(ss.scan.reserve(radix_scan_tmp_elems(matches)), "alloc sort");
  CHK(radix_sort_u64_u32(ws.raw_key.p, (uint32_t*)ws.raw_sim.p, ss.k2.p, ss.v32b.p, matches, key_bits, ss.hist.p,
                         ss.scan.p, ws.stream),
      "pair sort");
  return APSS_OK;
}

void take_counters(Workspace& ws, const unsigned long long* c) {
  ws.last.posting_visits = (int64_t)(c[C_VISITS] + c[C_TAILVISITS]);
  ws.last.candidates = (int64_t)c[C_CANDIDATES];
  ws.last.bound_survivors = (int64_t)c[C_SURVIVORS];
  ws.last.verified = (int64_t)c[C_VERIFIED];
  ws.last.band = (int64_t)c[C_BAND];
  ws.last.matches = (int64_t)c[C_MATCHES];
}

// Every call on a workspace starts here.  Any call other than a graph
// replay may rewrite buffers a captured graph reads, so it drops the graph.
int start_call(Workspace& ws, bool keep_graph = false) {
  if (!keep_graph) ws.graph.reset();
  memset(&ws.last, 0, sizeof(ws.last));
  for (int e = 0; e < 6; ++e)
    if (!ws.ev[e]) CHK(hipEventCreateWithFlags(&ws.ev[e], hipEventDefault), "event");
  CHK(hipEventRecord(ws.ev[0], ws.stream), "event");
  return APSS_OK;
}

int run_join(apss_index* ix, Workspace& ws, const QuerySet& Q, int triangle, float t, const float* qt_dev,
             int64_t cap_hint, int64_t* count) {
  hipStream_t s = ws.stream;
  *count = 0;
  int rc = start_call(ws);
  if (rc) return rc;
  if (Q.n == 0 || ix->n == 0) return APSS_OK;
  JoinPlan P;
  if ((rc = plan_join(ix, ws, Q, triangle, t, qt_dev, nullptr, P))) return rc;
  if ((rc = ensure_pair_capacity(ws, cap_hint))) return rc;
  if (ix->opts.remscore) {
    // each query's first component that admits new candidates (remscore)
    CHK(ws.qadm.reserve(Q.n), "alloc");
    CHK(launch_admit_pos(Q.rp, Q.rc, ix->mw_r.p, qt_dev, t, Q.n, ws.qadm.p, s), "admission");
    P.a.qadm = ws.qadm.p;
  }
  for (int attempt = 0; attempt < 2; ++attempt) {
    CHK(fill_u64((uint64_t*)ws.counters.p, 0ull, C_NUM, s), "fill");
    CHK(hipEventRecord(ws.ev[1], s), "event");
    if ((rc = launch_planned(ws, P))) return rc;
    CHK(hipEventRecord(ws.ev[2], s), "event");
    unsigned long long c[C_NUM];
    CHK(hipMemcpyAsync(c, ws.counters.p, sizeof(c), hipMemcpyDeviceToHost, s), "read counters");
    CHK(hipStreamSynchronize(s), "join");
    const int64_t matches = (int64_t)c[C_MATCHES];
    if (matches > ws.raw_key.n) {
      if ((rc = ensure_pair_capacity(ws, matches + matches / 8 + 1024))) return rc;
      ++ws.regrows;
      continue;  // rerun with room for every pair
    }
    take_counters(ws, c);
    float ms = 0.0f;
    CHK(hipEventElapsedTime(&ms, ws.ev[1], ws.ev[2]), "event");
    ws.last.ms_candidates = ms;
    if ((rc = sort_pairs(ws, matches, P.bi + P.bj))) return rc;
    int64_t distinct = matches;
    if (P.a.parts > 1 && matches > 1) {
      // a pair kept by several parts was emitted once by each, with the same
      // rescored similarity: keep one copy
      SortScratch& ss = ws.ss;
      CHK(ss.v64a.reserve(matches), "alloc");
      CHK(ss.v64b.reserve(scan_tmp_elems(matches)), "alloc");
      CHK(ws.uniq_total.reserve(1), "alloc");
      CHK(unique_sorted_u64_u32(ws.raw_key.p, (uint32_t*)ws.raw_sim.p, matches, (int64_t*)ss.v64a.p,
                                (int64_t*)ss.v64b.p, ws.uniq_total.p, ss.k2.p, ss.v32b.p, s),
          "unique pairs");
      CHK(hipMemcpyAsync(&distinct, ws.uniq_total.p, sizeof(int64_t), hipMemcpyDeviceToHost, s), "unique pairs");
      CHK(hipStreamSynchronize(s), "unique pairs");
      ws.last.matches = distinct;
    }
    *count = distinct;
    return APSS_OK;
  }
  set_error("pair buffer kept overflowing");
  return APSS_ENOMEM;
}

// Screened self-join: the bf16 MFMA head screen (pairs that share no tail
// dimension) and the sparse pass over the head-cut index (pairs that share
// one), written into one pair buffer and sorted together.
int run_screen_join(apss_index* ix, Workspace& ws, float t, int64_t cap_hint, int64_t* count) {
  apss_index* sx = ix->screen;
  hipStream_t s = ws.stream;
  *count = 0;
  if (!screen_variant_ok(sx->variant)) {
    set_error("tile variant %d is not available for the screened join", sx->variant);
    return APSS_EINVAL;
  }
  int rc = start_call(ws);
  if (rc) return rc;
  const int64_t n = sx->n;
  if (n == 0) return APSS_OK;
  const int32_t head = sx->head_cut;
  const int32_t ld = (int32_t)((head + kScreenK - 1) / kScreenK * kScreenK);
  const int bj = ceil_log2((uint64_t)n);

  // rows whose head norm reaches t, by decreasing head norm
  CHK(ws.s_keys.reserve(n), "alloc screen");
  CHK(ws.s_cnt.reserve(1), "alloc screen");
  CHK(fill_u64((uint64_t*)ws.s_cnt.p, 0ull, 1, s), "fill");
  CHK(launch_screen_select(sx->rs.p, n, t, ws.s_keys.p, ws.s_cnt.p, s), "screen select");
  unsigned long long S64 = 0;
  CHK(hipMemcpyAsync(&S64, ws.s_cnt.p, sizeof(S64), hipMemcpyDeviceToHost, s), "screen select");
  CHK(hipStreamSynchronize(s), "screen select");
  const int64_t S = (int64_t)S64;
  const int64_t Sp = (S + kScreenTileB - 1) / kScreenTileB * kScreenTileB;
  int64_t nc = 0, ntiles = 0, useful = 0;
  if (S > 1) {
    SortScratch& ss = ws.ss;
    CHK(ss.k2.reserve(S), "alloc sort");
    CHK(ss.v32a.reserve(S), "alloc sort");
    CHK(ss.v32b.reserve(S), "alloc sort");
    CHK(ss.hist.reserve(radix_hist_elems(S)), "alloc sort");
    CHK(ss.scan.reserve(radix_scan_tmp_elems(S)), "alloc sort");
    CHK(radix_sort_u64_u32(ws.s_keys.p, ss.v32a.p, ss.k2.p, ss.v32b.p, S, 64, ss.hist.p, ss.scan.p, s), "screen sort");
    CHK(ws.s_sid.reserve(Sp), "alloc screen");
    CHK(ws.s_nh.reserve(Sp), "alloc screen");
    CHK(launch_screen_unpack(ws.s_keys.p, S, Sp, ws.s_sid.p, ws.s_nh.p, s), "screen unpack");
    CHK(ws.s_X.reserve(Sp * ld), "alloc screen block");
    CHK(fill_u32((uint32_t*)ws.s_X.p, 0u, Sp * ld / 2, s), "fill");
    CHK(launch_screen_pack(sx->rows.rp.p, sx->rows.rc.p, ws.s_sid.p, S, head, ld, ws.s_X.p, s), "screen pack");
    // tiles (I, J) of kScreenTile x kScreenTileB rows that reach the upper
    // triangle (2 J + 1 >= I) and whose largest norm product reaches t (rows
    // are in decreasing head norm, so a tile's first rows have the largest);
    // `useful` counts the kScreenTile x kScreenTile pairs I <= J among them
    std::vector<float> nh((size_t)Sp);
    CHK(hipMemcpyAsync(nh.data(), ws.s_nh.p, sizeof(float) * Sp, hipMemcpyDeviceToHost, s), "screen norms");
    CHK(hipStreamSynchronize(s), "screen norms");
    const int64_t T = Sp / kScreenTile, TB = Sp / kScreenTileB;
    std::vector<int32_t> tl;
    for (int64_t I = 0; I < T; ++I) {
      const float nI = nh[(size_t)(I * kScreenTile)];
      for (int64_t J = I; J < T; ++J) {
        if (nI * nh[(size_t)(J * kScreenTile)] * (1.0f + 0x1p-20f) < t) break;
        ++useful;
      }
      for (int64_t J = I / 2; J < TB; ++J) {
        if (nI * nh[(size_t)(J * kScreenTileB)] * (1.0f + 0x1p-20f) < t) break;
        tl.push_back((int32_t)I);
        tl.push_back((int32_t)J);
      }
    }
    ntiles = (int64_t)tl.size() / 2;
    // blocks of kScreenBlock x kScreenBlock row tiles in turn: the
    // workgroups that run at once on an XCD then share a few panels of each
    // operand (from L2 and the last-level cache) instead of streaming a new
    // second operand panel per tile from HBM (C4 with 128 x 128 tiles:
    // 8.0 -> 6.6 ms; blocks of 4 and 16 within 0.1 ms of 8, of 32 7.5 ms)
    {
      const int B = kScreenBlock;
      if (B > 1) {
        std::vector<std::array<int32_t, 4>> key((size_t)ntiles);
        for (int64_t k = 0; k < ntiles; ++k) {
          const int32_t I = tl[(size_t)(2 * k)], J = tl[(size_t)(2 * k + 1)];
          key[(size_t)k] = {I / B, J / (B * kScreenTile / kScreenTileB), I, J};
        }
        std::sort(key.begin(), key.end());
        for (int64_t k = 0; k < ntiles; ++k) {
          tl[(size_t)(2 * k)] = key[(size_t)k][2];
          tl[(size_t)(2 * k + 1)] = key[(size_t)k][3];
        }
      }
    }
    if (ntiles > 0) {
      CHK(ws.s_tiles.reserve((int64_t)tl.size()), "alloc screen");
      CHK(hipMemcpyAsync(ws.s_tiles.p, tl.data(), sizeof(int32_t) * tl.size(), hipMemcpyHostToDevice, s),
          "screen tiles");
      CHK(ws.s_cand.reserve(std::max<int64_t>(1 << 16, 4 * S)), "alloc screen");
      for (int attempt = 0; attempt < 2; ++attempt) {
        CHK(fill_u64((uint64_t*)ws.s_cnt.p, 0ull, 1, s), "fill");
        ScreenArgs A{};
        A.X = ws.s_X.p;
        A.ld = ld;
        A.nh = ws.s_nh.p;
        A.sid = ws.s_sid.p;
        A.tiles = ws.s_tiles.p;
        A.ntiles = ntiles;
        A.t = t;
        A.bj = bj;
        A.out = ws.s_cand.p;
        A.cap = ws.s_cand.n;
        A.count = ws.s_cnt.p;
        CHK(hipEventRecord(ws.ev[4], s), "event");
        CHK(launch_screen_mfma(A, s), "screen kernel");
        CHK(hipEventRecord(ws.ev[5], s), "event");
        unsigned long long c = 0;
        CHK(hipMemcpyAsync(&c, ws.s_cnt.p, sizeof(c), hipMemcpyDeviceToHost, s), "screen count");
        CHK(hipStreamSynchronize(s), "screen kernel");
        nc = (int64_t)c;
        if (nc > ws.s_cand.n) {
          CHK(ws.s_cand.alloc(nc + nc / 8 + 1024), "alloc screen");
          continue;
        }
        float ms = 0.0f;
        CHK(hipEventElapsedTime(&ms, ws.ev[4], ws.ev[5]), "event");
        ws.last.ms_screen = ms;
        break;
      }
      if (nc > ws.s_cand.n) {
        set_error("screen candidate buffer kept overflowing");
        return APSS_ENOMEM;
      }
    }
  }

  // sparse pass over the head-cut index, then the exact check of the screen's candidates
  JoinPlan P;
  if ((rc = plan_join(sx, ws, QuerySet{sx->rows.rp.p, sx->rows.rc.p, sx->rows.mw.p, n, sx->nnz,
                                       sx->rows.rp_host.data()},
                      1, t, nullptr, sx->rs.p, P)))
    return rc;
  if ((rc = ensure_pair_capacity(ws, cap_hint))) return rc;
  for (int attempt = 0; attempt < 2; ++attempt) {
    CHK(fill_u64((uint64_t*)ws.counters.p, 0ull, C_NUM, s), "fill");
    CHK(hipEventRecord(ws.ev[1], s), "event");
    if ((rc = launch_planned(ws, P))) return rc;
    CHK(hipEventRecord(ws.ev[2], s), "event");
    CHK(launch_screen_verify(ws.s_cand.p, nc, bj, sx->rows.rp.p, sx->rows.rc.p, head, t, ws.raw_key.p, ws.raw_sim.p,
                             ws.raw_key.n, ws.counters.p, s),
        "screen verify");
    unsigned long long c[C_NUM];
    CHK(hipMemcpyAsync(c, ws.counters.p, sizeof(c), hipMemcpyDeviceToHost, s), "read counters");
    CHK(hipStreamSynchronize(s), "join");
    const int64_t matches = (int64_t)c[C_MATCHES];
    if (matches > ws.raw_key.n) {
      if ((rc = ensure_pair_capacity(ws, matches + matches / 8 + 1024))) return rc;
      ++ws.regrows;
      continue;
    }
    const double ms_screen = ws.last.ms_screen;
    take_counters(ws, c);
    ws.last.ms_screen = ms_screen;
    ws.last.screen_rows = S;
    ws.last.screen_tiles = useful;
    ws.last.screen_candidates = nc;
    ws.last.screen_ld = ld;
    float ms = 0.0f;
    CHK(hipEventElapsedTime(&ms, ws.ev[1], ws.ev[2]), "event");
    ws.last.ms_candidates = ms;
    if ((rc = sort_pairs(ws, matches, 2 * bj))) return rc;
    *count = matches;
    return APSS_OK;
  }
  set_error("pair buffer kept overflowing");
  return APSS_ENOMEM;
}

}  // namespace apss

namespace {

// Pair capacity a self-join starts with (grows on overflow, which reruns
// the join kernel): 32 pairs per vector, 384 MB of pair buffers per million
// vectors, which holds the matches of the million-vector workloads at their
// thresholds (about 22 per vector at t = 0.7) on the first call.
int64_t join_cap_hint(const apss_index* ix) { return std::max<int64_t>(1 << 20, 32 * ix->n); }

std::vector<const void*> graph_buffers(const apss_index* ix, const Workspace& ws) {
  return {ws.tstart.p, ws.qcum.p, ws.qctr.p, ws.counters.p, ws.wg_cur.p, ws.raw_key.p, ws.raw_sim.p, ws.ss.k2.p,
          ws.ss.v32b.p, ws.ss.hist.p, ws.ss.scan.p, ix->toff.p, ix->hoff[0].p, ix->hoff[1].p,
          (const void*)(intptr_t)ix->variant, (const void*)(intptr_t)ix->range_rows,
          (const void*)(intptr_t)ix->range_group};
}

// Capture the launch sequence of the self-join that just ran (count pairs).
int capture_join_graph(apss_index* ix, float t, uint32_t* out_i, uint32_t* out_j, float* out_sim, int64_t capacity,
                       int64_t cnt) {
  Workspace& ws = ix->ws;
  JoinGraph& g = ws.graph;
  hipStream_t s = ws.stream;
  g.reset();
  if (!s) return APSS_OK;  // the legacy default stream cannot be captured
  if (!g.hctr) CHK(hipHostMalloc((void**)&g.hctr, sizeof(unsigned long long) * C_NUM, hipHostMallocDefault),
                   "pinned counters");
  JoinPlan P;
  int rc = plan_join(ix, ws, QuerySet{ix->rows.rp.p, ix->rows.rc.p, ix->rows.mw.p, ix->n, ix->nnz,
                                      ix->rows.rp_host.data()},
                     1, t, nullptr, nullptr, P);
  if (rc) return rc;
  CHK(hipStreamSynchronize(s), "graph capture");
  CHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "graph capture");
  auto body = [&]() -> int {
    CHK(fill_u64((uint64_t*)ws.counters.p, 0ull, C_NUM, s), "fill");
    int r = launch_planned(ws, P);
    if (r) return r;
    CHK(hipMemcpyAsync(g.hctr, ws.counters.p, sizeof(unsigned long long) * C_NUM, hipMemcpyDeviceToHost, s),
        "read counters");
    if ((r = sort_pairs(ws, cnt, P.bi + P.bj))) return r;
    CHK(launch_unpack_pairs(ws.raw_key.p, ws.raw_sim.p, cnt, P.bj, out_i, out_j, out_sim, s), "unpack");
    return APSS_OK;
  };
  rc = body();
  hipGraph_t graph = nullptr;
  const hipError_t ee = hipStreamEndCapture(s, &graph);
  if (!rc && ee != hipSuccess) rc = dev_err(ee, "graph capture");
  if (!rc) {
    const hipError_t ei = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
      g.exec = nullptr;
      rc = dev_err(ei, "graph instantiate");
    }
  }
  if (graph) (void)hipGraphDestroy(graph);
  if (rc) return rc;
  g.t = t;
  g.out[0] = out_i;
  g.out[1] = out_j;
  g.out[2] = out_sim;
  g.capacity = capacity;
  g.count = cnt;
  g.baked = graph_buffers(ix, ws);
  return APSS_OK;
}

// apss_join_device with graph replay (plain self-join).
int graph_join(apss_index* ix, float t, uint32_t* out_i, uint32_t* out_j, float* out_sim, int64_t capacity,
               int64_t* count) {
  Workspace& ws = ix->ws;
  JoinGraph& g = ws.graph;
  hipStream_t s = ws.stream;
  int rc;
  if (g.exec && g.t == t && g.out[0] == out_i && g.out[1] == out_j && g.out[2] == out_sim &&
      g.capacity == capacity && g.baked == graph_buffers(ix, ws)) {
    if ((rc = start_call(ws, true))) return rc;
    CHK(hipEventRecord(ws.ev[1], s), "event");
    CHK(hipGraphLaunch(g.exec, s), "graph launch");
    CHK(hipEventRecord(ws.ev[2], s), "event");
    CHK(hipStreamSynchronize(s), "graph launch");
    if ((int64_t)g.hctr[C_MATCHES] == g.count) {
      take_counters(ws, g.hctr);
      float ms = 0.0f;
      CHK(hipEventElapsedTime(&ms, ws.ev[1], ws.ev[2]), "event");
      ws.last.ms_candidates = ms;
      CHK(hipEventElapsedTime(&ms, ws.ev[0], ws.ev[2]), "event");
      ws.last.ms_total = ms;
      *count = g.count;
      return APSS_OK;
    }
    g.reset();  // cannot happen for a deterministic join; recompute eagerly
  }
  int64_t cnt = 0;
  if ((rc = run_join(ix, ws, QuerySet{ix->rows.rp.p, ix->rows.rc.p, ix->rows.mw.p, ix->n, ix->nnz,
                                      ix->rows.rp_host.data()},
                     1, t, nullptr, join_cap_hint(ix), &cnt)))
    return rc;
  if ((rc = finish_device(ws, cnt, ceil_log2((uint64_t)ix->n), out_i, out_j, out_sim, capacity, count))) return rc;
  const apss_stats keep = ws.last;
  rc = capture_join_graph(ix, t, out_i, out_j, out_sim, capacity, cnt);
  ws.last = keep;
  return rc;
}

}  // namespace

namespace apss {

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

// wait = false leaves the stream running; the caller synchronises and then
// calls record_total.
int record_total(Workspace& ws) {
  float ms = 0.0f;
  CHK(hipEventElapsedTime(&ms, ws.ev[0], ws.ev[3]), "event");
  ws.last.ms_total = ms;
  return APSS_OK;
}

int finish_device(Workspace& ws, int64_t cnt, int bj, uint32_t* out_i, uint32_t* out_j, float* out_sim,
                  int64_t capacity, int64_t* count, bool wait) {
  *count = cnt;
  if (cnt > capacity) {
    set_error("output capacity %lld too small for %lld pairs", (long long)capacity, (long long)cnt);
    return APSS_ERANGE;
  }
  CHK(launch_unpack_pairs(ws.raw_key.p, ws.raw_sim.p, cnt, bj, out_i, out_j, out_sim, ws.stream), "unpack");
  CHK(hipEventRecord(ws.ev[3], ws.stream), "event");
  if (!wait) return APSS_OK;
  CHK(hipStreamSynchronize(ws.stream), "unpack");
  return record_total(ws);
}

int finish_host(Workspace& ws, int64_t cnt, int bj, apss_pairs* out) {
  out->count = 0;
  out->i = out->j = nullptr;
  out->sim = nullptr;
  // the sort's second key buffer is free once the pairs are sorted: unpack
  // there, i, j and sim one after another, so that one copy brings them over
  SortScratch& ss = ws.ss;
  CHK(ss.k2.reserve(cnt + cnt / 2 + 1), "alloc");
  uint32_t* di = (uint32_t*)ss.k2.p;
  uint32_t* dj = di + cnt;
  float* ds = (float*)(dj + cnt);
  int64_t c2 = 0;
  int rc = finish_device(ws, cnt, bj, di, dj, ds, cnt, &c2, false);
  if (rc) {
    (void)hipStreamSynchronize(ws.stream);
    return rc;
  }
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
    (void)hipStreamSynchronize(ws.stream);
    set_error("host allocation failed");
    return APSS_ENOMEM;
  }
  // up to 4M pairs through the workspace's pinned staging in one copy;
  // larger results straight into the output arrays
  if (cnt && cnt <= (4ll << 20) && ws.host_out.reserve((size_t)(3 * cnt))) {
    CHK(hipMemcpyAsync(ws.host_out.p, di, sizeof(uint32_t) * 3 * cnt, hipMemcpyDeviceToHost, ws.stream), "copy out");
    CHK(hipStreamSynchronize(ws.stream), "copy out");
    memcpy(out->i, ws.host_out.p, sizeof(uint32_t) * cnt);
    memcpy(out->j, ws.host_out.p + cnt, sizeof(uint32_t) * cnt);
    memcpy(out->sim, ws.host_out.p + 2 * cnt, sizeof(float) * cnt);
  } else {
    if (cnt) {
      CHK(hipMemcpyAsync(out->i, di, sizeof(uint32_t) * cnt, hipMemcpyDeviceToHost, ws.stream), "copy out");
      CHK(hipMemcpyAsync(out->j, dj, sizeof(uint32_t) * cnt, hipMemcpyDeviceToHost, ws.stream), "copy out");
      CHK(hipMemcpyAsync(out->sim, ds, sizeof(float) * cnt, hipMemcpyDeviceToHost, ws.stream), "copy out");
    }
    CHK(hipStreamSynchronize(ws.stream), "copy out");
  }
  if ((rc = record_total(ws))) return rc;
  out->count = cnt;
  return APSS_OK;
}

int stage_queries(apss_index* ix, Workspace& ws, int64_t nq, const int64_t* q_row_ptr, const int32_t* q_col,
                  const float* q_val, int on_device, const float* t_per_row, float t, RankRows& rows) {
  hipStream_t s = ws.stream;
  ws.graph.reset();  // the staging reuses buffers a captured join graph reads
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
  int64_t nnz = 0;
  int rc;
  if ((rc = reset_err(ws))) return rc;
  uint32_t* err = ws.err.p;
  unsigned long long* bad = ws.bad.p;
  const int64_t* prp;
  const int32_t* pcol;
  const float* pval;
  CsrDev in;
  rows.n = nq;
  if (on_device) {
    if ((rc = stage_csr(s, nq, q_row_ptr, q_col, q_val, on_device, &nnz, in))) return rc;
    CHK(launch_check_rowptr(in.prp, nq, nnz, err, bad, s), "check row_ptr");
    if ((rc = check_err(s, err, bad, "query"))) return rc;
    CHK(rows.rp.reserve(nq + 1), "alloc");
    CHK(hipMemcpyAsync(rows.rp.p, in.prp, sizeof(int64_t) * (nq + 1), hipMemcpyDeviceToDevice, s), "copy");
    rows.rp_host.resize((size_t)nq + 1);
    CHK(hipMemcpyAsync(rows.rp_host.data(), in.prp, sizeof(int64_t) * (nq + 1), hipMemcpyDeviceToHost, s), "copy");
    prp = in.prp;
    pcol = in.pcol;
    pval = in.pval;
  } else {
    // host rows: checked here, copied into the workspace's kept buffers,
    // with no synchronisation before the single error check below
    nnz = q_row_ptr[nq];
    if (q_row_ptr[0] != 0 || nnz < 0 || nnz >= (1ll << 32)) {
      set_error("row_ptr must start at 0 and end at nnz in [0, 2^32)");
      return APSS_EINVAL;
    }
    for (int64_t r = 0; r < nq; ++r)
      if (q_row_ptr[r + 1] < q_row_ptr[r]) {
        set_error("row_ptr must be non-decreasing (row %lld)", (long long)r);
        return APSS_EINVAL;
      }
    // every buffer is reserved before the first copy of the caller's
    // memory is queued, so no early return leaves such a copy in flight
    CHK(rows.rp.reserve(nq + 1), "alloc");
    CHK(ws.q_col.reserve(nnz), "alloc");
    CHK(ws.q_val.reserve(nnz), "alloc");
    CHK(rows.rc.reserve(nnz), "alloc");
    CHK(rows.mw.reserve(nq), "alloc");
    CHK(ws.ss.k1.reserve(nnz), "alloc");
    CHK(ws.ss.v32a.reserve(nnz), "alloc");
    CHK(ws.ss.k2.reserve(nnz), "sort scratch");
    CHK(ws.ss.v32b.reserve(nnz), "sort scratch");
    CHK(ws.ss.hist.reserve(radix_hist_elems(nnz)), "sort scratch");
    CHK(ws.ss.scan.reserve(radix_scan_tmp_elems(nnz)), "sort scratch");
    CHK(ws.ss.seg.reserve(nq + 2), "sort scratch");
    if (t_per_row) CHK(ws.qt.reserve(nq), "alloc");
    CHK(hipMemcpyAsync(rows.rp.p, q_row_ptr, sizeof(int64_t) * (nq + 1), hipMemcpyHostToDevice, s), "copy csr");
    if (nnz) {
      CHK(hipMemcpyAsync(ws.q_col.p, q_col, sizeof(int32_t) * nnz, hipMemcpyHostToDevice, s), "copy csr");
      CHK(hipMemcpyAsync(ws.q_val.p, q_val, sizeof(float) * nnz, hipMemcpyHostToDevice, s), "copy csr");
    }
    rows.rp_host.assign(q_row_ptr, q_row_ptr + nq + 1);
    prp = rows.rp.p;
    pcol = ws.q_col.p;
    pval = ws.q_val.p;
  }
  rows.nnz = nnz;
  if (t_per_row) {
    CHK(ws.qt.reserve(nq), "alloc");
    CHK(hipMemcpyAsync(ws.qt.p, t_per_row, sizeof(float) * nq, hipMemcpyHostToDevice, s), "copy thresholds");
  }
  CHK(rows.rc.reserve(nnz), "alloc");
  CHK(rows.mw.reserve(nq), "alloc");
  SortScratch& ss = ws.ss;
  CHK(ss.k1.reserve(nnz), "alloc");
  CHK(ss.v32a.reserve(nnz), "alloc");
  const int rbits = ceil_log2((uint64_t)ix->m);
  const int nbits = ceil_log2((uint64_t)std::max<int64_t>(nq, 1));
  // invalid dimensions get a valid key, so the sort runs before the check
  CHK(launch_query_keys(prp, pcol, pval, ix->rank.p, nq, ix->m, rbits, 1e-5, ss.k1.p, ss.v32a.p, rows.mw.p, err, bad, s),
      "query keys");
  if ((rc = sort_rows(ws, ss.k1.p, ss.v32a.p, nnz, nbits + rbits, rbits, rows.rc.p, err, rows.rp_host.data(), nq)))
    return rc;
  // also completes the copies of the caller's host buffers (borrowed)
  if ((rc = check_err(s, err, bad, "query"))) return rc;
  return APSS_OK;
}

}  // namespace apss

namespace {

QuerySet corpus_queries(const apss_index* ix) {
  return QuerySet{ix->rows.rp.p, ix->rows.rc.p, ix->rows.mw.p, ix->n, ix->nnz, ix->rows.rp_host.data()};
}

QuerySet staged_queries(const RankRows& r) {
  return QuerySet{r.rp.p, r.rc.p, r.mw.p, r.n, r.nnz, r.rp_host.data()};
}

int self_join(apss_index* ix, float t, int64_t* cnt) {
  if (ix->screen) return run_screen_join(ix, ix->ws, t, join_cap_hint(ix), cnt);
  return run_join(ix, ix->ws, corpus_queries(ix), 1, t, nullptr, join_cap_hint(ix), cnt);
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
  o->range_rows = 0;
  o->screen_dims = 0;
  o->graph = 0;
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
  if (o.variant < -1 || o.variant >= join_num_variants() || (o.variant >= 0 && !variant_available(o.variant))) {
    set_error("variant %d is not available (outside [-1, %d) or withdrawn)", o.variant, join_num_variants());
    return APSS_EINVAL;
  }
  if (o.range_rows < 0) {
    set_error("range_rows must be >= 0");
    return APSS_EINVAL;
  }
  if (o.range_group < 0 || o.range_group > kMaxRangeGroup) {
    set_error("range_group must be in [0, %d]", kMaxRangeGroup);
    return APSS_EINVAL;
  }
  if (o.screen_dims < 0 || o.screen_dims > kScreenMaxHead) {
    set_error("screen_dims must be in [0, %d]", kScreenMaxHead);
    return APSS_EINVAL;
  }
  if (o.index_all < 0 || o.index_all > 1 || o.remscore < 0 || o.remscore > 1) {
    set_error("index_all and remscore must be 0 or 1");
    return APSS_EINVAL;
  }
  if (!(o.local_parts == 0 || o.local_parts == 1 || o.local_parts == 2 || o.local_parts == 4 || o.local_parts == 8)) {
    set_error("local_parts must be 0, 1, 2, 4 or 8");
    return APSS_EINVAL;
  }
  if (o.screen_dims > 0 && (o.index_all || o.local_parts > 1 || o.remscore)) {
    set_error("screen_dims does not combine with index_all, local_parts or remscore");
    return APSS_EINVAL;
  }
  apss_index* ix = new (std::nothrow) apss_index();
  if (!ix) {
    set_error("host allocation failed");
    return APSS_ENOMEM;
  }
  ix->opts = o;
  ix->ws.stream = (hipStream_t)o.stream;
  ix->n = n;
  ix->m = m;
  ix->t_build = t_build;
  ix->variant = o.variant >= 0 ? o.variant : 1;
  if (const char* ev = getenv("APSS_VARIANT")) {
    const int v = atoi(ev);
    if (v >= 0 && v < join_num_variants() && variant_available(v)) ix->variant = v;
  }
  ix->range_rows = o.range_rows > 0 ? o.range_rows : default_range_rows(ix->variant);
  if (const char* ev = getenv("APSS_RANGE_ROWS")) {
    const long long rr = atoll(ev);
    if (rr > 0) ix->range_rows = rr;
  }
  ix->range_group = o.range_group > 0 ? o.range_group : 1;
  if (const char* ev = getenv("APSS_RANGE_GROUP")) {
    const int g = atoi(ev);
    if (g >= 1 && g <= kMaxRangeGroup) ix->range_group = g;
  }
  (void)hipGetDevice(&ix->device);
  if (o.screen_dims > 0 && !screen_variant_ok(ix->variant)) {
    set_error("tile variant %d is not available for the screened join", ix->variant);
    delete ix;
    return APSS_EINVAL;
  }
  int rc = build_impl(ix, row_ptr, col, val, on_device);
  if (!rc && o.screen_dims > 0) rc = build_screen(ix, (int32_t)std::min<int64_t>(o.screen_dims, m));
  // the join's lookup tables for the index's geometry and the call timers
  // exist from here on, so apss_join_device_noalloc needs no allocation
  if (!rc && o.screen_dims == 0 && n > 0) rc = prepare(ix, ix->ws.stream, ix->variant, ix->range_rows);
  for (int e = 0; !rc && e < 6; ++e)
    if (hipEventCreateWithFlags(&ix->ws.ev[e], hipEventDefault) != hipSuccess) {
      set_error("hipEventCreateWithFlags failed");
      rc = APSS_EDEVICE;
    }
  if (rc) {
    (void)hipStreamSynchronize(ix->ws.stream);
    apss_index_free(ix);
    return rc;
  }
  *out = ix;
  return APSS_OK;
}

void apss_index_free(apss_index* idx) {
  if (!idx) return;
  (void)hipStreamSynchronize(idx->ws.stream);
  apss_index_free(idx->screen);
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
  if (ix->opts.graph && !ix->screen && ix->parts == 1 && !ix->opts.remscore && ix->n > 0)
    return graph_join(ix, t, out_i, out_j, out_sim, capacity, count);
  int64_t cnt = 0;
  if ((rc = self_join(ix, t, &cnt))) return rc;
  return finish_device(ix->ws, cnt, ceil_log2((uint64_t)ix->n), out_i, out_j, out_sim, capacity, count);
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
  int64_t cnt = 0;
  if ((rc = self_join(ix, t, &cnt))) return rc;
  return finish_host(ix->ws, cnt, ceil_log2((uint64_t)ix->n), out);
}

int apss_query_device(apss_index* ix, int64_t nq, const int64_t* q_row_ptr, const int32_t* q_col, const float* q_val,
                      int on_device, const float* t_per_row, float t, uint32_t* out_i, uint32_t* out_j,
                      float* out_sim, int64_t capacity, int64_t* count) {
  if (!ix || !count || !q_row_ptr || nq < 0 || nq >= (1ll << 31) ||
      (capacity > 0 && (!out_i || !out_j || !out_sim))) {
    set_error("NULL or invalid argument");
    return APSS_EINVAL;
  }
  RankRows rows;
  int rc = stage_queries(ix, ix->ws, nq, q_row_ptr, q_col, q_val, on_device, t_per_row, t, rows);
  if (rc) return rc;
  int64_t cnt = 0;
  if ((rc = run_join(ix, ix->ws, staged_queries(rows), 0, t, t_per_row ? ix->ws.qt.p : nullptr, 16 * nq, &cnt)))
    return rc;
  return finish_device(ix->ws, cnt, ceil_log2((uint64_t)ix->n), out_i, out_j, out_sim, capacity, count);
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
  RankRows rows;
  int rc = stage_queries(ix, ix->ws, nq, q_row_ptr, q_col, q_val, on_device, t_per_row, t, rows);
  if (rc) return rc;
  int64_t cnt = 0;
  if ((rc = run_join(ix, ix->ws, staged_queries(rows), 0, t, t_per_row ? ix->ws.qt.p : nullptr, 16 * nq, &cnt)))
    return rc;
  return finish_host(ix->ws, cnt, ceil_log2((uint64_t)ix->n), out);
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
  *out = ix->ws.last;
  return APSS_OK;
}

int apss_index_export(const apss_index* ix, int32_t* rank, float* maxweight, int32_t* cut) {
  if (!ix) {
    set_error("NULL argument");
    return APSS_EINVAL;
  }
  hipStream_t s = ix->ws.stream;
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
