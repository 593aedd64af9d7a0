// Serving loop: continuous batching of query requests against a resident
// index (Find-Matches, Algorithm 2, for many queries at once).
//
// Requests are validated and copied at submit, then wait in one FIFO as
// chunks of consecutive rows (one chunk per request, or pieces of at most
// split_queries rows).  Each slot is a host thread with its own stream and
// workspace: whenever it is free it takes every waiting chunk that fits its
// batch (at most max_batch_queries queries, at least one chunk),
// concatenates them into one query set with per-row thresholds, runs the
// query kernels on its stream and splits the sorted pairs back per chunk; a
// request is complete when its last chunk is, and its pieces are joined in
// row order.  Slots run independently, so a batch formed from requests that
// arrived while another batch was on the GPU runs beside it, and the pieces
// of a large request run on several slots at once.
//
// Admission: each request reserves the device bytes its staging and pair
// buffers need (an estimate from its size, see request_bytes); submit
// refuses with APSS_EBUSY while the reservations of queued and running
// requests would exceed the budget, and the reservation returns when the
// request completes.
//
// The per-pair decision does not depend on which other queries share a
// batch: candidate scores are integer sums, and the final score of a pair
// is computed by one wavefront in a fixed order.  A request's result is
// therefore the same alone and in any mix.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "lib.h"

using namespace apss;

namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

// Device bytes one batch needs per query component, per query and per
// reserved output pair (staging copies, rank-space rows, sort scratch; raw
// pair keys and scores, their sort scratch and the unpacked output).
constexpr int64_t kBytesPerNnz = 40;
constexpr int64_t kBytesPerQuery = 32;
constexpr int64_t kBytesPerPair = 28;

struct Request {
  uint64_t id = 0;
  int64_t nq = 0, nnz = 0;
  std::vector<int64_t> rp;
  std::vector<int32_t> col;
  std::vector<float> val;
  std::vector<float> t;
  int64_t bytes = 0;  // reservation
  Clock::time_point t_submit, t_start, t_done;
  bool done = false;
  int status = APSS_OK;
  std::string error;
  apss_pairs pairs{0, nullptr, nullptr, nullptr};
  int64_t batch = -1;
  int32_t batch_requests = 0;
  int32_t slot = -1;
  // pieces of the request queued as separate chunks
  int chunks = 1, chunks_done = 0;
  bool started = false;
  std::vector<apss_pairs> parts;
};

// Rows [q0, q1) of a request, queued as one unit of batching.
struct Chunk {
  Request* r = nullptr;
  int64_t q0 = 0, q1 = 0;
  int idx = 0;
};

void free_pairs(apss_pairs& p) {
  free(p.i);
  free(p.j);
  free(p.sim);
  p = apss_pairs{0, nullptr, nullptr, nullptr};
}

}  // namespace

struct apss_server {
  apss_index* ix = nullptr;
  apss_server_opts o;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Chunk> queue;
  std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
  std::vector<std::thread> workers;
  bool stop = false;
  bool paused = false;
  uint64_t next_id = 1;
  int64_t next_batch = 0;
  int64_t reserved = 0;
  int running = 0;
  apss_server_counters st;
  int start_error = APSS_OK;
  std::string start_msg;
  int started = 0;
};

namespace {

int64_t request_bytes(const apss_server_opts& o, int64_t nq, int64_t nnz) {
  return kBytesPerNnz * nnz + kBytesPerQuery * nq + kBytesPerPair * o.pairs_per_query * nq;
}

// Host-side validation of a request (so that one bad request cannot fail a
// batch): the CSR conventions of the index, thresholds in [t_build, 1].
int validate_request(const apss_index* ix, int64_t nq, const int64_t* rp, const int32_t* col, const float* val,
                     const float* t_per_row, float t) {
  if (rp[0] != 0) {
    set_error("row_ptr must start at 0");
    return APSS_EINVAL;
  }
  std::vector<int32_t> dims;
  for (int64_t q = 0; q < nq; ++q) {
    const int64_t b = rp[q], e = rp[q + 1];
    if (e < b || e - b > (int64_t)ix->m) {
      set_error("row_ptr must be non-decreasing with rows of at most m entries (row %lld)", (long long)q);
      return APSS_EINVAL;
    }
    const float tq = t_per_row ? t_per_row[q] : t;
    const int rc = check_t(ix, tq);
    if (rc) return rc;
    double sq = 0.0;
    bool increasing = true;  // ids in increasing order have no repeats
    for (int64_t k = b; k < e; ++k) {
      if (k > b && col[k] <= col[k - 1]) increasing = false;
      if (col[k] < 0 || (int64_t)col[k] >= ix->m) {
        set_error("dimension id outside [0, m) (row %lld)", (long long)q);
        return APSS_EINVAL;
      }
      if (!(val[k] > 0.0f) || !isfinite(val[k])) {
        set_error("weights must be finite and > 0 (row %lld)", (long long)q);
        return APSS_EINVAL;
      }
      sq += (double)val[k] * (double)val[k];
    }
    if (e > b && fabs(sqrt(sq) - 1.0) > 1e-5) {
      set_error("non-empty rows must have unit L2 norm (|norm - 1| <= 1e-5) (row %lld)", (long long)q);
      return APSS_EINVAL;
    }
    if (!increasing) {
      dims.assign(col + b, col + e);
      std::sort(dims.begin(), dims.end());
      if (std::adjacent_find(dims.begin(), dims.end()) != dims.end()) {
        set_error("repeated dimension id inside a row (row %lld)", (long long)q);
        return APSS_EINVAL;
      }
    }
  }
  return APSS_OK;
}

// Run one batch on a slot's workspace; fills every request's result.
struct Staging {
  PinnedBuf<int64_t> rp;
  PinnedBuf<int32_t> col;
  PinnedBuf<float> val, tq;
};

// A chunk's status and pairs (rows numbered within its request).
void fail_chunk(const Chunk& c, int rc, const std::string& msg) {
  if (!c.r->status) {
    c.r->status = rc;
    c.r->error = msg;
  }
}

void run_batch(apss_server* S, Workspace& ws, RankRows& rows, Staging& hs, std::vector<Chunk>& batch) {
  apss_index* ix = S->ix;
  int64_t nq = 0, nnz = 0, cap = 0;
  for (const Chunk& c : batch) {
    nq += c.q1 - c.q0;
    nnz += c.r->rp[(size_t)c.q1] - c.r->rp[(size_t)c.q0];
    cap += S->o.pairs_per_query * (c.q1 - c.q0);
  }
  std::vector<int64_t> row0(batch.size() + 1);
  if (!hs.rp.reserve((size_t)nq + 1) || !hs.col.reserve((size_t)nnz) || !hs.val.reserve((size_t)nnz) ||
      !hs.tq.reserve((size_t)nq)) {
    for (const Chunk& c : batch) fail_chunk(c, APSS_ENOMEM, "pinned host allocation failed");
    return;
  }
  int64_t* const rp = hs.rp.p;
  int32_t* const col = hs.col.p;
  float* const val = hs.val.p;
  float* const tq = hs.tq.p;
  int64_t q0 = 0, k0 = 0;
  for (size_t b = 0; b < batch.size(); ++b) {
    const Chunk& c = batch[b];
    const Request* r = c.r;
    const int64_t kb = r->rp[(size_t)c.q0], ke = r->rp[(size_t)c.q1];
    row0[b] = q0;
    for (int64_t q = c.q0; q < c.q1; ++q) rp[(size_t)(q0 + q - c.q0)] = k0 + r->rp[(size_t)q] - kb;
    std::copy(r->col.begin() + kb, r->col.begin() + ke, col + k0);
    std::copy(r->val.begin() + kb, r->val.begin() + ke, val + k0);
    std::copy(r->t.begin() + c.q0, r->t.begin() + c.q1, tq + q0);
    q0 += c.q1 - c.q0;
    k0 += ke - kb;
  }
  row0[batch.size()] = q0;
  rp[(size_t)nq] = nnz;

  apss_pairs all{0, nullptr, nullptr, nullptr};
  int rc = APSS_OK;
  if (nq > 0) {
    rc = stage_queries(ix, ws, nq, rp, col, val, 0, tq, 1.0f, rows);
    int64_t cnt = 0;
    if (!rc) {
      const QuerySet Q{rows.rp.p, rows.rc.p, rows.mw.p, rows.n, rows.nnz, rows.rp_host.data()};
      rc = run_join(ix, ws, Q, 0, 1.0f, ws.qt.p, cap, &cnt);
    }
    if (!rc) rc = finish_host(ws, cnt, ceil_log2((uint64_t)ix->n), &all);
  }
  const std::string msg = rc ? last_error() : std::string();
  // split the (query row, corpus row)-sorted pairs by chunk
  int64_t k = 0;
  for (size_t b = 0; b < batch.size(); ++b) {
    const Chunk& ch = batch[b];
    if (rc) {
      fail_chunk(ch, rc, msg);
      continue;
    }
    const int64_t lo = k;
    while (k < all.count && (int64_t)all.i[k] < row0[b + 1]) ++k;
    const int64_t c = k - lo;
    const size_t nbytes = (size_t)(c > 0 ? c : 1);
    apss_pairs p{c, (uint32_t*)malloc(nbytes * 4), (uint32_t*)malloc(nbytes * 4), (float*)malloc(nbytes * 4)};
    if (!p.i || !p.j || !p.sim) {
      free_pairs(p);
      fail_chunk(ch, APSS_ENOMEM, "host allocation failed");
      continue;
    }
    for (int64_t x = 0; x < c; ++x) {
      p.i[x] = (uint32_t)((int64_t)all.i[lo + x] - row0[b] + ch.q0);
      p.j[x] = all.j[lo + x];
      p.sim[x] = all.sim[lo + x];
    }
    ch.r->parts[(size_t)ch.idx] = p;
  }
  free_pairs(all);
}

// The pieces of a request joined in row order into its result.
void assemble(Request* r) {
  if (r->status) {
    for (apss_pairs& p : r->parts) free_pairs(p);
    return;
  }
  if (r->parts.size() == 1) {
    r->pairs = r->parts[0];
    r->parts[0] = apss_pairs{0, nullptr, nullptr, nullptr};
    return;
  }
  int64_t total = 0;
  for (const apss_pairs& p : r->parts) total += p.count;
  const size_t nbytes = (size_t)(total > 0 ? total : 1);
  apss_pairs out{total, (uint32_t*)malloc(nbytes * 4), (uint32_t*)malloc(nbytes * 4), (float*)malloc(nbytes * 4)};
  if (!out.i || !out.j || !out.sim) {
    free_pairs(out);
    r->status = APSS_ENOMEM;
    r->error = "host allocation failed";
  } else {
    int64_t o = 0;
    for (const apss_pairs& p : r->parts) {
      if (p.count) {
        memcpy(out.i + o, p.i, sizeof(uint32_t) * (size_t)p.count);
        memcpy(out.j + o, p.j, sizeof(uint32_t) * (size_t)p.count);
        memcpy(out.sim + o, p.sim, sizeof(float) * (size_t)p.count);
      }
      o += p.count;
    }
    r->pairs = out;
  }
  for (apss_pairs& p : r->parts) free_pairs(p);
}

void worker(apss_server* S, int slot) {
  Staging hs;  // destroyed last, after the slot's stream has drained
  Workspace ws;
  RankRows rows;
  int rc = APSS_OK;
  std::string msg;
  hipError_t e = hipSetDevice(S->ix->device);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&ws.stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    rc = dev_err(e, "server slot stream");
    msg = last_error();
  }
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (rc && !S->start_error) {
      S->start_error = rc;
      S->start_msg = msg;
    }
    ++S->started;
  }
  S->cv_done.notify_all();
  if (rc) return;
  for (;;) {
    std::vector<Chunk> batch;
    int64_t bid = 0;
    bool more = false;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_work.wait(lk, [&] { return S->stop || (!S->paused && !S->queue.empty()); });
      if (S->stop) break;
      int64_t q = 0;
      while (!S->queue.empty()) {
        const Chunk& c = S->queue.front();
        if (!batch.empty() && q + (c.q1 - c.q0) > S->o.max_batch_queries) break;
        batch.push_back(c);
        q += c.q1 - c.q0;
        S->queue.pop_front();
      }
      bid = S->next_batch++;
      if (S->running > 0) ++S->st.overlapped_batches;
      ++S->running;
      S->st.peak_running = std::max<int64_t>(S->st.peak_running, S->running);
      ++S->st.batches;
      S->st.queries += q;
      const Clock::time_point now = Clock::now();
      for (const Chunk& c : batch) {
        Request* r = c.r;
        if (r->started) continue;
        r->started = true;
        r->t_start = now;
        r->batch = bid;
        r->batch_requests = (int32_t)batch.size();
        r->slot = slot;
      }
      more = !S->queue.empty();
    }
    if (more) S->cv_work.notify_one();
    const int64_t regrows0 = ws.regrows;
    run_batch(S, ws, rows, hs, batch);
    if (ws.regrows != regrows0) {
      // the batch's pairs outgrew its reservation and its buffers grew
      // beyond what the budget charged for: release them (after the slot's
      // stream has drained), so the slot holds no more than later batches
      // reserve; the next batch allocates its own size again
      (void)hipStreamSynchronize(ws.stream);
      ws.raw_key.release();
      ws.raw_sim.release();
      ws.ss.k2.release();
      ws.ss.v32b.release();
      ws.ss.hist.release();
      ws.ss.scan.release();
      ws.ss.v64a.release();
      ws.ss.v64b.release();
    }
    // requests whose last chunk this batch held are joined and handed over
    std::vector<Request*> finished;
    {
      std::lock_guard<std::mutex> lk(S->mu);
      for (const Chunk& c : batch)
        if (++c.r->chunks_done == c.r->chunks) finished.push_back(c.r);
      S->st.regrows += ws.regrows - regrows0;
      S->st.device_bytes[slot] = ws.bytes() + rows.rp.bytes() + rows.rc.bytes() + rows.mw.bytes();
      --S->running;
    }
    for (Request* r : finished) assemble(r);
    {
      std::lock_guard<std::mutex> lk(S->mu);
      const Clock::time_point now = Clock::now();
      for (Request* r : finished) {
        r->t_done = now;
        r->done = true;
        S->reserved -= r->bytes;
        ++S->st.completed;
        if (r->status) ++S->st.failed;
      }
    }
    S->cv_done.notify_all();
  }
  if (ws.stream) {
    (void)hipStreamSynchronize(ws.stream);
    (void)hipStreamDestroy(ws.stream);
  }
}

}  // namespace

extern "C" {

void apss_server_default_opts(apss_server_opts* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->struct_size = (int32_t)sizeof(apss_server_opts);
  o->slots = 2;
  o->max_batch_queries = 4096;
  o->memory_budget = 4ll << 30;
  o->pairs_per_query = 256;
  o->max_pending = 4096;
  o->split_queries = 0;
}

int apss_server_create(apss_index* ix, const apss_server_opts* opts, apss_server** out) {
  if (!ix || !out) {
    set_error("NULL argument");
    return APSS_EINVAL;
  }
  *out = nullptr;
  apss_server_opts o;
  apss_server_default_opts(&o);
  if (opts) {
    if (opts->struct_size != (int32_t)sizeof(apss_server_opts)) {
      set_error("apss_server_opts.struct_size mismatch (use apss_server_default_opts)");
      return APSS_EINVAL;
    }
    o = *opts;
  }
  if (o.slots < 1 || o.slots > APSS_SERVER_MAX_SLOTS || o.max_batch_queries < 1 ||
      o.max_batch_queries >= (1ll << 31) || o.memory_budget < 1 || o.pairs_per_query < 0 || o.max_pending < 1 ||
      o.split_queries < 0 || o.split_queries > o.max_batch_queries) {
    set_error("server options out of range");
    return APSS_EINVAL;
  }
  if (!ix->opts.query_safe) {
    set_error("index was built with query_safe = 0; serving needs the L2 cutoff clause");
    return APSS_EINVAL;
  }
  // build the lookup tables once, before several streams read them
  int rc = prepare(ix, ix->ws.stream, ix->variant, ix->range_rows);
  if (rc) return rc;
  apss_server* S = new (std::nothrow) apss_server();
  if (!S) {
    set_error("host allocation failed");
    return APSS_ENOMEM;
  }
  S->ix = ix;
  S->o = o;
  memset(&S->st, 0, sizeof(S->st));
  S->st.slots = o.slots;
  try {
    for (int k = 0; k < o.slots; ++k) S->workers.emplace_back(worker, S, k);
  } catch (...) {
    {
      std::lock_guard<std::mutex> lk(S->mu);
      S->stop = true;
    }
    S->cv_work.notify_all();
    for (auto& w : S->workers) w.join();
    delete S;
    set_error("could not start the server threads");
    return APSS_ENOMEM;
  }
  {
    std::unique_lock<std::mutex> lk(S->mu);
    S->cv_done.wait(lk, [&] { return S->started == o.slots; });
    rc = S->start_error;
  }
  if (rc) {
    const std::string msg = S->start_msg;
    apss_server_destroy(S);
    set_error("%s", msg.c_str());
    return rc;
  }
  *out = S;
  return APSS_OK;
}

int apss_submit(apss_server* S, int64_t nq, const int64_t* q_row_ptr, const int32_t* q_col, const float* q_val,
                const float* t_per_row, float t, uint64_t* req_id) {
  if (!S || !req_id || !q_row_ptr || nq < 0 || nq >= (1ll << 31)) {
    set_error("NULL or invalid argument");
    return APSS_EINVAL;
  }
  *req_id = 0;
  const int64_t nnz = q_row_ptr[nq];
  if (nnz < 0 || nnz >= (1ll << 32) || (nnz > 0 && (!q_col || !q_val))) {
    set_error("row_ptr[nq] must be in [0, 2^32), with col and val given");
    return APSS_EINVAL;
  }
  // a request is batched whole unless it is split into pieces, which then fit a batch
  if (S->o.split_queries == 0 && nq > S->o.max_batch_queries) {
    set_error("request of %lld queries exceeds max_batch_queries %lld", (long long)nq,
              (long long)S->o.max_batch_queries);
    return APSS_EINVAL;
  }
  int rc = validate_request(S->ix, nq, q_row_ptr, q_col, q_val, t_per_row, t);
  if (rc) return rc;
  const int64_t bytes = request_bytes(S->o, nq, nnz);
  if (bytes > S->o.memory_budget) {
    set_error("request needs %lld device bytes, more than the server budget %lld", (long long)bytes,
              (long long)S->o.memory_budget);
    return APSS_ENOMEM;
  }
  std::unique_ptr<Request> r(new (std::nothrow) Request());
  if (!r) {
    set_error("host allocation failed");
    return APSS_ENOMEM;
  }
  r->nq = nq;
  r->nnz = nnz;
  r->rp.assign(q_row_ptr, q_row_ptr + nq + 1);
  r->col.assign(q_col, q_col + nnz);
  r->val.assign(q_val, q_val + nnz);
  if (t_per_row) r->t.assign(t_per_row, t_per_row + nq);
  else r->t.assign((size_t)nq, t);
  r->bytes = bytes;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    const int64_t pending = (int64_t)S->reqs.size();
    if (S->reserved + bytes > S->o.memory_budget || pending >= S->o.max_pending) {
      ++S->st.rejected_busy;
      set_error("server busy: %lld of %lld budget bytes reserved, %lld requests held", (long long)S->reserved,
                (long long)S->o.memory_budget, (long long)pending);
      return APSS_EBUSY;
    }
    r->id = S->next_id++;
    r->t_submit = Clock::now();
    S->reserved += bytes;
    S->st.peak_reserved_bytes = std::max(S->st.peak_reserved_bytes, S->reserved);
    ++S->st.submitted;
    *req_id = r->id;
    // pieces of at most split_queries rows (one piece when 0 or larger)
    const int64_t piece = (S->o.split_queries > 0 && nq > S->o.split_queries) ? S->o.split_queries : std::max<int64_t>(nq, 1);
    r->chunks = (int)((std::max<int64_t>(nq, 1) + piece - 1) / piece);
    r->parts.assign((size_t)r->chunks, apss_pairs{0, nullptr, nullptr, nullptr});
    for (int c = 0; c < r->chunks; ++c) {
      Chunk ch;
      ch.r = r.get();
      ch.q0 = std::min<int64_t>(nq, (int64_t)c * piece);
      ch.q1 = std::min<int64_t>(nq, (int64_t)(c + 1) * piece);
      ch.idx = c;
      S->queue.push_back(ch);
    }
    S->reqs.emplace(r->id, std::move(r));
  }
  S->cv_work.notify_all();
  return APSS_OK;
}

int apss_poll(apss_server* S, uint64_t req_id, int timeout_ms, apss_pairs* out, apss_request_info* info) {
  if (!S || !out) {
    set_error("NULL argument");
    return APSS_EINVAL;
  }
  out->count = 0;
  out->i = out->j = nullptr;
  out->sim = nullptr;
  std::unique_ptr<Request> r;
  {
    std::unique_lock<std::mutex> lk(S->mu);
    // look the request up again after every wake-up: another thread may have collected it
    auto ready = [&] {
      auto it = S->reqs.find(req_id);
      return it == S->reqs.end() || it->second->done;
    };
    if (timeout_ms < 0) S->cv_done.wait(lk, ready);
    else if (!S->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready)) return APSS_PENDING;
    auto it = S->reqs.find(req_id);
    if (it == S->reqs.end()) {
      set_error("unknown or already collected request id %llu", (unsigned long long)req_id);
      return APSS_EINVAL;
    }
    r = std::move(it->second);
    S->reqs.erase(it);
  }
  if (info) {
    info->queue_ms = ms_between(r->t_submit, r->t_start);
    info->service_ms = ms_between(r->t_start, r->t_done);
    info->latency_ms = ms_between(r->t_submit, r->t_done);
    info->batch = r->batch;
    info->batch_requests = r->batch_requests;
    info->slot = r->slot;
  }
  if (r->status) {
    set_error("%s", r->error.c_str());
    return r->status;
  }
  *out = r->pairs;
  r->pairs = apss_pairs{0, nullptr, nullptr, nullptr};
  return APSS_OK;
}

int apss_server_pause(apss_server* S, int paused) {
  if (!S) {
    set_error("NULL argument");
    return APSS_EINVAL;
  }
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->paused = paused != 0;
  }
  S->cv_work.notify_all();
  return APSS_OK;
}

int apss_server_stats(apss_server* S, apss_server_counters* out) {
  if (!S || !out) {
    set_error("NULL argument");
    return APSS_EINVAL;
  }
  std::lock_guard<std::mutex> lk(S->mu);
  *out = S->st;
  out->reserved_bytes = S->reserved;
  out->queued = (int64_t)S->queue.size();
  out->running = S->running;
  return APSS_OK;
}

void apss_server_destroy(apss_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  for (auto& w : S->workers) w.join();
  for (auto& kv : S->reqs) {
    free_pairs(kv.second->pairs);
    for (apss_pairs& p : kv.second->parts) free_pairs(p);
  }
  delete S;
}

}  // extern "C"
