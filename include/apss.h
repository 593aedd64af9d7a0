/* apss -- exact all-pairs similarity join of sparse unit vectors on one
 * AMD Instinct MI355X (gfx950).
 *
 * Problem (Section 2.1 of Ozkural & Aykanat, "1-D and 2-D Parallel
 * Algorithms for All-Pairs Similarity Problem"): V = {v_0..v_{n-1}} sparse
 * vectors in R^m with positive weights and unit L2 norm; sim(x, y) is the
 * dot product; the join returns every unordered pair with sim >= t, with
 * its similarity (the match matrix M' of Section 2.1).
 *
 * Method: partial indexing (all-pairs-1, Section 3.2.2) with the size and
 * max-weight bounds of all-pairs-2, an exact completion of each surviving
 * candidate's score, and a final rescore.  The threshold is the float value
 * passed in; a pair belongs to the result iff its double-precision dot
 * product of the float weights is >= that value.  Pairs whose float rescore
 * lies within 1e-5 of t are decided by a double-precision rescore on the GPU.
 * Every reported sim is within 1e-5 of the double-precision value.
 *
 * Conventions for every entry point:
 *  - CSR input: row_ptr[n+1] (int64, row_ptr[0] = 0, non-decreasing),
 *    col[nnz] (int32 dimension ids in [0, m), unique within a row, any
 *    order), val[nnz] (float, finite, > 0).  A non-empty row must have
 *    |L2 norm - 1| <= 1e-5 (checked in double).  Empty rows are allowed and
 *    never match.  on_device = 1 means the three pointers are device
 *    pointers of the current HIP device, 0 means host memory.
 *  - Inputs are borrowed for the duration of the call only.
 *  - All work is issued on the stream given in apss_opts (NULL = the
 *    default stream); calls return after that work has finished.
 *  - An apss_index is not thread-safe: one call at a time per index.  While
 *    a server (below) is attached to it, use the index only through that
 *    server; the index must outlive the server.
 *  - Return value: APSS_OK or an error code below; apss_last_error() then
 *    holds a message for the calling thread.
 */
#ifndef APSS_H
#define APSS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  APSS_OK = 0,
  APSS_EINVAL = 1,   /* malformed input (CSR, weights, norms, sizes, NULL) */
  APSS_ETHRESH = 2,  /* t outside (0, 1], or below the index's build threshold */
  APSS_ENOMEM = 3,   /* device or host allocation failed */
  APSS_EDEVICE = 4,  /* HIP runtime error */
  APSS_ERANGE = 5,   /* caller's output buffer too small; *count holds the size needed */
  APSS_EBUSY = 6,    /* server admission refused: budget or queue full, retry later */
  APSS_PENDING = 100 /* apss_poll: request not finished yet (not an error) */
};

typedef struct apss_index apss_index;

/* Tuning and placement.  Fill with apss_default_opts, then override. */
typedef struct {
  int32_t struct_size;   /* sizeof(apss_opts) */
  void* stream;          /* hipStream_t for all work; NULL = default stream */
  int32_t query_safe;    /* 1 (default): the unindexed part of every vector also stops once its
                            own L2 norm reaches t, so dot(q, x') < t for any unit query q and the
                            index answers apss_query; 0: the paper's cutoff only (join only) */
  int32_t variant;       /* compiled tile variant of the join kernel (queries per tile x corpus
                            rows per block): 0, 1 or 2 (3 is withdrawn: APSS_EINVAL); -1 = the
                            library's default.  The environment variable APSS_VARIANT overrides it. */
  int32_t head_dims;     /* densest dimensions that get per-block list offsets (0 = default) */
  int32_t range_rows;    /* corpus rows per work item of the join (rounded down to a multiple of the
                            variant's block rows; 0 = default 16384).  The environment variable
                            APSS_RANGE_ROWS overrides it. */
  int32_t screen_dims;   /* > 0 (at most 8192): apss_join / apss_join_device use the screened join
                            with this many densest dimensions as the dense head (bf16 MFMA screen
                            plus a sparse pass over the rest); 0 (default): plain join only */
  int32_t graph;         /* 1: apss_join_device (plain join) captures its launch sequence in a HIP
                            graph and replays it on later calls with the same t and output
                            buffers (one launch, one synchronisation per call); the graph's
                            stats report its whole device time as ms_candidates.  0: default */
  int32_t index_all;     /* 1: index every component of every vector (no unindexed part): the
                            all-pairs-0-array algorithm of Section 4 (Algorithms 1 and 2 with a
                            dense score array per corpus block), the ablation of partial
                            indexing; not with screen_dims.  0 (default): partial indexing */
  int32_t local_parts;   /* p in {2, 4, 8}: local pruning (Section 5.1.3, Eq. 1 and Lemma 1).  The
                            indexed dimensions are split into p rank ranges of about equal
                            postings (the densest lists apart from the rest); every work item
                            scores one range, keeps a candidate only if its local score reaches
                            the local threshold t/p (with the unindexed part's bound shared
                            evenly), and the survivors are decided on their exact full score;
                            a pair kept by several ranges is reported once.  Not with
                            screen_dims.  0 or 1 (default): off */
  int32_t remscore;      /* 1: the remscore rule of all-pairs-2 (Section 3.2.2): components of a
                            query processed rarest first stop admitting new candidates once the
                            remaining bound sum q[d] * maxweight_d(V) of the components not yet
                            processed, the current one included, is below t; a candidate all of
                            whose indexed overlap lies in components past that point is dropped
                            before the bounds.  0 (default): off */
  int32_t range_group;   /* corpus ranges per work item of the join (1 to 64): an item stages its
                            query tile once and visits that many consecutive ranges in turn;
                            0 = 1.  The environment variable APSS_RANGE_GROUP overrides it. */
  int32_t reserved[4];
} apss_opts;

void apss_default_opts(apss_opts* opts);

/* Build the partial index of V for thresholds >= t_build (Section 3.2.2):
 * dimensions ordered by decreasing non-zero count (ties: smaller id first),
 * maxweight_d(V) per dimension, each vector split into its unindexed
 * leading part x' (densest dimensions first, while the running bound
 * sum x[d] * maxweight_d(V) stays below t_build) and its indexed rest, and
 * inverted lists of the indexed parts ordered by vector id.
 * The index owns device memory until apss_index_free.
 * Errors: APSS_EINVAL (bad CSR, n < 0, m <= 0, nnz >= 2^32, n >= 2^31),
 * APSS_ETHRESH (t_build outside (0, 1]), APSS_ENOMEM, APSS_EDEVICE. */
int apss_build_index(int64_t n, int64_t m, const int64_t* row_ptr, const int32_t* col, const float* val,
                     int on_device, float t_build, const apss_opts* opts, apss_index** out);

void apss_index_free(apss_index* idx);

/* Self-join (Algorithm 1 driving Find-Matches, Algorithm 2, with partial
 * indexing): every pair i < j with sim(v_i, v_j) >= t, written to caller
 * device buffers out_i[k], out_j[k] (uint32 row ids), out_sim[k] (float),
 * k < *count, sorted by (i, j).  capacity is the length of each buffer.
 * If more pairs exist than capacity, returns APSS_ERANGE with *count set to
 * the number needed and the buffers' contents undefined.
 * Errors: APSS_ETHRESH (t not in [t_build, 1]), APSS_EINVAL (NULL), APSS_ENOMEM, APSS_EDEVICE. */
int apss_join_device(apss_index* idx, float t, uint32_t* out_i, uint32_t* out_j, float* out_sim,
                     int64_t capacity, int64_t* count);

/* Allocation-free self-join, for callers that cannot allocate device
 * memory during the call: code under HIP stream capture, tight serving
 * loops, harnesses that forbid allocation.  Same contract and result as
 * apss_join_device on an index built without screen_dims, on the index's
 * stream and device (current at the call).  Every scratch buffer of the call
 * (work queues and counters, per-workgroup list cursors, raw pairs, sort
 * scratch) is placed in one fixed device array of
 * APSS_NOALLOC_SCRATCH_BYTES bytes, which the library holds on each device it
 * runs on until the process ends; the index's join tables are made by
 * apss_build_index (and remade by apss_autotune), so the call allocates
 * nothing.  All calls on one device share that device's array: calls that
 * overlap on one device (from several threads, streams or indexes) race and
 * must not be made.
 * Errors: as apss_join_device; APSS_EINVAL also for a screened index, a call
 * on another device than the index's, or an index whose tables are not
 * ready; APSS_ENOMEM when the join needs more scratch than the array holds
 * (its work queues, or more pairs than fit beside them -- then *count is the
 * number of pairs; apss_join_device has no such limit). */
#define APSS_NOALLOC_SCRATCH_BYTES (128ll << 20)
int apss_join_device_noalloc(apss_index* idx, float t, uint32_t* out_i, uint32_t* out_j, float* out_sim,
                             int64_t capacity, int64_t* count);

/* Pairs in library-owned host memory; free with apss_pairs_free. */
typedef struct {
  int64_t count;
  uint32_t* i;
  uint32_t* j;
  float* sim;
} apss_pairs;

/* apss_join_device with the result copied to host memory (sizes itself). */
int apss_join(apss_index* idx, float t, apss_pairs* out);

/* External queries (Find-Matches, Algorithm 2, against the resident index):
 * every (query row q, corpus row y) with sim(q, y) >= t_q, where t_q =
 * t_per_row[q] if t_per_row (host array of nq floats) is given, else t.
 * Query rows follow the CSR conventions above with dimension ids in
 * [0, m).  Output: out->i = query row, out->j = corpus row, sorted.
 * Requires an index built with query_safe = 1 and every t_q in
 * [t_build, 1] (else APSS_ETHRESH). */
int apss_query(apss_index* idx, int64_t nq, const int64_t* q_row_ptr, const int32_t* q_col, const float* q_val,
               int on_device, const float* t_per_row, float t, apss_pairs* out);

/* Device-output variant of apss_query; same contract as apss_join_device. */
int apss_query_device(apss_index* idx, int64_t nq, const int64_t* q_row_ptr, const int32_t* q_col,
                      const float* q_val, int on_device, const float* t_per_row, float t, uint32_t* out_i,
                      uint32_t* out_j, float* out_sim, int64_t capacity, int64_t* count);

void apss_pairs_free(apss_pairs* p);

/* Counters and device times of the last join or query on this index. */
typedef struct {
  int64_t posting_visits;   /* inverted-list entries streamed into accumulators */
  int64_t candidates;       /* distinct (x, y) pairs with an accumulated indexed score */
  int64_t bound_survivors;  /* candidates passing the size, max-weight and L2 bounds */
  int64_t verified;         /* survivors whose completed score A + dot(x, y') reached t - slack */
  int64_t band;             /* pairs rescored in double (float rescore within 1e-5 of t) */
  int64_t matches;          /* pairs returned */
  double ms_candidates;     /* device time of the candidate/filter/verify kernel */
  double ms_total;          /* device time of the whole call (kernels + sort) */
  /* screened join only (zero otherwise) */
  int64_t screen_rows;        /* rows whose head norm reaches t */
  int64_t screen_tiles;       /* 128 x 128 row-tile pairs of the head screen whose norm bound reaches t
                                 (2 * 128 * 128 * ld flops of useful work each) */
  int64_t screen_candidates;  /* pairs passing the screen's widened threshold */
  int64_t screen_ld;          /* head dimensions padded to the screen's K step */
  double ms_screen;           /* device time of the screen's MFMA kernel */
} apss_stats;

int apss_last_stats(const apss_index* idx, apss_stats* out);

/* Copies of the index ingredients to host arrays (any may be NULL):
 * rank[m] (position of each dimension in the density order), maxweight[m]
 * (by dimension id), cut[n] (length of each vector's unindexed part). */
int apss_index_export(const apss_index* idx, int32_t* rank, float* maxweight, int32_t* cut);

/* Sizes of the index: n, m, nnz, number of postings. Any pointer may be NULL. */
int apss_index_sizes(const apss_index* idx, int64_t* n, int64_t* m, int64_t* nnz, int64_t* postings);

const char* apss_strerror(int code);
const char* apss_last_error(void);

/* ---- Autotuning of the self-join ----
 * Times the join kernel at threshold t on this index under every compiled
 * tile variant (queries per tile x corpus rows per LDS accumulator block)
 * and several corpus-range widths of the persistent kernel's work items,
 * then, for the fastest of those, several numbers of ranges per work item,
 * and keeps the fastest for later joins on the index (for an index built
 * with screen_dims > 0: the sparse pass of the screened join).  budget_ms > 0
 * stops trying further configurations once that much host time has passed
 * (the current configuration is always timed first).  With cache_path, the
 * choice is first looked up in that JSON file under a key made of the device
 * architecture, the join kind and the workload class (n, m and nnz per row to
 * the nearest power of two, t to two decimals), and stored there after
 * tuning.  The index must not be in use by another call or a server. */
typedef struct {
  int32_t variant;             /* chosen tile variant */
  int32_t range_rows;          /* chosen corpus rows per work-item range */
  double ms;                   /* its join kernel time (from the cache if from_cache) */
  int32_t from_cache;          /* 1: taken from the cache file without timing */
  int32_t tried;               /* configurations timed */
  int32_t cache_write_failed;  /* 1: the cache file could not be written */
  int32_t range_group;         /* chosen ranges per work item */
  int32_t reserved[2];
} apss_tune_result;

int apss_autotune(apss_index* idx, float t, double budget_ms, const char* cache_path, apss_tune_result* out);

/* ---- Serving: continuous batching of query requests on a resident index ----
 *
 * A server answers external queries (apss_query semantics, Algorithm 2
 * against the resident index) for requests that arrive at any time from any
 * thread.  Each slot is a host thread with its own HIP stream and scratch;
 * a free slot takes every queued request that fits one batch (FIFO, at most
 * max_batch_queries queries), runs them as one query set with per-row
 * thresholds and hands each request its own part of the result.  Batches of
 * different slots run on the device at the same time.  A request's result
 * does not depend on what it was batched with.
 *
 * Admission: a request reserves
 *   40 * nnz + 32 * nq + 28 * pairs_per_query * nq
 * bytes of the device memory budget (query staging, sort scratch and its
 * candidate/pair buffers) from submit until it completes; submit returns
 * APSS_EBUSY instead of queueing while the reservations would exceed
 * memory_budget or max_pending requests are held.  A batch whose pairs
 * outgrow their reservation still completes (its buffers grow; counted in
 * apss_server_stats.regrows), and its slot releases the grown buffers when
 * it ends, so that between such batches the slots hold what the
 * reservations cover; apss_server_stats.device_bytes reports what each slot
 * holds.
 *
 * All server entry points are thread-safe, except apss_server_destroy, which
 * must not overlap any other call on the same server. */
typedef struct apss_server apss_server;

#define APSS_SERVER_MAX_SLOTS 8

typedef struct {
  int32_t struct_size;        /* sizeof(apss_server_opts) */
  int32_t slots;              /* batches in flight at once, 1..APSS_SERVER_MAX_SLOTS (default 2) */
  int64_t max_batch_queries;  /* queries merged into one batch, and the largest request unless requests
                                 are split (default 4096) */
  int64_t memory_budget;      /* device bytes that admitted requests may reserve (default 4 GiB) */
  int64_t pairs_per_query;    /* output pairs reserved per query (default 256) */
  int64_t max_pending;        /* requests held (queued, running or not yet polled) at most (default 4096) */
  int64_t split_queries;      /* > 0: a request of more rows is queued as pieces of at most this many rows,
                                 which free slots take (and run side by side) like separate requests; the
                                 request completes with its last piece, its result joined in row order;
                                 at most max_batch_queries.  0 (default): every request is one piece */
  int32_t reserved[6];
} apss_server_opts;

void apss_server_default_opts(apss_server_opts* opts);

/* Start a server on idx (built with query_safe = 1).  The server borrows
 * idx.  Errors: APSS_EINVAL (options, query_safe = 0), APSS_ENOMEM, APSS_EDEVICE. */
int apss_server_create(apss_index* idx, const apss_server_opts* opts, apss_server** out);

/* Queue a request of nq query rows (host CSR, copied before return; the
 * CSR conventions above) with thresholds t_per_row[q] (host, may be NULL:
 * t for every row).  *req_id identifies it for apss_poll.  nq = 0 is a
 * request with an empty result.
 * Errors: APSS_EINVAL (bad CSR, nq > max_batch_queries without split_queries), APSS_ETHRESH (a
 * threshold outside [t_build, 1]), APSS_EBUSY (not admitted now: retry),
 * APSS_ENOMEM (the request alone needs more than memory_budget). */
int apss_submit(apss_server* srv, int64_t nq, const int64_t* q_row_ptr, const int32_t* q_col, const float* q_val,
                const float* t_per_row, float t, uint64_t* req_id);

/* Timing of one completed request (host clock, milliseconds). */
typedef struct {
  double queue_ms;         /* submit -> its batch started */
  double service_ms;       /* batch start -> result ready */
  double latency_ms;       /* submit -> result ready */
  int64_t batch;           /* sequence number of its batch */
  int32_t batch_requests;  /* requests in that batch */
  int32_t slot;            /* slot that ran it */
} apss_request_info;

/* Wait up to timeout_ms (0: do not wait, < 0: no limit) for request req_id.
 * Returns APSS_PENDING if it has not finished; otherwise the request's own
 * status, with its pairs in *out on APSS_OK (out->i = row within the
 * request, out->j = corpus row, sorted; free with apss_pairs_free), and
 * forgets the request.  info (may be NULL) receives its timing once done.
 * Errors: APSS_EINVAL (unknown or already collected id), or the error that
 * ended its batch (APSS_ENOMEM, APSS_EDEVICE). */
int apss_poll(apss_server* srv, uint64_t req_id, int timeout_ms, apss_pairs* out, apss_request_info* info);

/* paused = 1: slots start no new batch (running batches finish; submit
 * still admits and queues); paused = 0: resume.  For draining a server. */
int apss_server_pause(apss_server* srv, int paused);

typedef struct {
  int32_t slots;
  int32_t running;              /* batches on the device now */
  int64_t submitted;            /* requests admitted */
  int64_t rejected_busy;        /* submits refused with APSS_EBUSY */
  int64_t completed;            /* requests finished (including failed) */
  int64_t failed;               /* requests finished with an error */
  int64_t queued;               /* request pieces waiting for a slot now */
  int64_t batches;              /* batches started */
  int64_t queries;              /* query rows in started batches */
  int64_t overlapped_batches;   /* batches started while another batch was running */
  int64_t peak_running;         /* most batches running at once */
  int64_t regrows;              /* batches rerun because their pairs outgrew the reservation */
  int64_t reserved_bytes;       /* budget reserved now */
  int64_t peak_reserved_bytes;  /* most budget reserved at once */
  int64_t device_bytes[APSS_SERVER_MAX_SLOTS]; /* scratch each slot holds on the device */
} apss_server_counters;

int apss_server_stats(apss_server* srv, apss_server_counters* out);

/* Stop the slots after their running batches; queued requests are dropped.
 * Frees results not yet collected. */
void apss_server_destroy(apss_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* APSS_H */
