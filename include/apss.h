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
 *  - An apss_index is not thread-safe: one call at a time per index.
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
  APSS_EBUSY = 6,    /* reserved for admission control */
  APSS_PENDING = 100 /* reserved: work not finished yet (not an error) */
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
                            rows per block); -1 = the library's default.  The environment
                            variable APSS_VARIANT overrides it. */
  int32_t head_dims;     /* densest dimensions that get per-block list offsets (0 = default) */
  int32_t reserved[8];
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

#ifdef __cplusplus
}
#endif

#endif /* APSS_H */
