/* CPU oracle for the all-pairs similarity join -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, double-precision implementations written from the paper
 * (Ozkural & Aykanat, "1-D and 2-D Parallel Algorithms for All-Pairs
 * Similarity Problem").  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code
 * with the GPU library.
 *
 * Problem (Section 2.1): V = {v_1..v_n}, sparse vectors in R^m with unit
 * norm and positive weights; sim(x,y) = dot(x,y); the matches are the
 * unordered pairs with sim >= t.  Weights arrive as float; every product
 * of two floats is exact in double and sums are taken in double.
 *
 * Entry points:
 *   oracle_validate      input checks (positive finite weights, unique dims
 *                        in range, unit norm within a tolerance);
 *   oracle_join_plain    all-pairs-0-array (Algorithms 1 and 2 with a dense
 *                        score array, Section 4): the plain definition;
 *   oracle_join_prefix   all-pairs-1 partial indexing (Section 3.2.2) with
 *                        the optional minsize, remscore and upperbound
 *                        tests of all-pairs-2; must return the same set;
 *   oracle_prefix_index  the ingredients of partial indexing (dimension
 *                        order, maxweight_i(V), unindexed prefix length);
 *   oracle_query         Find-Matches semantics for external query rows
 *                        against a corpus, by the plain definition.
 * Output pairs are sorted by (i, j).  Parity of the paper's own printed
 * results is unpinned: the paper prints no worked example and its datasets
 * are not available.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
  int64_t count;
  int64_t* i;
  int64_t* j;
  double* s;
  /* counters of the run (mode-dependent; zero when not applicable) */
  int64_t visits;      /* inverted-list entries touched */
  int64_t candidates;  /* distinct (x, y) pairs with an accumulated score */
  int64_t verified;    /* candidates whose score was completed with dot(x, y') */
} oracle_result;

enum { OR_OK = 0, OR_EINVAL = 1, OR_ENOMEM = 3 };

/* ------------------------------------------------------------------ */
/* growable pair buffer                                                */
/* ------------------------------------------------------------------ */
typedef struct {
  int64_t n, cap;
  int64_t *i, *j;
  double* s;
} pairbuf;

static int pb_push(pairbuf* b, int64_t i, int64_t j, double s) {
  if (b->n == b->cap) {
    int64_t nc = b->cap ? 2 * b->cap : 1024;
    int64_t* ni = (int64_t*)realloc(b->i, sizeof(int64_t) * nc);
    if (!ni) return -1;
    b->i = ni;
    int64_t* nj = (int64_t*)realloc(b->j, sizeof(int64_t) * nc);
    if (!nj) return -1;
    b->j = nj;
    double* ns = (double*)realloc(b->s, sizeof(double) * nc);
    if (!ns) return -1;
    b->s = ns;
    b->cap = nc;
  }
  b->i[b->n] = i;
  b->j[b->n] = j;
  b->s[b->n] = s;
  b->n++;
  return 0;
}

typedef struct { int64_t i, j; double s; } triple;

static int cmp_triple(const void* a, const void* b) {
  const triple* x = (const triple*)a;
  const triple* y = (const triple*)b;
  if (x->i != y->i) return x->i < y->i ? -1 : 1;
  if (x->j != y->j) return x->j < y->j ? -1 : 1;
  return 0;
}

/* merge per-thread buffers into one result sorted by (i, j) */
static int finish(pairbuf* bufs, int nb, oracle_result* out) {
  int64_t total = 0;
  for (int k = 0; k < nb; ++k) total += bufs[k].n;
  triple* all = (triple*)malloc(sizeof(triple) * (size_t)(total ? total : 1));
  if (!all) return OR_ENOMEM;
  int64_t p = 0;
  for (int k = 0; k < nb; ++k) {
    for (int64_t e = 0; e < bufs[k].n; ++e) {
      all[p].i = bufs[k].i[e];
      all[p].j = bufs[k].j[e];
      all[p].s = bufs[k].s[e];
      ++p;
    }
    free(bufs[k].i); free(bufs[k].j); free(bufs[k].s);
  }
  qsort(all, (size_t)total, sizeof(triple), cmp_triple);
  out->count = total;
  out->i = (int64_t*)malloc(sizeof(int64_t) * (size_t)(total ? total : 1));
  out->j = (int64_t*)malloc(sizeof(int64_t) * (size_t)(total ? total : 1));
  out->s = (double*)malloc(sizeof(double) * (size_t)(total ? total : 1));
  if (!out->i || !out->j || !out->s) { free(all); return OR_ENOMEM; }
  for (int64_t e = 0; e < total; ++e) {
    out->i[e] = all[e].i;
    out->j[e] = all[e].j;
    out->s[e] = all[e].s;
  }
  free(all);
  return OR_OK;
}

void oracle_result_free(oracle_result* r) {
  if (!r) return;
  free(r->i); free(r->j); free(r->s);
  r->i = r->j = NULL;
  r->s = NULL;
  r->count = 0;
}

/* ------------------------------------------------------------------ */
/* input checks (Section 2.1: positive weights, unit norm)             */
/* returns 0, or 1 + the first offending row                            */
/* ------------------------------------------------------------------ */
int64_t oracle_validate(int64_t n, int64_t m, const int64_t* rp, const int32_t* col, const float* val,
                        double norm_tol) {
  if (n < 0 || m <= 0 || rp[0] != 0) return 1;
  for (int64_t r = 0; r < n; ++r) {
    if (rp[r + 1] < rp[r]) return 1 + r;
    double ss = 0.0;
    for (int64_t k = rp[r]; k < rp[r + 1]; ++k) {
      if (col[k] < 0 || col[k] >= m) return 1 + r;
      double w = (double)val[k];
      if (!(w > 0.0) || !isfinite(w)) return 1 + r;
      for (int64_t k2 = rp[r]; k2 < k; ++k2)
        if (col[k2] == col[k]) return 1 + r; /* duplicate dimension */
      ss += w * w;
    }
    if (rp[r + 1] > rp[r] && fabs(sqrt(ss) - 1.0) > norm_tol) return 1 + r;
  }
  return 0;
}

/* ------------------------------------------------------------------ */
/* inverted index I = D^T (Section 3.2.3): for every dimension d the    */
/* list of (row, weight) for rows holding d, rows ascending.           */
/* keep[k] != 0 selects which entries go into the index (all if NULL). */
/* ------------------------------------------------------------------ */
typedef struct {
  int64_t* off; /* m + 1 */
  int64_t* row;
  double* w;
} invindex;

static int build_index(int64_t n, int64_t m, const int64_t* rp, const int32_t* col, const float* val,
                       const unsigned char* keep, invindex* I) {
  I->off = (int64_t*)calloc((size_t)m + 1, sizeof(int64_t));
  if (!I->off) return -1;
  int64_t total = 0;
  for (int64_t k = 0; k < rp[n]; ++k)
    if (!keep || keep[k]) { I->off[col[k] + 1]++; total++; }
  for (int64_t d = 0; d < m; ++d) I->off[d + 1] += I->off[d];
  I->row = (int64_t*)malloc(sizeof(int64_t) * (size_t)(total ? total : 1));
  I->w = (double*)malloc(sizeof(double) * (size_t)(total ? total : 1));
  int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)m);
  if (!I->row || !I->w || !fill) { free(fill); return -1; }
  memcpy(fill, I->off, sizeof(int64_t) * (size_t)m);
  for (int64_t r = 0; r < n; ++r)
    for (int64_t k = rp[r]; k < rp[r + 1]; ++k)
      if (!keep || keep[k]) {
        int64_t p = fill[col[k]]++;
        I->row[p] = r;
        I->w[p] = (double)val[k];
      }
  free(fill);
  return 0;
}

static void free_index(invindex* I) {
  free(I->off); free(I->row); free(I->w);
}

static int nthreads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

static int thread_id(void) {
#ifdef _OPENMP
  return omp_get_thread_num();
#else
  return 0;
#endif
}

/* ------------------------------------------------------------------ */
/* all-pairs-0-array: Algorithm 1 drives Algorithm 2 over every vector; */
/* the score map A is a dense array (Section 4).  Matching v_i against  */
/* the index of the vectors before it is the same as matching it        */
/* against the full index restricted to rows j < i, which lets threads  */
/* take different i.  Row i_begin..i_end-1 are the x vectors (all rows  */
/* when i_end <= 0).                                                    */
/* ------------------------------------------------------------------ */
int oracle_join_plain(int64_t n, int64_t m, const int64_t* rp, const int32_t* col, const float* val,
                      double t, int64_t i_begin, int64_t i_end, oracle_result* out) {
  memset(out, 0, sizeof(*out));
  if (i_end <= 0 || i_end > n) i_end = n;
  if (i_begin < 0) i_begin = 0;
  invindex I;
  if (build_index(n, m, rp, col, val, NULL, &I)) return OR_ENOMEM;
  int nt = nthreads();
  pairbuf* bufs = (pairbuf*)calloc((size_t)nt, sizeof(pairbuf));
  int64_t visits = 0, cands = 0;
  int fail = 0;
#pragma omp parallel reduction(+ : visits, cands)
  {
    int me = thread_id();
    double* A = (double*)calloc((size_t)(n ? n : 1), sizeof(double));
    int64_t* touched = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
    if (!A || !touched) {
#pragma omp atomic write
      fail = 1;
    } else {
#pragma omp for schedule(dynamic, 16)
      for (int64_t i = i_begin; i < i_end; ++i) {
        int64_t nt_ = 0;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
          int32_t d = col[k];
          double xw = (double)val[k];
          for (int64_t p = I.off[d]; p < I.off[d + 1]; ++p) {
            int64_t j = I.row[p];
            if (j >= i) break; /* lists are sorted by row */
            if (A[j] == 0.0) touched[nt_++] = j;
            A[j] += xw * I.w[p];
            visits++;
          }
        }
        cands += nt_;
        for (int64_t e = 0; e < nt_; ++e) {
          int64_t j = touched[e];
          if (A[j] >= t && pb_push(&bufs[me], j, i, A[j])) {
#pragma omp atomic write
            fail = 1;
          }
          A[j] = 0.0;
        }
      }
    }
    free(A);
    free(touched);
  }
  free_index(&I);
  if (fail) { for (int k = 0; k < nt; ++k) { free(bufs[k].i); free(bufs[k].j); free(bufs[k].s); } free(bufs); return OR_ENOMEM; }
  int rc = finish(bufs, nt, out);
  free(bufs);
  out->visits = visits;
  out->candidates = cands;
  return rc;
}

/* ------------------------------------------------------------------ */
/* Partial indexing ingredients (Section 3.2.2, all-pairs-1):           */
/*  - dimensions ordered by decreasing number of non-zeros (ties by     */
/*    ascending dimension id);                                          */
/*  - maxweight_d(V), the largest weight in dimension d;                */
/*  - for every vector, its components in that order, the running bound */
/*    b = sum x[d] * maxweight_d(V); the leading components whose b     */
/*    stays below t form the unindexed part x', the rest are indexed    */
/*    (a component is indexed as soon as b, including it, reaches t).   */
/*    With l2_clause, the unindexed part also stops once its own L2     */
/*    norm reaches t (compared as squared norm >= t*t, exact for a      */
/*    float t), which keeps dot(q, x') < t for any unit query q.        */
/* Outputs: rank[m] (position of each dim in the order), mw[m],         */
/* cut[n] (number of unindexed components of each row).                */
/* ------------------------------------------------------------------ */
typedef struct { int32_t rank; int32_t pos; } rankpos;

static int cmp_rankpos(const void* a, const void* b) {
  const rankpos* x = (const rankpos*)a;
  const rankpos* y = (const rankpos*)b;
  return (x->rank > y->rank) - (x->rank < y->rank);
}

typedef struct { int64_t cnt; int32_t d; } dimcnt;

static int cmp_dimcnt(const void* a, const void* b) {
  const dimcnt* x = (const dimcnt*)a;
  const dimcnt* y = (const dimcnt*)b;
  if (x->cnt != y->cnt) return x->cnt > y->cnt ? -1 : 1; /* decreasing count */
  return (x->d > y->d) - (x->d < y->d);                   /* then dimension id */
}

int oracle_prefix_index(int64_t n, int64_t m, const int64_t* rp, const int32_t* col, const float* val,
                        double t, int l2_clause, int32_t* rank, float* mw, int32_t* cut) {
  dimcnt* dc = (dimcnt*)malloc(sizeof(dimcnt) * (size_t)m);
  if (!dc) return OR_ENOMEM;
  for (int64_t d = 0; d < m; ++d) { dc[d].cnt = 0; dc[d].d = (int32_t)d; mw[d] = 0.0f; }
  for (int64_t k = 0; k < rp[n]; ++k) {
    dc[col[k]].cnt++;
    if (val[k] > mw[col[k]]) mw[col[k]] = val[k];
  }
  qsort(dc, (size_t)m, sizeof(dimcnt), cmp_dimcnt);
  for (int64_t r = 0; r < m; ++r) rank[dc[r].d] = (int32_t)r;
  free(dc);
  int fail = 0;
#pragma omp parallel
  {
    rankpos* rpbuf = NULL;
    int64_t cap = 0;
#pragma omp for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
      int64_t len = rp[i + 1] - rp[i];
      if (len > cap) { free(rpbuf); cap = len; rpbuf = (rankpos*)malloc(sizeof(rankpos) * (size_t)cap); }
      if (len && !rpbuf) {
#pragma omp atomic write
        fail = 1;
        continue;
      }
      for (int64_t k = 0; k < len; ++k) { rpbuf[k].rank = rank[col[rp[i] + k]]; rpbuf[k].pos = (int32_t)k; }
      qsort(rpbuf, (size_t)len, sizeof(rankpos), cmp_rankpos);
      double b = 0.0, sq = 0.0;
      int32_t c = (int32_t)len;
      for (int64_t k = 0; k < len; ++k) {
        int64_t e = rp[i] + rpbuf[k].pos;
        double w = (double)val[e];
        b += w * (double)mw[col[e]];
        sq += w * w;
        if (b >= t || (l2_clause && sq >= t * t)) { c = (int32_t)k; break; }
      }
      cut[i] = c;
    }
    free(rpbuf);
  }
  return fail ? OR_ENOMEM : OR_OK;
}

/* ------------------------------------------------------------------ */
/* all-pairs-1 (partial indexing) with the optional bounds of            */
/* all-pairs-2, run in the order of Algorithm 1: match v_i against the   */
/* index built so far, then add v_i's indexed components.               */
/*   flags & 1 : minsize -- a candidate y is only scored when           */
/*               |y| * maxweight(x) >= t   (x.y <= maxweight(x) |y|)     */
/*   flags & 2 : upperbound -- skip dot(x, y') when                      */
/*               A[y] + min(|y'|, |x|) maxweight(x) maxweight(y') < t    */
/*   flags & 4 : l2 clause in the cutoff (see oracle_prefix_index)      */
/*   flags & 8 : remscore -- x's components are processed rarest first;  */
/*               remscore starts at sum_i x[i] maxweight_i(V) and loses  */
/*               each component's term after it is processed; while it  */
/*               is below t a y not yet in the map is not added          */
/* The score is completed as A[y] + dot(x, y').                         */
/* ------------------------------------------------------------------ */
int oracle_join_prefix(int64_t n, int64_t m, const int64_t* rp, const int32_t* col, const float* val,
                       double t, int flags, oracle_result* out) {
  memset(out, 0, sizeof(*out));
  int32_t* rank = (int32_t*)malloc(sizeof(int32_t) * (size_t)m);
  float* mw = (float*)malloc(sizeof(float) * (size_t)m);
  int32_t* cut = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
  if (!rank || !mw || !cut) { free(rank); free(mw); free(cut); return OR_ENOMEM; }
  int rc = oracle_prefix_index(n, m, rp, col, val, t, (flags & 4) ? 1 : 0, rank, mw, cut);
  if (rc) { free(rank); free(mw); free(cut); return rc; }

  /* per row: components sorted by rank (densest dimension first), the
     unindexed part x' is the first cut[i] of them */
  int64_t nnz = rp[n];
  int32_t* sdim = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nnz ? nnz : 1));
  double* sw = (double*)malloc(sizeof(double) * (size_t)(nnz ? nnz : 1));
  double* xmax = (double*)malloc(sizeof(double) * (size_t)(n ? n : 1));  /* maxweight(x) */
  double* pmax = (double*)malloc(sizeof(double) * (size_t)(n ? n : 1));  /* maxweight(x') */
  /* dense map dim -> weight of the current x, for dot(x, y') */
  double* xdense = (double*)calloc((size_t)m, sizeof(double));
  /* index lists grown as vectors are indexed; sizes known in advance */
  int64_t* ioff = (int64_t*)calloc((size_t)m + 1, sizeof(int64_t));
  int64_t* ifill = (int64_t*)malloc(sizeof(int64_t) * (size_t)m);
  double* A = (double*)calloc((size_t)(n ? n : 1), sizeof(double));
  unsigned char* seen = (unsigned char*)calloc((size_t)(n ? n : 1), 1);
  int64_t* touched = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
  if (!sdim || !sw || !xmax || !pmax || !xdense || !ioff || !ifill || !A || !seen || !touched) {
    rc = OR_ENOMEM;
    goto done;
  }
  {
    int64_t cap = 0;
    rankpos* rpbuf = NULL;
    for (int64_t i = 0; i < n; ++i) {
      int64_t len = rp[i + 1] - rp[i];
      if (len > cap) { free(rpbuf); cap = len; rpbuf = (rankpos*)malloc(sizeof(rankpos) * (size_t)cap); }
      for (int64_t k = 0; k < len; ++k) { rpbuf[k].rank = rank[col[rp[i] + k]]; rpbuf[k].pos = (int32_t)k; }
      qsort(rpbuf, (size_t)len, sizeof(rankpos), cmp_rankpos);
      double mx = 0.0, px = 0.0;
      for (int64_t k = 0; k < len; ++k) {
        int64_t e = rp[i] + rpbuf[k].pos;
        sdim[rp[i] + k] = col[e];
        sw[rp[i] + k] = (double)val[e];
        if (sw[rp[i] + k] > mx) mx = sw[rp[i] + k];
        if (k < cut[i] && sw[rp[i] + k] > px) px = sw[rp[i] + k];
        if (k >= cut[i]) ioff[col[e] + 1]++;
      }
      xmax[i] = mx;
      pmax[i] = px;
    }
    free(rpbuf);
  }
  for (int64_t d = 0; d < m; ++d) ioff[d + 1] += ioff[d];
  memcpy(ifill, ioff, sizeof(int64_t) * (size_t)m);
  {
    int64_t ipost = ioff[m];
    int64_t* irow = (int64_t*)malloc(sizeof(int64_t) * (size_t)(ipost ? ipost : 1));
    double* iw = (double*)malloc(sizeof(double) * (size_t)(ipost ? ipost : 1));
    pairbuf buf = {0, 0, NULL, NULL, NULL};
    if (!irow || !iw) { free(irow); free(iw); rc = OR_ENOMEM; goto done; }
    int64_t visits = 0, cands = 0, verified = 0;
    for (int64_t i = 0; i < n; ++i) {
      int64_t a = rp[i], len = rp[i + 1] - rp[i];
      /* Find-Matches: every component of x against the lists */
      int64_t ntch = 0;
      double remscore = 0.0;
      if (flags & 8)
        for (int64_t k = 0; k < len; ++k) remscore += sw[a + k] * (double)mw[sdim[a + k]];
      for (int64_t kk = 0; kk < len; ++kk) {
        /* remscore processes the rarest dimension first */
        int64_t k = (flags & 8) ? len - 1 - kk : kk;
        int32_t d = sdim[a + k];
        double xw = sw[a + k];
        xdense[d] = xw;
        for (int64_t p = ioff[d]; p < ifill[d]; ++p) {
          int64_t y = irow[p];
          visits++;
          if ((flags & 1) && (double)(rp[y + 1] - rp[y]) * xmax[i] < t) continue;
          if (!seen[y]) {
            if ((flags & 8) && remscore < t) continue;
            seen[y] = 1;
            touched[ntch++] = y;
          }
          A[y] += xw * iw[p];
        }
        if (flags & 8) remscore -= xw * (double)mw[d];
      }
      cands += ntch;
      for (int64_t e = 0; e < ntch; ++e) {
        int64_t y = touched[e];
        double sc = A[y];
        int64_t yp = cut[y];
        int keep = 1;
        if (flags & 2) {
          double mn = (double)(yp < len ? yp : len);
          if (sc + mn * xmax[i] * pmax[y] < t) keep = 0;
        }
        if (keep) {
          verified++;
          for (int64_t k = 0; k < yp; ++k) sc += xdense[sdim[rp[y] + k]] * sw[rp[y] + k];
          if (sc >= t && pb_push(&buf, y, i, sc)) rc = OR_ENOMEM;
        }
        A[y] = 0.0;
        seen[y] = 0;
      }
      for (int64_t k = 0; k < len; ++k) xdense[sdim[a + k]] = 0.0;
      /* index the components from the cutoff on */
      for (int64_t k = cut[i]; k < len; ++k) {
        int32_t d = sdim[a + k];
        int64_t p = ifill[d]++;
        irow[p] = i;
        iw[p] = sw[a + k];
      }
    }
    free(irow);
    free(iw);
    if (rc == OR_OK) {
      rc = finish(&buf, 1, out);
      out->visits = visits;
      out->candidates = cands;
      out->verified = verified;
    }
  }
done:
  free(rank); free(mw); free(cut); free(sdim); free(sw); free(xmax); free(pmax); free(xdense);
  free(ioff); free(ifill); free(A); free(seen); free(touched);
  return rc;
}

/* ------------------------------------------------------------------ */
/* External queries (Find-Matches, Algorithm 2, against a corpus):      */
/* every (query row q, corpus row y) with dot(q, y) >= t_q, by the       */
/* plain definition over the full inverted index of the corpus.         */
/* t_per_row may be NULL (then t applies to every query).               */
/* Output (i = query row, j = corpus row).                               */
/* ------------------------------------------------------------------ */
int oracle_query(int64_t n, int64_t m, const int64_t* rp, const int32_t* col, const float* val,
                 int64_t nq, const int64_t* qrp, const int32_t* qcol, const float* qval,
                 const double* t_per_row, double t, oracle_result* out) {
  memset(out, 0, sizeof(*out));
  invindex I;
  if (build_index(n, m, rp, col, val, NULL, &I)) return OR_ENOMEM;
  int nt = nthreads();
  pairbuf* bufs = (pairbuf*)calloc((size_t)nt, sizeof(pairbuf));
  int fail = 0;
  int64_t visits = 0, cands = 0;
#pragma omp parallel reduction(+ : visits, cands)
  {
    int me = thread_id();
    double* A = (double*)calloc((size_t)(n ? n : 1), sizeof(double));
    int64_t* touched = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
    if (!A || !touched) {
#pragma omp atomic write
      fail = 1;
    } else {
#pragma omp for schedule(dynamic, 4)
      for (int64_t q = 0; q < nq; ++q) {
        double tq = t_per_row ? t_per_row[q] : t;
        int64_t ntch = 0;
        for (int64_t k = qrp[q]; k < qrp[q + 1]; ++k) {
          int32_t d = qcol[k];
          if (d < 0 || d >= m) continue;
          double xw = (double)qval[k];
          for (int64_t p = I.off[d]; p < I.off[d + 1]; ++p) {
            int64_t y = I.row[p];
            if (A[y] == 0.0) touched[ntch++] = y;
            A[y] += xw * I.w[p];
            visits++;
          }
        }
        cands += ntch;
        for (int64_t e = 0; e < ntch; ++e) {
          int64_t y = touched[e];
          if (A[y] >= tq && pb_push(&bufs[me], q, y, A[y])) {
#pragma omp atomic write
            fail = 1;
          }
          A[y] = 0.0;
        }
      }
    }
    free(A);
    free(touched);
  }
  free_index(&I);
  if (fail) { for (int k = 0; k < nt; ++k) { free(bufs[k].i); free(bufs[k].j); free(bufs[k].s); } free(bufs); return OR_ENOMEM; }
  int rc = finish(bufs, nt, out);
  free(bufs);
  out->visits = visits;
  out->candidates = cands;
  return rc;
}

int oracle_num_threads(void) { return nthreads(); }
