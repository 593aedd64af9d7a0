/* Seeded synthetic sparse corpora (input generation only).
 *
 * Holds none of the join's arithmetic.  Every random number is a pure
 * function of (seed, stream, row, counter) through the SplitMix64 finaliser
 * (Steele, Lea, Flood, "Fast splittable pseudorandom number generators",
 * OOPSLA 2014), so rows can be generated in parallel and the output does not
 * depend on the thread count.
 *
 * Row r:
 *   nnz_r   : uniform integer in [lo, hi], or round(lognormal(mu, sigma)) clipped;
 *   ranks   : k in [0, m) with P(k) proportional to (k+1)^-s, drawn in order,
 *             repeats rejected until nnz_r distinct ranks are held;
 *   dims    : perm[rank], perm a seeded Fisher-Yates permutation of [0, m);
 *             stored ascending;
 *   weights : lognormal(0,1) (Box-Muller normals), scaled to unit L2 norm
 *             in double precision, then rounded to float.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define STREAM_NNZ 1u
#define STREAM_DIM 2u
#define STREAM_W 3u
#define STREAM_PERM 4u

static inline uint64_t mix64(uint64_t z) {
  z += 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

static inline uint64_t draw(uint64_t seed, uint32_t stream, uint64_t row, uint64_t k) {
  uint64_t h = mix64(seed ^ ((uint64_t)stream << 56));
  h = mix64(h ^ row);
  return mix64(h ^ (k * 0xd1b54a32d192ed03ull));
}

/* uniform double in (0, 1): 53 random bits, offset by half an ulp */
static inline double unif(uint64_t x) { return ((double)(x >> 11) + 0.5) * (1.0 / 9007199254740992.0); }

static double normal(uint64_t seed, uint32_t stream, uint64_t row, uint64_t k) {
  double u1 = unif(draw(seed, stream, row, 2 * k));
  double u2 = unif(draw(seed, stream, row, 2 * k + 1));
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

/* nnz per row.  kind 0 = uniform [a, b]; kind 1 = lognormal with mean a, sigma b. */
void synth_nnz(int64_t n, uint64_t seed, int kind, double a, double b, int64_t lo, int64_t hi,
               int64_t* nnz_out) {
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < n; ++r) {
    int64_t k;
    if (kind == 0) {
      uint64_t span = (uint64_t)((int64_t)b - (int64_t)a + 1);
      k = (int64_t)a + (int64_t)(unif(draw(seed, STREAM_NNZ, (uint64_t)r, 0)) * (double)span);
      if (k > (int64_t)b) k = (int64_t)b;
    } else {
      double mu = log(a) - 0.5 * b * b;
      double z = normal(seed, STREAM_NNZ, (uint64_t)r, 0);
      k = (int64_t)llround(exp(mu + b * z));
    }
    if (k < lo) k = lo;
    if (k > hi) k = hi;
    nnz_out[r] = k;
  }
}

/* Fill col/val for rows [0, n) given row_ptr (prefix sums of nnz). */
int synth_rows(int64_t n, int64_t m, uint64_t seed, double s, const int64_t* row_ptr, int32_t* col,
               float* val) {
  if (m <= 0 || m > (1ll << 31) - 2) return -1;
  /* cdf over ranks and a guide table for the inverse-CDF search */
  double* cdf = (double*)malloc(sizeof(double) * (size_t)m);
  int32_t* perm = (int32_t*)malloc(sizeof(int32_t) * (size_t)m);
  const int64_t nguide = 1 << 22;
  int32_t* guide = (int32_t*)malloc(sizeof(int32_t) * (size_t)nguide);
  if (!cdf || !perm || !guide) { free(cdf); free(perm); free(guide); return -2; }
  double acc = 0.0;
  for (int64_t k = 0; k < m; ++k) { acc += pow((double)(k + 1), -s); cdf[k] = acc; }
  for (int64_t k = 0; k < m; ++k) cdf[k] /= acc;
  cdf[m - 1] = 1.0;
  {
    int64_t k = 0;
    for (int64_t g = 0; g < nguide; ++g) {
      double x = (double)g / (double)nguide;
      while (k < m - 1 && cdf[k] <= x) ++k;
      guide[g] = (int32_t)k;
    }
  }
  for (int64_t k = 0; k < m; ++k) perm[k] = (int32_t)k;
  for (int64_t k = m - 1; k > 0; --k) {
    int64_t j = (int64_t)(unif(draw(seed, STREAM_PERM, 0, (uint64_t)k)) * (double)(k + 1));
    if (j > k) j = k;
    int32_t tmp = perm[k]; perm[k] = perm[j]; perm[j] = tmp;
  }
  int err = 0;
#pragma omp parallel
  {
    int32_t* stamp = (int32_t*)malloc(sizeof(int32_t) * (size_t)m);
    double* w = NULL;
    int64_t wcap = 0;
    if (!stamp) {
#pragma omp atomic write
      err = -2;
    } else {
      for (int64_t k = 0; k < m; ++k) stamp[k] = -1;
#pragma omp for schedule(dynamic, 256)
      for (int64_t r = 0; r < n; ++r) {
        int64_t a = row_ptr[r], len = row_ptr[r + 1] - row_ptr[r];
        if (len > m) len = m;
        int32_t tag = (int32_t)(r & 0x7fffffff);
        int64_t got = 0;
        for (uint64_t k = 0; got < len; ++k) {
          double u = unif(draw(seed, STREAM_DIM, (uint64_t)r, k));
          int64_t lo = guide[(int64_t)(u * (double)nguide)];
          while (lo < m - 1 && cdf[lo] <= u) ++lo;
          if (stamp[lo] == tag) continue;
          stamp[lo] = tag;
          col[a + got++] = perm[lo];
        }
        qsort(col + a, (size_t)len, sizeof(int32_t), cmp_i32);
        if (len > wcap) { free(w); wcap = len; w = (double*)malloc(sizeof(double) * (size_t)wcap); }
        double ss = 0.0;
        for (int64_t k = 0; k < len; ++k) {
          double x = exp(normal(seed, STREAM_W, (uint64_t)r, (uint64_t)k));
          w[k] = x;
          ss += x * x;
        }
        double inv = 1.0 / sqrt(ss);
        for (int64_t k = 0; k < len; ++k) val[a + k] = (float)(w[k] * inv);
      }
      free(stamp);
      free(w);
    }
  }
  free(cdf); free(perm); free(guide);
  return err;
}
