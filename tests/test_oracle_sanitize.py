"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

apss_oracle.c is compiled with gcc's address and undefined-behaviour
sanitizers into a small driver that runs every entry point on seeded
corpora (empty rows included) and on the golden fixture, with leak checking
on.  A sanitizer finding fails the run; the driver's pair counts must equal
those of the ordinary build loaded through ``oracle``.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from synth.corpus import from_rows, make_corpus, spec_for
from tests.test_oracle import load_golden

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_C = os.path.join(ROOT, "oracle", "apss_oracle.c")

DRIVER = r"""
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
  int64_t count;
  int64_t* i;
  int64_t* j;
  double* s;
  int64_t visits, candidates, verified;
} oracle_result;

int64_t oracle_validate(int64_t, int64_t, const int64_t*, const int32_t*, const float*, double);
int oracle_join_plain(int64_t, int64_t, const int64_t*, const int32_t*, const float*, double, int64_t, int64_t,
                      oracle_result*);
int oracle_join_prefix(int64_t, int64_t, const int64_t*, const int32_t*, const float*, double, int, oracle_result*);
int oracle_prefix_index(int64_t, int64_t, const int64_t*, const int32_t*, const float*, double, int, int32_t*, float*,
                        int32_t*);
int oracle_query(int64_t, int64_t, const int64_t*, const int32_t*, const float*, int64_t, const int64_t*,
                 const int32_t*, const float*, const double*, double, oracle_result*);
void oracle_result_free(oracle_result*);

static void* slurp(const char* path, size_t* bytes) {
  FILE* f = fopen(path, "rb");
  if (!f) { perror(path); exit(2); }
  fseek(f, 0, SEEK_END);
  long b = ftell(f);
  fseek(f, 0, SEEK_SET);
  void* p = malloc(b > 0 ? (size_t)b : 1);
  if (b > 0 && fread(p, 1, (size_t)b, f) != (size_t)b) { perror(path); exit(2); }
  fclose(f);
  *bytes = (size_t)b;
  return p;
}

/* usage: driver dir n m t */
int main(int argc, char** argv) {
  if (argc != 5) return 2;
  char path[4096];
  size_t b;
  const int64_t n = atoll(argv[2]), m = atoll(argv[3]);
  const double t = atof(argv[4]);
  snprintf(path, sizeof(path), "%s/rp.bin", argv[1]);
  int64_t* rp = (int64_t*)slurp(path, &b);
  snprintf(path, sizeof(path), "%s/col.bin", argv[1]);
  int32_t* col = (int32_t*)slurp(path, &b);
  snprintf(path, sizeof(path), "%s/val.bin", argv[1]);
  float* val = (float*)slurp(path, &b);
  printf("validate %lld\n", (long long)oracle_validate(n, m, rp, col, val, 1e-5));
  oracle_result r;
  if (oracle_join_plain(n, m, rp, col, val, t, 0, 0, &r)) return 3;
  printf("plain %lld %lld\n", (long long)r.count, (long long)r.candidates);
  oracle_result_free(&r);
  if (oracle_join_plain(n, m, rp, col, val, t, n / 3, n / 2, &r)) return 3;
  printf("window %lld\n", (long long)r.count);
  oracle_result_free(&r);
  for (int flags = 0; flags < 16; ++flags) {
    if (oracle_join_prefix(n, m, rp, col, val, t, flags, &r)) return 4;
    printf("prefix %d %lld %lld\n", flags, (long long)r.count, (long long)r.candidates);
    oracle_result_free(&r);
  }
  int32_t* rank = (int32_t*)malloc(sizeof(int32_t) * (size_t)m);
  float* mw = (float*)malloc(sizeof(float) * (size_t)m);
  int32_t* cut = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  for (int l2 = 0; l2 < 2; ++l2) {
    if (oracle_prefix_index(n, m, rp, col, val, t, l2, rank, mw, cut)) return 5;
    long long s = 0;
    for (int64_t r2 = 0; r2 < n; ++r2) s += cut[r2];
    printf("cuts %d %lld\n", l2, s);
  }
  /* every third row as an external query, with per-row thresholds */
  const int64_t nq = (n + 2) / 3;
  int64_t* qrp = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nq + 1));
  double* tq = (double*)malloc(sizeof(double) * (size_t)(nq > 0 ? nq : 1));
  qrp[0] = 0;
  for (int64_t q = 0; q < nq; ++q) {
    const int64_t r2 = 3 * q;
    qrp[q + 1] = qrp[q] + (rp[r2 + 1] - rp[r2]);
    tq[q] = t + 0.3 * (double)(q % 4) / 4.0;
  }
  int32_t* qcol = (int32_t*)malloc(sizeof(int32_t) * (size_t)(qrp[nq] > 0 ? qrp[nq] : 1));
  float* qval = (float*)malloc(sizeof(float) * (size_t)(qrp[nq] > 0 ? qrp[nq] : 1));
  for (int64_t q = 0; q < nq; ++q)
    for (int64_t k = 0; k < qrp[q + 1] - qrp[q]; ++k) {
      qcol[qrp[q] + k] = col[rp[3 * q] + k];
      qval[qrp[q] + k] = val[rp[3 * q] + k];
    }
  if (oracle_query(n, m, rp, col, val, nq, qrp, qcol, qval, tq, t, &r)) return 6;
  printf("query %lld\n", (long long)r.count);
  oracle_result_free(&r);
  free(qrp); free(tq); free(qcol); free(qval); free(rank); free(mw); free(cut);
  free(rp); free(col); free(val);
  return 0;
}
"""


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    d = tmp_path_factory.mktemp("asan")
    src = d / "driver.c"
    src.write_text(DRIVER)
    exe = d / "driver"
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fopenmp", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-o", str(exe), str(src), ORACLE_C, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "asan" in (r.stderr or "").lower():
        pytest.skip("sanitizer runtime not available: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr
    return str(exe)


def run_case(driver, tmp_path, V, t):
    for name, arr, dt in (("rp", V.row_ptr, np.int64), ("col", V.col, np.int32), ("val", V.val, np.float32)):
        np.ascontiguousarray(arr, dtype=dt).tofile(str(tmp_path / (name + ".bin")))
    env = dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([driver, str(tmp_path), str(V.n), str(V.m), repr(float(t))], capture_output=True, text=True,
                       env=env, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
    out = {}
    for line in r.stdout.splitlines():
        f = line.split()
        out[" ".join(f[:2]) if f[0] in ("prefix", "cuts") else f[0]] = [int(x) for x in f[1:]]
    return out


@pytest.mark.parametrize("case", ["c1", "c2", "empty_rows", "golden"])
def test_oracle_under_sanitizers(driver, tmp_path, case):
    if case == "golden":
        V, _, _, cases = load_golden()
        t = cases[0]["t"]
    elif case == "empty_rows":
        base = make_corpus(spec_for("c1", n=200))
        rows = [dict(zip(base.row(k)[0].tolist(), base.row(k)[1].tolist())) for k in range(base.n)]
        rows = rows[:50] + [{}] * 7 + rows[50:] + [{}]
        V = from_rows(rows, base.m)
        t = 0.5
    else:
        V = make_corpus(spec_for(case, n=300 if case == "c1" else 900))
        t = 0.5
    out = run_case(driver, tmp_path, V, np.float32(t))
    assert out["validate"] == [0]
    ref = oracle.join_plain(V, np.float32(t))
    assert out["plain"] == [len(ref), ref.candidates]
    for flags in range(16):
        pre = oracle.join_prefix(V, np.float32(t), flags)
        assert out["prefix %d" % flags][1:] == [len(pre), pre.candidates]
