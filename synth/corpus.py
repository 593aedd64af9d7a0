"""Seeded synthetic sparse corpora shaped like the paper's workloads.

This module only generates inputs.  It holds none of the join's arithmetic:
no dimension ranking, no bounds, no dot products.  Both the CPU oracle and
the GPU library receive the arrays it produces.

Shape regime (Section 7, Table 1): document-term style data with a few very
dense dimensions and a long tail of rare ones, i.e. dimension popularity that
follows a power law.  Each vector is a list of (dimension, weight) pairs
(Section 2.1) with positive weights and unit L2 norm.

Recipe (implemented in synth.c; every random number is a pure function of
(seed, stream, row, counter), so the output does not depend on threading):

* nnz per vector: uniform integers, or a lognormal with the stated mean
  (mu = ln(mean) - sigma^2/2), rounded to the nearest integer and clipped.
* dimensions: a popularity rank k in [1, m] is drawn with probability
  proportional to k^-s; repeats inside a vector are rejected until the vector
  holds its nnz distinct ranks.  Ranks map to dimension ids through a seeded
  random permutation of [0, m), so the consumer must discover the popularity
  order itself.
* weights: i.i.d. lognormal(0, 1), normalised to unit L2 norm in float64 and
  then rounded to float32.  The float32 values are the ground truth.

Rows are stored in CSR form with dimension ids ascending inside a row.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np


@dataclasses.dataclass(frozen=True)
class CorpusSpec:
    n: int
    m: int
    nnz_kind: str            # "uniform" | "lognormal"
    nnz_a: float             # uniform: low  | lognormal: mean
    nnz_b: float             # uniform: high | lognormal: sigma
    nnz_lo: int
    nnz_hi: int
    zipf_s: float
    seed: int


@dataclasses.dataclass
class Csr:
    n: int
    m: int
    row_ptr: np.ndarray      # int64[n+1]
    col: np.ndarray          # int32[nnz], ascending within a row
    val: np.ndarray          # float32[nnz], > 0, unit L2 norm per non-empty row

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def row(self, i: int):
        a, b = int(self.row_ptr[i]), int(self.row_ptr[i + 1])
        return self.col[a:b], self.val[a:b]

    def take_rows(self, rows: np.ndarray) -> "Csr":
        rows = np.asarray(rows, dtype=np.int64)
        lens = self.row_ptr[rows + 1] - self.row_ptr[rows]
        rp = np.zeros(len(rows) + 1, dtype=np.int64)
        np.cumsum(lens, out=rp[1:])
        idx = np.repeat(self.row_ptr[rows] - rp[:-1], lens) + np.arange(rp[-1], dtype=np.int64)
        return Csr(len(rows), self.m, rp, self.col[idx].copy(), self.val[idx].copy())


# ---------------------------------------------------------------------------
# Named workloads.  Sizes, distributions and seeds of the five configurations.
# ---------------------------------------------------------------------------
CONFIGS = {
    "c1": dict(spec=CorpusSpec(2_000, 10_000, "uniform", 10, 60, 10, 60, 1.0, 1001), t=[0.5]),
    "c2": dict(spec=CorpusSpec(100_000, 200_000, "lognormal", 80, 1.0, 5, 2000, 1.1, 1002), t=[0.5, 0.7, 0.9]),
    "c3": dict(spec=CorpusSpec(1_000_000, 1_000_000, "lognormal", 120, 1.2, 5, 5000, 1.0, 1003), t=[0.7]),
    "c4": dict(spec=CorpusSpec(500_000, 500_000, "lognormal", 150, 1.0, 5, 2000, 0.9, 1004), t=[0.8]),
    "c5": dict(spec=CorpusSpec(2_000_000, 1_000_000, "lognormal", 100, 1.0, 5, 2000, 1.0, 1005), t=[0.5, 0.95]),
}


def spec_for(name: str, n: Optional[int] = None, seed: Optional[int] = None) -> CorpusSpec:
    """Named spec, optionally with fewer rows (same m and distributions) or another seed."""
    s = CONFIGS[name]["spec"]
    return dataclasses.replace(s, n=s.n if n is None else n, seed=s.seed if seed is None else seed)


_LIB = None


def _lib():
    """The compiled generator (synth.c), built in place on first use."""
    global _LIB
    if _LIB is None:
        import ctypes
        import os
        here = os.path.dirname(os.path.abspath(__file__))
        so = os.path.join(here, "libsynth.so")
        srcf = os.path.join(here, "synth.c")
        if not os.path.exists(so) or os.path.getmtime(so) < os.path.getmtime(srcf):
            build()
        lib = ctypes.CDLL(so)
        i64p = ctypes.POINTER(ctypes.c_int64)
        lib.synth_nnz.argtypes = [ctypes.c_int64, ctypes.c_uint64, ctypes.c_int, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_int64, ctypes.c_int64, i64p]
        lib.synth_nnz.restype = None
        lib.synth_rows.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double,
                                   i64p, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_float)]
        lib.synth_rows.restype = ctypes.c_int
        _LIB = lib
    return _LIB


def build() -> str:
    """Compile synth.c into libsynth.so next to it (gcc, OpenMP)."""
    import os
    import subprocess
    here = os.path.dirname(os.path.abspath(__file__))
    so = os.path.join(here, "libsynth.so")
    tmp = so + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp,
                           os.path.join(here, "synth.c"), "-lm"])
    os.replace(tmp, so)
    return so


def _ptr(a, ct):
    import ctypes
    return a.ctypes.data_as(ctypes.POINTER(ct))


def make_corpus(spec: CorpusSpec) -> Csr:
    import ctypes
    lib = _lib()
    kind = {"uniform": 0, "lognormal": 1}[spec.nnz_kind]
    nnz = np.empty(spec.n, dtype=np.int64)
    lib.synth_nnz(spec.n, spec.seed, kind, float(spec.nnz_a), float(spec.nnz_b), spec.nnz_lo,
                  min(spec.nnz_hi, spec.m), _ptr(nnz, ctypes.c_int64))
    row_ptr = np.zeros(spec.n + 1, dtype=np.int64)
    np.cumsum(nnz, out=row_ptr[1:])
    col = np.empty(int(row_ptr[-1]), dtype=np.int32)
    val = np.empty(int(row_ptr[-1]), dtype=np.float32)
    rc = lib.synth_rows(spec.n, spec.m, spec.seed, float(spec.zipf_s), _ptr(row_ptr, ctypes.c_int64),
                        _ptr(col, ctypes.c_int32), _ptr(val, ctypes.c_float))
    if rc != 0:
        raise MemoryError("synth_rows failed (%d)" % rc)
    return Csr(spec.n, spec.m, row_ptr, col, val)


def make_queries(corpus: Csr, nq: int, spec: CorpusSpec, seed: int, frac_copies: float = 0.10,
                 jitter_sigma: float = 0.05) -> Csr:
    """Query rows for the serving workload.

    Most rows come from the corpus generator with a fresh seed.  A fraction
    are perturbed copies of random corpus rows (each weight multiplied by
    lognormal(0, jitter_sigma), renormalised) so that high thresholds have hits.
    """
    ss = np.random.SeedSequence(seed)
    s_pick, s_jit, s_which = ss.spawn(3)
    fresh = make_corpus(dataclasses.replace(spec, n=nq, seed=seed))
    if frac_copies <= 0:
        return fresh
    rng = np.random.default_rng(s_which)
    is_copy = rng.random(nq) < frac_copies
    src = np.random.default_rng(s_pick).integers(0, corpus.n, size=nq)
    rng_j = np.random.default_rng(s_jit)
    rows_c, rows_v, lens = [], [], np.zeros(nq, dtype=np.int64)
    for q in range(nq):
        if is_copy[q]:
            c, v = corpus.row(int(src[q]))
            v = v.astype(np.float64) * rng_j.lognormal(0.0, jitter_sigma, size=len(v))
            v = v / math.sqrt(float(np.dot(v, v)))
            rows_c.append(c.copy())
            rows_v.append(v.astype(np.float32))
        else:
            c, v = fresh.row(q)
            rows_c.append(c)
            rows_v.append(v)
        lens[q] = len(rows_c[-1])
    rp = np.zeros(nq + 1, dtype=np.int64)
    np.cumsum(lens, out=rp[1:])
    return Csr(nq, corpus.m, rp, np.concatenate(rows_c).astype(np.int32),
               np.concatenate(rows_v).astype(np.float32))


def from_rows(rows, m: int) -> Csr:
    """CSR from a list of {dim: weight} dicts or (dims, weights) pairs, used for tiny hand cases."""
    cols, vals, lens = [], [], []
    for r in rows:
        if isinstance(r, dict):
            items = sorted(r.items())
            d = [k for k, _ in items]
            w = [v for _, v in items]
        else:
            d, w = r
            o = np.argsort(d)
            d = list(np.asarray(d)[o])
            w = list(np.asarray(w)[o])
        cols.extend(d)
        vals.extend(w)
        lens.append(len(d))
    rp = np.zeros(len(rows) + 1, dtype=np.int64)
    np.cumsum(lens, out=rp[1:])
    return Csr(len(rows), m, rp, np.asarray(cols, dtype=np.int32), np.asarray(vals, dtype=np.float32))
