"""CPU oracle for the all-pairs similarity join -- test infrastructure only.

Only the test suite, the GPU smoke check and the benchmark's CPU-baseline leg
may import this package.  The GPU library never does, and this package never
imports the GPU library.  The arithmetic lives in ``apss_oracle.c`` (double
precision, OpenMP over query rows); this module only marshals arrays.

Functions (each restates a passage of the paper, see apss_oracle.c):

* ``validate``      input checks of Section 2.1 (unit norm, positive weights).
* ``join_plain``    all-pairs-0-array: Algorithms 1 and 2 with a dense score
                    array (Section 4) -- the plain definition of the match set.
* ``join_prefix``   all-pairs-1 partial indexing (Section 3.2.2) with the
                    optional minsize / remscore / upperbound tests of
                    all-pairs-2.
* ``prefix_index``  dimension order, maxweight_i(V) and the unindexed-prefix
                    length of every vector (Section 3.2.2).
* ``query``         Find-Matches (Algorithm 2) for external query rows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "apss_oracle.c")
_LIB = None

FLAG_MINSIZE = 1
FLAG_UPPERBOUND = 2
FLAG_L2_CLAUSE = 4
FLAG_REMSCORE = 8


class _Result(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int64), ("i", ctypes.POINTER(ctypes.c_int64)),
                ("j", ctypes.POINTER(ctypes.c_int64)), ("s", ctypes.POINTER(ctypes.c_double)),
                ("visits", ctypes.c_int64), ("candidates", ctypes.c_int64), ("verified", ctypes.c_int64)]


@dataclass
class Pairs:
    i: np.ndarray        # int64
    j: np.ndarray        # int64
    s: np.ndarray        # float64
    visits: int = 0
    candidates: int = 0
    verified: int = 0

    def __len__(self):
        return len(self.i)

    def keys(self) -> np.ndarray:
        return self.i.astype(np.int64) * (1 << 32) + self.j.astype(np.int64)


def build() -> str:
    """Compile apss_oracle.c into liboracle.so (gcc -O2 -fopenmp)."""
    tmp = _SO + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _SO)
    return _SO


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_SO)
        i64, f64 = ctypes.c_int64, ctypes.c_double
        P = ctypes.c_void_p
        lib.oracle_validate.argtypes = [i64, i64, P, P, P, f64]
        lib.oracle_validate.restype = i64
        lib.oracle_join_plain.argtypes = [i64, i64, P, P, P, f64, i64, i64, ctypes.POINTER(_Result)]
        lib.oracle_join_plain.restype = ctypes.c_int
        lib.oracle_join_prefix.argtypes = [i64, i64, P, P, P, f64, ctypes.c_int, ctypes.POINTER(_Result)]
        lib.oracle_join_prefix.restype = ctypes.c_int
        lib.oracle_prefix_index.argtypes = [i64, i64, P, P, P, f64, ctypes.c_int, P, P, P]
        lib.oracle_prefix_index.restype = ctypes.c_int
        lib.oracle_query.argtypes = [i64, i64, P, P, P, i64, P, P, P, P, f64, ctypes.POINTER(_Result)]
        lib.oracle_query.restype = ctypes.c_int
        lib.oracle_result_free.argtypes = [ctypes.POINTER(_Result)]
        lib.oracle_result_free.restype = None
        lib.oracle_num_threads.argtypes = []
        lib.oracle_num_threads.restype = ctypes.c_int
        _LIB = lib
    return _LIB


def _arr(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(ctypes.c_void_p)


def _csr(V):
    rp, prp = _arr(V.row_ptr, np.int64)
    col, pcol = _arr(V.col, np.int32)
    val, pval = _arr(V.val, np.float32)
    return (rp, col, val), (prp, pcol, pval)


def _take(res: _Result) -> Pairs:
    c = res.count
    if c:
        i = np.ctypeslib.as_array(res.i, shape=(c,)).copy()
        j = np.ctypeslib.as_array(res.j, shape=(c,)).copy()
        s = np.ctypeslib.as_array(res.s, shape=(c,)).copy()
    else:
        i = np.zeros(0, np.int64)
        j = np.zeros(0, np.int64)
        s = np.zeros(0, np.float64)
    out = Pairs(i, j, s, res.visits, res.candidates, res.verified)
    _lib().oracle_result_free(ctypes.byref(res))
    return out


def num_threads() -> int:
    return int(_lib().oracle_num_threads())


def validate(V, norm_tol: float = 1e-5) -> int:
    """0 if V is a valid input, else 1 + the first offending row."""
    keep, p = _csr(V)
    return int(_lib().oracle_validate(V.n, V.m, *p, norm_tol))


def join_plain(V, t: float, i_begin: int = 0, i_end: int = 0) -> Pairs:
    """All (i, j), i < j, with dot(v_i, v_j) >= t; rows j in [i_begin, i_end) when i_end > 0."""
    keep, p = _csr(V)
    res = _Result()
    rc = _lib().oracle_join_plain(V.n, V.m, *p, float(t), int(i_begin), int(i_end), ctypes.byref(res))
    if rc:
        raise MemoryError("oracle_join_plain failed (%d)" % rc)
    return _take(res)


def join_prefix(V, t: float, flags: int = 0) -> Pairs:
    keep, p = _csr(V)
    res = _Result()
    rc = _lib().oracle_join_prefix(V.n, V.m, *p, float(t), int(flags), ctypes.byref(res))
    if rc:
        raise MemoryError("oracle_join_prefix failed (%d)" % rc)
    return _take(res)


def prefix_index(V, t: float, l2_clause: bool = True):
    """(rank[m], maxweight[m], cut[n]) of partial indexing at threshold t."""
    keep, p = _csr(V)
    rank = np.empty(V.m, np.int32)
    mw = np.empty(V.m, np.float32)
    cut = np.empty(max(V.n, 1), np.int32)
    rc = _lib().oracle_prefix_index(V.n, V.m, *p, float(t), int(bool(l2_clause)),
                                    rank.ctypes.data_as(ctypes.c_void_p), mw.ctypes.data_as(ctypes.c_void_p),
                                    cut.ctypes.data_as(ctypes.c_void_p))
    if rc:
        raise MemoryError("oracle_prefix_index failed (%d)" % rc)
    return rank, mw, cut[:V.n]


def query(V, Q, t: float = 0.0, t_per_row=None) -> Pairs:
    """All (q, y) with dot(Q_q, V_y) >= t_q (t_per_row[q] if given, else t)."""
    keep, p = _csr(V)
    qkeep, qp = _csr(Q)
    if t_per_row is not None:
        tq, ptq = _arr(t_per_row, np.float64)
    else:
        tq, ptq = None, None
    res = _Result()
    rc = _lib().oracle_query(V.n, V.m, *p, Q.n, *qp, ptq, float(t), ctypes.byref(res))
    if rc:
        raise MemoryError("oracle_query failed (%d)" % rc)
    return _take(res)
