"""Python binding of libapss.so: exact all-pairs similarity join on MI355X.

Argument marshalling only -- every step of the join runs in the library's
HIP kernels.  The functions carry the names of the C entry points
(``apss_build_index`` -> ``build_index`` and so on); ``Index`` wraps a
handle.  Inputs may be numpy arrays (host) or torch tensors on the GPU
(device); PyTorch is used for device memory and the current stream only.

The library must have been built (``python -m paper_1402_3010_amd.build`` or
``__graft_entry__.build()``).  Importing this package without it raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libapss.so")

APSS_OK = 0
APSS_EINVAL = 1
APSS_ETHRESH = 2
APSS_ENOMEM = 3
APSS_EDEVICE = 4
APSS_ERANGE = 5
APSS_EBUSY = 6
APSS_PENDING = 100
NOALLOC_SCRATCH_BYTES = 128 << 20  # APSS_NOALLOC_SCRATCH_BYTES of include/apss.h


class ApssError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("apss error %d (%s): %s" % (code, strerror(code) if _lib_ok() else "?", msg))
        self.code = code


class Opts(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_int32), ("stream", ctypes.c_void_p), ("query_safe", ctypes.c_int32),
                ("variant", ctypes.c_int32), ("head_dims", ctypes.c_int32), ("range_rows", ctypes.c_int32),
                ("screen_dims", ctypes.c_int32), ("graph", ctypes.c_int32), ("index_all", ctypes.c_int32),
                ("local_parts", ctypes.c_int32), ("remscore", ctypes.c_int32), ("range_group", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 4)]


class Pairs(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int64), ("i", ctypes.POINTER(ctypes.c_uint32)),
                ("j", ctypes.POINTER(ctypes.c_uint32)), ("sim", ctypes.POINTER(ctypes.c_float))]


class Stats(ctypes.Structure):
    _fields_ = [("posting_visits", ctypes.c_int64), ("candidates", ctypes.c_int64),
                ("bound_survivors", ctypes.c_int64), ("verified", ctypes.c_int64), ("band", ctypes.c_int64),
                ("matches", ctypes.c_int64), ("ms_candidates", ctypes.c_double), ("ms_total", ctypes.c_double),
                ("screen_rows", ctypes.c_int64), ("screen_tiles", ctypes.c_int64),
                ("screen_candidates", ctypes.c_int64), ("screen_ld", ctypes.c_int64), ("ms_screen", ctypes.c_double)]


SERVER_MAX_SLOTS = 8


class ServerOpts(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_int32), ("slots", ctypes.c_int32), ("max_batch_queries", ctypes.c_int64),
                ("memory_budget", ctypes.c_int64), ("pairs_per_query", ctypes.c_int64),
                ("max_pending", ctypes.c_int64), ("split_queries", ctypes.c_int64),
                ("reserved", ctypes.c_int32 * 6)]


class RequestInfo(ctypes.Structure):
    _fields_ = [("queue_ms", ctypes.c_double), ("service_ms", ctypes.c_double), ("latency_ms", ctypes.c_double),
                ("batch", ctypes.c_int64), ("batch_requests", ctypes.c_int32), ("slot", ctypes.c_int32)]


class ServerCounters(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int32), ("running", ctypes.c_int32)] + [
        (k, ctypes.c_int64) for k in ("submitted", "rejected_busy", "completed", "failed", "queued", "batches",
                                      "queries", "overlapped_batches", "peak_running", "regrows", "reserved_bytes",
                                      "peak_reserved_bytes")] + [("device_bytes", ctypes.c_int64 * SERVER_MAX_SLOTS)]


class TuneResult(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("range_rows", ctypes.c_int32), ("ms", ctypes.c_double),
                ("from_cache", ctypes.c_int32), ("tried", ctypes.c_int32), ("cache_write_failed", ctypes.c_int32),
                ("range_group", ctypes.c_int32), ("reserved", ctypes.c_int32 * 2)]


_LIB = None


def _lib_ok() -> bool:
    return _LIB is not None


def load(path: str = LIB_PATH):
    """Load libapss.so; raises if it has not been built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise ImportError("libapss.so not built at %s; run __graft_entry__.build()" % path)
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i64 = ctypes.c_int64
    f32 = ctypes.c_float
    lib.apss_default_opts.argtypes = [ctypes.POINTER(Opts)]
    lib.apss_default_opts.restype = None
    lib.apss_build_index.argtypes = [i64, i64, P, P, P, ctypes.c_int, f32, ctypes.POINTER(Opts),
                                     ctypes.POINTER(ctypes.c_void_p)]
    lib.apss_build_index.restype = ctypes.c_int
    lib.apss_index_free.argtypes = [P]
    lib.apss_index_free.restype = None
    lib.apss_join_device.argtypes = [P, f32, P, P, P, i64, ctypes.POINTER(i64)]
    lib.apss_join_device.restype = ctypes.c_int
    lib.apss_join_device_noalloc.argtypes = [P, f32, P, P, P, i64, ctypes.POINTER(i64)]
    lib.apss_join_device_noalloc.restype = ctypes.c_int
    # test hook outside the ABI header: the screen's raw head products
    lib.apss_probe_screen_products.argtypes = [P, P, i64, P, P]
    lib.apss_probe_screen_products.restype = ctypes.c_int
    lib.apss_join.argtypes = [P, f32, ctypes.POINTER(Pairs)]
    lib.apss_join.restype = ctypes.c_int
    lib.apss_query.argtypes = [P, i64, P, P, P, ctypes.c_int, P, f32, ctypes.POINTER(Pairs)]
    lib.apss_query.restype = ctypes.c_int
    lib.apss_query_device.argtypes = [P, i64, P, P, P, ctypes.c_int, P, f32, P, P, P, i64, ctypes.POINTER(i64)]
    lib.apss_query_device.restype = ctypes.c_int
    lib.apss_pairs_free.argtypes = [ctypes.POINTER(Pairs)]
    lib.apss_pairs_free.restype = None
    lib.apss_last_stats.argtypes = [P, ctypes.POINTER(Stats)]
    lib.apss_last_stats.restype = ctypes.c_int
    lib.apss_index_export.argtypes = [P, P, P, P]
    lib.apss_index_export.restype = ctypes.c_int
    lib.apss_index_sizes.argtypes = [P, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64),
                                     ctypes.POINTER(i64)]
    lib.apss_index_sizes.restype = ctypes.c_int
    lib.apss_strerror.argtypes = [ctypes.c_int]
    lib.apss_strerror.restype = ctypes.c_char_p
    lib.apss_last_error.argtypes = []
    lib.apss_last_error.restype = ctypes.c_char_p
    lib.apss_autotune.argtypes = [P, f32, ctypes.c_double, ctypes.c_char_p, ctypes.POINTER(TuneResult)]
    lib.apss_autotune.restype = ctypes.c_int
    lib.apss_server_default_opts.argtypes = [ctypes.POINTER(ServerOpts)]
    lib.apss_server_default_opts.restype = None
    lib.apss_server_create.argtypes = [P, ctypes.POINTER(ServerOpts), ctypes.POINTER(ctypes.c_void_p)]
    lib.apss_server_create.restype = ctypes.c_int
    lib.apss_submit.argtypes = [P, i64, P, P, P, P, f32, ctypes.POINTER(ctypes.c_uint64)]
    lib.apss_submit.restype = ctypes.c_int
    lib.apss_poll.argtypes = [P, ctypes.c_uint64, ctypes.c_int, ctypes.POINTER(Pairs), ctypes.POINTER(RequestInfo)]
    lib.apss_poll.restype = ctypes.c_int
    lib.apss_server_pause.argtypes = [P, ctypes.c_int]
    lib.apss_server_pause.restype = ctypes.c_int
    lib.apss_server_stats.argtypes = [P, ctypes.POINTER(ServerCounters)]
    lib.apss_server_stats.restype = ctypes.c_int
    lib.apss_server_destroy.argtypes = [P]
    lib.apss_server_destroy.restype = None
    _LIB = lib
    return lib


EXPORTED = ("apss_default_opts", "apss_build_index", "apss_index_free", "apss_join_device",
            "apss_join_device_noalloc", "apss_join",
            "apss_query", "apss_query_device", "apss_pairs_free", "apss_last_stats", "apss_index_export",
            "apss_index_sizes", "apss_strerror", "apss_last_error", "apss_autotune", "apss_server_default_opts",
            "apss_server_create", "apss_submit", "apss_poll", "apss_server_pause", "apss_server_stats",
            "apss_server_destroy")


def strerror(code: int) -> str:
    return load().apss_strerror(code).decode()


def last_error() -> str:
    return load().apss_last_error().decode()


def _check(rc: int):
    if rc != APSS_OK:
        raise ApssError(rc, last_error())


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _csr_args(row_ptr, col, val):
    """(pointers, on_device, keepalive) for numpy host arrays or torch GPU tensors."""
    if _is_torch(row_ptr):
        import torch
        assert row_ptr.dtype == torch.int64 and col.dtype == torch.int32 and val.dtype == torch.float32
        assert row_ptr.is_contiguous() and col.is_contiguous() and val.is_contiguous()
        on_dev = 1 if row_ptr.is_cuda else 0
        return (row_ptr.data_ptr(), col.data_ptr(), val.data_ptr()), on_dev, (row_ptr, col, val)
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    c = np.ascontiguousarray(col, dtype=np.int32)
    v = np.ascontiguousarray(val, dtype=np.float32)
    return (rp.ctypes.data, c.ctypes.data, v.ctypes.data), 0, (rp, c, v)


def current_stream_handle() -> Optional[int]:
    try:
        import torch
        if torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
    except Exception:
        pass
    return None


def default_opts(stream=None, query_safe: bool = True, head_dims: int = 0, variant: int = -1,
                 range_rows: int = 0, screen_dims: int = 0, graph: bool = False, index_all: bool = False,
                 local_parts: int = 0, remscore: bool = False, range_group: int = 0) -> Opts:
    o = Opts()
    load().apss_default_opts(ctypes.byref(o))
    o.stream = stream
    o.query_safe = 1 if query_safe else 0
    o.head_dims = head_dims
    o.variant = variant
    o.range_rows = range_rows
    o.screen_dims = screen_dims
    o.graph = 1 if graph else 0
    o.index_all = 1 if index_all else 0
    o.local_parts = local_parts
    o.remscore = 1 if remscore else 0
    o.range_group = range_group
    return o


def _take_pairs(p: Pairs):
    c = p.count
    if c:
        i = np.ctypeslib.as_array(p.i, shape=(c,)).copy()
        j = np.ctypeslib.as_array(p.j, shape=(c,)).copy()
        s = np.ctypeslib.as_array(p.sim, shape=(c,)).copy()
    else:
        i = np.zeros(0, np.uint32)
        j = np.zeros(0, np.uint32)
        s = np.zeros(0, np.float32)
    load().apss_pairs_free(ctypes.byref(p))
    return i, j, s


def build_index(n: int, m: int, row_ptr, col, val, t_build: float, opts: Optional[Opts] = None) -> int:
    """apss_build_index; returns the raw handle."""
    lib = load()
    ptrs, on_dev, keep = _csr_args(row_ptr, col, val)
    h = ctypes.c_void_p()
    o = opts if opts is not None else default_opts(current_stream_handle())
    _check(lib.apss_build_index(int(n), int(m), *ptrs, on_dev, float(t_build), ctypes.byref(o), ctypes.byref(h)))
    del keep
    return h.value


def index_free(h: int):
    load().apss_index_free(h)


def join(h: int, t: float):
    p = Pairs()
    _check(load().apss_join(h, float(t), ctypes.byref(p)))
    return _take_pairs(p)


def join_device(h: int, t: float, out_i, out_j, out_sim) -> int:
    """Pairs into caller tensors (uint32/int32 ids, float32 sims); returns the count.

    Raises ApssError(APSS_ERANGE) carrying the count needed if they are too small.
    """
    cnt = ctypes.c_int64()
    rc = load().apss_join_device(h, float(t), out_i.data_ptr(), out_j.data_ptr(), out_sim.data_ptr(),
                                 int(out_i.numel()), ctypes.byref(cnt))
    if rc == APSS_ERANGE:
        e = ApssError(rc, last_error())
        e.count = cnt.value
        raise e
    _check(rc)
    return cnt.value


def join_device_noalloc(h: int, t: float, out_i, out_j, out_sim) -> int:
    """apss_join_device_noalloc: join_device with every scratch buffer in the
    library's fixed device array (no allocation during the call)."""
    cnt = ctypes.c_int64()
    rc = load().apss_join_device_noalloc(h, float(t), out_i.data_ptr(), out_j.data_ptr(), out_sim.data_ptr(),
                                         int(out_i.numel()), ctypes.byref(cnt))
    if rc in (APSS_ERANGE, APSS_ENOMEM):
        e = ApssError(rc, last_error())
        e.count = cnt.value
        raise e
    _check(rc)
    return cnt.value


def probe_screen_products(h: int, rows):
    """Test hook (not part of include/apss.h): the bf16 MFMA screen's float
    head products H~ of the given rows (S x S, upper triangle) and their
    rounded-up head norms, on an index built with screen_dims > 0."""
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    S = len(rows)
    H = np.zeros((S, S), np.float32)
    N = np.zeros(S, np.float32)
    _check(load().apss_probe_screen_products(h, rows.ctypes.data, S, H.ctypes.data, N.ctypes.data))
    return H, N


def _query_args(Q_row_ptr, Q_col, Q_val, t_per_row):
    ptrs, on_dev, keep = _csr_args(Q_row_ptr, Q_col, Q_val)
    if t_per_row is not None:
        tq = np.ascontiguousarray(t_per_row, dtype=np.float32)
        return ptrs, on_dev, keep, tq, tq.ctypes.data
    return ptrs, on_dev, keep, None, None


def query(h: int, nq: int, q_row_ptr, q_col, q_val, t: float = 0.0, t_per_row=None):
    ptrs, on_dev, keep, tq, ptq = _query_args(q_row_ptr, q_col, q_val, t_per_row)
    p = Pairs()
    _check(load().apss_query(h, int(nq), *ptrs, on_dev, ptq, float(t), ctypes.byref(p)))
    return _take_pairs(p)


def query_device(h: int, nq: int, q_row_ptr, q_col, q_val, out_i, out_j, out_sim, t: float = 0.0,
                 t_per_row=None) -> int:
    ptrs, on_dev, keep, tq, ptq = _query_args(q_row_ptr, q_col, q_val, t_per_row)
    cnt = ctypes.c_int64()
    rc = load().apss_query_device(h, int(nq), *ptrs, on_dev, ptq, float(t), out_i.data_ptr(), out_j.data_ptr(),
                                  out_sim.data_ptr(), int(out_i.numel()), ctypes.byref(cnt))
    if rc == APSS_ERANGE:
        e = ApssError(rc, last_error())
        e.count = cnt.value
        raise e
    _check(rc)
    return cnt.value


def last_stats(h: int) -> dict:
    s = Stats()
    _check(load().apss_last_stats(h, ctypes.byref(s)))
    return {k: getattr(s, k) for k, _ in Stats._fields_}


def autotune(h: int, t: float, budget_ms: float = 0.0, cache: Optional[str] = None) -> dict:
    r = TuneResult()
    _check(load().apss_autotune(h, float(t), float(budget_ms), cache.encode() if cache else None, ctypes.byref(r)))
    return {k: getattr(r, k) for k, _ in TuneResult._fields_ if k != "reserved"}


def index_sizes(h: int) -> dict:
    v = [ctypes.c_int64() for _ in range(4)]
    _check(load().apss_index_sizes(h, *[ctypes.byref(x) for x in v]))
    return dict(n=v[0].value, m=v[1].value, nnz=v[2].value, postings=v[3].value)


def index_export(h: int):
    sz = index_sizes(h)
    rank = np.empty(sz["m"], np.int32)
    mw = np.empty(sz["m"], np.float32)
    cut = np.empty(max(sz["n"], 1), np.int32)
    _check(load().apss_index_export(h, rank.ctypes.data, mw.ctypes.data, cut.ctypes.data))
    return rank, mw, cut[:sz["n"]]


@dataclass
class Index:
    """Owning wrapper of an apss_index handle."""
    handle: int
    n: int
    m: int

    @classmethod
    def build(cls, V, t_build: float, stream=None, query_safe: bool = True, head_dims: int = 0,
              on_device: bool = False, variant: int = -1, range_rows: int = 0, screen_dims: int = 0,
              graph: bool = False, index_all: bool = False, local_parts: int = 0,
              remscore: bool = False, range_group: int = 0) -> "Index":
        """V: object with n, m, row_ptr, col, val (numpy), or a tuple (n, m, row_ptr, col, val) of tensors."""
        if isinstance(V, tuple):
            n, m, rp, col, val = V
        else:
            n, m, rp, col, val = V.n, V.m, V.row_ptr, V.col, V.val
        if on_device and not _is_torch(rp):
            import torch
            rp = torch.from_numpy(np.ascontiguousarray(rp, np.int64)).cuda()
            col = torch.from_numpy(np.ascontiguousarray(col, np.int32)).cuda()
            val = torch.from_numpy(np.ascontiguousarray(val, np.float32)).cuda()
        if stream is None:
            stream = current_stream_handle()
        h = build_index(n, m, rp, col, val, t_build, default_opts(stream, query_safe, head_dims, variant, range_rows,
                                                                      screen_dims, graph, index_all, local_parts,
                                                                      remscore, range_group))
        return cls(h, int(n), int(m))

    def join(self, t: float):
        return join(self.handle, t)

    def join_device(self, t: float, out_i, out_j, out_sim) -> int:
        return join_device(self.handle, t, out_i, out_j, out_sim)

    def join_device_noalloc(self, t: float, out_i, out_j, out_sim) -> int:
        return join_device_noalloc(self.handle, t, out_i, out_j, out_sim)

    def query(self, Q, t: float = 0.0, t_per_row=None):
        return query(self.handle, Q.n, Q.row_ptr, Q.col, Q.val, t, t_per_row)

    def query_device(self, Q, out_i, out_j, out_sim, t: float = 0.0, t_per_row=None) -> int:
        return query_device(self.handle, Q.n, Q.row_ptr, Q.col, Q.val, out_i, out_j, out_sim, t, t_per_row)

    def stats(self) -> dict:
        return last_stats(self.handle)

    def autotune(self, t: float, budget_ms: float = 0.0, cache: Optional[str] = None) -> dict:
        """apss_autotune: pick the tile variant and range width for joins at t (see the header)."""
        return autotune(self.handle, t, budget_ms, cache)

    def export(self):
        return index_export(self.handle)

    def sizes(self) -> dict:
        return index_sizes(self.handle)

    def close(self):
        if self.handle:
            index_free(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- serving ----

def server_default_opts(**kw) -> ServerOpts:
    o = ServerOpts()
    load().apss_server_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def server_create(index_handle: int, opts: Optional[ServerOpts] = None) -> int:
    h = ctypes.c_void_p()
    o = opts if opts is not None else server_default_opts()
    _check(load().apss_server_create(index_handle, ctypes.byref(o), ctypes.byref(h)))
    return h.value


def submit(server_handle: int, nq: int, q_row_ptr, q_col, q_val, t: float = 0.0, t_per_row=None) -> int:
    """apss_submit with host arrays; returns the request id (raises ApssError, code APSS_EBUSY when not admitted)."""
    rp = np.ascontiguousarray(q_row_ptr, dtype=np.int64)
    c = np.ascontiguousarray(q_col, dtype=np.int32)
    v = np.ascontiguousarray(q_val, dtype=np.float32)
    tq = None if t_per_row is None else np.ascontiguousarray(t_per_row, dtype=np.float32)
    rid = ctypes.c_uint64()
    _check(load().apss_submit(server_handle, int(nq), rp.ctypes.data, c.ctypes.data, v.ctypes.data,
                              None if tq is None else tq.ctypes.data, float(t), ctypes.byref(rid)))
    return rid.value


def poll(server_handle: int, req_id: int, timeout_ms: int = -1):
    """apss_poll: None while pending, else (i, j, sim, info dict)."""
    p = Pairs()
    info = RequestInfo()
    rc = load().apss_poll(server_handle, ctypes.c_uint64(req_id), int(timeout_ms), ctypes.byref(p),
                          ctypes.byref(info))
    if rc == APSS_PENDING:
        return None
    _check(rc)
    i, j, s = _take_pairs(p)
    return i, j, s, {k: getattr(info, k) for k, _ in RequestInfo._fields_}


def server_stats(server_handle: int) -> dict:
    c = ServerCounters()
    _check(load().apss_server_stats(server_handle, ctypes.byref(c)))
    d = {k: getattr(c, k) for k, _ in ServerCounters._fields_ if k != "device_bytes"}
    d["device_bytes"] = list(c.device_bytes)[:c.slots]
    return d


def server_destroy(server_handle: int):
    load().apss_server_destroy(server_handle)


class Server:
    """Owning wrapper of an apss_server attached to an Index (which must stay open)."""

    def __init__(self, index: Index, **opts):
        self.index = index
        self.handle = server_create(index.handle, server_default_opts(**opts))

    def submit(self, Q, t: float = 0.0, t_per_row=None) -> int:
        return submit(self.handle, Q.n, Q.row_ptr, Q.col, Q.val, t, t_per_row)

    def try_submit(self, Q, t: float = 0.0, t_per_row=None) -> Optional[int]:
        """Like submit, but None when the server refuses with APSS_EBUSY."""
        try:
            return self.submit(Q, t, t_per_row)
        except ApssError as e:
            if e.code == APSS_EBUSY:
                return None
            raise

    def poll(self, req_id: int, timeout_ms: int = -1):
        return poll(self.handle, req_id, timeout_ms)

    def pause(self, paused: bool = True):
        _check(load().apss_server_pause(self.handle, 1 if paused else 0))

    def stats(self) -> dict:
        return server_stats(self.handle)

    def close(self):
        if self.handle:
            server_destroy(self.handle)
            self.handle = 0

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
