"""The C-ABI library: loads, exports every declared symbol, argument checks (CPU only)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "apss.h")


def declared_symbols():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(apss_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    import paper_1402_3010_amd as apss
    lib = apss.load()
    syms = declared_symbols()
    assert len(syms) >= 12
    for s in syms:
        assert hasattr(lib, s), s
    assert set(syms) == set(apss.EXPORTED)


def test_strerror_and_opts():
    import paper_1402_3010_amd as apss
    assert apss.strerror(0) == "ok"
    assert apss.strerror(apss.APSS_ERANGE) == "output buffer too small"
    o = apss.default_opts()
    assert o.struct_size == ctypes.sizeof(apss.Opts)
    assert o.query_safe == 1


def test_argument_errors_before_device_work():
    import paper_1402_3010_amd as apss
    lib = apss.load()
    rp = np.array([0, 1], np.int64)
    col = np.array([0], np.int32)
    val = np.array([1.0], np.float32)
    h = ctypes.c_void_p()
    o = apss.default_opts()
    P = lambda a: a.ctypes.data
    assert lib.apss_build_index(1, 4, P(rp), P(col), P(val), 0, 0.0, ctypes.byref(o), ctypes.byref(h)) == apss.APSS_ETHRESH
    assert lib.apss_build_index(1, 4, P(rp), P(col), P(val), 0, 1.5, ctypes.byref(o), ctypes.byref(h)) == apss.APSS_ETHRESH
    assert lib.apss_build_index(-1, 4, P(rp), P(col), P(val), 0, 0.5, ctypes.byref(o), ctypes.byref(h)) == apss.APSS_EINVAL
    assert lib.apss_build_index(1, 0, P(rp), P(col), P(val), 0, 0.5, ctypes.byref(o), ctypes.byref(h)) == apss.APSS_EINVAL
    assert "m" in apss.last_error()
    bad = apss.Opts()
    bad.struct_size = 3
    assert lib.apss_build_index(1, 4, P(rp), P(col), P(val), 0, 0.5, ctypes.byref(bad), ctypes.byref(h)) == apss.APSS_EINVAL
    assert lib.apss_join(None, 0.5, None) == apss.APSS_EINVAL
    assert lib.apss_last_stats(None, None) == apss.APSS_EINVAL


def test_package_fails_loudly_without_library(tmp_path):
    import paper_1402_3010_amd as apss
    with pytest.raises(ImportError):
        apss._LIB, saved = None, apss._LIB
        try:
            apss.load(str(tmp_path / "missing.so"))
        finally:
            apss._LIB = saved


LAYOUT_PROBE = r"""
#include <stddef.h>
#include <stdio.h>
#include "apss.h"
#define F(T, f) printf(#T "." #f " %zu %zu\n", offsetof(T, f), sizeof(((T*)0)->f));
int main(void) {
  printf("apss_opts %zu\n", sizeof(apss_opts));
  printf("apss_pairs %zu\n", sizeof(apss_pairs));
  printf("apss_stats %zu\n", sizeof(apss_stats));
  printf("apss_server_opts %zu\n", sizeof(apss_server_opts));
  printf("apss_request_info %zu\n", sizeof(apss_request_info));
  printf("apss_server_counters %zu\n", sizeof(apss_server_counters));
  printf("apss_tune_result %zu\n", sizeof(apss_tune_result));
  F(apss_opts, stream) F(apss_opts, query_safe) F(apss_opts, variant) F(apss_opts, head_dims)
  F(apss_opts, range_rows) F(apss_opts, screen_dims) F(apss_opts, graph) F(apss_opts, index_all)
  F(apss_opts, local_parts) F(apss_opts, remscore) F(apss_opts, range_group) F(apss_opts, reserved)
  F(apss_server_opts, slots) F(apss_server_opts, max_batch_queries) F(apss_server_opts, memory_budget)
  F(apss_server_opts, pairs_per_query) F(apss_server_opts, max_pending) F(apss_server_opts, split_queries)
  F(apss_server_opts, reserved)
  F(apss_request_info, latency_ms) F(apss_request_info, batch) F(apss_request_info, batch_requests)
  F(apss_request_info, slot)
  F(apss_server_counters, running) F(apss_server_counters, submitted) F(apss_server_counters, peak_reserved_bytes)
  F(apss_server_counters, device_bytes)
  F(apss_stats, ms_candidates) F(apss_stats, ms_total) F(apss_stats, screen_rows) F(apss_stats, screen_ld)
  F(apss_stats, ms_screen)
  F(apss_tune_result, ms) F(apss_tune_result, from_cache) F(apss_tune_result, cache_write_failed)
  F(apss_tune_result, range_group)
  return 0;
}
"""


def test_struct_layouts_match_header(tmp_path):
    """The ctypes mirrors agree with the C structs (compiled against include/apss.h)."""
    import subprocess

    import paper_1402_3010_amd as apss
    src = tmp_path / "probe.c"
    src.write_text(LAYOUT_PROBE)
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    mirrors = {"apss_opts": apss.Opts, "apss_pairs": apss.Pairs, "apss_stats": apss.Stats,
               "apss_server_opts": apss.ServerOpts, "apss_request_info": apss.RequestInfo,
               "apss_server_counters": apss.ServerCounters, "apss_tune_result": apss.TuneResult}
    checked = 0
    for line in filter(None, out):
        parts = line.split()
        if len(parts) == 2:
            assert ctypes.sizeof(mirrors[parts[0]]) == int(parts[1]), line
        else:
            struct, field = parts[0].split(".")
            f = getattr(mirrors[struct], field)
            assert (f.offset, f.size) == (int(parts[1]), int(parts[2])), line
        checked += 1
    assert checked >= 25


def test_server_defaults_and_argument_errors():
    import paper_1402_3010_amd as apss
    lib = apss.load()
    o = apss.server_default_opts()
    assert o.struct_size == ctypes.sizeof(apss.ServerOpts)
    assert (o.slots, o.max_batch_queries, o.pairs_per_query, o.max_pending) == (2, 4096, 256, 4096)
    assert o.memory_budget == 4 << 30
    h = ctypes.c_void_p()
    assert lib.apss_server_create(None, ctypes.byref(o), ctypes.byref(h)) == apss.APSS_EINVAL
    rid = ctypes.c_uint64()
    rp = np.array([0, 1], np.int64)
    assert lib.apss_submit(None, 1, rp.ctypes.data, None, None, None, 0.5, ctypes.byref(rid)) == apss.APSS_EINVAL
    p = apss.Pairs()
    assert lib.apss_poll(None, 1, 0, ctypes.byref(p), None) == apss.APSS_EINVAL
    assert lib.apss_server_pause(None, 1) == apss.APSS_EINVAL
    c = apss.ServerCounters()
    assert lib.apss_server_stats(None, ctypes.byref(c)) == apss.APSS_EINVAL
    lib.apss_server_destroy(None)
    assert apss.strerror(apss.APSS_EBUSY) == "busy"
    assert apss.strerror(apss.APSS_PENDING) == "pending"


def test_variant_3_is_refused():
    """Variant 3 is withdrawn (refused before any device work), with or without the screen."""
    import paper_1402_3010_amd as apss
    lib = apss.load()
    rp = np.array([0, 1], np.int64)
    col = np.array([0], np.int32)
    val = np.array([1.0], np.float32)
    o = apss.default_opts(screen_dims=64, variant=3)
    h = ctypes.c_void_p()
    assert lib.apss_build_index(1, 4, rp.ctypes.data, col.ctypes.data, val.ctypes.data, 0, 0.5, ctypes.byref(o),
                                ctypes.byref(h)) == apss.APSS_EINVAL
    o = apss.default_opts(variant=3)
    assert lib.apss_build_index(1, 4, rp.ctypes.data, col.ctypes.data, val.ctypes.data, 0, 0.5, ctypes.byref(o),
                                ctypes.byref(h)) == apss.APSS_EINVAL
    assert "not available" in apss.last_error()
