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
