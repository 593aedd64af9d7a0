"""GPU test of the allocation-free self-join (apss_join_device_noalloc):
its output equals apss_join_device's bit for bit, and the oracle's within
the band, on two calls in a row, the second with a smaller input."""
import numpy as np
import pytest

import oracle
from synth.corpus import make_corpus, spec_for
from tests.parity import assert_parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def apss():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.init()
    import paper_1402_3010_amd as m
    m.load()
    return m


def buffers(n):
    import torch
    return (torch.empty(max(n, 1), dtype=torch.int32, device="cuda"),
            torch.empty(max(n, 1), dtype=torch.int32, device="cuda"),
            torch.empty(max(n, 1), dtype=torch.float32, device="cuda"))


def host(bufs, n):
    i, j, s = bufs
    return (i[:n].cpu().numpy().astype(np.uint32), j[:n].cpu().numpy().astype(np.uint32), s[:n].cpu().numpy())


def one_case(apss, V, t, **kw):
    t = np.float32(t)
    print("noalloc case n=%d t=%.2f %s" % (V.n, t, kw), flush=True)
    ix = apss.Index.build(V, t, on_device=True, **kw)
    try:
        ref_i, _, _ = ix.join(t)
        n = len(ref_i)
        a = buffers(n + 17)
        b = buffers(n + 17)
        ca = ix.join_device(t, *a)
        cb = ix.join_device_noalloc(t, *b)
        assert ca == cb == n
        st = ix.stats()
        assert st["matches"] == n and st["posting_visits"] > 0
        A, B = host(a, ca), host(b, cb)
        assert np.array_equal(A[0], B[0]) and np.array_equal(A[1], B[1])
        assert np.array_equal(A[2].view(np.uint32), B[2].view(np.uint32))
        # too small an output: the count needed comes back with APSS_ERANGE
        small = buffers(max(n // 3, 1))
        with pytest.raises(apss.ApssError) as e:
            ix.join_device_noalloc(t, *small)
        assert e.value.code == apss.APSS_ERANGE and e.value.count == n
    finally:
        ix.close()
    assert_parity(B[0], B[1], B[2], oracle.join_plain(V, t), float(t), V)
    return n


def test_noalloc_matches_join_device_two_calls(apss):
    big = make_corpus(spec_for("c2", n=21111))
    small = make_corpus(spec_for("c2", n=5000, seed=77))
    n1 = one_case(apss, big, 0.6)
    n2 = one_case(apss, small, 0.6)
    assert n1 > n2 > 0


def test_noalloc_with_range_groups(apss):
    # work items over several ranges use the same scratch layout
    big = make_corpus(spec_for("c2", n=21111))
    small = make_corpus(spec_for("c2", n=5000, seed=77))
    n1 = one_case(apss, big, 0.6, range_rows=2048, range_group=3)
    n2 = one_case(apss, small, 0.6, variant=2, range_rows=1024, range_group=4)
    assert n1 > n2 > 0


def test_noalloc_rejects_screened_index(apss):
    V = make_corpus(spec_for("c1", n=500))
    ix = apss.Index.build(V, np.float32(0.5), screen_dims=64)
    try:
        with pytest.raises(apss.ApssError) as e:
            ix.join_device_noalloc(np.float32(0.5), *buffers(10))
        assert e.value.code == apss.APSS_EINVAL
    finally:
        ix.close()
