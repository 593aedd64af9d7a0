"""GPU tests of the screened self-join (bf16 MFMA head screen + sparse pass
over the head-cut index): the output must equal the plain join's bit for
bit, and the oracle's within the band."""
import numpy as np
import pytest

import oracle
from synth.corpus import from_rows, make_corpus, spec_for
from tests.parity import assert_parity, exact_dot
from tests.test_oracle import load_golden

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def apss():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.init()
    import paper_1402_3010_amd as m
    m.load()
    return m


def join(apss, V, t, t_build=None, **kw):
    ix = apss.Index.build(V, np.float32(t if t_build is None else t_build), **kw)
    try:
        i, j, s = ix.join(np.float32(t))
        st = ix.stats()
    finally:
        ix.close()
    return i, j, s, st


def assert_identical(a, b):
    ai, aj, as_ = a[:3]
    bi, bj, bs = b[:3]
    assert len(ai) == len(bi), (len(ai), len(bi))
    assert np.array_equal(ai, bi) and np.array_equal(aj, bj)
    assert np.array_equal(as_.view(np.uint32), bs.view(np.uint32))


def test_golden_through_the_screen(apss):
    """Every dimension in the head: every pair is found by the MFMA screen,
    including the exact ties at t."""
    V, rank, mw, cases = load_golden()
    for c in cases:
        t = np.float32(c["t"])
        for sd in (V.m, 1, 3):
            i, j, s, st = join(apss, V, t, screen_dims=sd)
            assert list(zip(i.tolist(), j.tolist())) == [(a, b) for a, b, _ in c["pairs"]], (sd, c["t"])
            assert list(s) == [np.float32(x) for _, _, x in c["pairs"]]
        _, _, _, st = join(apss, V, t, screen_dims=V.m)
        nonempty = int(np.sum(np.diff(V.row_ptr) > 0))   # an empty row has head norm 0 < t
        assert st["screen_rows"] == nonempty and st["posting_visits"] == 0


@pytest.mark.parametrize("name,n,t,sd", [("c4", 20000, 0.8, 4096), ("c4", 20000, 0.6, 4096),
                                         ("c4", 20000, 0.8, 512), ("c1", None, 0.5, 64),
                                         ("c1", None, 0.5, 4096), ("c2", 15000, 0.7, 4096),
                                         ("c3", 12000, 0.7, 2048)])
def test_screened_equals_plain_and_oracle(apss, name, n, t, sd):
    V = make_corpus(spec_for(name, n=n))
    plain = join(apss, V, t)
    scr = join(apss, V, t, screen_dims=sd)
    assert_identical(plain, scr)
    st = scr[3]
    assert st["screen_ld"] == (min(sd, V.m) + 63) // 64 * 64
    assert st["matches"] == len(scr[0])
    assert_parity(scr[0], scr[1], scr[2], oracle.join_plain(V, np.float32(t)), float(np.float32(t)), V)


def test_screened_range_groups(apss):
    # the sparse pass with several ranges per work item (its tuned form at
    # full size): the plain join's pairs bit for bit
    V = make_corpus(spec_for("c4", n=20000))
    t = 0.8
    plain = join(apss, V, t)
    for kw in (dict(variant=2, range_rows=2048, range_group=4), dict(variant=1, range_rows=1024, range_group=3)):
        scr = join(apss, V, t, screen_dims=4096, **kw)
        assert_identical(plain, scr)


@pytest.mark.parametrize("variant,range_rows,sd,rg", [(2, 16384, 4096, 1), (1, 8192, 4096, 1), (2, 4096, 1024, 1),
                                                    (1, 4096, 1024, 2)])
def test_sparse_pass_wide_ranges(apss, variant, range_rows, sd, rg):
    # geometries where many ranges of the sparse pass hold more entries than
    # the hash table takes and go block by block, beside ranges that fit it:
    # the plain join's pairs bit for bit
    V = make_corpus(spec_for("c4", n=20000))
    t = 0.8
    plain = join(apss, V, t)
    scr = join(apss, V, t, screen_dims=sd, variant=variant, range_rows=range_rows, range_group=rg)
    assert_identical(plain, scr)
    assert_parity(scr[0], scr[1], scr[2], oracle.join_plain(V, np.float32(t)), float(np.float32(t)), V)


def test_screen_finds_pairs_with_no_tail_overlap(apss):
    """Near-duplicate rows that live almost entirely in the head: the
    matches must come from the MFMA screen (the sparse pass cannot see them)."""
    V = make_corpus(spec_for("c4", n=8000))
    rng = np.random.default_rng(5)
    cnt = np.bincount(V.col, minlength=V.m)
    head = np.argsort(-cnt, kind="stable")[:256]
    rows = []
    for _ in range(300):
        d = rng.choice(head, size=12, replace=False)
        w = rng.lognormal(0.0, 0.3, size=12)
        rows.append((d, w / np.sqrt(np.dot(w, w))))
        w2 = w * rng.lognormal(0.0, 0.02, size=12)      # a perturbed copy on the same dims
        rows.append((d, w2 / np.sqrt(np.dot(w2, w2))))
    base = [(V.row(k)[0], V.row(k)[1].astype(np.float64)) for k in range(V.n)]
    W = from_rows(base + rows, V.m)
    t = np.float32(0.95)
    plain = join(apss, W, t)
    scr = join(apss, W, t, screen_dims=512)
    assert_identical(plain, scr)
    st = scr[3]
    assert st["screen_candidates"] >= 280 and st["screen_tiles"] >= 1
    new_pairs = np.sum(scr[0] >= V.n)
    assert new_pairs >= 280
    for k in np.flatnonzero(scr[0] >= V.n)[:50]:
        assert abs(exact_dot(W, scr[0][k], scr[1][k]) - scr[2][k]) <= 1e-5


def test_screen_identical_vectors_and_empty_rows(apss):
    V = make_corpus(spec_for("c4", n=3000))
    idx = np.concatenate([np.arange(0, 3000), np.repeat(np.arange(0, 50), 3)])
    W = V.take_rows(idx)
    rows = [(W.row(k)[0], W.row(k)[1].astype(np.float64)) for k in range(W.n)] + [({})] * 5
    W = from_rows(rows, V.m)
    for t in (0.999, 1.0):
        assert_identical(join(apss, W, t), join(apss, W, t, screen_dims=4096))


def test_screen_dims_out_of_range(apss):
    V = make_corpus(spec_for("c1", n=100))
    with pytest.raises(apss.ApssError) as e:
        apss.Index.build(V, np.float32(0.5), screen_dims=8193)
    assert e.value.code == apss.APSS_EINVAL
