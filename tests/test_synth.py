"""Input generator: shapes, determinism and the stated distributions."""
import numpy as np

from synth.corpus import CorpusSpec, make_corpus, spec_for, from_rows


def test_deterministic_and_valid():
    s = spec_for("c1")
    a = make_corpus(s)
    b = make_corpus(s)
    assert np.array_equal(a.row_ptr, b.row_ptr)
    assert np.array_equal(a.col, b.col)
    assert np.array_equal(a.val, b.val)
    lens = np.diff(a.row_ptr)
    assert lens.min() >= 10 and lens.max() <= 60
    rows = np.repeat(np.arange(a.n), lens)
    nrm = np.sqrt(np.bincount(rows, weights=a.val.astype(np.float64) ** 2))
    assert np.abs(nrm - 1).max() < 1e-6
    assert (a.val > 0).all()
    # dims strictly ascending inside rows (so distinct)
    d = np.diff(a.col.astype(np.int64))
    inner = np.ones(len(d), bool)
    inner[a.row_ptr[1:-1] - 1] = False
    assert (d[inner] > 0).all()
    c = make_corpus(spec_for("c1", seed=7))
    assert not np.array_equal(a.col, c.col)


def test_zipf_popularity():
    # s = 1.0 over m dims: with few draws per row and many rows the count of the
    # k-th most popular dimension is close to n * (1 - (1 - p_k)^L) for p_k ~ 1/(k H_m).
    s = CorpusSpec(20000, 1000, "uniform", 10, 10, 10, 10, 1.0, 5)
    c = make_corpus(s)
    cnt = np.sort(np.bincount(c.col, minlength=c.m))[::-1]
    H = np.sum(1.0 / np.arange(1, c.m + 1))
    # rejection of repeats changes the law slightly for the head; check the tail ratio
    ratio = cnt[99] / cnt[199]
    assert 1.7 < ratio < 2.3
    assert cnt[0] > 0.5 * c.n
    assert abs(cnt[499] / (c.n * 10 / (500 * H)) - 1) < 0.3


def test_lognormal_mean():
    c = make_corpus(spec_for("c2", n=20000))
    lens = np.diff(c.row_ptr)
    assert 70 < lens.mean() < 90
    assert lens.min() >= 5 and lens.max() <= 2000


def test_from_rows():
    v = from_rows([{3: 0.6, 1: 0.8}, ([5, 2], [1.0, 0.0])], m=8)
    assert list(v.col) == [1, 3, 2, 5]
    assert np.allclose(v.val, [0.8, 0.6, 0.0, 1.0])
