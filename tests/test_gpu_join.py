"""GPU parity: the HIP join against the CPU oracle, through the C ABI."""
import numpy as np
import pytest

import oracle
from synth.corpus import CorpusSpec, Csr, from_rows, make_corpus, spec_for
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


def gpu_join(apss, V, t, t_build=None, **kw):
    ix = apss.Index.build(V, t if t_build is None else t_build, **kw)
    try:
        i, j, s = ix.join(t)
        st = ix.stats()
    finally:
        ix.close()
    return i, j, s, st


# ---------------------------------------------------------------- exact fixtures


def test_golden_dyadic(apss):
    V, rank, mw, cases = load_golden()
    for c in cases:
        t = np.float32(c["t"])
        i, j, s, _ = gpu_join(apss, V, t)
        assert list(zip(i.tolist(), j.tolist())) == [(a, b) for a, b, _ in c["pairs"]]
        assert list(s) == [np.float32(x) for _, _, x in c["pairs"]]
        ix = apss.Index.build(V, t)
        r, w, cut = ix.export()
        ix.close()
        assert list(r) == rank and list(w) == mw and list(cut) == c["cut_l2"]
        ix = apss.Index.build(V, t, query_safe=False)
        _, _, cut2 = ix.export()
        ix.close()
        assert list(cut2) == c["cut"]


@pytest.mark.parametrize("name,n,t", [("c1", None, 0.5), ("c2", 20000, 0.7), ("c3", 20000, 0.7)])
def test_index_matches_oracle(apss, name, n, t):
    V = make_corpus(spec_for(name, n=n))
    t = np.float32(t)
    for qs in (True, False):
        ix = apss.Index.build(V, t, query_safe=qs)
        r, w, cut = ix.export()
        sizes = ix.sizes()
        ix.close()
        orank, omw, ocut = oracle.prefix_index(V, t, l2_clause=qs)
        assert np.array_equal(r, orank)
        assert np.array_equal(w, omw)
        assert np.array_equal(cut, ocut)
        assert sizes["postings"] == V.nnz - int(ocut.sum())


# ---------------------------------------------------------------- joins


@pytest.mark.parametrize("t", [0.3, 0.5, 0.7, 0.9])
def test_c1_join(apss, t):
    V = make_corpus(spec_for("c1"))
    t = np.float32(t)
    i, j, s, st = gpu_join(apss, V, t)
    ref = oracle.join_plain(V, t)
    assert_parity(i, j, s, ref, float(t), V)
    assert st["matches"] == len(i)
    assert st["candidates"] >= st["bound_survivors"] >= st["verified"] >= st["matches"]


@pytest.mark.parametrize("t", [0.5, 0.7, 0.9])
def test_c2_subset_join(apss, t):
    # several tiles and corpus blocks, ragged last block
    V = make_corpus(spec_for("c2", n=21111))
    t = np.float32(t)
    i, j, s, st = gpu_join(apss, V, t)
    ref = oracle.join_plain(V, t)
    assert_parity(i, j, s, ref, float(t), V)
    # candidates equal the pairs sharing an indexed dimension of the earlier vector
    pre = oracle.join_prefix(V, t, 4)
    assert st["candidates"] == pre.candidates


def test_c3_shape_subset(apss):
    V = make_corpus(spec_for("c3", n=30000))
    t = np.float32(0.7)
    i, j, s, _ = gpu_join(apss, V, t)
    assert_parity(i, j, s, oracle.join_plain(V, t), float(t), V)


def test_join_above_build_threshold(apss):
    V = make_corpus(spec_for("c2", n=5000))
    ix = apss.Index.build(V, np.float32(0.5))
    try:
        for t in (0.5, 0.6, 0.8):
            t = np.float32(t)
            i, j, s = ix.join(t)
            assert_parity(i, j, s, oracle.join_plain(V, t), float(t), V)
        with pytest.raises(apss.ApssError) as e:
            ix.join(np.float32(0.4))
        assert e.value.code == apss.APSS_ETHRESH
    finally:
        ix.close()


def test_deterministic(apss):
    V = make_corpus(spec_for("c2", n=8000))
    a = gpu_join(apss, V, np.float32(0.6))
    b = gpu_join(apss, V, np.float32(0.6))
    for x, y in zip(a[:3], b[:3]):
        assert np.array_equal(x, y)


# ---------------------------------------------------------------- edge cases


def test_edge_empty_and_degenerate(apss):
    # no vectors at all
    V = Csr(0, 10, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.float32))
    i, j, s, _ = gpu_join(apss, V, 0.5)
    assert len(i) == 0
    # only empty rows
    V = Csr(5, 10, np.zeros(6, np.int64), np.zeros(0, np.int32), np.zeros(0, np.float32))
    assert len(gpu_join(apss, V, 0.5)[0]) == 0
    # one vector
    V = from_rows([{3: 1.0}], 10)
    assert len(gpu_join(apss, V, 0.5)[0]) == 0


def test_edge_identical_vectors_t1(apss):
    base = make_corpus(spec_for("c1", n=1))
    row = dict(zip(base.row(0)[0].tolist(), base.row(0)[1].tolist()))
    V = from_rows([row] * 3000, base.m)     # every pair has sim ~ 1, spans two blocks
    t = np.float32(0.999)
    i, j, s, _ = gpu_join(apss, V, t)
    assert len(i) == 3000 * 2999 // 2
    assert np.abs(s - 1.0).max() < 1e-5
    # dyadic rows: every similarity is exactly 1, so t = 1 keeps every pair
    V = from_rows([{1: 0.5, 5: 0.5, 9: 0.5, 13: 0.5}] * 2100 + [{2: 1.0}], 16)
    i, j, s, _ = gpu_join(apss, V, np.float32(1.0))
    assert len(i) == 2100 * 2099 // 2
    assert (s == 1.0).all()
    ref = oracle.join_plain(V, 1.0)
    assert len(ref) == len(i)


def test_edge_long_rows_and_dense_dim(apss):
    # a few rows with 5000 components among short rows; one dimension in every row
    rng = np.random.default_rng(5)
    m = 20000
    rows = []
    for r in range(4000):
        k = 5000 if r % 997 == 0 else int(rng.integers(5, 40))
        d = rng.choice(np.arange(1, m), size=k - 1, replace=False)
        w = rng.lognormal(size=k)
        dims = np.concatenate([[0], d])
        w = w / np.sqrt(np.sum(w * w))
        rows.append((dims, w.astype(np.float32)))
    V = from_rows(rows, m)
    # renormalise in float64 -> float32 rounding keeps |norm-1| tiny
    for t in (0.2, 0.5):
        t = np.float32(t)
        i, j, s, _ = gpu_join(apss, V, t)
        assert_parity(i, j, s, oracle.join_plain(V, t), float(t), V)


def test_edge_invalid_inputs(apss):
    dup = Csr(1, 4, np.array([0, 2]), np.array([1, 1], np.int32), np.array([0.6, 0.8], np.float32))
    bad_norm = from_rows([{0: 0.5}], 4)
    neg = from_rows([{0: -1.0}], 4)
    out = Csr(1, 4, np.array([0, 1]), np.array([7], np.int32), np.array([1.0], np.float32))
    for V in (dup, bad_norm, neg, out):
        with pytest.raises(apss.ApssError) as e:
            apss.Index.build(V, 0.5)
        assert e.value.code == apss.APSS_EINVAL
    # the same checks on device pointers
    with pytest.raises(apss.ApssError) as e:
        apss.Index.build(out, 0.5, on_device=True)
    assert e.value.code == apss.APSS_EINVAL


def test_device_output_and_erange(apss):
    import torch
    V = make_corpus(spec_for("c1"))
    t = np.float32(0.5)
    ix = apss.Index.build(V, t, on_device=True)
    try:
        ref_i, ref_j, ref_s = ix.join(t)
        n = len(ref_i)
        small = [torch.empty(max(n // 2, 1), dtype=torch.int32, device="cuda") for _ in range(2)]
        sim = torch.empty(max(n // 2, 1), dtype=torch.float32, device="cuda")
        with pytest.raises(apss.ApssError) as e:
            ix.join_device(t, small[0], small[1], sim)
        assert e.value.code == apss.APSS_ERANGE and e.value.count == n
        oi = torch.empty(n, dtype=torch.int32, device="cuda")
        oj = torch.empty(n, dtype=torch.int32, device="cuda")
        os_ = torch.empty(n, dtype=torch.float32, device="cuda")
        c = ix.join_device(t, oi, oj, os_)
        assert c == n
        assert np.array_equal(oi.cpu().numpy().astype(np.uint32), ref_i)
        assert np.array_equal(oj.cpu().numpy().astype(np.uint32), ref_j)
        assert np.array_equal(os_.cpu().numpy(), ref_s)
    finally:
        ix.close()


# ---------------------------------------------------------------- external queries


def test_query_per_row_thresholds(apss):
    V = make_corpus(spec_for("c2", n=12000))
    Qf = make_corpus(CorpusSpec(300, V.m, "lognormal", 80, 1.0, 5, 2000, 1.1, 4242))
    Qc = V.take_rows(np.arange(0, 12000, 97))
    rows = [dict(zip(*[a.tolist() for a in Q.row(k)])) for Q in (Qf, Qc) for k in range(Q.n)]
    Q = from_rows(rows, V.m)
    rng = np.random.default_rng(1)
    tq = rng.uniform(0.5, 0.95, size=Q.n).astype(np.float32)
    ix = apss.Index.build(V, np.float32(0.5))
    try:
        i, j, s = ix.query(Q, t_per_row=tq)
    finally:
        ix.close()
    ref = oracle.query(V, Q, t_per_row=tq.astype(np.float64))
    assert_parity(i, j, s, ref, None, Q, V, per_row_t=tq.astype(np.float64))
    assert len(ref) >= Qc.n


def test_query_needs_query_safe_index(apss):
    V = make_corpus(spec_for("c1", n=500))
    ix = apss.Index.build(V, np.float32(0.5), query_safe=False)
    try:
        with pytest.raises(apss.ApssError) as e:
            ix.query(V.take_rows(np.arange(5)), t=0.5)
        assert e.value.code == apss.APSS_EINVAL
    finally:
        ix.close()


# ---------------------------------------------------------------- full size, sampled


@pytest.mark.parametrize("name,t", [("c2", 0.5), ("c2", 0.9), ("c3", 0.7)])
def test_full_size_sampled(apss, name, t):
    """Full-size corpus in the benchmark's launch configuration; the oracle
    recomputes the matches of a sample of rows (all their earlier partners)."""
    V = make_corpus(spec_for(name))
    t = np.float32(t)
    i, j, s, st = gpu_join(apss, V, t)
    lo, hi = V.n - 300, V.n
    ref = oracle.join_plain(V, t, lo, hi)
    sel = (j >= lo) & (j < hi)
    assert_parity(i[sel], j[sel], s[sel], ref, float(t), V)
    # a sample of reported pairs anywhere: exact similarity above t - band
    rng = np.random.default_rng(0)
    for k in rng.integers(0, len(i), size=min(2000, len(i))):
        d = exact_dot(V, i[k], j[k])
        assert d >= float(t) - 1e-5 and abs(d - s[k]) <= 1e-5
    assert st["matches"] == len(i)


@pytest.mark.parametrize("variant", [0, 1, 2, pytest.param(3, marks=pytest.mark.skip(
    reason="variant 3 is withdrawn: it faulted the GPU (memory aperture violation) in two tuning runs on the "
           "500k-vector workloads, cause not yet identified"))])
def test_every_tile_variant(apss, variant):
    V = make_corpus(spec_for("c2", n=9000))
    t = np.float32(0.6)
    i, j, s, st = gpu_join(apss, V, t, variant=variant)
    assert_parity(i, j, s, oracle.join_plain(V, t), float(t), V)
    pre = oracle.join_prefix(V, t, 4)
    assert st["candidates"] == pre.candidates


@pytest.mark.parametrize("range_rows", [1024, 4096, 131072])
def test_range_widths(apss, range_rows):
    # narrow ranges (many work items, hashed items), and one range wider than
    # 65,536 rows, where survivors are drained after every block instead of
    # sharing the queue across the item's blocks (no hashed items either)
    V = make_corpus(spec_for("c2", n=9000))
    t = np.float32(0.6)
    i, j, s, st = gpu_join(apss, V, t, range_rows=range_rows)
    assert_parity(i, j, s, oracle.join_plain(V, t), float(t), V)
    pre = oracle.join_prefix(V, t, 4)
    assert st["candidates"] == pre.candidates
    assert st["matches"] == len(i)


@pytest.mark.parametrize("variant,range_rows,range_group", [(1, 1024, 2), (1, 2048, 3), (2, 1024, 8), (0, 4096, 64),
                                                          (1, 131072, 2)])
def test_range_groups(apss, variant, range_rows, range_group):
    # work items that stage their tile once and visit several ranges: the
    # same pairs and candidates as one range per item, hashed and block
    # ranges mixed within an item, groups cut short by the triangle and by
    # the last range
    V = make_corpus(spec_for("c2", n=9000))
    t = np.float32(0.6)
    i, j, s, st = gpu_join(apss, V, t, variant=variant, range_rows=range_rows, range_group=range_group)
    assert_parity(i, j, s, oracle.join_plain(V, t), float(t), V)
    pre = oracle.join_prefix(V, t, 4)
    assert st["candidates"] == pre.candidates
    i1, j1, s1, st1 = gpu_join(apss, V, t, variant=variant, range_rows=range_rows)
    assert np.array_equal(i, i1) and np.array_equal(j, j1) and np.array_equal(s.view(np.uint32), s1.view(np.uint32))
    assert st["posting_visits"] == st1["posting_visits"]
    # queries against the index (no triangle), per-row thresholds
    Q = V.take_rows(np.arange(5, 9000, 61))
    tq = np.random.default_rng(11).uniform(0.5, 0.9, size=Q.n).astype(np.float32)
    ix = apss.Index.build(V, np.float32(0.5), variant=variant, range_rows=range_rows, range_group=range_group)
    try:
        qi, qy, qs = ix.query(Q, t_per_row=tq)
    finally:
        ix.close()
    assert_parity(qi, qy, qs, oracle.query(V, Q, t_per_row=tq.astype(np.float64)), None, Q, V,
                  per_row_t=tq.astype(np.float64))


def test_query_device_input_matches_host(apss):
    # the same queries given as device tensors take the device staging path
    # (row offsets checked on the device); the pairs are bitwise the same
    import torch
    from types import SimpleNamespace
    V = make_corpus(spec_for("c2", n=6000))
    Q = V.take_rows(np.arange(3, 6000, 41))
    tq = np.random.default_rng(7).uniform(0.5, 0.9, size=Q.n).astype(np.float32)
    D = SimpleNamespace(n=Q.n, row_ptr=torch.from_numpy(Q.row_ptr).cuda(), col=torch.from_numpy(Q.col).cuda(),
                        val=torch.from_numpy(Q.val).cuda())
    ix = apss.Index.build(V, np.float32(0.5))
    try:
        hi, hj, hs = ix.query(Q, t_per_row=tq)
        di, dj, ds = ix.query(D, t_per_row=tq)
        # bad queries are refused by both paths and leave the index usable
        bad = Csr(2, V.m, np.array([0, 1, 2]), np.array([3, V.m + 5], np.int32), np.array([1.0, 1.0], np.float32))
        for B in (bad, SimpleNamespace(n=2, row_ptr=torch.from_numpy(bad.row_ptr).cuda(),
                                       col=torch.from_numpy(bad.col).cuda(), val=torch.from_numpy(bad.val).cuda())):
            with pytest.raises(apss.ApssError) as e:
                ix.query(B, t=0.6)
            assert e.value.code == apss.APSS_EINVAL
        ai, aj, as_ = ix.query(Q, t_per_row=tq)
    finally:
        ix.close()
    assert np.array_equal(hi, di) and np.array_equal(hj, dj) and np.array_equal(hs, ds)
    assert np.array_equal(hi, ai) and np.array_equal(hj, aj) and np.array_equal(hs, as_)
    ref = oracle.query(V, Q, t_per_row=tq.astype(np.float64))
    assert_parity(hi, hj, hs, ref, None, Q, V, per_row_t=tq.astype(np.float64))
