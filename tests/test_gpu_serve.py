"""GPU tests of the serving loop: continuous batching, admission, per-request
results identical alone and in a mix, and parity with the CPU oracle."""
import threading

import numpy as np
import pytest

import oracle
from synth.corpus import Csr, make_corpus, make_queries, spec_for
from tests.parity import assert_parity

pytestmark = pytest.mark.gpu

T_BUILD = np.float32(0.5)


@pytest.fixture(scope="module")
def apss():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.init()
    import paper_1402_3010_amd as m
    m.load()
    return m


@pytest.fixture(scope="module")
def corpus():
    spec = spec_for("c5", n=30000)
    V = make_corpus(spec)
    Q = make_queries(V, 1500, spec, seed=2005)
    return V, Q


@pytest.fixture()
def index(apss, corpus):
    ix = apss.Index.build(corpus[0], T_BUILD)
    yield ix
    ix.close()


def split_requests(Q, seed, max_rows=160):
    """Consecutive row ranges of Q with log-uniform sizes, each with per-row thresholds."""
    rng = np.random.default_rng(seed)
    out, q = [], 0
    while q < Q.n:
        k = int(min(Q.n - q, np.floor(np.exp(rng.uniform(0.0, np.log(max_rows + 1))))))
        k = max(k, 1)
        if len(out) % 3 == 2:
            t = rng.uniform(0.5, 0.95, size=k)  # mixed thresholds inside one request
        else:
            t = np.full(k, rng.uniform(0.5, 0.95))
        out.append((q, q + k, t.astype(np.float32)))
        q += k
    return out


def rows_of(Q, lo, hi):
    return Q.take_rows(np.arange(lo, hi))


def request_bytes(nq, nnz, pairs_per_query=256):
    return 40 * nnz + 32 * nq + 28 * pairs_per_query * nq


def test_alone_equals_mixed_and_oracle(apss, corpus, index):
    V, Q = corpus
    reqs = split_requests(Q, seed=7)
    assert len(reqs) >= 20
    tq = np.concatenate([t for _, _, t in reqs])

    # alone: one slot, each request submitted after the previous one finished
    alone = []
    with apss.Server(index, slots=1) as srv:
        for lo, hi, t in reqs:
            rid = srv.submit(rows_of(Q, lo, hi), t_per_row=t)
            i, j, s, info = srv.poll(rid)
            assert info["batch_requests"] == 1
            alone.append((i, j, s))
        st = srv.stats()
        assert st["completed"] == len(reqs) and st["failed"] == 0 and st["peak_running"] == 1

    # mixed: a burst from four threads into two slots with small batches, so
    # requests are merged into shared batches and batches overlap on the GPU
    mixed = [None] * len(reqs)
    infos = [None] * len(reqs)
    with apss.Server(index, slots=2, max_batch_queries=256) as srv:
        ids = [None] * len(reqs)

        def submitter(part):
            for k in part:
                lo, hi, t = reqs[k]
                ids[k] = srv.submit(rows_of(Q, lo, hi), t_per_row=t)

        parts = [list(range(w, len(reqs), 4)) for w in range(4)]
        th = [threading.Thread(target=submitter, args=(p,)) for p in parts]
        for x in th:
            x.start()
        for x in th:
            x.join()
        assert all(r is not None for r in ids)
        for k in range(len(reqs)):
            i, j, s, info = srv.poll(ids[k])
            mixed[k] = (i, j, s)
            infos[k] = info
        st = srv.stats()
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert st["batches"] < len(reqs), "no request shared a batch"
    assert max(x["batch_requests"] for x in infos) > 1
    assert st["peak_running"] >= 2 and st["overlapped_batches"] >= 1, st
    assert st["reserved_bytes"] == 0

    total = 0
    for k, ((ai, aj, as_), (mi, mj, ms)) in enumerate(zip(alone, mixed)):
        assert np.array_equal(ai, mi) and np.array_equal(aj, mj), "request %d pairs differ" % k
        assert np.array_equal(as_.view(np.uint32), ms.view(np.uint32)), "request %d sims differ" % k
        total += len(ai)

    # the same pairs as one direct query of all rows, and as the oracle
    gi = np.concatenate([m[0].astype(np.int64) + lo for m, (lo, _, _) in zip(mixed, reqs)])
    gj = np.concatenate([m[1] for m in mixed])
    gs = np.concatenate([m[2] for m in mixed])
    di, dj, ds = index.query(Q, t_per_row=tq)
    assert np.array_equal(gi, di.astype(np.int64)) and np.array_equal(gj, dj)
    assert np.array_equal(gs.view(np.uint32), ds.view(np.uint32))
    ref = oracle.query(V, Q, t_per_row=tq.astype(np.float64))
    assert_parity(gi, gj, gs, ref, None, Q, V, per_row_t=tq.astype(np.float64))
    assert total >= 100


def test_admission_by_memory_budget(apss, corpus, index):
    V, Q = corpus
    A, B = rows_of(Q, 0, 40), rows_of(Q, 40, 70)
    ba, bb = request_bytes(A.n, A.nnz), request_bytes(B.n, B.nnz)
    with apss.Server(index, slots=1, memory_budget=ba + bb - 1) as srv:
        srv.pause(True)
        ra = srv.submit(A, t=0.6)
        assert srv.stats()["reserved_bytes"] == ba
        with pytest.raises(apss.ApssError) as e:
            srv.submit(B, t=0.6)
        assert e.value.code == apss.APSS_EBUSY
        assert srv.try_submit(B, t=0.6) is None
        assert srv.poll(ra, timeout_ms=0) is None          # pending while paused
        assert srv.poll(ra, timeout_ms=20) is None
        st = srv.stats()
        assert st["rejected_busy"] == 2 and st["queued"] == 1 and st["submitted"] == 1
        srv.pause(False)
        ia, ja, sa, _ = srv.poll(ra)
        assert srv.stats()["reserved_bytes"] == 0
        rb = srv.submit(B, t=0.6)                          # admitted once A's reservation returned
        ib, jb, sb, _ = srv.poll(rb)
    ref = oracle.query(V, A, t=0.6)
    assert_parity(ia, ja, sa, ref, 0.6, A, V)
    ref = oracle.query(V, B, t=0.6)
    assert_parity(ib, jb, sb, ref, 0.6, B, V)
    # a request larger than the whole budget can never be admitted
    with apss.Server(index, slots=1, memory_budget=ba - 1) as srv:
        with pytest.raises(apss.ApssError) as e:
            srv.submit(A, t=0.6)
        assert e.value.code == apss.APSS_ENOMEM


def test_admission_by_held_requests(apss, corpus, index):
    V, Q = corpus
    A, B = rows_of(Q, 0, 5), rows_of(Q, 5, 9)
    with apss.Server(index, slots=1, max_pending=1) as srv:
        ra = srv.submit(A, t=0.7)
        with pytest.raises(apss.ApssError) as e:
            srv.submit(B, t=0.7)                           # A is held until polled
        assert e.value.code == apss.APSS_EBUSY
        srv.poll(ra)
        rb = srv.submit(B, t=0.7)
        srv.poll(rb)
        with pytest.raises(apss.ApssError) as e:
            srv.poll(rb)                                   # already collected
        assert e.value.code == apss.APSS_EINVAL


def test_submit_validation_and_edge_requests(apss, corpus, index):
    V, Q = corpus
    with apss.Server(index, slots=2) as srv:
        good = rows_of(Q, 0, 3)
        bad_dim = Csr(good.n, good.m, good.row_ptr.copy(), good.col.copy(), good.val.copy())
        bad_dim.col[1] = V.m
        bad_norm = Csr(good.n, good.m, good.row_ptr.copy(), good.col.copy(), good.val.copy() * np.float32(1.01))
        dup = Csr(good.n, good.m, good.row_ptr.copy(), good.col.copy(), good.val.copy())
        dup.col[1] = dup.col[0]
        for bad in (bad_dim, bad_norm, dup):
            with pytest.raises(apss.ApssError) as e:
                srv.submit(bad, t=0.6)
            assert e.value.code == apss.APSS_EINVAL
        for t in (0.3, 1.5):
            with pytest.raises(apss.ApssError) as e:
                srv.submit(good, t=t)
            assert e.value.code == apss.APSS_ETHRESH
        with pytest.raises(apss.ApssError) as e:
            srv.submit(good, t_per_row=np.array([0.6, 0.4, 0.6], np.float32))
        assert e.value.code == apss.APSS_ETHRESH
        # empty request, request of empty rows, one exact corpus row at t = 1
        empty = Csr(0, V.m, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.float32))
        blank = Csr(3, V.m, np.zeros(4, np.int64), np.zeros(0, np.int32), np.zeros(0, np.float32))
        same = V.take_rows(np.array([123]))
        r0, r1, r2 = srv.submit(empty, t=0.6), srv.submit(blank, t=0.6), srv.submit(same, t=0.5)
        r3 = srv.submit(good, t=0.6)
        assert len(srv.poll(r0)[0]) == 0
        assert len(srv.poll(r1)[0]) == 0
        i, j, s, _ = srv.poll(r2)
        assert 123 in j.tolist() and np.all(i == 0)
        i, j, s, _ = srv.poll(r3)
        assert_parity(i, j, s, oracle.query(V, good, t=0.6), 0.6, good, V)
        st = srv.stats()
        assert st["failed"] == 0 and st["submitted"] == 4


def test_regrown_slot_buffers_are_released(apss):
    """A batch whose pairs outgrow its reservation completes, and its slot
    gives the grown buffers back when it ends."""
    from synth.corpus import from_rows
    base = make_corpus(spec_for("c1", n=1))
    row = dict(zip(base.row(0)[0].tolist(), base.row(0)[1].tolist()))
    other = make_corpus(spec_for("c1", n=2000, seed=77))
    rows = [row] * 3000 + [dict(zip(*[a.tolist() for a in other.row(k)])) for k in range(other.n)]
    V = from_rows(rows, base.m)
    Q = from_rows([row] * 40, base.m)            # 40 x 3000 = 120,000 pairs
    ix = apss.Index.build(V, T_BUILD)
    try:
        with apss.Server(ix, slots=1, pairs_per_query=1) as srv:
            i, j, s, _ = srv.poll(srv.submit(Q, t=0.9))
            st = srv.stats()
            small = srv.poll(srv.submit(Q.take_rows(np.arange(1)), t=0.9))
            st2 = srv.stats()
    finally:
        ix.close()
    assert len(i) == 40 * 3000
    assert st["regrows"] >= 1
    # the slot holds far less than the 120,000-pair buffers it grew to
    assert st["device_bytes"][0] < 12 * 120000
    assert len(small[0]) == 3000 and st2["failed"] == 0
    assert_parity(i, j, s, oracle.query(V, Q, t=0.9), 0.9, Q, V)


def test_split_requests_equal_whole_requests(apss, corpus, index):
    """Requests queued as pieces of at most 7 rows, run by two slots side by
    side, give each request the same pairs, bit for bit, as whole requests."""
    V, Q = corpus
    reqs = split_requests(Q, seed=11)[:40]
    whole, pieces = [], []
    with apss.Server(index, slots=1) as srv:
        for lo, hi, t in reqs:
            whole.append(srv.poll(srv.submit(rows_of(Q, lo, hi), t_per_row=t))[:3])
    with apss.Server(index, slots=2, split_queries=7, max_batch_queries=16) as srv:
        ids = [srv.submit(rows_of(Q, lo, hi), t_per_row=t) for lo, hi, t in reqs]
        for rid in ids:
            pieces.append(srv.poll(rid)[:3])
        st = srv.stats()
    assert st["failed"] == 0 and st["completed"] == len(reqs)
    assert st["batches"] >= sum((hi - lo + 6) // 7 for lo, hi, _ in reqs) // 3
    for (ai, aj, as_), (bi, bj, bs) in zip(whole, pieces):
        assert np.array_equal(ai, bi) and np.array_equal(aj, bj)
        assert np.array_equal(as_.view(np.uint32), bs.view(np.uint32))
    lo, hi, t = max(reqs, key=lambda r: r[1] - r[0])
    R = rows_of(Q, lo, hi)
    k = reqs.index((lo, hi, t))
    assert_parity(*pieces[k], oracle.query(V, R, t_per_row=t.astype(np.float64)), None, R, V,
                  per_row_t=t.astype(np.float64))
