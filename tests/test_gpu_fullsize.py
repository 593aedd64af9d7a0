"""GPU parity at full size, in the configurations the benchmark times.

The oracle cannot recompute a whole full-size join in a test, so each case
checks every pair that involves a sample of rows: contiguous windows of rows
(all their earlier partners, by the plain definition) and rows drawn from
the GPU's own output (all their partners, earlier or later, by the oracle's
query mode over the whole corpus), plus exact similarities of a random
sample of reported pairs.  The match set is that of Section 2.1 computed by
Find-Matches-0 (Algorithm 2).
"""
import threading

import numpy as np
import pytest

import oracle
from synth.corpus import make_corpus, make_queries, spec_for
from tests.parity import assert_parity, assert_rows_parity, exact_dot

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def apss():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.init()
    import paper_1402_3010_amd as m
    m.load()
    return m


@pytest.fixture(scope="module")
def c4():
    return make_corpus(spec_for("c4"))


def join(apss, V, t, **kw):
    print("full-size join n=%d t=%.2f %s" % (V.n, t, kw), flush=True)
    ix = apss.Index.build(V, np.float32(t), **kw)
    try:
        i, j, s = ix.join(np.float32(t))
        st = ix.stats()
    finally:
        ix.close()
    return i, j, s, st


def check_sampled(V, t, i, j, s, windows=((None, 200),), drawn=200, seed=0):
    """Windows of rows against the oracle's plain join, rows drawn from the
    output against its query mode, and exact dots of reported pairs."""
    t = np.float32(t)
    for lo, k in windows:
        lo = V.n - k if lo is None else lo
        ref = oracle.join_plain(V, t, lo, lo + k)
        sel = (j >= lo) & (j < lo + k)
        assert_parity(i[sel], j[sel], s[sel], ref, float(t), V)
    rng = np.random.default_rng(seed)
    if len(i) and drawn:
        ends = np.concatenate([i, j]).astype(np.int64)
        rows = rng.choice(ends, size=min(drawn, len(ends)), replace=False)
        assert assert_rows_parity(i, j, s, V, float(t), rows, oracle) >= min(drawn, len(ends)) // 2
    for k in rng.integers(0, len(i), size=min(2000, len(i))):
        d = exact_dot(V, i[k], j[k])
        assert d >= float(t) - 1e-5 and abs(d - s[k]) <= 1e-5


def test_c2_t07_full(apss):
    V = make_corpus(spec_for("c2"))
    i, j, s, st = join(apss, V, 0.7)
    check_sampled(V, 0.7, i, j, s, windows=((None, 300), (V.n // 2, 300)))
    assert st["matches"] == len(i)


def test_c4_plain_and_screened_full(apss, c4):
    """C4 at n = 500,000, t = 0.8: the plain join with the tuned geometry and
    the screened join in the benchmark's tuned configuration (head of 4,096
    dimensions, tile variant 2 = 16 queries x 1,024 rows, hashed ranges of
    8,192 rows): identical outputs, both against the oracle."""
    V = c4
    plain = join(apss, V, 0.8, variant=1, range_rows=16384)
    scr = join(apss, V, 0.8, screen_dims=4096, variant=2, range_rows=8192)
    assert len(plain[0]) == len(scr[0])
    assert np.array_equal(plain[0], scr[0]) and np.array_equal(plain[1], scr[1])
    assert np.array_equal(plain[2].view(np.uint32), scr[2].view(np.uint32))
    st = scr[3]
    assert st["screen_tiles"] > 0 and st["screen_candidates"] > 0 and st["posting_visits"] > 0
    i, j, s = scr[:3]
    check_sampled(V, 0.8, i, j, s, windows=((None, 300), (V.n // 4, 200)), drawn=300)
    # pairs found by the screen alone: both rows' head norms reach t and the
    # pair shares no dimension outside the head -- sample them on purpose
    assert st["matches"] == len(i)


def test_c4_screened_from_tuning_cache(apss, c4):
    """The screened index as the benchmark builds it: geometry looked up in
    the shipped tuning cache, then joined; same pairs as the plain join."""
    import os
    V = c4
    t = np.float32(0.8)
    cache = os.path.join(os.path.dirname(apss.__file__), "tuning", "gfx950.json")
    ix = apss.Index.build(V, t, screen_dims=4096)
    try:
        res = ix.autotune(t, budget_ms=1.0, cache=cache)
        assert res["from_cache"] == 1, res
        i, j, s = ix.join(t)
    finally:
        ix.close()
    rows = np.arange(V.n - 150, V.n)
    assert_rows_parity(i, j, s, V, float(t), rows, oracle)
    assert len(i) > 100000


def test_c5_server_full(apss):
    """C5: the 2M-vector resident index built at t = 0.5 and a server with the
    benchmark's settings (2 slots, batches of up to 4,096 queries).  A burst of
    requests -- one of 4,096 queries, others of log-uniform size -- with
    queries from the corpus generator plus 10% perturbed corpus copies and a
    threshold per request in [0.5, 0.95]; sampled rows of every request
    against the oracle's query mode."""
    spec = spec_for("c5")
    V = make_corpus(spec)
    Q = make_queries(V, 8192, spec, seed=2005)
    rng = np.random.default_rng(11)
    sizes = [4096, 1, 37, 512, 1500, 9, 2000]
    reqs, q = [], 0
    for k in sizes:
        t = np.full(k, rng.uniform(0.5, 0.95), np.float32)
        if k > 100:
            t = rng.uniform(0.5, 0.95, size=k).astype(np.float32)  # mixed thresholds in one request
        reqs.append((q, q + k, t))
        q += k
    print("c5 index n=%d nnz=%d" % (V.n, V.nnz), flush=True)
    ix = apss.Index.build(V, np.float32(0.5))
    try:
        results = [None] * len(reqs)
        with apss.Server(ix, slots=2, max_batch_queries=4096) as srv:
            ids = [None] * len(reqs)

            def submitter(part):
                for k in part:
                    lo, hi, t = reqs[k]
                    ids[k] = srv.submit(Q.take_rows(np.arange(lo, hi)), t_per_row=t)

            th = [threading.Thread(target=submitter, args=([k for k in range(len(reqs)) if k % 2 == w],))
                  for w in range(2)]
            for x in th:
                x.start()
            for x in th:
                x.join()
            for k in range(len(reqs)):
                results[k] = srv.poll(ids[k])
            st = srv.stats()
        assert st["completed"] == len(reqs) and st["failed"] == 0
    finally:
        ix.close()
    checked = 0
    total = 0
    for (lo, hi, t), (i, j, s, info) in zip(reqs, results):
        total += len(i)
        nq = hi - lo
        pick = np.unique(np.concatenate([np.arange(0, nq, max(1, nq // 60)), [nq - 1]]))
        R = Q.take_rows(np.arange(lo, hi)[pick])
        ref = oracle.query(V, R, t_per_row=t[pick].astype(np.float64))
        sel = np.isin(i, pick)
        remap = np.full(nq, -1, np.int64)
        remap[pick] = np.arange(len(pick))
        gi = remap[i[sel].astype(np.int64)]
        assert_parity(gi, j[sel], s[sel], ref, None, R, V, per_row_t=t[pick].astype(np.float64))
        checked += len(pick)
    assert checked >= 200
    assert total > 1000
