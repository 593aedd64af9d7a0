"""GPU tests of the autotuner (variant / range choice, JSON cache) and of
graph replay of the self-join."""
import json
import os

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


def same(a, b):
    return (len(a[0]) == len(b[0]) and np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
            and np.array_equal(np.asarray(a[2]).view(np.uint32), np.asarray(b[2]).view(np.uint32)))


@pytest.mark.parametrize("name,n,t,sd", [("c2", 20000, 0.7, 0), ("c4", 20000, 0.8, 4096)])
def test_autotune_choice_and_cache(apss, tmp_path, name, n, t, sd):
    V = make_corpus(spec_for(name, n=n))
    t = np.float32(t)
    cache = str(tmp_path / "tune.json")
    ix = apss.Index.build(V, t, screen_dims=sd)
    try:
        before = ix.join(t)
        r = ix.autotune(t, cache=cache)
        assert r["from_cache"] == 0 and r["tried"] >= 4 and r["cache_write_failed"] == 0
        assert 0 <= r["variant"] < 4 and r["range_rows"] in (2048, 4096, 8192, 16384) and r["ms"] > 0
        after = ix.join(t)
        assert same(before, after)
    finally:
        ix.close()
    text = open(cache).read()
    entries = json.loads(text)
    assert len(entries) == 1
    key = next(iter(entries))
    assert key.startswith("gfx950|") and ("|screened|" in key) == (sd > 0)
    assert entries[key]["variant"] == r["variant"] and entries[key]["range_rows"] == r["range_rows"]
    ix = apss.Index.build(V, t, screen_dims=sd)
    try:
        r2 = ix.autotune(t, cache=cache)
        assert r2["from_cache"] == 1 and r2["tried"] == 0
        assert (r2["variant"], r2["range_rows"]) == (r["variant"], r["range_rows"])
        again = ix.join(t)
        assert same(before, again)
        r3 = ix.autotune(t, budget_ms=1e-3)   # no cache: only the current configuration
        assert r3["tried"] == 1 and r3["from_cache"] == 0
    finally:
        ix.close()
    assert_parity(*before, oracle.join_plain(V, t), float(t), V)


def test_graph_replay_matches_eager(apss):
    import torch
    V = make_corpus(spec_for("c2", n=12000))
    t = np.float32(0.6)
    eager = apss.Index.build(V, t)
    ref = eager.join(t)
    stream = torch.cuda.Stream()
    g = apss.Index.build(V, t, stream=stream.cuda_stream, graph=True)
    try:
        cap = len(ref[0]) + 100
        oi = torch.zeros(cap, dtype=torch.int32, device="cuda")
        oj = torch.zeros(cap, dtype=torch.int32, device="cuda")
        os_ = torch.zeros(cap, dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        Q = V.take_rows(np.arange(0, 12000, 37))
        for k in range(6):
            if k == 3:
                g.query(Q, t=0.7)          # other work on the index drops the graph
            oi.fill_(-1)
            oj.fill_(-1)
            os_.fill_(-1.0)
            torch.cuda.synchronize()
            cnt = g.join_device(t, oi, oj, os_)
            got = (oi[:cnt].cpu().numpy().view(np.uint32), oj[:cnt].cpu().numpy().view(np.uint32),
                   os_[:cnt].cpu().numpy())
            assert same(got, ref), "replay %d differs" % k
            st = g.stats()
            assert st["matches"] == cnt and st["posting_visits"] > 0
            eager.query(Q, t=0.7)          # eager work between replays
            torch.cuda.synchronize()
        # other outputs or threshold: recaptured, still exact
        oi2 = torch.zeros(cap, dtype=torch.int32, device="cuda")
        cnt = g.join_device(t, oi2, oj, os_)
        assert np.array_equal(oi2[:cnt].cpu().numpy().view(np.uint32), ref[0])
        ref2 = eager.join(np.float32(0.75))
        cnt = g.join_device(np.float32(0.75), oi2, oj, os_)
        assert cnt == len(ref2[0]) and np.array_equal(oj[:cnt].cpu().numpy().view(np.uint32), ref2[1])
    finally:
        g.close()
        eager.close()
