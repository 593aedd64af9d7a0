"""Pins of the CPU oracle against things other than itself.

* a hand-derived dyadic fixture (exact values, exact ties at t);
* brute force with dense numpy products and with scipy.sparse SpGEMM (the
  matrix view S = D D^T of Section 2.1 is a library product);
* exact rational arithmetic on small dyadic inputs;
* invariants of the definition: symmetry, self-similarity 1, monotonicity
  in t, relabelling, duplicates, disjoint supports;
* the lossless claims of Section 3.2.2: partial indexing, minsize and
  upperbound return exactly the plain set, and every unindexed part has
  dot(x, y') < t for every x.
"""
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from synth.corpus import CorpusSpec, Csr, from_rows, make_corpus, spec_for

GOLD = os.path.join(os.path.dirname(__file__), "golden", "dyadic_ties.txt")


def load_golden():
    rows, m, cases, rank, mw = {}, None, [], None, None
    cur = None
    for line in open(GOLD):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        tok = line.split()
        if tok[0] == "m":
            m = int(tok[1])
        elif tok[0] == "v":
            rows[int(tok[1])] = {int(a): float(b) for a, b in (x.split(":") for x in tok[2:])}
        elif tok[0] == "rank":
            rank = [int(x) for x in tok[1:]]
        elif tok[0] == "maxweight":
            mw = [float(x) for x in tok[1:]]
        elif tok[0] == "case":
            cur = dict(t=float(tok[1].split("=")[1]), pairs=[])
            cases.append(cur)
        elif tok[0] in ("cut", "cut_l2"):
            cur[tok[0]] = [int(x) for x in tok[1:]]
        elif tok[0] == "p":
            cur["pairs"].append((int(tok[1]), int(tok[2]), float(tok[3])))
    V = from_rows([rows[k] for k in range(len(rows))], m)
    return V, rank, mw, cases


def dense(V: Csr) -> np.ndarray:
    D = np.zeros((V.n, V.m), np.float64)
    rows = np.repeat(np.arange(V.n), np.diff(V.row_ptr))
    D[rows, V.col] = V.val
    return D


def brute_pairs(V: Csr, t: float):
    D = dense(V)
    S = D @ D.T
    i, j = np.nonzero(np.triu(S >= t, 1))
    return i, j, S[i, j]


def same_set(a_keys, a_s, b_keys, b_s, band_keys=None, tol=1e-12):
    """Equal as sets, scores within tol; keys in band_keys may differ."""
    A = dict(zip(a_keys.tolist(), a_s.tolist()))
    B = dict(zip(b_keys.tolist(), b_s.tolist()))
    band = set() if band_keys is None else set(band_keys.tolist())
    only_a = set(A) - set(B) - band
    only_b = set(B) - set(A) - band
    assert not only_a, "only in first: %d e.g. %s" % (len(only_a), sorted(only_a)[:5])
    assert not only_b, "only in second: %d e.g. %s" % (len(only_b), sorted(only_b)[:5])
    common = set(A) & set(B)
    if common:
        d = max(abs(A[k] - B[k]) for k in common)
        assert d <= tol, d


def keys(i, j):
    return np.asarray(i, np.int64) * (1 << 32) + np.asarray(j, np.int64)


# ---------------------------------------------------------------- fixtures


def test_golden_dyadic_plain_and_prefix():
    V, rank, mw, cases = load_golden()
    assert oracle.validate(V) == 0
    for c in cases:
        t = np.float32(c["t"])
        assert float(t) == c["t"]
        want = sorted((a, b) for a, b, _ in c["pairs"])
        wants = {(a, b): s for a, b, s in c["pairs"]}
        for res in (oracle.join_plain(V, t), oracle.join_prefix(V, t, 0), oracle.join_prefix(V, t, 7)):
            got = list(zip(res.i.tolist(), res.j.tolist()))
            assert got == want
            for a, b, s in zip(res.i, res.j, res.s):
                assert s == wants[(a, b)]          # dyadic: exact
        r, w, cut = oracle.prefix_index(V, t, l2_clause=False)
        assert list(r) == rank
        assert list(w) == mw
        assert list(cut) == c["cut"]
        _, _, cut2 = oracle.prefix_index(V, t, l2_clause=True)
        assert list(cut2) == c["cut_l2"]


def test_exact_rational_small():
    # random dyadic inputs: weights k/8 normalised only when the norm is exact
    rng = np.random.default_rng(3)
    rows = []
    for _ in range(40):
        d = rng.choice(12, size=4, replace=False)
        rows.append({int(x): 0.5 for x in d})            # norm exactly 1
    V = from_rows(rows, 12)
    F = [{k: Fraction(v) for k, v in r.items()} for r in rows]
    for t in (0.25, 0.5, 0.75, 1.0):
        exp = sorted((a, b) for a in range(len(F)) for b in range(a + 1, len(F))
                     if sum(F[a][k] * F[b].get(k, 0) for k in F[a]) >= Fraction(t))
        for res in (oracle.join_plain(V, t), oracle.join_prefix(V, t, 3)):
            assert list(zip(res.i.tolist(), res.j.tolist())) == exp


def test_plain_vs_dense_numpy_c1():
    V = make_corpus(spec_for("c1"))
    for t in (0.3, 0.5, 0.7):
        bi, bj, bs = brute_pairs(V, t)
        res = oracle.join_plain(V, t)
        # scores are sums of exact float products in double: differences only from order
        band = keys(*np.nonzero(np.triu(np.abs(dense(V) @ dense(V).T - t) <= 1e-12, 1)))
        same_set(res.keys(), res.s, keys(bi, bj), bs, band, tol=1e-12)
        assert len(res) > 0


def test_plain_vs_scipy_spgemm():
    V = make_corpus(spec_for("c2", n=3000))
    A = sp.csr_matrix((V.val.astype(np.float64), V.col, V.row_ptr), shape=(V.n, V.m))
    S = sp.triu(A @ A.T, 1).tocoo()
    t = 0.5
    sel = S.data >= t
    res = oracle.join_plain(V, t)
    band = keys(S.row[np.abs(S.data - t) <= 1e-12], S.col[np.abs(S.data - t) <= 1e-12])
    same_set(res.keys(), res.s, keys(S.row[sel], S.col[sel]), S.data[sel], band)
    # visits of all-pairs-0 are sum_d C(|I_d|, 2) (Section 3.2.3)
    cnt = np.bincount(V.col, minlength=V.m).astype(np.int64)
    assert res.visits == int(np.sum(cnt * (cnt - 1) // 2))
    # candidates are exactly the pairs with a shared dimension
    assert res.candidates == S.nnz


def test_range_of_rows():
    V = make_corpus(spec_for("c1"))
    full = oracle.join_plain(V, 0.5)
    part = oracle.join_plain(V, 0.5, 700, 1300)
    sel = (full.j >= 700) & (full.j < 1300)
    assert np.array_equal(part.keys(), full.keys()[sel])


# ---------------------------------------------------------------- invariants


def test_invariants_symmetry_self_monotone():
    V = make_corpus(spec_for("c1", n=600))
    q = oracle.query(V, V, 0.5)
    diag = q.i == q.j
    assert diag.sum() == V.n                              # every row matches itself
    assert np.abs(q.s[diag] - 1.0).max() < 1e-6           # sim(x, x) = 1
    off = ~diag
    fwd = set(zip(q.i[off].tolist(), q.j[off].tolist()))
    assert fwd == {(b, a) for a, b in fwd}                # symmetric
    j = oracle.join_plain(V, 0.5)
    assert set(zip(j.i.tolist(), j.j.tolist())) == {(a, b) for a, b in fwd if a < b}
    prev = None
    for t in (0.3, 0.4, 0.5, 0.6, 0.8):
        cur = set(oracle.join_plain(V, t).keys().tolist())
        if prev is not None:
            assert cur <= prev                            # monotone in t
        prev = cur


def test_relabel_invariance():
    V = make_corpus(spec_for("c1", n=500))
    rng = np.random.default_rng(11)
    prow = rng.permutation(V.n)          # new row r holds old row prow[r]
    pdim = rng.permutation(V.m)          # old dim d becomes pdim[d]
    W = V.take_rows(prow)
    W = Csr(W.n, W.m, W.row_ptr, pdim[W.col].astype(np.int32), W.val)
    a = oracle.join_plain(V, 0.5)
    b = oracle.join_plain(W, 0.5)
    inv = np.empty(V.n, np.int64)
    inv[prow] = np.arange(V.n)
    mapped = {tuple(sorted((int(inv[x]), int(inv[y])))) for x, y in zip(a.i, a.j)}
    assert mapped == set(zip(b.i.tolist(), b.j.tolist()))
    bp = oracle.join_prefix(W, 0.5, 3)
    assert np.array_equal(bp.keys(), b.keys())


def test_duplicates_and_disjoint():
    V = make_corpus(spec_for("c1", n=50))
    rows = [dict(zip(V.row(k)[0].tolist(), V.row(k)[1].tolist())) for k in range(V.n)]
    rows.append(rows[7])                                  # duplicate of row 7
    rows.append({9999: 1.0})                              # a dim nobody else has
    W = from_rows(rows, V.m)
    res = oracle.join_plain(W, 0.999)
    pairs = set(zip(res.i.tolist(), res.j.tolist()))
    assert (7, V.n) in pairs
    assert all(V.n + 1 not in p for p in pairs)
    s = res.s[(res.i == 7) & (res.j == V.n)][0]
    assert abs(s - 1.0) < 1e-6


def test_empty_rows_never_match():
    V = from_rows([{0: 1.0}, {}, {0: 1.0}, {}], 3)
    res = oracle.join_plain(V, 0.1)
    assert list(zip(res.i.tolist(), res.j.tolist())) == [(0, 2)]
    pre = oracle.join_prefix(V, 0.1, 7)
    assert list(zip(pre.i.tolist(), pre.j.tolist())) == [(0, 2)]


# ---------------------------------------------------------------- lossless pruning


@pytest.mark.parametrize("flags", [0, 1, 2, 3, 4, 7, 8, 12, 15])
def test_prefix_equals_plain(flags):
    V = make_corpus(spec_for("c2", n=4000))
    for t in (0.5, 0.7, 0.9):
        a = oracle.join_plain(V, t)
        b = oracle.join_prefix(V, t, flags)
        # scores differ only by summation order: compare outside a 1e-12 band
        sa = dict(zip(a.keys().tolist(), a.s.tolist()))
        sb = dict(zip(b.keys().tolist(), b.s.tolist()))
        diff = set(sa) ^ set(sb)
        for k in diff:
            s = sa.get(k, sb.get(k))
            assert abs(s - t) < 1e-12
        assert len(a) > 0 or t == 0.9
        assert b.visits < a.visits                        # partial indexing touches less


def test_remscore_candidates_by_definition():
    """Remscore (all-pairs-2, Section 3.2.2) admits y when some indexed
    component of y meets a component of x processed while the remaining
    bound was at least t.  With x's components in rank order (densest
    first), the remaining bound at component k is the prefix sum
    sum_{i <= k} x_i maxweight_i(V), so the admitted candidates are the pairs
    y < x whose indexed part meets x where that prefix sum reaches t -- the
    rule stated here by prefix sums, independently of the oracle's running
    subtraction."""
    V = make_corpus(spec_for("c1", n=400))
    for t in (0.3, 0.5, 0.7):
        rank, mw, cut = oracle.prefix_index(V, t, l2_clause=True)
        rows = []
        for i in range(V.n):
            c, w = V.row(i)
            o = np.argsort(rank[c], kind="stable")
            rows.append((c[o], w[o].astype(np.float64)))
        indexed = [set(rows[i][0][cut[i]:].tolist()) for i in range(V.n)]
        cand = 0
        for x in range(V.n):
            d, w = rows[x]
            pre = np.cumsum(w * mw[d].astype(np.float64))
            adm = set(d[pre >= t].tolist())
            cand += sum(1 for y in range(x) if adm & indexed[y])
        res = oracle.join_prefix(V, t, oracle.FLAG_REMSCORE | oracle.FLAG_L2_CLAUSE)
        base = oracle.join_prefix(V, t, oracle.FLAG_L2_CLAUSE)
        assert res.candidates == cand
        assert res.candidates < base.candidates
        assert set(res.keys().tolist()) == set(base.keys().tolist())


def test_unindexed_part_bound():
    """dot(x, y') < t for all x, y: the guarantee behind partial indexing."""
    V = make_corpus(spec_for("c1"))
    D = dense(V)
    for t, l2 in ((0.5, False), (0.5, True), (0.7, True)):
        rank, mw, cut = oracle.prefix_index(V, t, l2_clause=l2)
        Dp = np.zeros_like(D)
        for y in range(V.n):
            c, w = V.row(y)
            o = np.argsort(rank[c])[: cut[y]]             # densest-first prefix
            Dp[y, c[o]] = w[o]
            # defining property of the cutoff
            b = np.cumsum(w[np.argsort(rank[c])].astype(np.float64) * mw[c[np.argsort(rank[c])]])
            if cut[y] < len(c):
                assert b[cut[y]] >= t or (l2 and np.sqrt(np.sum(w[np.argsort(rank[c])][: cut[y] + 1].astype(np.float64) ** 2)) >= t)
        assert (D @ Dp.T).max() < t
        if l2:
            assert np.sqrt((Dp ** 2).sum(1)).max() < t


def test_rank_and_maxweight_definition():
    V = make_corpus(spec_for("c2", n=2000))
    rank, mw, cut = oracle.prefix_index(V, 0.7)
    cnt = np.bincount(V.col, minlength=V.m)
    inv = np.argsort(rank)
    assert np.array_equal(np.sort(rank), np.arange(V.m))
    c = cnt[inv]
    assert (np.diff(c) <= 0).all()
    tie = np.diff(c) == 0
    assert (np.diff(inv)[tie] > 0).all()
    ref = np.zeros(V.m, np.float32)
    np.maximum.at(ref, V.col, V.val)
    assert np.array_equal(ref, mw)


# ---------------------------------------------------------------- queries


def test_query_vs_dense():
    V = make_corpus(spec_for("c1", n=800))
    Q = make_corpus(CorpusSpec(100, V.m, "uniform", 10, 60, 10, 60, 1.0, 77))
    # plus copies of corpus rows, so high thresholds have hits
    Q2 = V.take_rows(np.arange(0, 800, 40))
    rows = [dict(zip(*[a.tolist() for a in Q.row(k)])) for k in range(Q.n)]
    rows += [dict(zip(*[a.tolist() for a in Q2.row(k)])) for k in range(Q2.n)]
    Qa = from_rows(rows, V.m)
    tq = np.linspace(0.3, 0.95, Qa.n)
    res = oracle.query(V, Qa, t_per_row=tq)
    S = dense(Qa) @ dense(V).T
    qi, yi = np.nonzero(S >= tq[:, None])
    band = keys(*np.nonzero(np.abs(S - tq[:, None]) <= 1e-12))
    same_set(res.keys(), res.s, keys(qi, yi), S[qi, yi], band)
    assert len(res) >= Q2.n


# ---------------------------------------------------------------- validation


def test_validate():
    ok = from_rows([{0: 0.6, 1: 0.8}, {}], 4)
    assert oracle.validate(ok) == 0
    bad_neg = from_rows([{0: 1.0}, {0: -0.6, 1: 0.8}], 4)
    assert oracle.validate(bad_neg) == 2
    bad_nan = from_rows([{0: float("nan")}], 4)
    assert oracle.validate(bad_nan) == 1
    bad_norm = from_rows([{0: 0.5}], 4)
    assert oracle.validate(bad_norm) == 1
    bad_dim = Csr(1, 4, np.array([0, 1]), np.array([4], np.int32), np.array([1.0], np.float32))
    assert oracle.validate(bad_dim) == 1
    dup = Csr(1, 4, np.array([0, 2]), np.array([1, 1], np.int32), np.array([0.6, 0.8], np.float32))
    assert oracle.validate(dup) == 1
