"""Comparison helpers shared by the GPU parity tests (test infrastructure)."""
import numpy as np

BAND = 1e-5     # pairs whose exact similarity is within BAND of t may differ
SIM_TOL = 1e-5  # every reported similarity within SIM_TOL of the double value


def exact_dot(V, a: int, b: int, W=None) -> float:
    """Double-precision dot product of row a of V and row b of W (default V)."""
    W = V if W is None else W
    ca, va = V.row(int(a))
    cb, vb = W.row(int(b))
    common, ia, ib = np.intersect1d(ca, cb, assume_unique=True, return_indices=True)
    return float(np.dot(va[ia].astype(np.float64), vb[ib].astype(np.float64)))


def pair_keys(i, j):
    return np.asarray(i, np.int64) * (1 << 32) + np.asarray(j, np.int64)


def assert_parity(gi, gj, gs, ref, t, V, W=None, per_row_t=None):
    """GPU pairs (gi, gj, gs) against the oracle's ref (Pairs) at threshold t.

    Equal outside |sim - t| <= BAND; common pairs' sims within SIM_TOL; the
    output must be sorted by (i, j) without duplicates.
    """
    gk = pair_keys(gi, gj)
    assert np.all(np.diff(gk) > 0), "GPU output not strictly sorted by (i, j)"
    G = dict(zip(gk.tolist(), np.asarray(gs, np.float64).tolist()))
    O = dict(zip(ref.keys().tolist(), ref.s.tolist()))
    thr = lambda k: (per_row_t[k >> 32] if per_row_t is not None else t)
    only_g = set(G) - set(O)
    only_o = set(O) - set(G)
    for k in only_g:
        s = exact_dot(V, k >> 32, k & 0xFFFFFFFF, W) if W is not None else exact_dot(V, k >> 32, k & 0xFFFFFFFF)
        assert abs(s - thr(k)) <= BAND, "extra pair %s sim %.9f t %.9f" % ((k >> 32, k & 0xFFFFFFFF), s, thr(k))
    for k in only_o:
        assert abs(O[k] - thr(k)) <= BAND, "missing pair %s sim %.9f t %.9f" % ((k >> 32, k & 0xFFFFFFFF), O[k], thr(k))
    common = set(G) & set(O)
    if common:
        d = max(abs(G[k] - O[k]) for k in common)
        assert d <= SIM_TOL, "sim error %g" % d
    return len(common), len(only_g), len(only_o)


def assert_rows_parity(gi, gj, gs, V, t, rows, oracle):
    """Self-join pairs (gi, gj, gs) against the oracle on every pair that
    involves one of `rows` (as i or as j), whatever its partner.

    The oracle finds the partners of each selected row by the plain
    definition over the whole corpus (query mode), so the check does not
    depend on how the rows were chosen.  Returns the number of pairs compared.
    """
    rows = np.unique(np.asarray(rows, np.int64))
    ref = oracle.query(V, V.take_rows(rows), t=float(t))
    O = {}
    for q, y, s in zip(ref.i.tolist(), ref.j.tolist(), ref.s.tolist()):
        r = int(rows[q])
        if r == y:
            continue
        O[(min(r, y) << 32) | max(r, y)] = s
    gi = np.asarray(gi, np.int64)
    gj = np.asarray(gj, np.int64)
    sel = np.isin(gi, rows) | np.isin(gj, rows)
    gk = (gi[sel] << 32) | gj[sel]
    G = dict(zip(gk.tolist(), np.asarray(gs, np.float64)[sel].tolist()))
    for k in set(G) - set(O):
        s = exact_dot(V, k >> 32, k & 0xFFFFFFFF)
        assert abs(s - t) <= BAND, "extra pair %s sim %.9f t %.9f" % ((k >> 32, k & 0xFFFFFFFF), s, t)
    for k in set(O) - set(G):
        assert abs(O[k] - t) <= BAND, "missing pair %s sim %.9f t %.9f" % ((k >> 32, k & 0xFFFFFFFF), O[k], t)
    common = set(G) & set(O)
    if common:
        d = max(abs(G[k] - O[k]) for k in common)
        assert d <= SIM_TOL, "sim error %g" % d
    return len(common)
