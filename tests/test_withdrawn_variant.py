"""CPU checks of the two leads on the memory-aperture faults of tile variant 3
(4 queries x 2,048 rows, 256 threads), which occurred while it was timed on the
500k-vector C4 workloads (plain index at t = 0.8 and the head-cut index of the
screened join), with a short-segment stream that located each entry's segment
by a binary search over the wave's lanes (six shuffles) -- since replaced.

A fault of this kind needs a global access outside every allocation: LDS
accesses and the list loads' vector offsets are range-checked by the
hardware.  The two unchecked or computed addressings examined here:

1. the long-segment stream puts a chunk's base in the scalar offset of its
   buffer loads, outside the range check, so a chunk of a long segment that
   ends within 63 entries of the packed list array's end reads past it.
   Long segments come only from the dense lists (the H = 32,768 densest
   ranks, whose entries lead the array), so this needs those lists to end
   within 64 entries of the array's end.  Checked on both workloads: they end
   tens of millions of entries before it.
2. the shuffle-search stream: a model of it at the variant's geometry (4
   waves, 8 chunks in flight) over random segment layouts finds every lane's
   segment index inside the segment table and every live lane's entry inside
   its segment.

Neither lead is the cause; the variant stays withdrawn.
"""
import numpy as np
import pytest

import oracle
from synth.corpus import make_corpus, spec_for

H = 32768        # ranks with per-block offsets (dense lists) in every index
HEAD = 4096      # head of the screened join at C4


def postings_per_rank(V, rank, indexed):
    """Entries of each rank's inverted list, given which components are indexed."""
    return np.bincount(rank[V.col][indexed], minlength=V.m)


@pytest.mark.slow
def test_dense_lists_end_far_from_the_array_end():
    V = make_corpus(spec_for("c4"))
    t = np.float32(0.8)
    rank, mw, cut = oracle.prefix_index(V, t, l2_clause=True)
    pos = np.arange(V.nnz) - np.repeat(V.row_ptr[:-1], np.diff(V.row_ptr))
    # component k of a row (rank order) is indexed from the cut on; the
    # position in rank order is the order of its rank within the row
    r = rank[V.col]
    order = np.lexsort((r, np.repeat(np.arange(V.n), np.diff(V.row_ptr))))
    pos_in_rank_order = np.empty(V.nnz, np.int64)
    pos_in_rank_order[order] = pos
    plain = postings_per_rank(V, rank, pos_in_rank_order >= np.repeat(cut, np.diff(V.row_ptr)))
    headcut = postings_per_rank(V, rank, r >= HEAD)
    for cnt in (plain, headcut):
        off = np.concatenate([[0], np.cumsum(cnt)])
        P = int(off[-1])
        dense_end = int(off[min(H, V.m)])
        assert P - dense_end > 64 * 1000, (P, dense_end)
    assert headcut[:HEAD].sum() == 0


def old_shuffle_stream(segpre, ns, nw, u_depth):
    """The replaced short-segment stream: returns every lane's segment index
    and the (entry, segment) of every live lane."""
    L = int(segpre[ns])
    lanes = np.arange(64)
    reads, live_pairs = [], []
    per = (((L + nw - 1) // nw) + 63) & ~63
    for wave in range(nw):
        vbeg = wave * per
        vend = min(vbeg + per, L)
        if vbeg >= vend:
            continue
        lo, hi = 0, ns - 1
        while lo < hi:
            mid = (lo + hi + 1) >> 1
            if segpre[mid] <= vbeg:
                lo = mid
            else:
                hi = mid - 1
        sa = lo
        for base in range(vbeg, vend, 64 * u_depth):
            for u in range(u_depth):
                c = base + u * 64
                sj = sa + 1 + lanes
                rel = np.where(sj < ns, segpre[np.minimum(sj, ns - 1)] - c, 0x7FFFFFFF)
                k = np.zeros(64, np.int64)
                for step in (32, 16, 8, 4, 2, 1):
                    r = rel[k + step - 1]          # shuffle from lane k + step - 1
                    k = np.where(r <= lanes, k + step, k)
                sg = sa + k
                reads.append(sg.copy())
                v = c + lanes
                live = v < vend
                live_pairs.append((v[live], sg[live]))
                last = int(sg[63])
                sa = last + 1 if (last + 1 < ns and segpre[last + 1] <= c + 64) else last
    return reads, live_pairs


@pytest.mark.parametrize("seed", range(8))
def test_replaced_shuffle_stream_stays_in_range(seed):
    rng = np.random.default_rng(seed)
    for trial in range(30):
        # block path: short segments of 1..31 entries; hashed items: whole-range
        # segments of any length, at most 3 / 4 of the 4,096-slot table in all
        if trial % 2:
            lens = rng.integers(1, 32, size=int(rng.integers(1, 1025)))
        else:
            lens = rng.integers(1, 300, size=int(rng.integers(1, 60)))
            lens = lens[np.cumsum(lens) <= 3072]
            if len(lens) == 0:
                lens = np.array([1])
        ns = len(lens)
        segpre = np.concatenate([[0], np.cumsum(lens)])
        reads, live = old_shuffle_stream(segpre, ns, nw=4, u_depth=8)
        for sg in reads:
            assert sg.min() >= 0 and sg.max() < ns
        for v, sg in live:
            assert np.all(segpre[sg] <= v) and np.all(v < segpre[sg + 1])
