"""CPU model of the join kernel's short-segment stream indexing.

The kernel maps each streamed list entry to its segment without branches:
a chunk table gives the segment holding each 64-entry chunk's first entry,
every lane stores the start of one later segment as a tagged flag in the
chunk's row (lanes whose segment does not start in the chunk store to a
sink), the prefix sums are read at an index clamped to the total, and a
lane's segment is the chunk's first segment plus the number of flags at or
before it.  Lanes past the wave's slice still run the whole sequence and
must land on a valid segment, since they read it and add zero.  This model
checks, over random segment layouts, that every live lane finds the segment
that holds its entry and that every lane reads a segment in range.
"""
import numpy as np
import pytest

LONG_SEG = 32  # segments at least this long go to the long stream


def chunk_table(segpre, ns):
    """Segment holding the first entry of every 64-entry chunk."""
    L = int(segpre[ns])
    first = np.zeros((L + 63) // 64 + 1, dtype=np.int64)
    for e in range(ns):
        s0, s1 = int(segpre[e]), int(segpre[e + 1])
        c = (s0 + 63) & ~63
        while c < s1:
            first[c >> 6] = e
            c += 64
    return first


def stream(segpre, ns, nw, u_depth):
    """(entry, segment) of every live lane, and every segment index read."""
    L = int(segpre[ns])
    first = chunk_table(segpre, ns)
    lanes = np.arange(64)
    live_pairs, reads = [], []
    per = (((L + nw - 1) // nw) + 63) & ~63
    for wave in range(nw):
        vbeg = wave * per
        vend = min(vbeg + per, L)
        if vbeg >= vend:
            continue
        flag = np.zeros((u_depth, 64), dtype=np.int64)
        tag = 0
        for base in range(vbeg, vend, 64 * u_depth):
            tag += 1
            assert tag < 255  # the flags hold the tag in a byte
            sa = np.zeros(u_depth, dtype=np.int64)
            for u in range(u_depth):
                c = base + u * 64
                sa[u] = first[c >> 6] if c < vend else 0
                sj = sa[u] + 1 + lanes
                d = segpre[np.minimum(sj, ns)] - c  # clamped read: segpre[ns] is the total
                rel = np.where((c < vend) & (sj < ns), d, 0x7FFFFFFF)
                hit = (rel >= 0) & (rel < 64)
                # a segment that starts in the chunk starts after its first entry
                assert np.all(rel[hit] >= 1)
                flag[u, rel[hit]] = tag  # the others go to the sink
            for u in range(u_depth):
                c = base + u * 64
                f = flag[u] == tag
                sg = sa[u] + np.cumsum(f)
                reads.append(sg)
                v = c + lanes
                live = v < vend
                live_pairs.append((v[live], sg[live]))
    return live_pairs, reads


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("nw,u_depth", [(8, 4), (8, 8), (4, 8)])
def test_every_lane_finds_a_valid_segment(seed, nw, u_depth):
    rng = np.random.default_rng(1000 * seed + 10 * nw + u_depth)
    for _ in range(40):
        ns = int(rng.integers(1, 600))
        # short segments of the block path (1..31 entries), or the longer
        # whole-range segments of a hashed item
        hi = int(rng.choice([2, 3, 8, LONG_SEG, 300]))
        lens = rng.integers(1, hi, size=ns)
        segpre = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
        owner = np.repeat(np.arange(ns), lens)
        live_pairs, reads = stream(segpre, ns, nw, u_depth)
        covered = np.zeros(int(segpre[ns]), dtype=bool)
        for v, sg in live_pairs:
            assert np.array_equal(sg, owner[v])
            covered[v] = True
        assert covered.all()  # every entry is streamed by some lane
        for sg in reads:
            assert sg.min() >= 0 and sg.max() < ns


def test_short_segments_start_at_most_one_chunk():
    # the block path stores one chunk-table entry per short segment
    for s0 in range(0, 256):
        for sl in range(1, LONG_SEG):
            c = (s0 + 63) & ~63
            starts = len(range(c, s0 + sl, 64))
            assert starts == (1 if c < s0 + sl else 0)
