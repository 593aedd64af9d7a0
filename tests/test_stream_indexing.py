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

A second model covers the block path's segment placement, which stores
without branches too: long segments fill the front of the segment array,
short ones its back, and the prefix sums and chunk table agree with them.
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


def place(kinds, lens, QB, KMAX, NT):
    """The block path's placement: thread t owns components t*KMAX..t*KMAX+KMAX-1
    in the scan (component j*NT + t in the tile); an exclusive scan over the
    threads of (long count, short count, short entries) gives each its
    offsets; long segments fill seg[0..nl), short ones seg[QB-ns..QB), with
    their prefix sums and one chunk-table entry each."""
    # per-thread totals in thread order, as the wave scans compute them
    cnt_l = np.zeros(NT, dtype=np.int64)
    cnt_s = np.zeros(NT, dtype=np.int64)
    len_s = np.zeros(NT, dtype=np.int64)
    for t in range(NT):
        for j in range(KMAX):
            k = j * NT + t
            cnt_l[t] += kinds[k] == 2
            cnt_s[t] += kinds[k] == 1
            len_s[t] += lens[k] if kinds[k] == 1 else 0
    nl, ns, L = int(cnt_l.sum()), int(cnt_s.sum()), int(len_s.sum())
    ex_l = np.concatenate([[0], np.cumsum(cnt_l)[:-1]])
    ex_s = np.concatenate([[0], np.cumsum(cnt_s)[:-1]])
    ex_len = np.concatenate([[0], np.cumsum(len_s)[:-1]])
    sbase = QB - ns
    seg = np.full(QB, -1, dtype=np.int64)  # component placed at each slot
    segpre = np.full(QB + 1, -1, dtype=np.int64)
    first = {}
    for t in range(NT):
        lb, sb, lp = int(ex_l[t]), int(ex_s[t]), int(ex_len[t])
        for j in range(KMAX):
            k = j * NT + t
            isl, iss = kinds[k] == 2, kinds[k] == 1
            sl = int(lens[k]) if iss else 0
            if isl or iss:  # (the kernel stores the rest to sinks)
                idx = lb if isl else sbase + sb
                assert seg[idx] == -1
                seg[idx] = k
            if iss:
                segpre[sb] = lp
                c = (lp + 63) & ~63
                if c < lp + sl:
                    assert (c >> 6) not in first
                    first[c >> 6] = sb
            lb += isl
            sb += iss
            lp += sl
    segpre[ns] = L
    return seg, segpre, first, nl, ns, L


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("QB,NT", [(1024, 512), (1536, 512), (1024, 256)])
def test_block_path_placement(seed, QB, NT):
    rng = np.random.default_rng(7 * seed + QB + NT)
    KMAX = QB // NT
    for _ in range(20):
        kinds = rng.choice([0, 1, 2], size=QB, p=rng.dirichlet([1, 1, 1]))
        lens = np.where(kinds == 1, rng.integers(1, LONG_SEG, size=QB), rng.integers(LONG_SEG, 5000, size=QB))
        seg, segpre, first, nl, ns, L = place(kinds, lens, QB, KMAX, NT)
        longs = set(np.nonzero(kinds == 2)[0])
        shorts_in_order = [k for t in range(NT) for j in range(KMAX) if kinds[(k := j * NT + t)] == 1]
        # long segments at the front, short ones at the back, none lost or shared
        assert set(seg[:nl]) == longs and nl + ns <= QB
        assert list(seg[QB - ns:]) == shorts_in_order
        assert np.all(seg[nl:QB - ns] == -1)
        # prefix sums and the chunk table agree with the short segments' lengths
        sl = np.array([lens[k] for k in shorts_in_order], dtype=np.int64)
        assert np.array_equal(segpre[:ns + 1], np.concatenate([[0], np.cumsum(sl)]))
        owner = np.repeat(np.arange(ns), sl)
        for c in range(0, L, 64):
            assert first[c >> 6] == owner[c]
