"""Pins of the oracle's HSIG construction that do not run its own code twice.

* With one segment, HSIGInsert (Alg. 6) is the HNSW insertion (Alg. 3) on every
  layer.  An independent HNSW written here from Alg. 1 and Alg. 3 (plain Python
  lists and tuples, no code shared with the oracle) must give the oracle's
  chunks edge for edge.
* A six-object, two-segment input traced by hand through Alg. 6: forward chunks
  (Alg. 4), reverse edges into chunk i of the neighbour, the
  re-prune of an overflowing chunk, the global-edge marks of Alg. 5
  with their own re-prune, and a mark dropped when its edge is pruned away.
* The hybrid search's entry rule (the entry of the active segment whose top
  level is highest; among equals the nearer, then the smaller id) on a
  three-segment index built so that two segments share the top level.
"""
import math

import numpy as np

from oracle import hsig


# ---------------------------------------------------------------------------
# Independent HNSW (Alg. 1 ANNSearch, Alg. 3 InsertLayer, the Prune rule of
# Sec. 2.2, the level draw of Alg. 6).  Keys are (FP64 squared distance, id).
# ---------------------------------------------------------------------------
def _hnsw(X, level_u, M, ef_cons):
    Xd = np.asarray(X, np.float64)
    n = len(Xd)
    mL = 1.0 / math.log(M)

    def dist(a, b):
        e = Xd[a] - Xd[b]
        return float(np.dot(e, e))

    def prune(v, cands, cap):
        # sort by distance to v; drop r when an already kept e has d(e, r) < d(v, r)
        kept = []
        for dvr, r in sorted(cands):
            if len(kept) >= cap:
                break
            if r == v:
                continue
            if all(not dist(e, r) < dvr for _, e in kept):
                kept.append((dvr, r))
        return kept

    def ann_search(v, ep, ef, G, l):
        seen = {ep}
        first = (dist(v, ep), ep)
        cand, ann = [first], [first]
        while cand:
            o = min(cand)
            cand.remove(o)
            if o > max(ann):
                break
            for _, x in G[o[1]][l]:
                if x in seen:
                    continue
                seen.add(x)
                kx = (dist(v, x), x)
                if kx < max(ann) or len(ann) < ef:
                    cand.append(kx)
                    ann.append(kx)
                    if len(ann) > ef:
                        ann.remove(max(ann))
        return sorted(ann)

    levels = [int(math.floor(-math.log(u) * mL)) for u in level_u]
    G = [None] * n
    entry, top = -1, -1
    for v in range(n):
        lev = levels[v]
        G[v] = [[] for _ in range(lev + 1)]
        if entry < 0:
            entry, top = v, lev
            continue
        ep = entry
        for l in range(top, lev, -1):
            ep = ann_search(v, ep, 1, G, l)[0][1]
        for l in range(min(lev, top), -1, -1):
            ann = ann_search(v, ep, ef_cons, G, l)
            G[v][l] = prune(v, ann, M)
            for dvo, o in G[v][l]:
                G[o][l] = sorted(G[o][l] + [(dvo, v)])
                if len(G[o][l]) > M:
                    G[o][l] = prune(o, G[o][l], M)
            ep = ann[0][1]
        if lev > top:
            entry, top = v, lev
    return levels, G, entry


def test_single_segment_build_equals_independent_hnsw():
    """Catches, in the oracle's insertion: a wrong Prune comparison or order, a
    reverse edge that is not added or not re-pruned, the wrong entry for the
    next layer, a wrong level draw, the entry not moving to a higher object."""
    for seed, n, d, M, ef in ((1, 200, 8, 6, 24), (2, 160, 4, 4, 12), (3, 120, 16, 8, 200)):
        rng = np.random.default_rng(seed)
        X = rng.standard_normal((n, d)).astype(np.float32)
        attr = rng.permutation(n).astype(np.int64)
        u = 1.0 - rng.random(n)
        levels, G, entry = _hnsw(X, u, M, ef)
        ix = hsig.Index.build(X, attr, u, 1, M, ef)
        assert max(levels) >= 2  # the upper layers are exercised
        for v in range(n):
            assert ix.build_level(v) == levels[v]
            for l in range(levels[v] + 1):
                assert ix.build_chunk(v, l, 0) == [o for _, o in G[v][l]], (seed, v, l)
        _, seg_entry, seg_top = ix.segments()
        assert ix.ext_ids()[seg_entry[0]] == entry and seg_top[0] == max(levels)


# ---------------------------------------------------------------------------
# Hand-traced HSIGInsert on six objects of a line, two segments, M = 2.
# ---------------------------------------------------------------------------
# object: position on the first axis, attribute (segment boundary b_1 = 3:
# segment 0 = attributes 0..2, segment 1 = 3..5); inserted in this order.
_LINE = [(0.0, 0), (10.0, 3), (2.0, 1), (6.0, 4), (3.0, 5), (5.0, 2)]
# e0..e5 by external id; chunk lists ordered by distance to the owner.
_CHUNKS = {
    0: ([2], [1]),
    1: ([2, 0], [3]),
    2: ([0, 5], [4]),
    3: ([5, 2], [4, 1]),
    4: ([2, 5], [3]),
    5: ([2], [3, 4]),
}
_MARKS = {0: {1, 2}, 1: {3}, 2: {0, 4}, 3: {1, 5}, 4: {2, 5}, 5: {3, 4}}
# The trace (squared distances; segment of each object in brackets):
#  e0 [0]: entry of segment 0.
#  e1 [1]: chunk 0 <- Prune{e0} = [e0]; reverse e1 into e0's chunk 1.  Entry of
#     segment 1.  Marks: e1 -> {e0}; e0 holds e1, so e0 -> {e1}.
#  e2 [0]: chunk 0 = [e0] (reverse: e0.c0 = [e2]); chunk 1 = [e1] (reverse:
#     e1.c0 = [e2 64, e0 100]).  Marks: Prune(e2, [e0 4, e1 64]) keeps both
#     (d(e0,e1) = 100 is not < 64): e2 -> {e0, e1}; e0 -> {e1, e2}; e1 -> {e0, e2}.
#  e3 [1]: segment-0 search finds [e2 16, e0 36]; e0 is pruned by e2 (4 < 36):
#     chunk 0 = [e2], reverse e2.c1 = [e3 16, e1 64].  Chunk 1 = [e1], reverse
#     e1.c1 = [e3].  Marks: [e1 16, e2 16] (tie: smaller id first), both kept:
#     e3 -> {e1, e2}; e1 gets e3, now 3 > M: Prune(e1, [e3 16, e2 64, e0 100])
#     keeps {e3}; e2 gets e3: Prune(e2, [e0 4, e3 16, e1 64]) keeps {e0, e3}.
#  e4 [1]: segment 0: [e2 1, e0 9], e0 pruned by e2: chunk 0 = [e2]; reverse into
#     e2.c1 = [e4 1, e3 16, e1 64] overflows; Prune(e2, .) keeps [e4] (e3 and e1
#     are nearer e4 than e2: 9 < 16, 49 < 64) and e2's mark on e3 is dropped:
#     e2 -> {e0}.  Segment 1: [e3 9, e1 49], e1 pruned by e3: chunk 1 = [e3],
#     reverse e3.c1 = [e4 9, e1 16].  Marks: e4 -> {e2, e3}; e2 -> {e0, e4};
#     e3 -> {e1, e2, e4} overflows: Prune(e3, [e4 9, e1 16, e2 16]) = {e1, e4}.
#  e5 [0]: segment 0: [e2 9, e0 25], chunk 0 = [e2], reverse e2.c0 = [e0 4, e5 9].
#     Segment 1: [e3 1, e4 4, e1 25], Prune keeps [e3, e4]; reverse e3.c0 =
#     [e5 1, e2 16], e4.c0 = [e2 1, e5 4].  Marks: Prune(e5, [e3 1, e4 4, e2 9])
#     = {e3, e4}; e3 -> Prune(e3, [e5 1, e4 9, e1 16, e2 16]) = {e5, e1} (e4 is
#     nearer e5: 4 < 9); e4 -> Prune(e4, [e2 1, e5 4, e3 9]) = {e2, e5}.


def _line_index():
    X = np.zeros((6, 4), np.float32)
    X[:, 0] = [p for p, _ in _LINE]
    attr = np.array([a for _, a in _LINE], np.int64)
    u = np.ones(6)  # every object on layer 0
    return hsig.Index.build(X, attr, u, 2, 2, 16)


def test_hand_traced_backbone_and_masking():
    """Catches: a reverse edge put in the neighbour's chunk j instead of chunk i,
    an overflowing chunk left unpruned or pruned with the wrong owner, chunks not
    kept sorted, Alg. 5 marks taken over one chunk instead of all chunks, a mark
    added when v is not in o's lists, a missing re-prune of o's marks, and a mark
    kept after its edge was pruned."""
    ix = _line_index()
    for v, (c0, c1) in _CHUNKS.items():
        assert ix.build_level(v) == 0
        assert ix.build_chunk(v, 0, 0) == c0, v
        assert ix.build_chunk(v, 0, 1) == c1, v
    ext = ix.ext_ids()
    _, gl = ix.layer(0)
    internal = {int(e): i for i, e in enumerate(ext)}
    for v, marks in _MARKS.items():
        got = {int(ext[t]) for t in gl[internal[v]] if t >= 0}
        assert got == marks, (v, got)
    ss, entry, top = ix.segments()
    assert ss.tolist() == [0, 3, 6]
    assert [int(ext[e]) for e in entry] == [0, 1] and top.tolist() == [0, 0]


# ---------------------------------------------------------------------------
# Hybrid entry rule
# ---------------------------------------------------------------------------
def test_hybrid_entry_rule():
    """Three segments; the first object of segments 0 and 1 reaches layer 1, all
    others stay on layer 0.  Catches: an entry from a lower-level segment, the
    farther of two top-level entries, the larger id on a distance tie, and
    entries taken from inactive segments."""
    M = 4
    # external id: (position, attribute, level variate); segment b = 3, 6
    objs = [((1.0, 0.0), 0, 0.2), ((-1.0, 0.0), 3, 0.2), ((0.0, 0.5), 6, 1.0),
            ((7.0, 5.0), 1, 1.0), ((8.0, 5.0), 4, 1.0), ((9.0, 5.0), 7, 1.0),
            ((7.0, 6.0), 2, 1.0), ((8.0, 6.0), 5, 1.0), ((9.0, 6.0), 8, 1.0)]
    X = np.zeros((9, 4), np.float32)
    X[:, :2] = [p for p, _, _ in objs]
    attr = np.array([a for _, a, _ in objs], np.int64)
    u = np.array([x for _, _, x in objs])
    assert [hsig.level_of(x, M) for x in u[:3]] == [1, 1, 0]
    ix = hsig.Index.build(X, attr, u, 3, M, 16)
    ext = ix.ext_ids()
    internal = {int(e): i for i, e in enumerate(ext)}
    cases = [  # query position, range, expected entry (external id)
        ((0.0, 0.0), (0, 8), 0),    # e0 and e1 tie at distance 1: smaller id; e2 (level 0) is nearer
        ((-0.5, 0.0), (0, 8), 1),   # e1 nearer than e0
        ((1.0, 0.0), (3, 8), 1),    # segment 0 inactive: e1, although e2 is nearer
        ((0.0, 0.5), (6, 8), 2),    # only segment 2 active: its level-0 entry
        # attribute 2 (object e6) puts segment 0 in range: its entry e0 (distance 0)
        # wins although e0 itself is out of range
        ((1.0, 0.0), (2, 8), 0),
    ]
    Q = np.zeros((len(cases), 4), np.float32)
    Q[:, :2] = [c[0] for c in cases]
    lo = np.array([c[1][0] for c in cases], np.int64)
    hi = np.array([c[1][1] for c in cases], np.int64)
    _, _, cnt = ix.search(Q, lo, hi, 3, 8, strategy=hsig.HYBRID, counters=True)
    assert [int(c) for c in cnt[:, hsig.ENTRY]] == [internal[c[2]] for c in cases]


# ---------------------------------------------------------------------------
# Independent HSIGInsert (Alg. 6 with Alg. 4 per segment and layer and Alg. 5
# per layer), written here from the paper with the readings the oracle states:
# segment boundaries at ranks floor(j n / S) (values equal to a boundary go up);
# chunks sorted by (distance to the owner, id); an empty segment is skipped and a
# segment's entry moves only for its own objects; marks are kept as target ids,
# a mark is dropped when its edge is pruned, Alg. 5 prunes over all chunks with
# capacity M.  Keys are (FP64 squared distance, id).
# ---------------------------------------------------------------------------
def _hsig(X, attr, level_u, S, M, ef_cons):
    Xd = np.asarray(X, np.float64)
    n = len(Xd)
    mL = 1.0 / math.log(M)
    srt = sorted(int(a) for a in attr)
    bounds = [srt[j * n // S] for j in range(1, S)]
    seg = [sum(1 for b in bounds if int(a) >= b) for a in attr]

    def dist(a, b):
        e = Xd[a] - Xd[b]
        return float(np.dot(e, e))

    def prune(v, cands, cap):
        kept = []
        for dvr, r in sorted(cands):
            if len(kept) >= cap:
                break
            if r != v and all(not dist(e, r) < dvr for _, e in kept):
                kept.append((dvr, r))
        return kept

    adj, marks = [None] * n, [None] * n

    def ann_search(v, ep, ef, l, j):
        seen = {ep}
        first = (dist(v, ep), ep)
        cand, ann = [first], [first]
        while cand:
            o = min(cand)
            cand.remove(o)
            if o > max(ann):
                break
            for _, x in adj[o[1]][l][j]:
                if x not in seen:
                    seen.add(x)
                    kx = (dist(v, x), x)
                    if kx < max(ann) or len(ann) < ef:
                        cand.append(kx)
                        ann.append(kx)
                        if len(ann) > ef:
                            ann.remove(max(ann))
        return sorted(ann)

    def every_chunk(o, l):
        return sorted(e for ch in adj[o][l] for e in ch)

    levels = [int(math.floor(-math.log(u) * mL)) for u in level_u]
    entry, top = [-1] * S, [-1] * S
    gentry, gtop = -1, -1
    for v in range(n):
        i, lev = seg[v], levels[v]
        adj[v] = [[[] for _ in range(S)] for _ in range(lev + 1)]
        marks[v] = [set() for _ in range(lev + 1)]
        for j in range(S):
            if entry[j] < 0:
                if j == i:
                    entry[j], top[j] = v, lev
                continue
            ep = entry[j]
            for l in range(top[j], lev, -1):
                ep = ann_search(v, ep, 1, l, j)[0][1]
            for l in range(min(lev, top[j]), -1, -1):
                ann = ann_search(v, ep, ef_cons, l, j)
                adj[v][l][j] = prune(v, ann, M)
                for dvo, o in adj[v][l][j]:
                    adj[o][l][i] = sorted(adj[o][l][i] + [(dvo, v)])
                    if len(adj[o][l][i]) > M:
                        adj[o][l][i] = prune(o, adj[o][l][i], M)
                        held = {e for _, e in every_chunk(o, l)}
                        marks[o][l] &= held
                ep = ann[0][1]
            if j == i and lev > top[j]:
                entry[j], top[j] = v, lev
        for l in range(lev + 1):
            N = prune(v, every_chunk(v, l), M)
            marks[v][l] = {o for _, o in N}
            for _, o in N:
                if any(e == v for _, e in every_chunk(o, l)):
                    marks[o][l].add(v)
                    if len(marks[o][l]) > M:
                        marks[o][l] = {e for _, e in prune(o, every_chunk(o, l), M)}
        if lev > gtop:
            gentry, gtop = v, lev
    return levels, adj, marks, entry, gentry


def test_build_equals_independent_hsig_insert():
    """Integer coordinates on a small grid make equal distances common, so the
    (distance, id) order and the strict Prune test decide many choices.  Catches,
    besides the mistakes the hand trace catches: a non-strict Prune comparison,
    marks kept after their edge is pruned (they then count towards the M limit),
    ties broken by the larger id, and wrong segment entries."""
    cases = ((5, 48, 2, 3, 2, 16), (6, 60, 3, 2, 3, 8), (7, 64, 4, 3, 2, 32), (8, 40, 2, 2, 4, 4))
    for seed, n, d, S, M, ef in cases:
        rng = np.random.default_rng(seed)
        X = rng.integers(0, 5, (n, 4)).astype(np.float32)
        X[:, d:] = 0
        attr = rng.integers(0, n // 2, n).astype(np.int64)  # with duplicate attributes
        u = 1.0 - rng.random(n)
        levels, adj, marks, entry, gentry = _hsig(X, attr, u, S, M, ef)
        ix = hsig.Index.build(X, attr, u, S, M, ef)
        ext = ix.ext_ids()
        internal = {int(e): t for t, e in enumerate(ext)}
        for v in range(n):
            assert ix.build_level(v) == levels[v]
            for l in range(levels[v] + 1):
                for j in range(S):
                    assert ix.build_chunk(v, l, j) == [o for _, o in adj[v][l][j]], (seed, v, l, j)
        for l in range(max(levels) + 1):
            _, gl = ix.layer(l)
            for v in range(n):
                if levels[v] >= l:
                    got = {int(ext[t]) for t in gl[internal[v]] if t >= 0}
                    assert got == marks[v][l], (seed, v, l)
        _, seg_entry, _ = ix.segments()
        assert [int(ext[e]) if e >= 0 else -1 for e in seg_entry] == entry
        assert int(ext[ix.gentry]) == gentry
