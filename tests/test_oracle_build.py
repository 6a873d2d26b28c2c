"""Pins of the reference HSIG build (Sec. 3-4.1, Alg. 3-6) against the paper's
worked example, exact reductions and structural invariants."""
import os

import numpy as np
import pytest

from oracle import hsig
from synth import workloads as w


def test_prune_hand_cases():
    # Owner at the origin.  (2,0) is pruned by (1,0): d((1,0),(2,0)) = 1 < d(o,(2,0)) = 4.
    # (0,1) is kept (d to (1,0) is 2, not < 1).  (0,3) is pruned by (0,1) (4 < 9).
    # (-1.5, 0) is kept: d to (1,0) = 6.25, d to (0,1) = 3.25, both >= 2.25.
    o = np.zeros(4, np.float32)
    c = np.zeros((5, 4), np.float32)
    c[:, :2] = [[2, 0], [0, 3], [1, 0], [0, 1], [-1.5, 0]]
    assert hsig.prune(o, c, 8) == [2, 3, 4]
    assert hsig.prune(o, c, 2) == [2, 3]
    # Equal distances are kept (strict comparison): r = (0.5, 1) is exactly as far
    # from e = (1, 0) as from the owner (1.25 both), so it survives.
    c2 = np.zeros((2, 4), np.float32)
    c2[:, :2] = [[0.5, 1], [1, 0]]
    assert hsig.prune(o, c2, 8) == [1, 0]
    c2[0, :2] = [0.6, 1]                          # now nearer to e than to the owner: pruned
    assert hsig.prune(o, c2, 8) == [1]


def _tiny_build(n, S, M, ef=32, seed=5, d=8, attr=None):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, d)).astype(np.float32)
    if attr is None:
        attr = rng.permutation(n).astype(np.int64)
    u = 1.0 - rng.random(n)
    return X, attr, u, hsig.Index.build(X, attr, u, S, M, ef, seed=seed)


def test_example2_segments():
    # Example 2 of Sec. 3.2: v_i = i for i = 1..8, two segments [1,5) and [5,8].
    X, attr, u, ix = _tiny_build(8, 2, 4, attr=np.arange(1, 9, dtype=np.int64))
    ss, entry, maxlev = ix.segments()
    a = ix.attr_sorted()
    assert ss.tolist() == [0, 4, 8]
    assert a[ss[0]:ss[1]].tolist() == [1, 2, 3, 4]
    assert a[ss[1]:ss[2]].tolist() == [5, 6, 7, 8]


def test_equi_depth_and_duplicates():
    n, S = 1000, 8
    _, _, _, ix = _tiny_build(n, S, 8)
    ss, _, _ = ix.segments()
    assert np.all(np.diff(ss) == n // S)           # a permutation splits into equal segments
    # duplicates of a boundary value go to the higher segment
    attr = np.array([0, 1, 2, 3, 3, 3, 4, 5], np.int64)
    _, _, _, ix = _tiny_build(8, 2, 4, attr=attr)
    ss, _, _ = ix.segments()
    a = ix.attr_sorted()
    # b_1 = attr_sorted[4] = 3: every 3 is in segment 1
    assert ss.tolist() == [0, 3, 8] and a[3:6].tolist() == [3, 3, 3]


def test_structure_invariants(small_index, small_workload):
    ix = small_index
    X = small_workload.base
    ext = ix.ext_ids()
    Xs = X[ext]
    ss, entry, maxlev = ix.segments()
    seg_of = np.searchsorted(ss, np.arange(ix.n), side="right") - 1
    lev = ix.levels()
    assert entry.min() >= 0 and (lev[entry] == maxlev).all()
    for l in range(ix.L + 1):
        adj, gl = ix.layer(l)
        mc = adj.shape[2]
        have = np.nonzero(lev >= l)[0]
        for v in have[:: max(1, len(have) // 300)]:
            marked = [t for t in gl[v] if t >= 0]
            allnb = set()
            for j in range(ix.S):
                ch = adj[v, j]
                k = int((ch >= 0).sum())
                assert (ch[:k] >= 0).all() and (ch[k:] == -1).all()      # packed, -1 padded
                nb = ch[:k]
                assert len(set(nb.tolist())) == k and v not in nb          # no duplicates or loops
                assert (seg_of[nb] == j).all()                            # chunk j holds segment j
                assert (lev[nb] >= l).all()                               # neighbours live on layer l
                dd = ((Xs[nb].astype(np.float64) - Xs[v]) ** 2).sum(1)
                assert np.all(np.diff(dd) >= -1e-9)                       # sorted by distance (R5)
                allnb |= set(nb.tolist())
            assert len(marked) <= ix.MU and set(marked) <= allnb          # Alg. 5: <= M marks
            assert len(marked) >= 1 or len(allnb) == 0


def test_single_segment_masking_leaves_backbone():
    # With S = 1 the oracle's insertion run with and without Alg. 5's masking and
    # the skip list gives the same chunks: those steps never edit the backbone.
    # (The backbone itself is pinned against an independent HNSW in
    # test_oracle_build_pins.py.)
    rng = np.random.default_rng(8)
    n, d, M = 600, 8, 6
    X = rng.standard_normal((n, d)).astype(np.float32)
    attr = rng.permutation(n).astype(np.int64)
    u = 1.0 - rng.random(n)
    a = hsig.Index.build(X, attr, u, 1, M, 24)
    b = hsig.Index.build(X, attr, u, 1, M, 24, hnsw=True)
    for v in range(n):
        assert a.build_level(v) == b.build_level(v)
        for l in range(a.build_level(v) + 1):
            assert a.build_chunk(v, l, 0) == b.build_chunk(v, l, 0)


def test_skiplist_slice(small_index):
    ix = small_index
    a = ix.attr_sorted()
    rng = np.random.default_rng(3)
    for _ in range(100):
        l, h = sorted(rng.integers(a.min() - 5, a.max() + 5, 2))
        got = ix.skiplist_range(l, h)
        lo, hi = np.searchsorted(a, l, "left"), np.searchsorted(a, h, "right")
        assert got.tolist() == list(range(lo, hi))


def test_sig_knng_inclusivity_theorem1():
    """Lemma 1 / Theorem 1 (Sec. 3.2) on the oracle's exact range search: the k-NN
    graph of every union of contiguous segments (what a range query selects) is
    contained in the segmented k-NN graph, each object's exact k-NN in every
    segment.  Both sides come from the oracle's pre-filter search, so a slice that
    drops or adds an object at a segment edge breaks the containment."""
    rng = np.random.default_rng(4)
    n, S, k, d = 48, 4, 3, 4
    X = rng.standard_normal((n, d)).astype(np.float32)
    attr = rng.permutation(n).astype(np.int64)
    ix = hsig.Index.build(X, attr, 1.0 - rng.random(n), S, 4, 16)
    ss, _, _ = ix.segments()
    a = ix.attr_sorted()
    lo_attr = [int(a[ss[j]]) for j in range(S)]
    hi_attr = [int(a[ss[j + 1] - 1]) for j in range(S)]

    def knn_in(j0, j1):
        # k nearest other objects of every object among segments j0..j1 (k + 1 with itself)
        ids, _ = ix.search(X, np.full(n, lo_attr[j0]), np.full(n, hi_attr[j1]), k + 1, k + 1,
                           strategy=hsig.PRE)
        return [set(int(t) for t in row if t >= 0 and t != v) for v, row in enumerate(ids)], ids

    per_seg = [knn_in(j, j)[0] for j in range(S)]
    F = [set().union(*(per_seg[j][v] for j in range(S))) for v in range(n)]
    seg_of = np.searchsorted(ss, np.argsort(np.lexsort((np.arange(n), attr))), side="right") - 1
    checked = 0
    for j0 in range(S):
        for j1 in range(j0, S):
            _, ids = knn_in(j0, j1)
            for v in range(n):
                if not j0 <= seg_of[v] <= j1:
                    continue
                got = [int(t) for t in ids[v] if t >= 0 and t != v][:k]
                assert set(got) <= F[v], (j0, j1, v)
                checked += 1
    assert checked == n * sum(j1 - j0 + 1 for j0 in range(S) for j1 in range(j0, S)) // S


def test_inclusiveness_vs_multi_segment_hnsw():
    # Sec. 5.4: HNSWs built over 1, 2, 4, 6 and 8 contiguous segments of an S = 8
    # HSIG share, on average, more than 80% of their edges with the HSIG.
    spec = w.scaled(w.SPECS["hybrid10k"], n=4000, nq=1)
    W = w.make(spec, base_seed=21)
    S, M, ef = 8, 16, 100
    hs = hsig.Index.build(W.base, W.attr, W.level_u, S, M, ef)
    order = np.lexsort((np.arange(spec.n), W.attr))          # external ids in attribute order
    per = spec.n // S
    vals = []
    for width in (1, 2, 4, 6, 8):
        sub = order[: width * per]
        sub_sorted = np.sort(sub)                               # insertion order = external id order
        h = hsig.Index.build(W.base[sub_sorted], W.attr[sub_sorted], W.level_u[sub_sorted], 1, M, ef, hnsw=True)
        common = total = 0
        for loc, v in enumerate(sub_sorted):
            for l in range(h.build_level(loc) + 1):
                he = {int(sub_sorted[t]) for t in h.build_chunk(loc, l, 0)}
                se = set()
                for j in range(width):
                    se |= set(hs.build_chunk(int(v), l, j))
                total += len(he)
                common += len(he & se)
        vals.append(common / total)
    # One segment: chunk 0 of segment-0 objects evolves exactly like that HNSW.
    assert vals[0] == 1.0
    assert np.mean(vals) > 0.8, vals


def test_file_round_trip_and_rejection(small_index, small_workload, tmp_path):
    W = small_workload
    p = str(tmp_path / "ix.bin")
    small_index.write(p)
    rd = hsig.Index.read(p)
    for name in ("attr_sorted", "ext_ids", "levels"):
        assert np.array_equal(getattr(rd, name)(), getattr(small_index, name)())
    for l in range(small_index.L + 1):
        for A, B in zip(rd.layer(l), small_index.layer(l)):
            assert np.array_equal(A, B)
    a = small_index.search(W.queries, W.l, W.h, 10, 64)
    b = rd.search(W.queries, W.l, W.h, 10, 64)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    raw = open(p, "rb").read()
    bad = bytearray(raw)
    bad[len(raw) // 2] ^= 0x40
    open(p, "wb").write(bytes(bad))
    with pytest.raises(RuntimeError):
        hsig.Index.read(p)
    open(p, "wb").write(raw[:-100])
    with pytest.raises(RuntimeError):
        hsig.Index.read(p)
    bad = bytearray(raw)
    bad[0:8] = b"NOTANIDX"
    open(p, "wb").write(bytes(bad))
    with pytest.raises(RuntimeError):
        hsig.Index.read(p)


def test_index_size_formula(small_index, tmp_path):
    # Sec. 4.3: per node and level, M S edge slots, M S / 32 bitmap words and one
    # successor (implicit here: internal ids follow attribute order).  The file holds
    # exactly those tables plus the vectors and per-node attribute/id/level/row data.
    ix = small_index
    p = str(tmp_path / "ix.bin")
    ix.write(p)
    lev = ix.levels()
    node_levels = int((lev + 1).sum())
    units = node_levels * ix.S * ix.MU + node_levels * ((ix.S * ix.MU + 31) // 32)
    per_node = ix.n * (8 + 8 + 1 + 4) + ix.n * ix.d * 4
    expect = 256 + 4 * units + per_node + 8 * (ix.S + 1) + 8 * ix.S + 4
    size = os.path.getsize(p)
    assert expect <= size <= expect + 13 * 64
