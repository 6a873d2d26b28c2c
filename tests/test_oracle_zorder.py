"""Pins of the z-order composite attribute in the reference (the paper's
multi-attribute extension, approach 2: one HSIG over a z-order key of the pair
(A1, A2), searched on the key range of a query box with the box test at Alg. 7's
ann admission, the post-filter test and the pre-filter scan).

Pinned against: the quadtree (base-4 digit) address of a grid cell, the recursive
quadrant enumeration of a small grid, hand-computed key maps (spans at the 2^31
boundary and the full int64 range), brute-force containment of every box object in
the searched key range, brute-force box answers (pre-filter), the unfiltered search
when the box holds every object, and the box membership of every returned object.
Each test names the mistake it catches."""
import numpy as np
import pytest

from oracle import hsig
from synth import workloads as w

I64_MIN, I64_MAX = -(1 << 63), (1 << 63) - 1


def _quad_address(u1: int, u2: int) -> int:
    # the cell's address in the quadtree of the 2^31 x 2^31 grid: one base-4 digit per
    # level from the root, the A1 half (0 / 1) times 2 plus the A2 half
    a = 0
    for j in range(30, -1, -1):
        a = 4 * a + 2 * ((u1 >> j) & 1) + ((u2 >> j) & 1)
    return a


def test_keys_are_quadtree_addresses():
    # catches: swapped coordinate roles, bits placed one position off, a dropped top level
    rng = np.random.default_rng(5)
    u1 = rng.integers(0, 1 << 31, 400, dtype=np.int64)
    u2 = rng.integers(0, 1 << 31, 400, dtype=np.int64)
    u1[:4] = [0, (1 << 31) - 1, 0, (1 << 31) - 1]
    u2[:4] = [0, 0, (1 << 31) - 1, (1 << 31) - 1]
    zmap = np.array([0, 0, 0, 0], np.int64)  # base 0, shift 0: the coordinates are the values
    keys = hsig.zorder_keys(zmap, u1, u2)
    for a, b, z in zip(u1.tolist(), u2.tolist(), keys.tolist()):
        assert z == _quad_address(a, b)
    assert keys[3] == (1 << 62) - 1 and keys.min() >= 0


def test_small_grid_follows_recursive_quadrants():
    # catches: an order that is not the Z curve (row-major, or A2 as the major half)
    def quads(x0, y0, size):
        if size == 1:
            yield (x0, y0)
            return
        h = size // 2
        for dx, dy in ((0, 0), (0, 1), (1, 0), (1, 1)):
            yield from quads(x0 + dx * h, y0 + dy * h, h)

    order = list(quads(0, 0, 16))
    x = np.array([p[0] for p in order], np.int64)
    y = np.array([p[1] for p in order], np.int64)
    keys = hsig.zorder_keys(np.zeros(4, np.int64), x, y)
    assert keys.tolist() == list(range(256))


def test_key_map_hand_cases():
    # catches: a base that is not the minimum, an off-by-one shift at the 2^31 boundary,
    # signed overflow of the span
    m = hsig.zorder_map(np.array([5, 7, 100]), np.array([-3, 4, 9]))
    assert m.tolist() == [5, -24, -3, -27]  # spans 95 (7 bits), 12 (4 bits)
    k = hsig.zorder_keys(m, np.array([100, 7, 1000]), np.array([9, -3, -4]))
    assert k[0] == _quad_address(95 << 24, 12 << 27)
    assert k[1] == _quad_address(2 << 24, 0)
    assert k[2] == _quad_address((1 << 31) - 1, 0)  # beyond the data: the axis's last cell
    m = hsig.zorder_map(np.array([10, 10 + (1 << 31) - 1]), np.array([0, 1 << 31]))
    assert m.tolist() == [10, 0, 0, 1]
    m = hsig.zorder_map(np.array([4, 4, 4]), np.array([0, 1, 1]))
    assert m.tolist() == [4, 0, 0, -30]  # one value only: every coordinate 0
    m = hsig.zorder_map(np.array([I64_MIN, I64_MAX]), np.array([-(1 << 40), 0]))
    assert m.tolist() == [I64_MIN, 33, -(1 << 40), 10]
    # coordinates: (x - base) >> shift, clamped to [0, 2^31 - 1]
    k = hsig.zorder_keys(m, np.array([I64_MIN, I64_MAX, 0]), np.array([-(1 << 40), 0, -(1 << 39)]))
    assert k[0] == 0
    assert k[1] == _quad_address((1 << 31) - 1, 1 << 30)
    assert k[2] == _quad_address(1 << 30, 1 << 29)
    # query bounds outside the data clamp to the grid's edges
    lo, hi = hsig.zorder_range(np.array([0, 0, 0, 0]), [-5], [I64_MAX], [-7], [1 << 40])
    assert lo[0] == 0 and hi[0] == (1 << 62) - 1
    lo, hi = hsig.zorder_range(np.array([0, -20, 0, -20]), [-5], [I64_MAX], [-7], [1 << 40])
    assert lo[0] == 0 and hi[0] == (1 << 62) - 1
    lo, hi = hsig.zorder_range(np.array([0, 0, 0, 0]), [3], [2], [0], [9])  # empty box
    assert lo[0] > hi[0]


@pytest.mark.parametrize("wide", [False, True])
def test_box_objects_lie_in_the_searched_key_range(wide):
    # catches: a key range that drops box objects (non-monotone coordinates, wrong corner,
    # rounding of shifted coordinates the wrong way)
    rng = np.random.default_rng(7 + wide)
    n = 3000
    if wide:
        a1 = rng.integers(-(1 << 45), 1 << 45, n, dtype=np.int64)
        a2 = rng.integers(I64_MIN // 2, I64_MAX // 2, n, dtype=np.int64)
    else:
        a1 = rng.integers(0, 500, n, dtype=np.int64)
        a2 = rng.integers(-1000, 1000, n, dtype=np.int64)
    m = hsig.zorder_map(a1, a2)
    assert (m[1] > 0 and m[3] > 0) if wide else (m[1] < 0 and m[3] < 0)
    keys = hsig.zorder_keys(m, a1, a2)
    nb = 300
    c1 = rng.choice(a1, (nb, 2))
    c2 = rng.choice(a2, (nb, 2))
    l1, h1 = c1.min(1), c1.max(1)
    l2, h2 = c2.min(1), c2.max(1)
    l1[:10] -= 1 << 20  # bounds outside the data
    h2[10:20] += 1 << 20
    lo, hi = hsig.zorder_range(m, l1, h1, l2, h2)
    for i in range(nb):
        inside = (a1 >= l1[i]) & (a1 <= h1[i]) & (a2 >= l2[i]) & (a2 <= h2[i])
        assert np.all((keys[inside] >= lo[i]) & (keys[inside] <= hi[i])), i


@pytest.fixture(scope="module")
def zindex(small_workload):
    W = small_workload
    s = W.spec
    a2, l2, h2 = w.second_attribute(len(W.attr), len(W.queries), base_seed=6)
    m = hsig.zorder_map(W.attr, a2)
    z = hsig.zorder_keys(m, W.attr, a2)
    ix = hsig.Index.build(W.base, z, W.level_u, s.S, s.M, s.ef_cons, seed=11)
    ix.set_zorder(m, W.attr, a2)
    return ix, W, m, z, a2, l2, h2


def _brute(W, a2, i, l1, h1, l2, h2, k):
    ok = (W.attr >= l1) & (W.attr <= h1) & (a2 >= l2) & (a2 <= h2)
    idx = np.nonzero(ok)[0]
    d = ((W.base[idx].astype(np.float64) - W.queries[i].astype(np.float64)) ** 2).sum(1)
    o = np.lexsort((idx, d))[:k]
    return idx[o], d[o]


def test_pre_filter_box_is_brute_force(zindex):
    # catches: a box test that checks one attribute only, or the key range instead of the box
    ix, W, m, z, a2, l2, h2 = zindex
    ids, dist = ix.search_box(W.queries, W.l, W.h, l2, h2, 10, 10, strategy=hsig.PRE)
    bound = (W.base.shape[1] / 16 + 8) * 2.0 ** -24
    for i in range(len(W.queries)):
        tid, td = _brute(W, a2, i, W.l[i], W.h[i], l2[i], h2[i], 10)
        assert ids[i, : len(tid)].tolist() == tid.tolist()
        assert (ids[i, len(tid):] == -1).all()
        np.testing.assert_array_less(np.abs(dist[i, : len(tid)] - td), bound * td + 1e-30)


@pytest.mark.parametrize("strategy", [hsig.PRE, hsig.HYBRID, hsig.POST])
def test_full_box_is_the_unfiltered_key_search(zindex, strategy):
    # catches: a box test that rejects objects on the box's edges; a key range that is not
    # the corners' keys
    ix, W, m, z, a2, _, _ = zindex
    nq = len(W.queries)
    l1 = np.full(nq, W.attr.min())
    h1 = np.full(nq, W.attr.max())
    lo2 = np.full(nq, a2.min())
    hi2 = np.full(nq, a2.max())
    a = ix.search(W.queries, np.full(nq, z.min()), np.full(nq, z.max()), 10, 48, p=2, strategy=strategy)
    b = ix.search_box(W.queries, l1, h1, lo2, hi2, 10, 48, p=2, strategy=strategy)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("strategy", [hsig.AUTO, hsig.HYBRID, hsig.POST])
def test_box_results_lie_in_the_box(zindex, strategy):
    # catches: the filter of Alg. 7 or of the post-filter admitting key-range objects outside
    # the box
    ix, W, m, z, a2, l2, h2 = zindex
    ids, dist, cnt = ix.search_box(W.queries, W.l, W.h, l2, h2, 10, 64, p=2, strategy=strategy, counters=True)
    rec = []
    for i in range(len(W.queries)):
        row = ids[i][ids[i] >= 0]
        assert np.all((W.attr[row] >= W.l[i]) & (W.attr[row] <= W.h[i]))
        assert np.all((a2[row] >= l2[i]) & (a2[row] <= h2[i]))
        assert np.all(np.diff(dist[i][ids[i] >= 0]) >= 0)
        tid, _ = _brute(W, a2, i, W.l[i], W.h[i], l2[i], h2[i], 10)
        if len(tid):
            rec.append(len(set(tid.tolist()) & set(row.tolist())) / len(tid))
    if strategy == hsig.AUTO:
        assert np.mean(rec) >= 0.9, np.mean(rec)


def test_strategy_rule_extremes(zindex):
    # catches: the rule reading the key range instead of the box estimate (a tiny box whose
    # key range is wide), or the full box not reaching the post-filter
    ix, W, m, z, a2, _, _ = zindex
    nq = len(W.queries)
    # the full box: every sampled pair is inside
    _, _, cnt = ix.search_box(W.queries, np.full(nq, W.attr.min()), np.full(nq, W.attr.max()),
                              np.full(nq, a2.min()), np.full(nq, a2.max()), 10, 32, counters=True)
    assert (cnt[:, hsig.STRAT] == hsig.POST).all()
    # boxes one A2 value wide across A1's whole span: their key ranges hold far more than
    # tau_a n objects, but the box holds one object, so the rule pre-filters
    v = np.sort(a2)[len(a2) // 2]
    ids, _, cnt = ix.search_box(W.queries, np.full(nq, W.attr.min()), np.full(nq, W.attr.max()),
                                np.full(nq, v), np.full(nq, v), 10, 32, counters=True)
    assert ((cnt[:, hsig.HI] - cnt[:, hsig.LO]) > 0.01 * len(z)).all()
    assert (cnt[:, hsig.STRAT] == hsig.PRE).all()
    want = np.nonzero(a2 == v)[0]
    assert set(ids[0][ids[0] >= 0].tolist()) <= set(want.tolist()) and (ids[0] >= 0).sum() == min(10, want.size)


def test_errors(zindex, small_workload):
    ix, W, m, z, a2, l2, h2 = zindex
    with pytest.raises(ValueError):  # swapped attributes: the index is not built on their keys
        ix.set_zorder(m, a2, W.attr)
    plain = hsig.Index.build(W.base[:200], W.attr[:200], W.level_u[:200], 2, 8, 32, seed=1)
    with pytest.raises(ValueError):  # no z-order attributes
        plain.search_box(W.queries[:2], W.l[:2], W.h[:2], l2[:2], h2[:2], 10, 16)
    # an empty box (l1 > h1): padded rows
    ids, dist = ix.search_box(W.queries[:3], W.h[:3] + 1, W.h[:3], l2[:3], h2[:3], 10, 16)
    assert (ids == -1).all() and np.isinf(dist).all()
