"""Pins of conjunctive two-attribute queries in the reference search (the paper's
multi-attribute extension, approach 1: the HSIG indexes the first attribute and
the filter of Alg. 7 -- its ann admission -- and the post-filter test both).

Pinned against: brute force over the objects satisfying both ranges (the
pre-filter), the single-attribute search when the second range admits every
object, and the ranges of every returned object."""
import numpy as np
import pytest

from oracle import hsig
from synth import workloads as w


@pytest.fixture(scope="module")
def multi(small_index, small_workload):
    W = small_workload
    a2, l2, h2 = w.second_attribute(len(W.attr), len(W.queries), base_seed=4)
    small_index.set_attr2(a2)
    return small_index, W, a2, l2, h2


def _brute(W, a2, i, l2, h2, k):
    ok = (W.attr >= W.l[i]) & (W.attr <= W.h[i]) & (a2 >= l2) & (a2 <= h2)
    idx = np.nonzero(ok)[0]
    d = ((W.base[idx].astype(np.float64) - W.queries[i].astype(np.float64)) ** 2).sum(1)
    o = np.lexsort((idx, d))[:k]
    return idx[o], d[o]


def test_pre_filter_is_brute_force(multi):
    ix, W, a2, l2, h2 = multi
    ids, dist = ix.search(W.queries, W.l, W.h, 10, 10, strategy=hsig.PRE, l2=l2, h2=h2)
    bound = (W.base.shape[1] / 16 + 8) * 2.0 ** -24
    for i in range(len(W.queries)):
        tid, td = _brute(W, a2, i, l2[i], h2[i], 10)
        assert ids[i, : len(tid)].tolist() == tid.tolist()
        assert (ids[i, len(tid):] == -1).all()
        np.testing.assert_array_less(np.abs(dist[i, : len(tid)] - td), bound * td + 1e-30)


@pytest.mark.parametrize("strategy", [hsig.AUTO, hsig.PRE, hsig.HYBRID, hsig.POST])
def test_full_second_range_is_single_attribute(multi, strategy):
    ix, W, a2, _, _ = multi
    lo = np.full(len(W.queries), a2.min())
    hi = np.full(len(W.queries), a2.max())
    a = ix.search(W.queries, W.l, W.h, 10, 48, p=2, strategy=strategy)
    b = ix.search(W.queries, W.l, W.h, 10, 48, p=2, strategy=strategy, l2=lo, h2=hi)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("strategy", [hsig.AUTO, hsig.HYBRID, hsig.POST])
def test_results_satisfy_both_ranges(multi, strategy):
    ix, W, a2, l2, h2 = multi
    ids, dist = ix.search(W.queries, W.l, W.h, 10, 64, strategy=strategy, l2=l2, h2=h2)
    rec = []
    for i in range(len(W.queries)):
        row = ids[i][ids[i] >= 0]
        assert np.all((W.attr[row] >= W.l[i]) & (W.attr[row] <= W.h[i]))
        assert np.all((a2[row] >= l2[i]) & (a2[row] <= h2[i]))
        d32 = np.array([hsig.dist32(W.queries[i], W.base[e]) for e in row], np.float32)
        assert np.array_equal(d32, dist[i][: len(row)])
        tid, _ = _brute(W, a2, i, l2[i], h2[i], 10)
        if len(tid):
            rec.append(len(set(row.tolist()) & set(tid.tolist())) / len(tid))
    if strategy == hsig.HYBRID:
        assert np.mean(rec) > 0.85


def test_empty_second_range_and_errors(multi, small_workload):
    ix, W, a2, l2, h2 = multi
    ids, dist = ix.search(W.queries, W.l, W.h, 10, 32, l2=h2 + 1, h2=h2)  # l2 > h2: nothing qualifies
    assert (ids == -1).all() and np.isinf(dist).all()
    with pytest.raises(ValueError):
        ix.search(W.queries, W.l, W.h, 10, 32, l2=l2)
    with pytest.raises(ValueError):
        ix.set_attr2(a2[:-1])
    fresh = hsig.Index.build(W.base[:300], W.attr[:300], W.level_u[:300], 4, 8, 32)
    with pytest.raises(ValueError):
        fresh.search(W.queries[:2], W.l[:2], W.h[:2], 10, 32, l2=l2[:2], h2=h2[:2])


def test_strategy_rule_uses_joint_estimate(multi):
    """The rule for conjunctive queries compares Y * c2 / ns with tau_A and tau_B (c2 of
    the ns sample values of the second attribute lie in its range): a second range that
    admits everything keeps the single-attribute choice, an empty one makes every query
    a pre-filter scan, and a narrow one never turns a query into a post-filter search."""
    ix, W, a2, l2, h2 = multi
    nq = len(W.queries)
    _, _, c0 = ix.search(W.queries, W.l, W.h, 10, 32, counters=True)
    lo, hi = np.full(nq, a2.min()), np.full(nq, a2.max())
    _, _, c1 = ix.search(W.queries, W.l, W.h, 10, 32, counters=True, l2=lo, h2=hi)
    assert np.array_equal(c0[:, hsig.STRAT], c1[:, hsig.STRAT])
    _, _, ce = ix.search(W.queries, W.l, W.h, 10, 32, counters=True, l2=hi, h2=lo)
    Y = ce[:, hsig.HI] - ce[:, hsig.LO]
    assert (ce[Y > 0, hsig.STRAT] == hsig.PRE).all()
    srt = np.sort(a2)
    narrow_l = np.full(nq, srt[len(srt) // 2])
    narrow_h = np.full(nq, srt[len(srt) // 2 + len(srt) // 100])  # about 1% of the objects
    _, _, cn = ix.search(W.queries, W.l, W.h, 10, 32, counters=True, l2=narrow_l, h2=narrow_h)
    assert (cn[:, hsig.STRAT] != hsig.POST).all()
    assert (cn[c0[:, hsig.STRAT] == hsig.PRE, hsig.STRAT] == hsig.PRE).all()
