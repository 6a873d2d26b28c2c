"""Pins of disjunctive two-attribute queries (the paper's multi-attribute
extension, approach 1: one HSIG per attribute, results merged): the merge of two
exact pre-filter answers is the brute-force answer of the OR query, and the merge
itself drops an object found by both searches."""
import numpy as np

from oracle import hsig
from synth import workloads as w


def test_merge_of_exact_answers_is_brute_force(small_workload):
    W = small_workload
    s = W.spec
    n = len(W.attr)
    a2, l2, h2 = w.second_attribute(n, len(W.queries), base_seed=8, f_lo=0.001, f_hi=0.05)
    ia = hsig.Index.build(W.base, W.attr, W.level_u, s.S, s.M, s.ef_cons)
    ib = hsig.Index.build(W.base, a2, W.level_u, s.S, s.M, s.ef_cons)
    k = 10
    ra = ia.search(W.queries, W.l, W.h, k, k, strategy=hsig.PRE)
    rb = ib.search(W.queries, l2, h2, k, k, strategy=hsig.PRE)
    ids, dist = hsig.merge_or(ra[0], ra[1], rb[0], rb[1])
    bound = (W.base.shape[1] / 16 + 8) * 2.0 ** -24
    both = 0
    for i in range(len(W.queries)):
        ok = ((W.attr >= W.l[i]) & (W.attr <= W.h[i])) | ((a2 >= l2[i]) & (a2 <= h2[i]))
        idx = np.nonzero(ok)[0]
        d = ((W.base[idx].astype(np.float64) - W.queries[i].astype(np.float64)) ** 2).sum(1)
        o = np.lexsort((idx, d))[:k]
        assert ids[i, : len(o)].tolist() == idx[o].tolist()
        np.testing.assert_array_less(np.abs(dist[i, : len(o)] - d[o]), bound * d[o] + 1e-30)
        both += len(set(ra[0][i]) & set(rb[0][i]) - {-1})
    assert both > 0  # some objects come from both searches and appear once


def test_merge_special_cases():
    ia = np.array([[1, 2, -1], [4, -1, -1]])
    da = np.array([[0.5, 1.0, np.inf], [2.0, np.inf, np.inf]], np.float32)
    ib = np.array([[2, 3, 1], [-1, -1, -1]])
    db = np.array([[1.0, 1.0, 1.5], [np.inf, np.inf, np.inf]], np.float32)
    ids, dist = hsig.merge_or(ia, da, ib, db)
    # object 2 appears in both lists at distance 1.0 and once in the result; the third
    # slot goes to object 3 (distance 1.0) before b's 1.5
    assert ids.tolist() == [[1, 2, 3], [4, -1, -1]]
    assert dist.tolist()[0] == [0.5, 1.0, 1.0]
