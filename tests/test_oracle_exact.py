"""Pins of the exact definitions (Definition 1, Eq. 1) and of the canonical FP32 distance."""
import math

import numpy as np
import pytest
from scipy.spatial.distance import cdist

from oracle import exact, hsig

U32 = 2.0 ** -24  # unit roundoff of FP32


def test_rfknn_hand_example():
    # Objects on a line (first coordinate), attribute = index.  Query at 2.2 in [1, 4].
    X = np.zeros((6, 4), np.float32)
    X[:, 0] = [0.0, 1.0, 2.0, 3.0, 4.0, 5.0]
    attr = np.arange(6)
    q = np.array([2.2, 0, 0, 0], np.float32)
    ids, d = exact.rfknn(X, attr, q, 1, 4, 3)
    assert ids.tolist() == [2, 3, 1]
    np.testing.assert_allclose(d, [0.04, 0.64, 1.44], rtol=1e-6)
    # object 0 and 5 are out of range even though 5 is not nearer than 1
    ids, _ = exact.rfknn(X, attr, q, 0, 5, 6)
    assert ids.tolist() == [2, 3, 1, 4, 0, 5]


def test_rfknn_ties_small_and_empty_ranges():
    X = np.zeros((5, 4), np.float32)
    X[:, 0] = [1.0, -1.0, 1.0, -1.0, 0.0]
    attr = np.array([10, 20, 30, 40, 50])
    q = np.zeros(4, np.float32)
    ids, d = exact.rfknn(X, attr, q, 10, 40, 2)       # four objects at distance 1: smaller ids first
    assert ids.tolist() == [0, 1]
    ids, d = exact.rfknn(X, attr, q, 15, 35, 10)      # |R| = 2 < k: all of R
    assert ids.tolist() == [1, 2]
    ids, d = exact.rfknn(X, attr, q, 21, 29, 10)      # no object in range
    assert ids.size == 0
    ids, d = exact.rfknn(X, attr, q, 40, 10, 10)      # l > h
    assert ids.size == 0


def test_rfknn_matches_library_distances():
    rng = np.random.default_rng(0)
    X = rng.standard_normal((300, 16)).astype(np.float32)
    attr = rng.integers(0, 50, 300)
    for t in range(20):
        q = rng.standard_normal(16).astype(np.float32)
        l, h = sorted(rng.integers(0, 50, 2))
        ids, d = exact.rfknn(X, attr, q, l, h, 7)
        sel = np.nonzero((attr >= l) & (attr <= h))[0]
        lib = cdist(q[None].astype(np.float64), X[sel].astype(np.float64), "sqeuclidean")[0]
        order = np.argsort(lib, kind="stable")[:7]      # sel is ascending, so stable = id tie-break
        assert ids.tolist() == sel[order].tolist()
        np.testing.assert_allclose(d, lib[order], rtol=1e-12)
        # the sorted-store form gives the same answer
        perm = np.lexsort((np.arange(300), attr))
        ids2, d2, Y = exact.rfknn_sorted(X[perm], attr[perm], q, l, h, 7, perm)
        assert ids2.tolist() == ids.tolist() and Y == sel.size


def test_recall_closed_forms():
    assert exact.recall([1, 2, 3], [1, 2, 3], 3, 100) == 1.0
    assert exact.recall([1, 2, 9], [1, 2, 3], 3, 100) == pytest.approx(2 / 3)
    assert exact.recall([5, -1, -1], [5], 3, 1) == 1.0          # |R| < k: denominator |R|
    assert exact.recall([-1, -1], [], 2, 0) == 1.0              # empty R
    assert exact.recall([7, 8], [1, 2], 2, 2) == 0.0


def test_dist32_exact_on_integers():
    # Small integer coordinates: every partial sum is an integer below 2^24,
    # so the canonical FP32 result equals the exact squared distance.
    rng = np.random.default_rng(1)
    for d in (4, 96, 128, 960):
        for _ in range(20):
            q = rng.integers(-20, 21, d).astype(np.float32)
            x = rng.integers(-20, 21, d).astype(np.float32)
            exact_val = int(((x.astype(np.int64) - q.astype(np.int64)) ** 2).sum())
            assert float(hsig.dist32(q, x)) == float(exact_val)
            assert hsig.dist64(q, x) == float(exact_val)


def test_dist32_summation_tree():
    # e_0 = 4096 (partial 0 holds 2^24) and e = 1 in groups 1 and 3 (partials 1 and 3).
    # The butterfly adds partials 1 and 3 first (= 2), then 2^24 + 2 is exact.
    # A left-to-right sum would round 2^24 + 1 back to 2^24 twice.
    d = 128
    q = np.zeros(d, np.float32)
    x = np.zeros(d, np.float32)
    x[0] = 4096.0
    x[4] = 1.0
    x[12] = 1.0
    assert float(hsig.dist32(q, x)) == 16777218.0
    # Moving the second 1 into group 2 (partial 2) makes the tree add 2^24 + 1 twice.
    x[12] = 0.0
    x[8] = 1.0
    assert float(hsig.dist32(q, x)) == 16777216.0


def test_dist32_error_bound_vs_fp64():
    rng = np.random.default_rng(2)
    for d in (96, 128, 960):
        bound = (d / 16 + 8) * U32
        for _ in range(200):
            q = rng.standard_normal(d).astype(np.float32)
            x = (q + 0.3 * rng.standard_normal(d)).astype(np.float32)
            a = float(hsig.dist32(q, x))
            b = hsig.dist64(q, x)
            assert abs(a - b) <= bound * b


def test_level_distribution():
    # Alg. 6: level = floor(-ln(U) mL) with mL = 1/ln(M) gives P(level >= l) = M^-l.
    from synth import workloads as w
    M = 16
    u = w.level_uniforms(200_000, 3)
    lv = np.array([hsig.level_of(x, M) for x in u[:200_000:4]])
    n = lv.size
    for l in (1, 2):
        p = M ** -l
        frac = (lv >= l).mean()
        assert abs(frac - p) <= 5 * math.sqrt(p * (1 - p) / n) + 1e-9
    assert hsig.level_of(1.0, M) == 0
    assert hsig.level_of(1.001 / M, M) == 0        # just above the level-1 edge U = 1/M
    assert hsig.level_of(0.999 / M, M) == 1
    assert hsig.level_of(1.0 / M ** 2 * 0.999, M) == 2
