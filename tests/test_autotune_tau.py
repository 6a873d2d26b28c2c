"""The strategy-threshold calibration of Sec. 4.2 ("Range-aware Strategy Selection"):
turning points from per-bucket recall and latency records, on hand-made tables, and
the random ranges the calibration samples."""
import numpy as np

from paper_2412_02448_amd import autotune


def _table(pre, hyb, post, rec_h=None, rec_p=None):
    nb = len(pre)
    rec = {"pre": [1.0] * nb, "hybrid": rec_h or [1.0] * nb, "post": rec_p or [1.0] * nb}
    return rec, {"pre": pre, "hybrid": hyb, "post": post}


def test_turning_points_hand_cases():
    n = 1000
    y_lo = [1, 10, 100, 300, 600]
    y_hi = [9, 99, 299, 599, 1000]
    # pre fastest on the first two buckets, hybrid in the middle, post on the last
    rec, us = _table([1, 2, 9, 20, 40], [3, 3, 3, 3, 3], [9, 9, 5, 4, 1])
    ta, tb = autotune.turning_points(y_lo, y_hi, rec, us, 0.9, n)
    assert int(np.floor(ta * n)) == 99 and int(np.ceil(tb * n)) == 600
    # hybrid misses the target on the last two buckets: post takes them even when slower
    rec, us = _table([1, 2, 9, 20, 40], [3, 3, 3, 3, 3], [9, 9, 5, 4, 4], rec_h=[1, 1, 1, 0.5, 0.5])
    ta, tb = autotune.turning_points(y_lo, y_hi, rec, us, 0.9, n)
    assert int(np.ceil(tb * n)) == 300
    # a post bucket below a hybrid one is not a turning point: post must win every bucket above it
    rec, us = _table([1, 5, 9, 20, 40], [3, 3, 3, 3, 3], [9, 1, 5, 1, 1])
    ta, tb = autotune.turning_points(y_lo, y_hi, rec, us, 0.9, n)
    assert int(np.floor(ta * n)) == 9 and int(np.ceil(tb * n)) == 300
    # pre wins everywhere: no hybrid or post zone
    rec, us = _table([1, 1, 1, 1, 1], [3, 3, 3, 3, 3], [9, 9, 9, 9, 9])
    ta, tb = autotune.turning_points(y_lo, y_hi, rec, us, 0.9, n)
    assert ta == 1.0 and tb == 1.0
    # post wins everywhere and pre nowhere: tau_A = 0, post from the smallest bucket
    rec, us = _table([9, 9, 9, 9, 9], [3, 3, 3, 3, 3], [1, 1, 1, 1, 1])
    ta, tb = autotune.turning_points(y_lo, y_hi, rec, us, 0.9, n)
    assert 0.0 < ta and int(np.floor(ta * n)) == 0 and int(np.ceil(tb * n)) == 1
    # a tie goes to the cheaper-to-plan strategy of the edge (pre / post), not hybrid
    rec, us = _table([3, 3, 9, 9, 9], [3, 3, 3, 3, 3], [9, 9, 9, 9, 3])
    ta, tb = autotune.turning_points(y_lo, y_hi, rec, us, 0.9, n)
    assert int(np.floor(ta * n)) == 99 and int(np.ceil(tb * n)) == 600


def test_sample_ranges_hold_their_cardinality():
    rng = np.random.default_rng(4)
    attr = rng.integers(0, 500, 4000)  # many equal attributes
    l, h, y = autotune.sample_ranges(attr, 3000, np.random.default_rng(5))
    inr = (attr[None, :] >= l[:, None]) & (attr[None, :] <= h[:, None])
    assert np.array_equal(inr.sum(1), y)
    assert y.min() >= 1 and y.max() <= len(attr)
    # log-uniform fractions: every decade from 1/n to 1 is hit
    dec = np.floor(np.log10(y / len(attr)) + 1e-9)
    assert set(dec.tolist()) >= {-3.0, -2.0, -1.0}
