"""TEST INFRASTRUCTURE -- NOT PART OF THE PRODUCT.

The plain definitions the search approximates, in FP64:

* exact range-filtered k-NN (Definition 1, Sec. 2.1): R = {v : l <= v[A] <= h};
  return the k objects of R nearest to q, all of R when |R| < k.  Ties in
  distance are broken by the smaller identifier (the definition's strict "<"
  leaves tied sets open); squared Euclidean distance gives the same order as
  Euclidean distance (Sec. 5.1).
* recall (Eq. 1): |kNN' intersect kNN| / min(k, |R|); 1 when R is empty.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this module.
"""
from __future__ import annotations

import numpy as np


def sqdist64(q: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Squared Euclidean distances from q to every row of X, in FP64."""
    diff = X.astype(np.float64) - q.astype(np.float64)[None, :]
    return np.einsum("ij,ij->i", diff, diff)


def rfknn(X: np.ndarray, attr: np.ndarray, q: np.ndarray, l: int, h: int, k: int,
          ids: np.ndarray | None = None):
    """Exact range-filtered k-NN of one query (Definition 1).

    X, attr are indexed by object; ids[i] is the identifier used for ties and
    returned (default: the row number).  Returns (ids, distances) of length
    min(k, |R|), ascending by (distance, id).
    """
    if ids is None:
        ids = np.arange(X.shape[0], dtype=np.int64)
    sel = np.nonzero((attr >= l) & (attr <= h))[0]
    if sel.size == 0:
        return np.zeros(0, np.int64), np.zeros(0, np.float64)
    dist = sqdist64(q, X[sel])
    order = np.lexsort((ids[sel], dist))[:k]
    return ids[sel][order], dist[order]


def rfknn_sorted(Xs: np.ndarray, attr_sorted: np.ndarray, q: np.ndarray, l: int, h: int, k: int,
                 ids: np.ndarray):
    """The same on a store already ordered by attribute: the in-range objects are one slice."""
    lo = int(np.searchsorted(attr_sorted, l, side="left"))
    hi = int(np.searchsorted(attr_sorted, h, side="right"))
    if l > h or hi <= lo:
        return np.zeros(0, np.int64), np.zeros(0, np.float64), 0
    dist = sqdist64(q, Xs[lo:hi])
    order = np.lexsort((ids[lo:hi], dist))[:k]
    return ids[lo:hi][order], dist[order], hi - lo


def recall(found, truth, k: int, size_R: int) -> float:
    """Eq. 1: |found intersect truth| / min(k, |R|); 1 when R is empty."""
    denom = min(k, size_R)
    if denom == 0:
        return 1.0
    f = {int(x) for x in found if int(x) >= 0}
    t = {int(x) for x in truth if int(x) >= 0}
    return len(f & t) / denom
