"""Recall as the tuner computes it (Eq. 1: |found & exact| / min(k, |R|), a query
with an empty range counting 1), on hand-made rows."""
import numpy as np

from paper_2412_02448_amd import autotune


def test_recall_hand_cases():
    truth = np.array([[1, 2, 3, -1], [5, 6, 7, 8], [-1, -1, -1, -1], [9, -1, -1, -1]])
    ids = np.array([[3, 1, 4, -1], [8, 7, 6, 5], [2, -1, -1, -1], [-1, -1, -1, -1]])
    # rows: 2/3, 4/4, empty range -> 1, 0/1
    assert autotune.recall_at_k(ids, truth) == np.mean([2 / 3, 1.0, 1.0, 0.0])
    assert autotune.recall_at_k(ids[:0], truth[:0]) == 1.0


def test_recall_blocks_agree():
    rng = np.random.default_rng(3)
    nq, k = 3000, 64  # several blocks of comparisons
    truth = np.stack([rng.choice(500, k, replace=False) for _ in range(nq)])
    ids = np.stack([rng.choice(500, k, replace=False) for _ in range(nq)])
    ids[::7, k // 2:] = -1
    ref = np.mean([len(set(ids[i][ids[i] >= 0]) & set(truth[i])) / k for i in range(nq)])
    assert abs(autotune.recall_at_k(ids, truth) - ref) < 1e-12
