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


def test_pick_best_rule():
    """Among the settings reaching the target, those within 2% of the fastest tie; the smallest
    beam width wins, then the more accurate, then the faster."""
    S = autotune.Setting
    table = [S(64, 16, 6, 0.9694, 12.14e6), S(64, 16, 4, 0.9673, 12.08e6), S(64, 16, 2, 0.9645, 11.1e6),
             S(64, 16, 8, 0.9713, 11.3e6), S(32, 16, 3, 0.94, 13e6)]  # the last misses the target
    assert autotune.pick_best(table, 0.953) == table[1]  # p = 2 is 8.6% slower: outside the tie
    table.append(S(96, 16, 4, 0.9690, 12.0e6))  # same beam width, more accurate, within 2%
    assert autotune.pick_best(table, 0.953) == table[-1]
    assert autotune.pick_best(table, 0.99) is None
    assert autotune.pick_best([S(64, 16, 4, 0.97, 0.0)], 0.95) is None  # recall-only rows carry no timing
