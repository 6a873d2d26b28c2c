"""The builder's Prune (Sec. 2.2; the selection step of Alg. 4 and Alg. 5) on the GPU
against the oracle's Prune, candidate list for candidate list.

Vectors sit on a small integer grid, so every squared distance is an integer that FP32
(the GPU) and FP64 (the oracle) both hold exactly, and ties are frequent: the GPU's
(distance, id) order and the oracle's (distance, position) order agree because each
candidate list is passed in ascending id order.  Shapes cover the kernel's three
variants: kept vectors in registers (M <= 32, d <= 256), the wider register variant
(M <= 64, d <= 128) and kept vectors read from memory (larger d)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import hsig


@pytest.mark.parametrize("d,M", [(8, 8), (64, 24), (128, 48), (256, 32), (300, 24), (960, 16)])
def test_prune_equals_oracle(d, M):
    import torch
    import paper_2412_02448_amd as u
    assert torch.cuda.is_available()
    rng = np.random.default_rng(d * 100 + M)
    n, t = 3000, 400
    X = rng.integers(-3, 4, size=(n, d)).astype(np.float32)
    owners = rng.integers(0, n, t).astype(np.int32)
    c = 160
    cand = np.full((t, c), -1, np.int32)
    for i in range(t):
        cnt = int(rng.integers(1, c + 1)) if i % 5 else c  # ragged lists, some full
        ids = rng.choice(np.delete(np.arange(n), owners[i]), cnt, replace=False)
        cand[i, :cnt] = np.sort(ids)
    dev = torch.device("cuda", 0)
    print(f"[case] prune d={d} M={M}", flush=True)
    got = u.prune(torch.from_numpy(X).to(dev), torch.from_numpy(owners).to(dev), torch.from_numpy(cand).to(dev), M)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    for i in range(t):
        ids = cand[i][cand[i] >= 0]
        sel = hsig.prune(X[owners[i]], X[ids], M)
        want = np.full(M, -1, np.int32)
        want[:len(sel)] = ids[sel]
        assert np.array_equal(got[i], want), (i, got[i], want)


def test_prune_edge_cases():
    """The owner among its own candidates and repeated ids are dropped; a task with no
    candidate keeps none; t = 0 is a no-op; sizes out of range are refused."""
    import torch
    import paper_2412_02448_amd as u
    dev = torch.device("cuda", 0)
    X = torch.tensor([[0, 0, 0, 0], [1, 0, 0, 0], [2, 0, 0, 0], [0, 3, 0, 0]], dtype=torch.float32, device=dev)
    owners = torch.tensor([0, 1, 2], dtype=torch.int32, device=dev)
    cand = torch.tensor([[0, 1, 1, 2, 3], [-1, -1, -1, -1, -1], [0, 1, 2, 3, -1]], dtype=torch.int32, device=dev)
    got = u.prune(X, owners, cand, 3).cpu().numpy()
    # owner 0: 1 (d=1) kept; 2 (d=4) dropped, as 1 is nearer to it (1 < 4); 3 (d=9) kept (d(1,3)=10 >= 9)
    assert got[0].tolist() == [1, 3, -1]
    assert got[1].tolist() == [-1, -1, -1]
    # owner 2: 1 (d=1) kept; 0 (d=4): d(1,0)=1 < 4, dropped; 3 (d=13): d(1,3)=10 < 13, dropped
    assert got[2].tolist() == [1, -1, -1]
    empty = torch.empty((0, 5), dtype=torch.int32, device=dev)
    assert u.prune(X, owners[:0], empty, 3).shape == (0, 3)
    with pytest.raises(u.UnifyError):
        u.prune(X, owners, cand, 65)
