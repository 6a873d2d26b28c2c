"""Disjunctive two-attribute queries on the GPU: the merge kernel against the
oracle's merge (bit for bit, with shared objects and equal distances), and the
whole path -- one index per attribute, each searched with its range, merged --
against the oracle on the same two index files."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import hsig
from synth import workloads as w


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


def test_merge_kernel_matches_oracle():
    torch = _torch()
    import paper_2412_02448_amd as u
    rng = np.random.default_rng(31)
    dev = torch.device("cuda", 0)
    for nq, k in ((1, 1), (257, 10), (300, 64)):
        ia = np.full((nq, k), -1, np.int64)
        ib = np.full((nq, k), -1, np.int64)
        da = np.full((nq, k), np.inf, np.float32)
        db = np.full((nq, k), np.inf, np.float32)
        for q in range(nq):
            pool = rng.choice(10 * k + 10, 2 * k, replace=False)
            dist = rng.integers(0, 3 * k, 2 * k).astype(np.float32) / 4  # many equal distances
            na, nb = rng.integers(0, k + 1), rng.integers(0, k + 1)
            sa = rng.choice(2 * k, na, replace=False)
            sb = rng.choice(2 * k, nb, replace=False)  # overlaps sa: shared objects, same distance
            for arr_i, arr_d, sel in ((ia, da, sa), (ib, db, sb)):
                o = sorted(sel, key=lambda j: (dist[j], rng.random()))  # ties in any order, as two indexes give
                arr_i[q, : len(o)] = pool[o]
                arr_d[q, : len(o)] = dist[o]
        oi, od = hsig.merge_or(ia, da, ib, db)
        gi, gd = u.merge_or((torch.from_numpy(ia).to(dev), torch.from_numpy(da).to(dev)),
                            (torch.from_numpy(ib).to(dev), torch.from_numpy(db).to(dev)))
        torch.cuda.synchronize()
        assert np.array_equal(gi.cpu().numpy(), oi)
        assert np.array_equal(gd.cpu().numpy().view(np.uint32), od.view(np.uint32))


@pytest.mark.parametrize("strategy", [hsig.AUTO, hsig.PRE, hsig.HYBRID])
def test_disjunctive_search_matches_oracle(tmp_path, strategy):
    torch = _torch()
    import paper_2412_02448_amd as u
    spec = w.scaled(w.SPECS["hybrid10k"], n=5000, nq=200)
    W = w.make(spec, base_seed=33)
    a2, l2, h2 = w.second_attribute(spec.n, len(W.queries), base_seed=33, f_lo=0.001, f_hi=0.2)
    ox = hsig.Index.build(W.base, W.attr, W.level_u, spec.S, spec.M, spec.ef_cons)
    oy = hsig.Index.build(W.base, a2, W.level_u, spec.S, spec.M, spec.ef_cons)
    px, py = str(tmp_path / "x.uix"), str(tmp_path / "y.uix")
    ox.write(px)
    oy.write(py)
    print(f"[case] disjunctive strategy={strategy}", flush=True)
    gx, gy = u.Index.load(px, device=0), u.Index.load(py, device=0)
    dev = torch.device("cuda", 0)
    Q = torch.from_numpy(W.queries).to(dev)
    st = None if strategy == hsig.AUTO else strategy
    ra = gx.search(Q, torch.from_numpy(W.l).to(dev), torch.from_numpy(W.h).to(dev), 10, 40, strategy=st)
    rb = gy.search(Q, torch.from_numpy(l2).to(dev), torch.from_numpy(h2).to(dev), 10, 40, strategy=st)
    gi, gd = u.merge_or(ra[:2], rb[:2])
    torch.cuda.synchronize()
    xa = ox.search(W.queries, W.l, W.h, 10, 40, strategy=strategy)
    xb = oy.search(W.queries, l2, h2, 10, 40, strategy=strategy)
    oi, od = hsig.merge_or(xa[0], xa[1], xb[0], xb[1])
    assert np.array_equal(gi.cpu().numpy(), oi)
    assert np.array_equal(gd.cpu().numpy().view(np.uint32), od.view(np.uint32))
    gx.close()
    gy.close()
