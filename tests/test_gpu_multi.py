"""Conjunctive two-attribute queries on the GPU against the oracle (the paper's
multi-attribute extension, approach 1): identical ids and FP32 distances for
every strategy, both stores, split pre-filter scans, and the error paths."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import hsig
from synth import workloads as w


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


@pytest.fixture(scope="module")
def c1(tmp_path_factory):
    spec = w.SPECS["hybrid10k"]
    W = w.make(spec, base_seed=17)
    path = str(tmp_path_factory.mktemp("multi") / "m.uix")
    print(f"[fixture] oracle build {spec.name}", flush=True)
    ix = hsig.Index.build(W.base, W.attr, W.level_u, spec.S, spec.M, spec.ef_cons, seed=17)
    ix.write(path)
    a2, l2, h2 = w.second_attribute(spec.n, len(W.queries), base_seed=17)
    ix.set_attr2(a2)
    return W, ix, path, a2, l2, h2


def _dev(*arrs):
    torch = _torch()
    dev = torch.device("cuda", 0)
    return [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in arrs]


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("strategy", [hsig.AUTO, hsig.PRE, hsig.HYBRID, hsig.POST])
def test_parity_conjunctive(c1, precision, strategy):
    torch = _torch()
    import paper_2412_02448_amd as u
    W, ix, path, a2, l2, h2 = c1
    print(f"[case] conjunctive {precision} strategy={strategy}", flush=True)
    g = u.Index.load(path, device=0, precision=precision)
    g.set_attr2(a2)
    ix.set_store(hsig.BF16 if precision == "bf16" else hsig.FP32, 4)
    try:
        Q, L, H, L2, H2 = _dev(W.queries, W.l, W.h, l2, h2)
        for ef, p, chunk in ((48, 1, 0), (64, 2, 64)):
            rid, rd, rc = ix.search(W.queries, W.l, W.h, 10, ef, p=p, strategy=strategy, l2=l2, h2=h2, counters=True)
            ids, dist, srun, st = g.search(Q, L, H, 10, ef, beam_p=p, strategy=None if strategy == hsig.AUTO else strategy,
                                        stats=True, pre_chunk=chunk, l2=L2, h2=H2)
            torch.cuda.synchronize()
            assert ((st.cpu().numpy()[:, 3] & 0xFF) != 2).all()
            assert np.array_equal(srun.cpu().numpy().astype(np.int64), rc[:, hsig.STRAT])
            gid, gd = ids.cpu().numpy(), dist.cpu().numpy()
            bad = np.nonzero((gid != rid).any(1) | (gd.view(np.uint32) != rd.view(np.uint32)).any(1))[0]
            assert bad.size == 0, f"ef={ef} p={p} chunk={chunk}: {bad.size} rows differ, first {bad[:5]}"
            row = gid[gid >= 0]
            assert np.all((a2[row] >= np.repeat(l2, 10)[(gid >= 0).ravel()]))
    finally:
        ix.set_store(hsig.FP32)
        g.close()


def test_conjunctive_edges_and_errors(c1):
    torch = _torch()
    import paper_2412_02448_amd as u
    W, ix, path, a2, l2, h2 = c1
    g = u.Index.load(path, device=0)
    Q, L, H, L2, H2 = _dev(W.queries, W.l, W.h, l2, h2)
    with pytest.raises(u.UnifyError):  # no second attribute yet
        g.search(Q, L, H, 10, 32, l2=L2, h2=H2)
    with pytest.raises(u.UnifyError):
        g.set_attr2(a2[:-1])
    g.set_attr2(a2)
    ids, dist, _ = g.search(Q, L, H, 10, 32, l2=H2 + 1, h2=H2)  # l2 > h2: nothing qualifies
    assert (ids.cpu().numpy() == -1).all() and torch.isinf(dist).all().item()
    # a second range covering everything gives the single-attribute answer
    lo = torch.full_like(L2, int(a2.min()))
    hi = torch.full_like(H2, int(a2.max()))
    a = g.search(Q, L, H, 10, 32)[0]
    b = g.search(Q, L, H, 10, 32, l2=lo, h2=hi)[0]
    assert torch.equal(a, b)
    # replacing the attribute takes effect for later searches
    g.set_attr2(np.zeros_like(a2))
    ids, _, _ = g.search(Q, L, H, 10, 32, l2=torch.zeros_like(L2), h2=torch.zeros_like(H2))
    assert torch.equal(ids, a)
    g.close()
