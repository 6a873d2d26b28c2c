"""The graph-captured batch (unify_batch_*) against the eager search and the oracle.

A batch captures plan, work list, search, merge and re-run into one HIP graph
over fixed buffers.  Each replay must return exactly what unify_search_ex
returns on the same inputs; replays are interleaved with eager searches and
synchronisations, and the inputs are rewritten in place between replays.
"""
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
    spec = w.SPECS["batch100k"]
    spec = w.scaled(spec, nq=800)
    W = w.make(spec, base_seed=2)
    path = str(tmp_path_factory.mktemp("batch") / "b.uix")
    print(f"[fixture] oracle build {spec.name}", flush=True)
    ix = hsig.Index.build(W.base, W.attr, W.level_u, spec.S, spec.M, spec.ef_cons, seed=2)
    ix.write(path)
    W2 = w.more_queries(spec, W.attr, 800, base_seed=2, stream=3)
    return W, W2, ix, path


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("chunk,wpq", [(0, 1), (64, 1), (0, 4)])
def test_batch_replays_equal_eager(c1, precision, chunk, wpq):
    """wpq = 4: the captured graph forks the cooperative kernel onto a side branch."""
    W, W2, ix, path = c1
    torch = _torch()
    import paper_2412_02448_amd as u
    print(f"[case] batch {precision} chunk={chunk} wpq={wpq}", flush=True)
    dev = torch.device("cuda", 0)
    g = u.Index.load(path, device=0, precision=precision)
    Q = torch.from_numpy(W.queries).to(dev)
    L = torch.from_numpy(W.l).to(dev)
    H = torch.from_numpy(W.h).to(dev)
    kw = dict(m=24, beam_p=2, pre_chunk=chunk, waves_per_query=wpq)
    b = u.Batch(g, Q, L, H, 10, 48, stats=True, **kw)
    sets = [(W.queries, W.l, W.h), (W2[0], W2[1], W2[2])]
    for rep in range(6):
        q, l, h = sets[rep % 2]
        Q.copy_(torch.from_numpy(q))
        L.copy_(torch.from_numpy(l))
        H.copy_(torch.from_numpy(h))
        b.run()
        torch.cuda.synchronize()
        got = [t.cpu().numpy() for t in (b.ids, b.dist, b.strategy_run, b.stats)]
        ref = [t.cpu().numpy() for t in g.search(Q, L, H, 10, 48, stats=True, **kw)]
        torch.cuda.synchronize()
        if wpq > 1:  # which searches ran cooperatively (flag bits 8-9) depends on timing
            got[3][:, 3] &= 0xFF
            ref[3][:, 3] &= 0xFF
        for x, y, name in zip(got, ref, ("ids", "dist", "strategy", "stats")):
            assert np.array_equal(x, y), f"replay {rep}: {name} differs"
        if rep < 2:  # and the oracle agrees with both
            ix.set_store(hsig.BF16 if precision == "bf16" else hsig.FP32, 4)
            oid, od = ix.search(q, l, h, 10, 48, m=24, p=2)
            ix.set_store(hsig.FP32)
            assert np.array_equal(oid, got[0]) and np.array_equal(od.view(np.uint32), got[1].view(np.uint32))
    b.close()
    g.close()


def test_batch_invalid_arguments(c1):
    W, W2, ix, path = c1
    torch = _torch()
    import paper_2412_02448_amd as u
    dev = torch.device("cuda", 0)
    g = u.Index.load(path, device=0)
    Q = torch.from_numpy(W.queries).to(dev)
    L = torch.from_numpy(W.l).to(dev)
    H = torch.from_numpy(W.h).to(dev)
    with pytest.raises(u.UnifyError):
        u.Batch(g, Q, L, H, 0, 10)
    with pytest.raises(u.UnifyError):
        u.Batch(g, Q, L, H, 10, 300)
    with pytest.raises(u.UnifyError):
        u.Batch(g, Q[:0], L[:0], H[:0], 10, 10)
    g.close()
