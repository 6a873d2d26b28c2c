"""Continuous-batching server: a request's result does not depend on its batch.

Requests arrive at random times and are admitted into batches of up to
max_batch by the library's worker, so every batch mixes different queries and
strategies.  Each result must equal the one a search of that query alone
returns (and the oracle's), bit for bit.
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
    spec = w.scaled(w.SPECS["serve10m"], n=8000, nq=600, d=96, S=8, M=12, ef_cons=60)
    W = w.make(spec, base_seed=4)
    path = str(tmp_path_factory.mktemp("serve") / "s.uix")
    print(f"[fixture] oracle build {spec.name}", flush=True)
    ix = hsig.Index.build(W.base, W.attr, W.level_u, spec.S, spec.M, spec.ef_cons, seed=4)
    ix.write(path)
    return W, ix, path


def alone(g, W, i, k, ef, **kw):
    torch = _torch()
    dev = torch.device("cuda", 0)
    ids, dist, _ = g.search(torch.from_numpy(W.queries[i:i + 1]).to(dev), torch.from_numpy(W.l[i:i + 1]).to(dev),
                            torch.from_numpy(W.h[i:i + 1]).to(dev), k, ef, **kw)
    return ids.cpu().numpy()[0], dist.cpu().numpy()[0]


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_served_equals_alone(c1, precision):
    W, ix, path = c1
    _torch()
    import paper_2412_02448_amd as u
    print(f"[case] serve {precision}", flush=True)
    g = u.Index.load(path, device=0, precision=precision)
    k, ef = 10, 40
    kw = dict(m=16, beam_p=2)
    srv = u.Server(g, k, ef, max_batch=37, inflight=3, **kw)
    n = len(W.queries)
    rng = np.random.default_rng(9)
    arrive = np.sort(rng.uniform(0, 0.05, n))
    order = rng.permutation(n)  # submission order differs from query order
    tickets = np.empty(n, np.int64)
    for part in np.array_split(order, 5):
        tickets[part] = srv.submit(W.queries[part], W.l[part], W.h[part], arrive_s=arrive[part])
    ids, dist, lat = srv.wait(tickets, timeout_s=60)
    done, batches, busy = srv.stats()
    srv.close()
    assert done == n and batches >= n // 37 and (lat >= 0).all()
    ix.set_store(hsig.BF16 if precision == "bf16" else hsig.FP32, 4)
    oid, od = ix.search(W.queries, W.l, W.h, k, ef, m=16, p=2)
    ix.set_store(hsig.FP32)
    assert np.array_equal(oid, ids) and np.array_equal(od.view(np.uint32), dist.view(np.uint32))
    for i in range(0, n, 23):
        a_ids, a_dist = alone(g, W, i, k, ef, **kw)
        assert np.array_equal(a_ids, ids[i]) and np.array_equal(a_dist.view(np.uint32), dist[i].view(np.uint32))
    g.close()


def test_server_waits_and_errors(c1):
    W, ix, path = c1
    import paper_2412_02448_amd as u
    g = u.Index.load(path, device=0)
    with pytest.raises(u.UnifyError):
        u.Server(g, 0, 10)
    with pytest.raises(u.UnifyError):
        u.Server(g, 10, 5)
    srv = u.Server(g, 10, 20, max_batch=8, inflight=1, max_wait_s=0.002)
    t = srv.submit(W.queries[:20], W.l[:20], W.h[:20])
    ids, dist, lat = srv.wait(t, timeout_s=30)
    assert (ids[:, 0] >= -1).all() and len(lat) == 20
    with pytest.raises(u.UnifyError):
        srv.wait(np.array([10 ** 6]))
    srv.close()
    g.close()


def test_concurrent_streams_equal_serial(c1):
    """Searches issued on two streams without waiting for each other share the
    index's visited-set memory; the library orders their search kernels."""
    W, ix, path = c1
    torch = _torch()
    import paper_2412_02448_amd as u
    print("[case] concurrent streams", flush=True)
    dev = torch.device("cuda", 0)
    g = u.Index.load(path, device=0)
    Q = torch.from_numpy(W.queries).to(dev)
    L = torch.from_numpy(W.l).to(dev)
    H = torch.from_numpy(W.h).to(dev)
    ref = g.search(Q, L, H, 10, 40, m=16, beam_p=2)[0].cpu().numpy()
    streams = [torch.cuda.Stream(device=dev), torch.cuda.Stream(device=dev)]
    torch.cuda.synchronize()
    outs = []
    for i in range(6):
        s = streams[i % 2]
        outs.append(g.search(Q, L, H, 10, 40, m=16, beam_p=2, stream=s)[0])
    torch.cuda.synchronize()
    for o in outs:
        assert np.array_equal(o.cpu().numpy(), ref)
    g.close()


def test_served_k100_equals_batch(c1):
    """The serving workload's other result size: k = 100."""
    W, ix, path = c1
    torch = _torch()
    import paper_2412_02448_amd as u
    print("[case] serve k=100", flush=True)
    g = u.Index.load(path, device=0)
    dev = torch.device("cuda", 0)
    n = 300
    srv = u.Server(g, 100, 128, max_batch=64, inflight=2, m=16, beam_p=2)
    arrive = np.sort(np.random.default_rng(2).uniform(0, 0.02, n))
    ids, dist, lat = srv.wait(srv.submit(W.queries[:n], W.l[:n], W.h[:n], arrive_s=arrive), timeout_s=60)
    srv.close()
    ref = g.search(torch.from_numpy(W.queries[:n]).to(dev), torch.from_numpy(W.l[:n]).to(dev),
                   torch.from_numpy(W.h[:n]).to(dev), 100, 128, m=16, beam_p=2)
    assert np.array_equal(ids, ref[0].cpu().numpy())
    assert np.array_equal(dist.view(np.uint32), ref[1].cpu().numpy().view(np.uint32))
    oid, od = ix.search(W.queries[:n], W.l[:n], W.h[:n], 100, 128, m=16, p=2)
    assert np.array_equal(oid, ids)
    g.close()


def test_memory_budget_admission(c1):
    """A small device-memory budget shrinks the batch size, then each slot's visited
    rows, until the slots fit; results stay those of the oracle.  A budget that holds
    no slot is refused."""
    W, ix, path = c1
    _torch()
    import paper_2412_02448_amd as u
    print("[case] serve under a 12 MB budget", flush=True)
    g = u.Index.load(path, device=0)
    with pytest.raises(u.UnifyError):
        u.Server(g, 10, 40, inflight=3, mem_budget=1 << 16, m=16, beam_p=2)
    srv = u.Server(g, 10, 40, max_batch=4096, inflight=3, mem_budget=12 << 20, m=16, beam_p=2)
    batch, rows, nbytes = srv.limits()
    assert batch == 64 and 1 <= rows <= 128 and 0 < nbytes <= 12 << 20
    n = len(W.queries)
    arrive = np.sort(np.random.default_rng(5).uniform(0, 0.02, n))
    ids, dist, _ = srv.wait(srv.submit(W.queries, W.l, W.h, arrive_s=arrive), timeout_s=60)
    done, batches, _ = srv.stats()
    srv.close()
    assert done == n and batches >= n // 64
    oid, od = ix.search(W.queries, W.l, W.h, 10, 40, m=16, p=2)
    assert np.array_equal(oid, ids) and np.array_equal(od.view(np.uint32), dist.view(np.uint32))
    g.close()
