"""Incremental insertion into a resident index (Alg. 6 on more objects; the
paper's incremental-construction objective).

The GPU inserts a batch at a time (exact candidates, Prune, reverse edges, marks
recomputed from the final chunks), so its graph is not the oracle's sequential
one edge for edge.  Checked here: every structural property of an HSIG over all
objects, identical searches to the oracle's on the grown index's file, recall
close to a single build over all objects, and insertion while searches and a
server run.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import exact, hsig
from synth import workloads as w
from test_gpu_build import check_structure, read_index


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


def _q(W):
    torch = _torch()
    dev = torch.device("cuda", 0)
    return (torch.from_numpy(W.queries).to(dev), torch.from_numpy(W.l).to(dev), torch.from_numpy(W.h).to(dev))


SPLITS = (4000, 7000)


@pytest.fixture(scope="module")
def grown(tmp_path_factory):
    torch = _torch()
    import paper_2412_02448_amd as u
    W = w.make(w.SPECS["hybrid10k"], base_seed=6)
    s = W.spec
    n0 = SPLITS[0]
    print(f"[fixture] GPU build {n0} of {s.n}, then insert", flush=True)
    g = u.Index.build(W.base[:n0], W.attr[:n0], W.level_u[:n0], s.S, s.M, s.ef_cons)
    ss0 = read_seg_bounds(g, tmp_path_factory)
    for a, b in zip(SPLITS, SPLITS[1:] + (s.n,)):
        g.insert(W.base[a:b], W.attr[a:b], W.level_u[a:b])
        print(f"[fixture] inserted {a}..{b}", flush=True)
    assert g.n == s.n
    path = str(tmp_path_factory.mktemp("ins") / "grown.uix")
    g.save(path)
    return W, g, path, ss0


def read_seg_bounds(g, tmp_path_factory):
    path = str(tmp_path_factory.mktemp("ins0") / "first.uix")
    g.save(path)
    F = read_index(path)
    return F["attr"][F["seg_start"][1:-1]]


def test_structure_after_insertion(grown):
    W, g, path, bvals = grown
    F = read_index(path)
    check_structure(W, F, equi_depth=False)
    # segment boundaries are those of the first build
    assert np.array_equal(F["attr"][F["seg_start"][1:-1]], bvals)
    assert np.all(F["attr"][F["seg_start"][1:-1] - 1] < bvals)
    # upper layers: every object of a layer >= 1 has a row, chunks hold layer objects of the right segment
    n, S, MU = F["n"], F["S"], F["MU"]
    adjU = F["adjU"].reshape(-1, S, MU)
    seg_of = np.searchsorted(F["seg_start"], np.arange(n), side="right") - 1
    for v in np.nonzero(F["level"] >= 1)[0][::7]:
        for l in range(1, F["level"][v] + 1):
            row = adjU[F["uprow"][v] + l - 1]
            for j in range(S):
                nb = row[j][row[j] >= 0]
                assert (F["level"][nb] >= l).all() and (seg_of[nb] == j).all() and v not in nb


@pytest.mark.parametrize("strategy", [hsig.AUTO, hsig.PRE, hsig.HYBRID, hsig.POST])
def test_parity_on_grown_index(grown, strategy):
    """The oracle, reading the grown index's file, returns exactly the GPU's results."""
    torch = _torch()
    W, g, path, _ = grown
    print(f"[case] grown index strategy={strategy}", flush=True)
    ref = hsig.Index.read(path)
    rid, rd = ref.search(W.queries, W.l, W.h, 10, 48, p=2, strategy=strategy)
    Q, L, H = _q(W)
    ids, dist, _, st = g.search(Q, L, H, 10, 48, beam_p=2, strategy=None if strategy == hsig.AUTO else strategy,
                                stats=True)
    torch.cuda.synchronize()
    assert ((st.cpu().numpy()[:, 3] & 0xFF) != 2).all()
    assert np.array_equal(ids.cpu().numpy(), rid)
    assert np.array_equal(dist.cpu().numpy().view(np.uint32), rd.view(np.uint32))


def test_recall_close_to_single_build(grown):
    torch = _torch()
    import paper_2412_02448_amd as u
    W, g, path, _ = grown
    s = W.spec
    whole = u.Index.build(W.base, W.attr, W.level_u, s.S, s.M, s.ef_cons)
    Q, L, H = _q(W)
    truth = [exact.rfknn(W.base, W.attr, W.queries[i], W.l[i], W.h[i], 10) for i in range(len(W.queries))]
    sizes = [int(((W.attr >= W.l[i]) & (W.attr <= W.h[i])).sum()) for i in range(len(W.queries))]
    for strategy in (None, hsig.HYBRID):
        rec = []
        for ix in (g, whole):
            ids = ix.search(Q, L, H, 10, 48, strategy=strategy)[0].cpu().numpy()
            rec.append(np.mean([exact.recall(ids[i], truth[i][0], 10, sizes[i]) for i in range(len(ids))]))
        print(f"strategy={strategy}: grown {rec[0]:.4f}, single build {rec[1]:.4f}", flush=True)
        assert rec[0] >= rec[1] - 0.02 and rec[0] >= 0.9
    whole.close()


def test_insert_into_loaded_low_precision_index(tmp_path):
    """An oracle-built file, loaded with the BF16 store: insertion keeps that store and
    its searches match the oracle's on the saved result (BF16 ranking + FP32 rerank)."""
    torch = _torch()
    import paper_2412_02448_amd as u
    spec = w.scaled(w.SPECS["hybrid10k"], n=3000, nq=120)
    W = w.make(spec, base_seed=9)
    base = hsig.Index.build(W.base[:1800], W.attr[:1800], W.level_u[:1800], spec.S, spec.M, spec.ef_cons)
    p0 = str(tmp_path / "o.uix")
    base.write(p0)
    g = u.Index.load(p0, device=0, precision="bf16")
    print("[case] insert into loaded bf16 index", flush=True)
    g.insert(W.base[1800:], W.attr[1800:], W.level_u[1800:])
    assert g.n == 3000 and g.precision == hsig.BF16
    p1 = str(tmp_path / "g.uix")
    g.save(p1)
    F = read_index(p1)
    check_structure(W, F, equi_depth=False)
    ref = hsig.Index.read(p1)
    ref.set_store(hsig.BF16, 4)
    rid, rd = ref.search(W.queries, W.l, W.h, 10, 40, p=2)
    Q, L, H = _q(W)
    ids, dist, _ = g.search(Q, L, H, 10, 40, beam_p=2)
    assert np.array_equal(ids.cpu().numpy(), rid)
    assert np.array_equal(dist.cpu().numpy().view(np.uint32), rd.view(np.uint32))
    g.close()


def test_insert_invalidates_batches_and_checks_arguments(tmp_path):
    torch = _torch()
    import paper_2412_02448_amd as u
    spec = w.scaled(w.SPECS["hybrid10k"], n=2000, nq=50)
    W = w.make(spec, base_seed=12)
    g = u.Index.build(W.base[:1500], W.attr[:1500], W.level_u[:1500], spec.S, spec.M, spec.ef_cons)
    Q, L, H = _q(W)
    b = u.Batch(g, Q, L, H, 10, 32)
    b.run()
    with pytest.raises(u.UnifyError):
        g.insert(W.base[1500:1510], W.attr[1500:1510], np.zeros(10))  # level variates outside (0, 1]
    assert g.n == 1500
    b.run()  # a failed insertion leaves the index (and its batches) as they were
    g.insert(W.base[1500:], W.attr[1500:], W.level_u[1500:])
    with pytest.raises(u.UnifyError):
        b.run()
    b.close()
    b2 = u.Batch(g, Q, L, H, 10, 32)
    b2.run()
    torch.cuda.synchronize()
    ref = g.search(Q, L, H, 10, 32)[0]
    assert torch.equal(b2.ids, ref)
    b2.close()
    g.insert(W.base[:0], W.attr[:0], W.level_u[:0])  # nothing to insert
    assert g.n == 2000
    g.close()


def test_insert_while_serving(tmp_path):
    """A server keeps answering while objects are inserted; requests submitted after
    the insertion returns see the new objects (equal to a search of the grown index)."""
    torch = _torch()
    import paper_2412_02448_amd as u
    spec = w.scaled(w.SPECS["hybrid10k"], n=4000, nq=300)
    W = w.make(spec, base_seed=13)
    g = u.Index.build(W.base[:2500], W.attr[:2500], W.level_u[:2500], spec.S, spec.M, spec.ef_cons)
    srv = u.Server(g, 10, 32, max_batch=64, inflight=2)
    rng = np.random.default_rng(3)
    t_before = srv.submit(W.queries, W.l, W.h, arrive_s=np.sort(rng.uniform(0, 0.02, len(W.queries))))
    print("[case] insert while serving", flush=True)
    g.insert(W.base[2500:], W.attr[2500:], W.level_u[2500:])
    t_after = srv.submit(W.queries, W.l, W.h)
    ids_b, _, _ = srv.wait(t_before, timeout_s=60)
    ids_a, dist_a, _ = srv.wait(t_after, timeout_s=60)
    srv.close()
    Q, L, H = _q(W)
    ref_ids, ref_dist, _ = g.search(Q, L, H, 10, 32)
    assert np.array_equal(ids_a, ref_ids.cpu().numpy())
    assert np.array_equal(dist_a.view(np.uint32), ref_dist.cpu().numpy().view(np.uint32))
    assert (ids_b < 4000).all() and (ids_b[:, 0] >= 0).any()
    g.close()
