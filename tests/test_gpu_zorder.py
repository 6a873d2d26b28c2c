"""Box searches on a z-order index on the GPU against the oracle (the paper's
multi-attribute extension, approach 2: one HSIG over the z-order key of the pair
(A1, A2)): identical ids, FP32 distances and strategies for every strategy and both
stores, the full box against the plain key-range search, and the error paths."""
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
def zc(tmp_path_factory):
    spec = w.SPECS["hybrid10k"]
    W = w.make(spec, base_seed=23)
    a2, l2, h2 = w.second_attribute(spec.n, len(W.queries), base_seed=23)
    zmap = hsig.zorder_map(W.attr, a2)
    z = hsig.zorder_keys(zmap, W.attr, a2)
    path = str(tmp_path_factory.mktemp("zorder") / "z.uix")
    print(f"[fixture] oracle build {spec.name} on z-order keys", flush=True)
    ix = hsig.Index.build(W.base, z, W.level_u, spec.S, spec.M, spec.ef_cons, seed=23)
    ix.write(path)
    ix.set_zorder(zmap, W.attr, a2)
    return W, ix, path, zmap, z, a2, l2, h2


def _dev(*arrs):
    torch = _torch()
    dev = torch.device("cuda", 0)
    return [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in arrs]


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("strategy", [hsig.AUTO, hsig.PRE, hsig.HYBRID, hsig.POST])
def test_parity_box(zc, precision, strategy):
    torch = _torch()
    import paper_2412_02448_amd as u
    W, ix, path, zmap, z, a2, l2, h2 = zc
    print(f"[case] box {precision} strategy={strategy}", flush=True)
    g = u.Index.load(path, device=0, precision=precision)
    g.set_zorder(u.zorder_map(W.attr, a2), W.attr, a2)
    ix.set_store(hsig.BF16 if precision == "bf16" else hsig.FP32, 4)
    try:
        Q, L, H, L2, H2 = _dev(W.queries, W.l, W.h, l2, h2)
        for ef, p, chunk in ((48, 1, 0), (64, 2, 64)):
            rid, rd, rc = ix.search_box(W.queries, W.l, W.h, l2, h2, 10, ef, p=p, strategy=strategy, counters=True)
            ids, dist, srun, st = g.search(Q, L, H, 10, ef, beam_p=p, strategy=None if strategy == hsig.AUTO else strategy,
                                           stats=True, pre_chunk=chunk, l2=L2, h2=H2, box=True)
            torch.cuda.synchronize()
            assert ((st.cpu().numpy()[:, 3] & 0xFF) != 2).all()
            assert np.array_equal(srun.cpu().numpy().astype(np.int64), rc[:, hsig.STRAT])
            gid, gd = ids.cpu().numpy(), dist.cpu().numpy()
            bad = np.nonzero((gid != rid).any(1) | (gd.view(np.uint32) != rd.view(np.uint32)).any(1))[0]
            assert bad.size == 0, f"ef={ef} p={p} chunk={chunk}: {bad.size} rows differ, first {bad[:5]}"
            ok = gid >= 0
            e = gid[ok]
            assert np.all((W.attr[e] >= np.repeat(W.l, 10)[ok.ravel()]) & (W.attr[e] <= np.repeat(W.h, 10)[ok.ravel()]))
            assert np.all((a2[e] >= np.repeat(l2, 10)[ok.ravel()]) & (a2[e] <= np.repeat(h2, 10)[ok.ravel()]))
        if strategy == hsig.AUTO:
            # the rule reached all three strategies on this workload
            assert set(rc[:, hsig.STRAT].tolist()) >= {hsig.PRE, hsig.HYBRID}
    finally:
        ix.set_store(hsig.FP32)
        g.close()


def test_full_box_is_the_key_range_search(zc):
    torch = _torch()
    import paper_2412_02448_amd as u
    W, ix, path, zmap, z, a2, l2, h2 = zc
    g = u.Index.load(path, device=0)
    try:
        g.set_zorder(zmap, W.attr, a2)
        nq = len(W.queries)
        full = [np.full(nq, v, np.int64) for v in (W.attr.min(), W.attr.max(), a2.min(), a2.max())]
        Q, L1, H1, L2, H2 = _dev(W.queries, *full)
        ZL, ZH = _dev(np.full(nq, z.min(), np.int64), np.full(nq, z.max(), np.int64))
        for s in (hsig.PRE, hsig.HYBRID, hsig.POST):
            a = g.search(Q, ZL, ZH, 10, 48, strategy=s)
            b = g.search(Q, L1, H1, 10, 48, strategy=s, l2=L2, h2=H2, box=True)
            torch.cuda.synchronize()
            assert torch.equal(a[0], b[0]) and torch.equal(a[1].view(torch.int32), b[1].view(torch.int32))
    finally:
        g.close()


def test_box_edges_and_errors(zc):
    torch = _torch()
    import paper_2412_02448_amd as u
    W, ix, path, zmap, z, a2, l2, h2 = zc
    g = u.Index.load(path, device=0)
    try:
        Q, L, H, L2, H2 = _dev(W.queries, W.l, W.h, l2, h2)
        with pytest.raises(u.UnifyError):  # no pairs attached yet
            g.search(Q, L, H, 10, 32, l2=L2, h2=H2, box=True)
        with pytest.raises(u.UnifyError):  # the index is not built on these pairs' keys
            g.set_zorder(zmap, a2, W.attr)
        with pytest.raises(u.UnifyError):
            g.set_zorder(zmap, W.attr[:-1], a2[:-1])
        g.set_zorder(zmap, W.attr, a2)
        ids, dist, _ = g.search(Q, H + 1, H, 10, 32, l2=L2, h2=H2, box=True)  # l1 > h1: nothing qualifies
        torch.cuda.synchronize()
        assert (ids.cpu().numpy() == -1).all() and torch.isinf(dist).all().item()
        # a conjunctive search still needs a second attribute of its own
        with pytest.raises(u.UnifyError):
            g.search(Q, L, H, 10, 32, l2=L2, h2=H2)
        # nq = 0 is a no-op
        e = _dev(np.zeros((0, W.queries.shape[1]), np.float32), *[np.zeros(0, np.int64)] * 4)
        g.search(e[0], e[1], e[2], 10, 32, l2=e[3], h2=e[4], box=True)
    finally:
        g.close()


def test_gpu_built_zorder_index_and_insertion():
    """A z-order index built on the GPU: box pre-filter answers equal brute force; an
    insertion drops the attached pairs (box searches refused) until they are attached again
    for the grown index, whose box pre-filter answers again equal brute force."""
    torch = _torch()
    import paper_2412_02448_amd as u
    spec = w.scaled(w.SPECS["hybrid10k"], n=3000, nq=40)
    W = w.make(spec, base_seed=31)
    a2, l2, h2 = w.second_attribute(spec.n, len(W.queries), base_seed=31)
    zmap = u.zorder_map(W.attr, a2)
    z = u.zorder_keys(zmap, W.attr, a2)
    print("[case] GPU-built z-order index, then an insertion", flush=True)
    g = u.Index.build(W.base[:2400], z[:2400], W.level_u[:2400], spec.S, spec.M, spec.ef_cons)
    try:
        Q, L, H, L2, H2 = _dev(W.queries, W.l, W.h, l2, h2)

        def check(nobj):
            ids, dist, _ = g.search(Q, L, H, 10, 32, strategy=hsig.PRE, l2=L2, h2=H2, box=True)
            torch.cuda.synchronize()
            ids, dist = ids.cpu().numpy(), dist.cpu().numpy()
            X, A1, A2 = W.base[:nobj], W.attr[:nobj], a2[:nobj]
            for i in range(len(W.queries)):
                ok = (A1 >= W.l[i]) & (A1 <= W.h[i]) & (A2 >= l2[i]) & (A2 <= h2[i])
                idx = np.nonzero(ok)[0]
                dd = ((X[idx].astype(np.float64) - W.queries[i].astype(np.float64)) ** 2).sum(1)
                want = np.sort(dd)[:10]
                got = ids[i][ids[i] >= 0]
                assert len(got) == len(want) and ok[got].all(), i
                gd = ((X[got].astype(np.float64) - W.queries[i].astype(np.float64)) ** 2).sum(1)
                np.testing.assert_allclose(gd, want, rtol=1e-6)  # the exact top 10 (ties aside)

        g.set_zorder(zmap, W.attr[:2400], a2[:2400])
        check(2400)
        g.insert(W.base[2400:], z[2400:], W.level_u[2400:])
        with pytest.raises(u.UnifyError):
            g.search(Q, L, H, 10, 32, l2=L2, h2=H2, box=True)
        g.set_zorder(zmap, W.attr, a2)
        check(3000)
    finally:
        g.close()
