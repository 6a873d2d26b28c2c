"""The GPU batch builder: structure of the index it produces (Sec. 4.1) and the
recall of searches on it against the exact FP64 answer (Definition 1, Eq. 1).

The builder's graph is not compared edge for edge with the oracle's: it inserts
all objects at once from exact candidates rather than one at a time (Alg. 6), so
only properties that hold for any HSIG are checked here.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import exact
from synth import workloads as w


def read_index(path):
    """Test-local reader of the index file layout (header + 64-byte aligned sections)."""
    raw = open(path, "rb").read()
    hdr = np.frombuffer(raw[:256], dtype=np.uint8)
    n = int(np.frombuffer(raw[16:24], np.int64)[0])
    d, S, M0, MU, L, efc, gentry, _ = np.frombuffer(raw[24:56], np.int32)
    R = int(np.frombuffer(raw[72:80], np.int64)[0])
    W0, WU = np.frombuffer(raw[80:88], np.int32)
    off = 256
    out = {}
    for name, dt, cnt in (("attr", np.int64, n), ("ext", np.int64, n), ("seg_start", np.int64, S + 1),
                          ("seg_entry", np.int32, S), ("seg_maxlevel", np.int32, S), ("level", np.uint8, n),
                          ("uprow", np.int32, n), ("vec", np.float32, n * d), ("adj0", np.int32, n * S * M0),
                          ("gbits0", np.uint32, n * W0), ("adjU", np.int32, R * S * MU),
                          ("gbitsU", np.uint32, R * WU)):
        off = (off + 63) // 64 * 64
        nb = np.dtype(dt).itemsize * cnt
        out[name] = np.frombuffer(raw[off:off + nb], dtype=dt)
        off += nb
    out.update(n=n, d=int(d), S=int(S), M0=int(M0), MU=int(MU), L=int(L), gentry=int(gentry), R=R,
               W0=int(W0), WU=int(WU))
    out["adj0"] = out["adj0"].reshape(n, S, M0)
    out["vec"] = out["vec"].reshape(n, d)
    out["gbits0"] = out["gbits0"].reshape(n, W0)
    return out


@pytest.fixture(scope="module")
def built(tmp_path_factory):
    import torch
    import paper_2412_02448_amd as u
    assert torch.cuda.is_available()
    W = w.make(w.SPECS["hybrid10k"], base_seed=5)
    s = W.spec
    print("[fixture] GPU build hybrid10k", flush=True)
    g = u.Index.build(W.base, W.attr, W.level_u, s.S, s.M, s.ef_cons)
    path = str(tmp_path_factory.mktemp("b") / "gpu_built.uix")
    g.save(path)
    assert u.validate_index_file(path)["n"] == s.n
    return W, g, read_index(path)


def test_structure(built):
    W, g, F = built
    check_structure(W, F)


def check_structure(W, F, equi_depth=True):
    n, S, M = F["n"], F["S"], F["M0"]
    order = np.lexsort((np.arange(n), W.attr))
    assert np.array_equal(F["ext"], order) and np.array_equal(F["attr"], W.attr[order])
    assert np.array_equal(F["vec"], W.base[order])
    ss = F["seg_start"]
    if W.spec.attr == "perm" and equi_depth:
        assert np.all(np.diff(ss) == n // S)
    seg_of = np.searchsorted(ss, np.arange(n), side="right") - 1
    M_L = 1.0 / np.log(M)
    lev = np.minimum(np.floor(-np.log(W.level_u[order]) * M_L), 30).astype(int)
    assert np.array_equal(F["level"], lev)
    adj = F["adj0"]
    X = F["vec"].astype(np.float64)
    for v in range(0, n, 37):
        marked = []
        allnb = set()
        for j in range(S):
            ch = adj[v, j]
            k = int((ch >= 0).sum())
            assert (ch[:k] >= 0).all() and (ch[k:] == -1).all()
            nb = ch[:k]
            assert len(set(nb.tolist())) == k and v not in nb
            assert (seg_of[nb] == j).all()
            dd = ((X[nb] - X[v]) ** 2).sum(1)
            assert np.all(np.diff(dd) >= -1e-3 * (1 + dd[:-1]))
            allnb |= set(nb.tolist())
            for r in range(k):
                pos = j * M + r
                if (F["gbits0"][v, pos >> 5] >> (pos & 31)) & 1:
                    marked.append(int(nb[r]))
        assert 1 <= len(marked) <= M and set(marked) <= allnb
    # most chunks are non-empty (each object reaches every segment)
    assert (adj[:, :, 0] >= 0).mean() > 0.99


def test_first_entries_are_segment_nearest(built):
    """Candidates are ranked on the matrix cores over BF16 copies, and Prune re-scores
    them in FP32 and always keeps the nearest: the first entry of every chunk is the
    owner's exact nearest object of that segment (up to distance ties)."""
    W, g, F = built
    assert first_entry_misses(F, 29) == 0


@pytest.mark.parametrize("ef_cons", [200, 256])
def test_wide_candidate_lists(tmp_path, ef_cons):
    """efCons above 128: candidate lists of up to 256 per (object, segment), merged in
    four 64-entry blocks.  Structure, first entries and recall as for efCons = 100."""
    import torch
    import paper_2412_02448_amd as u
    spec = w.scaled(w.SPECS["hybrid10k"], n=4000, nq=100)
    W = w.make(spec, base_seed=12)
    print(f"[case] GPU build efCons={ef_cons}", flush=True)
    g = u.Index.build(W.base, W.attr, W.level_u, spec.S, spec.M, ef_cons)
    try:
        path = str(tmp_path / "efc.uix")
        g.save(path)
        F = read_index(path)
        check_structure(W, F)
        assert first_entry_misses(F, 13) == 0
        dev = torch.device("cuda", 0)
        truth = [exact.rfknn(W.base, W.attr, W.queries[i], W.l[i], W.h[i], 10) for i in range(len(W.queries))]
        sizes = [int(((W.attr >= W.l[i]) & (W.attr <= W.h[i])).sum()) for i in range(len(W.queries))]
        ids, _, _ = g.search(torch.from_numpy(W.queries).to(dev), torch.from_numpy(W.l).to(dev),
                             torch.from_numpy(W.h).to(dev), 10, 64)
        ids = ids.cpu().numpy()
        rec = np.mean([exact.recall(ids[i], truth[i][0], 10, sizes[i]) for i in range(len(ids))])
        print(f"efCons={ef_cons} recall={rec:.4f}", flush=True)
        assert rec >= 0.95
    finally:
        g.close()


def first_entry_misses(F, step):
    """Objects (every step-th) whose chunk of some segment does not start with the owner's
    exact nearest object of that segment (up to distance ties)."""
    n, S = F["n"], F["S"]
    X = F["vec"].astype(np.float64)
    ss = F["seg_start"]
    adj = F["adj0"]
    bad = 0
    for v in range(0, n, step):
        dd = ((X - X[v]) ** 2).sum(1)
        dd[v] = np.inf
        for j in range(S):
            seg = dd[ss[j]:ss[j + 1]]
            if not np.isfinite(seg).any():
                continue
            first = adj[v, j, 0]
            if first < 0 or dd[first] > seg.min() * (1 + 1e-6) + 1e-12:
                bad += 1
    return bad


def test_recall_against_exact(built):
    import torch
    W, g, F = built
    dev = torch.device("cuda", 0)
    Q = torch.from_numpy(W.queries).to(dev)
    l = torch.from_numpy(W.l).to(dev)
    h = torch.from_numpy(W.h).to(dev)
    truth = [exact.rfknn(W.base, W.attr, W.queries[i], W.l[i], W.h[i], 10) for i in range(len(W.queries))]
    sizes = [int(((W.attr >= W.l[i]) & (W.attr <= W.h[i])).sum()) for i in range(len(W.queries))]
    for strategy, floor in ((None, 0.95), (2, 0.9), (3, 0.5)):
        ids, dist, _, stats = g.search(Q, l, h, 10, 64, strategy=strategy, stats=True)
        torch.cuda.synchronize()
        ids = ids.cpu().numpy()
        dist = dist.cpu().numpy()
        assert ((stats.cpu().numpy()[:, 3] & 0xFF) != 2).all()
        rec = np.mean([exact.recall(ids[i], truth[i][0], 10, sizes[i]) for i in range(len(ids))])
        print(f"strategy={strategy} recall={rec:.4f}", flush=True)
        assert rec >= floor
        # returned distances are the FP32 distances of the returned objects
        for i in range(0, len(ids), 17):
            ok = ids[i] >= 0
            ref = ((W.base[ids[i][ok]].astype(np.float64) - W.queries[i]) ** 2).sum(1)
            np.testing.assert_allclose(dist[i][ok], ref, rtol=1e-5)


def test_wide_vectors(tmp_path):
    """d = 960 (the GIST-like shape): the prune path that evaluates kept neighbours
    from memory instead of registers."""
    import torch
    import paper_2412_02448_amd as u
    spec = w.scaled(w.SPECS["gist1m"], n=3000, nq=60)
    W = w.make(spec, base_seed=8)
    print("[case] GPU build d=960", flush=True)
    g = u.Index.build(W.base, W.attr, W.level_u, spec.S, spec.M, spec.ef_cons)
    path = str(tmp_path / "wide.uix")
    g.save(path)
    check_structure(W, read_index(path))
    dev = torch.device("cuda", 0)
    truth = [exact.rfknn(W.base, W.attr, W.queries[i], W.l[i], W.h[i], 10) for i in range(len(W.queries))]
    sizes = [int(((W.attr >= W.l[i]) & (W.attr <= W.h[i])).sum()) for i in range(len(W.queries))]
    for prec in ("fp32", "bf16", "fp8"):
        g.set_precision(prec)
        ids, _, _ = g.search(torch.from_numpy(W.queries).to(dev), torch.from_numpy(W.l).to(dev),
                             torch.from_numpy(W.h).to(dev), 10, 64)
        ids = ids.cpu().numpy()
        rec = np.mean([exact.recall(ids[i], truth[i][0], 10, sizes[i]) for i in range(len(ids))])
        print(f"d=960 {prec} recall={rec:.4f}", flush=True)
        assert rec >= 0.9
    g.close()

