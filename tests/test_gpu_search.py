"""GPU parity: the HIP search against the CPU oracle on the same index file.

The oracle builds the index (Alg. 6) and writes it; the library loads that file.
Both then search the same graph with the same parameters.  The bar: identical
ids and bit-identical FP32 distances (canonical summation order on both sides)
for every query; pre-filter results additionally within 1e-5 relative of the
FP64 exact answer.
"""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import exact, hsig
from synth import workloads as w


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


def gpu_search(g, W, k, ef, strategy=None, **kw):
    torch = _torch()
    dev = torch.device("cuda", 0)
    Q = torch.from_numpy(W.queries).to(dev)
    l = torch.from_numpy(W.l).to(dev)
    h = torch.from_numpy(W.h).to(dev)
    out = g.search(Q, l, h, k, ef, strategy=strategy, stats=True, **kw)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in out]


def _build(spec, seed, path):
    W = w.make(spec, base_seed=seed)
    print(f"[fixture] oracle build {spec.name} n={spec.n} d={spec.d}", flush=True)
    ix = hsig.Index.build(W.base, W.attr, W.level_u, spec.S, spec.M, spec.ef_cons, seed=seed)
    ix.write(path)
    import paper_2412_02448_amd as u
    g = u.Index.load(path, device=0)
    return W, ix, g


@pytest.fixture(scope="module")
def c1(tmp_path_factory):
    path = str(tmp_path_factory.mktemp("c1") / "hybrid10k.uix")
    return _build(w.SPECS["hybrid10k"], 0, path)


def assert_parity(ref, got, what):
    rid, rd = ref
    gid, gd, gst, gstats = got
    bad = np.nonzero((rid != gid).any(1) | (rd.view(np.uint32) != gd.view(np.uint32)).any(1))[0]
    assert ((gstats[:, 3] & 0xFF) != 2).all(), f"{what}: capacity overflow on {np.nonzero((gstats[:, 3] & 0xFF) == 2)[0][:5]}"
    assert bad.size == 0, f"{what}: {bad.size} queries differ, first {bad[:5]}: ref {rid[bad[0]]} got {gid[bad[0]]}"


@pytest.mark.parametrize("strategy", [hsig.AUTO, hsig.PRE, hsig.HYBRID, hsig.POST])
def test_parity_hybrid10k(c1, strategy):
    W, ix, g = c1
    k, ef = 10, 64
    print(f"[case] hybrid10k strategy={strategy} k={k} ef={ef}", flush=True)
    ref = ix.search(W.queries, W.l, W.h, k, ef, strategy=strategy)
    got = gpu_search(g, W, k, ef, strategy=None if strategy == hsig.AUTO else strategy)
    assert_parity(ref, got, f"strategy {strategy}")
    if strategy == hsig.AUTO:
        _, _, cnt = ix.search(W.queries, W.l, W.h, k, ef, strategy=strategy, counters=True)
        assert (got[2] == cnt[:, hsig.STRAT]).all()


@pytest.mark.parametrize("p", [2, 4])
@pytest.mark.parametrize("strategy", [hsig.HYBRID, hsig.POST])
def test_parity_beam_width(c1, strategy, p):
    W, ix, g = c1
    print(f"[case] hybrid10k beam p={p} strategy={strategy}", flush=True)
    ref = ix.search(W.queries, W.l, W.h, 10, 48, p=p, strategy=strategy)
    got = gpu_search(g, W, 10, 48, strategy=strategy, beam_p=p)
    assert_parity(ref, got, f"p={p}")


@pytest.mark.parametrize("m", [4, 8, 64])
def test_parity_neighbour_budget(c1, m):
    W, ix, g = c1
    print(f"[case] hybrid10k m={m}", flush=True)
    ref = ix.search(W.queries, W.l, W.h, 10, 32, m=m, strategy=hsig.HYBRID)
    got = gpu_search(g, W, 10, 32, strategy=hsig.HYBRID, m=m)
    assert_parity(ref, got, f"m={m}")


@pytest.mark.parametrize("m,p", [(4, 1), (16, 2), (64, 1)])
@pytest.mark.parametrize("strategy", [hsig.HYBRID, hsig.AUTO])
def test_parity_selection_s1(c1, strategy, m, p):
    """Selection S1: each expanded object's active-chunk entries ranked by distance."""
    W, ix, g = c1
    print(f"[case] hybrid10k S1 m={m} p={p} strategy={strategy}", flush=True)
    ref = ix.search(W.queries, W.l, W.h, 10, 32, m=m, p=p, strategy=strategy, select_s1=True)
    got = gpu_search(g, W, 10, 32, strategy=None if strategy == hsig.AUTO else strategy, m=m, beam_p=p,
                     select_s1=True)
    assert_parity(ref, got, f"S1 m={m} p={p}")
    if strategy == hsig.HYBRID and m == 16:
        # S1 and S2 are different selections: the searches are not all the same
        s2 = ix.search(W.queries, W.l, W.h, 10, 32, m=m, p=p, strategy=strategy)
        assert (s2[0] != ref[0]).any()


@pytest.mark.parametrize("chunk", [64, 100, 1000])
def test_parity_split_pre_filter(c1, chunk):
    """Pre-filter scans split into chunks on several wavefronts and merged."""
    W, ix, g = c1
    print(f"[case] split pre-filter chunk={chunk}", flush=True)
    for k in (1, 10, 32, 33, 100, 128, 129):
        for strategy in (hsig.PRE, hsig.AUTO):
            ref = ix.search(W.queries, W.l, W.h, k, max(k, 40), strategy=strategy)
            got = gpu_search(g, W, k, max(k, 40), strategy=None if strategy == hsig.AUTO else strategy,
                             pre_chunk=chunk)
            assert_parity(ref, got, f"chunk={chunk} k={k} strategy={strategy}")
            pre = got[3][:, 5] == hsig.PRE
            # every object of the slice scanned once, whatever the split
            assert (got[3][pre, 0] == got[3][pre, 6]).all()


def test_pre_filter_matches_fp64_exact(c1):
    W, ix, g = c1
    print("[case] pre vs FP64 exact", flush=True)
    gid, gd, _, _ = gpu_search(g, W, 10, 10, strategy=hsig.PRE)
    for i in range(len(W.queries)):
        tid, td = exact.rfknn(W.base, W.attr, W.queries[i], W.l[i], W.h[i], 10)
        assert gid[i, : len(tid)].tolist() == tid.tolist()
        np.testing.assert_allclose(gd[i, : len(tid)], td, rtol=1e-5)


def test_edge_cases_and_large_k(c1):
    W, ix, g = c1
    torch = _torch()
    print("[case] edge cases", flush=True)
    a = ix.attr_sorted()
    n = len(a)
    Q = W.queries[:6]
    l = np.array([10, a[-1] + 1, a[7], a[0], a[100], a[0]], np.int64)
    h = np.array([5, a[-1] + 50, a[7], a[-1], a[130], a[n // 3]], np.int64)
    Wc = w.Workload(W.spec, W.base, W.attr, Q, l, h, None, None)
    for strategy in (hsig.AUTO, hsig.PRE, hsig.HYBRID, hsig.POST):
        for k, ef in ((1, 1), (10, 10), (256, 256), (37, 100)):
            ref = ix.search(Q, l, h, k, ef, strategy=strategy)
            got = gpu_search(g, Wc, k, ef, strategy=None if strategy == hsig.AUTO else strategy)
            assert_parity(ref, got, f"edge strategy={strategy} k={k} ef={ef}")
            assert (got[0][0] == -1).all() and (got[0][1] == -1).all()


def test_invalid_arguments(c1):
    W, ix, g = c1
    torch = _torch()
    import paper_2412_02448_amd as u
    dev = torch.device("cuda", 0)
    Q = torch.from_numpy(W.queries[:4]).to(dev)
    l = torch.from_numpy(W.l[:4]).to(dev)
    h = torch.from_numpy(W.h[:4]).to(dev)
    for k, ef in ((0, 10), (257, 300), (10, 5), (10, 257)):
        with pytest.raises(u.UnifyError) as e:
            g.search(Q, l, h, k, ef)
        assert e.value.code == -22
    with pytest.raises(u.UnifyError):
        g.search(Q, l, h, 10, 10, beam_p=9)
    # nq = 0 is a no-op
    ids, dist, st = g.search(Q[:0], l[:0], h[:0], 10, 10)
    assert ids.shape == (0, 10)


def test_deterministic(c1):
    W, ix, g = c1
    a = gpu_search(g, W, 10, 64)
    b = gpu_search(g, W, 10, 64)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("d", [4, 96, 200, 260, 960, 2048])  # every kernel width: 2, 4, 8, 15 and 32 groups
def test_parity_other_dimensions(tmp_path, d):
    spec = w.scaled(w.SPECS["hybrid10k"], n=3000, nq=40, d=d, S=4, M=8, ef_cons=40)
    W, ix, g = _build(spec, 3, str(tmp_path / f"d{d}.uix"))
    print(f"[case] d={d}", flush=True)
    for strategy in (hsig.AUTO, hsig.PRE, hsig.HYBRID, hsig.POST):
        ref = ix.search(W.queries, W.l, W.h, 10, 32, strategy=strategy)
        got = gpu_search(g, W, 10, 32, strategy=None if strategy == hsig.AUTO else strategy)
        assert_parity(ref, got, f"d={d} strategy={strategy}")


@pytest.mark.parametrize("p", [1, 4])
@pytest.mark.parametrize("strategy", [hsig.HYBRID, hsig.POST, hsig.AUTO])
def test_parity_small_capacities(c1, strategy, p):
    """A 64-entry candidate array and a 256-entry visited cache: graph searches outgrow
    the candidate array (the query is abandoned and re-run by the second launch with a
    larger one: status 1) or the visited cache (the visited set continues in the wave's
    HBM tag row: flag bit 8).  Both paths are reached here and every row still equals
    the oracle's."""
    W, ix, g = c1
    print(f"[case] small capacities strategy={strategy} p={p}", flush=True)
    ref = ix.search(W.queries, W.l, W.h, 10, 64, p=p, strategy=strategy)
    got = gpu_search(g, W, 10, 64, strategy=None if strategy == hsig.AUTO else strategy, beam_p=p,
                     cand_cap=64, visit_cap=256)
    assert_parity(ref, got, f"small capacities strategy={strategy} p={p}")
    st = got[3]
    graph = np.isin(st[:, 5], [hsig.HYBRID, hsig.POST])
    assert graph.any()
    assert ((st[:, 3] & 0xFF) == 1)[graph].any(), "no query reached the re-run launch"
    assert ((st[:, 3] & 0x100) != 0)[graph].any(), "no visited set spilled to HBM"


def test_unknown_strategy_rows(c1):
    """Strategies outside AUTO..POST are read on the device: their rows are padded and
    reported as strategy -2 with status 3; the other rows are searched as usual."""
    W, ix, g = c1
    torch = _torch()
    dev = torch.device("cuda", 0)
    print("[case] unknown strategies", flush=True)
    nq = len(W.queries)
    s = np.zeros(nq, np.int8)
    s[::7] = 4
    s[3::11] = -1
    s[5::13] = 127
    bad = (s < 0) | (s > 3)
    Q, l, h = (torch.from_numpy(a).to(dev) for a in (W.queries, W.l, W.h))
    ids, dist, ost, st = g.search(Q, l, h, 10, 64, strategy=torch.from_numpy(s).to(dev), stats=True)
    torch.cuda.synchronize()
    ids, dist, ost, st = (t.cpu().numpy() for t in (ids, dist, ost, st))
    assert (ids[bad] == -1).all() and np.isinf(dist[bad]).all()
    assert (ost[bad] == -2).all() and (st[bad, 3] == 3).all() and (st[bad, 5] == -2).all()
    rid, rd = ix.search(W.queries[~bad], W.l[~bad], W.h[~bad], 10, 64)
    assert np.array_equal(ids[~bad], rid) and np.array_equal(dist[~bad].view(np.uint32), rd.view(np.uint32))


@pytest.mark.parametrize("k", [1, 10, 32])
def test_matrix_core_scan_equals_wave_scan(c1, k):
    """The pre-filter scan on the matrix cores (norm expansion on MFMA, then FP32 re-scores of
    the objects its bounds cannot exclude) returns exactly the per-wavefront FP32 scan's rows
    and the oracle's; every forced pre-filter row within the record budget took that path."""
    W, ix, g = c1
    print(f"[case] matrix-core scan k={k}", flush=True)
    ref = ix.search(W.queries, W.l, W.h, k, max(k, 16), strategy=hsig.PRE)
    tile = gpu_search(g, W, k, max(k, 16), strategy=hsig.PRE)
    wave = gpu_search(g, W, k, max(k, 16), strategy=hsig.PRE, wave_scan=True)
    assert_parity(ref, tile, f"matrix-core scan k={k}")
    assert_parity(ref, wave, f"wave scan k={k}")
    took = tile[3][:, 4] > 0
    assert took.sum() >= len(W.queries) // 2, took.sum()
    assert (wave[3][:, 4] == 0).all()
    # far fewer FP32 evaluations than objects in range
    assert tile[3][took, 2].sum() < 0.2 * tile[3][took, 6].sum()


def test_serial_phases_equal_concurrent(c1):
    """The matrix-core scan runs beside the graph search on a second stream by default;
    run before it (UNIFY_FLAG_SERIAL_PHASES), every row is the same, and the oracle's."""
    W, ix, g = c1
    print("[case] serial phases vs concurrent", flush=True)
    ref = ix.search(W.queries, W.l, W.h, 10, 32, m=16, p=2)
    side = gpu_search(g, W, 10, 32, m=16, beam_p=2)
    serial = gpu_search(g, W, 10, 32, m=16, beam_p=2, serial_phases=True)
    assert_parity(ref, side, "concurrent phases")
    assert_parity(ref, serial, "serial phases")
    assert (side[3][:, 4][side[2] == hsig.PRE] > 0).any()  # the matrix-core scan ran


def test_matrix_core_scan_record_overflow(tmp_path):
    """Four distinct vectors repeated over 4096 objects: about 64 objects of every super-block
    tie at the smallest distance, more than a record holds, and those queries are answered
    by the FP32 scan (status 1) with the (distance, id) order of the oracle."""
    rng = np.random.default_rng(9)
    n, d = 4096, 64
    base = rng.standard_normal((4, d)).astype(np.float32)
    X = base[rng.integers(0, 4, n)]
    attr = rng.permutation(n).astype(np.int64)
    ix = hsig.Index.build(X, attr, 1.0 - rng.random(n), 4, 8, 32)
    path = str(tmp_path / "ties.uix")
    ix.write(path)
    import paper_2412_02448_amd as u
    g = u.Index.load(path, device=0)
    nq = 64
    Q = (base[rng.integers(0, 4, nq)] + 0.01 * rng.standard_normal((nq, d))).astype(np.float32)
    lo = rng.integers(0, n // 2, nq).astype(np.int64)
    hi = (lo + rng.integers(300, n // 2, nq)).astype(np.int64)
    Wq = w.Workload(None, X, attr, Q, lo, hi, None, None)
    print("[case] matrix-core scan record overflow", flush=True)
    for k in (1, 10):
        ref = ix.search(Q, lo, hi, k, 16, strategy=hsig.PRE)
        got = gpu_search(g, Wq, k, 16, strategy=hsig.PRE)
        assert_parity(ref, got, f"ties k={k}")
        assert ((got[3][:, 3] & 0xFF) == 1).any(), "no record overflowed"
    g.close()


@pytest.mark.parametrize("wpq", [2, 4])
@pytest.mark.parametrize("strategy,p", [(hsig.HYBRID, 1), (hsig.HYBRID, 4), (hsig.POST, 2), (hsig.AUTO, 4),
                                        (hsig.PRE, 1)])
def test_parity_cooperative_search(c1, wpq, strategy, p):
    """Heavy graph searches run by 2 or 4 wavefronts together (the adjacency gather, the
    visited checks and the distance evaluations split between them, admissions by one):
    every row equals the oracle's, for a few heavy queries and for all of them.  The
    cooperative kernel takes graph searches only: with per-wavefront pre-filter scans
    every pre-filter chunk stays with the one-wavefront kernel (forced pre-filter: no
    graph search at all)."""
    W, ix, g = c1
    print(f"[case] cooperative wpq={wpq} strategy={strategy} p={p}", flush=True)
    ref = ix.search(W.queries, W.l, W.h, 10, 48, p=p, strategy=strategy)
    for heavy in (16, 100000):
        got = gpu_search(g, W, 10, 48, strategy=None if strategy == hsig.AUTO else strategy, beam_p=p,
                         waves_per_query=wpq, heavy_queries=heavy, wave_scan=strategy in (hsig.AUTO, hsig.PRE))
        assert_parity(ref, got, f"cooperative wpq={wpq} heavy={heavy}")
        coop = (got[3][:, 3] & 0x200) != 0
        graph = np.isin(got[3][:, 5], [hsig.HYBRID, hsig.POST])
        assert coop[graph].sum() >= min(heavy, graph.sum()), (coop.sum(), heavy)
        assert not coop[~graph].any()
