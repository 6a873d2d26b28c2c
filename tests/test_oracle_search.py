"""Pins of the reference searches (Sec. 4.2: strategies A/B/C, Alg. 1, 2, 7 and the
range-aware rule) against brute force, reachability and exact reductions."""
import numpy as np
import pytest

from oracle import exact, hsig

U32 = 2.0 ** -24


def _truth(W, i, k):
    return exact.rfknn(W.base, W.attr, W.queries[i], W.l[i], W.h[i], k)


def test_pre_filter_equals_exact(small_index, small_workload):
    W = small_workload
    ids, dist = small_index.search(W.queries, W.l, W.h, 10, 64, strategy=hsig.PRE)
    bound = (W.base.shape[1] / 16 + 8) * U32
    for i in range(len(W.queries)):
        tid, td = _truth(W, i, 10)
        assert ids[i, : len(tid)].tolist() == tid.tolist()
        assert (ids[i, len(tid):] == -1).all() and np.isinf(dist[i, len(tid):]).all()
        np.testing.assert_array_less(np.abs(dist[i, : len(tid)] - td), bound * td + 1e-30)


def _bfs(adj_rows, ep):
    seen = {ep}
    todo = [ep]
    while todo:
        v = todo.pop()
        for t in adj_rows(v):
            if t not in seen:
                seen.add(t)
                todo.append(t)
    return seen


@pytest.mark.parametrize("mode", ["hybrid", "post"])
def test_layer0_with_huge_ef_is_brute_force_over_reachable(small_index, small_workload, mode):
    # With ef >= n, ann never fills, the stopping test never fires, and the layer
    # search expands every object reachable from its entry: the result is the
    # brute-force order of the reachable (in-range, for hybrid) objects.
    ix = small_index
    W = small_workload
    adj, gl = ix.layer(0)
    ext = ix.ext_ids()
    Xs = W.base[ext]
    a_sorted = ix.attr_sorted()
    ss, _, _ = ix.segments()
    rng = np.random.default_rng(0)
    for t in range(6):
        q = W.queries[t]
        ep = int(rng.integers(0, ix.n))
        if mode == "hybrid":
            a, b = sorted(rng.integers(0, ix.S, 2))
            c = int(rng.integers(1, ix.M0 + 1))
            lo, hi = ss[a], ss[b + 1]
            l, h = int(a_sorted[lo + 3]), int(a_sorted[hi - 4])
            rows = lambda v: [x for j in range(a, b + 1) for x in adj[v, j, :c] if x >= 0]
            reach = _bfs(rows, ep)
            keep = [v for v in reach if l <= a_sorted[v] <= h]
            got_i, got_d = ix.layer_search(q, ep, 0, ix.n + 5, True, a, b, c, True, l, h)
        else:
            rows = lambda v: [x for x in gl[v] if x >= 0]
            keep = list(_bfs(rows, ep))
            got_i, got_d = ix.layer_search(q, ep, 0, ix.n + 5, False)
        dd = np.array([hsig.dist32(q, Xs[v]) for v in keep], np.float32)
        order = np.lexsort((np.array(keep), dd))
        assert got_i.tolist() == [keep[o] for o in order]
        assert np.array_equal(got_d, dd[order])


def test_upper_layer_search_is_greedy_descent(small_index, small_workload):
    # Alg. 1 with k = 1 keeps one result; from any entry it ends at an object none
    # of whose neighbours (through the same edges) is nearer to q.
    ix = small_index
    W = small_workload
    ext = ix.ext_ids()
    Xs = W.base[ext]
    lev = ix.levels()
    adj, gl = ix.layer(1)
    nodes = np.nonzero(lev >= 1)[0]
    for t in range(10):
        q = W.queries[t]
        ep = int(nodes[t % len(nodes)])
        got, gd = ix.layer_search(q, ep, 1, 1, True, 0, ix.S - 1, ix.MU)
        assert len(got) == 1
        v = int(got[0])
        nb = [x for x in adj[v].reshape(-1) if x >= 0]
        dv = hsig.dist32(q, Xs[v])
        assert all((hsig.dist32(q, Xs[x]), x) >= (dv, v) for x in nb)


def test_batch_form_equals_sequential(small_index, small_workload):
    # Evaluating one expansion's neighbours against the threshold from before the
    # expansion gives the sequential result (p = 1).
    W = small_workload
    for st in (hsig.HYBRID, hsig.POST):
        for ef in (10, 32, 64):
            a = small_index.search(W.queries, W.l, W.h, 10, ef, strategy=st)
            b = small_index.search(W.queries, W.l, W.h, 10, ef, strategy=st, batch_form=True)
            assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_results_in_range_sorted_and_distances_exact(small_index, small_workload):
    W = small_workload
    ext_to_row = {int(e): r for r, e in enumerate(small_index.ext_ids())}
    for st in (hsig.HYBRID, hsig.POST, hsig.AUTO):
        for p in (1, 2, 4):
            ids, dist = small_index.search(W.queries, W.l, W.h, 10, 48, p=p, strategy=st)
            for i in range(len(W.queries)):
                got = ids[i][ids[i] >= 0]
                assert len(set(got.tolist())) == len(got)
                a = W.attr[got]
                assert ((a >= W.l[i]) & (a <= W.h[i])).all()
                d = dist[i, : len(got)]
                keys = [(float(x), ext_to_row[int(g)]) for x, g in zip(d, got)]
                assert keys == sorted(keys)
                for g, x in zip(got, d):
                    assert x == hsig.dist32(W.queries[i], W.base[g])


def test_strategy_rule_thresholds(small_workload):
    # hybrid10k recipe: tau_A = floor(1% n) = 100, tau_B = ceil(50% n) = 5000.
    from synth import workloads as w
    spec = w.scaled(w.SPECS["hybrid10k"], nq=3)
    W = w.make(spec, base_seed=2)
    ix = hsig.Index.build(W.base[:0 + spec.n], W.attr, W.level_u, 2, 4, 8)   # structure irrelevant here
    a = ix.attr_sorted()
    l = np.array([a[0], a[0], a[0], a[0], a[0], a[0]])
    Ys = np.array([99, 100, 101, 4999, 5000, 5001])
    h = a[Ys - 1]
    Q = np.repeat(W.queries[:1], 6, 0)
    _, _, cnt = ix.search(Q, l, h, 5, 16, counters=True)
    assert (cnt[:, hsig.HI] - cnt[:, hsig.LO]).tolist() == Ys.tolist()
    assert cnt[:, hsig.STRAT].tolist() == [hsig.PRE, hsig.PRE, hsig.HYBRID, hsig.HYBRID, hsig.POST, hsig.POST]


def test_edge_cases(small_index, small_workload):
    W = small_workload
    a = small_index.attr_sorted()
    q = W.queries[:4]
    # l > h, a gap between attributes (no object), a single object, k > |R|
    gap = [int(x) + 1 for x in a[:-1] if a[a.searchsorted(x, "right")] > x + 1][:1] or [int(a[-1]) + 10]
    l = np.array([10, gap[0], a[5], a[0]])
    h = np.array([5, gap[0], a[5], a[-1]])
    for st in (hsig.PRE, hsig.HYBRID, hsig.POST, hsig.AUTO):
        ids, dist = small_index.search(q, l, h, 7, 16, strategy=st)
        assert (ids[0] == -1).all() and np.isinf(dist[0]).all()
        assert (ids[1] == -1).all()
        assert (ids[2, 1:] == -1).all()
        if st in (hsig.PRE, hsig.AUTO):          # exact strategies must find the one object
            assert ids[2, 0] == W.attr.tolist().index(a[5]) or W.attr[ids[2, 0]] == a[5]
        assert (ids[3] >= 0).all()
    ids, dist = small_index.search(q[:1], l[3:], h[3:], small_index.n + 3, small_index.n + 3, strategy=hsig.PRE)
    assert (ids[0, : small_index.n] >= 0).all() and (ids[0, small_index.n:] == -1).all()


def test_recall_grows_with_ef(small_index, small_workload):
    # Sec. 5.7: recall rises with ef (m fixed); here averaged over all queries.
    W = small_workload
    rec = []
    for ef in (10, 20, 40, 80):
        ids, _ = small_index.search(W.queries, W.l, W.h, 10, ef, strategy=hsig.HYBRID)
        r = []
        for i in range(len(W.queries)):
            tid, _ = _truth(W, i, 10)
            Y = int(((W.attr >= W.l[i]) & (W.attr <= W.h[i])).sum())
            r.append(exact.recall(ids[i], tid, 10, Y))
        rec.append(np.mean(r))
    assert rec == sorted(rec) and rec[-1] > 0.97, rec


def test_neighbour_selection_brute_force(small_index, small_workload):
    """One expansion's neighbours (Sec. 4.2) against the chunks themselves: S2 = the
    first ceil(m / S') entries of each active chunk in chunk order; S1 = the m entries
    of the active chunks nearest the expanded object, checked with FP64 distances
    (any FP32 rounding can only swap entries whose FP64 distances nearly tie)."""
    ix, W = small_index, small_workload
    ext = ix.ext_ids()
    X = W.base[ext].astype(np.float64)  # rows in internal-id order
    rng = np.random.default_rng(5)
    checked = 0
    for l in (0, 1):
        adj, _ = ix.layer(l)
        lev = ix.levels()
        objs = np.nonzero(lev >= l)[0]
        for o in rng.choice(objs, size=min(40, objs.size), replace=False):
            a = int(rng.integers(0, ix.S))
            b = int(rng.integers(a, ix.S))
            for m in (1, 3, 8, 40):
                sa = b - a + 1
                c = -(-m // sa)
                s2 = ix.neighbours(int(o), l, a, b, m)
                want2 = [int(u) for j in range(a, b + 1) for u in adj[o, j, :c] if u >= 0]
                assert s2.tolist() == want2
                s1 = ix.neighbours(int(o), l, a, b, m, select_s1=True)
                ent = np.array([u for j in range(a, b + 1) for u in adj[o, j] if u >= 0], np.int64)
                assert len(s1) == min(m, ent.size)
                if ent.size == 0:
                    continue
                d64 = ((X[ent] - X[o]) ** 2).sum(1)
                order = np.lexsort((ent, d64))
                t = d64[order[len(s1) - 1]]  # the m-th smallest FP64 distance
                ds1 = ((X[s1] - X[o]) ** 2).sum(1)
                # S1's picks are the nearest: none beyond the m-th FP64 distance,
                # and every entry strictly nearer than it is picked
                assert np.all(ds1 <= t * (1 + 1e-5) + 1e-30)
                nearer = ent[d64 < t * (1 - 1e-5)]
                assert np.isin(nearer, s1).all()
                # in (distance, id) order, duplicates (an object in two chunks) kept
                assert np.all(np.diff(ds1) >= -1e-5 * t - 1e-30)
                checked += 1
    assert checked > 100


def test_selection_s1_special_cases(small_index, small_workload):
    """Hybrid selection S1 (Sec. 4.2: the m entries of the active chunks nearest to
    the expanded object): with m covering every entry it picks the same neighbours as
    S2 (so results are identical); with a smaller m it never examines more than m
    neighbours per expansion; its results are in range, sorted, with exact distances."""
    ix, W = small_index, small_workload
    mall = ix.S * ix.M0
    a = ix.search(W.queries, W.l, W.h, 10, 40, m=mall, strategy=hsig.HYBRID)
    b = ix.search(W.queries, W.l, W.h, 10, 40, m=mall, strategy=hsig.HYBRID, select_s1=True)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    for m in (4, 12):
        ids, dist, cnt = ix.search(W.queries, W.l, W.h, 10, 40, m=m, strategy=hsig.HYBRID, select_s1=True,
                                   counters=True)
        # entry distances of each active segment (<= S per query) plus m per expansion
        assert np.all(cnt[:, hsig.NDIST] <= ix.S + m * cnt[:, hsig.NEXP])
        for i in range(len(ids)):
            row = ids[i][ids[i] >= 0]
            assert np.all((W.attr[row] >= W.l[i]) & (W.attr[row] <= W.h[i]))
            d32 = np.array([hsig.dist32(W.queries[i], W.base[e]) for e in row], np.float32)
            assert np.array_equal(d32, dist[i][: len(row)])
    # S1 and S2 differ once m is smaller than the active entries (the test above is not vacuous)
    s2 = ix.search(W.queries, W.l, W.h, 10, 40, m=4, strategy=hsig.HYBRID, counters=True)
    s1 = ix.search(W.queries, W.l, W.h, 10, 40, m=4, strategy=hsig.HYBRID, select_s1=True, counters=True)
    assert not np.array_equal(s1[2][:, hsig.NDIST], s2[2][:, hsig.NDIST])
