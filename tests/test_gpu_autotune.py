"""The search-parameter tuner (Sec. 5.7's sweep, Sec. 4.2's thresholds from
sample queries): every setting it reports carries the recall that setting
actually reaches (beam width included), and the one it returns is the fastest
of those meeting the target, up to its 2% tie rule."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from synth import workloads as w


def test_tuner_reports_true_recall(tmp_path):
    import torch
    import paper_2412_02448_amd as u
    from paper_2412_02448_amd import autotune
    assert torch.cuda.is_available()
    spec = w.scaled(w.SPECS["hybrid10k"], n=6000, nq=300)
    W = w.make(spec, base_seed=23)
    g = u.Index.build(W.base, W.attr, W.level_u, spec.S, spec.M, spec.ef_cons)
    dev = torch.device("cuda", 0)
    Q, L, H = (torch.from_numpy(a).to(dev) for a in (W.queries, W.l, W.h))
    best, table = autotune.tune(g, Q, L, H, 10, 0.9, ms=(8, 16), efs=(16, 32, 64), ps=(1, 4),
                                taus=((0.01, 0.5), (0.005, 0.3)), pre_chunks=(64, 512), reps=2)
    assert best is not None and best.recall >= 0.9
    truth = autotune.exact_answers(g, Q, L, H, 10)
    assert {s.pre_chunk for s in table} >= {64, 512}
    for s in table:
        ids, _, _ = g.search(Q, L, H, 10, s.ef, **dict(s.kwargs(), visit_cap=0))
        assert autotune.recall_at_k(ids.cpu().numpy(), truth) == pytest.approx(s.recall, abs=0)
    ok = [s for s in table if s.recall >= 0.9 and s.qps > 0 and s.visit_cap == 0 and s.pre_chunk == 0]
    assert best.qps >= 0.98 * max(s.qps for s in ok) or best.visit_cap != 0 or best.pre_chunk != 0
    g.close()


def test_tau_calibration_turning_points():
    """Sec. 4.2's calibration on the GPU: base objects as queries with random ranges,
    every bucket timed under the three strategies; the pre-filter records are exact,
    the thresholds are the turning points of those records, and a search with them
    runs pre-filtering below tau_A and post-filtering above tau_B."""
    import torch
    import paper_2412_02448_amd as u
    from paper_2412_02448_amd import autotune
    assert torch.cuda.is_available()
    spec = w.scaled(w.SPECS["hybrid10k"], n=6000, nq=300)
    W = w.make(spec, base_seed=29)
    g = u.Index.build(W.base, W.attr, W.level_u, spec.S, spec.M, spec.ef_cons)
    rng = np.random.default_rng(1)
    sample = W.base[rng.choice(len(W.base), 512, replace=False)]
    cal = autotune.calibrate_tau(g, sample, W.attr, 10, 32, 0.9, m=16, beam_p=2, buckets=8, per_bucket=64, reps=2)
    assert all(r == 1.0 for r in cal.recall["pre"])
    assert 0.0 <= cal.tau_a <= cal.tau_b <= 1.0
    assert (cal.tau_a, cal.tau_b) == autotune.turning_points(cal.y_lo, cal.y_hi, cal.recall, cal.us_per_query, 0.9,
                                                             len(W.attr))
    assert cal.y_lo == sorted(cal.y_lo) and all(a <= b for a, b in zip(cal.y_lo, cal.y_hi))
    dev = torch.device("cuda", 0)
    Q, L, H = (torch.from_numpy(a).to(dev) for a in (W.queries, W.l, W.h))
    _, _, strat, st = g.search(Q, L, H, 10, 32, m=16, beam_p=2, tau_a=cal.tau_a, tau_b=cal.tau_b, stats=True)
    strat, y = strat.cpu().numpy(), st.cpu().numpy()[:, 6]
    n = len(W.attr)
    assert (strat[(y > 0) & (y <= np.floor(cal.tau_a * n))] == u.PRE).all()
    assert (strat[y >= np.ceil(cal.tau_b * n)] == u.POST).all()
    g.close()
