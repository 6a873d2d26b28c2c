"""Benchmark: range-filtered k-NN search over HSIG on one MI355X.

Workload (synthetic, seeded): 1,000,000 x 128 FP32 vectors from a 1024-centre
Gaussian mixture (sigma 0.2), attribute uniform in [0, 2^31), HSIG with 32
segments and M = 32 (built on the GPU), 10,000 queries from the same mixture
with range fraction log-uniform in [1e-3, 1], k = 10.  One step = one search of
the whole 10,000-query batch with the range-aware strategy (plan, pre-filter
scans, hybrid and post-filter searches, FP32 rerank), inputs already resident
in HBM, run as one replay of the captured launch sequence (unify_batch_run); the
same step through per-call launches (unify_search) is reported beside it.

For each vector store (FP32, and BF16 / FP8 E4M3 copies ranked in low precision
and re-scored in FP32), (m, ef, beam width) is tuned on 10,000 held-out queries
of the same recipe for recall@10 >= 0.95 against the exact answer (the
pre-filter scan forced on every query), then the batch is timed.  The headline
value is the fastest store whose recall on the benchmark queries reaches the
target (stores within 2% of the fastest are a tie, which the most accurate of
them wins).  The JSON line also reports every store, each strategy timed
separately, the roofline of the search kernel (algorithmic bytes from the
kernel's own counters / its HIP-event duration) and the CPU oracle's HSIG
search on the same index as a baseline.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import tempfile
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
# HIP shares GPU_MAX_HW_QUEUES hardware queues (4 by default) among a process's streams,
# and kernels of streams that share a queue run one after another: the serving slots,
# the index's side streams and the default stream each get a queue of their own.
os.environ.setdefault("GPU_MAX_HW_QUEUES", "8")

HBM_PEAK_GBS = 8000.0
# searches whose HIP-event phases are averaged for the rooflines (each synchronised)
TIMED_REPS = 10
HOST_SHARE = 16  # host cores that go with one GPU of the box
METRIC = "QPS @ recall@10≥0.95, 1M×128 mixed ranges, FP32 vs BF16/FP8; HBM GB/s"
PRECISIONS = ("fp32", "bf16", "fp8")
DTYPE = {"fp32": "f32", "bf16": "bf16", "fp8": "fp8e4m3"}
KCODE = {"fp32": 0, "bf16": 1, "fp8": 2}
TUNE_MARGIN = 0.003


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--ef", type=int, default=0, help="fixed ef (0: tuned)")
    ap.add_argument("--m", type=int, default=0, help="fixed neighbour budget m (0: tuned)")
    ap.add_argument("--p", type=int, default=0, help="fixed beam width (0: tuned)")
    ap.add_argument("--tau-a", type=float, default=0.0, help="fixed tau_A fraction (0: tuned, with --tau-b)")
    ap.add_argument("--tau-b", type=float, default=0.5, help="tau_B fraction used with --tau-a")
    ap.add_argument("--visit-cap", type=int, default=0,
                    help="visited-cache entries for --profile-run and the --c5-only server (0: default)")
    ap.add_argument("--precisions", default=",".join(PRECISIONS),
                    help="comma-separated vector stores to measure (fp32, bf16, fp8)")
    ap.add_argument("--recall-target", type=float, default=0.95)
    ap.add_argument("--n", type=int, default=0, help="override n (smaller runs for development only)")
    ap.add_argument("--profile-run", action="store_true",
                    help="profiling run: one store (--precisions), fixed --m/--ef/--p, only the timed steps "
                         "and one counted call (every search-kernel launch has the same configuration)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch100k", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-wide", action="store_true")
    ap.add_argument("--no-insert", action="store_true")
    ap.add_argument("--no-multi", action="store_true")
    ap.add_argument("--wide-n", type=int, default=1_000_000, help="objects of the 960-wide workload")
    ap.add_argument("--wide-M", type=int, default=0, help="chunk capacity of the 960-wide index (0: the recipe's)")
    ap.add_argument("--wide-efc", type=int, default=256,
                    help="efCons of the 960-wide index (0: the recipe's 100, which leaves layer 0 without links "
                         "out of a cluster at n = 1M: 244 objects of a cluster per segment, more than 100 candidates)")
    ap.add_argument("--cpu-queries", type=int, default=0, help="queries in the CPU sample (0: all)")
    ap.add_argument("--wpq", type=int, default=0, help="wavefronts per heavy graph search (0: the library default)")
    ap.add_argument("--heavy", type=int, default=0, help="heavy graph searches per batch (0: the library default)")
    ap.add_argument("--inflight", type=int, default=3, help="serving slots in flight")
    ap.add_argument("--wave-scan", action="store_true",
                    help="--profile-run: pre-filter scans per wavefront instead of the matrix-core scan")
    ap.add_argument("--c5-only", action="store_true",
                    help="only the 10M x 96 serving configuration (S = 64, M = 24): GPU build, recall, "
                         "Poisson serving at 5k-100k requests/s for k = 10 and k = 100; prints its record")
    ap.add_argument("--serving-only", action="store_true",
                    help="development/profiling run: build the index, then only the serving section with one "
                         "store (--precisions) and --m/--ef/--p (no tuning); prints the serving record")
    return ap.parse_args()


def bytes_per_query(st, d, k, prec):
    """Algorithmic HBM bytes of each query from its kernel counters:
    distances to the ranking store (d * b bytes, + 4 B scale for FP8, + 4 B error
    bound for pre-filter rows of a low-precision store), FP32 re-scores (d * 4),
    adjacency entries read (4 B), the query vector and the k outputs."""
    b = {"fp32": 4, "bf16": 2, "fp8": 1}[prec]
    row = d * b + (4 if prec == "fp8" else 0)
    pre = st[:, 5] == 1
    per_dist = row + ((4 if prec != "fp32" else 0) * pre)
    return st[:, 0] * per_dist + st[:, 2] * d * 4 + st[:, 4] * 4 + (st[:, 5] >= 0) * (d * 4 + k * 12)


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: every box here has one MI355X; run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2412_02448_amd as u
    from synth import workloads as w

    precs = [p for p in args.precisions.split(",") if p]
    assert all(p in PRECISIONS for p in precs), precs
    if args.c5_only:
        print(json.dumps({"c5": c5_bench(args)}), flush=True)
        return
    spec = w.SPECS["mixed1m"]
    if args.n:
        spec = w.scaled(spec, n=args.n)
    dev = torch.device("cuda", 0)
    t0 = time.time()
    W = w.make(spec, base_seed=0)
    log(f"workload {spec.name}: n={spec.n} d={spec.d} nq={len(W.queries)} ({time.time() - t0:.1f}s)")
    t0 = time.time()
    index = u.Index.build(W.base, W.attr, W.level_u, spec.S, spec.M, spec.ef_cons, device=0)
    build_s = time.time() - t0
    log(f"GPU build: {build_s:.1f}s, {index.levels} layers")

    Q = torch.from_numpy(W.queries).to(dev)
    L = torch.from_numpy(W.l).to(dev)
    H = torch.from_numpy(W.h).to(dev)
    nq, k, d = Q.shape[0], spec.k, spec.d
    # A copy of known size, for scaling HBM counters in a profiling run.
    cp_src = torch.empty(256 << 20, dtype=torch.uint8, device=dev)
    cp_dst = torch.empty_like(cp_src)
    cp_dst.copy_(cp_src)

    if args.serving_only:
        if not (args.m and args.ef and args.p and len(precs) == 1):
            print("--serving-only needs --m, --ef, --p and one store in --precisions", file=sys.stderr)
            sys.exit(2)
        index.set_precision(precs[0])
        rec = serve_bench(args, index, spec, W, args.m, args.ef, args.p, 0.01, 0.5, 0, precs[0])
        print(json.dumps({"serving": rec}), flush=True)
        return

    if args.profile_run:
        if not (args.m and args.ef and args.p and len(precs) == 1):
            print("--profile-run needs --m, --ef, --p and one store in --precisions", file=sys.stderr)
            sys.exit(2)
        return profile_run(args, index, Q, L, H, k, spec, nq, build_s, precs[0])

    # exact answer: the FP32 pre-filter scan on every query
    t0 = time.time()
    truth, _, _ = index.search(Q, L, H, k, k, strategy=u.PRE)
    torch.cuda.synchronize()
    truth = truth.cpu().numpy()
    log(f"exact answers by forced pre-filter scan ({time.time() - t0:.1f}s)")

    def recall_of(ids, rows=None):
        ids = ids.cpu().numpy()
        rows = range(nq) if rows is None else rows
        r = []
        for i in rows:
            t = truth[i][truth[i] >= 0]
            if t.size == 0:
                r.append(1.0)
                continue
            r.append(len(set(ids[i][ids[i] >= 0].tolist()) & set(t.tolist())) / t.size)
        return float(np.mean(r)) if r else 1.0

    from paper_2412_02448_amd import autotune
    # held-out tuning queries: as many as the benchmark batch, so that the tuner sees the
    # same batch dynamics (the longest searches bound a step)
    cq, cl, ch, _ = w.more_queries(spec, W.attr, len(W.queries), base_seed=0, stream=1)
    Qc = torch.from_numpy(cq).to(dev)
    Lc = torch.from_numpy(cl).to(dev)
    Hc = torch.from_numpy(ch).to(dev)

    coop = {"waves_per_query": args.wpq, "heavy_queries": args.heavy}

    def timed(m, ef, bp, strategy=None, steps=args.steps, warmup=args.warmup, ta=0.01, tb=0.5, vc=0, **kw):
        # cooperative searches do not run selection S1
        kw = {**({} if kw.get("select_s1") else coop), **kw}
        out = None
        for _ in range(warmup):
            out = index.search(Q, L, H, k, ef, strategy=strategy, m=m, beam_p=bp, tau_a=ta, tau_b=tb, visit_cap=vc, **kw)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            out = index.search(Q, L, H, k, ef, strategy=strategy, m=m, beam_p=bp, tau_a=ta, tau_b=tb, visit_cap=vc, **kw)
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / steps, out

    # ---- every store: tune on held-out queries, then K timed steps of the batch ----
    by_prec = {}
    store_rows = {}  # store -> (ids, dist) of the timed batch, scored against FP64 in the CPU leg
    for prec in precs:
        index.set_precision(prec)
        t0 = time.time()
        ms_grid = (args.m,) if args.m else None
        efs_grid = (args.ef,) if args.ef else (16, 24, 32, 48, 64, 128, 256)
        ps_grid = (args.p,) if args.p else (2, 3, 4, 6, 8)
        if not args.m:
            Mi = index.M
            ms_grid = (Mi // 2, (3 * Mi) // 4, Mi, (3 * Mi) // 2, 2 * Mi, 3 * Mi)
        kw_t = {"taus": ((args.tau_a, args.tau_b),)} if args.tau_a else {}
        cal = None
        if not args.tau_a:
            # Sec. 4.2: base objects as sample queries with random ranges, the three strategies
            # timed per cardinality bucket; the turning points join the tuner's threshold grid
            rs = np.random.default_rng(41)
            sample = W.base[rs.choice(len(W.base), 8192, replace=False)]
            cal = autotune.calibrate_tau(index, sample, W.attr, k, 32, args.recall_target, m=2 * index.M, beam_p=4,
                                         log=lambda s, p=prec: log(f"[{p}] {s}"))
            log(f"[{prec}] calibrated tau = ({cal.tau_a:.6f}, {cal.tau_b:.6f})")
            kw_t = {"taus": ((cal.tau_a, cal.tau_b), (0.01, 0.5), (0.02, 0.5), (0.03, 0.5), (0.01, 0.3),
                             (0.005, 0.3))}
        # a small margin above the target on the held-out queries keeps the benchmark
        # queries above it too
        # the knobs that leave results unchanged: the per-wavefront pre-filter scan against the
        # matrix-core scan, and 2 or 4 wavefronts for the heaviest graph searches
        coop.pop("wave_scan", None)
        if not args.wpq:
            coop["waves_per_query"] = 0
        best, table = autotune.tune(index, Qc, Lc, Hc, k, args.recall_target + TUNE_MARGIN, ms=ms_grid,
                                    efs=efs_grid, ps=ps_grid, log=lambda s, p=prec: log(f"[{p}] {s}"),
                                    wave_scans=(True,), wpqs=() if args.wpq else (2, 4), **kw_t)
        if best is None:
            best = max(table, key=lambda s: s.recall)
        m, ef, bp, ta, tb, vc = best.m, best.ef, best.beam_p, best.tau_a, best.tau_b, best.visit_cap
        coop["wave_scan"] = best.wave_scan
        if not args.wpq:
            coop["waves_per_query"] = best.waves_per_query
        log(f"[{prec}] tuned on {Qc.shape[0]} held-out queries ({time.time() - t0:.1f}s): m={m} ef={ef} p={bp} "
            f"tau=({ta}, {tb})")
        sec, out = timed(m, ef, bp, ta=ta, tb=tb, vc=vc)
        rec = recall_of(out[0])
        store_rows[prec] = (out[0].cpu().numpy(), out[1].cpu().numpy())
        ph, _, (ids, _, _, stats) = timed_calls(index, Q, L, H, k, ef, m=m, beam_p=bp, tau_a=ta, tau_b=tb,
                                                visit_cap=vc, **coop)
        pre_ms, rerun_ms = ph["plan"], ph["rerun"]
        search_ms = ph["search"]
        st = stats.cpu().numpy().astype(np.int64)
        first = ((st[:, 3] & 0xFF) == 0) & ~tile_rows(st)
        bts = int(bytes_per_query(st, d, k, prec)[first].sum())
        by_prec[prec] = {
            "qps": round(nq / sec, 1), "ms_per_step": round(sec * 1e3, 4), "recall@10": round(rec, 4),
            "m": m, "ef": ef, "beam_p": bp, "tau_a": ta, "tau_b": tb, "visit_cap": vc,
            "wave_scan": bool(coop["wave_scan"]), "waves_per_query": int(coop["waves_per_query"] or 1),
            "search_launch_ms": round(search_ms, 4),
            "plan_ms": round(pre_ms, 4), "rerun_launch_ms": round(rerun_ms, 4),
            "rerun_queries": int(((st[:, 3] & 0xFF) == 1).sum()), "failed_queries": int(((st[:, 3] & 0xFF) == 2).sum()),
            "bytes_per_launch": bts, "achieved_GBps": round(bts / (search_ms * 1e-3) / 1e9, 1),
            "fp32_rescores_per_query": round(float(st[:, 2].mean()), 2),
            "same_ids_as_stats_call": bool((ids == out[0]).all().item()),
            "phases_ms": {kk: round(v, 4) for kk, v in ph.items()},
            "tile_scan": tile_roofline(st, ph, d, k, prec, spec.n),
            "tau_calibration": None if cal is None else {
                "tau_a": round(cal.tau_a, 6), "tau_b": round(cal.tau_b, 6), "setting": "k=10 ef=32 m=2M p=4",
                "chosen": bool(abs(ta - cal.tau_a) < 1e-12 and abs(tb - cal.tau_b) < 1e-12),
                "buckets": [{"y": [a, b], "recall": [round(cal.recall[s_][i], 3) for s_ in ("pre", "hybrid", "post")],
                             "us_per_query": [round(cal.us_per_query[s_][i], 3) for s_ in ("pre", "hybrid", "post")]}
                            for i, (a, b) in enumerate(zip(cal.y_lo, cal.y_hi))]},
        }
        log(f"[{prec}] {nq / sec:,.0f} QPS ({sec * 1e3:.3f} ms/step), recall@10 {rec:.4f}; search kernel "
            f"{search_ms:.3f} ms, {by_prec[prec]['achieved_GBps']} GB/s algorithmic, rerun {rerun_ms:.3f} ms "
            f"({by_prec[prec]['rerun_queries']} queries)")

    ok = [p for p in precs if by_prec[p]["recall@10"] >= args.recall_target]
    if ok:
        # stores within 2% of the fastest are within the timing noise: the most accurate of them
        top = max(by_prec[p]["qps"] for p in ok)
        head = max((p for p in ok if by_prec[p]["qps"] >= 0.98 * top), key=lambda p: by_prec[p]["recall@10"])
    else:
        head = max(precs, key=lambda p: by_prec[p]["recall@10"])
    H0 = by_prec[head]
    m, ef, bp, ta, tb, vc = H0["m"], H0["ef"], H0["beam_p"], H0["tau_a"], H0["tau_b"], H0["visit_cap"]
    coop["wave_scan"] = H0["wave_scan"]
    if not args.wpq:
        coop["waves_per_query"] = H0["waves_per_query"]
    index.set_precision(head)
    log(f"headline store: {head} (m={m} ef={ef} p={bp} tau=({ta}, {tb}))")

    # the auto strategy's QPS-recall curve over the ef grid of the 1M configuration (headline store)
    recalls, qps_by_ef = {}, {}
    for e in (32, 64, 128, 256):
        s_e, o_e = timed(m, e, bp, steps=3, warmup=1, ta=ta, tb=tb, vc=vc)
        recalls[e] = recall_of(o_e[0])
        qps_by_ef[e] = round(nq / s_e, 1)
    log("recall@10 by ef: " + ", ".join(f"ef={e}: {r:.4f} ({qps_by_ef[e]:,.0f} QPS)" for e, r in recalls.items()))

    # ---- timed region of the headline: K steps of the whole path ----
    # A step is one replay of the captured launch sequence (plan, work list, search, merge,
    # re-run) over the resident batch; the same step through per-call launches is reported
    # beside it.
    sec_eager, out_eager = timed(m, ef, bp, ta=ta, tb=tb, vc=vc)
    batch = u.Batch(index, Q, L, H, k, ef, m=m, beam_p=bp, tau_a=ta, tau_b=tb, visit_cap=vc, **coop)
    for _ in range(args.warmup):
        batch.run()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        batch.run()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t) / args.steps
    out = (batch.ids, batch.dist)
    same = bool(torch.equal(batch.ids, out_eager[0]))
    batch.close()  # the output tensors stay
    qps = nq / sec
    log(f"auto ({head}): {qps:,.0f} QPS ({sec * 1e3:.3f} ms/step) as a graph replay; "
        f"{nq / sec_eager:,.0f} QPS ({sec_eager * 1e3:.3f} ms/step) through per-call launches; same ids {same}")
    # the same step from pinned host buffers: queries and ranges copied in, results copied out
    # (the boundary takes device buffers; this is the rate a host-side caller sees)
    hq, hl, hh = Q.cpu().pin_memory(), L.cpu().pin_memory(), H.cpu().pin_memory()
    hids = torch.empty((nq, k), dtype=torch.int64).pin_memory()
    hdist = torch.empty((nq, k), dtype=torch.float32).pin_memory()
    dq, dl, dh = torch.empty_like(Q), torch.empty_like(L), torch.empty_like(H)

    def host_step():
        dq.copy_(hq, non_blocking=True)
        dl.copy_(hl, non_blocking=True)
        dh.copy_(hh, non_blocking=True)
        o = index.search(dq, dl, dh, k, ef, m=m, beam_p=bp, tau_a=ta, tau_b=tb, visit_cap=vc, **coop)
        hids.copy_(o[0], non_blocking=True)
        hdist.copy_(o[1], non_blocking=True)

    for _ in range(args.warmup):
        host_step()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        host_step()
    torch.cuda.synchronize()
    sec_host = (time.perf_counter() - t) / args.steps
    host_same = bool(torch.equal(hids, out[0].cpu()))
    # the copies alone, for the split of that step
    t = time.perf_counter()
    for _ in range(args.steps):
        dq.copy_(hq, non_blocking=True)
        dl.copy_(hl, non_blocking=True)
        dh.copy_(hh, non_blocking=True)
    torch.cuda.synchronize()
    sec_in = (time.perf_counter() - t) / args.steps
    t = time.perf_counter()
    for _ in range(args.steps):
        hids.copy_(out[0], non_blocking=True)
        hdist.copy_(out[1], non_blocking=True)
    torch.cuda.synchronize()
    sec_out = (time.perf_counter() - t) / args.steps
    in_b = hq.numel() * 4 + hl.numel() * 8 + hh.numel() * 8
    out_b = hids.numel() * 8 + hdist.numel() * 4
    log(f"from pinned host buffers (PCIe copies in the step): {nq / sec_host:,.0f} QPS "
        f"({sec_host * 1e3:.3f} ms/step); same ids {host_same}; copies alone: in {sec_in * 1e3:.3f} ms "
        f"({in_b / sec_in / 1e9:.1f} GB/s), out {sec_out * 1e3:.3f} ms ({out_b / sec_out / 1e9:.1f} GB/s)")
    per_strategy = {}
    for name, sv in (("pre", u.PRE), ("hybrid", u.HYBRID), ("post", u.POST)):
        s, o = timed(m, ef, bp, sv, steps=max(1, args.steps // 2 + 1), warmup=1, ta=ta, tb=tb, vc=vc)
        per_strategy[name] = {"qps": round(nq / s, 1), "recall@10": round(recall_of(o[0]), 4)}
        log(f"{name}: {nq / s:,.0f} QPS recall {per_strategy[name]['recall@10']}")
    # each strategy timed separately on the FP32 store over the ef grid of the 1M configuration
    index.set_precision("fp32")
    fp32_by_ef = {}
    for e in (32, 64, 128, 256):
        row = {}
        for name, sv in (("auto", None), ("pre", u.PRE), ("hybrid", u.HYBRID), ("post", u.POST)):
            s, o = timed(m, e, bp, sv, steps=2, warmup=1, ta=ta, tb=tb, vc=vc)
            row[name] = {"qps": round(nq / s, 1), "recall@10": round(recall_of(o[0]), 4)}
        fp32_by_ef[e] = row
        log(f"fp32 ef={e}: " + ", ".join(f"{nm} {r['qps']:,.0f} QPS r={r['recall@10']}" for nm, r in row.items()))
    index.set_precision(head)

    # ---- hybrid neighbour selections S1 and S2 (Sec. 4.2) on the forced hybrid search ----
    selection = {}
    for sel_name, s1 in (("S2", False), ("S1", True)):
        for e in (16, 32, 64, 128):
            s, o = timed(m, e, bp, u.HYBRID, steps=max(1, args.steps // 2 + 1), warmup=1, ta=ta, tb=tb, vc=vc,
                         select_s1=s1)
            selection[f"{sel_name}_ef{e}"] = {"qps": round(nq / s, 1), "recall@10": round(recall_of(o[0]), 4)}
        log(f"hybrid selection {sel_name}: " + ", ".join(
            f"ef={e}: {selection[f'{sel_name}_ef{e}']['qps']:,.0f} QPS r={selection[f'{sel_name}_ef{e}']['recall@10']}"
            for e in (16, 32, 64, 128)))

    # ---- roofline of the search kernel: counters of identical calls, HIP events averaged ----
    phases, (smin, smax), (ids, dist, strat, stats) = timed_calls(index, Q, L, H, k, ef, m=m, beam_p=bp, tau_a=ta,
                                                                  tau_b=tb, visit_cap=vc, **coop)
    pre_ms, rerun_ms = phases["plan"], phases["rerun"]
    search_ms = phases["search"]
    st = stats.cpu().numpy().astype(np.int64)
    first = ((st[:, 3] & 0xFF) == 0) & ~tile_rows(st)
    bytes_first = int(bytes_per_query(st, d, k, head)[first].sum())
    achieved = bytes_first / (search_ms * 1e-3) / 1e9
    copy_gbs = copy_peak(torch, dev)
    log(f"device copy: {copy_gbs:,.0f} GB/s (read + write)")
    mix = np.bincount(np.maximum(st[:, 5], 0), minlength=4)
    kern = f"k_search<*, {KCODE[head]}, 0, false>"
    roofline = {"bound": "hbm", "kernel": f"{kern} (first pass)", "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": profiled_traffic(head, m, ef, bp, ta, tb, vc, coop.get("wave_scan"),
                                            coop.get("waves_per_query")), "bytes_per_launch": bytes_first,
                "launch_ms": round(search_ms, 4), "launch_ms_min_max": [round(smin, 4), round(smax, 4)],
                "timed_calls": TIMED_REPS, "rerun_launch_ms": round(rerun_ms, 4),
                "measured_copy_GBps": round(copy_gbs, 1), "frac_of_copy": round(achieved / copy_gbs, 4),
                "rerun_queries": int(((st[:, 3] & 0xFF) == 1).sum()), "failed_queries": int(((st[:, 3] & 0xFF) == 2).sum()),
                "phases_ms": {kk: round(v, 4) for kk, v in phases.items()}}
    # the whole step against the same peak, two ways.  Batched reads: the graph searches' and
    # the per-wavefront scans' algorithmic bytes, plus the matrix-core scan's super-blocks,
    # each read once per group of up to 16 queries (rows, norms, bounds), its FP32 re-scores
    # and each query's vector and outputs.  Per-query sum (every pre-filter query's own whole
    # slice, however many queries share its rows): it counts shared rows again and can pass
    # the peak, so it bounds nothing; it is reported for comparison only.
    per_q = bytes_per_query(st, d, k, head)
    trows = tile_rows(st)
    items = tile_items(W, st, spec.n)
    b = {"fp32": 4, "bf16": 2, "fp8": 1}[head]
    blk_row = d * b + 4 + (4 if head != "fp32" else 0) + (4 if head == "fp8" else 0)
    tile_b = items * TILE_ROWS * blk_row + int((st[trows, 2] * d * 4).sum()) + int(trows.sum()) * (d * 4 + k * 12)
    step_bytes = int(per_q[~trows].sum()) + int(tile_b)
    roofline["step_algorithmic_bytes"] = step_bytes
    roofline["step_tile_items"] = int(items)
    roofline["step_GBps"] = round(step_bytes / sec / 1e9, 1)
    roofline["step_frac"] = round(step_bytes / sec / 1e9 / HBM_PEAK_GBS, 4)
    roofline["step_bytes_per_query_sum"] = int(per_q.sum())
    roofline["step_GBps_per_query_sum"] = round(int(per_q.sum()) / sec / 1e9, 1)
    roofline["wave_scan"] = bool(coop.get("wave_scan"))
    roofline["waves_per_query"] = int(coop.get("waves_per_query") or 1)
    roofline_tile = tile_roofline(st, phases, d, k, head, spec.n)
    ids_np = ids.cpu().numpy()
    for sname, sv in (("pre", 1), ("hybrid", 2), ("post", 3)):
        sel = np.nonzero(st[:, 5] == sv)[0]
        if sel.size:
            per_strategy.setdefault(sname, {})["recall@10_in_auto"] = round(recall_of(ids, sel), 4)
    log(f"search kernel {search_ms:.3f} ms, rerun {rerun_ms:.3f} ms, {achieved:.1f} GB/s algorithmic")

    # ---- batched form: 100k queries on the 10k index, one graph replay per step ----
    b100 = None
    if not args.no_batch100k:
        try:
            b100 = batch100k(args, "fp32")  # the batched form of the plain FP32 search
        except Exception as e:  # the headline line is still reported
            log(f"batch100k failed: {e!r}")
            b100 = {"failed": repr(e)}

    # ---- the small plain-FP32 hybrid configuration ----
    c1 = None
    try:
        c1 = c1_bench(args)
    except Exception as e:  # the headline line is still reported
        log(f"c1 failed: {e!r}")
        c1 = {"failed": repr(e)}

    # ---- the 960-wide workload: every store on the GIST-like shape ----
    wide = None
    if not args.no_wide:
        try:
            wide = wide_bench(args)
        except Exception as e:  # the headline line is still reported
            log(f"wide workload failed: {e!r}")
            wide = {"failed": repr(e)}

    # ---- conjunctive queries: a second attribute, range fraction log-uniform in [0.05, 1] ----
    multi = None
    if not args.no_multi:
        try:
            multi = multi_bench(args, index, spec, W, Q, L, H, k, m, ef, bp, ta, tb, vc, head)
        except Exception as e:  # the headline line is still reported
            log(f"conjunctive queries failed: {e!r}")
            multi = {"failed": repr(e)}

    # ---- incremental insertion: 200k objects, then four insertions of 200k (1M in the end) ----
    ins = None
    if not args.no_insert:
        try:
            ins = insert_bench(args, spec, W, Q, L, H, k, m, ef, bp, ta, tb, vc, head, build_s,
                               recall_of(out[0]), nq / sec)
        except Exception as e:  # the headline line is still reported
            log(f"insertion failed: {e!r}")
            ins = {"failed": repr(e)}

    # ---- serving: open-loop Poisson arrivals through the continuous-batching server ----
    serving = None
    if not args.no_serving:
        try:
            serving = serve_bench(args, index, spec, W, m, ef, bp, ta, tb, vc, head)
        except Exception as e:  # the headline line is still reported
            log(f"serving failed: {e!r}")
            serving = {"failed": repr(e)}

    # ---- CPU baseline: the oracle's HSIG search on the same index ----
    cpu = None
    fp64 = None
    if not args.no_cpu_baseline:
        try:
            cpu = cpu_baseline(args, W, index, ids_np, k, ef, m, bp, ta, tb, nq, head)
        except Exception as e:  # the GPU line is still reported
            log(f"CPU baseline failed: {e!r}")
            cpu = {"value": None, "unit": "queries/s", "cores": 0, "kind": "oracle", "sample": f"failed: {e!r}"}
        try:
            store_rows["headline_graph_replay"] = (out[0].cpu().numpy(), out[1].cpu().numpy())
            fp64 = fp64_scoring(W, truth, store_rows, k, st[:, 6])
        except Exception as e:  # the GPU line is still reported
            log(f"FP64 scoring failed: {e!r}")
            fp64 = {"failed": repr(e)}
    line = {
        "metric": METRIC, "value": round(qps, 1), "unit": "queries/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(sec * 1e3, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": DTYPE[head], "data": "synthetic",
        "config": {"workload": f"mixed1m: n={spec.n} d={spec.d} (1024-centre mixture, sigma 0.2), attribute "
                               f"uniform in [0, 2^31), HSIG S={spec.S} M={spec.M} efCons={spec.ef_cons} built on GPU; "
                               f"{nq} queries, range fraction log-uniform [1e-3, 1], k={k}, auto strategy",
                   "n": spec.n, "d": d, "nq": nq, "k": k, "store": head, "ef": ef, "m": m, "beam_p": bp,
                   "tau_a": ta, "tau_b": tb, "visit_cap": vc,
                   "recall@10": round(recall_of(out[0]), 4),
                   "recall@10_vs_fp64_sample": (fp64 or {}).get("headline_graph_replay", {}).get("recall@10"),
                   "qps_by_ef": {str(e_): v for e_, v in qps_by_ef.items()}, "recall_by_ef": {str(e): round(r, 4) for e, r in recalls.items()},
                   "strategy_mix": {"pre": int(mix[1]), "hybrid": int(mix[2]), "post": int(mix[3])},
                   "build_s": round(build_s, 1)},
        "eager": {"qps": round(nq / sec_eager, 1), "ms_per_step": round(sec_eager * 1e3, 4),
                  "same_ids_as_graph": same},
        "host_buffers": {"qps": round(nq / sec_host, 1), "ms_per_step": round(sec_host * 1e3, 4),
                         "same_ids_as_graph": host_same, "copy_in_ms": round(sec_in * 1e3, 4),
                         "copy_out_ms": round(sec_out * 1e3, 4), "copy_in_bytes": int(in_b),
                         "copy_out_bytes": int(out_b),
                         "what": "per-call search with the queries and ranges copied from pinned host "
                                 "memory and the ids and distances copied back inside the step"},
        "by_precision": by_prec,
        "per_strategy": per_strategy,
        "fp32_strategies_by_ef": fp32_by_ef,
        "hybrid_selection": selection,
        "roofline": roofline,
        "roofline_tile_scan": roofline_tile,
        "fp64_check": fp64,
        "batch100k": b100,
        "wide960": wide,
        "insertion": ins,
        "two_attribute": multi,
        "serving": serving,
        "c1_hybrid_fp32": c1,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


TILE_ROWS, TILE_Q = 256, 16  # objects per super-block and queries per item of the matrix-core scan


def tile_items(W, st, n):
    """Work items of the matrix-core scan: every super-block its queries' slices touch, once
    per group of up to 16 of those queries."""
    import numpy as np
    rows = tile_rows(st)
    if not rows.any():
        return 0
    asorted = np.sort(W.attr)
    lo = np.searchsorted(asorted, W.l, "left")[rows]
    hi = np.searchsorted(asorted, W.h, "right")[rows]
    cnt = np.zeros((n + TILE_ROWS - 1) // TILE_ROWS + 1, np.int64)
    np.add.at(cnt, lo // TILE_ROWS, 1)
    np.add.at(cnt, (hi - 1) // TILE_ROWS + 1, -1)
    per_sb = np.cumsum(cnt)[:-1]
    return int(((per_sb + TILE_Q - 1) // TILE_Q).sum())


def tile_rows(st):
    """Rows answered by the matrix-core pre-filter scan (stats[4] = its super-block records)."""
    return (st[:, 5] == 1) & (st[:, 4] > 0)


def tile_roofline(st, ph, d, k, prec, n):
    """The matrix-core pre-filter scan: its kernel time (HIP events around it), the products
    it runs on the matrix cores, and the bytes of the super-blocks it reads.  Every super-block
    a record names is read once per group of up to 16 queries; the per-query algorithmic
    bytes (Y d b summed over the queries) are reported beside them."""
    import numpy as np
    rows = tile_rows(st)
    if not rows.any():
        return None
    b = {"fp32": 4, "bf16": 2, "fp8": 1}[prec]
    row_b = d * b + 4 + (4 if prec != "fp32" else 0) + (4 if prec == "fp8" else 0)  # + norm, eps, scale
    Y = st[rows, 6].astype(np.int64)
    alg_bytes = int((Y * d * b).sum())
    # products: each (query, object in range) pair is one d-long dot product; BF16 inputs run it twice
    # (the query in two parts)
    alg_flop = int((Y * 2 * d).sum()) * (2 if prec != "fp32" else 1)
    ms = ph["tile_scan"]
    peak = 2500.0 if prec != "fp32" else 157.3
    tf = alg_flop / (ms * 1e-3) / 1e12 if ms > 0 else None
    return {"bound": "hbm", "kernel": f"k_tile_scan<{KCODE[prec]}>", "launch_ms": round(ms, 4),
            "setup_ms": round(ph["tile_setup"], 4), "final_ms": round(ph["tile_final"], 4),
            "queries": int(rows.sum()), "records": int(st[rows, 4].sum()),
            "per_query_bytes": alg_bytes, "per_query_GBps": round(alg_bytes / (ms * 1e-3) / 1e9, 1) if ms > 0 else None,
            "row_bytes": row_b, "mfma_flop": alg_flop, "mfma_TFLOPs": round(tf, 2) if tf else None,
            "mfma_peak_TFLOPs": peak, "mfma_frac": round(tf / peak, 5) if tf else None,
            "fp32_rescores_per_query": round(float(st[rows, 2].mean()), 2)}


def copy_peak(torch, dev):
    """Device-to-device copy bandwidth (bytes read + written per second), the achievable
    HBM rate beside the 8 TB/s specification."""
    a = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s0.record()
    for _ in range(10):
        b.copy_(a)
    s1.record()
    torch.cuda.synchronize()
    gbs = 10 * 2 * a.numel() / (s0.elapsed_time(s1) * 1e-3) / 1e9
    del a, b
    return gbs


def fp64_scoring(W, truth_gpu, rows, k, Ysize, nsample=1000):
    """Part of the CPU leg: the exact FP64 answer (Definition 1, the oracle's brute force) of a
    fixed sample of queries spread over all range sizes (every (nq / nsample)-th query in order of
    Y), recall@10 of each store's rows against it (Eq. 1), the relative error of every returned
    distance against the FP64 distance of the same object, and how often the GPU's exact scan
    (the recall truth of the rest of the line) returns the FP64 answer."""
    import concurrent.futures as cf

    import numpy as np
    from oracle import exact
    nq = len(W.queries)
    order = np.argsort(Ysize, kind="stable")
    sample = np.sort(order[np.linspace(0, nq - 1, min(nsample, nq)).astype(np.int64)])
    ext = np.arange(len(W.attr), dtype=np.int64)
    perm = np.lexsort((ext, W.attr))
    Xs, As, Es = W.base[perm], W.attr[perm], ext[perm]
    t0 = time.time()
    ncpu = min(HOST_SHARE, len(os.sched_getaffinity(0)))

    def one(i):
        ids, dd, size = exact.rfknn_sorted(Xs, As, W.queries[i], W.l[i], W.h[i], k, Es)
        return ids, dd, size
    with cf.ThreadPoolExecutor(max_workers=ncpu) as pool:
        res = list(pool.map(one, sample))
    truth_s = time.time() - t0
    log(f"FP64 exact answers of {len(sample)} sample queries: {truth_s:.1f}s on {ncpu} threads")
    X64 = W.base.astype(np.float64)
    out = {"sample": f"{len(sample)} of the {nq} queries, every {nq // len(sample)}-th in order of range size "
                     f"(Y from {int(Ysize[sample].min())} to {int(Ysize[sample].max())})",
           "truth_s": round(truth_s, 1), "threads": ncpu}
    agree = 0
    for j, i in enumerate(sample):
        t = truth_gpu[i][truth_gpu[i] >= 0]
        agree += int(np.array_equal(t, res[j][0]))
    out["gpu_exact_scan_equals_fp64"] = round(agree / len(sample), 4)
    for name, (ids, dist) in rows.items():
        rec, errs = [], []
        for j, i in enumerate(sample):
            tid, _, size = res[j]
            rec.append(exact.recall(ids[i], tid, k, size))
            got = ids[i] >= 0
            if got.any():
                e = ids[i][got]
                d64 = ((X64[e] - W.queries[i].astype(np.float64)) ** 2).sum(1)
                nz = d64 > 0
                errs.append(np.abs(dist[i][got][nz].astype(np.float64) - d64[nz]) / d64[nz])
        errs = np.concatenate(errs) if errs else np.zeros(1)
        out[name] = {"recall@10": round(float(np.mean(rec)), 4), "dist_rel_err_max": float(errs.max()),
                     "dist_rel_err_mean": float(errs.mean())}
        log(f"FP64 check {name}: recall@10 {np.mean(rec):.4f}, distance error max {errs.max():.2e} "
            f"mean {errs.mean():.2e}")
    return out


def wide_bench(args):
    """GIST-like shape (d = 960, 512-centre mixture, S = 8, M = 16) at n = --wide-n:
    FP32 vs BF16 vs FP8 stores, each tuned for recall@10 >= 0.95 on held-out queries."""
    import numpy as np
    import torch

    import paper_2412_02448_amd as u
    from paper_2412_02448_amd import autotune
    from synth import workloads as w
    over = {}
    if args.wide_M:
        over["M"] = args.wide_M
    if args.wide_efc:
        over["ef_cons"] = args.wide_efc
    spec = w.scaled(w.SPECS["gist1m"], n=args.wide_n, **over)
    dev = torch.device("cuda", 0)
    t0 = time.time()
    W = w.make(spec, base_seed=0)
    index = u.Index.build(W.base, W.attr, W.level_u, spec.S, spec.M, spec.ef_cons, device=0)
    build_s = time.time() - t0
    Q = torch.from_numpy(W.queries).to(dev)
    L = torch.from_numpy(W.l).to(dev)
    H = torch.from_numpy(W.h).to(dev)
    nq, k, d = Q.shape[0], spec.k, spec.d
    truth = index.search(Q, L, H, k, k, strategy=u.PRE)[0].cpu().numpy()
    cq, cl, ch, _ = w.more_queries(spec, W.attr, 1000, base_seed=0, stream=1)
    Qc, Lc, Hc = (torch.from_numpy(a).to(dev) for a in (cq, cl, ch))
    out = {"workload": f"gist-like: n={spec.n} d={d} (512-centre mixture, sigma 0.2), attribute uniform in "
                       f"[0, 2^31), HSIG S={spec.S} M={spec.M} efCons={spec.ef_cons} built on GPU ({build_s:.0f}s); {nq} queries, "
                       f"range fraction log-uniform [1e-3, 1], k={k}"}
    for prec in ("fp32", "bf16", "fp8"):
        index.set_precision(prec)
        best, table = autotune.tune(index, Qc, Lc, Hc, k, args.recall_target, efs=(32, 64, 128, 256),
                                    ms=(index.M, (3 * index.M) // 2, 2 * index.M, 3 * index.M, 4 * index.M))
        if best is None:
            best = max(table, key=lambda s: s.recall)
        m, ef, bp, ta, tb, vc = best.m, best.ef, best.beam_p, best.tau_a, best.tau_b, best.visit_cap
        for _ in range(2):
            index.search(Q, L, H, k, ef, m=m, beam_p=bp, tau_a=ta, tau_b=tb, visit_cap=vc)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(5):
            o = index.search(Q, L, H, k, ef, m=m, beam_p=bp, tau_a=ta, tau_b=tb, visit_cap=vc)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t) / 5
        ph, _, (_, _, _, st) = timed_calls(index, Q, L, H, k, ef, reps=5, m=m, beam_p=bp, tau_a=ta, tau_b=tb,
                                           visit_cap=vc)
        search_ms = ph["search"]
        st = st.cpu().numpy().astype(np.int64)
        b = int(bytes_per_query(st, d, k, prec)[(st[:, 3] & 0xFF) == 0].sum())
        ids = o[0].cpu().numpy()
        rec = float(np.mean([len(set(ids[i][ids[i] >= 0]) & set(truth[i][truth[i] >= 0]))
                             / max(1, (truth[i] >= 0).sum()) if (truth[i] >= 0).any() else 1.0
                             for i in range(nq)]))
        out[prec] = {"qps": round(nq / sec, 1), "recall@10": round(rec, 4), "m": m, "ef": ef, "beam_p": bp,
                     "tau_a": ta, "tau_b": tb, "visit_cap": vc, "visit_cap": vc,
                     "search_launch_ms": round(search_ms, 4), "bytes_per_launch": b,
                     "achieved_GBps": round(b / (search_ms * 1e-3) / 1e9, 1),
                     "fp32_rescores_per_query": round(float(st[:, 2].mean()), 2)}
        log(f"wide960 {prec}: {nq / sec:,.0f} QPS, recall {rec:.4f} (m={m} ef={ef} p={bp}), "
            f"{out[prec]['achieved_GBps']} GB/s algorithmic")
    index.close()
    return out


def multi_bench(args, index, spec, W, Q, L, H, k, m, ef, bp, ta, tb, vc, prec):
    """Two-attribute queries on the mixed1m objects: the benchmark queries with a second
    range (fraction log-uniform in [0.05, 1]) on an independent uniform second attribute.
    Conjunctive (AND) on the mixed1m index, recall against the exact conjunctive answer
    (the pre-filter scan with both ranges); disjunctive (OR) with a second index built on
    the second attribute, recall against the merge of the two exact answers; the same
    conjunctive boxes on one index over the z-order key of both attributes."""
    import numpy as np
    import torch

    import paper_2412_02448_amd as u
    from synth import workloads as w
    dev = torch.device("cuda", 0)
    nq = Q.shape[0]
    a2, l2, h2 = w.second_attribute(spec.n, nq, base_seed=0)
    index.set_attr2(a2)
    L2 = torch.from_numpy(l2).to(dev)
    H2 = torch.from_numpy(h2).to(dev)
    truth = index.search(Q, L, H, k, k, strategy=u.PRE, l2=L2, h2=H2)[0].cpu().numpy()
    truth_and = truth
    out = {"workload": f"mixed1m index ({prec} store), the {nq} benchmark queries plus a second range "
                       f"(fraction log-uniform in [0.05, 1]) on an independent uniform attribute; k={k}"}
    for name, sv, e in (("auto", None, ef), ("auto_ef64", None, 64), ("hybrid", u.HYBRID, ef)):
        for _ in range(2):
            o = index.search(Q, L, H, k, e, strategy=sv, m=m, beam_p=bp, tau_a=ta, tau_b=tb, visit_cap=vc,
                             l2=L2, h2=H2)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(5):
            o = index.search(Q, L, H, k, e, strategy=sv, m=m, beam_p=bp, tau_a=ta, tau_b=tb, visit_cap=vc,
                             l2=L2, h2=H2)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t) / 5
        ids = o[0].cpu().numpy()
        rec = float(np.mean([len(set(ids[i][ids[i] >= 0]) & set(truth[i][truth[i] >= 0]))
                             / max(1, (truth[i] >= 0).sum()) if (truth[i] >= 0).any() else 1.0
                             for i in range(nq)]))
        out[name] = {"ef": e, "qps": round(nq / sec, 1), "recall@10": round(rec, 4)}
        log(f"conjunctive {name} (ef={e}): {nq / sec:,.0f} QPS, recall {rec:.4f}")
    # disjunctive: a second index over the same objects on the second attribute, each
    # searched with its own range, results merged per query
    t0 = time.time()
    other = u.Index.build(W.base, a2, W.level_u, spec.S, spec.M, spec.ef_cons, device=0,
                          precision=prec)
    build2 = time.time() - t0
    try:
        ta_ = index.search(Q, L, H, k, k, strategy=u.PRE)
        tb_ = other.search(Q, L2, H2, k, k, strategy=u.PRE)
        truth = u.merge_or(ta_[:2], tb_[:2])[0].cpu().numpy()

        def both(e):
            ra = index.search(Q, L, H, k, e, m=m, beam_p=bp, tau_a=ta, tau_b=tb, visit_cap=vc)
            rb = other.search(Q, L2, H2, k, e, m=m, beam_p=bp, tau_a=ta, tau_b=tb, visit_cap=vc)
            return u.merge_or(ra[:2], rb[:2])
        for name, e in (("disjunctive", ef), ("disjunctive_ef64", 64)):
            for _ in range(2):
                o = both(e)
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(5):
                o = both(e)
            torch.cuda.synchronize()
            sec = (time.perf_counter() - t) / 5
            ids = o[0].cpu().numpy()
            rec = float(np.mean([len(set(ids[i][ids[i] >= 0]) & set(truth[i][truth[i] >= 0]))
                                 / max(1, (truth[i] >= 0).sum()) if (truth[i] >= 0).any() else 1.0
                                 for i in range(nq)]))
            out[name] = {"ef": e, "qps": round(nq / sec, 1), "recall@10": round(rec, 4),
                         "second_index_build_s": round(build2, 1)}
            log(f"disjunctive (two indexes, merged; ef={e}): {nq / sec:,.0f} QPS, recall {rec:.4f}")
    finally:
        other.close()
    # approach 2: one index over the z-order key of (attribute, second attribute), searched
    # with the same boxes; recall against the exact conjunctive answer above
    zmap = u.zorder_map(W.attr, a2)
    t0 = time.time()
    zix = u.Index.build(W.base, u.zorder_keys(zmap, W.attr, a2), W.level_u, spec.S, spec.M, spec.ef_cons,
                        device=0, precision=prec)
    build3 = time.time() - t0
    try:
        zix.set_zorder(zmap, W.attr, a2)
        for name, e in (("zorder", ef), ("zorder_ef64", 64)):
            for _ in range(2):
                o = zix.search(Q, L, H, k, e, m=m, beam_p=bp, tau_a=ta, tau_b=tb, visit_cap=vc, l2=L2, h2=H2,
                               box=True)
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(5):
                o = zix.search(Q, L, H, k, e, m=m, beam_p=bp, tau_a=ta, tau_b=tb, visit_cap=vc, l2=L2, h2=H2,
                               box=True)
            torch.cuda.synchronize()
            sec = (time.perf_counter() - t) / 5
            ids = o[0].cpu().numpy()
            sr = o[2].cpu().numpy()
            rec = float(np.mean([len(set(ids[i][ids[i] >= 0]) & set(truth_and[i][truth_and[i] >= 0]))
                                 / max(1, (truth_and[i] >= 0).sum()) if (truth_and[i] >= 0).any() else 1.0
                                 for i in range(nq)]))
            mix = {nm: int((sr == v).sum()) for nm, v in (("pre", u.PRE), ("hybrid", u.HYBRID), ("post", u.POST))}
            out[name] = {"ef": e, "qps": round(nq / sec, 1), "recall@10": round(rec, 4), "strategies": mix,
                         "zorder_index_build_s": round(build3, 1)}
            log(f"z-order composite (one index, box search; ef={e}): {nq / sec:,.0f} QPS, recall {rec:.4f}, "
                f"strategies {mix}")
    finally:
        zix.close()
    return out


def insert_bench(args, spec, W, Q, L, H, k, m, ef, bp, ta, tb, vc, prec, build_s, rec_single, qps_single):
    """The insertion experiment's shape on the mixed1m objects: an index of the first
    200k, then four insertions of 200k each.  Per round: insertion time, then QPS and
    recall@10 (against the exact answer over the objects present) at the headline
    setting.  After the last insertion the index holds the same 1M objects as the single build."""
    import numpy as np
    import torch

    import paper_2412_02448_amd as u
    n = spec.n
    step = n // 5
    nq = Q.shape[0]
    t0 = time.perf_counter()
    g = u.Index.build(W.base[:step], W.attr[:step], W.level_u[:step], spec.S, spec.M, spec.ef_cons, device=0)
    first_s = time.perf_counter() - t0
    rounds = []
    try:
        for r in range(5):
            if r > 0:
                a, b = r * step, (r + 1) * step if r < 4 else n
                t0 = time.perf_counter()
                g.insert(W.base[a:b], W.attr[a:b], W.level_u[a:b])
                ins_s = time.perf_counter() - t0
            else:
                ins_s = None
            g.set_precision(prec)
            truth = g.search(Q, L, H, k, k, strategy=u.PRE)[0].cpu().numpy()
            for _ in range(2):
                o = g.search(Q, L, H, k, ef, m=m, beam_p=bp, tau_a=ta, tau_b=tb, visit_cap=vc)
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(5):
                o = g.search(Q, L, H, k, ef, m=m, beam_p=bp, tau_a=ta, tau_b=tb, visit_cap=vc)
            torch.cuda.synchronize()
            sec = (time.perf_counter() - t) / 5
            ids = o[0].cpu().numpy()
            rec = float(np.mean([len(set(ids[i][ids[i] >= 0]) & set(truth[i][truth[i] >= 0]))
                                 / max(1, (truth[i] >= 0).sum()) if (truth[i] >= 0).any() else 1.0
                                 for i in range(nq)]))
            row = {"n": int(g.n), "insert_s": None if ins_s is None else round(ins_s, 2),
                   "qps": round(nq / sec, 1), "recall@10": round(rec, 4)}
            rounds.append(row)
            log(f"insertion round {r}: n={g.n}, insert {row['insert_s']} s, {nq / sec:,.0f} QPS, recall {rec:.4f}")
    finally:
        g.close()
    return {"workload": f"mixed1m objects in ext-id order: GPU build of the first {step} ({first_s:.1f} s), then "
                        f"four insertions of {step}; {prec} store at the headline setting (m={m} ef={ef} p={bp} "
                        f"tau=({ta}, {tb})), {nq} queries",
            "rounds": rounds,
            "single_build": {"n": n, "build_s": round(build_s, 1), "qps": round(qps_single, 1),
                             "recall@10": round(rec_single, 4)}}


def serve_bench(args, index, spec, W, m, ef, bp, ta, tb, vc, prec):
    """Poisson arrivals at several rates into the server over the mixed1m index, with
    the serving range mix (30% of fractions log-uniform in [1e-5, 1e-3), 40% in
    [1e-3, 0.1), 30% in [0.1, 1]); latency = completion - arrival per request."""
    import dataclasses

    import numpy as np
    import torch

    import paper_2412_02448_amd as u
    from synth import workloads as w
    sspec = dataclasses.replace(spec, ranges="serving")
    k = spec.k
    n = 40000
    q, l, h, _ = w.more_queries(sspec, W.attr, n, base_seed=0, stream=5)
    # the same requests searched as one batch: each served result must equal its row
    dev = torch.device("cuda", 0)
    ref = index.search(torch.from_numpy(q).to(dev), torch.from_numpy(l).to(dev), torch.from_numpy(h).to(dev), k,
                       ef, m=m, beam_p=bp, tau_a=ta, tau_b=tb, visit_cap=vc)[0].cpu().numpy()
    rng = np.random.default_rng(12)
    rows = []
    limits = None
    for rate in (10_000, 100_000, 1_000_000, None):
        cnt = n if rate is None or rate >= 100_000 else 20_000
        arrive = np.zeros(cnt) if rate is None else np.cumsum(rng.exponential(1.0 / rate, cnt))
        srv = u.Server(index, k, ef, max_batch=4096, inflight=args.inflight, m=m, beam_p=bp, tau_a=ta, tau_b=tb,
                       visit_cap=vc)
        b_, r_, m_ = srv.limits()
        limits = {"max_batch": b_, "visit_rows_per_slot": r_, "device_MB": round(m_ / 2 ** 20, 1)}
        t0 = time.perf_counter()
        tickets = srv.submit(q[:cnt], l[:cnt], h[:cnt], arrive_s=arrive)
        ids, _, lat = srv.wait(tickets, timeout_s=120)
        wall = time.perf_counter() - t0
        done, batches, busy = srv.stats()
        srv.close()
        span = max(wall, 1e-9)
        row = {"offered_qps": rate if rate else "all at t=0", "requests": cnt, "achieved_qps": round(cnt / span, 1),
               "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
               "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3), "batches": batches,
               # requests after the first tenth of arrivals (the server's start-up excluded)
               "p99_ms_after_first_10pct": round(float(np.percentile(lat[cnt // 10:], 99)) * 1e3, 3),
               "max_ms": round(float(lat.max()) * 1e3, 3),
               "mean_batch": round(cnt / max(batches, 1), 1),
               "equal_to_batch_search": bool(np.array_equal(ids, ref[:cnt]))}
        rows.append(row)
        log(f"serving {row['offered_qps']}: {row['achieved_qps']:,.0f} QPS, p50 {row['p50_ms']} ms, "
            f"p99 {row['p99_ms']} ms, {batches} batches, identical {row['equal_to_batch_search']}")
    # k = 100 (the other result size of the serving workload), ef = 128
    k2, ef2, cnt = 100, 128, 20_000
    ref2 = index.search(torch.from_numpy(q[:cnt]).to(dev), torch.from_numpy(l[:cnt]).to(dev),
                        torch.from_numpy(h[:cnt]).to(dev), k2, ef2, m=m, beam_p=bp, tau_a=ta, tau_b=tb,
                        visit_cap=vc)[0].cpu().numpy()
    k100 = []
    for rate in (10_000, 100_000):
        arrive = np.cumsum(rng.exponential(1.0 / rate, cnt))
        srv = u.Server(index, k2, ef2, max_batch=4096, inflight=args.inflight, m=m, beam_p=bp, tau_a=ta, tau_b=tb,
                       visit_cap=vc)
        t0 = time.perf_counter()
        ids, _, lat = srv.wait(srv.submit(q[:cnt], l[:cnt], h[:cnt], arrive_s=arrive), timeout_s=120)
        wall = time.perf_counter() - t0
        _, batches, _ = srv.stats()
        srv.close()
        row = {"k": k2, "ef": ef2, "offered_qps": rate, "requests": cnt, "achieved_qps": round(cnt / wall, 1),
               "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
               "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3), "batches": batches,
               "equal_to_batch_search": bool(np.array_equal(ids, ref2))}
        k100.append(row)
        log(f"serving k=100 at {rate}/s: {row['achieved_qps']:,.0f} QPS, p50 {row['p50_ms']} ms, "
            f"p99 {row['p99_ms']} ms, identical {row['equal_to_batch_search']}")
    return {"workload": f"mixed1m index ({prec} store, m={m} ef={ef} p={bp} tau=({ta}, {tb})), k={k}, "
                        f"serving range mix",
            "max_batch": 4096, "inflight": args.inflight, "admitted": limits, "rates": rows, "k100": k100}


def c1_bench(args):
    """The plain FP32 hybrid search of the small configuration: 10,000 x 128 vectors
    (16-centre mixture, sigma 0.3), attribute a permutation, HSIG S = 8, M = 16, efCons =
    100 built on the GPU, FP32 store; 200 queries with in-range fractions in {0.01, 0.1,
    0.5} (random placement), k = 10, ef = 64, every query forced to the hybrid search."""
    import numpy as np
    import torch

    import paper_2412_02448_amd as u
    from paper_2412_02448_amd import autotune
    from synth import workloads as w
    spec = w.SPECS["hybrid10k"]
    dev = torch.device("cuda", 0)
    W = w.make(spec, base_seed=0)
    index = u.Index.build(W.base, W.attr, W.level_u, spec.S, spec.M, spec.ef_cons, device=0, precision="fp32")
    Q, L, H = (torch.from_numpy(a).to(dev) for a in (W.queries, W.l, W.h))
    truth = autotune.exact_answers(index, Q, L, H, spec.k)
    out = {"workload": "hybrid10k: n=10000 d=128 (16-centre mixture, sigma 0.3), permutation attribute, HSIG S=8 "
                       "M=16 efCons=100 built on GPU, FP32 store; 200 queries, fractions {0.01, 0.1, 0.5}, k=10, "
                       "ef=64; p1, p4: hybrid forced with beam width 1, 4; auto_p4: the range-aware rule"}
    for name, strat, p in (("p1", u.HYBRID, 1), ("p4", u.HYBRID, 4), ("auto_p4", None, 4)):
        kw = dict(strategy=strat, m=0, beam_p=p)
        for _ in range(3):
            index.search(Q, L, H, spec.k, 64, **kw)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(50):
            o = index.search(Q, L, H, spec.k, 64, **kw)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t) / 50
        rec = autotune.recall_at_k(o[0].cpu().numpy(), truth)
        out[name] = {"qps": round(len(W.queries) / sec, 1), "ms_per_batch": round(sec * 1e3, 4),
                     "recall@10": round(rec, 4)}
        log(f"c1 FP32 ef=64 {name} ({'hybrid forced' if strat else 'auto strategy'}): {len(W.queries) / sec:,.0f} "
            f"QPS ({sec * 1e3:.3f} ms per 200), recall {rec:.4f}")
    index.close()
    return out


def c5_bench(args):
    """The serving configuration at full size: 10,000,000 x 96 vectors (4096-centre
    mixture, sigma 0.2), attribute uniform in [0, 2^31), HSIG with S = 64 and M = 24
    (efCons = 100) built on the GPU, BF16 store.  (m, ef, p) tuned for recall@10 >= 0.95
    on 2,000 held-out queries of the serving range mix; then Poisson arrivals at 5k-100k
    requests/s for k = 10 and k = 100 (ef = 128); every served row equals the batch
    search's; recall against the exact answer (the FP32 pre-filter scan)."""
    import numpy as np
    import torch

    import paper_2412_02448_amd as u
    from paper_2412_02448_amd import autotune
    from synth import workloads as w
    spec = w.SPECS["serve10m"]
    if args.n:
        spec = w.scaled(spec, n=args.n)
    dev = torch.device("cuda", 0)
    t0 = time.time()
    W = w.make(spec, base_seed=0)
    log(f"c5 workload n={spec.n} d={spec.d}: {time.time() - t0:.1f}s")
    free0 = torch.cuda.mem_get_info(dev)[0]
    t0 = time.time()
    index = u.Index.build(W.base, W.attr, W.level_u, spec.S, spec.M, spec.ef_cons, device=0, precision="bf16")
    build_s = time.time() - t0
    index_gb = (free0 - torch.cuda.mem_get_info(dev)[0]) / 1e9
    log(f"c5 GPU build: {build_s:.1f}s, {index.levels} layers, {index_gb:.1f} GB resident (tables, stores, "
        f"visited rows)")
    k = spec.k
    cq, cl, ch, _ = w.more_queries(spec, W.attr, 2000, base_seed=0, stream=1)
    Qc, Lc, Hc = (torch.from_numpy(a).to(dev) for a in (cq, cl, ch))
    best, table = autotune.tune(index, Qc, Lc, Hc, k, args.recall_target + TUNE_MARGIN, ms=(24, 48, 72),
                                efs=(16, 32, 64, 128), ps=(2, 4, 6), taus=((0.01, 0.5),), visit_caps=(),
                                log=lambda s: log(f"[c5] {s}"))
    if best is None:
        best = max(table, key=lambda s: s.recall)
    m, ef, bp = best.m, best.ef, best.beam_p
    n_eval = 5000
    q, l, h = W.queries[:n_eval], W.l[:n_eval], W.h[:n_eval]
    Q, L, H = (torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (q, l, h))
    truth = autotune.exact_answers(index, Q, L, H, k)
    ids, _, strat = index.search(Q, L, H, k, ef, m=m, beam_p=bp)
    torch.cuda.synchronize()
    rec = autotune.recall_at_k(ids.cpu().numpy(), truth)
    mix = np.bincount(strat.cpu().numpy().astype(np.int64) + 1, minlength=5)
    log(f"c5 m={m} ef={ef} p={bp}: recall@10 {rec:.4f} on {n_eval} queries")
    rng = np.random.default_rng(17)
    rows = []
    for kk, e2, rates in ((k, ef, (5_000, 10_000, 20_000, 50_000, 100_000)), (100, 128, (5_000, 20_000, 100_000))):
        ref = index.search(Q, L, H, kk, e2, m=m, beam_p=bp)[0].cpu().numpy()
        for rate in rates:
            cnt = min(n_eval, max(2000, int(rate * 0.5)))
            arrive = np.cumsum(rng.exponential(1.0 / rate, cnt))
            srv = u.Server(index, kk, e2, max_batch=4096, inflight=args.inflight, m=m, beam_p=bp,
                           visit_cap=args.visit_cap)
            batch_cap, vrows, dev_b = srv.limits()
            t1 = time.perf_counter()
            got, _, lat = srv.wait(srv.submit(q[:cnt], l[:cnt], h[:cnt], arrive_s=arrive), timeout_s=300)
            wall = time.perf_counter() - t1
            _, batches, _ = srv.stats()
            srv.close()
            row = {"k": kk, "ef": e2, "offered_qps": rate, "requests": cnt, "achieved_qps": round(cnt / wall, 1),
                   "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
                   "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3), "batches": batches,
                   "equal_to_batch_search": bool(np.array_equal(got, ref[:cnt])),
                   "slot_device_MB": round(dev_b / 2 ** 20, 1), "visit_rows_per_slot": vrows}
            rows.append(row)
            log(f"c5 serving k={kk} at {rate}/s: {row['achieved_qps']:,.0f} QPS, p50 {row['p50_ms']} ms, "
                f"p99 {row['p99_ms']} ms, identical {row['equal_to_batch_search']}")
    index.close()
    return {"workload": f"serve10m: n={spec.n} d={spec.d} (4096-centre mixture, sigma 0.2), attribute uniform in "
                        f"[0, 2^31), HSIG S={spec.S} M={spec.M} efCons={spec.ef_cons} built on GPU, BF16 store; "
                        f"serving range mix (30% of fractions in [1e-5, 1e-3), 40% in [1e-3, 0.1), 30% in [0.1, 1])",
            "build_s": round(build_s, 1), "resident_GB": round(index_gb, 1), "m": m, "ef": ef, "beam_p": bp,
            "recall@10": round(rec, 4), "eval_queries": n_eval,
            "strategy_mix": {"pre": int(mix[2]), "hybrid": int(mix[3]), "post": int(mix[4])},
            "inflight": args.inflight, "rates": rows}


def batch100k(args, prec):
    """100,000 queries (range fraction log-uniform in [1e-4, 1]) on the 10k x 128 index
    (S = 8, M = 16): one graph-captured replay per step vs the same batch through
    unify_search and vs one launch sequence per query."""
    import numpy as np
    import torch

    import paper_2412_02448_amd as u
    from paper_2412_02448_amd import autotune
    from synth import workloads as w
    spec = w.SPECS["batch100k"]
    dev = torch.device("cuda", 0)
    W = w.make(spec, base_seed=0)
    index = u.Index.build(W.base, W.attr, W.level_u, spec.S, spec.M, spec.ef_cons, device=0, precision=prec)
    Q = torch.from_numpy(W.queries).to(dev)
    L = torch.from_numpy(W.l).to(dev)
    H = torch.from_numpy(W.h).to(dev)
    nq, k = Q.shape[0], spec.k
    cq, cl, ch, _ = w.more_queries(spec, W.attr, 2000, base_seed=0, stream=1)
    best, table = autotune.tune(index, torch.from_numpy(cq).to(dev), torch.from_numpy(cl).to(dev),
                                torch.from_numpy(ch).to(dev), k, args.recall_target, efs=(16, 32, 64, 128),
                                wave_scans=(True,), wpqs=(2, 4))
    if best is None:
        best = max(table, key=lambda s: s.recall)
    m, ef, bp, ta, tb, vc = best.m, best.ef, best.beam_p, best.tau_a, best.tau_b, best.visit_cap
    kw = best.kwargs()
    truth = index.search(Q, L, H, k, k, strategy=u.PRE)[0].cpu().numpy()
    b = u.Batch(index, Q, L, H, k, ef, **kw)
    steps = max(args.steps, 5)
    for _ in range(2):
        b.run()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        b.run()
    torch.cuda.synchronize()
    g_s = (time.perf_counter() - t) / steps
    ids = b.ids.cpu().numpy()
    rec = float(np.mean([len(set(ids[i][ids[i] >= 0]) & set(truth[i][truth[i] >= 0])) / max(1, (truth[i] >= 0).sum())
                         if (truth[i] >= 0).any() else 1.0 for i in range(nq)]))
    eager = index.search(Q, L, H, k, ef, **kw)
    same = bool((eager[0] == b.ids).all().item())
    for _ in range(2):
        index.search(Q, L, H, k, ef, **kw)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        index.search(Q, L, H, k, ef, **kw)
    torch.cuda.synchronize()
    e_s = (time.perf_counter() - t) / steps
    # one launch sequence per query (the first 2,000 queries)
    npq = 2000
    views = [(Q[i:i + 1], L[i:i + 1], H[i:i + 1]) for i in range(npq)]
    for i in range(50):
        index.search(*views[i], k, ef, **kw)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for v in views:
        index.search(*v, k, ef, **kw)
    torch.cuda.synchronize()
    pq_s = time.perf_counter() - t
    b.close()
    out = {"workload": f"batch100k: n={spec.n} d={spec.d} (16-centre mixture, sigma 0.3), permutation attribute, "
                       f"HSIG S={spec.S} M={spec.M} built on GPU; {nq} queries, range fraction log-uniform "
                       f"[1e-4, 1], k={k}, auto strategy, {prec} store",
           "m": m, "ef": ef, "beam_p": bp, "tau_a": ta, "tau_b": tb, "visit_cap": vc,
           "wave_scan": best.wave_scan, "waves_per_query": best.waves_per_query or 1, "recall@10": round(rec, 4),
           "graph_qps": round(nq / g_s, 1), "graph_ms_per_step": round(g_s * 1e3, 4),
           "eager_qps": round(nq / e_s, 1), "per_query_launch_qps": round(npq / pq_s, 1),
           "graph_equals_eager": same, "per_query_sample": npq}
    log(f"batch100k ({prec}, m={m} ef={ef} p={bp}, recall {rec:.4f}): graph {nq / g_s:,.0f} QPS, "
        f"eager {nq / e_s:,.0f} QPS, one launch per query {npq / pq_s:,.0f} QPS")
    index.close()
    return out


def cpu_baseline(args, W, index, ids, k, ef, m, bp, ta, tb, nq, prec):
    """The oracle's HSIG search (plain C++, one query per thread) on the same index file and store."""
    import numpy as np
    from oracle import hsig
    with tempfile.TemporaryDirectory(dir="/tmp") as td:
        path = os.path.join(td, "bench.uix")
        t0 = time.time()
        index.save(path)
        ref = hsig.Index.read(path)
        log(f"index file written and read by the oracle ({time.time() - t0:.1f}s)")
    if prec != "fp32":
        t0 = time.time()
        ref.set_store({"bf16": hsig.BF16, "fp8": hsig.FP8E4M3}[prec], 4)
        log(f"oracle {prec} copy ({time.time() - t0:.1f}s)")
    naff = len(os.sched_getaffinity(0))
    ncpu = min(HOST_SHARE, naff)  # this GPU's share of the host's cores
    sample = np.arange(min(args.cpu_queries, nq)) if args.cpu_queries else np.arange(nq)
    parts = np.array_split(sample, ncpu)
    res = [None] * ncpu

    def work(i):
        p = parts[i]
        res[i] = ref.search(W.queries[p], W.l[p], W.h[p], k, ef, m=m, p=bp, tau_a=ta, tau_b=tb)[0]

    # whole passes over the sample until about 10 s of work (at most 30 passes)
    passes, cpu_s = 0, 0.0
    while passes < 30 and cpu_s < 10.0:
        t0 = time.perf_counter()
        th = [threading.Thread(target=work, args=(i,)) for i in range(ncpu)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        cpu_s += time.perf_counter() - t0
        passes += 1
        if passes == 1:
            cpu_ids = np.concatenate(res)
            agree = float(np.mean([np.array_equal(cpu_ids[i], ids[i]) for i in range(len(sample))]))
    # one thread over a fixed 2,000-query slice of the same batch (the strategy mix of the whole)
    one = sample[:: max(1, len(sample) // 2000)]
    t0 = time.perf_counter()
    ref.search(W.queries[one], W.l[one], W.h[one], k, ef, m=m, p=bp, tau_a=ta, tau_b=tb)
    one_s = time.perf_counter() - t0
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    cpu = {"value": round(passes * len(sample) / cpu_s, 1), "unit": "queries/s", "cores": ncpu, "kind": "oracle",
           "sample": f"{passes} passes over {len(sample)} of the {nq} queries ({cpu_s:.1f} s) on {ncpu} threads "
                     f"(the GPU's share of the host; the affinity mask holds {naff} cores), auto strategy, {prec} "
                     f"store, ef={ef}, m={m}, p={bp}, tau=({ta}, {tb}), same index; {agree:.4f} of them return the "
                     f"GPU's ids",
           "affinity_cores": naff,
           "cpu_model": model, "single_thread_qps": round(len(one) / one_s, 1),
           "single_thread_sample": f"every {max(1, len(sample) // 2000)}-th query, {len(one)} queries"}
    log(f"CPU oracle: {cpu['value']:,.0f} QPS on {ncpu} threads ({cpu_s:.1f}s), id agreement {agree:.4f}; "
        f"1 thread {cpu['single_thread_qps']:,.0f} QPS; {model}")
    return cpu


def timed_calls(index, Q, L, H, k, ef, reps=TIMED_REPS, **kw):
    """reps searches with HIP-event timing, each synchronised before the next: the mean of
    every phase (ms), its min and max for the graph-search phase, and the last call's
    outputs (ids, dist, strategy, stats)."""
    import torch
    acc, lo, hi, out = {}, float("inf"), 0.0, None
    for _ in range(reps):
        out = index.search(Q, L, H, k, ef, stats=True, timing=True, **kw)
        torch.cuda.synchronize()
        ph = index.last_timing_phases()
        for kk, v in ph.items():
            acc[kk] = acc.get(kk, 0.0) + v
        lo, hi = min(lo, ph["search"]), max(hi, ph["search"])
    mean = {kk: v / reps for kk, v in acc.items()}
    return mean, (lo, hi), out


def source_hash():
    src = b"".join(open(os.path.join(ROOT, "paper_2412_02448_amd", "csrc", x), "rb").read()
                   for x in ("search.hip", "wave.h", "lowp.h", "unify_internal.h", "zorder.h"))
    return hashlib.sha256(src).hexdigest()


def profiled_traffic(prec, m, ef, bp, ta, tb, vc, wave_scan=False, wpq=1):
    """HBM bytes per launch of the search kernel from the committed rocprofv3 counter summary,
    or None when the kernel sources or the setting differ from what was profiled."""
    import glob
    want = f"--m {m} --ef {ef} --p {bp} --tau-a {ta} --tau-b {tb} --visit-cap {vc} "
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", f"k_search_mixed1m_{prec}*.json"))):
        prof = json.load(open(path))
        if (source_hash() == prof["source_sha256"] and want in prof["args"] + " "
                and bool(prof.get("wave_scan", False)) == bool(wave_scan)
                and int(prof.get("waves_per_query", 1)) == int(wpq or 1)):
            return int(prof["traffic_bytes"])
    return None


def profile_run(args, index, Q, L, H, k, spec, nq, build_s, prec):
    """Timed steps at a fixed setting plus one counted call: the search kernel's
    launches all share one configuration, so a profiler's average matches."""
    import numpy as np
    import torch
    index.set_precision(prec)
    m, ef, bp = args.m, args.ef, args.p
    ta, tb = (args.tau_a, args.tau_b) if args.tau_a else (0.01, 0.5)
    vc = args.visit_cap
    xk = dict(wave_scan=args.wave_scan, waves_per_query=args.wpq, heavy_queries=args.heavy)
    for _ in range(args.warmup):
        index.search(Q, L, H, k, ef, m=m, beam_p=bp, tau_a=ta, tau_b=tb, visit_cap=vc, **xk)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        index.search(Q, L, H, k, ef, m=m, beam_p=bp, tau_a=ta, tau_b=tb, visit_cap=vc, **xk)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t) / args.steps
    ph, (smin, smax), (ids, dist, strat, stats) = timed_calls(index, Q, L, H, k, ef, m=m, beam_p=bp, tau_a=ta,
                                                              tau_b=tb, visit_cap=vc, **xk)
    search_ms, rerun_ms = ph["search"], ph["rerun"]
    st = stats.cpu().numpy().astype(np.int64)
    b = int(bytes_per_query(st, spec.d, k, prec)[((st[:, 3] & 0xFF) == 0) & ~tile_rows(st)].sum())
    print(json.dumps({"profile_run": True, "store": prec, "m": m, "ef": ef, "beam_p": bp, "tau_a": ta, "tau_b": tb,
                      "visit_cap": vc, "wave_scan": args.wave_scan, "waves_per_query": args.wpq or 1,
                      "qps": round(nq / sec, 1), "phases_ms": {kk: round(v, 4) for kk, v in ph.items()},
                      "tile_scan": tile_roofline(st, ph, spec.d, k, prec, spec.n),
                      "ms_per_step": round(sec * 1e3, 4), "search_launch_ms": round(search_ms, 4),
                      "search_launch_ms_min_max": [round(smin, 4), round(smax, 4)], "timed_calls": TIMED_REPS,
                      "rerun_launch_ms": round(rerun_ms, 4), "bytes_per_launch": b,
                      "achieved_GBps": round(b / (search_ms * 1e-3) / 1e9, 1), "build_s": round(build_s, 1),
                      "source_sha256": source_hash()}),
          flush=True)


if __name__ == "__main__":
    main()
