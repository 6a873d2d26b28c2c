"""Benchmark: range-filtered k-NN search over HSIG on one MI355X.

Workload (synthetic, seeded): 1,000,000 x 128 FP32 vectors from a 1024-centre
Gaussian mixture (sigma 0.2), attribute uniform in [0, 2^31), HSIG with 32
segments and M = 32 (built on the GPU), 10,000 queries from the same mixture
with range fraction log-uniform in [1e-3, 1], k = 10.  One step = one search of
the whole 10,000-query batch with the range-aware strategy (plan, pre-filter
scans, hybrid and post-filter searches), inputs already resident in HBM.

ef is the smallest of {32, 64, 128, 256} whose recall@10 against the exact
answer (the pre-filter scan forced on every query) reaches 0.95.  The JSON line
also reports each strategy timed separately, the roofline of the search kernel
(algorithmic bytes from the kernel's own counters / its HIP-event duration),
and the CPU oracle's HSIG search on the same index file as a baseline.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import tempfile
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "QPS @ recall@10≥0.95, 1M×128 mixed ranges, FP32 vs BF16/FP8; HBM GB/s"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--ef", type=int, default=0, help="fixed ef (0: tuned)")
    ap.add_argument("--m", type=int, default=0, help="fixed neighbour budget m (0: tuned)")
    ap.add_argument("--recall-target", type=float, default=0.95)
    ap.add_argument("--n", type=int, default=0, help="override n (smaller runs for development only)")
    ap.add_argument("--p", type=int, default=0, help="fixed beam width (0: tuned)")
    ap.add_argument("--profile-run", action="store_true",
                    help="profiling run: fixed --m/--ef/--p, only the timed steps and one counted call "
                         "(every search-kernel launch has the same configuration)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-queries", type=int, default=2000)
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: every box here has one MI355X; run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2412_02448_amd as u
    from synth import workloads as w

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
    nq, k = Q.shape[0], spec.k
    # A small copy of known size, for scaling HBM counters in a profiling run.
    cp_src = torch.empty(256 << 20, dtype=torch.uint8, device=dev)
    cp_dst = torch.empty_like(cp_src)
    cp_dst.copy_(cp_src)

    if args.profile_run:
        if not (args.m and args.ef and args.p):
            print("--profile-run needs --m, --ef and --p", file=sys.stderr)
            sys.exit(2)
        return profile_run(args, index, Q, L, H, k, spec, nq, build_s)

    # exact answer: the pre-filter scan on every query
    t0 = time.time()
    truth, tdist, _ = index.search(Q, L, H, k, k, strategy=u.PRE)
    torch.cuda.synchronize()
    truth = truth.cpu().numpy()
    log(f"exact answers by forced pre-filter scan ({time.time() - t0:.1f}s)")

    def recall_of(ids):
        ids = ids.cpu().numpy()
        r = []
        for i in range(nq):
            t = truth[i][truth[i] >= 0]
            if t.size == 0:
                r.append(1.0)
                continue
            r.append(len(set(ids[i][ids[i] >= 0].tolist()) & set(t.tolist())) / t.size)
        return float(np.mean(r))

    # search parameters: tuned on held-out sample queries of the same recipe
    from paper_2412_02448_amd import autotune
    cq, cl, ch, _ = w.more_queries(spec, W.attr, 2000, base_seed=0, stream=1)
    Qc = torch.from_numpy(cq).to(dev)
    Lc = torch.from_numpy(cl).to(dev)
    Hc = torch.from_numpy(ch).to(dev)
    t0 = time.time()
    if args.ef:
        ms_grid, efs_grid = ((args.m,) if args.m else None), (args.ef,)
    else:
        ms_grid, efs_grid = ((args.m,) if args.m else None), (32, 64, 128, 256)
    best, table = autotune.tune(index, Qc, Lc, Hc, k, args.recall_target, ms=ms_grid, efs=efs_grid, log=log)
    if best is None:
        best = max(table, key=lambda s: s.recall)
    m, ef, bp = best.m, best.ef, best.beam_p
    log(f"tuned on 2000 held-out queries ({time.time() - t0:.1f}s): m={m} ef={ef} p={bp}")
    recalls = {}
    for e in (32, 64, 128, 256):
        ids, _, _ = index.search(Q, L, H, k, e, m=m, beam_p=bp)
        torch.cuda.synchronize()
        recalls[e] = recall_of(ids)
    rec = recalls[ef]
    log(f"recall@10 on the benchmark queries at m={m}: " + ", ".join(f"ef={e}: {r:.4f}" for e, r in recalls.items()))

    def timed(strategy=None, steps=args.steps, warmup=args.warmup, **kw):
        out = None
        for _ in range(warmup):
            out = index.search(Q, L, H, k, ef, strategy=strategy, m=m, beam_p=bp, **kw)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            out = index.search(Q, L, H, k, ef, strategy=strategy, m=m, beam_p=bp, **kw)
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / steps, out

    # ---- timed region: K steps of the whole path (auto strategy) ----
    sec, out = timed()
    qps = nq / sec
    log(f"auto: {qps:,.0f} QPS ({sec * 1e3:.2f} ms/step), ef={ef}")
    per_strategy = {}
    for name, st in (("pre", u.PRE), ("hybrid", u.HYBRID), ("post", u.POST)):
        s, o = timed(st, steps=max(1, args.steps // 2 + 1), warmup=1)
        per_strategy[name] = {"qps": round(nq / s, 1), "recall@10": round(recall_of(o[0]), 4)}
        log(f"{name}: {nq / s:,.0f} QPS recall {per_strategy[name]['recall@10']}")

    # the same step with narrow pre-filter queries answered by the tile-shared scan
    s, o = timed(steps=max(1, args.steps // 2 + 1), warmup=1, tiled_prescan=True)
    same = bool((o[0] == out[0]).all().item())
    _, _, _, tst = index.search(Q, L, H, k, ef, m=m, beam_p=bp, stats=True, timing=True, tiled_prescan=True)
    torch.cuda.synchronize()
    tpre_ms = index.last_timing()[0]
    ntiled = int((tst[:, 3] == 3).sum().item())
    tiled_alt = {"qps": round(nq / s, 1), "same_ids_as_default": same, "tiled_queries": ntiled,
                 "prescan_ms": round(tpre_ms, 4)}
    log(f"auto with tiled pre-filter scan: {nq / s:,.0f} QPS ({ntiled} tiled queries, "
        f"{tpre_ms:.3f} ms), same ids: {same}")

    # ---- roofline of the search kernel: counters of one more (identical) call ----
    ids, dist, strat, stats = index.search(Q, L, H, k, ef, m=m, beam_p=bp, stats=True, timing=True)
    torch.cuda.synchronize()
    pre_ms, search_ms, rerun_ms = index.last_timing()
    st = stats.cpu().numpy().astype(np.int64)
    d = spec.d
    first = st[:, 3] == 0
    # algorithmic bytes: vectors whose distance is evaluated, adjacency entries read,
    # the query vector and the k (id, distance) outputs of each query
    per_q = st[:, 0] * d * 4 + st[:, 4] * 4 + (st[:, 5] >= 0) * (d * 4 + k * 12)
    bytes_first = int(per_q[first].sum())
    achieved = bytes_first / (search_ms * 1e-3) / 1e9
    mix = np.bincount(np.maximum(st[:, 5], 0), minlength=4)
    roofline = {"bound": "hbm", "kernel": "k_search (first pass)", "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None, "bytes_per_launch": bytes_first, "launch_ms": round(search_ms, 4),
                "rerun_launch_ms": round(rerun_ms, 4), "rerun_queries": int((st[:, 3] == 1).sum()),
                "failed_queries": int((st[:, 3] == 2).sum())}
    roofline["traffic"] = profiled_traffic(m, ef, bp)
    ids_np = ids.cpu().numpy()
    for sname, sv in (("pre", 1), ("hybrid", 2), ("post", 3)):
        sel = np.nonzero(st[:, 5] == sv)[0]
        if sel.size:
            r = [len(set(ids_np[i][ids_np[i] >= 0].tolist()) & set(truth[i][truth[i] >= 0].tolist()))
                 / max(1, int((truth[i] >= 0).sum())) for i in sel]
            per_strategy.setdefault(sname, {})["recall@10_in_auto"] = round(float(np.mean(r)), 4)
    log(f"work list {pre_ms:.3f} ms; search kernel {search_ms:.3f} ms, "
        f"rerun {rerun_ms:.3f} ms, {achieved:.1f} GB/s algorithmic")

    # ---- CPU baseline: the oracle's HSIG search on the same index file ----
    cpu = None
    if not args.no_cpu_baseline:
        try:
            cpu = cpu_baseline(args, W, index, ids, k, ef, m, bp, nq)
        except Exception as e:  # the GPU line is still reported
            log(f"CPU baseline failed: {e!r}")
            cpu = {"value": None, "unit": "queries/s", "cores": 0, "kind": "oracle", "sample": f"failed: {e!r}"}
    line = {
        "metric": METRIC, "value": round(qps, 1), "unit": "queries/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(sec * 1e3, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"mixed1m: n={spec.n} d={spec.d} (1024-centre mixture, sigma 0.2), attribute "
                               f"uniform in [0, 2^31), HSIG S={spec.S} M={spec.M} efCons={spec.ef_cons} built on GPU; "
                               f"{nq} queries, range fraction log-uniform [1e-3, 1], k={k}, auto strategy",
                   "n": spec.n, "d": spec.d, "nq": nq, "k": k, "ef": ef, "m": m, "beam_p": bp,
                   "recall@10": round(rec, 4),
                   "recall_by_ef": {str(e): round(r, 4) for e, r in recalls.items()},
                   "strategy_mix": {"pre": int(mix[1]), "hybrid": int(mix[2]), "post": int(mix[3])},
                   "build_s": round(build_s, 1)},
        "per_strategy": per_strategy,
        "roofline": roofline,
        "alt_tiled_prescan": tiled_alt,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def cpu_baseline(args, W, index, ids, k, ef, m, bp, nq):
    """The oracle's HSIG search (plain C++, one query per thread) on the same index file."""
    import numpy as np
    from oracle import hsig
    with tempfile.TemporaryDirectory(dir="/tmp") as td:
        path = os.path.join(td, "bench.uix")
        t0 = time.time()
        index.save(path)
        ref = hsig.Index.read(path)
        log(f"index file written and read by the oracle ({time.time() - t0:.1f}s)")
    ncpu = min(16, len(os.sched_getaffinity(0)))
    sample = np.arange(min(args.cpu_queries, nq))
    parts = np.array_split(sample, ncpu)
    res = [None] * ncpu

    def work(i):
        p = parts[i]
        res[i] = ref.search(W.queries[p], W.l[p], W.h[p], k, ef, m=m, p=bp)[0]

    t0 = time.perf_counter()
    th = [threading.Thread(target=work, args=(i,)) for i in range(ncpu)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    cpu_s = time.perf_counter() - t0
    cpu_ids = np.concatenate(res)
    agree = float(np.mean([np.array_equal(cpu_ids[i], ids.cpu().numpy()[i]) for i in range(len(sample))]))
    cpu = {"value": round(len(sample) / cpu_s, 1), "unit": "queries/s", "cores": ncpu, "kind": "oracle",
           "sample": f"first {len(sample)} of the {nq} queries, auto strategy, ef={ef}, m={m}, p={bp}, same index file; "
                     f"{agree:.4f} of them return the GPU's ids"}
    log(f"CPU oracle: {cpu['value']:,.0f} QPS on {ncpu} threads ({cpu_s:.1f}s), id agreement {agree:.4f}")

    return cpu


def profiled_traffic(m, ef, bp):
    """HBM bytes per launch of the search kernel from the committed rocprofv3 counter summary,
    or None when the kernel sources or the setting differ from what was profiled."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_search_mixed1m.json")
    if not os.path.exists(path):
        return None
    prof = json.load(open(path))
    src = b"".join(open(os.path.join(ROOT, "paper_2412_02448_amd", "csrc", x), "rb").read()
                   for x in ("search.hip", "wave.h"))
    if hashlib.sha256(src).hexdigest() != prof["source_sha256"]:
        return None
    if f"--m {m} --ef {ef} --p {bp} " not in prof["args"] + " ":
        return None
    return int(prof["traffic_bytes"])


def profile_run(args, index, Q, L, H, k, spec, nq, build_s):
    """Timed steps at a fixed setting plus one counted call: the search kernel's
    launches all share one configuration, so a profiler's average matches."""
    import numpy as np
    import torch
    m, ef, bp = args.m, args.ef, args.p
    for _ in range(args.warmup):
        index.search(Q, L, H, k, ef, m=m, beam_p=bp)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        index.search(Q, L, H, k, ef, m=m, beam_p=bp)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t) / args.steps
    ids, dist, strat, stats = index.search(Q, L, H, k, ef, m=m, beam_p=bp, stats=True, timing=True)
    torch.cuda.synchronize()
    pre_ms, search_ms, rerun_ms = index.last_timing()
    st = stats.cpu().numpy().astype(np.int64)
    per_q = st[:, 0] * spec.d * 4 + st[:, 4] * 4 + (st[:, 5] >= 0) * (spec.d * 4 + k * 12)
    b = int(per_q[st[:, 3] == 0].sum())
    print(json.dumps({"profile_run": True, "m": m, "ef": ef, "beam_p": bp, "qps": round(nq / sec, 1),
                      "ms_per_step": round(sec * 1e3, 4), "search_launch_ms": round(search_ms, 4),
                      "rerun_launch_ms": round(rerun_ms, 4), "bytes_per_launch": b,
                      "achieved_GBps": round(b / (search_ms * 1e-3) / 1e9, 1), "build_s": round(build_s, 1)}),
          flush=True)


if __name__ == "__main__":
    main()
