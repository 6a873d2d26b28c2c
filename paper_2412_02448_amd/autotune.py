"""Search-parameter tuning for a resident index.

The paper sets its search parameters by sweeping them (Sec. 5.7: ef and m trade
recall for speed; Sec. 4.2: tau_A and tau_B come from sample queries).  This
tuner does the same on the GPU: for sample queries with known exact answers
(the pre-filter scan forced on every sample query gives them), it measures
recall@k and throughput of the range-aware search over a grid of
(tau_A, tau_B, m, ef, beam width p) and returns the fastest setting whose
recall reaches the target (the GPU's cost crossovers between the strategies
differ from the CPU's that the paper's 1% / 50% reflect).  Every measurement
runs the library's kernels; this module only orchestrates calls and computes
recall.
"""
from __future__ import annotations

import dataclasses
import time

import numpy as np


@dataclasses.dataclass
class Setting:
    m: int
    ef: int
    beam_p: int
    recall: float
    qps: float
    tau_a: float = 0.01
    tau_b: float = 0.5
    visit_cap: int = 0  # 0: the library's default
    pre_chunk: int = 0  # 0: the library's default

    def kwargs(self) -> dict:
        """Search keyword arguments of this setting."""
        return dict(m=self.m, beam_p=self.beam_p, tau_a=self.tau_a, tau_b=self.tau_b, visit_cap=self.visit_cap,
                    pre_chunk=self.pre_chunk)


def recall_at_k(ids: np.ndarray, truth: np.ndarray) -> float:
    """Mean over queries of |found & exact| / |exact| (Eq. 1; |exact| = min(k, |R|)).
    Rows hold distinct ids padded with -1; a query with no exact answer counts 1."""
    if len(ids) == 0:
        return 1.0
    valid = truth >= 0
    hit = np.empty(len(ids), np.int64)
    step = max(1, (1 << 24) // max(1, truth.shape[1] * ids.shape[1]))  # rows per block of comparisons
    for a in range(0, len(ids), step):
        t, f = truth[a:a + step], ids[a:a + step]
        hit[a:a + step] = ((t[:, :, None] == f[:, None, :]).any(2) & valid[a:a + step]).sum(1)
    n = valid.sum(1)
    return float(np.where(n > 0, hit / np.maximum(n, 1), 1.0).mean())


def exact_answers(index, Q, L, H, k):
    """Exact range-filtered k-NN ids of every query (strategy A on all of them)."""
    import torch
    from . import PRE
    ids, _, _ = index.search(Q, L, H, k, k, strategy=PRE)
    torch.cuda.synchronize()
    return ids.cpu().numpy()


def tune(index, Q, L, H, k: int, target: float, ms=None, efs=(32, 64, 128, 256), ps=(1, 2, 4),
         taus=((0.01, 0.5), (0.01, 0.3), (0.005, 0.3), (0.01, 0.2)), visit_caps=(512, 1024), pre_chunks=(),
         reps: int = 10, log=None):
    """Fastest (tau_A, tau_B, m, ef, p) reaching recall@k >= target on the given sample
    queries; taus lists the (tau_A, tau_B) fractions of the strategy rule to try.  The
    visited-cache sizes in visit_caps, then the pre-filter chunk lengths in pre_chunks, are
    timed on the best setting (results do not depend on either); one replaces the default
    only when it is more than 3% faster.

    Returns (best Setting or None, list of every Setting measured)."""
    import torch
    if ms is None:
        M = index.M
        ms = (M, (3 * M) // 2, 2 * M, 3 * M)
    truth = exact_answers(index, Q, L, H, k)
    table = []
    for ta, tb in taus:
        for m in ms:
            if m > index.S * index.M:
                continue
            pending = list(ps)  # beam widths still below the target at the efs tried so far
            for ef in efs:
                if ef < k or not pending:
                    continue
                for p in list(pending):
                    kw = dict(m=m, beam_p=p, tau_a=ta, tau_b=tb)
                    ids, _, _ = index.search(Q, L, H, k, ef, **kw)
                    torch.cuda.synchronize()
                    rec = recall_at_k(ids.cpu().numpy(), truth)  # beam width changes the results
                    if rec < target:
                        table.append(Setting(m, ef, p, rec, 0.0, ta, tb))
                        continue
                    t = time.perf_counter()
                    for _ in range(reps):
                        index.search(Q, L, H, k, ef, **kw)
                    torch.cuda.synchronize()
                    qps = Q.shape[0] * reps / (time.perf_counter() - t)
                    table.append(Setting(m, ef, p, rec, qps, ta, tb))
                    pending.remove(p)  # larger ef only costs more once the target is met
                    if log:
                        log(f"tune tau=({ta}, {tb}) m={m} ef={ef} p={p}: recall {rec:.4f}, {qps:,.0f} QPS")
    ok = [s for s in table if s.recall >= target and s.qps > 0]
    best = None
    if ok:
        # settings within 2% of the fastest are within the timing noise: take the most accurate
        top = max(s.qps for s in ok)
        best = max((s for s in ok if s.qps >= 0.98 * top), key=lambda s: (s.recall, s.qps))
    if best is not None:
        # the on-chip visited cache trades LDS (waves per CU) against HBM tag reads;
        # results do not depend on it
        for vc in visit_caps:
            kw = dict(best.kwargs(), visit_cap=vc)
            index.search(Q, L, H, k, best.ef, **kw)
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(reps):
                index.search(Q, L, H, k, best.ef, **kw)
            torch.cuda.synchronize()
            qps = Q.shape[0] * reps / (time.perf_counter() - t)
            cand = dataclasses.replace(best, qps=qps, visit_cap=vc)
            table.append(cand)
            if log:
                log(f"tune visit_cap={vc}: {qps:,.0f} QPS")
            if qps > 1.03 * best.qps:  # the default stays unless another size is clearly faster
                best = cand
        base = best
        for pc in pre_chunks:
            kw = dict(base.kwargs(), pre_chunk=pc)
            index.search(Q, L, H, k, base.ef, **kw)
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(reps):
                index.search(Q, L, H, k, base.ef, **kw)
            torch.cuda.synchronize()
            qps = Q.shape[0] * reps / (time.perf_counter() - t)
            cand = dataclasses.replace(base, qps=qps, pre_chunk=pc)
            table.append(cand)
            if log:
                log(f"tune pre_chunk={pc}: {qps:,.0f} QPS")
            if qps > 1.03 * best.qps:
                best = cand
    return best, table
