"""Seeded synthetic workloads for range-filtered k-NN search.

This module only draws random inputs: base vectors, attributes, query vectors,
query ranges and the uniform variates an index build consumes.  It holds none
of the search or build arithmetic, so both the oracle and the HIP path can use
it without sharing any of the method.

Shapes follow the paper's workloads (Section 5.1, Table 1: SIFT1M-like 1M x 128,
GIST1M-like 1M x 960; Section 5.8: the 10M scalability point).  The real
datasets are not available; Gaussian mixtures stand in for them:

* centres ~ N(0, I_d), mixture weights uniform, point = centre + sigma * N(0, I_d);
* queries are fresh draws from the same mixture;
* a query of range fraction f covers Y = max(1, round(f * n)) objects: a start
  rank r ~ U{0 .. n - Y} is drawn in attribute order and the range is
  [attr_sorted[r], attr_sorted[r + Y - 1]] (inclusive), so |R| = Y up to
  duplicate attribute values at the two ends.

Seeds (numpy PCG64): data = 1, attributes = 2, queries = 3, ranges = 4,
level variates = 5, each offset by the caller's base seed.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED_DATA, SEED_ATTR, SEED_QUERY, SEED_RANGE, SEED_LEVEL = 1, 2, 3, 4, 5


@dataclasses.dataclass(frozen=True)
class WorkloadSpec:
    name: str
    n: int
    d: int
    centers: int
    sigma: float
    attr: str                 # "perm" (permutation of 0..n-1) or "uniform31" (uniform int in [0, 2^31))
    S: int                    # segments
    M: int                    # per-chunk degree
    ef_cons: int
    nq: int
    ranges: str               # "fixed" (each query at every fraction in `fractions`) or "loguniform"
    fractions: tuple = ()
    f_lo: float = 1e-3
    f_hi: float = 1.0
    k: int = 10
    efs: tuple = (64,)


# The paper's configuration family, as the workloads of this repository name them.
SPECS = {
    # 10k x 128, 16-centre mixture (sigma 0.3), permutation attribute, HSIG S=8 M=16 efCons=100,
    # 200 queries at each of the fractions {0.01, 0.1, 0.5}, k=10, ef=64.
    "hybrid10k": WorkloadSpec("hybrid10k", 10_000, 128, 16, 0.3, "perm", 8, 16, 100, 200,
                              "fixed", fractions=(0.01, 0.1, 0.5), k=10, efs=(64,)),
    # 1M x 128, 1024-centre mixture (sigma 0.2), uniform int attribute, HSIG S=32 M=32,
    # 10k queries with log-uniform range fraction in [1e-3, 1], k=10, ef in {32,64,128,256}.
    "mixed1m": WorkloadSpec("mixed1m", 1_000_000, 128, 1024, 0.2, "uniform31", 32, 32, 100, 10_000,
                            "loguniform", f_lo=1e-3, f_hi=1.0, k=10, efs=(32, 64, 128, 256)),
    # Batched form of hybrid10k: 100k queries, log-uniform fractions in [1e-4, 1].
    "batch100k": WorkloadSpec("batch100k", 10_000, 128, 16, 0.3, "perm", 8, 16, 100, 100_000,
                              "loguniform", f_lo=1e-4, f_hi=1.0, k=10, efs=(64,)),
    # Precision form: 1M x 960, 512 centres (sigma assumed 0.2), S=8 M=16.
    "gist1m": WorkloadSpec("gist1m", 1_000_000, 960, 512, 0.2, "uniform31", 8, 16, 100, 10_000,
                           "loguniform", f_lo=1e-3, f_hi=1.0, k=10, efs=(64,)),
    # Serving form: 10M x 96, 4096 centres, S=64 M=24.
    "serve10m": WorkloadSpec("serve10m", 10_000_000, 96, 4096, 0.2, "uniform31", 64, 24, 100, 100_000,
                             "serving", k=10, efs=(64,)),
}


def scaled(spec: WorkloadSpec, n: int | None = None, nq: int | None = None, **kw) -> WorkloadSpec:
    """The same recipe at another size (for tests that must finish in seconds)."""
    upd = dict(kw)
    if n is not None:
        upd["n"] = n
    if nq is not None:
        upd["nq"] = nq
    upd.setdefault("name", f"{spec.name}@n{upd.get('n', spec.n)}")
    return dataclasses.replace(spec, **upd)


def _rng(base_seed: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64([base_seed, stream]))


def mixture(n: int, d: int, centers: int, sigma: float, base_seed: int, stream: int,
            chunk: int = 1 << 18) -> np.ndarray:
    """n points of the Gaussian mixture whose centres are drawn from the data stream."""
    crng = _rng(base_seed, SEED_DATA)
    cen = crng.standard_normal((centers, d), dtype=np.float32)
    rng = _rng(base_seed, stream) if stream != SEED_DATA else crng
    out = np.empty((n, d), dtype=np.float32)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        lab = rng.integers(0, centers, size=e - s)
        noise = rng.standard_normal((e - s, d), dtype=np.float32)
        out[s:e] = cen[lab] + np.float32(sigma) * noise
    return out


def attributes(spec: WorkloadSpec, base_seed: int) -> np.ndarray:
    rng = _rng(base_seed, SEED_ATTR)
    if spec.attr == "perm":
        return rng.permutation(spec.n).astype(np.int64)
    if spec.attr == "uniform31":
        return rng.integers(0, 1 << 31, size=spec.n, dtype=np.int64)
    raise ValueError(spec.attr)


def range_fractions(spec: WorkloadSpec, base_seed: int) -> np.ndarray:
    """One range fraction per search (len = number of searches)."""
    rng = _rng(base_seed, SEED_RANGE)
    if spec.ranges == "fixed":
        return np.repeat(np.asarray(spec.fractions, dtype=np.float64)[None, :], spec.nq, 0).reshape(-1)
    if spec.ranges == "loguniform":
        u = rng.random(spec.nq)
        return np.exp(math.log(spec.f_lo) + u * (math.log(spec.f_hi) - math.log(spec.f_lo)))
    if spec.ranges == "serving":
        # 30% in [1e-5, 1e-3), 40% in [1e-3, 0.1), 30% in [0.1, 1], each log-uniform.
        c = rng.random(spec.nq)
        u = rng.random(spec.nq)
        lo = np.where(c < 0.3, 1e-5, np.where(c < 0.7, 1e-3, 0.1))
        hi = np.where(c < 0.3, 1e-3, np.where(c < 0.7, 0.1, 1.0))
        return np.exp(np.log(lo) + u * (np.log(hi) - np.log(lo)))
    raise ValueError(spec.ranges)


def ranges_for(attr: np.ndarray, fractions: np.ndarray, base_seed: int, stream_offset: int = 0):
    """Inclusive [l, h] per search covering about fraction * n objects."""
    n = attr.shape[0]
    srt = np.sort(attr, kind="stable")
    rng = _rng(base_seed + stream_offset, SEED_RANGE + 100)
    Y = np.maximum(1, np.rint(fractions * n).astype(np.int64))
    Y = np.minimum(Y, n)
    r = (rng.random(len(Y)) * (n - Y + 1)).astype(np.int64)
    r = np.minimum(r, n - Y)
    return srt[r].copy(), srt[r + Y - 1].copy()


def level_uniforms(n: int, base_seed: int) -> np.ndarray:
    """U in (0, 1] per object, consumed by an index build's level draw."""
    rng = _rng(base_seed, SEED_LEVEL)
    return 1.0 - rng.random(n)  # random() is in [0, 1)


@dataclasses.dataclass
class Workload:
    spec: WorkloadSpec
    base: np.ndarray          # [n, d] float32, row = external id
    attr: np.ndarray          # [n] int64
    queries: np.ndarray       # [nsearch, d] float32
    l: np.ndarray             # [nsearch] int64 (inclusive)
    h: np.ndarray             # [nsearch] int64 (inclusive)
    fractions: np.ndarray     # [nsearch] float64
    level_u: np.ndarray       # [n] float64 in (0, 1]


def more_queries(spec: WorkloadSpec, attr: np.ndarray, nq: int, base_seed: int = 0, stream: int = 1):
    """Another query set of the same recipe over the same data (e.g. held-out tuning queries).

    Query vectors come from the same mixture (same centres); vectors, range
    fractions and placements use their own streams.  Returns (queries, l, h, fractions)."""
    sub = dataclasses.replace(spec, nq=nq)
    q = mixture(nq, spec.d, spec.centers, spec.sigma, base_seed, SEED_QUERY + 1000 * stream)
    fr = range_fractions(sub, base_seed + 7919 * stream)
    if spec.ranges == "fixed":
        q = np.repeat(q, len(spec.fractions), axis=0)
    l, h = ranges_for(attr, fr, base_seed, stream_offset=104729 * stream)
    return np.ascontiguousarray(q), l, h, fr


def make(spec: WorkloadSpec, base_seed: int = 0) -> Workload:
    base = mixture(spec.n, spec.d, spec.centers, spec.sigma, base_seed, SEED_DATA)
    attr = attributes(spec, base_seed)
    q = mixture(spec.nq, spec.d, spec.centers, spec.sigma, base_seed, SEED_QUERY)
    fr = range_fractions(spec, base_seed)
    if spec.ranges == "fixed":
        q = np.repeat(q, len(spec.fractions), axis=0)
    l, h = ranges_for(attr, fr, base_seed)
    return Workload(spec, base, attr, np.ascontiguousarray(q), l, h, fr, level_uniforms(spec.n, base_seed))


def second_attribute(n: int, nsearch: int, base_seed: int = 0, f_lo: float = 0.05, f_hi: float = 1.0):
    """A second attribute per object (uniform in [0, 2^31), independent of the first)
    and, per search, an inclusive range on it covering a fraction log-uniform in
    [f_lo, f_hi] of the objects.  Returns (attr2 [n], l2 [nsearch], h2 [nsearch])."""
    rng = _rng(base_seed, SEED_ATTR + 500)
    attr2 = rng.integers(0, 1 << 31, size=n, dtype=np.int64)
    u = _rng(base_seed, SEED_RANGE + 500).random(nsearch)
    fr = np.exp(math.log(f_lo) + u * (math.log(f_hi) - math.log(f_lo)))
    l2, h2 = ranges_for(attr2, fr, base_seed, stream_offset=31337)
    return attr2, l2, h2
