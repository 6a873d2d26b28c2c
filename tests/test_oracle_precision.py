"""Oracle pins for the low-precision vector stores and the FP32 rerank.

The BF16 and FP8 E4M3 roundings are pinned against PyTorch's own conversions
(a library routine, round to nearest even) and the format's value table; the
rerank is pinned by a special case: on vectors that both formats hold exactly,
a search over a low-precision copy must return exactly what the FP32 search
returns.
"""
import numpy as np
import pytest
import torch

from oracle import exact, hsig
from synth import workloads as w


def test_e4m3_value_table():
    codes = np.arange(256, dtype=np.uint8)
    ours = hsig.e4m3_decode(codes)
    lib = torch.from_numpy(codes.copy()).view(torch.float8_e4m3fn).float().numpy()
    nan = np.isnan(lib)
    assert np.array_equal(np.isnan(ours), nan)
    assert nan.sum() == 2  # S.1111.111 only
    assert np.array_equal(ours[~nan].view(np.uint32), lib[~nan].view(np.uint32))
    # landmarks of the format: smallest subnormal, smallest normal, one, largest
    assert ours[0x01] == 2.0 ** -9 and ours[0x08] == 2.0 ** -6 and ours[0x38] == 1.0 and ours[0x7E] == 448.0
    # codes 0x00..0x7E increase, which the nearest-code search relies on
    assert np.all(np.diff(ours[:0x7F]) > 0)


def test_e4m3_encode_matches_library():
    rng = np.random.default_rng(0)
    pos = hsig.e4m3_decode(np.arange(0x7F, dtype=np.uint8)).astype(np.float64)
    mids = (pos[:-1] + pos[1:]) / 2  # exact in FP32: ties must go to the even code
    vals = np.concatenate([
        pos, -pos, mids, -mids,
        rng.uniform(-448, 448, 20000), rng.standard_normal(20000) * 3, rng.uniform(-1e-3, 1e-3, 5000),
        np.nextafter(mids, 0), np.nextafter(mids, 1000),
    ]).astype(np.float32)
    ours = hsig.e4m3_encode(vals)
    lib = torch.from_numpy(vals).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    # the library keeps the sign of zero; so do we
    assert np.array_equal(ours, lib)
    ties = hsig.e4m3_encode(mids.astype(np.float32))
    assert np.all((ties & 1) == 0)
    # beyond the largest finite value: clamp (the library returns NaN there)
    big = np.array([448.0, 449.0, 463.9, 464.0, 1e6, -500.0], np.float32)
    assert hsig.e4m3_encode(big).tolist() == [0x7E] * 5 + [0xFE]


def test_bf16_matches_library():
    rng = np.random.default_rng(1)
    x = np.concatenate([
        rng.standard_normal(50000).astype(np.float32),
        (rng.standard_normal(5000) * 1e30).astype(np.float32),
        np.array([0.0, -0.0, 1e-40, -3e-39, 3.3895e38, np.inf, -np.inf], np.float32),
    ])
    # exact midpoints between neighbouring bfloat16 values
    b = rng.integers(0, 0x7F00, 5000).astype(np.uint32) << 16
    x = np.concatenate([x, (b | 0x8000).view(np.float32)])
    ours = hsig.bf16_bits(x)
    lib = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(ours, lib)
    assert np.all((hsig.bf16_bits((b | 0x8000).view(np.float32)) & 1) == 0)


def test_fp8_rows_invariants():
    rng = np.random.default_rng(2)
    X = (rng.standard_normal((300, 64)) * rng.uniform(0.01, 100, (300, 1))).astype(np.float32)
    X[7] = 0.0
    codes, sc, back = hsig.fp8_rows(X)
    mx = np.abs(X).max(1)
    assert sc[7] == 1.0 and np.all(codes[7] == 0) and np.all(back[7] == 0)
    nz = mx > 0
    assert np.array_equal(sc[nz], (mx[nz] / np.float32(448)).astype(np.float32))
    # the largest component of every non-zero row maps to +-448
    am = np.abs(X).argmax(1)
    assert np.all((codes[np.arange(300), am] & 0x7F)[nz] == 0x7E)
    # read-back = code value * scale in FP32, within half a code spacing of the input
    assert np.array_equal(back, (hsig.e4m3_decode(codes) * sc[:, None]).astype(np.float32))
    y = np.abs(X) / sc[:, None]
    half_step = np.where(y < 2.0 ** -6, 2.0 ** -10, 2.0 ** (np.floor(np.log2(np.maximum(y, 2.0 ** -6))) - 4))
    assert np.all(np.abs(back - X) <= (half_step * 1.0001 + 1e-30) * sc[:, None])


@pytest.fixture(scope="module")
def exact_grid_index():
    """Vectors with integer components in [-7, 7] and max |component| = 7 per row:
    BF16 holds them exactly, and the FP8 scale 7/448 = 2^-6 makes every x / s an
    E4M3 value (multiples of 64 up to 448)."""
    spec = w.scaled(w.SPECS["hybrid10k"], n=1500, nq=30, S=4, M=8, ef_cons=40)
    W = w.make(spec, base_seed=5)
    X = np.clip(np.rint(W.base * 2.5), -7, 7).astype(np.float32)
    X[:, 0] = 7.0
    Q = np.rint(W.queries * 2.5).astype(np.float32)
    ix = hsig.Index.build(X, W.attr, W.level_u, spec.S, spec.M, spec.ef_cons)
    return X, Q, W, ix


def test_exact_store_search_equals_fp32(exact_grid_index):
    X, Q, W, ix = exact_grid_index
    assert np.array_equal(hsig.bf16_values(X), X)
    assert np.array_equal(hsig.fp8_rows(X)[2], X)
    for strategy in (hsig.AUTO, hsig.PRE, hsig.HYBRID, hsig.POST):
        ix.set_store(hsig.FP32)
        ref = ix.search(Q, W.l, W.h, 10, 32, strategy=strategy)
        for prec in (hsig.BF16, hsig.FP8E4M3):
            ix.set_store(prec, 4)
            got = ix.search(Q, W.l, W.h, 10, 32, strategy=strategy)
            assert np.array_equal(ref[0], got[0]) and np.array_equal(ref[1], got[1])
    ix.set_store(hsig.FP32)


@pytest.fixture(scope="module")
def mixture_index():
    spec = w.scaled(w.SPECS["hybrid10k"], n=3000, nq=60, S=4, M=12, ef_cons=60)
    W = w.make(spec, base_seed=6)
    ix = hsig.Index.build(W.base, W.attr, W.level_u, spec.S, spec.M, spec.ef_cons)
    return W, ix


@pytest.mark.parametrize("prec", [hsig.BF16, hsig.FP8E4M3])
def test_rerank_outputs_exact_distances(mixture_index, prec):
    W, ix = mixture_index
    ix.set_store(prec, 4)
    try:
        for strategy in (hsig.HYBRID, hsig.POST, hsig.PRE):
            ids, dist, cnt = ix.search(W.queries, W.l, W.h, 10, 48, strategy=strategy, counters=True)
            ext = ix.ext_ids()
            pos = np.empty(ix.n, np.int64)
            pos[ext] = np.arange(ix.n)
            for i in range(len(ids)):
                row = ids[i][ids[i] >= 0]
                d32 = [hsig.dist32(W.queries[i], W.base[e]) for e in row]
                # distances are the exact FP32 ones, sorted by (distance, internal id)
                assert np.array_equal(np.asarray(d32, np.float32), dist[i][: len(row)])
                keys = list(zip(dist[i][: len(row)].tolist(), pos[row].tolist()))
                assert keys == sorted(keys)
                assert np.all((W.attr[row] >= W.l[i]) & (W.attr[row] <= W.h[i]))
            if strategy == hsig.PRE:  # the scan ignores the copy: exact
                assert cnt[:, hsig.NRERANK].sum() == 0
                for i in range(len(ids)):
                    tid, _ = exact.rfknn(W.base, W.attr, W.queries[i], W.l[i], W.h[i], 10)
                    assert ids[i][: len(tid)].tolist() == tid.tolist()
            else:
                found = cnt[:, hsig.NRERANK]
                assert np.all(found <= 40) and found.sum() > 0
    finally:
        ix.set_store(hsig.FP32)


def test_rerank_improves_low_precision_recall(mixture_index):
    """Re-scoring more results in FP32 cannot lose a true neighbour the search found:
    recall with rerank_mult = ef / k (every result re-scored) is at least that
    with rerank_mult = 1 (the copy's own order)."""
    W, ix = mixture_index
    truth = [exact.rfknn(W.base, W.attr, W.queries[i], W.l[i], W.h[i], 10)[0] for i in range(len(W.queries))]
    rec = {}
    for mult in (1, 5):
        ix.set_store(hsig.FP8E4M3, mult)
        ids, _ = ix.search(W.queries, W.l, W.h, 10, 50, strategy=hsig.HYBRID)
        rec[mult] = np.mean([exact.recall(ids[i], truth[i], 10, len(truth[i])) for i in range(len(truth))])
    ix.set_store(hsig.FP32)
    assert rec[5] >= rec[1]
