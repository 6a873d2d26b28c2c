"""TEST INFRASTRUCTURE -- NOT PART OF THE PRODUCT.

ctypes wrapper of the plain C++ HSIG reference (``hsig_ref.cpp``): the build by
Alg. 6 (with Alg. 1, 4, 5 and the skip list), the plain HNSW build by Alg. 3,
the search strategies of Sec. 4.2 and the index file.  Only the tests, the
smoke check and the CPU-baseline leg of the benchmark may import it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hsig_ref.cpp")
_LIB = os.path.join(_HERE, "liboracle_hsig.so")

AUTO, PRE, HYBRID, POST = 0, 1, 2, 3
# per-query counters written by search(): see the C_* enum in hsig_ref.cpp
NDIST, NEXP, NVISIT0, MAXCAND, MAXLIVE, STRAT, LO, HI, NRERANK, ENTRY, NCOUNT = range(11)
FP32, BF16, FP8E4M3 = 0, 1, 2


def compile_oracle(force: bool = False) -> str:
    """Compiles the reference with g++ (no fast-math, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
                               "-fno-fast-math", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(compile_oracle())
        P, I64, I32, D, F = C.c_void_p, C.c_int64, C.c_int, C.c_double, C.c_float
        L.orc_build.restype = P
        L.orc_build.argtypes = [P, P, P, I64, I32, I32, I32, I32, I32, D, C.c_uint64, I32, I64]
        L.orc_insert.restype = I32
        L.orc_insert.argtypes = [P, P, P, P, I64]
        L.orc_read.restype = P
        L.orc_read.argtypes = [C.c_char_p]
        L.orc_write.restype = I32
        L.orc_write.argtypes = [P, C.c_char_p]
        L.orc_free.argtypes = [P]
        L.orc_info.argtypes = [P, P]
        L.orc_last_error.restype = C.c_char_p
        L.orc_dist32.restype = F
        L.orc_dist32.argtypes = [P, P, I32]
        L.orc_level_of.restype = I32
        L.orc_level_of.argtypes = [D, D]
        L.orc_dist64.restype = D
        L.orc_dist64.argtypes = [P, P, I32]
        L.orc_search.restype = I32
        L.orc_search.argtypes = [P, P, I64, P, P, I32, I32, I32, I32, I32, D, D, P, P, P, I32, I32, P, P]
        L.orc_set_attr2.restype = I32
        L.orc_set_attr2.argtypes = [P, P, I64]
        L.orc_zorder_map.restype = I32
        L.orc_zorder_map.argtypes = [P, P, I64, P]
        L.orc_zorder_keys.restype = I32
        L.orc_zorder_keys.argtypes = [P, P, P, I64, P]
        L.orc_zorder_range.restype = I32
        L.orc_zorder_range.argtypes = [P, P, P, P, P, I64, P, P]
        L.orc_set_zorder.restype = I32
        L.orc_set_zorder.argtypes = [P, P, P, P, I64]
        L.orc_search_box.restype = I32
        L.orc_search_box.argtypes = [P, P, I64, P, P, P, P, I32, I32, I32, I32, I32, D, D, P, P, P, I32, I32]
        L.orc_layer_search.restype = I32
        L.orc_layer_search.argtypes = [P, P, I32, I32, I32, I32, I32, I32, I32, I32, I64, I64, P, P]
        L.orc_prune.restype = I32
        L.orc_prune.argtypes = [P, P, I32, I32, I32, P]
        L.orc_get_attr.argtypes = [P, P]
        L.orc_get_ext.argtypes = [P, P]
        L.orc_get_level.argtypes = [P, P]
        L.orc_get_segments.argtypes = [P, P, P, P]
        L.orc_get_layer.argtypes = [P, I32, P, P]
        L.orc_skiplist_range.restype = I64
        L.orc_skiplist_range.argtypes = [P, I64, I64, P, I64]
        L.orc_build_chunk.restype = I32
        L.orc_build_chunk.argtypes = [P, I64, I32, I32, P, I32]
        L.orc_build_level.restype = I32
        L.orc_build_level.argtypes = [P, I64]
        L.orc_bf16.argtypes = [P, I64, P]
        L.orc_e4m3_encode.argtypes = [P, I64, P]
        L.orc_e4m3_decode.argtypes = [P, I64, P]
        L.orc_fp8_rows.argtypes = [P, I64, I32, P, P, P]
        L.orc_neighbours.restype = I32
        L.orc_neighbours.argtypes = [P, I32, I32, I32, I32, I32, I32, P, I32]
        L.orc_set_store.restype = I32
        L.orc_set_store.argtypes = [P, I32, I32]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def dist32(q: np.ndarray, x: np.ndarray) -> np.float32:
    q = np.ascontiguousarray(q, np.float32)
    x = np.ascontiguousarray(x, np.float32)
    return np.float32(lib().orc_dist32(_p(q), _p(x), q.shape[0]))


def dist64(q: np.ndarray, x: np.ndarray) -> float:
    q = np.ascontiguousarray(q, np.float32)
    x = np.ascontiguousarray(x, np.float32)
    return float(lib().orc_dist64(_p(q), _p(x), q.shape[0]))


def level_of(u: float, M: int) -> int:
    """Level drawn for uniform variate u with mL = 1/ln(M) (Alg. 6)."""
    import math
    return int(lib().orc_level_of(float(u), 1.0 / math.log(M)))


def bf16_bits(x: np.ndarray) -> np.ndarray:
    """Bit patterns of the nearest bfloat16 values (ties to even)."""
    x = np.ascontiguousarray(x, np.float32)
    out = np.zeros(x.shape, np.uint16)
    lib().orc_bf16(_p(x), x.size, _p(out))
    return out


def bf16_values(x: np.ndarray) -> np.ndarray:
    return (bf16_bits(x).astype(np.uint32) << 16).view(np.float32)


def e4m3_encode(y: np.ndarray) -> np.ndarray:
    """Nearest OCP E4M3 codes (ties to even, magnitudes above 448 clamp)."""
    y = np.ascontiguousarray(y, np.float32)
    out = np.zeros(y.shape, np.uint8)
    lib().orc_e4m3_encode(_p(y), y.size, _p(out))
    return out


def e4m3_decode(c: np.ndarray) -> np.ndarray:
    c = np.ascontiguousarray(c, np.uint8)
    out = np.zeros(c.shape, np.float32)
    lib().orc_e4m3_decode(_p(c), c.size, _p(out))
    return out


def fp8_rows(X: np.ndarray):
    """FP8 copy of each row: (codes [n, d] u8, scales [n] f32, values read back [n, d] f32)."""
    X = np.ascontiguousarray(X, np.float32)
    n, d = X.shape
    codes = np.zeros((n, d), np.uint8)
    sc = np.zeros(n, np.float32)
    back = np.zeros((n, d), np.float32)
    lib().orc_fp8_rows(_p(X), n, d, _p(codes), _p(sc), _p(back))
    return codes, sc, back


def prune(owner: np.ndarray, cands: np.ndarray, M: int) -> list[int]:
    owner = np.ascontiguousarray(owner, np.float32)
    cands = np.ascontiguousarray(cands, np.float32)
    out = np.zeros(max(1, len(cands)), np.int32)
    c = lib().orc_prune(_p(owner), _p(cands), len(cands), owner.shape[0], M, _p(out))
    return out[:c].tolist()


class Index:
    """A reference HSIG (or plain HNSW) built or read by the C++ oracle."""

    def __init__(self, handle):
        if not handle:
            raise RuntimeError(lib().orc_last_error().decode())
        self._h = handle
        info = np.zeros(9, np.int64)
        lib().orc_info(self._h, _p(info))
        (self.n, self.d, self.S, self.M0, self.MU, self.L, self.gentry, self.R, self.ef_cons) = map(int, info)

    @classmethod
    def build(cls, X, attr, level_u, S, M, ef_cons, M0=0, mL=0.0, seed=0, hnsw=False, bnd_n=0):
        """HSIG over X (Alg. 6, objects inserted in row order); segment boundaries from
        the attributes of the first bnd_n rows (0: all)."""
        X = np.ascontiguousarray(X, np.float32)
        attr = np.ascontiguousarray(attr, np.int64)
        level_u = np.ascontiguousarray(level_u, np.float64)
        n, d = X.shape
        h = lib().orc_build(_p(X), _p(attr), _p(level_u), n, d, S, M, M0, ef_cons, mL, seed, int(hnsw), int(bnd_n))
        return cls(h)

    def insert(self, X, attr, level_u) -> None:
        """Inserts more objects (Alg. 6) into an index built here; they take the next
        external ids.  Segment boundaries do not move."""
        X = np.ascontiguousarray(X, np.float32)
        attr = np.ascontiguousarray(attr, np.int64)
        level_u = np.ascontiguousarray(level_u, np.float64)
        if lib().orc_insert(self._h, _p(X), _p(attr), _p(level_u), X.shape[0]) != 0:
            raise ValueError(lib().orc_last_error().decode())
        info = np.zeros(9, np.int64)
        lib().orc_info(self._h, _p(info))
        (self.n, self.d, self.S, self.M0, self.MU, self.L, self.gentry, self.R, self.ef_cons) = map(int, info)

    @classmethod
    def read(cls, path: str):
        return cls(lib().orc_read(path.encode()))

    def write(self, path: str) -> None:
        rc = lib().orc_write(self._h, path.encode())
        if rc != 0:
            raise OSError(f"orc_write failed ({rc})")

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            try:
                _lib.orc_free(self._h)
            except Exception:
                pass
            self._h = None

    # --- tables of the frozen view (internal ids = attribute rank) ---
    def attr_sorted(self):
        a = np.zeros(self.n, np.int64)
        lib().orc_get_attr(self._h, _p(a))
        return a

    def ext_ids(self):
        a = np.zeros(self.n, np.int64)
        lib().orc_get_ext(self._h, _p(a))
        return a

    def levels(self):
        a = np.zeros(self.n, np.int32)
        lib().orc_get_level(self._h, _p(a))
        return a

    def segments(self):
        ss = np.zeros(self.S + 1, np.int64)
        en = np.zeros(self.S, np.int32)
        ml = np.zeros(self.S, np.int32)
        lib().orc_get_segments(self._h, _p(ss), _p(en), _p(ml))
        return ss, en, ml

    def layer(self, l: int):
        """(adj [n, S, mcap], glist [n, S*mcap]) of layer l, internal ids, -1 padded."""
        mc = self.M0 if l == 0 else self.MU
        adj = np.zeros((self.n, self.S, mc), np.int32)
        gl = np.zeros((self.n, self.S * mc), np.int32)
        lib().orc_get_layer(self._h, l, _p(adj), _p(gl))
        return adj, gl

    def neighbours(self, o: int, l: int, a: int, b: int, m: int, select_s1: bool = False) -> np.ndarray:
        """Internal ids a hybrid expansion of o on layer l takes (active segments a..b, budget m;
        selection S1 or S2 of Sec. 4.2, distances in the current store)."""
        out = np.zeros(self.S * max(self.M0, self.MU), np.int32)
        c = lib().orc_neighbours(self._h, o, l, a, b, m, int(select_s1), _p(out), out.size)
        if c < 0:
            raise IndexError((o, l, a, b, m))
        return out[:c]

    def skiplist_range(self, l: int, h: int):
        out = np.zeros(self.n, np.int64)
        c = lib().orc_skiplist_range(self._h, l, h, _p(out), self.n)
        if c < 0:
            raise RuntimeError("no build-side skip list (index was read from a file)")
        return out[:c]

    def build_chunk(self, v: int, l: int, j: int):
        out = np.zeros(4096, np.int64)
        c = lib().orc_build_chunk(self._h, v, l, j, _p(out), 4096)
        if c < 0:
            raise IndexError((v, l, j))
        return out[:c].tolist()

    def build_level(self, v: int) -> int:
        return lib().orc_build_level(self._h, v)

    def set_store(self, precision: int, rerank_mult: int = 4) -> None:
        """Graph searches rank by FP32 (0), a BF16 copy (1) or an FP8 E4M3 copy (2) of the
        vectors; with a copy, the best rerank_mult * k results are re-scored in FP32."""
        if lib().orc_set_store(self._h, precision, rerank_mult) != 0:
            raise ValueError(lib().orc_last_error().decode())

    def set_attr2(self, attr2) -> None:
        """Second attribute of every object, indexed by external id (conjunctive queries)."""
        a = np.ascontiguousarray(attr2, np.int64)
        if lib().orc_set_attr2(self._h, _p(a), a.size) != 0:
            raise ValueError(lib().orc_last_error().decode())

    def search(self, Q, l, h, k, ef, m=0, p=1, strategy=AUTO, tau_a=0.01, tau_b=0.5,
               counters=False, batch_form=False, select_s1=False, l2=None, h2=None):
        """l2, h2: optional inclusive ranges on the second attribute (both or neither)."""
        Q = np.ascontiguousarray(Q, np.float32)
        l = np.ascontiguousarray(l, np.int64)
        h = np.ascontiguousarray(h, np.int64)
        if (l2 is None) != (h2 is None):
            raise ValueError("l2 and h2 go together")
        l2p = h2p = None
        if l2 is not None:
            l2 = np.ascontiguousarray(l2, np.int64)
            h2 = np.ascontiguousarray(h2, np.int64)
            l2p, h2p = _p(l2), _p(h2)
        nq = Q.shape[0]
        ids = np.zeros((nq, k), np.int64)
        dist = np.zeros((nq, k), np.float32)
        cnt = np.zeros((nq, NCOUNT), np.int64)
        rc = lib().orc_search(self._h, _p(Q), nq, _p(l), _p(h), k, ef, m, p, strategy, tau_a, tau_b,
                              _p(ids), _p(dist), _p(cnt), int(batch_form), int(select_s1), l2p, h2p)
        if rc != 0:
            raise ValueError(lib().orc_last_error().decode())
        return (ids, dist, cnt) if counters else (ids, dist)

    def set_zorder(self, zmap, a1, a2) -> None:
        """Both attributes of a z-order index, indexed by external id (box searches); the
        index must have been built on zorder_keys(zmap, a1, a2)."""
        m = np.ascontiguousarray(zmap, np.int64)
        a1 = np.ascontiguousarray(a1, np.int64)
        a2 = np.ascontiguousarray(a2, np.int64)
        if a1.size != a2.size or m.size != 4:
            raise ValueError("one pair per object and a map of 4 values")
        if lib().orc_set_zorder(self._h, _p(m), _p(a1), _p(a2), a1.size) != 0:
            raise ValueError(lib().orc_last_error().decode())

    def search_box(self, Q, l1, h1, l2, h2, k, ef, m=0, p=1, strategy=AUTO, tau_a=0.01, tau_b=0.5,
                   counters=False, batch_form=False, select_s1=False):
        """Box search on a z-order index: objects with l1 <= A1 <= h1 and l2 <= A2 <= h2."""
        Q = np.ascontiguousarray(Q, np.float32)
        r = [np.ascontiguousarray(x, np.int64) for x in (l1, h1, l2, h2)]
        nq = Q.shape[0]
        ids = np.zeros((nq, k), np.int64)
        dist = np.zeros((nq, k), np.float32)
        cnt = np.zeros((nq, NCOUNT), np.int64)
        rc = lib().orc_search_box(self._h, _p(Q), nq, *[_p(x) for x in r], k, ef, m, p, strategy, tau_a, tau_b,
                                  _p(ids), _p(dist), _p(cnt), int(batch_form), int(select_s1))
        if rc != 0:
            raise ValueError(lib().orc_last_error().decode())
        return (ids, dist, cnt) if counters else (ids, dist)

    def layer_search(self, q, ep, layer, ef, hybrid, a=0, b=0, c=0, filter=False, l=0, h=0):
        q = np.ascontiguousarray(q, np.float32)
        ids = np.zeros(max(ef, 1), np.int32)
        dist = np.zeros(max(ef, 1), np.float32)
        cnt = lib().orc_layer_search(self._h, _p(q), ep, layer, ef, int(hybrid), a, b, c, int(filter),
                                     l, h, _p(ids), _p(dist))
        return ids[:cnt], dist[:cnt]


def zorder_map(a1, a2) -> np.ndarray:
    """The z-order key map of two attributes (the multi-attribute extension, approach 2):
    [base1, shift1, base2, shift2]: each attribute's smallest value, and the shift that puts its
    largest value in the upper half of a 2^31-cell axis (negative: a left shift)."""
    a1 = np.ascontiguousarray(a1, np.int64)
    a2 = np.ascontiguousarray(a2, np.int64)
    out = np.zeros(4, np.int64)
    lib().orc_zorder_map(_p(a1), _p(a2), a1.size, _p(out))
    return out


def zorder_keys(zmap, a1, a2) -> np.ndarray:
    """The z-order keys of the pairs (a1[i], a2[i]): the two coordinates' bits interleaved,
    a1's in the odd positions."""
    m = np.ascontiguousarray(zmap, np.int64)
    a1 = np.ascontiguousarray(a1, np.int64)
    a2 = np.ascontiguousarray(a2, np.int64)
    out = np.zeros(a1.size, np.int64)
    if lib().orc_zorder_keys(_p(m), _p(a1), _p(a2), a1.size, _p(out)) != 0:
        raise ValueError(lib().orc_last_error().decode())
    return out


def zorder_range(zmap, l1, h1, l2, h2):
    """The key range [lo, hi] a box search runs on (lo > hi for an empty box)."""
    m = np.ascontiguousarray(zmap, np.int64)
    r = [np.ascontiguousarray(x, np.int64) for x in (l1, h1, l2, h2)]
    lo = np.zeros(r[0].size, np.int64)
    hi = np.zeros(r[0].size, np.int64)
    lib().orc_zorder_range(_p(m), *[_p(x) for x in r], r[0].size, _p(lo), _p(hi))
    return lo, hi


def merge_or(ids_a, dist_a, ids_b, dist_b):
    """Disjunctive two-attribute queries (the paper's multi-attribute extension,
    approach 1): the results of one index per attribute, each searched with its own
    range, merged per query.  Both lists ascend by distance (-1 / +inf padded); the
    merged list takes the smaller distance first (ties: the smaller id), and an id
    already taken at the same distance (the same object from the other list) is
    skipped.  Returns the first k of the merged list, padded."""
    ids_a, ids_b = np.asarray(ids_a), np.asarray(ids_b)
    dist_a, dist_b = np.asarray(dist_a, np.float32), np.asarray(dist_b, np.float32)
    nq, k = ids_a.shape
    oi = np.full((nq, k), -1, np.int64)
    od = np.full((nq, k), np.inf, np.float32)
    for q in range(nq):
        a = [(float(d), int(i)) for d, i in zip(dist_a[q], ids_a[q]) if i >= 0]
        b = [(float(d), int(i)) for d, i in zip(dist_b[q], ids_b[q]) if i >= 0]
        out = []
        while len(out) < k and (a or b):
            if a and (not b or a[0] <= b[0]):
                d, i = a.pop(0)
            else:
                d, i = b.pop(0)
            if any(dd == d and ii == i for dd, ii in out):
                continue
            out.append((d, i))
        for t, (d, i) in enumerate(out):
            oi[q, t], od[q, t] = i, d
    return oi, od
