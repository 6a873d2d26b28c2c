"""Range-filtered k-NN search over an HSIG (UNIFY, PVLDB 18(4), 2024) on MI355X.

A thin ctypes binding of ``libunify.so`` (the C ABI declared in
``include/unify.h``).  Every step of a search runs in the library's HIP kernels;
this module only marshals arguments: torch tensors supply device memory and the
current HIP stream.  The library must be built first
(``python -m paper_2412_02448_amd.build_native``); importing without it raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

__all__ = ["Index", "UnifyError", "AUTO", "PRE", "HYBRID", "POST", "FP32", "BF16", "FP8E4M3",
           "validate_index_file", "library_path", "load_library"]

AUTO, PRE, HYBRID, POST = 0, 1, 2, 3
FLAG_TIMING = 1
FLAG_SELECT_S1 = 2
FLAG_PRE_WAVE_SCAN = 4
FLAG_SERIAL_PHASES = 8
FP32, BF16, FP8E4M3 = 0, 1, 2
_PRECISIONS = {"fp32": FP32, "bf16": BF16, "fp8": FP8E4M3, "fp8e4m3": FP8E4M3}

_HERE = os.path.dirname(os.path.abspath(__file__))


def library_path() -> str:
    return os.path.join(_HERE, "libunify.so")


class UnifyError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"unify error {code}: {msg}")
        self.code = code


class _Params(C.Structure):
    _fields_ = [("m", C.c_int32), ("beam_p", C.c_int32), ("rerank_mult", C.c_int32),
                ("tau_a_frac", C.c_double), ("tau_b_frac", C.c_double), ("flags", C.c_uint32),
                ("cand_cap", C.c_int32), ("visit_cap", C.c_int32), ("pre_chunk", C.c_int32),
                ("waves_per_query", C.c_int32), ("heavy_queries", C.c_int32)]


class _ZMap(C.Structure):
    _fields_ = [("base1", C.c_int64), ("base2", C.c_int64), ("shift1", C.c_int32), ("shift2", C.c_int32)]


def _zmap(zmap) -> _ZMap:
    b1, s1, b2, s2 = (int(x) for x in zmap)
    return _ZMap(base1=b1, base2=b2, shift1=s1, shift2=s2)


def zorder_map(a1, a2) -> np.ndarray:
    """The z-order key map of two attributes (the multi-attribute extension, approach 2), as
    [base1, shift1, base2, shift2]: each attribute's smallest value and the shift that puts its
    largest value in the upper half of a 2^31-cell axis (negative: a left shift)."""
    a1 = np.ascontiguousarray(a1, np.int64)
    a2 = np.ascontiguousarray(a2, np.int64)
    if a1.shape != a2.shape or a1.ndim != 1:
        raise ValueError("a1 and a2 are [n] arrays")
    m = _ZMap()
    _check(load_library().unify_zorder_map(a1.ctypes.data, a2.ctypes.data, a1.size, C.byref(m)))
    return np.array([m.base1, m.shift1, m.base2, m.shift2], np.int64)


def zorder_keys(zmap, a1, a2) -> np.ndarray:
    """The z-order keys of the pairs (a1[i], a2[i]) under zmap: the attribute to build the index on."""
    a1 = np.ascontiguousarray(a1, np.int64)
    a2 = np.ascontiguousarray(a2, np.int64)
    if a1.shape != a2.shape or a1.ndim != 1:
        raise ValueError("a1 and a2 are [n] arrays")
    out = np.empty(a1.size, np.int64)
    m = _zmap(zmap)
    _check(load_library().unify_zorder_keys(C.byref(m), a1.ctypes.data, a2.ctypes.data, a1.size, out.ctypes.data))
    return out


def _params(m=0, beam_p=0, rerank_mult=0, tau_a=0.0, tau_b=0.0, flags=0, cand_cap=0, visit_cap=0,
            pre_chunk=0, waves_per_query=0, heavy_queries=0) -> _Params:
    return _Params(m=m, beam_p=beam_p, rerank_mult=rerank_mult, tau_a_frac=tau_a, tau_b_frac=tau_b, flags=flags,
                   cand_cap=cand_cap, visit_cap=visit_cap, pre_chunk=pre_chunk, waves_per_query=waves_per_query,
                   heavy_queries=heavy_queries)


_lib = None

# name -> (restype, argtypes) of every symbol include/unify.h declares
_P, _I64, _I32, _S = C.c_void_p, C.c_int64, C.c_int32, C.c_char_p
SIGNATURES = {
    "unify_load_index": (_I32, [_S, _I32, _I32, _P]),
    "unify_build_index": (_I32, [_P, _P, _P, _I64, _I32, _I32, _I32, _I32, _I32, _I32, _P]),
    "unify_validate_index_file": (_I32, [_S, _P, _P, _P, _P]),
    "unify_save_index": (_I32, [_P, _S]),
    "unify_index_info": (_I32, [_P, _P, _P, _P, _P, _P]),
    "unify_search": (_I32, [_P, _P, _I64, _P, _P, _I32, _I32, _P, _P, _P, _P, _P, _P]),
    "unify_search_ex": (_I32, [_P, _P, _I64, _P, _P, _I32, _I32, _P, _P, _P, _P, _P, _P, _P]),
    "unify_search_ex_noalloc": (_I32, [_P, _P, _I64, _P, _P, _I32, _I32, _P, _P, _P, _P, _P, _P, _P]),
    "unify_last_timing": (_I32, [_P, _P, _P, _P]),
    "unify_last_timing_ex": (_I32, [_P, _P, _I32]),
    "unify_copy_store": (_I32, [_P, _I32, _P, _P, _P, _P]),
    "unify_set_precision": (_I32, [_P, _I32]),
    "unify_insert": (_I32, [_P, _P, _P, _P, _I64]),
    "unify_set_attr2": (_I32, [_P, _P, _I64]),
    "unify_merge_or": (_I32, [_P, _P, _P, _P, _I64, _I32, _P, _P, _P]),
    "unify_search_multi": (_I32, [_P, _P, _I64, _P, _P, _P, _P, _I32, _I32, _P, _P, _P, _P, _P, _P, _P]),
    "unify_zorder_map": (_I32, [_P, _P, _I64, _P]),
    "unify_zorder_keys": (_I32, [_P, _P, _P, _I64, _P]),
    "unify_set_zorder": (_I32, [_P, _P, _P, _P, _I64]),
    "unify_search_box": (_I32, [_P, _P, _I64, _P, _P, _P, _P, _I32, _I32, _P, _P, _P, _P, _P, _P, _P]),
    "unify_batch_create": (_I32, [_P, _P, _I64, _P, _P, _I32, _I32, _P, _P, _P, _P, _P, _P, _P]),
    "unify_server_create": (_I32, [_P, _P, _P]),
    "unify_server_submit": (_I32, [_P, _I64, _P, _P, _P, _P, _P, _P]),
    "unify_server_wait": (_I32, [_P, _I64, _P, _P, _P, _P, C.c_double]),
    "unify_prune": (_I32, [_P, _I64, _I32, _P, _P, _I64, _I32, _I32, _P, _P]),
    "unify_server_limits": (_I32, [_P, _P, _P, _P]),
    "unify_server_stats": (_I32, [_P, _P, _P, _P]),
    "unify_server_free": (_I32, [_P]),
    "unify_batch_run": (_I32, [_P, _P]),
    "unify_batch_free": (_I32, [_P]),
    "unify_free_index": (_I32, [_P]),
    "unify_last_error": (_S, []),
}


def load_library():
    global _lib
    if _lib is None:
        # torch ships its own HIP runtime; it must be the one in the process before
        # libunify binds to libamdhip64.so.7, or two runtimes would share the GPU.
        import torch  # noqa: F401
        path = library_path()
        if not os.path.exists(path):
            raise ImportError(f"{path} is missing: run `python -m paper_2412_02448_amd.build_native`")
        lib = C.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(rc: int):
    if rc != 0:
        raise UnifyError(rc, load_library().unify_last_error().decode(errors="replace"))


def validate_index_file(path: str) -> dict:
    """Host-only check of an index file; returns its sizes."""
    n, d, S, M = C.c_int64(), C.c_int32(), C.c_int32(), C.c_int32()
    _check(load_library().unify_validate_index_file(path.encode(), C.byref(n), C.byref(d), C.byref(S),
                                                    C.byref(M)))
    return {"n": n.value, "d": d.value, "S": S.value, "M": M.value}


def merge_or(a, b, stream=None):
    """Disjunctive query results: a and b are (ids, dist) of the same queries searched on two
    indexes over the same objects (one per attribute, each with its range); returns the k
    nearest distinct objects of the two lists per query, as new device tensors."""
    import torch
    ia, da = a[0], a[1]
    ib, db = b[0], b[1]
    if ia.shape != ib.shape or da.shape != ia.shape or db.shape != ia.shape or ia.dim() != 2:
        raise ValueError("both results must be [nq, k] ids and distances")
    for t, dt in ((ia, torch.int64), (ib, torch.int64), (da, torch.float32), (db, torch.float32)):
        if t.dtype != dt or not t.is_contiguous() or t.device != ia.device:
            raise ValueError("ids int64 and dist float32, contiguous, on one device")
    oi, od = torch.empty_like(ia), torch.empty_like(da)
    s = stream if stream is not None else torch.cuda.current_stream(ia.device)
    _check(load_library().unify_merge_or(_ptr(ia), _ptr(da), _ptr(ib), _ptr(db), ia.shape[0], ia.shape[1],
                                         _ptr(oi), _ptr(od), s.cuda_stream))
    if s != torch.cuda.current_stream(ia.device):
        for t in (ia, da, ib, db, oi, od):
            t.record_stream(s)  # in use on s until it passes this point
    return oi, od


def prune(vectors, owners, cand, M: int):
    """The builder's Prune on the GPU: vectors cuda float32 [n, d]; owners cuda int32 [t];
    cand cuda int32 [t, c] candidate ids (-1: none).  Returns cuda int32 [t, M], the kept ids
    of each task in selection order, -1 padded."""
    import torch
    if vectors.dtype != torch.float32 or vectors.dim() != 2 or not vectors.is_contiguous():
        raise ValueError("vectors must be a contiguous float32 [n, d] tensor")
    dev = vectors.device
    for t_, nd in ((owners, 1), (cand, 2)):
        if t_.dtype != torch.int32 or t_.dim() != nd or not t_.is_contiguous() or t_.device != dev:
            raise ValueError("owners int32 [t] and cand int32 [t, c], contiguous, on the vectors' device")
    t = owners.shape[0]
    if cand.shape[0] != t:
        raise ValueError("one candidate row per owner")
    out = torch.empty((t, M), dtype=torch.int32, device=dev)
    s = torch.cuda.current_stream(dev)
    _check(load_library().unify_prune(_ptr(vectors), vectors.shape[0], vectors.shape[1], _ptr(owners), _ptr(cand),
                                      t, cand.shape[1] if cand.dim() == 2 else 0, M, _ptr(out), s.cuda_stream))
    return out


def _ptr(t) -> int:
    return t.data_ptr() if t is not None else None


class Index:
    """An HSIG resident on one GPU."""

    def __init__(self, handle: int, device: int):
        self._h = C.c_void_p(handle)
        self.device = device
        n, d, S, M, L = C.c_int64(), C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        _check(load_library().unify_index_info(self._h, C.byref(n), C.byref(d), C.byref(S), C.byref(M),
                                               C.byref(L)))
        self.n, self.d, self.S, self.M, self.levels = n.value, d.value, S.value, M.value, L.value
        self.precision = FP32

    @staticmethod
    def _prec(precision) -> int:
        return _PRECISIONS[precision] if isinstance(precision, str) else int(precision)

    @classmethod
    def load(cls, path: str, device: int = 0, precision="fp32") -> "Index":
        h = C.c_void_p()
        prec = cls._prec(precision)
        _check(load_library().unify_load_index(path.encode(), device, prec, C.byref(h)))
        ix = cls(h.value, device)
        ix.precision = prec
        return ix

    @classmethod
    def build(cls, vectors: np.ndarray, attr: np.ndarray, level_u: np.ndarray, S: int, M: int,
              ef_cons: int, device: int = 0, precision="fp32") -> "Index":
        X = np.ascontiguousarray(vectors, np.float32)
        a = np.ascontiguousarray(attr, np.int64)
        u = np.ascontiguousarray(level_u, np.float64)
        h = C.c_void_p()
        _check(load_library().unify_build_index(X.ctypes.data, a.ctypes.data, u.ctypes.data, X.shape[0],
                                                X.shape[1], S, M, ef_cons, device, cls._prec(precision),
                                                C.byref(h)))
        ix = cls(h.value, device)
        ix.precision = cls._prec(precision)
        return ix

    def insert(self, vectors: np.ndarray, attr: np.ndarray, level_u: np.ndarray) -> None:
        """Inserts more objects (Alg. 6) into the resident index; they take the next external
        ids.  Searches enqueued afterwards see them; Batch objects must be created again."""
        X = np.ascontiguousarray(vectors, np.float32)
        a = np.ascontiguousarray(attr, np.int64)
        u = np.ascontiguousarray(level_u, np.float64)
        if X.ndim != 2 or X.shape[1] != self.d or a.shape != (X.shape[0],) or u.shape != (X.shape[0],):
            raise ValueError(f"vectors must be [m, {self.d}] with attr and level_u of length m")
        _check(load_library().unify_insert(self._h, X.ctypes.data, a.ctypes.data, u.ctypes.data, X.shape[0]))
        n, L = C.c_int64(), C.c_int32()
        _check(load_library().unify_index_info(self._h, C.byref(n), None, None, None, C.byref(L)))
        self.n, self.levels = n.value, L.value

    def set_attr2(self, attr2: np.ndarray) -> None:
        """Second attribute of every object, indexed by external id, for conjunctive queries
        (search with l2, h2).  Dropped by insert()."""
        a = np.ascontiguousarray(attr2, np.int64)
        _check(load_library().unify_set_attr2(self._h, a.ctypes.data, a.size))

    def set_zorder(self, zmap, a1, a2) -> None:
        """Both attributes of an index built on zorder_keys(zmap, a1, a2), indexed by external id,
        for box searches (search with box=True).  Dropped by insert()."""
        a1 = np.ascontiguousarray(a1, np.int64)
        a2 = np.ascontiguousarray(a2, np.int64)
        if a1.shape != a2.shape:
            raise ValueError("a1 and a2 differ in size")
        m = _zmap(zmap)
        _check(load_library().unify_set_zorder(self._h, C.byref(m), a1.ctypes.data, a2.ctypes.data, a1.size))

    def set_precision(self, precision) -> None:
        """Store later searches rank by ("fp32", "bf16", "fp8"); builds the copy on first use."""
        prec = self._prec(precision)
        _check(load_library().unify_set_precision(self._h, prec))
        self.precision = prec

    def copy_store(self, precision=None, stream=None):
        """A resident BF16 / FP8 copy of the vectors in internal-id order, as device tensors:
        (codes [n, d] int16 or uint8, scales [n] float32 or None, eps [n] float32)."""
        import torch
        dev = torch.device("cuda", self.device)
        prec = self.precision if precision is None else self._prec(precision)
        if prec == BF16:
            codes, sc = torch.empty((self.n, self.d), dtype=torch.int16, device=dev), None
        elif prec == FP8E4M3:
            codes = torch.empty((self.n, self.d), dtype=torch.uint8, device=dev)
            sc = torch.empty(self.n, dtype=torch.float32, device=dev)
        else:
            raise UnifyError(-22, "the index has no low-precision store")
        eps = torch.empty(self.n, dtype=torch.float32, device=dev)
        s = stream if stream is not None else torch.cuda.current_stream(dev)
        _check(load_library().unify_copy_store(self._h, prec, _ptr(codes), _ptr(sc), _ptr(eps), s.cuda_stream))
        if s != torch.cuda.current_stream(dev):
            for t in (codes, sc, eps):
                if t is not None:
                    t.record_stream(s)  # in use on s until it passes this point
        return codes, sc, eps

    def save(self, path: str) -> None:
        _check(load_library().unify_save_index(self._h, path.encode()))

    def close(self) -> None:
        if getattr(self, "_h", None) and self._h.value:
            load_library().unify_free_index(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def last_timing(self):
        """(plan_ms, search_ms, rerun_ms) of the last search issued with timing=True (waits for it)."""
        a, b, c = C.c_float(), C.c_float(), C.c_float()
        _check(load_library().unify_last_timing(self._h, C.byref(a), C.byref(b), C.byref(c)))
        return a.value, b.value, c.value

    def last_timing_phases(self) -> dict:
        """Per-phase milliseconds of the last search issued with timing=True (waits for it)."""
        t = (C.c_float * 7)()
        _check(load_library().unify_last_timing_ex(self._h, t, 7))
        names = ("plan", "tile_setup", "tile_scan", "tile_final", "search", "merge", "rerun")
        return {nm: float(v) for nm, v in zip(names, t)}

    def search(self, queries, l, h, k: int, ef: int, strategy=None, m: int = 0, beam_p: int = 1,
               rerank_mult: int = 0, tau_a: float = 0.0, tau_b: float = 0.0, stats: bool = False,
               out=None, stream=None, timing: bool = False, cand_cap: int = 0, visit_cap: int = 0, pre_chunk: int = 0,
               select_s1: bool = False, l2=None, h2=None, wave_scan: bool = False, waves_per_query: int = 0,
               heavy_queries: int = 0, serial_phases: bool = False, box: bool = False):
        """Enqueues a search on the current stream (or `stream`) and returns torch tensors.

        queries: cuda float32 [nq, d]; l, h: cuda int64 [nq] (inclusive); strategy: None (auto),
        an int for every query, or a cuda int8 [nq] tensor.  select_s1: hybrid neighbour selection S1
        (the m entries of the active chunks nearest the expanded object) instead of S2 (the first
        ceil(m / S') of each chunk).  l2, h2: cuda int64 [nq] inclusive ranges on the second
        attribute (conjunctive query; set_attr2 first).  wave_scan: pre-filter scans per
        wavefront instead of the shared matrix-core scan (same results).  serial_phases: the
        matrix-core scan before the graph search rather than beside it (same results; for
        timing each phase alone).  box: a box search on a z-order index (set_zorder first): l, h
        range over the first attribute and l2, h2 over the second.  Returns (ids, dist,
        strategy[, stats]).
        """
        import torch
        dev = torch.device("cuda", self.device)
        nq = queries.shape[0]
        if queries.dtype != torch.float32 or queries.device != dev or not queries.is_contiguous():
            raise ValueError("queries must be a contiguous float32 tensor on the index's device")
        if queries.dim() != 2 or queries.shape[1] != self.d:
            raise ValueError(f"queries must be [nq, {self.d}]")
        for t in (l, h):
            if t.dtype != torch.int64 or t.device != dev or not t.is_contiguous() or t.shape != (nq,):
                raise ValueError("l and h must be contiguous int64 [nq] tensors on the index's device")
        st = None
        if strategy is not None:
            st = strategy if isinstance(strategy, torch.Tensor) else torch.full((nq,), int(strategy),
                                                                                 dtype=torch.int8, device=dev)
            if st.dtype != torch.int8 or st.device != dev or st.shape != (nq,):
                raise ValueError("strategy must be an int8 [nq] tensor on the index's device")
        if out is None:
            ids = torch.empty((nq, k), dtype=torch.int64, device=dev)
            dist = torch.empty((nq, k), dtype=torch.float32, device=dev)
            ost = torch.empty((nq,), dtype=torch.int8, device=dev)
            sts = torch.empty((nq, 8), dtype=torch.int32, device=dev) if stats else None
        else:
            ids, dist, ost, sts = out
        flags = ((FLAG_TIMING if timing else 0) | (FLAG_SELECT_S1 if select_s1 else 0)
                 | (FLAG_PRE_WAVE_SCAN if wave_scan else 0) | (FLAG_SERIAL_PHASES if serial_phases else 0))
        prm = _params(m, beam_p, rerank_mult, tau_a, tau_b, flags, cand_cap, visit_cap, pre_chunk, waves_per_query,
                      heavy_queries)
        s = stream if stream is not None else torch.cuda.current_stream(dev)
        lib = load_library()
        if (l2 is None) != (h2 is None) or (box and l2 is None):
            raise ValueError("l2 and h2 go together (and a box search needs them)")
        if l2 is not None:
            for t in (l2, h2):
                if t.dtype != torch.int64 or t.device != dev or not t.is_contiguous() or t.shape != (nq,):
                    raise ValueError("l2 and h2 must be contiguous int64 [nq] tensors on the index's device")
            fn = lib.unify_search_box if box else lib.unify_search_multi
            rc = fn(self._h, _ptr(queries), nq, _ptr(l), _ptr(h), _ptr(l2), _ptr(h2), k, ef, _ptr(st), C.byref(prm),
                    _ptr(ids), _ptr(dist), _ptr(ost), _ptr(sts), s.cuda_stream)
        elif stats:
            rc = lib.unify_search_ex(self._h, _ptr(queries), nq, _ptr(l), _ptr(h), k, ef, _ptr(st), C.byref(prm),
                                     _ptr(ids), _ptr(dist), _ptr(ost), _ptr(sts), s.cuda_stream)
        else:
            rc = lib.unify_search(self._h, _ptr(queries), nq, _ptr(l), _ptr(h), k, ef, _ptr(st), C.byref(prm),
                                  _ptr(ids), _ptr(dist), _ptr(ost), s.cuda_stream)
        _check(rc)
        if s != torch.cuda.current_stream(dev):
            # the kernels use these tensors on `s`: the caching allocator must not hand their
            # memory out again before that stream has passed this point
            for t in (queries, l, h, st, ids, dist, ost, sts, l2, h2):
                if t is not None:
                    t.record_stream(s)
        return (ids, dist, ost, sts) if stats else (ids, dist, ost)


class Batch:
    """A fixed-size batch whose whole search is captured once as a HIP graph and
    replayed by run().  The query tensors passed in are read at every replay
    (write new queries into them in place); results land in .ids, .dist,
    .strategy_run and .stats (when stats=True).  Keyword arguments are those of
    Index.search."""

    def __init__(self, index: Index, queries, l, h, k: int, ef: int, strategy=None, stats: bool = False,
                 m: int = 0, beam_p: int = 1, rerank_mult: int = 0, tau_a: float = 0.0, tau_b: float = 0.0,
                 cand_cap: int = 0, visit_cap: int = 0, pre_chunk: int = 0, select_s1: bool = False,
                 wave_scan: bool = False, waves_per_query: int = 0, heavy_queries: int = 0,
                 serial_phases: bool = False):
        import torch
        dev = torch.device("cuda", index.device)
        nq = queries.shape[0]
        if queries.dtype != torch.float32 or queries.device != dev or not queries.is_contiguous() \
                or queries.shape != (nq, index.d):
            raise ValueError("queries must be a contiguous float32 [nq, d] tensor on the index's device")
        for t in (l, h):
            if t.dtype != torch.int64 or t.device != dev or not t.is_contiguous() or t.shape != (nq,):
                raise ValueError("l and h must be contiguous int64 [nq] tensors on the index's device")
        if strategy is not None and not isinstance(strategy, torch.Tensor):
            strategy = torch.full((nq,), int(strategy), dtype=torch.int8, device=dev)
        self.index, self.queries, self.l, self.h, self.strategy = index, queries, l, h, strategy
        self.ids = torch.empty((nq, k), dtype=torch.int64, device=dev)
        self.dist = torch.empty((nq, k), dtype=torch.float32, device=dev)
        self.strategy_run = torch.empty((nq,), dtype=torch.int8, device=dev)
        self.stats = torch.empty((nq, 8), dtype=torch.int32, device=dev) if stats else None
        flags = ((FLAG_SELECT_S1 if select_s1 else 0) | (FLAG_PRE_WAVE_SCAN if wave_scan else 0)
                 | (FLAG_SERIAL_PHASES if serial_phases else 0))
        prm = _params(m, beam_p, rerank_mult, tau_a, tau_b, flags, cand_cap, visit_cap, pre_chunk, waves_per_query,
                      heavy_queries)
        torch.cuda.synchronize(dev)  # the tensors above exist before the capture reads their addresses
        self._b = C.c_void_p()
        _check(load_library().unify_batch_create(index._h, _ptr(queries), nq, _ptr(l), _ptr(h), k, ef,
                                                 _ptr(strategy), C.byref(prm), _ptr(self.ids), _ptr(self.dist),
                                                 _ptr(self.strategy_run), _ptr(self.stats), C.byref(self._b)))

    def run(self, stream=None) -> None:
        import torch
        s = stream if stream is not None else torch.cuda.current_stream(torch.device("cuda", self.index.device))
        _check(load_library().unify_batch_run(self._b, s.cuda_stream))

    def close(self) -> None:
        if getattr(self, "_b", None) and self._b.value:
            load_library().unify_batch_free(self._b)
            self._b = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _ServerConfig(C.Structure):
    _fields_ = [("k", C.c_int32), ("ef", C.c_int32), ("max_batch", C.c_int32), ("inflight", C.c_int32),
                ("max_wait_s", C.c_double), ("params", _Params), ("mem_budget", C.c_int64)]


class Server:
    """Continuous-batching server over a resident index (the library's worker
    thread admits arrived requests into batches whenever one of `inflight`
    slots is free; each slot has its own visited memory, so slots overlap on the
    device; the batch size and visited rows fit mem_budget bytes, 0 = half the
    free device memory).  Requests come from host arrays."""

    def __init__(self, index: Index, k: int, ef: int, max_batch: int = 4096, inflight: int = 2,
                 max_wait_s: float = 0.0, m: int = 0, beam_p: int = 1, rerank_mult: int = 0, tau_a: float = 0.0,
                 tau_b: float = 0.0, cand_cap: int = 0, visit_cap: int = 0, pre_chunk: int = 0,
                 select_s1: bool = False, waves_per_query: int = 0, heavy_queries: int = 0, mem_budget: int = 0):
        self.index, self.k = index, k
        flags = FLAG_SELECT_S1 if select_s1 else 0
        cfg = _ServerConfig(k, ef, max_batch, inflight, max_wait_s,
                            _params(m, beam_p, rerank_mult, tau_a, tau_b, flags, cand_cap, visit_cap, pre_chunk,
                                    waves_per_query, heavy_queries), int(mem_budget))
        self._s = C.c_void_p()
        _check(load_library().unify_server_create(index._h, C.byref(cfg), C.byref(self._s)))

    def submit(self, queries, l, h, strategy=None, arrive_s=None) -> np.ndarray:
        """Submits len(l) requests; arrive_s: seconds from now at which each arrives (None: now).
        Returns their tickets."""
        q = np.ascontiguousarray(queries, np.float32)
        lo = np.ascontiguousarray(l, np.int64)
        hi = np.ascontiguousarray(h, np.int64)
        n = lo.shape[0]
        if q.shape != (n, self.index.d) or hi.shape != (n,):
            raise ValueError("queries must be [n, d] and l, h [n]")
        st = None if strategy is None else np.ascontiguousarray(strategy, np.int8)
        ar = None if arrive_s is None else np.ascontiguousarray(arrive_s, np.float64)
        t = np.zeros(n, np.int64)
        p = lambda a: None if a is None else a.ctypes.data  # noqa: E731
        _check(load_library().unify_server_submit(self._s, n, p(q), p(lo), p(hi), p(st), p(ar), p(t)))
        return t

    def wait(self, tickets, timeout_s: float = 0.0):
        """(ids [n, k], dist [n, k], latency_s [n]) of the given tickets, waiting for them."""
        t = np.ascontiguousarray(tickets, np.int64)
        n = t.shape[0]
        ids = np.zeros((n, self.k), np.int64)
        dist = np.zeros((n, self.k), np.float32)
        lat = np.zeros(n, np.float64)
        _check(load_library().unify_server_wait(self._s, n, t.ctypes.data, ids.ctypes.data, dist.ctypes.data,
                                                lat.ctypes.data, float(timeout_s)))
        return ids, dist, lat

    def limits(self):
        """(requests per batch, visited rows per slot, device bytes of the slots) the budget admitted."""
        b, r, m = C.c_int64(), C.c_int64(), C.c_int64()
        _check(load_library().unify_server_limits(self._s, C.byref(b), C.byref(r), C.byref(m)))
        return b.value, r.value, m.value

    def stats(self):
        """(requests completed, batches launched, seconds with a batch in flight)."""
        c, b, s = C.c_int64(), C.c_int64(), C.c_double()
        _check(load_library().unify_server_stats(self._s, C.byref(c), C.byref(b), C.byref(s)))
        return c.value, b.value, s.value

    def close(self) -> None:
        if getattr(self, "_s", None) and self._s.value:
            load_library().unify_server_free(self._s)
            self._s = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

