"""The C-ABI library loads and exports every entry point its header declares; the
host-only index-file check accepts the oracle's files and rejects damaged ones."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "unify.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(unify_[a-z_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported_and_bound():
    import paper_2412_02448_amd as u
    lib = u.load_library()
    names = _declared()
    assert len(names) >= 9
    for n in names:
        assert hasattr(lib, n), n
        assert n in u.SIGNATURES, n


def test_validate_index_file(small_index, tmp_path):
    import paper_2412_02448_amd as u
    p = str(tmp_path / "ix.bin")
    small_index.write(p)
    info = u.validate_index_file(p)
    assert info == {"n": small_index.n, "d": small_index.d, "S": small_index.S, "M": small_index.M0}
    raw = open(p, "rb").read()
    bad = bytearray(raw)
    bad[300] ^= 1
    open(p, "wb").write(bytes(bad))
    with pytest.raises(u.UnifyError) as e:
        u.validate_index_file(p)
    assert e.value.code == -74
    open(p, "wb").write(raw[:1000])
    with pytest.raises(u.UnifyError) as e:
        u.validate_index_file(p)
    assert e.value.code == -74
    with pytest.raises(u.UnifyError) as e:
        u.validate_index_file(str(tmp_path / "missing.bin"))
    assert e.value.code == -5


def test_validate_rejects_out_of_range_edge(tmp_path):
    # A file whose checksum is right but whose adjacency names a non-existent
    # object is rejected by the table check (the kernels trust loaded tables).
    import zlib

    import paper_2412_02448_amd as u
    from oracle import hsig
    rng = np.random.default_rng(0)
    X = rng.standard_normal((64, 8)).astype(np.float32)
    ix = hsig.Index.build(X, np.arange(64), 1.0 - rng.random(64), 2, 4, 8)
    p = str(tmp_path / "ix.bin")
    ix.write(p)
    raw = bytearray(open(p, "rb").read())
    # adj0 section: after header and the per-node tables; find it from the layout
    n, d, S, M0 = 64, 8, 2, 4
    off = 256
    def sec(off, nbytes):
        off = (off + 63) // 64 * 64
        return off, off + nbytes
    for nbytes in (8 * n, 8 * n, 8 * (S + 1), 4 * S, 4 * S, n, 4 * n, 4 * n * d):
        _, off = sec(off, nbytes)
    a0, _ = sec(off, 4 * n * S * M0)
    raw[a0:a0 + 4] = np.int32(10 ** 6).tobytes()
    body = bytes(raw[:-4])
    raw[-4:] = np.uint32(zlib.crc32(body)).tobytes()
    open(p, "wb").write(bytes(raw))
    with pytest.raises(u.UnifyError) as e:
        u.validate_index_file(p)
    assert e.value.code == -74 and "adjacency" in str(e.value)


def test_entry_points_reject_bad_arguments_on_the_host():
    """Argument checks that run before any device call: every entry point answers a
    null handle or an out-of-range size with UNIFY_EINVAL (-22) and a message, and the
    free functions accept null."""
    import ctypes as C

    import paper_2412_02448_amd as u
    lib = u.load_library()
    EINVAL = -22
    null = None
    assert lib.unify_search(null, null, 1, null, null, 10, 10, null, null, null, null, null, null) == EINVAL
    assert lib.unify_search_ex(null, null, 1, null, null, 10, 10, null, null, null, null, null, null, null) == EINVAL
    assert lib.unify_search_multi(null, null, 1, null, null, null, null, 10, 10, null, null, null, null, null, null,
                                  null) == EINVAL
    assert lib.unify_search_box(null, null, 1, null, null, null, null, 10, 10, null, null, null, null, null, null,
                                null) == EINVAL
    assert lib.unify_set_zorder(null, null, null, null, 5) == EINVAL
    assert lib.unify_zorder_map(null, null, 5, null) == EINVAL
    assert lib.unify_zorder_keys(null, null, null, 5, null) == EINVAL
    assert lib.unify_insert(null, null, null, null, 5) == EINVAL
    assert lib.unify_set_attr2(null, null, 5) == EINVAL
    assert lib.unify_set_precision(null, 1) == EINVAL
    assert lib.unify_index_info(null, null, null, null, null, null) == EINVAL
    assert lib.unify_save_index(null, b"/nonexistent") == EINVAL
    assert lib.unify_batch_run(null, null) == EINVAL
    assert lib.unify_server_create(null, null, null) == EINVAL
    assert lib.unify_server_submit(null, 1, null, null, null, null, null, null) == EINVAL
    assert lib.unify_server_wait(null, 1, null, null, null, null, 1.0) == EINVAL
    assert lib.unify_server_stats(null, null, null, null) == EINVAL
    assert lib.unify_server_limits(null, null, null, null) == EINVAL
    # the merge checks its sizes before launching anything
    buf = (C.c_int64 * 4)()
    assert lib.unify_merge_or(buf, buf, buf, buf, 1, 0, buf, buf, null) == EINVAL
    assert lib.unify_merge_or(buf, buf, buf, buf, -1, 2, buf, buf, null) == EINVAL
    assert lib.unify_merge_or(null, null, null, null, 0, 2, null, null, null) == 0  # nothing to merge
    assert lib.unify_last_error()  # a message is left
    for free in (lib.unify_free_index, lib.unify_batch_free, lib.unify_server_free):
        assert free(null) == 0


def test_params_struct_matches_header():
    """The binding's parameter struct has the header's fields in the header's order, and
    the search's own parameters (m, beam width, rerank depth, the two strategy thresholds,
    flags) come first, so a caller compiled against that six-field prefix keeps working."""
    import ctypes as C

    import paper_2412_02448_amd as u
    src = open(os.path.join(ROOT, "include", "unify.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    body = re.search(r"typedef struct \{(.*?)\} unify_params;", src, flags=re.S).group(1)
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        typ, names = decl.split(None, 1)
        fields += [(n.strip(), typ) for n in names.split(",")]
    ctype = {"int32_t": C.c_int32, "uint32_t": C.c_uint32, "double": C.c_double}
    assert [(n, ctype[t]) for n, t in fields] == list(u._Params._fields_)
    assert [n for n, _ in fields[:6]] == ["m", "beam_p", "rerank_mult", "tau_a_frac", "tau_b_frac", "flags"]
    assert u._Params.tau_a_frac.offset == 16 and u._Params.flags.offset == 32


def test_server_config_struct_matches_header():
    """The binding's server configuration has the header's fields in its order."""
    import ctypes as C

    import paper_2412_02448_amd as u
    src = open(os.path.join(ROOT, "include", "unify.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    body = re.search(r"typedef struct \{([^{}]*?)\} unify_server_config;", src, flags=re.S).group(1)
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        typ, names = decl.split(None, 1)
        fields += [(n.strip(), typ) for n in names.split(",")]
    ctype = {"int32_t": C.c_int32, "int64_t": C.c_int64, "double": C.c_double, "unify_params": u._Params}
    assert [(n, ctype[t]) for n, t in fields] == list(u._ServerConfig._fields_)


@pytest.mark.parametrize("kind", ["narrow", "wide", "full", "constant"])
def test_zorder_map_and_keys_equal_oracle(kind):
    # the library's host-side z-order map and keys (mask-spread interleave) against the
    # oracle's bit-by-bit ones, integer for integer
    import paper_2412_02448_amd as u
    from oracle import hsig
    rng = np.random.default_rng({"narrow": 1, "wide": 2, "full": 3, "constant": 4}[kind])
    n = 5000
    if kind == "narrow":
        a1 = rng.integers(0, 1000, n, dtype=np.int64)
        a2 = rng.integers(-50, 50, n, dtype=np.int64)
    elif kind == "wide":
        a1 = rng.integers(-(1 << 50), 1 << 50, n, dtype=np.int64)
        a2 = rng.integers(0, 1 << 33, n, dtype=np.int64)
    elif kind == "full":
        a1 = rng.integers(-(1 << 63), (1 << 63) - 1, n, dtype=np.int64)
        a2 = rng.integers(-(1 << 63), (1 << 63) - 1, n, dtype=np.int64)
    else:
        a1 = np.full(n, 7, np.int64)
        a2 = rng.integers(0, 2, n, dtype=np.int64)
    m = u.zorder_map(a1, a2)
    assert m.tolist() == hsig.zorder_map(a1, a2).tolist()
    # keys of the objects and of query bounds around and beyond them
    b1 = np.concatenate([a1, a1 - 1, a1 + 1, [-(1 << 63), (1 << 63) - 1]])
    b2 = np.concatenate([a2, a2 + 3, a2 - 3, [(1 << 63) - 1, -(1 << 63)]])
    assert np.array_equal(u.zorder_keys(m, b1, b2), hsig.zorder_keys(m, b1, b2))


def test_zorder_bad_map():
    import paper_2412_02448_amd as u
    with pytest.raises(u.UnifyError):
        u.zorder_keys([0, -31, 0, 0], np.zeros(3, np.int64), np.zeros(3, np.int64))
    with pytest.raises(u.UnifyError):
        u.zorder_keys([0, 0, 0, 64], np.zeros(3, np.int64), np.zeros(3, np.int64))
