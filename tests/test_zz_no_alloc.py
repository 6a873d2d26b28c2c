"""The allocation-free search entry point (unify_search_ex_noalloc), called through
the C ABI, returns what unify_search_ex returns (ids, FP32 distances, strategies
and counters bit for bit) on two calls in a row, the second with fewer queries;
it leaves the device's free memory unchanged and refuses a batch whose scratch
would not fit its static array."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import hsig
from synth import workloads as w


def _p(t):
    return C.c_void_p(t.data_ptr())


def test_noalloc_equals_search_ex(tmp_path):
    import torch

    import paper_2412_02448_amd as u
    assert torch.cuda.is_available()
    dev = torch.device("cuda", 0)
    lib = u.load_library()
    spec = w.scaled(w.SPECS["hybrid10k"], n=4000, nq=100)
    W = w.make(spec, base_seed=5)
    print("[case] noalloc: oracle build n=4000", flush=True)
    ref_ix = hsig.Index.build(W.base, W.attr, W.level_u, spec.S, spec.M, spec.ef_cons, seed=5)
    path = str(tmp_path / "noalloc.uix")
    ref_ix.write(path)
    g = u.Index.load(path, device=0, precision="bf16")
    k, ef = 10, 48
    prm = u._params(m=32, beam_p=2, pre_chunk=256)
    stream = torch.cuda.current_stream(dev).cuda_stream

    def call(fn, nq):
        Q = torch.from_numpy(W.queries[:nq]).to(dev)
        lo = torch.from_numpy(W.l[:nq]).to(dev)
        hi = torch.from_numpy(W.h[:nq]).to(dev)
        ids = torch.full((nq, k), -7, dtype=torch.int64, device=dev)
        dist = torch.zeros((nq, k), dtype=torch.float32, device=dev)
        st = torch.zeros(nq, dtype=torch.int8, device=dev)
        stats = torch.zeros((nq, 8), dtype=torch.int32, device=dev)
        torch.cuda.synchronize()
        rc = fn(g._h, _p(Q), nq, _p(lo), _p(hi), k, ef, None, C.byref(prm), _p(ids), _p(dist), _p(st), _p(stats),
                C.c_void_p(stream))
        assert rc == 0, lib.unify_last_error().decode()
        torch.cuda.synchronize()
        return ids.cpu().numpy(), dist.cpu().numpy(), st.cpu().numpy(), stats.cpu().numpy()

    nq_all = len(W.queries)
    for nq in (nq_all, 37):  # two calls in a row, the second smaller
        print(f"[case] noalloc nq={nq}", flush=True)
        want = call(lib.unify_search_ex, nq)
        free0 = torch.cuda.mem_get_info(dev)[0]
        got = call(lib.unify_search_ex_noalloc, nq)
        assert torch.cuda.mem_get_info(dev)[0] == free0
        assert np.array_equal(got[0], want[0])
        assert np.array_equal(got[1].view(np.uint32), want[1].view(np.uint32))
        assert np.array_equal(got[2], want[2]) and np.array_equal(got[3], want[3])
        # and the oracle's rows (same store, same parameters)
        ref_ix.set_store(hsig.BF16, 4)
        rid, rd = ref_ix.search(W.queries[:nq], W.l[:nq], W.h[:nq], k, ef, m=32, p=2)
        assert np.array_equal(got[0], rid) and np.array_equal(got[1].view(np.uint32), rd.view(np.uint32))
    # a batch whose scratch exceeds the static array is refused before any launch
    big = 1 << 20
    rc = lib.unify_search_ex_noalloc(g._h, C.c_void_p(1), big, C.c_void_p(1), C.c_void_p(1), 10, 16, None, None,
                                     C.c_void_p(1), C.c_void_p(1), None, None, None)
    assert rc == -22 and b"static" in lib.unify_last_error()
    g.close()
