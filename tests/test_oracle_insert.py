"""Pins of incremental insertion in the reference build (Alg. 6 HSIGInsert; the
paper's incremental-construction objective and its insertion experiment).

HSIG is built by inserting objects one at a time, so inserting more objects into
an existing index must leave exactly the index a single build over all of them
produces when that build uses the same segment boundaries (those of the objects
present at creation).  Searches on the grown index are then checked against the
exact answer over all objects.
"""
import numpy as np
import pytest

from oracle import exact, hsig
from synth import workloads as w


def _tables(ix):
    t = {"attr": ix.attr_sorted(), "ext": ix.ext_ids(), "level": ix.levels()}
    ss, en, ml = ix.segments()
    t.update(seg_start=ss, seg_entry=en, seg_maxlevel=ml)
    for l in range(ix.L + 1):
        adj, gl = ix.layer(l)
        t[f"adj{l}"], t[f"glist{l}"] = adj, gl
    return t


@pytest.fixture(scope="module")
def parts():
    spec = w.scaled(w.SPECS["hybrid10k"], n=1500, nq=20)
    W = w.make(spec, base_seed=21)
    return W, spec


@pytest.mark.parametrize("splits", [(600,), (600, 1000), (1499,)])
def test_insert_equals_build_with_same_boundaries(parts, splits):
    W, s = parts
    n = len(W.attr)
    n0 = splits[0]
    whole = hsig.Index.build(W.base, W.attr, W.level_u, s.S, s.M, s.ef_cons, seed=3, bnd_n=n0)
    grown = hsig.Index.build(W.base[:n0], W.attr[:n0], W.level_u[:n0], s.S, s.M, s.ef_cons, seed=3)
    for a, b in zip(splits, splits[1:] + (n,)):
        grown.insert(W.base[a:b], W.attr[a:b], W.level_u[a:b])
    assert grown.n == n and grown.L == whole.L and grown.gentry == whole.gentry
    A, B = _tables(whole), _tables(grown)
    assert A.keys() == B.keys()
    for key in A:
        assert np.array_equal(A[key], B[key]), key


def test_boundaries_stay_fixed(parts):
    W, s = parts
    n0 = 500
    ix = hsig.Index.build(W.base[:n0], W.attr[:n0], W.level_u[:n0], s.S, s.M, s.ef_cons)
    ss0, _, _ = ix.segments()
    a0 = ix.attr_sorted()
    bvals = a0[ss0[1:-1]]  # the boundary values b_1 .. b_{S-1}
    ix.insert(W.base[n0:], W.attr[n0:], W.level_u[n0:])
    ss, _, _ = ix.segments()
    a = ix.attr_sorted()
    # every segment still starts at its boundary value: attributes below it lie to the left
    assert np.array_equal(a[ss[1:-1]], bvals)
    assert np.all(a[ss[1:-1] - 1] < bvals)
    # the ext ids of the inserted objects continue the build's
    assert sorted(ix.ext_ids().tolist()) == list(range(len(W.attr)))


def test_grown_index_searches(parts):
    """After insertion every strategy searches all objects: the pre-filter equals the
    exact answer over the full set and hybrid/post reach high recall."""
    W, s = parts
    n0 = 700
    ix = hsig.Index.build(W.base[:n0], W.attr[:n0], W.level_u[:n0], s.S, s.M, s.ef_cons)
    ix.insert(W.base[n0:], W.attr[n0:], W.level_u[n0:])
    ids, _ = ix.search(W.queries, W.l, W.h, 10, 64, strategy=hsig.PRE)
    rec = {hsig.HYBRID: [], hsig.AUTO: []}
    hy, _ = ix.search(W.queries, W.l, W.h, 10, 64, strategy=hsig.HYBRID)
    au, _ = ix.search(W.queries, W.l, W.h, 10, 64)
    for i in range(len(W.queries)):
        tid, _ = exact.rfknn(W.base, W.attr, W.queries[i], W.l[i], W.h[i], 10)
        assert ids[i, : len(tid)].tolist() == tid.tolist()
        if len(tid):
            rec[hsig.HYBRID].append(len(set(hy[i]) & set(tid)) / len(tid))
            rec[hsig.AUTO].append(len(set(au[i]) & set(tid)) / len(tid))
    assert np.mean(rec[hsig.HYBRID]) > 0.9 and np.mean(rec[hsig.AUTO]) > 0.9


def test_insert_rejects_read_index(parts, tmp_path):
    W, s = parts
    ix = hsig.Index.build(W.base[:300], W.attr[:300], W.level_u[:300], s.S, s.M, s.ef_cons)
    path = str(tmp_path / "x.uix")
    ix.write(path)
    r = hsig.Index.read(path)
    with pytest.raises(ValueError):
        r.insert(W.base[300:310], W.attr[300:310], W.level_u[300:310])
    with pytest.raises(ValueError):
        ix.insert(W.base[300:310], W.attr[300:310], np.zeros(10))
