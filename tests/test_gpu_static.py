"""Connected components from the sketches alone (Boruvka over supernodes,
App. A.1.1) on the GPU against the oracle's run of the same algorithm on the
same sketch: labels, merge edges (in merge order), rounds and failed queries
must all be identical; and against the true components of the final graph.
"""
import math

import numpy as np
import pytest

import oracle
import streamgen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cupk():
    import torch
    assert torch.cuda.is_available()
    import paper_2509_14433_amd as m
    return m


def _run(cupk, V, u, v, d, S, batch=None, mode=None):
    C = max(1, math.ceil(math.log2(V)))
    D = 2 * C
    kw = {} if mode is None else {"scatter_mode": mode}
    ctx = cupk.Context(V, C, D, S, **kw)
    n = len(u)
    b = max(1, n if batch is None else batch)
    for s in range(0, n, b):
        ctx.apply_updates(u[s:s + b], v[s:s + b], d[s:s + b])
    sk = oracle.Sketch(V, C, D, S)
    if n:
        sk.apply(u, v)
    got = ctx.static_components()
    want = oracle.static_components(sk)
    forest_labels = ctx.component_labels()
    ctx.close()
    return got, want, forest_labels


def _check(V, u, v, d, got, want, forest_labels):
    labels, edges, info = got
    wl, we, wr, wf = want
    assert labels.tolist() == wl.tolist()
    assert edges == we
    assert info["rounds"] == wr and info["sample_failed"] == wf
    assert info["n_components"] == len(set(wl.tolist()))
    assert info["n_edges"] == V - info["n_components"]
    fu, fv = streamgen.final_edges(u, v, d)
    truth = oracle.components_truth(V, fu, fv)
    assert labels.tolist() == truth.tolist()
    # the maintained forest induces the same partition
    assert all(forest_labels[w] == forest_labels[truth[w]] for w in range(V))


@pytest.mark.parametrize("name,V,p,df,seed,batch", [
    ("dense", 1024, 0.5, 0.25, 1, 65536),
    ("sparse_many_components", 3000, 0.0008, 0.3, 2, 4096),
    ("mid", 500, 0.01, 0.5, 3, 997),
])
def test_static_components_match_oracle(cupk, name, V, p, df, seed, batch):
    u, v, d = streamgen.er_standard(V, p, df, seed)
    print(f"static {name} V={V} n={len(u)}", flush=True)
    got, want, fl = _run(cupk, V, u, v, d, 0x5EED0000 + seed, batch)
    _check(V, u, v, d, got, want, fl)


def test_static_components_degenerate(cupk):
    # no edges: every vertex is its own component, one round of EMPTY queries
    V = 64
    e = np.zeros(0, np.uint32)
    got, want, fl = _run(cupk, V, e, e, np.zeros(0, np.uint8), 0x5EED)
    assert got[2]["rounds"] == 1 and got[1] == []
    _check(V, e, e, np.zeros(0, np.uint8), got, want, fl)
    # every edge inserted then deleted: the sketch is zero again
    u, v, d = streamgen.er_standard(V, 0.3, 0.0, 5)
    u2 = np.concatenate([u, u]); v2 = np.concatenate([v, v])
    d2 = np.concatenate([np.zeros(len(u), np.uint8), np.ones(len(u), np.uint8)])
    got, want, fl = _run(cupk, V, u2, v2, d2, 0x5EED)
    assert got[2]["n_components"] == V and got[2]["rounds"] == 1
    _check(V, u2, v2, d2, got, want, fl)
    # two vertices, one edge
    one = np.array([0], np.uint32)
    got, want, fl = _run(cupk, 2, one, one + 1, np.zeros(1, np.uint8), 7)
    assert got[1] == [(0, 1)] and got[2]["n_components"] == 1
    _check(2, one, one + 1, np.zeros(1, np.uint8), got, want, fl)
