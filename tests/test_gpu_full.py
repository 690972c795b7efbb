"""Full-size parity on the benchmark workload (V=16384, G(V,0.3) inserts then
10% deletions, 44,276,290 updates in 1,000,000-update device batches: the
launch configuration bench.py times).

The whole oracle sketch takes about half a minute on the CPU, so it is
compared through its digest (stored by tests/golden/make_oracle_digests.py,
which calls only the oracle), plus exact sketches of sampled vertices that
the oracle recomputes from the stream one by one, plus properties that hold
at any size: connectivity equals scipy's connected components of the final
edge set, the forest is a spanning forest of it, sampled edges are real cut
edges, and a true component's aggregate sketch is empty.
"""
import json
import os

import numpy as np
import pytest

import oracle
import streamgen

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "oracle_digests.json")


@pytest.fixture(scope="module")
def workload():
    import torch
    assert torch.cuda.is_available()
    import paper_2509_14433_amd as cupk
    cfg = streamgen.CONFIGS[1]
    u, v, d = streamgen.config_stream(1)
    packed = torch.from_numpy(cupk.pack_updates(u, v, d).view(np.int64)).cuda()
    V = cfg["V"]
    keys_ins = u[d == 0].astype(np.uint64) * V + v[d == 0]
    keys_del = u[d == 1].astype(np.uint64) * V + v[d == 1]
    final = np.setdiff1d(keys_ins, keys_del, assume_unique=True)
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    fu = (final // V).astype(np.int64)
    fv = (final % V).astype(np.int64)
    m = coo_matrix((np.ones(len(fu), np.int8), (fu, fv)), shape=(V, V))
    ncomp, comp = connected_components(m, directed=False)
    return dict(cupk=cupk, torch=torch, cfg=cfg, u=u, v=v, d=d, packed=packed, final=final,
                ncomp=ncomp, comp=comp)


@pytest.mark.parametrize("mode", ["staged", "pair", "atomic"])
def test_benchmark_workload_full_size(workload, mode):
    W = workload
    cupk, cfg = W["cupk"], W["cfg"]
    V = cfg["V"]
    C = streamgen.ceil_log2(V)
    D = 2 * C
    S = cfg["S"]
    sm = cupk.SCATTER_ATOMIC if mode == "atomic" else cupk.SCATTER_STAGED
    lay = {"staged": cupk.LAYOUT_RECORD, "pair": cupk.LAYOUT_PAIR}.get(mode, 0)
    ctx = cupk.Context(V, C, D, S, scatter_mode=sm, max_batch=cfg["batch"], tile_layout=lay)
    n = len(W["u"])
    print(f"full workload mode={mode} n={n}", flush=True)
    for s in range(0, n, cfg["batch"]):
        ctx.apply_updates_device(W["packed"][s:min(n, s + cfg["batch"])])
    ctx.sync()
    # whole-sketch digest against the oracle's
    gold = json.load(open(GOLDEN))[cfg["name"]]
    assert (gold["V"], gold["C"], gold["D"], gold["S"], gold["n_updates"]) == (V, C, D, S, n)
    assert ctx.digest() == int(gold["digest"], 16)
    # sampled vertices, exact
    rng = np.random.default_rng(5)
    for w in [0, V - 1] + rng.choice(V, size=6, replace=False).tolist():
        oa, og = oracle.vertex_from_stream(V, C, D, S, int(w), W["u"], W["v"])
        ga, gg = ctx.get_sketch(int(w), 1)
        assert np.array_equal(ga[0], oa) and np.array_equal(gg[0], og), w
    # connectivity and forest
    lab = ctx.component_labels()
    comp = W["comp"]
    assert ctx.num_components() == W["ncomp"]
    m = {}
    for w in range(V):
        m.setdefault(int(lab[w]), set()).add(int(comp[w]))
    assert all(len(s) == 1 for s in m.values())
    fe = np.array(ctx.forest_edges(), dtype=np.uint64)
    assert len(fe) == V - W["ncomp"]
    keys = fe[:, 0] * V + fe[:, 1]
    assert np.isin(keys, W["final"]).all()
    # component sketch of everything is empty; samples of random sets are cut edges
    a, g = ctx.component_sketch(np.arange(V, dtype=np.uint32))
    assert not a.any() and not g.any()
    final_set = W["final"]
    for _ in range(20):
        U = np.sort(rng.choice(V, size=int(rng.integers(1, 50)), replace=False)).astype(np.uint32)
        a, g = ctx.component_sketch(U)
        st, x, y = ctx.sample_cut_edge(a, g)
        assert st == cupk.OK
        assert x < y and np.isin(np.uint64(x * V + y), final_set)
        assert (x in U) != (y in U)
    ctr = ctx.counters()
    print(ctr, flush=True)
    assert ctr["sample_failed"] == 0
    # components from the sketches alone: same partition, merge edges are a
    # spanning forest of the final graph, Boruvka's round bound
    sl, se, si = ctx.static_components()
    assert si["sample_failed"] == 0 and si["n_components"] == W["ncomp"]
    assert all(comp[w] == comp[sl[w]] for w in range(V))
    assert len(set(sl.tolist())) == W["ncomp"]
    assert si["n_edges"] == V - W["ncomp"] and si["rounds"] <= C + 1
    sk_keys = np.array([a * V + b for a, b in se], dtype=np.uint64)
    assert np.isin(sk_keys, W["final"]).all()
    par = list(range(V))

    def find(x):
        while par[x] != x:
            par[x] = par[par[x]]
            x = par[x]
        return x
    for a, b in se:
        ra, rb = find(a), find(b)
        assert ra != rb
        par[ra] = rb
    ctx.close()


def test_benchmark_workload_first_batch_forest(workload):
    # the first 1,000,000-update batch flags every insert (every vertex is
    # its own tree); its forest must equal the oracle's replay exactly
    W = workload
    cupk, cfg = W["cupk"], W["cfg"]
    V, B = cfg["V"], cfg["batch"]
    C = streamgen.ceil_log2(V)
    D = 2 * C
    ctx = cupk.Context(V, C, D, cfg["S"], max_batch=B)
    ctx.apply_updates_device(W["packed"][:B])
    fr = oracle.ForestReplay(oracle.Sketch(V, C, D, cfg["S"]))
    fr.apply_batch(W["u"][:B], W["v"][:B], W["d"][:B])
    assert ctx.forest_edges() == fr.forest_edges()
    assert ctx.counters()["links"] == fr.n_links
    ctx.close()
