"""Exact mode (speculative buffering with undo, Sec. 4.3): whatever the
batch size, the forest equals the oracle's replay of the stream one update
at a time, and so do the sketch and the link / cut / round counts.  The
streams delete most edges, so many deletions cut forest edges inside a
batch and force the undo path."""
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


def _per_update(V, C, D, S, u, v, d):
    sk = oracle.Sketch(V, C, D, S)
    fr = oracle.ForestReplay(sk)
    for i in range(len(u)):
        fr.apply_batch(u[i:i + 1], v[i:i + 1], d[i:i + 1])
    return sk, fr


STREAMS = {
    "sparse_heavy_delete": (80, 0.15, 0.6, 21),
    "dense_heavy_delete": (300, 0.05, 0.9, 22),
}


@pytest.fixture(scope="module", params=sorted(STREAMS))
def ref(request):
    V, p, df, seed = STREAMS[request.param]
    u, v, d = streamgen.er_standard(V, p, df, seed)
    C = streamgen.ceil_log2(V)
    D = 2 * C
    S = 0x5EED2000 + seed
    sk, fr = _per_update(V, C, D, S, u, v, d)
    return dict(name=request.param, V=V, C=C, D=D, S=S, u=u, v=v, d=d, digest=sk.digest(),
                forest=fr.forest_edges(), links=fr.n_links, cuts=fr.n_cuts, rounds=fr.n_rounds,
                failed=fr.n_failed)


@pytest.mark.parametrize("batch,mode", [(1, "staged"), (7, "staged"), (257, "atomic"),
                                        (257, "staged"), (None, "staged")])
def test_exact_mode_equals_per_update_replay(cupk, ref, batch, mode):
    R = ref
    sm = cupk.SCATTER_STAGED if mode == "staged" else cupk.SCATTER_ATOMIC
    ctx = cupk.Context(R["V"], R["C"], R["D"], R["S"], scatter_mode=sm, exact=True)
    n = len(R["u"])
    b = n if batch is None else batch
    print(f"exact {R['name']} n={n} batch={b} mode={mode}", flush=True)
    for s in range(0, n, b):
        ctx.apply_updates(R["u"][s:s + b], R["v"][s:s + b], R["d"][s:s + b])
    assert R["failed"] == 0
    assert ctx.digest() == R["digest"]
    assert ctx.forest_edges() == R["forest"]
    ctr = ctx.counters()
    assert (ctr["links"], ctr["cuts"], ctr["rounds"]) == (R["links"], R["cuts"], R["rounds"])
    assert ctr["sample_failed"] == 0
    if b > 1:
        assert ctr["reverts"] > 0
    ctx.close()


def test_exact_mode_batches_agree_on_queries(cupk):
    # connectivity after every batch of an exact run equals BFS truth, and
    # device-resident batches take the same path
    V, p, df, seed = 200, 0.04, 0.7, 23
    u, v, d = streamgen.er_standard(V, p, df, seed)
    C = streamgen.ceil_log2(V)
    import torch
    packed = torch.from_numpy(cupk.pack_updates(u, v, d).view(np.int64)).cuda()
    ctx = cupk.Context(V, C, 2 * C, 0x5EED, exact=True)
    live = set()
    B = 101
    rng = np.random.default_rng(1)
    for s in range(0, len(u), B):
        ctx.apply_updates_device(packed[s:s + B])
        for a, b, x in zip(u[s:s + B].tolist(), v[s:s + B].tolist(), d[s:s + B].tolist()):
            (live.remove if x else live.add)((a, b))
        eu = np.array([e[0] for e in live], np.uint32)
        ev = np.array([e[1] for e in live], np.uint32)
        truth = oracle.components_truth(V, eu, ev)
        for _ in range(20):
            a, b = (int(x) for x in rng.integers(0, V, 2))
            assert ctx.connected(a, b) == (truth[a] == truth[b])
    ctx.close()
