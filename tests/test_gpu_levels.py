"""Levels mode (the multi-level hierarchy, Sec. 2.2.2 and Alg. 1) against the
oracle's replay of the same batches (oracle/levels.py): the forest of every
level, the sketch, and the counts of links, cuts, passes, repairs, failed
one-column queries and top rounds must be identical; connectivity against
BFS.  Streams with heavy deletion exercise deletes of forest edges at
several weights and repairs that remove cycle edges."""
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


CASES = [
    # name, V, p, delete fraction, seed, batch
    ("sparse_per_update", 48, 0.12, 0.6, 31, 1),
    ("sparse_small_batches", 120, 0.05, 0.6, 32, 13),
    ("dense_batches", 300, 0.2, 0.4, 33, 2000),
    ("whole_stream", 200, 0.03, 0.5, 34, None),
]


@pytest.mark.parametrize("name,V,p,df,seed,batch", CASES)
@pytest.mark.parametrize("mode", ["staged", "atomic"])
def test_levels_mode_matches_oracle(cupk, name, V, p, df, seed, batch, mode):
    u, v, d = streamgen.er_standard(V, p, df, seed)
    C = streamgen.ceil_log2(V)
    D = 2 * C
    S = 0x5EED3000 + seed
    sm = cupk.SCATTER_STAGED if mode == "staged" else cupk.SCATTER_ATOMIC
    ctx = cupk.Context(V, C, D, S, scatter_mode=sm, levels=True)
    sk = oracle.Sketch(V, C, D, S)
    fr = oracle.LevelsReplay(sk)
    n = len(u)
    b = max(1, n if batch is None else batch)
    print(f"levels {name} V={V} n={n} batch={b} mode={mode}", flush=True)
    live = set()
    rng = np.random.default_rng(seed)
    checks = 0
    for s in range(0, n, b):
        e = min(n, s + b)
        ctx.apply_updates(u[s:e], v[s:e], d[s:e])
        fr.apply_batch(u[s:e], v[s:e], d[s:e])
        for a, c, x in zip(u[s:e].tolist(), v[s:e].tolist(), d[s:e].tolist()):
            (live.remove if x else live.add)((a, c))
        if (s // b) % max(1, (n // b) // 5) == 0 or e == n:
            checks += 1
            for j in range(1, C + 1):
                assert ctx.level_forest_edges(j) == fr.forest_edges(j), (s, j)
            eu = np.array([q[0] for q in live], np.uint32)
            ev = np.array([q[1] for q in live], np.uint32)
            truth = oracle.components_truth(V, eu, ev)
            for _ in range(20):
                a, c = (int(x) for x in rng.integers(0, V, 2))
                assert ctx.connected(a, c) == (truth[a] == truth[c])
    assert checks > 0
    assert ctx.forest_edges() == fr.forest_edges()
    assert ctx.digest() == sk.digest()
    ctr = ctx.counters()
    assert (ctr["links"], ctr["cuts"]) == (fr.n_links, fr.n_cuts)
    assert (ctr["level_passes"], ctr["level_repairs"], ctr["level_failed"]) == \
        (fr.n_passes, fr.n_repairs, fr.n_level_failed)
    assert (ctr["rounds"], ctr["sample_failed"]) == (fr.n_top_rounds, fr.n_failed)
    assert fr.n_repairs > 0
    ctx.close()


def test_levels_mode_rejects_exact(cupk):
    with pytest.raises(cupk.CupkError):
        cupk.Context(64, 6, 12, 1, levels=True, exact=True)
    ctx = cupk.Context(64, 6, 12, 1)
    with pytest.raises(cupk.CupkError):
        ctx.level_forest_edges(1)
    ctx.close()
