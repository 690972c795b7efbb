"""Pins of the multi-level oracle (oracle/levels.py) against what the paper
fixes: Invariants 1-3 of Sec. 2.2.2 checked by brute force after every
batch, the top forest a spanning forest of the live graph, forests made of
live edges only, and hand-worked repairs that remove the heaviest edge of a
cycle (tie: the smaller edge) from its weight up."""
import math

import numpy as np
import pytest

import oracle
import streamgen


def _check_invariants(fr, live):
    V, top = fr.V, fr.top
    for j in range(1, top + 1):
        fe = set(fr.forest_edges(j))
        assert fe <= live, "forest edge not in the graph"
        # a forest: V - #components == #edges
        assert len(fe) == V - len(fr.comps(j))
        if j < top:
            assert fe <= set(fr.forest_edges(j + 1)), "Invariant 2"
    for i in range(top):
        for K in fr.comps(i):
            st, x, y = fr._query_level(i, K)
            if st == oracle.OK:
                assert len(fr.comp(i + 1, K[0])) > len(K), f"Invariant 3 at level {i}"


@pytest.mark.parametrize("V,p,df,batch,seed", [
    (24, 0.2, 0.6, 1, 1),
    (40, 0.15, 0.5, 9, 2),
    (64, 0.1, 0.7, 40, 3),
    (90, 0.05, 0.5, None, 4),
])
def test_levels_invariants_and_spanning(V, p, df, batch, seed):
    u, v, d = streamgen.er_standard(V, p, df, seed)
    C = math.ceil(math.log2(V))
    sk = oracle.Sketch(V, C, 2 * C, 0x5EED + seed)
    fr = oracle.LevelsReplay(sk)
    n = len(u)
    b = n if batch is None else batch
    live = set()
    for s in range(0, n, b):
        e = min(n, s + b)
        fr.apply_batch(u[s:e], v[s:e], d[s:e])
        for a, c, x in zip(u[s:e].tolist(), v[s:e].tolist(), d[s:e].tolist()):
            (live.remove if x else live.add)((a, c))
        if (s // b) % max(1, (n // b) // 6) == 0 or e == n:
            _check_invariants(fr, live)
            eu = np.array([q[0] for q in live], np.uint32)
            ev = np.array([q[1] for q in live], np.uint32)
            truth = oracle.components_truth(V, eu, ev)
            oracle.check_spanning_forest(V, fr.forest_edges(), live, truth)
    assert fr.n_failed == 0
    assert fr.n_repairs > 0


def _manual(paths):
    """Three vertices; the sketch holds only edge (0, 2); forest levels set by
    hand from {level: edges}."""
    sk = oracle.Sketch(3, 5, 10, 0x5EED)
    sk.apply(np.array([0], np.uint32), np.array([2], np.uint32))
    fr = oracle.LevelsReplay(sk)
    for j, edges in paths.items():
        for a, b in edges:
            fr._link(j, a, b)
    return fr


def test_levels_repair_removes_heaviest_cycle_edge_tie_smaller():
    # top forest path 0-1-2, both edges of weight 2: the query of {0} at
    # level 0 returns (0, 2); the tie goes to (0, 1), removed from level 2 up
    top = 5
    fr = _manual({j: [(0, 1), (1, 2)] for j in range(2, top + 1)})
    fr._restore()
    assert fr.forest_edges(1) == [(0, 2)]
    for j in range(2, top + 1):
        assert fr.forest_edges(j) == [(0, 2), (1, 2)]
    assert (fr.n_cuts, fr.n_links, fr.n_repairs) == (1, 1, 1)


def test_levels_repair_removes_heaviest_cycle_edge_by_weight():
    # (0, 1) has weight 2 and (1, 2) weight 3: (1, 2) goes, from level 3 up
    top = 5
    levels = {2: [(0, 1)]}
    levels.update({j: [(0, 1), (1, 2)] for j in range(3, top + 1)})
    fr = _manual(levels)
    fr._restore()
    assert fr.forest_edges(1) == [(0, 2)]
    assert fr.forest_edges(2) == [(0, 1), (0, 2)]
    for j in range(3, top + 1):
        assert fr.forest_edges(j) == [(0, 1), (0, 2)]
    assert fr.weight(0, 1) == 2 and fr.weight(0, 2) == 1


def test_levels_single_edge_insert_and_delete():
    sk = oracle.Sketch(2, 1, 2, 7)
    fr = oracle.LevelsReplay(sk)
    fr.apply_batch([0], [1], [0])
    assert fr.forest_edges() == [(0, 1)] and fr.weight(0, 1) == 1
    assert fr.n_passes == 1 and fr.n_repairs == 1   # top == 1: one pass over level 0
    fr.apply_batch([0], [1], [1])
    assert fr.forest_edges() == [] and fr.n_cuts == 1
