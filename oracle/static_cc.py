"""Oracle: connected components of the whole graph from its vertex sketches
(test infrastructure only).

This is the sketch connectivity algorithm the paper builds on (App. A.1.1,
AGM): Boruvka's algorithm over supernodes, where a supernode's incident edges
are recovered by querying its sketch, and merging supernodes merges (XORs)
their sketches.  Written out:

* supernodes start as the single vertices; all are active;
* each round takes the active supernodes in ascending order of their
  smallest vertex, sums (XORs) each one's member sketches and queries the
  sum (the oracle's ``sample``);
* then, in that order, every sampled edge (x, y) merges the supernodes of x
  and y unless they are already one; a merge records (x, y) as a spanning
  forest edge;
* a supernode whose query is EMPTY has no edge leaving it: it is a whole
  component and stops being active (unless a merge in the same round joined
  it to another supernode);
* a round that merges nothing ends the algorithm.  Supernodes whose query
  FAILED are then left as they are (their components may be split).

Result: per vertex the smallest vertex of its final supernode, the merge
edges in merge order, the number of rounds and of failed queries.  On the
same sketch the GPU library must reproduce all of it exactly.
"""
from __future__ import annotations

import numpy as np


def static_components(sk):
    V = sk.V
    parent = list(range(V))
    size = [1] * V

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    finished = set()   # roots of supernodes known to be whole components
    edges = []
    rounds = 0
    n_failed = 0
    while True:
        groups = {}
        for w in range(V):
            groups.setdefault(find(w), []).append(w)
        active = sorted((m for r, m in groups.items() if r not in finished), key=lambda m: m[0])
        if not active:
            break
        rounds += 1
        results = []
        for m in active:
            a, g = sk.set_sketch(np.asarray(m, np.uint32))
            results.append(sk.sample(a, g))
        merged = False
        for m, (st, x, y) in zip(active, results):
            if st != 0:
                continue
            rx, ry = find(x), find(y)
            if rx != ry:
                parent[rx] = ry
                size[ry] += size[rx]
                edges.append((min(x, y), max(x, y)))
                merged = True
        for m, (st, x, y) in zip(active, results):
            if st == 1:
                r = find(m[0])
                # still exactly this supernode: nothing merged into it
                if size[r] == len(m):
                    finished.add(r)
            elif st == 2:
                n_failed += 1
        if not merged:
            break
    labels = np.empty(V, np.int64)
    low = {}
    for w in range(V):
        r = find(w)
        if r not in low:
            low[r] = w
        labels[w] = low[r]
    return labels, edges, rounds, n_failed
