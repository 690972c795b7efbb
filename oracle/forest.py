"""Oracle forest replay and connectivity truth (test infrastructure only).

Spanning-forest maintenance on top of the oracle sketch, in plain Python.

The paper keeps a spanning forest of the current graph and, when a forest
edge is deleted, queries the cutset of the broken component for a
replacement (Sec. 2.2.1 cutset Query; Alg. 1 restoration; AGM Boruvka rounds
in App. A.1.1 merge fragments by adding their sketches).  This module replays
one level of that scheme with the batch semantics the GPU library uses:

Per batch of updates, with ``L`` the component labels of the forest at the
start of the batch:

1. every update toggles its edge in the sketch;
2. walking the updates in stream order, an insert (u,v) with
   ``L[u] != L[v]`` whose endpoints are in different trees of the current
   forest is linked; a delete of a current forest edge is cut, and both
   resulting trees are marked dirty.  Any other update only touches the
   sketch (an insert inside a batch-start component that a cut separated is
   left to step 3);
3. replacement rounds over the dirty trees.  Clean trees are whole
   components, so every edge leaving a dirty tree ends in another dirty tree
   (the search-from-the-smaller-side argument).  Each round therefore skips
   the largest dirty tree (ties: smallest vertex id) and samples all the
   others: each is reduced to one sketch (XOR of its members' sketches) and
   queried; then, in ascending order of smallest vertex id, each sampled
   edge (x,y) is linked if x and y are in different trees at that moment.  A
   tree whose sample is EMPTY has no cut edge (it is a whole component) and
   becomes clean.  A single remaining dirty tree is a whole component and
   becomes clean.  If a round links nothing, the rounds stop: when no sample
   FAILED the skipped tree is a whole component too and becomes clean;
   otherwise the failed trees and the skipped one stay dirty for the next
   batch.

With batches of one update this is the per-update method; larger batches
defer replacement search to the end of the batch, where queries observe the
state (queries flush pending updates first, Sec. 4.3).
"""
from __future__ import annotations

from collections import deque

import numpy as np


class _UF:
    def __init__(self, n):
        self.p = list(range(n))

    def find(self, x):
        p = self.p
        while p[x] != x:
            p[x] = p[p[x]]
            x = p[x]
        return x

    def union(self, a, b):
        ra, rb = self.find(a), self.find(b)
        if ra != rb:
            self.p[ra] = rb


class ForestReplay:
    """Plain replay of forest maintenance over an oracle ``Sketch``."""

    def __init__(self, sketch):
        self.sk = sketch
        self.V = sketch.V
        self.adj = [set() for _ in range(self.V)]
        self.mark = set()          # vertices whose tree is dirty
        self.uf = _UF(self.V)
        self._stale = False
        self.n_links = 0
        self.n_cuts = 0
        self.n_rounds = 0
        self.n_failed = 0
        self.round_log = []        # per round: list of (min_vertex, status, u, v)

    # -- forest primitives ---------------------------------------------------
    def _rebuild_uf(self):
        self.uf = _UF(self.V)
        for a in range(self.V):
            for b in self.adj[a]:
                if a < b:
                    self.uf.union(a, b)

    def _uf_now(self):
        # cuts only mark the union-find stale; it is rebuilt once, when the
        # next connectivity question comes (same answers, one rebuild per
        # run of cuts instead of one per cut)
        if self._stale:
            self._rebuild_uf()
            self._stale = False
        return self.uf

    def connected(self, a, b):
        uf = self._uf_now()
        return uf.find(a) == uf.find(b)

    def _link(self, a, b):
        assert not self.connected(a, b)
        self.adj[a].add(b)
        self.adj[b].add(a)
        self._uf_now().union(a, b)
        self.n_links += 1

    def _cut(self, a, b):
        self.adj[a].discard(b)
        self.adj[b].discard(a)
        self._stale = True
        self.n_cuts += 1

    def tree_of(self, w):
        seen = {w}
        q = deque([w])
        while q:
            x = q.popleft()
            for y in self.adj[x]:
                if y not in seen:
                    seen.add(y)
                    q.append(y)
        return seen

    def labels(self):
        uf = self._uf_now()
        lab = np.empty(self.V, np.int64)
        for w in range(self.V):
            lab[w] = uf.find(w)
        return lab

    def forest_edges(self):
        out = sorted((a, b) for a in range(self.V) for b in self.adj[a] if a < b)
        return out

    # -- one batch -------------------------------------------------------------
    def apply_batch(self, u, v, is_delete):
        u = np.asarray(u, np.uint32)
        v = np.asarray(v, np.uint32)
        is_delete = np.asarray(is_delete, np.uint8)
        self.sk.apply(u, v)
        # batch-start labels; for a batch of one update they are the current
        # labels, and the test below reduces to "not connected"
        L = self.labels() if len(u) > 1 else None
        for a, b, dl in zip(u.tolist(), v.tolist(), is_delete.tolist()):
            if a > b:
                a, b = b, a
            if not dl:
                crosses = (L[a] != L[b]) if L is not None else True
                if crosses and not self.connected(a, b):
                    self._link(a, b)
            else:
                if b in self.adj[a]:
                    self._cut(a, b)
                    self.mark.add(a)
                    self.mark.add(b)
        self._rounds()

    def _dirty_trees(self):
        trees, seen = [], set()
        for w in sorted(self.mark):
            if w in seen:
                continue
            t = self.tree_of(w)
            seen |= t
            trees.append(t)
        return trees

    def _rounds(self):
        while True:
            D = self._dirty_trees()
            if not D:
                return
            if len(D) == 1:
                self.mark -= D[0]
                return
            L = max(D, key=lambda t: (len(t), -min(t)))
            S = sorted((t for t in D if t is not L), key=min)
            self.n_rounds += 1
            results = []
            for t in S:
                a, g = self.sk.set_sketch(np.fromiter(sorted(t), np.uint32, len(t)))
                results.append(self.sk.sample(a, g))
            self.round_log.append([(min(t), r[0], r[1], r[2]) for t, r in zip(S, results)])
            linked = False
            for t, (st, x, y) in zip(S, results):
                if st == 0 and not self.connected(x, y):
                    self._link(x, y)
                    linked = True
            failed = False
            for t, (st, x, y) in zip(S, results):
                if st == 1:
                    if self.tree_of(min(t)) == t:   # not merged this round
                        self.mark -= t
                elif st == 2:
                    self.n_failed += 1
                    failed = True
            if not linked:
                if not failed:
                    self.mark -= L
                return


def components_truth(V, u, v):
    """Component label (smallest member id) of every vertex of the graph with
    edge list (u, v), by breadth-first search over adjacency lists."""
    adj = [[] for _ in range(V)]
    for a, b in zip(np.asarray(u).tolist(), np.asarray(v).tolist()):
        adj[a].append(b)
        adj[b].append(a)
    lab = np.full(V, -1, np.int64)
    for s in range(V):
        if lab[s] >= 0:
            continue
        lab[s] = s
        q = deque([s])
        while q:
            x = q.popleft()
            for y in adj[x]:
                if lab[y] < 0:
                    lab[y] = s
                    q.append(y)
    return lab


def check_spanning_forest(V, forest, edge_set, truth_labels):
    """Assert that ``forest`` (list of (a,b), a<b) is a spanning forest of the
    graph whose edges are ``edge_set`` and components ``truth_labels``."""
    uf = _UF(V)
    for a, b in forest:
        assert (a, b) in edge_set, f"forest edge {(a, b)} not in graph"
        assert uf.find(a) != uf.find(b), f"forest edge {(a, b)} closes a cycle"
        uf.union(a, b)
    n_comp_truth = len(set(truth_labels.tolist()))
    assert V - len(forest) == n_comp_truth, (V - len(forest), n_comp_truth)
    # same partition
    for w in range(V):
        assert (uf.find(w) == uf.find(int(truth_labels[w])))
