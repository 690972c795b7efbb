"""Oracle: multi-level forest maintenance (Gibb's hierarchy, Sec. 2.2.2 and
Alg. 1; test infrastructure only).

Levels 0..C.  Level i < C keeps a forest F_i and queries components with the
sampler of sketch column i alone (``sample_col``); the top level C keeps the
forest that answers connectivity and queries with all C columns (``sample``).
F_0 has no edges and F_i is contained in F_(i+1) (Invariants 1 and 2).  The
weight of a forest edge is the lowest level whose forest holds it.

A batch of updates is applied in three steps:

1. every update toggles its edge in the sketch;
2. walking the batch in stream order, a delete of an edge of the top forest
   removes it from every level from its weight up; inserts touch only the
   sketch;
3. restoration of Invariant 3 (a component K of F_i whose level-i query
   succeeds must be a proper subset of its F_(i+1) component), in passes.  A
   pass looks at the levels from ``lo`` up to C-1 and finds the lowest level
   i with a violating component: K whose F_(i+1) component has the same size
   as K and whose query returns an edge (x, y).  Taking those K in ascending
   order of smallest vertex, each one that still violates (its F_(i+1)
   component may have grown meanwhile) is repaired as in Alg. 1: if x and y
   are connected in the top forest, the heaviest edge on the top-forest path
   between them (ties: the smallest edge (a, b), a < b) is removed from every
   level from its weight up; then (x, y) joins every forest from level i+1
   up.  The next pass starts at level i+1 (no level at or below i changed).
4. top completion: the replacement rounds of the single-level replay on
   the top forest with the all-column sampler, every tree dirty to begin
   with (every dirty tree but the largest sampled, links in ascending order
   of smallest vertex, EMPTY trees clean, until a round links nothing).  This stands in for the
   levels beyond C that Gibb's bound would ask for: the top forest is then a
   spanning forest w.h.p.
"""
from __future__ import annotations

from collections import deque

import numpy as np

from . import OK, EMPTY, FAILED, sample_col


class LevelsReplay:
    def __init__(self, sketch):
        self.sk = sketch
        self.V, self.C, self.D, self.S = sketch.V, sketch.C, sketch.D, sketch.S
        self.top = self.C
        # adj[j] for j = 1..top (adj[0] would be empty)
        self.adj = [None] + [[set() for _ in range(self.V)] for _ in range(self.top)]
        self.n_links = 0          # (x, y) joins, counted once per repair / top link
        self.n_cuts = 0           # edges removed (deletes and cycle edges), once per edge
        self.n_passes = 0
        self.n_repairs = 0
        self.n_top_rounds = 0
        self.n_level_failed = 0   # level queries that failed (expected: one column)
        self.n_failed = 0         # all-column queries of the top completion that failed

    # -- per-level forests ---------------------------------------------------
    def comp(self, j, w):
        if j == 0:
            return {w}
        seen = {w}
        q = deque([w])
        adj = self.adj[j]
        while q:
            x = q.popleft()
            for y in adj[x]:
                if y not in seen:
                    seen.add(y)
                    q.append(y)
        return seen

    def comps(self, j):
        """Components of F_j as sorted member lists, ascending smallest vertex."""
        out, seen = [], set()
        for w in range(self.V):
            if w in seen:
                continue
            c = self.comp(j, w)
            seen |= c
            out.append(sorted(c))
        return out

    def weight(self, a, b):
        for j in range(1, self.top + 1):
            if b in self.adj[j][a]:
                return j
        raise AssertionError("not a forest edge")

    def _link(self, j, a, b):
        self.adj[j][a].add(b)
        self.adj[j][b].add(a)

    def _unlink(self, j, a, b):
        self.adj[j][a].discard(b)
        self.adj[j][b].discard(a)

    def remove(self, a, b):
        """Remove forest edge (a, b) from every level from its weight up."""
        w = self.weight(a, b)
        for j in range(w, self.top + 1):
            self._unlink(j, a, b)
        self.n_cuts += 1

    def top_path(self, x, y):
        """Vertices of the top-forest path from x to y (None if not connected)."""
        par = {x: None}
        q = deque([x])
        adj = self.adj[self.top]
        while q:
            a = q.popleft()
            if a == y:
                break
            for b in adj[a]:
                if b not in par:
                    par[b] = a
                    q.append(b)
        if y not in par:
            return None
        path = [y]
        while path[-1] != x:
            path.append(par[path[-1]])
        return path[::-1]

    def forest_edges(self, j=None):
        j = self.top if j is None else j
        return sorted((a, b) for a in range(self.V) for b in self.adj[j][a] if a < b)

    def connected(self, a, b):
        return b in self.comp(self.top, a)

    # -- one batch ---------------------------------------------------------
    def apply_batch(self, u, v, is_delete):
        u = np.asarray(u, np.uint32)
        v = np.asarray(v, np.uint32)
        is_delete = np.asarray(is_delete, np.uint8)
        self.sk.apply(u, v)
        for a, b, dl in zip(u.tolist(), v.tolist(), is_delete.tolist()):
            if a > b:
                a, b = b, a
            if dl and b in self.adj[self.top][a]:
                self.remove(a, b)
        self._restore()
        self._top_completion()

    def _query_level(self, i, K):
        a, g = self.sk.set_sketch(np.asarray(K, np.uint32))
        return sample_col(self.V, self.C, self.D, self.S, i, a, g)

    def _restore(self):
        lo = 0
        while lo < self.top:
            self.n_passes += 1
            found_level, found = None, []
            for i in range(lo, self.top):
                for K in self.comps(i):
                    if len(self.comp(i + 1, K[0])) != len(K):
                        continue
                    st, x, y = self._query_level(i, K)
                    if st == FAILED:
                        self.n_level_failed += 1
                    if st == OK:
                        found.append((K, x, y))
                if found:
                    found_level = i
                    break
            if found_level is None:
                return
            i = found_level
            for K, x, y in found:
                inside = x if x in K else y     # the sampled edge leaves K
                if len(self.comp(i + 1, inside)) != len(K):
                    continue            # joined by an earlier repair of this pass
                path = self.top_path(x, y)
                if path is not None:
                    best = None
                    for p, q in zip(path, path[1:]):
                        e = (min(p, q), max(p, q))
                        key = (-self.weight(*e), e)
                        if best is None or key < best[0]:
                            best = (key, e)
                    self.remove(*best[1])
                for j in range(i + 1, self.top + 1):
                    self._link(j, x, y)
                self.n_links += 1
                self.n_repairs += 1
            lo = i + 1

    def _top_completion(self):
        # the replacement rounds of the single-level replay, with every tree
        # of the top forest dirty to begin with
        mark = set(range(self.V))
        while True:
            trees, seen = [], set()
            for w in sorted(mark):
                if w in seen:
                    continue
                t = self.comp(self.top, w)
                seen |= t
                trees.append(t)
            if not trees:
                return
            if len(trees) == 1:
                return
            L = max(trees, key=lambda t: (len(t), -min(t)))
            S = sorted((t for t in trees if t is not L), key=min)
            self.n_top_rounds += 1
            results = []
            for t in S:
                a, g = self.sk.set_sketch(np.fromiter(sorted(t), np.uint32, len(t)))
                results.append(self.sk.sample(a, g))
            linked = False
            for t, (st, x, y) in zip(S, results):
                if st == OK and not self.connected(x, y):
                    self._link(self.top, x, y)
                    self.n_links += 1
                    linked = True
            failed = False
            for t, (st, x, y) in zip(S, results):
                if st == EMPTY:
                    if self.comp(self.top, min(t)) == t:
                        mark -= t
                elif st == FAILED:
                    self.n_failed += 1
                    failed = True
            if not linked:
                return
