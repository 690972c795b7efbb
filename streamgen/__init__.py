"""Seeded synthetic update streams for sketch-based dynamic connectivity.

This module only draws graphs and update orders.  It holds none of the
method's arithmetic (no hashing, no sketches, no forests), so that both the
CPU oracle and the GPU library can be fed the same inputs without sharing any
code of the method itself.

A stream is three equal-length numpy arrays ``(u, v, is_delete)`` with
``u, v`` uint32 vertex ids (``u < v``) and ``is_delete`` uint8.  Streams are
legal in the sense of the graph-stream model (App. A.1 of the paper): an
edge is inserted only when absent and deleted only when present, and there are
no self loops.

Workloads (stand-ins for the paper's Kronecker / random streams of Table 1,
which are not available here; they keep the dense regime and the "insert
all, then delete" stream shape of Sec. 5 / App. C):

* ``er_standard(V, p, del_frac, seed)``: every pair ``u<v`` is inserted with
  probability ``p`` in a seeded random order, then a seeded random fraction
  ``del_frac`` of the inserted edges is deleted in random order.
* ``rmat_interleaved``: R-MAT edges with interleaved deletions (C helper).
* ``clustered_churn``: dense clusters joined by bridges, with fixed-forest
  style churn and an adversarial bridge toggling phase.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libstreamgen.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile gen.c (the long-stream generators) with gcc, in place."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-shared", "-fPIC", "-o",
                               tmp, os.path.join(_HERE, "gen.c"), "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _c():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        L = ctypes.CDLL(_SO)
        p, u32, u64, sz, dbl = (ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64,
                                ctypes.c_size_t, ctypes.c_double)
        L.sg_rmat_new.restype = p
        L.sg_rmat_new.argtypes = [u32, u64, sz]
        L.sg_rmat_free.restype = None
        L.sg_rmat_free.argtypes = [p]
        L.sg_rmat_next.restype = sz
        L.sg_rmat_next.argtypes = [p, sz, dbl, dbl, dbl, dbl, p, p, p]
        L.sg_ftd_new.restype = p
        L.sg_ftd_new.argtypes = [u32, dbl, dbl, dbl, u64]
        L.sg_ftd_free.restype = None
        L.sg_ftd_free.argtypes = [p]
        for f in (L.sg_ftd_m, L.sg_ftd_k, L.sg_ftd_deleted):
            f.restype = sz
            f.argtypes = [p]
        L.sg_ftd_inserts.restype = sz
        L.sg_ftd_inserts.argtypes = [p, sz, sz, p]
        L.sg_ftd_delete_chunk.restype = sz
        L.sg_ftd_delete_chunk.argtypes = [p, sz, p, sz, p]
        L.sg_clu_new.restype = p
        L.sg_clu_new.argtypes = [u32, u32, dbl, u32, u32, u32, u32, u64]
        L.sg_clu_free.restype = None
        L.sg_clu_free.argtypes = [p]
        for f in (L.sg_clu_setup_len, L.sg_clu_round_cap, L.sg_clu_m2):
            f.restype = sz
            f.argtypes = [p]
        L.sg_clu_setup.restype = sz
        L.sg_clu_setup.argtypes = [p, p]
        L.sg_clu_round.restype = sz
        L.sg_clu_round.argtypes = [p, u32, p]
        L.sg_forest_mask.restype = sz
        L.sg_forest_mask.argtypes = [u32, sz, p, p, p]
        _lib = L
    return _lib


def _arrays(n):
    return (np.zeros(n, np.uint32), np.zeros(n, np.uint32), np.zeros(n, np.uint8))


def _p(a):
    return ctypes.c_void_p(a.ctypes.data)


def rmat_chunks(logV: int, n: int, del_prob: float, seed: int, chunk: int = 1 << 24,
                a: float = 0.57, b: float = 0.19, c: float = 0.19):
    """R-MAT (a, b, c, d=1-a-b-c) inserts with interleaved deletions (each
    step deletes a uniformly random live edge with probability del_prob),
    yielded in pieces of ``chunk`` updates; the pieces concatenate to the
    stream ``rmat_interleaved`` returns."""
    L = _c()
    h = L.sg_rmat_new(logV, seed, n)
    if not h:
        raise MemoryError("R-MAT generator allocation failed")
    try:
        done = 0
        while done < n:
            m = min(chunk, n - done)
            u, v, d = _arrays(m)
            if L.sg_rmat_next(h, m, del_prob, a, b, c, _p(u), _p(v), _p(d)) != m:
                raise MemoryError("R-MAT generator failed")
            done += m
            yield u, v, d
    finally:
        L.sg_rmat_free(h)


def rmat_interleaved(logV: int, n: int, del_prob: float, seed: int,
                     a: float = 0.57, b: float = 0.19, c: float = 0.19):
    """The whole R-MAT stream as (u, v, is_delete) arrays."""
    parts = list(rmat_chunks(logV, n, del_prob, seed, a=a, b=b, c=c))
    if not parts:
        return _arrays(0)
    return tuple(np.concatenate([p[k] for p in parts]) for k in range(3))


class ForestTargetedDeletes:
    """G(V, p) inserts in random order, then ``del_frac`` of the inserted
    edges deleted, in chunks of ``rho`` updates (C generator).

    Before each deletion chunk the caller passes the current spanning-forest
    edges of whatever engine replays the stream (batch boundaries = chunk
    boundaries; the library and the oracle hold the same forest there).  A
    Binomial(chunk, ``forest_frac``) share of the chunk's deletions are
    distinct uniform forest edges (at most all of them); the rest are
    uniform live non-forest edges.  The order inside a chunk is random.
    This module only picks edges; it computes no forest itself.  The
    ``*_packed`` forms give uint64 updates (u | v<<32 | del<<63)."""

    def __init__(self, V: int, p: float, del_frac: float, forest_frac: float, seed: int,
                 rho: int):
        self.V, self.rho, self.forest_frac = V, rho, forest_frac
        self._L = _c()
        self._h = self._L.sg_ftd_new(V, p, del_frac, forest_frac, seed)
        if not self._h:
            raise MemoryError("forest-targeted generator allocation failed")
        self.m = self._L.sg_ftd_m(self._h)
        self.k = self._L.sg_ftd_k(self._h)

    def close(self):
        if getattr(self, "_h", None):
            self._L.sg_ftd_free(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def insert_chunks_packed(self):
        """The insert phase, in chunks of rho packed updates."""
        for s in range(0, self.m, self.rho):
            e = min(self.m, s + self.rho)
            out = np.empty(e - s, np.uint64)
            if self._L.sg_ftd_inserts(self._h, s, e, _p(out)) != e - s:
                raise RuntimeError("inserts drawn out of order")
            yield out

    def insert_chunks(self):
        """The insert phase, in chunks of rho updates, as (u, v, is_delete)."""
        for out in self.insert_chunks_packed():
            yield unpack(out)

    def deletes_left(self) -> int:
        return self.k - self._L.sg_ftd_deleted(self._h)

    def delete_chunk_packed(self, forest_keys):
        """The next chunk of deletions (packed) given the current forest as
        keys u*V + v (u < v); None when every deletion has been drawn."""
        fk = np.array(forest_keys, dtype=np.uint64, copy=True)
        out = np.empty(self.rho, np.uint64)
        n = self._L.sg_ftd_delete_chunk(self._h, self.rho, _p(fk), fk.size, _p(out))
        if n == ctypes.c_size_t(-1).value:
            raise MemoryError("forest-targeted generator")
        return out[:n] if n else None

    def delete_chunk(self, forest_u, forest_v):
        """The next chunk of deletions given the current forest edges, as
        (u, v, is_delete); None when every deletion has been drawn."""
        fu = np.asarray(forest_u, np.uint64)
        fv = np.asarray(forest_v, np.uint64)
        out = self.delete_chunk_packed(np.minimum(fu, fv) * np.uint64(self.V) +
                                       np.maximum(fu, fv))
        return None if out is None else unpack(out)


class ClusteredChurn:
    """Clustered churn drawn one phase at a time (C generator): the setup
    phase (sparse part, bridges, every cluster's first-arrival forest), then
    churn rounds in order, each inserting every other cluster edge in a fresh
    random order and deleting them all in another one; every adv_every
    updates from the forest on, adv_k random bridges are toggled.  Phases
    come packed (uint64: u | v<<32 | is_delete<<63, u < v); ``unpack`` gives
    (u, v, is_delete).  Vertices: clusters first, then the sparse part."""

    def __init__(self, K, S, p_in, n_sparse, extra_bridges, adv_every, adv_k, seed):
        self._L = _c()
        self._h = self._L.sg_clu_new(K, S, p_in, n_sparse, extra_bridges, adv_every, adv_k, seed)
        if not self._h:
            raise MemoryError("clustered churn generator allocation failed")
        self.next_round = 0

    def close(self):
        if getattr(self, "_h", None):
            self._L.sg_clu_free(self._h)
            self._h = None

    def __del__(self):
        self.close()

    @property
    def churn_edges(self) -> int:
        """Cluster edges outside the fixed forest (inserted and deleted once
        per round)."""
        return self._L.sg_clu_m2(self._h)

    def setup(self) -> np.ndarray:
        out = np.empty(self._L.sg_clu_setup_len(self._h), np.uint64)
        n = self._L.sg_clu_setup(self._h, _p(out))
        if n == 0:
            raise RuntimeError("setup phase already drawn")
        return out[:n]

    def round(self) -> np.ndarray:
        out = np.empty(self._L.sg_clu_round_cap(self._h), np.uint64)
        n = self._L.sg_clu_round(self._h, self.next_round, _p(out))
        if n == 0:
            raise RuntimeError("churn round out of order or out of memory")
        self.next_round += 1
        return out[:n]


def unpack(packed):
    """(u, v, is_delete) arrays of packed updates (u | v<<32 | del<<63)."""
    p = np.asarray(packed, np.uint64)
    return ((p & np.uint64(0xFFFFFFFF)).astype(np.uint32),
            ((p >> np.uint64(32)) & np.uint64(0x7FFFFFFF)).astype(np.uint32),
            (p >> np.uint64(63)).astype(np.uint8))


def clustered_churn(K: int, S: int, p_in: float, n_sparse: int, extra_bridges: int,
                    rounds: int, adv_every: int, adv_k: int, seed: int):
    """The whole clustered-churn stream (setup phase, then `rounds` churn
    rounds) as (u, v, is_delete) arrays; see ``ClusteredChurn``."""
    g = ClusteredChurn(K, S, p_in, n_sparse, extra_bridges, adv_every, adv_k, seed)
    parts = [g.setup()] + [g.round() for _ in range(rounds)]
    g.close()
    return unpack(np.concatenate(parts))


def clustered_phases(cfg: dict):
    """Generator over the packed phases (setup, round 0, round 1, ...) of a
    clustered-churn workload description."""
    g = ClusteredChurn(cfg["K"], cfg["Sc"], cfg["p_in"], cfg["n_sparse"], cfg["extra_bridges"],
                       cfg["adv_every"], cfg["adv_k"], cfg["seed"])
    try:
        yield g.setup()
        for _ in range(cfg["rounds"]):
            yield g.round()
    finally:
        g.close()

__all__ = [
    "build",
    "rmat_interleaved",
    "rmat_chunks",
    "ForestTargetedDeletes",
    "clustered_churn",
    "ClusteredChurn",
    "clustered_phases",
    "unpack",
    "stream_of",
    "SCALED",
    "er_standard",
    "er_pairs",
    "ragged_sizes",
    "fixed_sizes",
    "star_stream",
    "final_edges",
    "CONFIGS",
    "config_stream",
]


def er_pairs(V: int, p: float, rng: np.random.Generator, row_block: int = 512):
    """All pairs ``u<v`` of an Erdos-Renyi G(V, p) graph, row-major order.

    Returns ``(u, v)`` uint32 arrays.  The random draw is one float32 uniform
    per ordered cell of a ``row_block x V`` block, so the result depends only
    on ``(V, p, rng state)``.
    """
    us, vs = [], []
    cols = np.arange(V, dtype=np.uint32)
    for r0 in range(0, V, row_block):
        r1 = min(V, r0 + row_block)
        rows = np.arange(r0, r1, dtype=np.uint32)
        rnd = rng.random((r1 - r0, V), dtype=np.float32)
        mask = (rnd < np.float32(p)) & (cols[None, :] > rows[:, None])
        rr, cc = np.nonzero(mask)
        us.append(rows[rr])
        vs.append(cols[cc].astype(np.uint32))
    if not us:
        return np.zeros(0, np.uint32), np.zeros(0, np.uint32)
    return np.concatenate(us).astype(np.uint32), np.concatenate(vs).astype(np.uint32)


def er_standard(V: int, p: float, del_frac: float, seed: int):
    """Insert each pair with probability p in random order, then delete a
    random ``del_frac`` of the inserted edges in random order."""
    rng = np.random.default_rng(seed)
    u, v = er_pairs(V, p, rng)
    m = u.shape[0]
    order = rng.permutation(m)
    u, v = u[order], v[order]
    k = int(math.floor(del_frac * m))
    dsel = rng.permutation(m)[:k]
    du, dv = u[dsel], v[dsel]
    uu = np.concatenate([u, du])
    vv = np.concatenate([v, dv])
    dd = np.concatenate([np.zeros(m, np.uint8), np.ones(k, np.uint8)])
    return uu, vv, dd


def forest_mask(V: int, u, v) -> np.ndarray:
    """Boolean mask of the first-arrival spanning forest of the edge
    sequence (u, v): an edge is in it iff it joins two components of the
    edges before it."""
    u = np.ascontiguousarray(u, np.uint32)
    v = np.ascontiguousarray(v, np.uint32)
    m = np.zeros(u.shape[0], np.uint8)
    k = _c().sg_forest_mask(V, u.shape[0], _p(u), _p(v), _p(m))
    if k == ctypes.c_size_t(-1).value:
        raise MemoryError("forest mask")
    return m.astype(bool)


def fixed_forest(V: int, p: float, reps: int, seed: int):
    """Fixed-forest stream of G(V, p) (the paper's second stream type,
    Sec. 5 and App. C.1): insert a spanning forest of the graph (the
    first-arrival forest of a random edge order), then ``reps`` times insert
    every other edge in random order and delete them all in random order.
    The forest is never deleted, so after the forest no update changes the
    components: almost every update is a non-tree-edge update."""
    rng = np.random.default_rng(seed)
    u, v = er_pairs(V, p, rng)
    order = rng.permutation(u.shape[0])
    u, v = u[order], v[order]
    fm = forest_mask(V, u, v)
    parts_u, parts_v, parts_d = [u[fm]], [v[fm]], [np.zeros(int(fm.sum()), np.uint8)]
    ou, ov = u[~fm], v[~fm]
    m = ou.shape[0]
    for _ in range(reps):
        pi = rng.permutation(m)
        pd = rng.permutation(m)
        parts_u += [ou[pi], ou[pd]]
        parts_v += [ov[pi], ov[pd]]
        parts_d += [np.zeros(m, np.uint8), np.ones(m, np.uint8)]
    return np.concatenate(parts_u), np.concatenate(parts_v), np.concatenate(parts_d)


def star_stream(V: int, n_rounds: int, seed: int, center: int = 0):
    """Hot-vertex adversary: every update touches ``center``.  Inserts the
    star edges in random order, then toggles random star edges
    ``n_rounds`` times (delete when present, insert when absent)."""
    rng = np.random.default_rng(seed)
    others = np.array([w for w in range(V) if w != center], dtype=np.uint32)
    present = np.zeros(V, dtype=bool)
    us, vs, ds = [], [], []
    order = rng.permutation(others)
    for w in order:
        us.append(min(center, int(w)))
        vs.append(max(center, int(w)))
        ds.append(0)
        present[w] = True
    picks = rng.choice(others, size=n_rounds)
    for w in picks:
        us.append(min(center, int(w)))
        vs.append(max(center, int(w)))
        ds.append(1 if present[w] else 0)
        present[w] = not present[w]
    return (np.array(us, np.uint32), np.array(vs, np.uint32), np.array(ds, np.uint8))


def final_edges(u, v, d):
    """Edge set left after replaying the stream, as sorted (u, v) arrays.
    Asserts stream legality (insert only if absent, delete only if present)."""
    live = set()
    for a, b, x in zip(u.tolist(), v.tolist(), d.tolist()):
        e = (a, b)
        if x:
            assert e in live, f"delete of absent edge {e}"
            live.remove(e)
        else:
            assert e not in live, f"insert of present edge {e}"
            live.add(e)
    if not live:
        return np.zeros(0, np.uint32), np.zeros(0, np.uint32)
    arr = np.array(sorted(live), dtype=np.uint32)
    return arr[:, 0].copy(), arr[:, 1].copy()


def ragged_sizes(total: int, lo: int, hi: int, seed: int):
    """Batch sizes drawn log-uniform in [lo, hi] until they cover ``total``
    (the last one is cut to fit)."""
    rng = np.random.default_rng(seed)
    out = []
    left = total
    llo, lhi = math.log(lo), math.log(hi)
    while left > 0:
        s = int(round(math.exp(rng.uniform(llo, lhi))))
        s = max(lo, min(hi, s))
        s = min(s, left)
        out.append(s)
        left -= s
    return out


def fixed_sizes(total: int, size: int):
    """Batch sizes of a fixed ``size`` with a ragged tail."""
    out = [size] * (total // size)
    if total % size:
        out.append(total % size)
    return out


# Workload table.  C and D follow ceil(log2 V) columns and 2*ceil(log2 V)
# depth buckets per vertex; ``S`` is the 64-bit master seed of the hash.
CONFIGS = {
    0: dict(name="er1024_p0.5_del25", V=1024, p=0.5, del_frac=0.25, seed=1,
            S=0x5EED0000 + 0, batch=None),
    1: dict(name="er16384_p0.3_del10", V=16384, p=0.3, del_frac=0.10, seed=2,
            S=0x5EED0000 + 1, batch=1_000_000),
    # R-MAT (0.57, 0.19, 0.19, 0.05) over 2^17 vertices, 5e8 updates, 15%
    # interleaved deletions; ragged batches log-uniform in [1e3, 4e6]
    2: dict(name="rmat17_del15", V=1 << 17, logV=17, n=500_000_000, del_prob=0.15, seed=3,
            S=0x5EED0000 + 2, batch=(1000, 4_000_000)),
    # G(65536, 0.2) inserts then 10% deletions, 30% of them on forest edges;
    # a connectivity query every 1e5 updates
    3: dict(name="er65536_p0.2_forestdel", V=65536, p=0.2, del_frac=0.10, forest_frac=0.30,
            seed=4, S=0x5EED0000 + 3, rho=100_000),
    # 64 clusters of 2048 (p=0.5) + sparse G(n, 2n) on the other 917,504
    # vertices, 63 tree + 65 extra bridges, 11 churn rounds, 100 bridges
    # toggled every 1e5 updates
    4: dict(name="clusters64x2048_churn", V=1 << 20, K=64, Sc=2048, p_in=0.5, n_sparse=917_504,
            extra_bridges=65, rounds=11, adv_every=100_000, adv_k=100, seed=5,
            S=0x5EED0000 + 4, batch=1_000_000),
    # fixed-forest stream of G(16384, 0.3): the forest, then every other edge
    # inserted and deleted once (the paper repeats once for large graphs)
    5: dict(name="er16384_p0.3_fixedforest", V=16384, p=0.3, reps=1, seed=6,
            S=0x5EED0000 + 5, batch=1_000_000),
}

# The same recipes at sizes the CPU oracle replays in seconds (parity tests).
SCALED = {
    2: dict(name="rmat12_del15", V=1 << 12, logV=12, n=1_000_000, del_prob=0.15, seed=13,
            S=0x5EED1002, batch=(100, 100_000)),
    3: dict(name="er1024_p0.2_forestdel", V=1024, p=0.2, del_frac=0.10, forest_frac=0.30,
            seed=14, S=0x5EED1003, rho=2_000),
    4: dict(name="clusters8x128_churn", V=8 * 128 + 1024, K=8, Sc=128, p_in=0.5, n_sparse=1024,
            extra_bridges=4, rounds=2, adv_every=3000, adv_k=3, seed=15, S=0x5EED1004,
            batch=20_000),
    5: dict(name="er1024_p0.3_fixedforest", V=1024, p=0.3, reps=2, seed=16, S=0x5EED1005,
            batch=50_000),
}


def stream_of(cfg: dict):
    """The update stream of a workload description (CONFIGS / SCALED); the
    forest-targeted workload needs an engine and is built with
    ``ForestTargetedDeletes`` instead."""
    if "logV" in cfg:
        return rmat_interleaved(cfg["logV"], cfg["n"], cfg["del_prob"], cfg["seed"])
    if "forest_frac" in cfg:
        raise ValueError("forest-targeted deletions need the current forest: "
                         "use ForestTargetedDeletes")
    if "reps" in cfg:
        return fixed_forest(cfg["V"], cfg["p"], cfg["reps"], cfg["seed"])
    if "K" in cfg:
        return clustered_churn(cfg["K"], cfg["Sc"], cfg["p_in"], cfg["n_sparse"],
                               cfg["extra_bridges"], cfg["rounds"], cfg["adv_every"],
                               cfg["adv_k"], cfg["seed"])
    return er_standard(cfg["V"], cfg["p"], cfg["del_frac"], cfg["seed"])


def config_stream(i: int, scaled: bool = False):
    """The update stream of workload ``i`` as (u, v, is_delete)."""
    return stream_of((SCALED if scaled else CONFIGS)[i])


def ceil_log2(V: int) -> int:
    return max(1, int(math.ceil(math.log2(V))))
