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

import math
import numpy as np

__all__ = [
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
}


def config_stream(i: int):
    """The update stream of workload ``i`` (0 or 1) as (u, v, is_delete)."""
    cfg = CONFIGS[i]
    return er_standard(cfg["V"], cfg["p"], cfg["del_frac"], cfg["seed"])


def ceil_log2(V: int) -> int:
    return max(1, int(math.ceil(math.log2(V))))
