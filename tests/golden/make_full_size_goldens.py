"""Write tests/golden/full_size_parity.json: what the CPU oracle computes for
two long workload streams at their full vertex count and sketch size, for
the full-size GPU parity tests.

Per workload: the digest of the whole oracle sketch after the stream, the
exact nonzero buckets of eight sampled vertices, and the partition of the
final graph (number of components, and a SHA-256 of the array that labels
every vertex with the smallest vertex of its component).  The final edge set
is taken from the stream alone: an edge is live at the end iff it occurs an
odd number of times (a legal stream toggles it).  Connectivity truth is the
oracle's union-find over that edge set.

  clusters64x2048_churn  the whole stream (setup phase and 11 churn rounds,
                         1.48e9 updates; V = 2^20, C = 20, D = 40)
  rmat17_del15           the first 1e8 of its 5e8 updates (V = 2^17, C = 17,
                         D = 34): the generator is sequential and draws the
                         whole stream in about 3 minutes on one core
  er65536_p0.2_forestdel the digest after its insert phase (4.3e8 inserts; its
                         deletions are drawn from the engine's forest)

Calls only the oracle and the stream generators.  Run from the repository
root (about 10 minutes on 8 cores, 16 GB of memory):
    python tests/golden/make_full_size_goldens.py
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import streamgen  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "full_size_parity.json")
RMAT_PREFIX = 100_000_000
THREADS = os.cpu_count() or 1


def odd_keys(keys):
    """Keys that occur an odd number of times (sorted)."""
    k = np.sort(keys)
    if k.size == 0:
        return k
    starts = np.flatnonzero(np.concatenate([[True], k[1:] != k[:-1]]))
    counts = np.diff(np.concatenate([starts, [k.size]]))
    return k[starts[counts % 2 == 1]]


def partition_sha(labels):
    return hashlib.sha256(np.ascontiguousarray(labels, np.uint32).tobytes()).hexdigest()


def record(name, V, C, D, S, phases, sample_vertices):
    t0 = time.time()
    sk = oracle.Sketch(V, C, D, S)
    live = np.zeros(0, np.uint64)
    n = 0
    for k, (u, v) in enumerate(phases):
        sk.apply_threads(u, v, THREADS)
        live = np.setxor1d(live, odd_keys(u.astype(np.uint64) * V + v), assume_unique=True)
        n += len(u)
        print(f"{name}: phase {k}, {n} updates, {len(live)} live edges, "
              f"{time.time() - t0:.0f} s", flush=True)
    fu = (live // V).astype(np.uint32)
    fv = (live % V).astype(np.uint32)
    ncomp, lab = oracle.uf_components(V, fu, fv)
    slabs = {}
    a, g = sk.alpha, sk.gamma
    for w in sample_vertices:
        nz = np.argwhere((a[w] != 0) | (g[w] != 0))
        slabs[str(w)] = [[int(c), int(d), "0x%016x" % int(a[w, c, d]), "0x%016x" % int(g[w, c, d])]
                         for c, d in nz]
    res = {"V": V, "C": C, "D": D, "S": S, "n_updates": n, "digest": "0x%016x" % sk.digest(),
           "live_edges": int(len(live)), "n_components": ncomp,
           "partition_sha256": partition_sha(lab), "slabs": slabs}
    print(f"{name}: digest {res['digest']}, {ncomp} components, {time.time() - t0:.0f} s",
          flush=True)
    return res


def clusters():
    cfg = streamgen.CONFIGS[4]
    V = cfg["V"]
    C = streamgen.ceil_log2(V)
    rng = np.random.default_rng(404)
    ncl = cfg["K"] * cfg["Sc"]
    ws = sorted(set([0, ncl - 1, ncl, V - 1] + rng.integers(0, ncl, 3).tolist() +
                    rng.integers(ncl, V, 2).tolist()))

    def phases():
        for ph in streamgen.clustered_phases(cfg):
            u, v, _ = streamgen.unpack(ph)
            yield u, v

    return record(cfg["name"], V, C, 2 * C, cfg["S"], phases(), ws)


def rmat():
    cfg = streamgen.CONFIGS[2]
    V = cfg["V"]
    C = streamgen.ceil_log2(V)
    rng = np.random.default_rng(202)
    ws = sorted(set([0, 1, 2, 3, V - 1] + rng.integers(0, V, 4).tolist()))

    def phases():
        for u, v, _ in streamgen.rmat_chunks(cfg["logV"], RMAT_PREFIX, cfg["del_prob"],
                                             cfg["seed"]):
            yield u, v

    res = record(cfg["name"] + "_first1e8", V, C, 2 * C, cfg["S"], phases(), ws)
    res["prefix"] = RMAT_PREFIX
    return res


def forest_targeted_inserts():
    """Digest after the insert phase of er65536_p0.2_forestdel (4.3e8
    inserts; the deletions that follow depend on the engine's forest)."""
    cfg = streamgen.CONFIGS[3]
    V = cfg["V"]
    C = streamgen.ceil_log2(V)
    g = streamgen.ForestTargetedDeletes(V, cfg["p"], cfg["del_frac"], cfg["forest_frac"],
                                        cfg["seed"], cfg["rho"])
    t0 = time.time()
    sk = oracle.Sketch(V, C, 2 * C, cfg["S"])
    buf = []
    for ch in g.insert_chunks_packed():
        buf.append(ch)
        if len(buf) == 200:
            u, v, _ = streamgen.unpack(np.concatenate(buf))
            sk.apply_threads(u, v, THREADS)
            buf = []
    if buf:
        u, v, _ = streamgen.unpack(np.concatenate(buf))
        sk.apply_threads(u, v, THREADS)
    res = {"V": V, "C": C, "D": 2 * C, "S": cfg["S"], "n_inserts": int(g.m),
           "digest": "0x%016x" % sk.digest()}
    print(f"{cfg['name']} inserts: digest {res['digest']}, {time.time() - t0:.0f} s", flush=True)
    return res


def main():
    out = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            out = json.load(f)
    which = sys.argv[1:] or ["clusters", "rmat", "forest_targeted"]
    if "forest_targeted" in which:
        out["er65536_p0.2_forestdel_inserts"] = forest_targeted_inserts()
    if "rmat" in which:
        out["rmat17_del15_first1e8"] = rmat()
    if "clusters" in which:
        out["clusters64x2048_churn"] = clusters()
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
        f.write("\n")


if __name__ == "__main__":
    main()
