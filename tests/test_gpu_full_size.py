"""Full-size parity of the largest workloads.

clusters64x2048_churn (V = 2^20, C = 20, D = 40, 13.4 GB of sketches, 1.48e9
updates) runs in the launch configuration the benchmark times: lane layout,
geometry and batch size from the autotuner on a warm-up context (64M-update
sample), then the setup phase and all 11 churn rounds.  rmat17_del15 runs the first 1e8 of its updates (full V,
C, D and recipe) in its ragged batches.  Both are compared with what the
oracle computed for the same streams (tests/golden/full_size_parity.json,
written by tests/golden/make_full_size_goldens.py, which calls only the
oracle and the stream generators): the whole-sketch digest, the exact
sketches of eight sampled vertices, and the partition of the final graph
(union-find over its edges); the forest must be acyclic and span that
partition.

er65536_p0.2_forestdel runs whole (4.7e8 updates): G(65536, 0.2) inserts,
then deletions chunk by chunk, 30% of them on the library's current forest
edges, with two queries after every 1e5-update chunk (a random pair and the
endpoints of the last deleted forest edge).  Truth: while edges are only
inserted, a union-find over the edges so far; during the deletions every
graph contains the final one, and the test checks that never-deleted edges
alone connect all vertices, so the true answer there is always 1.  Those
deletions depend on the library's forest, so they can drain a sampler (see
the test); answers are exact up to the first failed sample, and every
failure is one the oracle's sampler shows on the same sketch.
"""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle
import streamgen

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "full_size_parity.json")


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU test on a machine without a GPU"
    import paper_2509_14433_amd as cupk
    with open(GOLDEN) as f:
        gold = json.load(f)
    return cupk, torch, gold


def _canonical_sha(lab):
    """SHA-256 of the labelling that maps every vertex to the smallest vertex
    carrying its label."""
    lab = np.asarray(lab)
    order = np.argsort(lab, kind="stable")
    sl = lab[order]
    starts = np.flatnonzero(np.concatenate([[True], sl[1:] != sl[:-1]]))
    counts = np.diff(np.concatenate([starts, [len(sl)]]))
    canon = np.empty(len(lab), np.uint32)
    canon[order] = np.repeat(order[starts].astype(np.uint32), counts)
    return hashlib.sha256(canon.tobytes()).hexdigest(), len(starts)


def _check_against_golden(ctx, g):
    V = g["V"]
    assert ctx.digest() == int(g["digest"], 16)
    for w, buckets in g["slabs"].items():
        a, gm = ctx.get_sketch(int(w), 1)
        ea = np.zeros_like(a[0])
        eg = np.zeros_like(gm[0])
        for c, d, x, h in buckets:
            ea[c, d] = int(x, 16)
            eg[c, d] = int(h, 16)
        assert np.array_equal(a[0], ea) and np.array_equal(gm[0], eg), f"vertex {w}"
    sha, k = _canonical_sha(ctx.component_labels())
    assert k == g["n_components"] and sha == g["partition_sha256"]
    assert ctx.num_components() == g["n_components"]
    fu, fv = ctx.forest_edge_arrays()
    assert len(fu) == V - g["n_components"]
    nf, flab = oracle.uf_components(V, fu, fv)
    assert nf == g["n_components"]               # acyclic: V - |F| trees
    assert _canonical_sha(flab)[0] == g["partition_sha256"]


def test_clusters_full_size_in_the_benchmark_configuration(env):
    cupk, torch, gold = env
    g = gold["clusters64x2048_churn"]
    cfg = streamgen.CONFIGS[4]
    V, C, D, S = g["V"], g["C"], g["D"], g["S"]
    phases = []
    for k, ph in enumerate(streamgen.clustered_phases(cfg)):
        phases.append(torch.from_numpy(ph.view(np.int64)).to("cuda"))
        print(f"clusters: phase {k} drawn, {len(ph)} updates", flush=True)
    assert sum(int(p.shape[0]) for p in phases) == g["n_updates"]
    one_m = 1_000_000

    def apply(ctx, ph, b):
        for s in range(0, ph.shape[0], b):
            ctx.apply_updates_device(ph[s:s + b])

    # the benchmark's tuning: a warm-up context with 8 batches of host
    # history, then the autotuner on a 64M-update sample of round 0
    w = cupk.Context(V, C, D, S, max_batch=one_m)
    apply(w, phases[0], one_m)
    apply(w, phases[1][:8 * one_m], one_m)
    tuned = w.autotune(phases[1][8 * one_m:8 * one_m + (1 << 26)].contiguous())
    w.close()
    batch = tuned["batch_target"]
    print(f"clusters: tuned layout {tuned['tile_layout']} {tuned['tile_vertices']} "
          f"{tuned['lds_rows']} "
          f"{tuned['chunk_records']} coarse {tuned['coarse_tiles']} batch {batch}", flush=True)
    ctx = cupk.Context(V, C, D, S, max_batch=batch, tile_vertices=tuned["tile_vertices"],
                       lds_rows=tuned["lds_rows"], chunk_records=tuned["chunk_records"],
                       tile_layout=tuned["tile_layout"], coarse_tiles=tuned["coarse_tiles"])
    for k, ph in enumerate(phases):
        apply(ctx, ph, batch)
        ctx.sync()
        print(f"clusters: phase {k} applied", flush=True)
    del phases
    _check_against_golden(ctx, g)
    ctr = ctx.counters()
    assert ctr["cuts"] > 0 and ctr["rounds"] > 0
    ctx.close()


def test_rmat17_prefix_full_size(env):
    cupk, torch, gold = env
    g = gold["rmat17_del15_first1e8"]
    cfg = streamgen.CONFIGS[2]
    V, C, D, S = g["V"], g["C"], g["D"], g["S"]
    n = g["prefix"]
    packed = torch.empty(n, dtype=torch.int64, device="cuda")
    off = 0
    for u, v, d in streamgen.rmat_chunks(cfg["logV"], n, cfg["del_prob"], cfg["seed"]):
        m = len(u)
        packed[off:off + m].copy_(torch.from_numpy(cupk.pack_updates(u, v, d).view(np.int64)))
        off += m
        print(f"rmat17: {off} updates drawn", flush=True)
    sizes = streamgen.ragged_sizes(n, cfg["batch"][0], cfg["batch"][1], cfg["seed"])
    ctx = cupk.Context(V, C, D, S, max_batch=max(sizes))
    ctx.autotune(packed[: 1 << 22].contiguous())
    off = 0
    for k, sz in enumerate(sizes):
        ctx.apply_updates_device(packed[off:off + sz])
        off += sz
    ctx.sync()
    print(f"rmat17: {len(sizes)} ragged batches applied", flush=True)
    _check_against_golden(ctx, g)
    ctx.close()


def _incident_updates(chunks, members, V):
    """The updates of `chunks` (packed) with an endpoint in `members`."""
    inset = np.zeros(V, bool)
    inset[np.asarray(members, np.int64)] = True
    us, vs = [], []
    for ch in chunks:
        u, v, _ = streamgen.unpack(ch)
        m = inset[u] | inset[v]
        us.append(u[m])
        vs.append(v[m])
    return np.concatenate(us), np.concatenate(vs)


def _check_failed_trees(ctx, cfg, C, chunks, V, limit=6):
    """Every tree of the forest but the largest: its set sketch equals the
    oracle's, built from the updates incident to its members, and the
    oracle's sampler fails on it as well (status 2).  Checks the `limit`
    smallest such trees; returns how many trees there are."""
    lab = ctx.component_labels()
    roots, counts = np.unique(lab, return_counts=True)
    order = np.argsort(counts, kind="stable")
    others = [int(r) for r in roots[order[:-1]]]
    if not others:
        return 0
    trees = [np.flatnonzero(lab == r).astype(np.uint32) for r in others[:limit]]
    members = np.concatenate(trees)
    u, v = _incident_updates(chunks, members, V)
    sk = oracle.Sketch(V, C, 2 * C, cfg["S"])
    sk.apply(u, v)
    for t in trees:
        la, lg = ctx.component_sketch(t)
        oa, og = sk.set_sketch(t)
        assert np.array_equal(la, oa) and np.array_equal(lg, og), f"tree of {int(t[0])}"
        st, _, _ = sk.sample(oa, og)
        assert st == 2, (f"tree of {int(t[0])} ({len(t)} vertices): the oracle's sampler "
                         f"returns status {st}, the library's forest left it unmerged")
    return len(others)


def test_forest_targeted_deletions_full_size(env):
    """The deletions of this workload are drawn from the library's current
    forest, so they depend on the sketch's own samples: an adaptive
    adversary, outside the w.h.p. guarantee of a stream fixed in advance
    (Sec. 2.2.1, Sec. 2.2.2).  What is checked is what holds regardless:
    the sketch equals the oracle's (the insert-phase digest, and the set
    sketch of every tree the rounds left unmerged), every answer is exact
    until the first failed sample, a tree is left unmerged only where the
    oracle's sampler fails on the very same sketch, and the forest is
    always a forest of live edges."""
    cupk, torch, gold = env
    g = gold["er65536_p0.2_forestdel_inserts"]
    cfg = streamgen.CONFIGS[3]
    V = cfg["V"]
    C = streamgen.ceil_log2(V)
    assert (g["V"], g["C"], g["D"], g["S"]) == (V, C, 2 * C, cfg["S"])
    rho = cfg["rho"]
    gen = streamgen.ForestTargetedDeletes(V, cfg["p"], cfg["del_frac"], cfg["forest_frac"],
                                          cfg["seed"], rho)
    print(f"forest-targeted: {gen.m} inserts, {gen.k} deletions", flush=True)
    assert gen.m == g["n_inserts"]
    ctx = cupk.Context(V, C, 2 * C, cfg["S"], max_batch=rho)
    uf = oracle.UnionFind(V)
    rng = np.random.default_rng(cfg["seed"])
    chunks = []         # every update so far, packed
    early = []          # the first 4e6 inserts (to show the final graph connected)
    bad = 0
    for k, ch in enumerate(gen.insert_chunks_packed()):
        ctx.apply_updates_device(torch.from_numpy(ch.view(np.int64)).to("cuda"))
        chunks.append(ch)
        u, v, _ = streamgen.unpack(ch)
        uf.add(u, v)
        if len(early) < 40:
            early.append(ch)
        a, b = (int(x) for x in rng.integers(0, V, 2))
        bad += int(ctx.connected(a, b)) != int(uf.same(a, b))
        if k % 500 == 0:
            print(f"forest-targeted: insert chunk {k}, {uf.n_components} components", flush=True)
    assert bad == 0
    assert ctx.digest() == int(g["digest"], 16)
    assert uf.n_components == 1 and ctx.num_components() == 1
    dels = []
    last = (0, 1)
    n_forest_del = 0
    first_fail = None   # deletion chunk of the first failed sample
    exact = []          # answers up to the first failed sample
    later = []          # answers after it
    while True:
        fu, fv = ctx.forest_edge_arrays()
        fkeys = fu.astype(np.uint64) * np.uint64(V) + fv
        ch = gen.delete_chunk_packed(fkeys)
        if ch is None:
            break
        ctx.apply_updates_device(torch.from_numpy(ch.view(np.int64)).to("cuda"))
        chunks.append(ch)
        u, v, _ = streamgen.unpack(ch)
        keys = u.astype(np.uint64) * np.uint64(V) + v
        dels.append(keys)
        hit = np.flatnonzero(np.isin(keys, fkeys))
        n_forest_del += len(hit)
        if len(hit):
            last = (int(u[hit[-1]]), int(v[hit[-1]]))
        a, b = (int(x) for x in rng.integers(0, V, 2))
        ans = [int(ctx.connected(a, b)), int(ctx.connected(*last))]
        failed = ctx.counters()["sample_failed"]
        if failed and first_fail is None:
            first_fail = len(dels)
            n_other = _check_failed_trees(ctx, cfg, C, chunks, V)
            print(f"forest-targeted: first failed sample in deletion chunk {first_fail}, "
                  f"{n_other} trees left unmerged", flush=True)
        if first_fail is None:
            exact += ans
            assert ctx.num_components() == 1, f"deletion chunk {len(dels)}"
        else:
            later += ans
        if len(dels) % 100 == 0:
            print(f"forest-targeted: deletion chunk {len(dels)}", flush=True)
    ctr = ctx.counters()
    print(f"forest-targeted: {n_forest_del} forest-edge deletions of {gen.k}, cuts "
          f"{ctr['cuts']}, rounds {ctr['rounds']}, failed {ctr['sample_failed']}, "
          f"first failure in chunk {first_fail}, {later.count(0)} of {len(later)} later "
          f"answers 0", flush=True)
    assert n_forest_del > 0 and ctr["cuts"] >= n_forest_del
    # never-deleted early inserts alone connect every vertex, so every graph
    # of the deletion phase (each contains them) is connected
    deleted = np.sort(np.concatenate(dels))
    e = np.concatenate(early)
    eu, ev, _ = streamgen.unpack(e)
    ek = eu.astype(np.uint64) * np.uint64(V) + ev
    keep = ~np.isin(ek, deleted, assume_unique=True)
    k_final, _ = oracle.uf_components(V, eu[keep], ev[keep])
    assert k_final == 1
    assert exact and all(x == 1 for x in exact)
    # the final forest: live edges only (inserted, not deleted), acyclic,
    # one tree per component the library reports; every tree but the
    # largest is one whose sample fails in the oracle too
    fu, fv = ctx.forest_edge_arrays()
    fk = np.sort(fu.astype(np.uint64) * np.uint64(V) + fv)
    assert not np.isin(fk, deleted).any()
    found = np.zeros(len(fk), bool)
    for ch in chunks[: len(chunks) - len(dels)]:
        u, v, _ = streamgen.unpack(ch)
        ik = (np.minimum(u, v).astype(np.uint64) * np.uint64(V) + np.maximum(u, v))
        idx = np.minimum(np.searchsorted(fk, ik), len(fk) - 1)
        m = fk[idx] == ik
        found[idx[m]] = True
    assert found.all()
    nf, _ = oracle.uf_components(V, fu, fv)
    assert nf == V - len(fu) == ctx.num_components()
    n_other = _check_failed_trees(ctx, cfg, C, chunks, V)
    assert n_other == ctx.num_components() - 1
    assert (ctr["sample_failed"] > 0) == (first_fail is not None)
    ctx.close()
