"""Parity of the library with the oracle on the other workload recipes, at
sizes the oracle replays in seconds (same generators, same batch-boundary
rules as the full-size workloads):

* R-MAT with 15% interleaved deletions in ragged, log-uniform batches
  (plain, staged and graph-replayed paths);
* forest-targeted deletions: 30% of deletions hit current forest edges,
  forcing cuts and replacement rounds over components of uneven size, with
  connectivity queries every rho updates, direct and through the serving
  loop;
* clustered churn with adversarial bridge toggles that split and merge
  clusters.
"""
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


def _cd(V):
    C = max(1, math.ceil(math.log2(V)))
    return C, 2 * C


def _truth_labels(V, live):
    eu = np.array([e[0] for e in live], np.uint32)
    ev = np.array([e[1] for e in live], np.uint32)
    return oracle.uf_components(V, eu, ev)[1]


@pytest.fixture(scope="module")
def rmat_ref():
    cfg = streamgen.SCALED[2]
    V = cfg["V"]
    C, D = _cd(V)
    u, v, d = streamgen.config_stream(2, scaled=True)
    sizes = streamgen.ragged_sizes(len(u), cfg["batch"][0], cfg["batch"][1], cfg["seed"])
    sk = oracle.Sketch(V, C, D, cfg["S"])
    fr = oracle.ForestReplay(sk)
    off = 0
    for s in sizes:
        fr.apply_batch(u[off:off + s], v[off:off + s], d[off:off + s])
        off += s
    fu, fv = streamgen.final_edges(u, v, d)
    truth = oracle.components_truth(V, fu, fv)
    return dict(cfg=cfg, V=V, C=C, D=D, u=u, v=v, d=d, sizes=sizes, digest=sk.digest(),
                alpha=sk.alpha.copy(), gamma=sk.gamma.copy(), forest=fr.forest_edges(),
                truth=truth)


@pytest.mark.parametrize("mode,graph,walk_plain,split", [("atomic", False, False, False),
                                                         ("staged", False, False, False),
                                                         ("staged", True, False, False),
                                                         ("staged", False, True, False),
                                                         ("staged", False, False, True)])
def test_rmat_ragged_batches(cupk, rmat_ref, mode, graph, walk_plain, split):
    R = rmat_ref
    sm = cupk.SCATTER_ATOMIC if mode == "atomic" else cupk.SCATTER_STAGED
    ctx = cupk.Context(R["V"], R["C"], R["D"], R["cfg"]["S"], scatter_mode=sm, use_graph=graph,
                       max_batch=4096, walk_plain=walk_plain, split_rounds=split)
    print(f"rmat n={len(R['u'])} batches={len(R['sizes'])} mode={mode} graph={graph} "
          f"walk_plain={walk_plain} split_rounds={split}", flush=True)
    off = 0
    for s in R["sizes"]:
        ctx.apply_updates(R["u"][off:off + s], R["v"][off:off + s], R["d"][off:off + s])
        off += s
    a, g = ctx.get_sketch()
    assert np.array_equal(a, R["alpha"]) and np.array_equal(g, R["gamma"])
    assert ctx.digest() == R["digest"]
    assert ctx.forest_edges() == R["forest"]
    lab = ctx.component_labels()
    truth = R["truth"]
    assert ctx.num_components() == len(set(truth.tolist()))
    assert all(lab[w] == lab[truth[w]] for w in range(R["V"]))
    assert ctx.counters()["sample_failed"] == 0
    ctx.close()


def _forest_targeted_run(cupk, ctx_apply, ctx_query, want_forest_fn, cfg):
    """Drive the forest-targeted generator from the oracle's forest, apply
    every chunk to the oracle and (through ctx_apply) to the library, query
    after each chunk.  Returns (answers, wants, oracle sketch, replay,
    forest-edge deletions, deletions), where wants[i] is the oracle replay's
    answer to query i; every want is also checked here against the live
    graph's connectivity for as long as no oracle sample has failed.

    The deletions hit the forest, whose edges are the sampler's own
    outputs, so the stream depends on the sketch's randomness: it can drain
    every verifying bucket of a vertex, and then a replacement exists that
    no sample finds.  From the first such failure on, the replay's answers
    (and the library's, which must equal them) may differ from the truth."""
    V = cfg["V"]
    C, D = _cd(V)
    g = streamgen.ForestTargetedDeletes(V, cfg["p"], cfg["del_frac"], cfg["forest_frac"],
                                        cfg["seed"], cfg["rho"])
    sk = oracle.Sketch(V, C, D, cfg["S"])
    fr = oracle.ForestReplay(sk)
    live = set()
    rng = np.random.default_rng(cfg["seed"])
    answers, wants = [], []
    last_forest_del = (0, 1)
    n_forest_del = 0

    def step(u, v, d):
        nonlocal last_forest_del, n_forest_del
        fset = set(fr.forest_edges())
        for a, b, x in zip(u.tolist(), v.tolist(), d.tolist()):
            if x:
                live.remove((a, b))
                if (a, b) in fset:
                    last_forest_del = (a, b)
                    n_forest_del += 1
            else:
                live.add((a, b))
        fr.apply_batch(u, v, d)
        ctx_apply(u, v, d)
        # connectivity of the live graph at this point of the stream
        lab = _truth_labels(V, live)
        qa, qb = (int(x) for x in rng.integers(0, V, 2))
        for (x, y) in ((qa, qb), last_forest_del):
            answers.append(ctx_query(x, y))
            wants.append(int(fr.connected(x, y)))
            if fr.n_failed == 0:
                assert wants[-1] == int(lab[x] == lab[y]), (len(wants), x, y)

    for u, v, d in g.insert_chunks():
        step(u, v, d)
    while True:
        fe = fr.forest_edges()
        ch = g.delete_chunk([e[0] for e in fe], [e[1] for e in fe])
        if ch is None:
            break
        step(*ch)
    return answers, wants, sk, fr, n_forest_del, g.k


@pytest.mark.parametrize("split", [False, True])
def test_forest_targeted_deletions_direct(cupk, split):
    """Cuts of forest edges in every chunk: the first replacement round runs
    on the pieces (default) or after a split; both give the oracle's forest
    and counts."""
    cfg = streamgen.SCALED[3]
    V = cfg["V"]
    C, D = _cd(V)
    print(f"forest-targeted split_rounds={split}", flush=True)
    ctx = cupk.Context(V, C, D, cfg["S"], split_rounds=split)
    ans, want, sk, fr, nfd, k = _forest_targeted_run(
        cupk, lambda u, v, d: ctx.apply_updates(u, v, d),
        lambda a, b: int(ctx.connected(a, b)), None, cfg)
    print(f"forest-targeted: {nfd} of {k} deletions hit forest edges; queries {len(ans)}",
          flush=True)
    assert nfd > 0.2 * k
    assert ans == want
    assert ctx.digest() == sk.digest()
    assert ctx.forest_edges() == fr.forest_edges()
    ctr = ctx.counters()
    assert ctr["cuts"] == fr.n_cuts and ctr["rounds"] == fr.n_rounds
    assert ctr["links"] == fr.n_links
    ctx.close()


def test_forest_targeted_deletions_served(cupk):
    cfg = streamgen.SCALED[3]
    V = cfg["V"]
    C, D = _cd(V)
    ctx = cupk.Context(V, C, D, cfg["S"])
    # one device batch per chunk: the serving loop may not merge chunks, so
    # its forest equals the oracle's; queries follow each chunk
    ctx.serve_start(max_batch=cfg["rho"], mem_budget_bytes=8 * cfg["rho"] * 4)
    pending = []

    def apply(u, v, d):
        pending.append(ctx.submit_updates(u, v, d))

    def query(a, b):
        t = ctx.submit_query(a, b)
        return ctx.wait(t)

    ans, want, sk, fr, nfd, k = _forest_targeted_run(cupk, apply, query, None, cfg)
    for t in pending:
        assert ctx.wait(t) == 0
    st = ctx.serve_stats()
    ctx.serve_stop()
    assert ans == want
    assert ctx.digest() == sk.digest()
    assert ctx.forest_edges() == fr.forest_edges()
    assert st["query_p99_us"] >= st["query_p50_us"] > 0
    ctx.close()


@pytest.mark.parametrize("mode,walk_plain", [("atomic", False), ("staged", False),
                                             ("staged", True)])
def test_clustered_churn(cupk, mode, walk_plain):
    """Bridges toggled many times per batch: the flagged runs are walked
    contracted (or one by one), with the oracle's forest, links, cuts and
    rounds either way."""
    cfg = streamgen.SCALED[4]
    V = cfg["V"]
    C, D = _cd(V)
    u, v, d = streamgen.config_stream(4, scaled=True)
    sm = cupk.SCATTER_ATOMIC if mode == "atomic" else cupk.SCATTER_STAGED
    print(f"clusters n={len(u)} mode={mode} walk_plain={walk_plain}", flush=True)
    ctx = cupk.Context(V, C, D, cfg["S"], scatter_mode=sm, walk_plain=walk_plain)
    sk = oracle.Sketch(V, C, D, cfg["S"])
    fr = oracle.ForestReplay(sk)
    B = cfg["batch"]
    live = set()
    rng = np.random.default_rng(3)
    for s in range(0, len(u), B):
        e = min(len(u), s + B)
        ctx.apply_updates(u[s:e], v[s:e], d[s:e])
        fr.apply_batch(u[s:e], v[s:e], d[s:e])
        for a, b, x in zip(u[s:e].tolist(), v[s:e].tolist(), d[s:e].tolist()):
            (live.remove if x else live.add)((a, b))
        lab = _truth_labels(V, live)
        for _ in range(50):
            a, b = (int(x) for x in rng.integers(0, V, 2))
            assert ctx.connected(a, b) == (lab[a] == lab[b])
    assert ctx.digest() == sk.digest()
    assert ctx.forest_edges() == fr.forest_edges()
    ctr = ctx.counters()
    assert (ctr["links"], ctr["cuts"], ctr["rounds"]) == (fr.n_links, fr.n_cuts, fr.n_rounds)
    if walk_plain:
        assert ctr["walks_contracted"] == 0
    else:
        assert ctr["walks_contracted"] > 0
    ctx.close()


@pytest.mark.parametrize("mode", ["atomic", "staged"])
def test_fixed_forest_stream(cupk, mode):
    # the forest first, then every other edge inserted and deleted twice:
    # the forest never changes after it is built and no update is a cut
    cfg = streamgen.SCALED[5]
    V = cfg["V"]
    C, D = _cd(V)
    u, v, d = streamgen.config_stream(5, scaled=True)
    sm = cupk.SCATTER_ATOMIC if mode == "atomic" else cupk.SCATTER_STAGED
    ctx = cupk.Context(V, C, D, cfg["S"], scatter_mode=sm)
    sk = oracle.Sketch(V, C, D, cfg["S"])
    fr = oracle.ForestReplay(sk)
    B = cfg["batch"]
    print(f"fixed forest n={len(u)} mode={mode}", flush=True)
    for s in range(0, len(u), B):
        ctx.apply_updates(u[s:s + B], v[s:s + B], d[s:s + B])
        fr.apply_batch(u[s:s + B], v[s:s + B], d[s:s + B])
    assert ctx.digest() == sk.digest()
    assert ctx.forest_edges() == fr.forest_edges()
    fu, fv = streamgen.final_edges(u, v, d)
    assert set(ctx.forest_edges()) == set(zip(fu.tolist(), fv.tolist()))
    ctr = ctx.counters()
    assert ctr["cuts"] == 0 and ctr["links"] == len(fu) == fr.n_links
    ctx.close()
