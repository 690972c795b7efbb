"""Parity of the HIP path with the CPU oracle (bit-exact).

Every case runs the same seeded stream through the library (via the C ABI)
and through the oracle with the same batch boundaries, then compares the
whole sketch array, the digest, the forest edges, component sketches and
samples.  Sizes span several vertex tiles and leave a ragged last tile and
a ragged last batch.
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
    assert torch.cuda.is_available(), "GPU test on a machine without a GPU"
    import paper_2509_14433_amd as m
    return m


# "staged": the staged scatter in the record layout (the default at these
# batch sizes); "pair": the staged scatter in the pair layout
MODES = ["atomic", "staged", "pair"]


def _mode(cupk, name):
    return cupk.SCATTER_ATOMIC if name == "atomic" else cupk.SCATTER_STAGED


def _mkw(cupk, name):
    """Context keyword arguments of a scatter mode name."""
    kw = {"scatter_mode": _mode(cupk, name)}
    if name == "pair":
        kw["tile_layout"] = cupk.LAYOUT_PAIR
    elif name == "staged":
        kw["tile_layout"] = cupk.LAYOUT_RECORD
    return kw


def _replay(cupk, mode, V, C, D, S, u, v, d, bs, **kw):
    ctx = cupk.Context(V, C, D, S, **_mkw(cupk, mode), **kw)
    ref = oracle.Sketch(V, C, D, S)
    fr = oracle.ForestReplay(ref)
    n = len(u)
    bs = n if bs is None else bs
    for s in range(0, n, bs):
        e = min(n, s + bs)
        print(f"batch {s}:{e}", flush=True)
        ctx.apply_updates(u[s:e], v[s:e], d[s:e])
        fr.apply_batch(u[s:e], v[s:e], d[s:e])
    return ctx, ref, fr


def _assert_same_sketch(ctx, ref):
    a, g = ctx.get_sketch()
    assert a.shape == ref.alpha.shape
    bad = np.argwhere((a != ref.alpha) | (g != ref.gamma))
    assert bad.size == 0, f"{len(bad)} buckets differ, first (w,c,d) = {bad[:5].tolist()}"
    assert ctx.digest() == ref.digest()


CASES = [
    # V, p, del_frac, batch, tile_vertices, lds_rows
    (200, 0.15, 0.4, 97, 8, 0),
    (200, 0.15, 0.4, None, 0, 0),
    (333, 0.1, 0.5, 1000, 16, 2),
    (1000, 0.02, 0.3, 777, 4, 0),
    (2, 1.0, 0.0, None, 0, 0),
    # one vertex per tile: 2048 tiles (the most for which classify blocks
    # store their bin starts), then 2049 (fill reserves per record)
    (2048, 0.004, 0.3, 5000, 1, 0),
    (2049, 0.004, 0.3, 5000, 1, 0),
]


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("V,p,df,bs,tv,rows", CASES)
def test_stream_parity(cupk, mode, V, p, df, bs, tv, rows):
    C = max(1, math.ceil(math.log2(V)))
    D = 2 * C
    S = 0x5EED0000 + V
    u, v, d = streamgen.er_standard(V, p, df, V * 7 + 1)
    print(f"case V={V} n={len(u)} mode={mode} bs={bs} tv={tv} rows={rows}", flush=True)
    ctx, ref, fr = _replay(cupk, mode, V, C, D, S, u, v, d, bs, tile_vertices=tv,
                           lds_rows=rows)
    _assert_same_sketch(ctx, ref)
    assert ctx.forest_edges() == fr.forest_edges()
    fu, fv = streamgen.final_edges(u, v, d)
    truth = oracle.components_truth(V, fu, fv)
    lab = ctx.component_labels()
    assert ctx.num_components() == len(set(truth.tolist()))
    for w in range(V):
        assert (lab[w] == lab[truth[w]])
    # queries
    rng = np.random.default_rng(V)
    for _ in range(200):
        a, b = (int(x) for x in rng.integers(0, V, 2))
        assert ctx.connected(a, b) == (truth[a] == truth[b])
    ctx.close()


@pytest.mark.parametrize("mode", MODES)
def test_hot_vertex_star(cupk, mode):
    # every update touches vertex 0: one tile's bin spans several work items
    # (multi-chunk fold with device atomics) and LDS atomics collide
    V, C, D, S = 6000, 5, 10, 99
    u, v, d = streamgen.star_stream(V, 12000, 5)
    print(f"star n={len(u)} mode={mode}", flush=True)
    ctx, ref, fr = _replay(cupk, mode, V, C, D, S, u, v, d, 9000)
    _assert_same_sketch(ctx, ref)
    assert ctx.forest_edges() == fr.forest_edges()
    ctx.close()


@pytest.mark.parametrize("mode", MODES)
def test_config0_full(cupk, mode):
    V, C, D, S = 1024, 10, 20, 0x5EED0000
    u, v, d = streamgen.config_stream(0)
    for bs in (None, 65536):
        print(f"config0 bs={bs} mode={mode}", flush=True)
        ctx, ref, fr = _replay(cupk, mode, V, C, D, S, u, v, d, bs)
        _assert_same_sketch(ctx, ref)
        assert ctx.forest_edges() == fr.forest_edges()
        fu, fv = streamgen.final_edges(u, v, d)
        truth = oracle.components_truth(V, fu, fv)
        lab = ctx.component_labels()
        # all 523,776 pairs: equal partitions
        assert len(set(lab.tolist())) == len(set(truth.tolist()))
        pairs = {}
        for w in range(V):
            pairs.setdefault(int(lab[w]), set()).add(int(truth[w]))
        assert all(len(s) == 1 for s in pairs.values())
        ctx.close()


def test_component_sketch_and_sample_parity(cupk):
    V, C, D, S = 300, 9, 18, 4321
    u, v, d = streamgen.er_standard(V, 0.05, 0.3, 77)
    ctx, ref, fr = _replay(cupk, "staged", V, C, D, S, u, v, d, 500)
    rng = np.random.default_rng(1)
    sets = [np.array([], np.uint32), np.arange(V, dtype=np.uint32),
            np.array([5], np.uint32)]
    for _ in range(40):
        k = int(rng.integers(1, V))
        sets.append(np.sort(rng.choice(V, size=k, replace=False)).astype(np.uint32))
    ga, gg = ctx.component_sketch_batch(sets)
    for j, s in enumerate(sets):
        oa, og = ref.set_sketch(s)
        assert np.array_equal(ga[j], oa) and np.array_equal(gg[j], og), j
        one_a, one_g = ctx.component_sketch(s)
        assert np.array_equal(one_a, oa) and np.array_equal(one_g, og)
        assert ctx.sample_cut_edge(oa, og) == ref.sample(oa, og)
    st, su, sv = ctx.sample_cut_edge_batch(ga, gg)
    for j in range(len(sets)):
        want = ref.sample(ga[j], gg[j])
        assert (int(st[j]), int(su[j]) if st[j] == 0 else 0, int(sv[j]) if st[j] == 0 else 0) \
            == want
    ctx.close()


def test_sample_statuses(cupk):
    # EMPTY for a whole component, SAMPLE_FAILED for two colliding indices
    V, C, D, S = 1000, 1, 4, 55
    ctx = cupk.Context(V, C, D, S)
    ref = oracle.Sketch(V, C, D, S)
    first, pair = {}, None
    for b in range(1, V):
        x = oracle.edge_index(V, 0, b)
        dd = oracle.depth_of_hash(oracle.hash_c(S, 0, x), D)
        if dd in first:
            pair = (first[dd], b)
            break
        first[dd] = b
    uu = np.array([0, 0], np.uint32)
    vv = np.array(pair, np.uint32)
    ctx.apply_updates(uu, vv, np.zeros(2, np.uint8))
    ref.apply(uu, vv)
    a, g = ctx.component_sketch([0])
    assert ctx.sample_cut_edge(a, g)[0] == cupk.SAMPLE_FAILED
    assert ref.sample(a, g)[0] == oracle.FAILED
    a, g = ctx.component_sketch([0, int(pair[0]), int(pair[1])])
    assert ctx.sample_cut_edge(a, g)[0] == cupk.EMPTY
    ctx.close()


@pytest.mark.parametrize("mode", MODES)
def test_invalid_batch_applies_nothing(cupk, mode):
    V, C, D, S = 100, 7, 14, 3
    ctx = cupk.Context(V, C, D, S, **_mkw(cupk, mode))
    u, v, d = streamgen.er_standard(V, 0.1, 0.0, 4)
    ctx.apply_updates(u, v, d)
    dg = ctx.digest()
    edges = ctx.forest_edges()
    for bad in ((5, 5), (3, 100)):
        uu = np.array([1, bad[0], 2], np.uint32)
        vv = np.array([9, bad[1], 8], np.uint32)
        with pytest.raises(cupk.CupkError) as ei:
            ctx.apply_updates(uu, vv, np.zeros(3, np.uint8))
        assert ei.value.code == cupk.EINVAL
        # the device path validates on the GPU; the call that completes the
        # batch's host part (here cupk_sync) reports it
        import torch
        packed = torch.from_numpy(cupk.pack_updates(uu, vv, np.zeros(3)).view(np.int64)).cuda()
        ctx.apply_updates_device(packed)
        with pytest.raises(cupk.CupkError) as ei:
            ctx.sync()
        assert ei.value.code == cupk.EINVAL
        # reported once: the context goes on
        ctx.sync()
    assert ctx.digest() == dg and ctx.forest_edges() == edges
    ctx.apply_updates(np.zeros(0, np.uint32), np.zeros(0, np.uint32), np.zeros(0, np.uint8))
    assert ctx.digest() == dg
    ctx.close()


@pytest.mark.parametrize("mode", MODES)
def test_device_batches_match_host_batches(cupk, mode):
    import torch
    V, C, D, S = 500, 9, 18, 8
    u, v, d = streamgen.er_standard(V, 0.08, 0.5, 12)
    # endpoints in either order on the device path
    sw = np.arange(len(u)) % 2 == 1
    uu = np.where(sw, v, u)
    vv = np.where(sw, u, v)
    packed = torch.from_numpy(cupk.pack_updates(uu, vv, d).view(np.int64)).cuda()
    ctx = cupk.Context(V, C, D, S, **_mkw(cupk, mode))
    ref = oracle.Sketch(V, C, D, S)
    fr = oracle.ForestReplay(ref)
    bs = 3001
    for s in range(0, len(u), bs):
        e = min(len(u), s + bs)
        ctx.apply_updates_device(packed[s:e])
        fr.apply_batch(u[s:e], v[s:e], d[s:e])
    _assert_same_sketch(ctx, ref)
    assert ctx.forest_edges() == fr.forest_edges()
    ctx.close()


def test_autotune_leaves_sketch_unchanged_and_parity_holds(cupk):
    import torch
    V, C, D, S = 3000, 12, 24, 31337
    u, v, d = streamgen.er_standard(V, 0.02, 0.3, 8)
    half = len(u) // 2
    ctx = cupk.Context(V, C, D, S)
    ref = oracle.Sketch(V, C, D, S)
    fr = oracle.ForestReplay(ref)
    ctx.apply_updates(u[:half], v[:half], d[:half])
    fr.apply_batch(u[:half], v[:half], d[:half])
    dg = ctx.digest()
    sample = torch.from_numpy(cupk.pack_updates(u, v, d).view(np.int64)).cuda()
    res = ctx.autotune(sample)
    print(res, flush=True)
    assert ctx.digest() == dg
    # (the best few are timed again: the chosen one's second timing may sit
    # a little above the first timing of the setting in force before)
    assert res["candidates"] > 10 and res["best_ms"] <= 1.1 * res["before_ms"]
    assert res["tile_vertices"] in (4, 8, 16, 32, 64)
    assert res["batch_target"] in res["batch_sizes"]
    ctx.apply_updates(u[half:], v[half:], d[half:])
    fr.apply_batch(u[half:], v[half:], d[half:])
    _assert_same_sketch(ctx, ref)
    assert ctx.forest_edges() == fr.forest_edges()
    ctx.close()


@pytest.mark.parametrize("V,p,bs", [(3000, 0.002, None), (3000, 0.01, 20000), (500, 0.3, 9000)])
def test_insert_only_batches(cupk, V, p, bs):
    # batches whose flagged updates are all inserts take the union-find walk
    # (with early stop once one tree remains) and bulk linking; sparse cases
    # end with many trees, dense ones with one
    C = math.ceil(math.log2(V))
    D = 2 * C
    S = 4242
    u, v, d = streamgen.er_standard(V, p, 0.0, 40 + V)
    ctx, ref, fr = _replay(cupk, "staged", V, C, D, S, u, v, d, bs)
    assert ctx.forest_edges() == fr.forest_edges()
    assert ctx.num_components() == len(set(fr.labels().tolist()))
    _assert_same_sketch(ctx, ref)
    ctx.close()


@pytest.mark.parametrize("mode", MODES)
def test_graph_replay_ragged_batches(cupk, mode):
    # captured graphs are replayed for ragged batch sizes (the kernels read
    # the size from device memory), re-captured when the capacity grows, and
    # checked against the oracle between replays
    V, C, D, S = 700, 10, 20, 9
    u, v, d = streamgen.er_standard(V, 0.05, 0.5, 99)
    sizes = streamgen.ragged_sizes(len(u), 1, 3000, 5)
    ctx = cupk.Context(V, C, D, S, **_mkw(cupk, mode), use_graph=True, max_batch=512)
    ref = oracle.Sketch(V, C, D, S)
    fr = oracle.ForestReplay(ref)
    off = 0
    for k, sz in enumerate(sizes):
        ctx.apply_updates(u[off:off + sz], v[off:off + sz], d[off:off + sz])
        fr.apply_batch(u[off:off + sz], v[off:off + sz], d[off:off + sz])
        off += sz
        if k % 7 == 0:
            assert ctx.digest() == ref.digest(), k
    assert off == len(u) and len(sizes) > 10
    _assert_same_sketch(ctx, ref)
    assert ctx.forest_edges() == fr.forest_edges()
    ctx.close()


@pytest.mark.parametrize("mode", MODES)
def test_small_batch_boundary(cupk, mode):
    # batches just below, at and above the small-batch limit (4096), and a
    # batch of one, in sequence: both batch paths must agree with the oracle
    V, C, D, S = 700, 10, 20, 0x5EED77
    u, v, d = streamgen.er_standard(V, 0.05, 0.5, 12)
    sizes = [4095, 4096, 4097, 1, 3000]
    assert len(u) >= sum(sizes)
    ctx = cupk.Context(V, C, D, S, **_mkw(cupk, mode))
    ref = oracle.Sketch(V, C, D, S)
    fr = oracle.ForestReplay(ref)
    off = 0
    for sz in sizes + [len(u) - sum(sizes)]:
        print(f"boundary batch {off}:{off + sz} mode={mode}", flush=True)
        ctx.apply_updates(u[off:off + sz], v[off:off + sz], d[off:off + sz])
        fr.apply_batch(u[off:off + sz], v[off:off + sz], d[off:off + sz])
        off += sz
    _assert_same_sketch(ctx, ref)
    assert ctx.forest_edges() == fr.forest_edges()
    ctx.close()


@pytest.mark.parametrize("mode", MODES)
def test_flag_list_boundary(cupk, mode):
    # Batches above the small-batch limit whose every update is flagged:
    # 16384 flags (the longest list that comes back with the batch header)
    # and 16385 (compacted and copied), then deletions of tree edges mixed
    # with inserts; both flag paths must agree with the oracle.
    V, C, D, S = 40000, 8, 18, 0x1F1A6
    k = 16384
    ua = np.arange(0, 2 * k, 2, dtype=np.uint32)
    ub = np.arange(1, 2 * k + 2, 2, dtype=np.uint32)
    batches = [
        (ua, ua + 1, np.zeros(k, np.uint8)),          # 16384 pairs
        (ub, ub + 1, np.zeros(k + 1, np.uint8)),      # 16385 links joining them
    ]
    rng = np.random.default_rng(5)
    m = 200
    cu = ua[:m]
    ru = rng.integers(0, V, 6000).astype(np.uint32)
    rv = rng.integers(0, V, 6000).astype(np.uint32)
    keep = ru != rv
    u3 = np.concatenate([cu, ru[keep]])
    v3 = np.concatenate([cu + 1, rv[keep]])
    d3 = np.concatenate([np.ones(m, np.uint8), np.zeros(int(keep.sum()), np.uint8)])
    perm = rng.permutation(len(u3))
    batches.append((u3[perm], v3[perm], d3[perm]))
    ctx = cupk.Context(V, C, D, S, **_mkw(cupk, mode))
    ref = oracle.Sketch(V, C, D, S)
    fr = oracle.ForestReplay(ref)
    flagged = []
    for i, (u, v, d) in enumerate(batches):
        print(f"flag boundary batch {i} n={len(u)} mode={mode}", flush=True)
        before = ctx.counters()["flagged"]
        ctx.apply_updates(u, v, d)
        flagged.append(ctx.counters()["flagged"] - before)
        fr.apply_batch(u, v, d)
    assert flagged[:2] == [k, k + 1]
    _assert_same_sketch(ctx, ref)
    assert ctx.forest_edges() == fr.forest_edges()
    ctx.close()


def test_sketchless_root_piece(cupk):
    # One spanning tree over nearly all vertices, then batches that each cut
    # 120 of its edges (chosen from the oracle's forest): the first round
    # leaves the old root's piece out without listing or reducing it, and a
    # tree that holds it in the second round is reduced from the other
    # pieces.  Sketch, forest and counts must match the oracle.
    V, C, D, S = 3000, 10, 20, 0x5EED99
    rng = np.random.default_rng(11)
    m = 15000
    a = rng.integers(0, V, 3 * m)
    b = rng.integers(0, V, 3 * m)
    keep = a != b
    key = np.unique(np.minimum(a, b)[keep].astype(np.int64) * V + np.maximum(a, b)[keep])[:m]
    rng.shuffle(key)
    eu, ev = (key // V).astype(np.uint32), (key % V).astype(np.uint32)
    ctx = cupk.Context(V, C, D, S)
    ref = oracle.Sketch(V, C, D, S)
    fr = oracle.ForestReplay(ref)
    print("sketchless root: inserts", flush=True)
    ctx.apply_updates(eu, ev, np.zeros(m, np.uint8))
    fr.apply_batch(eu, ev, np.zeros(m, np.uint8))
    for it in range(4):
        fe = fr.forest_edges()
        pick = rng.choice(len(fe), 120, replace=False)
        du = np.array([fe[i][0] for i in pick], np.uint32)
        dv = np.array([fe[i][1] for i in pick], np.uint32)
        print(f"sketchless root: cut batch {it}", flush=True)
        ctx.apply_updates(du, dv, np.ones(len(du), np.uint8))
        fr.apply_batch(du, dv, np.ones(len(du), np.uint8))
        _assert_same_sketch(ctx, ref)
        assert ctx.forest_edges() == fr.forest_edges()
    ctr = ctx.counters()
    assert ctr["cuts"] == fr.n_cuts and ctr["rounds"] == fr.n_rounds
    assert ctr["links"] == fr.n_links
    print(f"sketchless={ctr['pieces_sketchless']} complemented={ctr['sets_complemented']}",
          flush=True)
    assert ctr["pieces_sketchless"] >= 1 and ctr["sets_complemented"] >= 1
    ctx.close()


def test_fill_reserve_option(cupk):
    # The staged fill reserving its own bin ranges (one set of tile counts)
    # gives the oracle's sketch and forest like the default, where classify
    # blocks store their bin starts.
    V, p, df = 1000, 0.02, 0.3
    C = max(1, math.ceil(math.log2(V)))
    D = 2 * C
    S = 0x5EEDF111
    u, v, d = streamgen.er_standard(V, p, df, 4242)
    for reserve, lay in ((True, "staged"), (False, "staged"), (True, "pair")):
        print(f"fill_reserve={reserve} layout={lay} n={len(u)}", flush=True)
        ctx, ref, fr = _replay(cupk, lay, V, C, D, S, u, v, d, 4500, tile_vertices=8,
                               fill_reserve=reserve)
        _assert_same_sketch(ctx, ref)
        assert ctx.forest_edges() == fr.forest_edges()
        ctx.close()


def _forest_cut_batches(rng, V, eu, ev, fr, nb, n_forest, n_other, n_new):
    """Batches after an insert phase: each deletes n_forest edges of the
    oracle's current forest and n_other other live edges, and inserts n_new
    fresh pairs, in random order (applied by the caller to both sides)."""
    live = set(zip(eu.tolist(), ev.tolist()))
    for _ in range(nb):
        fe = fr.forest_edges()
        pick_f = [fe[i] for i in rng.choice(len(fe), n_forest, replace=False)]
        fset = set(fe)
        others = [e for e in live if e not in fset]
        pick_o = [others[i] for i in rng.choice(len(others), n_other, replace=False)]
        new = set()
        while len(new) < n_new:
            a, b = (int(t) for t in rng.integers(0, V, 2))
            e = (min(a, b), max(a, b))
            if a != b and e not in live:
                new.add(e)
        dels = pick_f + pick_o
        ups = [(a, b, 1) for a, b in dels] + [(a, b, 0) for a, b in sorted(new)]
        order = rng.permutation(len(ups))
        u = np.array([ups[i][0] for i in order], np.uint32)
        v = np.array([ups[i][1] for i in order], np.uint32)
        d = np.array([ups[i][2] for i in order], np.uint8)
        live -= set(dels)
        live |= new
        yield u, v, d


# More than 8192 vertex tiles: the classify kernel counts tile records with
# global atomics instead of an LDS histogram, and the fill reserves one bin
# slot per record.  (V, tile_vertices): one-vertex tiles over 9000 vertices,
# and the default 16-vertex tiles over 140,000 vertices (8750 tiles).
@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("V,tv", [(9000, 1), (140_000, 16)])
def test_many_tiles_parity(cupk, mode, V, tv):
    _many_tiles(cupk, mode, V, tv, 0)


# The same with coarse bins of a given size (cupk_opts.coarse_tiles): 2 tiles
# (4500 coarse bins: the coarse fill takes the per-record path) and 8 tiles
# (1094 coarse bins: staged coarse fill, long fine runs).
@pytest.mark.parametrize("V,tv,coarse", [(9000, 1, 2), (140_000, 16, 8)])
def test_many_tiles_coarse_bins_parity(cupk, V, tv, coarse):
    _many_tiles(cupk, "pair", V, tv, coarse)


def _many_tiles(cupk, mode, V, tv, coarse):
    C = max(1, math.ceil(math.log2(V)))
    D = 2 * C
    S = 0x5EED8192 + V
    rng = np.random.default_rng(V + tv)
    m = 3 * V
    a = rng.integers(0, V, 2 * m)
    b = rng.integers(0, V, 2 * m)
    keep = a != b
    key = np.unique(np.minimum(a, b)[keep].astype(np.int64) * V + np.maximum(a, b)[keep])[:m]
    rng.shuffle(key)
    eu, ev = (key // V).astype(np.uint32), (key % V).astype(np.uint32)
    ctx = cupk.Context(V, C, D, S, **_mkw(cupk, mode), tile_vertices=tv, coarse_tiles=coarse)
    ref = oracle.Sketch(V, C, D, S)
    fr = oracle.ForestReplay(ref)
    bs = 5000 if V < 20000 else 60000
    for s in range(0, m, bs):
        e = min(m, s + bs)
        print(f"many tiles V={V} tv={tv} coarse={coarse} mode={mode} insert batch {s}:{e}",
              flush=True)
        z = np.zeros(e - s, np.uint8)
        ctx.apply_updates(eu[s:e], ev[s:e], z)
        fr.apply_batch(eu[s:e], ev[s:e], z)
    assert ctx.digest() == ref.digest()
    nfor = 25 if V < 20000 else 30
    for k, (u, v, d) in enumerate(_forest_cut_batches(rng, V, eu, ev, fr, 3, nfor, 3000, 3000)):
        print(f"many tiles V={V} tv={tv} coarse={coarse} mode={mode} cut batch {k} n={len(u)}",
              flush=True)
        ctx.apply_updates(u, v, d)
        fr.apply_batch(u, v, d)
        assert ctx.digest() == ref.digest()
        assert ctx.forest_edges() == fr.forest_edges()
    _assert_same_sketch(ctx, ref)
    ctr = ctx.counters()
    assert ctr["cuts"] == fr.n_cuts >= 3 * nfor
    assert ctr["links"] == fr.n_links and ctr["rounds"] == fr.n_rounds
    ctx.close()


@pytest.mark.parametrize("mode", MODES)
def test_device_batches_stream_ordered(cupk, mode):
    # Eight device batches produced on a side torch stream and queued back
    # to back without waiting in between: each call returns once its device
    # work is queued (the host part runs at the next call); after cupk_sync
    # the sketch, digest and forest equal the oracle's for the same batch
    # boundaries.  The batches are built on the side stream right before
    # each call and their tensors dropped at once, so the caching allocator
    # reuses the memory in stream order.
    import torch
    V, C, D, S = 3000, 12, 24, 0x5EED5757
    u, v, d = streamgen.er_standard(V, 0.01, 0.3, 77)
    nb = 8
    bounds = np.linspace(0, len(u), nb + 1).astype(int)
    ctx = cupk.Context(V, C, D, S, **_mkw(cupk, mode))
    ref = oracle.Sketch(V, C, D, S)
    fr = oracle.ForestReplay(ref)
    side = torch.cuda.Stream()
    host = [cupk.pack_updates(u[a:b], v[a:b], d[a:b]).view(np.int64)
            for a, b in zip(bounds[:-1], bounds[1:])]
    with torch.cuda.stream(side):
        for k, h in enumerate(host):
            print(f"stream-ordered batch {k} n={len(h)} mode={mode}", flush=True)
            t = torch.from_numpy(h).pin_memory().to("cuda", non_blocking=True)
            ctx.apply_updates_device(t, stream=side.cuda_stream)
            del t
    for a, b in zip(bounds[:-1], bounds[1:]):
        fr.apply_batch(u[a:b], v[a:b], d[a:b])
    ctx.sync()
    side.synchronize()
    _assert_same_sketch(ctx, ref)
    assert ctx.forest_edges() == fr.forest_edges()
    assert ctx.counters()["batches"] == nb
    # component sketches written straight into device memory equal the host
    # copies and the oracle's
    rng = np.random.default_rng(3)
    sets = [sorted(rng.choice(V, size=int(s), replace=False).tolist()) for s in (1, 17, 900)]
    ha, hg = ctx.component_sketch_batch(sets)
    out = torch.zeros(len(sets) * C * D * 2, dtype=torch.int64, device="cuda")
    ctx.component_sketch_batch(sets, out=out)
    dv = out.cpu().numpy().view(np.uint64).reshape(len(sets), C, D, 2)
    for j, U in enumerate(sets):
        oa, og = ref.set_sketch(U)
        assert np.array_equal(dv[j, ..., 0], oa) and np.array_equal(dv[j, ..., 1], og)
        assert np.array_equal(ha[j], oa) and np.array_equal(hg[j], og)
    ctx.close()


@pytest.mark.parametrize("mode", MODES)
def test_mass_forest_deletion_batch(cupk, mode):
    # One batch whose flagged updates are more than 16384 deletions of
    # forest edges (the compacted flag list, not the inline one) shatters a
    # spanning tree into about 20000 pieces, and the replacement rounds
    # reconnect them: sketch, forest edges and counts equal the oracle's,
    # and no sample fails.
    V = 30000
    C = max(1, math.ceil(math.log2(V)))
    D = 2 * C
    S = 0x5EEDDE1
    rng = np.random.default_rng(7)
    m = 8 * V
    a = rng.integers(0, V, 2 * m)
    b = rng.integers(0, V, 2 * m)
    keep = a != b
    key = np.unique(np.minimum(a, b)[keep].astype(np.int64) * V + np.maximum(a, b)[keep])[:m]
    rng.shuffle(key)
    eu, ev = (key // V).astype(np.uint32), (key % V).astype(np.uint32)
    ctx = cupk.Context(V, C, D, S, **_mkw(cupk, mode))
    ref = oracle.Sketch(V, C, D, S)
    fr = oracle.ForestReplay(ref)
    for s in range(0, m, 60000):
        e = min(m, s + 60000)
        print(f"mass deletion mode={mode}: insert batch {s}:{e}", flush=True)
        z = np.zeros(e - s, np.uint8)
        ctx.apply_updates(eu[s:e], ev[s:e], z)
        fr.apply_batch(eu[s:e], ev[s:e], z)
    (u, v, d), = _forest_cut_batches(rng, V, eu, ev, fr, 1, 20000, 5000, 3000)
    print(f"mass deletion mode={mode}: batch of {len(u)} with 20000 forest-edge deletions",
          flush=True)
    ctx.apply_updates(u, v, d)
    fr.apply_batch(u, v, d)
    _assert_same_sketch(ctx, ref)
    assert ctx.forest_edges() == fr.forest_edges()
    ctr = ctx.counters()
    assert ctr["cuts"] == fr.n_cuts and ctr["rounds"] == fr.n_rounds
    assert ctr["links"] == fr.n_links
    assert ctr["sample_failed"] == fr.n_failed == 0
    fu, fv = streamgen.final_edges(np.concatenate([eu, u]), np.concatenate([ev, v]),
                                   np.concatenate([np.zeros(m, np.uint8), d]))
    truth = oracle.components_truth(V, fu, fv)
    assert ctx.num_components() == len(set(truth.tolist()))
    ctx.close()


@pytest.mark.parametrize("coarse", [1, 3, 16384])
def test_coarse_tiles_rejected(cupk, coarse):
    # not a power of two in [2, 8192]: the context is not created
    with pytest.raises(cupk.CupkError) as ei:
        cupk.Context(9000, 14, 28, 1, scatter_mode=cupk.SCATTER_STAGED, tile_vertices=1,
                     coarse_tiles=coarse)
    assert ei.value.code == cupk.EINVAL
