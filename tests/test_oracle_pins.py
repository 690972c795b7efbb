"""Pins of the oracle against facts fixed outside it.

Each test checks the oracle against something other than itself:
published SplitMix64 outputs, closed-form probabilities, the cancellation
invariant of characteristic vectors (App. A.1.1), brute force over all
vertex subsets, and breadth-first search.  The tests are chosen so that a
plausible slip in the oracle (a wrong seed, an endpoint-dependent depth, a
swapped decode, a transposed bucket index, a missing checksum check) fails
at least one of them.
"""
import math
import os

import numpy as np
import pytest

import streamgen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "splitmix64_state0.txt")
M64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15


def _golden():
    vals = []
    for line in open(GOLDEN):
        line = line.strip()
        if line and not line.startswith("#"):
            vals.append(int(line, 16))
    return vals


def test_seed_sequence_matches_published_splitmix64(orc):
    vals = _golden()
    assert [orc.seed(0, c) for c in range(len(vals))] == vals


def test_hash_is_finalizer_of_index_xor_column_seed(orc):
    # h_c(x) = mix(x ^ seed_c): choosing x = seed_c ^ (k * gamma) makes the
    # hash input the k-th SplitMix64 state from 0, whose output is published.
    vals = _golden()
    S = 0x5EED0001
    for c in range(4):
        sc = orc.seed(S, c)
        for k, want in enumerate(vals, start=1):
            x = sc ^ ((k * GAMMA) & M64)
            assert orc.hash_c(S, c, x) == want


def test_depth_is_capped_trailing_zero_count(orc):
    D = 20
    for k in range(64):
        assert orc.depth_of_hash(1 << k, D) == min(k, D - 1)
        assert orc.depth_of_hash((1 << k) | (1 << 63), D) == min(k, D - 1)
    assert orc.depth_of_hash(0, D) == D - 1


def test_depth_distribution_chi_square(orc):
    # P(d) = 2^-(d+1) for d < D-1 and 2^-(D-1) at the cap.
    from scipy.stats import chisquare
    D = 8
    S = 0xABCDEF
    rng = np.random.default_rng(7)
    n = 60000
    xs = rng.integers(1, 1 << 62, size=n, dtype=np.uint64)
    counts = np.zeros(D)
    for i, x in enumerate(xs.tolist()):
        c = i % 3
        counts[orc.depth_of_hash(orc.hash_c(S, c, x), D)] += 1
    p = np.array([2.0 ** -(d + 1) for d in range(D - 1)] + [2.0 ** -(D - 1)])
    assert abs(p.sum() - 1) < 1e-12
    stat, pval = chisquare(counts, n * p)
    assert pval > 1e-4, (counts, n * p, pval)


def _small_stream(V, p, del_frac, seed):
    return streamgen.er_standard(V, p, del_frac, seed)


def test_bucket_contents_follow_definition(orc):
    # bucket (c, d) of vertex w = XOR of x_e (and of h_c(x_e)) over live
    # edges e at w with d_c(x_e) = d.  Catches a transposed [w][c][d] index.
    V, C, D, S = 20, 3, 6, 12345
    u, v, d = _small_stream(V, 0.4, 0.3, 3)
    sk = orc.Sketch(V, C, D, S)
    sk.apply(u, v)
    fu, fv = streamgen.final_edges(u, v, d)
    A = np.zeros((V, C, D), np.uint64)
    G = np.zeros((V, C, D), np.uint64)
    for a, b in zip(fu.tolist(), fv.tolist()):
        x = a * V + b
        for c in range(C):
            h = orc.hash_c(S, c, x)
            dd = orc.depth_of_hash(h, D)
            for w in (a, b):
                A[w, c, dd] ^= np.uint64(x)
                G[w, c, dd] ^= np.uint64(h)
    assert np.array_equal(sk.alpha, A)
    assert np.array_equal(sk.gamma, G)


def test_stream_sketch_depends_only_on_final_edge_set(orc):
    V, C, D, S = 64, 6, 12, 99
    u, v, d = _small_stream(V, 0.3, 0.4, 5)
    a = orc.Sketch(V, C, D, S)
    a.apply(u, v)
    fu, fv = streamgen.final_edges(u, v, d)
    b = orc.Sketch(V, C, D, S)
    b.apply(fu, fv)
    assert np.array_equal(a.alpha, b.alpha) and np.array_equal(a.gamma, b.gamma)
    # order independence
    perm = np.random.default_rng(1).permutation(len(u))
    c = orc.Sketch(V, C, D, S)
    c.apply(u[perm], v[perm])
    assert np.array_equal(a.alpha, c.alpha) and np.array_equal(a.gamma, c.gamma)
    assert a.digest() == c.digest()


def test_insert_then_delete_all_is_zero(orc):
    V, C, D, S = 50, 5, 10, 3
    u, v, _ = _small_stream(V, 0.5, 0.0, 8)
    sk = orc.Sketch(V, C, D, S)
    sk.apply(u, v)
    assert sk.alpha.any()
    sk.apply(u[::-1].copy(), v[::-1].copy())
    assert not sk.alpha.any() and not sk.gamma.any()


def test_cancellation_all_subsets_bruteforce(orc):
    # Sum over U of the vertex sketches == sketch of exactly the cut edges
    # delta(U) (App. A.1.1), for every subset U of a 10-vertex graph.
    V, C, D, S = 10, 4, 8, 777
    u, v, d = _small_stream(V, 0.5, 0.3, 11)
    fu, fv = streamgen.final_edges(u, v, d)
    sk = orc.Sketch(V, C, D, S)
    sk.apply(u, v)
    edges = list(zip(fu.tolist(), fv.tolist()))
    # (column, depth, index, checksum) of every live edge
    cells = {}
    for a, b in edges:
        x = a * V + b
        cells[(a, b)] = []
        for c in range(C):
            h = orc.hash_c(S, c, x)
            cells[(a, b)].append((c, orc.depth_of_hash(h, D), x, h))
    for mask in range(1, 1 << V):
        U = [w for w in range(V) if mask >> w & 1]
        inU = set(U)
        cut = [(a, b) for a, b in edges if (a in inU) != (b in inU)]
        a_, g_ = sk.set_sketch(U)
        ra = np.zeros((C, D), np.uint64)
        rg = np.zeros((C, D), np.uint64)
        for e in cut:
            for c, dd, x, h in cells[e]:
                ra[c, dd] ^= np.uint64(x)
                rg[c, dd] ^= np.uint64(h)
        assert np.array_equal(a_, ra) and np.array_equal(g_, rg), U
        assert (a_.any() or g_.any()) == bool(cut)


def test_true_component_sketch_is_zero_and_samples_empty(orc):
    V, C, D, S = 200, 8, 16, 31
    u, v, d = _small_stream(V, 0.012, 0.2, 4)
    fu, fv = streamgen.final_edges(u, v, d)
    lab = orc.components_truth(V, fu, fv)
    sk = orc.Sketch(V, C, D, S)
    sk.apply(u, v)
    comps = {}
    for w, l in enumerate(lab.tolist()):
        comps.setdefault(l, []).append(w)
    assert len(comps) > 3
    for members in comps.values():
        a, g = sk.set_sketch(members)
        assert not a.any() and not g.any()
        assert orc.sample(V, C, D, S, a, g)[0] == orc.EMPTY


def test_single_cut_edge_is_always_recovered(orc):
    # |delta(U)| = 1: every column holds that one index alone, so the first
    # column's bucket verifies and the sample is exactly that edge.
    rng = np.random.default_rng(3)
    for trial in range(40):
        V = int(rng.integers(8, 300))
        C, D = 3, 2 * math.ceil(math.log2(V))
        S = int(rng.integers(0, 1 << 62))
        # two cliques-ish blocks joined by one bridge
        k = int(rng.integers(2, V - 2))
        A, B = list(range(k)), list(range(k, V))
        edges = set()
        for blk in (A, B):
            for i in range(1, len(blk)):
                edges.add((blk[int(rng.integers(0, i))], blk[i]))
        a0, b0 = int(rng.choice(A)), int(rng.choice(B))
        bridge = (min(a0, b0), max(a0, b0))
        edges.add(bridge)
        eu = np.array([e[0] for e in edges], np.uint32)
        ev = np.array([e[1] for e in edges], np.uint32)
        sk = orc.Sketch(V, C, D, S)
        sk.apply(eu, ev)
        for U in (A, B):
            st, x, y = sk.sample(*sk.set_sketch(U))
            assert st == orc.OK and (x, y) == bridge, (trial, st, x, y, bridge)


def test_sampled_edge_is_a_real_cut_edge(orc):
    rng = np.random.default_rng(9)
    V, C, D, S = 120, 7, 14, 2024
    u, v, d = _small_stream(V, 0.2, 0.3, 13)
    fu, fv = streamgen.final_edges(u, v, d)
    edges = set(zip(fu.tolist(), fv.tolist()))
    sk = orc.Sketch(V, C, D, S)
    sk.apply(u, v)
    n_ok = 0
    for _ in range(300):
        U = set(np.flatnonzero(rng.random(V) < rng.random()).tolist())
        if not U:
            continue
        st, x, y = sk.sample(*sk.set_sketch(sorted(U)))
        cut = [(a, b) for a, b in edges if (a in U) != (b in U)]
        if st == orc.OK:
            n_ok += 1
            assert x < y and (x, y) in edges and ((x in U) != (y in U))
        elif st == orc.EMPTY:
            assert not cut
        else:
            assert cut
    assert n_ok > 250


def test_two_edge_column_success_matches_closed_form(orc):
    # With two indices in a column, the column recovers an index iff they
    # fall at different depths: p = 1 - sum_d P(d)^2.
    D = 12
    P = [2.0 ** -(d + 1) for d in range(D - 1)] + [2.0 ** -(D - 1)]
    p = 1 - sum(q * q for q in P)
    rng = np.random.default_rng(21)
    V = 256
    n, ok = 20000, 0
    for t in range(n):
        w = int(rng.integers(0, V))
        a, b = rng.choice(V - 1, size=2, replace=False)
        a = int(a) + (a >= w)
        b = int(b) + (b >= w)
        S = int(rng.integers(0, 1 << 62))
        sk = orc.Sketch(V, 1, D, S)
        sk.toggle(w, a)
        sk.toggle(w, b)
        st, x, y = sk.sample(*sk.set_sketch([w]))
        if st == orc.OK:
            ok += 1
            assert (x, y) in ((min(w, a), max(w, a)), (min(w, b), max(w, b)))
        else:
            assert st == orc.FAILED
    sd = math.sqrt(p * (1 - p) / n)
    assert abs(ok / n - p) < 5 * sd, (ok / n, p)


def test_colliding_indices_give_failed_not_empty(orc):
    # Two edges at the same depth in the only column: the bucket holds the
    # XOR of two indices, which does not verify.
    V, C, D, S = 1000, 1, 4, 55
    w = 0
    found = None
    first = {}
    for b in range(1, V):
        x = orc.edge_index(V, w, b)
        dd = orc.depth_of_hash(orc.hash_c(S, 0, x), D)
        if dd in first:
            found = (first[dd], b)
            break
        first[dd] = b
    assert found
    sk = orc.Sketch(V, C, D, S)
    sk.toggle(w, found[0])
    sk.toggle(w, found[1])
    st, _, _ = sk.sample(*sk.set_sketch([w]))
    assert st == orc.FAILED


def test_sample_takes_first_good_bucket_in_canonical_order(orc):
    # Reading: columns ascending, depths descending inside a column.
    V, C, D, S = 64, 4, 8, 4242
    u, v, d = _small_stream(V, 0.15, 0.0, 17)
    sk = orc.Sketch(V, C, D, S)
    sk.apply(u, v)
    rng = np.random.default_rng(5)
    for _ in range(100):
        U = sorted(set(rng.choice(V, size=int(rng.integers(1, V)), replace=False).tolist()))
        a, g = sk.set_sketch(U)
        want = None
        for c in range(C):
            for dd in range(D - 1, -1, -1):
                x, h = int(a[c, dd]), int(g[c, dd])
                if x == 0:
                    continue
                uu, vv = divmod(x, V)
                if not (uu < vv < V):
                    continue
                hh = orc.hash_c(S, c, x)
                if hh == h and orc.depth_of_hash(hh, D) == dd:
                    want = (uu, vv)
                    break
            if want:
                break
        st, x, y = sk.sample(a, g)
        if want is None:
            assert st != orc.OK
        else:
            assert st == orc.OK and (x, y) == want


# ---- the one-column sampler (level c of the hierarchy uses column c) -------
#
# These pins fix orc_sample_col from outside: which edges a column holds,
# and how many, follows from the cut edge list and the depth function alone
# (pinned above), not from the sampler's verification.


def _column_from_edges(orc, V, C, D, S, c, edges):
    """Column c of the aggregate sketch of an explicit edge list, built by
    XOR-ing (x, h_c(x)) into depth d_c(x): the streaming definition written
    out for one column.  Returns (alpha, gamma) as C x D arrays that are zero
    outside column c, and {depth: [edges]}."""
    a = np.zeros((C, D), np.uint64)
    g = np.zeros((C, D), np.uint64)
    at = {}
    for (x0, y0) in edges:
        x = orc.edge_index(V, x0, y0)
        h = orc.hash_c(S, c, x)
        dd = orc.depth_of_hash(h, D)
        a[c, dd] ^= np.uint64(x)
        g[c, dd] ^= np.uint64(h)
        at.setdefault(dd, []).append((min(x0, y0), max(x0, y0)))
    return a, g, at


def test_column_sampler_returns_a_lone_cut_edge(orc):
    # |delta(U)| = 1: every column holds that edge alone, so the query of
    # any single column returns it.
    rng = np.random.default_rng(31)
    for trial in range(30):
        V = int(rng.integers(8, 300))
        C, D = 5, 2 * math.ceil(math.log2(V))
        S = int(rng.integers(0, 1 << 62))
        k = int(rng.integers(2, V - 2))
        A, B = list(range(k)), list(range(k, V))
        edges = set()
        for blk in (A, B):
            for i in range(1, len(blk)):
                edges.add((blk[int(rng.integers(0, i))], blk[i]))
        a0, b0 = int(rng.choice(A)), int(rng.choice(B))
        bridge = (min(a0, b0), max(a0, b0))
        edges.add(bridge)
        sk = orc.Sketch(V, C, D, S)
        sk.apply(np.array([e[0] for e in edges], np.uint32),
                 np.array([e[1] for e in edges], np.uint32))
        for U in (A, B):
            a, g = sk.set_sketch(U)
            for c in range(C):
                assert orc.sample_col(V, C, D, S, c, a, g) == (orc.OK,) + bridge, (trial, c)


def test_column_sampler_two_indices_at_one_depth_fail(orc):
    # Two edges that land at the same depth of column c, and nothing else in
    # the column: the bucket holds the XOR of two indices and does not
    # verify, the column is not all zero, so the status is FAILED.
    rng = np.random.default_rng(32)
    V, C, D = 1000, 4, 12
    n = 0
    while n < 300:
        S = int(rng.integers(0, 1 << 62))
        c = int(rng.integers(0, C))
        w = int(rng.integers(0, V))
        first = {}
        pair = None
        for b in rng.permutation(V).tolist():
            if b == w:
                continue
            x = orc.edge_index(V, w, b)
            dd = orc.depth_of_hash(orc.hash_c(S, c, x), D)
            if dd in first:
                pair = [(w, first[dd]), (w, b)]
                break
            first[dd] = b
        a, g, at = _column_from_edges(orc, V, C, D, S, c, pair)
        assert len(at) == 1
        assert orc.sample_col(V, C, D, S, c, a, g)[0] == orc.FAILED
        n += 1


def test_column_sampler_empty_only_when_the_column_is_zero(orc):
    # EMPTY is decided by the queried column alone; any nonzero word in it
    # (even a checksum with a zero index word) makes an unverified column
    # FAILED.
    V, C, D, S = 500, 3, 10, 77
    a = np.zeros((C, D), np.uint64)
    g = np.zeros((C, D), np.uint64)
    for c in range(C):
        assert orc.sample_col(V, C, D, S, c, a, g)[0] == orc.EMPTY
    a[2, 3] = np.uint64(orc.edge_index(V, 4, 9))
    g[2, 3] = np.uint64(12345)
    for c in (0, 1):
        assert orc.sample_col(V, C, D, S, c, a, g)[0] == orc.EMPTY
    assert orc.sample_col(V, C, D, S, 2, a, g)[0] == orc.FAILED
    a[2, 3] = 0
    assert orc.sample_col(V, C, D, S, 2, a, g)[0] == orc.FAILED


def test_column_sampler_returns_the_deepest_lone_edge(orc):
    # For random edge sets, the expected answer is found by counting edges
    # per depth of column c: among depths that hold exactly one edge, the
    # deepest one's edge.  (A depth holding several edges does not verify
    # except with probability about 2^-64.)
    rng = np.random.default_rng(33)
    V, C, D = 400, 6, 18
    seen_multi = 0
    for trial in range(400):
        S = int(rng.integers(0, 1 << 62))
        c = int(rng.integers(0, C))
        m = int(rng.integers(1, 9))
        edges = set()
        while len(edges) < m:
            x0, y0 = (int(t) for t in rng.integers(0, V, 2))
            if x0 != y0:
                edges.add((min(x0, y0), max(x0, y0)))
        a, g, at = _column_from_edges(orc, V, C, D, S, c, sorted(edges))
        lone = [dd for dd, es in at.items() if len(es) == 1]
        got = orc.sample_col(V, C, D, S, c, a, g)
        if lone:
            want = at[max(lone)][0]
            assert got == (orc.OK,) + want, (trial, got, want, at)
            seen_multi += len(lone) > 1
        else:
            assert got[0] == orc.FAILED, (trial, got, at)
    assert seen_multi > 50


def test_vertex_from_stream_matches_full_replay(orc):
    V, C, D, S = 90, 7, 14, 606
    u, v, d = _small_stream(V, 0.3, 0.2, 23)
    sk = orc.Sketch(V, C, D, S)
    sk.apply(u, v)
    for w in (0, 1, 45, 89):
        a, g = orc.vertex_from_stream(V, C, D, S, w, u, v)
        assert np.array_equal(a, sk.alpha[w]) and np.array_equal(g, sk.gamma[w])


def test_digest_is_order_independent_and_sensitive(orc):
    V, C, D, S = 40, 5, 10, 9
    u, v, d = _small_stream(V, 0.4, 0.2, 2)
    a = orc.Sketch(V, C, D, S)
    a.apply(u, v)
    dg = a.digest()
    # partial digests over vertex ranges add up (mod 2^64)
    part = (orc.digest_arrays(C, D, S, 0, a.alpha[:17], a.gamma[:17])
            + orc.digest_arrays(C, D, S, 17, a.alpha[17:], a.gamma[17:])) & M64
    assert part == dg
    # one extra toggle changes it
    a.toggle(0, 1)
    assert a.digest() != dg


def test_components_truth_matches_scipy(orc):
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    V = 500
    u, v, d = _small_stream(V, 0.003, 0.3, 31)
    fu, fv = streamgen.final_edges(u, v, d)
    lab = orc.components_truth(V, fu, fv)
    m = coo_matrix((np.ones(len(fu)), (fu, fv)), shape=(V, V))
    n, sl = connected_components(m, directed=False)
    assert len(set(lab.tolist())) == n
    for a in range(0, V, 7):
        for b in range(0, V, 11):
            assert (lab[a] == lab[b]) == (sl[a] == sl[b])


@pytest.mark.parametrize("V,p,df,batch", [
    (60, 0.08, 0.5, 1),        # per-update replay, sparse: many components
    (60, 0.08, 0.5, 17),
    (128, 0.2, 0.4, 1),
    (128, 0.2, 0.4, 64),
    (128, 0.2, 0.4, None),     # whole stream in one batch
    (300, 0.01, 0.3, 50),
])
def test_forest_replay_is_spanning_forest_at_every_boundary(orc, V, p, df, batch):
    C = math.ceil(math.log2(V))
    D = 2 * C
    u, v, d = _small_stream(V, p, df, V + int(p * 1000))
    sk = orc.Sketch(V, C, D, 0x5EED)
    fr = orc.ForestReplay(sk)
    n = len(u)
    bs = n if batch is None else batch
    live = set()
    for s in range(0, n, bs):
        e = min(n, s + bs)
        fr.apply_batch(u[s:e], v[s:e], d[s:e])
        for a, b, x in zip(u[s:e].tolist(), v[s:e].tolist(), d[s:e].tolist()):
            (live.remove if x else live.add)((a, b))
        if batch is None or (s // bs) % max(1, (n // bs) // 25) == 0 or e == n:
            eu = np.array([x[0] for x in live], np.uint32)
            ev = np.array([x[1] for x in live], np.uint32)
            truth = orc.components_truth(V, eu, ev)
            orc.check_spanning_forest(V, fr.forest_edges(), live, truth)
        # with no failed sample every tree is known to be a whole component
        # at the end of a batch, including the one the rounds left out
        assert not fr.mark
    assert fr.n_failed == 0


def test_rounds_leave_out_the_largest_dirty_tree(orc):
    """Cutting a path splits it into sides of 3 and 5 vertices; the only
    edge between them is an insert of this batch (same batch-start tree, so
    not linked directly).  One round samples only the smaller side, whose
    single cut edge is always recovered; the larger side is never reduced and
    ends clean with the rest."""
    V = 8
    sk = orc.Sketch(V, 3, 6, 0x5EED)
    fr = orc.ForestReplay(sk)
    path = np.arange(V - 1, dtype=np.uint32)
    fr.apply_batch(path, path + 1, np.zeros(V - 1, np.uint8))
    assert fr.n_rounds == 0 and not fr.mark
    fr.apply_batch(np.array([2, 0], np.uint32), np.array([3, 7], np.uint32),
                   np.array([1, 0], np.uint8))
    assert fr.n_cuts == 1 and fr.n_rounds == 1
    assert fr.round_log[-1] == [(0, orc.OK, 0, 7)]
    assert (0, 7) in fr.forest_edges() and (2, 3) not in fr.forest_edges()
    assert not fr.mark


def test_static_components_hand_worked(orc):
    """Two disjoint edges on four vertices: round 1 samples the four
    singletons (each has one incident edge, always recovered) and merges
    {0,1} then {2,3}; round 2 finds both supernodes EMPTY."""
    sk = orc.Sketch(4, 2, 4, 0x5EED)
    sk.apply(np.array([0, 2], np.uint32), np.array([1, 3], np.uint32))
    labels, edges, rounds, failed = orc.static_components(sk)
    assert labels.tolist() == [0, 0, 2, 2]
    assert edges == [(0, 1), (2, 3)]
    assert rounds == 2 and failed == 0


@pytest.mark.parametrize("V,p,seed", [(40, 0.05, 1), (120, 0.02, 2), (200, 0.3, 3),
                                      (300, 0.004, 4)])
def test_static_components_match_bfs(orc, V, p, seed):
    """Boruvka over the sketch finds the true components (w.h.p.; no query
    fails at these sizes), its merge edges are a spanning forest of the
    graph, and the rounds at most halve the active supernodes each time."""
    C = math.ceil(math.log2(V))
    u, v, d = _small_stream(V, p, 0.3, seed)
    sk = orc.Sketch(V, C, 2 * C, 0x5EED + seed)
    sk.apply(u, v)
    fu, fv = streamgen.final_edges(u, v, d)
    truth = orc.components_truth(V, fu, fv)
    labels, edges, rounds, failed = orc.static_components(sk)
    assert failed == 0
    assert labels.tolist() == truth.tolist()
    orc.check_spanning_forest(V, edges, set(zip(fu.tolist(), fv.tolist())), truth)
    assert rounds <= math.ceil(math.log2(V)) + 1


def test_threaded_apply_equals_plain_apply(orc):
    # The all-core baseline (vertex ranges per thread) gives the sketch of the
    # one-thread replay bit for bit, for any thread count.
    V, C, D, S = 777, 10, 20, 0x5EEDC0DE
    u, v, d = _small_stream(V, 0.05, 0.4, 23)
    ref = orc.Sketch(V, C, D, S)
    ref.apply(u, v)
    for t in (1, 2, 3, 8):
        sk = orc.Sketch(V, C, D, S)
        used = sk.apply_threads(u, v, t)
        assert 1 <= used <= t
        assert np.array_equal(sk.alpha, ref.alpha) and np.array_equal(sk.gamma, ref.gamma)
        assert sk.digest() == ref.digest()


def test_union_find_truth_equals_bfs(orc):
    # The union-find connectivity truth (used for graphs too large for the
    # BFS) gives the BFS partition, labelled by smallest member.
    rng = np.random.default_rng(41)
    for trial in range(20):
        V = int(rng.integers(2, 400))
        m = int(rng.integers(0, 2 * V))
        a = rng.integers(0, V, m).astype(np.uint32)
        b = rng.integers(0, V, m).astype(np.uint32)
        keep = a != b
        k, lab = orc.uf_components(V, a[keep], b[keep])
        truth = orc.components_truth(V, a[keep], b[keep])
        assert np.array_equal(lab.astype(np.int64), truth)
        assert k == len(set(truth.tolist()))
        # incremental form: edges added in two parts, same answers
        uf = orc.UnionFind(V)
        h = int(keep.sum()) // 2
        uf.add(a[keep][:h], b[keep][:h])
        assert uf.add(a[keep][h:], b[keep][h:]) == k
        for x, y in rng.integers(0, V, (20, 2)).tolist():
            assert uf.same(x, y) == (truth[x] == truth[y])
