"""The seeded workload generators: legality, determinism and the shapes
their recipes promise (CPU only)."""
import numpy as np

import streamgen


def test_generators_are_legal_and_deterministic():
    for i in (2, 4):
        a = streamgen.config_stream(i, scaled=True)
        b = streamgen.config_stream(i, scaled=True)
        assert all(np.array_equal(x, y) for x, y in zip(a, b))
        u, v, d = a
        assert (u < v).all()
        streamgen.final_edges(u, v, d)  # asserts insert-if-absent / delete-if-present


def test_rmat_is_skewed_and_deletes_fifteen_percent():
    cfg = streamgen.SCALED[2]
    u, v, d = streamgen.config_stream(2, scaled=True)
    assert abs(d.mean() - cfg["del_prob"]) < 0.01
    deg = np.bincount(np.concatenate([u[d == 0], v[d == 0]]), minlength=cfg["V"])
    # quadrant a = 0.57 concentrates endpoints on small ids
    assert deg[: cfg["V"] // 16].sum() > 4 * deg[-cfg["V"] // 16:].sum()


def test_clustered_churn_shape():
    cfg = streamgen.SCALED[4]
    u, v, d = streamgen.config_stream(4, scaled=True)
    K, S = cfg["K"], cfg["Sc"]
    Vc = K * S
    inside = (u < Vc) & (v < Vc) & (u // S == v // S)
    bridge = (u < Vc) & (v < Vc) & (u // S != v // S)
    sparse = (u >= Vc) & (v >= Vc)
    assert (inside | bridge | sparse).all()
    assert sparse.sum() == 2 * cfg["n_sparse"]
    # churn inserts and deletes every non-forest cluster edge; the fixed
    # forest (S-1 edges per connected cluster) stays
    ins, dels = int((d[inside] == 0).sum()), int(d[inside].sum())
    assert ins - dels == K * (S - 1)
    assert dels % cfg["rounds"] == 0 and dels > 0
    # bridges are toggled adversarially
    assert d[bridge].sum() > 0


def test_forest_targeted_deletes_picks_supplied_forest_edges():
    cfg = streamgen.SCALED[3]
    g = streamgen.ForestTargetedDeletes(cfg["V"], 0.05, 0.5, 0.3, 7, 500)
    live = set()
    for u, v, d in g.insert_chunks():
        live |= set(zip(u.tolist(), v.tolist()))
    # a fake "forest": any 100 live edges
    forest = sorted(live)[:100]
    fu = np.array([e[0] for e in forest], np.uint32)
    fv = np.array([e[1] for e in forest], np.uint32)
    u, v, d = g.delete_chunk(fu, fv)
    got = set(zip(u.tolist(), v.tolist()))
    assert d.all() and len(got) == len(u) == 500
    assert got <= live
    nf = len(got & set(forest))
    assert 100 <= nf <= 200  # Binomial(500, 0.3) capped at the 100 forest edges


def test_fixed_forest_stream():
    """The forest comes first and is never deleted; every other edge is
    inserted and deleted reps times; replaying it links exactly the forest
    and never cuts."""
    import oracle
    V, reps = 300, 2
    u, v, d = streamgen.fixed_forest(V, 0.05, reps, 9)
    fu, fv = streamgen.final_edges(u, v, d)
    k = len(fu)
    assert set(zip(u[:k].tolist(), v[:k].tolist())) == set(zip(fu.tolist(), fv.tolist()))
    assert not d[:k].any()
    rest = len(u) - k
    assert rest % (2 * reps) == 0
    m = rest // (2 * reps)
    truth = oracle.components_truth(V, fu, fv)
    assert k == V - len(set(truth.tolist()))     # a spanning forest
    sk = oracle.Sketch(V, 9, 18, 0x5EED)
    fr = oracle.ForestReplay(sk)
    for s in range(0, len(u), 997):
        fr.apply_batch(u[s:s + 997], v[s:s + 997], d[s:s + 997])
    assert fr.n_cuts == 0 and fr.n_links == k
    assert set(fr.forest_edges()) == set(zip(fu.tolist(), fv.tolist()))
    for r in range(reps):
        ins = slice(k + 2 * r * m, k + (2 * r + 1) * m)
        dele = slice(k + (2 * r + 1) * m, k + (2 * r + 2) * m)
        assert not d[ins].any() and d[dele].all()
        assert set(zip(u[ins].tolist(), v[ins].tolist())) == set(zip(u[dele].tolist(), v[dele].tolist()))
