"""Serving loop: continuous batching, memory admission, query semantics.

* Each query is answered on exactly the updates submitted before it
  (checked against breadth-first search at that point of the stream).
* The final sketch equals the one from applying the same stream without
  the loop (XOR is order- and batching-independent).
* Several clients on disjoint vertex ranges: each client's answers are the
  same when it runs alone and when its requests are mixed with the others'
  (the forest answers do not depend on how the loop batched them).
* Admission: a tiny budget refuses (non-blocking) or waits (blocking).
"""
import threading

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


def _requests(u, v, d, rng, max_req=400, q_every=3):
    """Cut a stream into update requests of random sizes with queries in
    between; returns a list of ("u", lo, hi) / ("q", a, b)."""
    out = []
    i, n, V = 0, len(u), int(max(u.max(), v.max())) + 1
    k = 0
    while i < n:
        s = int(rng.integers(1, max_req))
        out.append(("u", i, min(n, i + s)))
        i = min(n, i + s)
        k += 1
        if k % q_every == 0:
            a, b = (int(x) for x in rng.integers(0, V, 2))
            out.append(("q", a, b))
    return out


def _truth_answers(V, u, v, d, reqs):
    live = set()
    ans = []
    for r in reqs:
        if r[0] == "u":
            for a, b, x in zip(u[r[1]:r[2]].tolist(), v[r[1]:r[2]].tolist(),
                               d[r[1]:r[2]].tolist()):
                (live.remove if x else live.add)((a, b))
        else:
            eu = np.array([e[0] for e in live], np.uint32)
            ev = np.array([e[1] for e in live], np.uint32)
            lab = oracle.components_truth(V, eu, ev)
            ans.append(int(lab[r[1]] == lab[r[2]]))
    return ans


@pytest.mark.parametrize("max_batch", [64, 1000, 1 << 20])
def test_served_queries_match_bfs_and_sketch_matches_unserved(cupk, max_batch):
    V, C, D, S = 300, 9, 18, 77
    u, v, d = streamgen.er_standard(V, 0.03, 0.6, 3)
    rng = np.random.default_rng(1)
    reqs = _requests(u, v, d, rng)
    want = _truth_answers(V, u, v, d, reqs)
    print(f"served n={len(u)} requests={len(reqs)} max_batch={max_batch}", flush=True)
    ctx = cupk.Context(V, C, D, S)
    ctx.serve_start(max_batch=max_batch, mem_budget_bytes=1 << 20)
    tickets = []
    for r in reqs:
        if r[0] == "u":
            tickets.append(("u", ctx.submit_updates(u[r[1]:r[2]], v[r[1]:r[2]], d[r[1]:r[2]])))
        else:
            tickets.append(("q", ctx.submit_query(r[1], r[2])))
    got = []
    for kind, t in tickets:
        res = ctx.wait(t)
        if kind == "q":
            got.append(res)
        else:
            assert res == 0
    st = ctx.serve_stats()
    ctx.serve_stop()
    assert got == want
    assert st["queries"] == len(want) and st["updates"] == len(u)
    assert st["query_p50_us"] > 0 and st["query_p99_us"] >= st["query_p50_us"]
    # same sketch as the plain, unserved path
    ref = cupk.Context(V, C, D, S)
    ref.apply_updates(u, v, d)
    assert ctx.digest() == ref.digest()
    sk = oracle.Sketch(V, C, D, S)
    sk.apply(u, v)
    assert ctx.digest() == sk.digest()
    # the context is usable again after stop
    ctx.apply_updates(u[:1], v[:1], 1 - d[:1])
    ctx.close()
    ref.close()


def test_clients_alone_and_in_the_mix(cupk):
    # 3 clients, each owning a disjoint block of 100 vertices
    V, C, D, S = 300, 9, 18, 5
    streams, reqs = [], []
    for k in range(3):
        u, v, d = streamgen.er_standard(100, 0.05, 0.5, 10 + k)
        u = u + 100 * k
        v = v + 100 * k
        streams.append((u, v, d))
        rng = np.random.default_rng(20 + k)
        rr = []
        for r in _requests(u, v, d, rng, max_req=50, q_every=2):
            if r[0] == "q":   # queries inside the client's own block
                rr.append(("q", 100 * k + r[1] % 100, 100 * k + r[2] % 100))
            else:
                rr.append(r)
        reqs.append(rr)

    def run_client(ctx, k, out):
        u, v, d = streams[k]
        ans = []
        for r in reqs[k]:
            if r[0] == "u":
                t = ctx.submit_updates(u[r[1]:r[2]], v[r[1]:r[2]], d[r[1]:r[2]])
                assert ctx.wait(t) == 0
            else:
                ans.append(ctx.wait(ctx.submit_query(r[1], r[2])))
        out[k] = ans

    alone = {}
    for k in range(3):
        ctx = cupk.Context(V, C, D, S)
        ctx.serve_start(max_batch=256)
        run_client(ctx, k, alone)
        ctx.serve_stop()
        ctx.close()
    mixed = {}
    ctx = cupk.Context(V, C, D, S)
    ctx.serve_start(max_batch=256)
    ths = [threading.Thread(target=run_client, args=(ctx, k, mixed)) for k in range(3)]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    st = ctx.serve_stats()
    ctx.serve_stop()
    for k in range(3):
        u, v, d = streams[k]
        want = _truth_answers(V, u, v, d, reqs[k])
        assert alone[k] == want
        assert mixed[k] == want
    assert st["batches"] >= 1
    ctx.close()


def test_memory_admission(cupk):
    V, C, D, S = 100, 7, 14, 1
    u, v, d = streamgen.er_standard(V, 0.2, 0.0, 2)
    ctx = cupk.Context(V, C, D, S)
    # a request larger than the whole budget can never be admitted
    ctx.serve_start(max_batch=16, mem_budget_bytes=8 * 32, nonblocking=True)
    with pytest.raises(cupk.CupkError) as ei:
        ctx.submit_updates(u[:33], v[:33], d[:33])
    assert ei.value.code == cupk.EINVAL
    ok, busy, tickets = 0, 0, []
    for i in range(0, 600, 8):
        try:
            tickets.append(ctx.submit_updates(u[i:i + 8], v[i:i + 8], d[i:i + 8]))
            ok += 1
        except cupk.CupkError as e:
            assert e.code == cupk.EBUSY
            busy += 1
            break
    for t in tickets:
        assert ctx.wait(t) == 0
    ctx.serve_stop()
    # blocking mode: the same flood always gets in, some submissions wait
    ctx2 = cupk.Context(V, C, D, S)
    ctx2.serve_start(max_batch=16, mem_budget_bytes=8 * 32)
    ts = [ctx2.submit_updates(u[i:i + 8], v[i:i + 8], d[i:i + 8]) for i in range(0, 600, 8)]
    for t in ts:
        assert ctx2.wait(t) == 0
    st = ctx2.serve_stats()
    ctx2.serve_stop()
    ref = oracle.Sketch(V, C, D, S)
    ref.apply(u[:600], v[:600])
    assert ctx2.digest() == ref.digest()
    assert st["updates"] == 600
    ctx.close()
    ctx2.close()


@pytest.mark.parametrize("mode", ["single", "exact", "levels"])
def test_query_bursts(cupk, mode):
    # the paper's query pattern: update periods of random length, each
    # followed by a burst of about period/9 queries; every answer of a burst
    # reflects exactly the updates submitted before it, in every mode
    V, C, D, S = 300, 9, 18, 78
    u, v, d = streamgen.er_standard(V, 0.03, 0.6, 4)
    rng = np.random.default_rng(2)
    live = set()
    ctx = cupk.Context(V, C, D, S, exact=(mode == "exact"), levels=(mode == "levels"))
    ctx.serve_start(max_batch=1 << 16, mem_budget_bytes=1 << 20)
    i, n = 0, len(u)
    bursts = []
    while i < n:
        period = int(rng.integers(100, 200))
        e = min(n, i + period)
        ctx.submit_updates(u[i:e], v[i:e], d[i:e])
        for a, b, x in zip(u[i:e].tolist(), v[i:e].tolist(), d[i:e].tolist()):
            (live.remove if x else live.add)((a, b))
        i = e
        k = max(1, period // 9)
        qa = rng.integers(0, V, k).astype(np.uint32)
        qb = rng.integers(0, V, k).astype(np.uint32)
        eu = np.array([q[0] for q in live], np.uint32)
        ev = np.array([q[1] for q in live], np.uint32)
        lab = oracle.components_truth(V, eu, ev)
        want = [int(lab[a] == lab[b]) for a, b in zip(qa.tolist(), qb.tolist())]
        t, out = ctx.submit_queries(qa, qb)
        bursts.append((t, out, want))
    print(f"bursts mode={mode} n={n} bursts={len(bursts)}", flush=True)
    for t, out, want in bursts:
        assert ctx.wait(t) == 0
        assert out.tolist() == want
    st = ctx.serve_stats()
    ctx.serve_stop()
    assert st["queries"] == sum(len(w) for _, _, w in bursts)
    assert st["query_p99_us"] >= st["query_p50_us"] > 0
    ctx.close()


def test_pipelined_requests_merge_and_match_the_unmerged_run(cupk):
    # One client submits many small update requests without waiting for
    # them, with a query after every 5th: requests admitted while a batch is
    # on the GPU (uploaded into their device slots meanwhile) join the next
    # batch, so there are fewer batches than requests.  Every answer equals
    # the union-find truth at its position and the answer of the same
    # requests applied one at a time (each waited for).
    V, C, D, S = 2000, 11, 22, 0x5EED5E
    u, v, d = streamgen.er_standard(V, 0.002, 0.4, 31)
    sz = 40
    reqs = [(s, min(len(u), s + sz)) for s in range(0, len(u), sz)]
    rng = np.random.default_rng(6)
    qpos = {i: tuple(int(x) for x in rng.integers(0, V, 2)) for i in range(4, len(reqs), 5)}
    uf_truth = {}
    uf = oracle.UnionFind(V)
    live = set()
    for i, (a, b) in enumerate(reqs):
        for x, y, z in zip(u[a:b].tolist(), v[a:b].tolist(), d[a:b].tolist()):
            (live.remove if z else live.add)((x, y))
        if i in qpos:
            lu = np.array([e[0] for e in live], np.uint32)
            lv = np.array([e[1] for e in live], np.uint32)
            _, lab = oracle.uf_components(V, lu, lv)
            uf_truth[i] = int(lab[qpos[i][0]] == lab[qpos[i][1]])

    def run(pipelined):
        ctx = cupk.Context(V, C, D, S)
        ctx.serve_start(max_batch=4096, mem_budget_bytes=64 * sz * 8)
        ans, pend = {}, []
        for i, (a, b) in enumerate(reqs):
            t = ctx.submit_updates(u[a:b], v[a:b], d[a:b])
            if pipelined:
                pend.append(t)
            else:
                assert ctx.wait(t) == 0
            if i in qpos:
                ans[i] = ctx.submit_query(*qpos[i])
        for t in pend:
            assert ctx.wait(t) == 0
        ans = {i: ctx.wait(t) for i, t in ans.items()}
        st = ctx.serve_stats()
        ctx.serve_stop()
        dg = ctx.digest()
        ctx.close()
        return ans, st, dg

    alone, st1, dg1 = run(False)
    mixed, st2, dg2 = run(True)
    print(f"pipelined: {st2['update_requests']} requests in {st2['batches']} batches "
          f"(one at a time: {st1['batches']})", flush=True)
    assert alone == uf_truth and mixed == uf_truth
    assert st1["batches"] == len(reqs)
    assert st2["batches"] < st2["update_requests"] == len(reqs)
    ref = oracle.Sketch(V, C, D, S)
    ref.apply(u, v)
    assert dg1 == dg2 == ref.digest()
