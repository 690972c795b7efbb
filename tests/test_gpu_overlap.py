"""Overlapped device batches.  A device batch of more than 4096 updates that
follows a pending device batch is classified against the forest as the
pending batch's flag walk left it and binned while that batch's replacement
rounds run; its flags are then checked again against the forest after the
rounds, before its scatter.  The result must be the oracle's batch-by-batch
replay (sketch digest, forest, links, cuts, rounds) and, counter for
counter, the serial order's (serial_rounds): on the ragged R-MAT stream
(small and large batches interleaved, 15% deletions), on clustered churn
(bridges cut and relinked in every batch) and on the fixed-forest stream
(no cut at all: every batch takes the serial order, since its rounds have
nothing to search), with every scatter timed and untimed, staged and plain.
An invalid batch is reported by the next call, which then applies nothing.
"""
import numpy as np
import pytest

import oracle
import streamgen

pytestmark = pytest.mark.gpu

SMALL_MAX = 4096  # larger batches take the staged pass (and may overlap)
# (scaled workload, batch size; None: the recipe's ragged sizes)
WORKLOADS = {"rmat": (2, None), "clusters": (4, 5000), "fixed": (5, 50_000)}
# (not timed_buckets: a bucket changed by records of two work items of one
# tile counts twice, and where the fill's atomics put a tile's records
# decides that, in any order of passes)
SAME = ("updates", "batches", "flagged", "links", "cuts", "rounds", "sets_reduced",
        "slabs_reduced", "sample_failed", "scatter_launches", "walks_contracted",
        "walks_fallback", "timed_launches", "timed_updates", "pieces_sketchless",
        "sets_complemented")


@pytest.fixture(scope="module")
def cupk():
    import torch
    assert torch.cuda.is_available()
    import paper_2509_14433_amd as m
    return m


def _sizes(k, batch, n):
    if batch is None:
        cfg = streamgen.SCALED[k]
        return streamgen.ragged_sizes(n, cfg["batch"][0], cfg["batch"][1], cfg["seed"])
    return [min(batch, n - s) for s in range(0, n, batch)]


_REF = {}


def _reference(name, skip=None):
    """Oracle replay of the workload in its batches (batch `skip` left out)."""
    key = (name, skip)
    if key not in _REF:
        k, batch = WORKLOADS[name]
        cfg = streamgen.SCALED[k]
        V = cfg["V"]
        C = streamgen.ceil_log2(V)
        D = 2 * C
        u, v, d = streamgen.config_stream(k, scaled=True)
        sizes = _sizes(k, batch, len(u))
        sk = oracle.Sketch(V, C, D, cfg["S"])
        fr = oracle.ForestReplay(sk)
        off = 0
        for i, s in enumerate(sizes):
            if i != skip:
                fr.apply_batch(u[off:off + s], v[off:off + s], d[off:off + s])
            off += s
        _REF[key] = dict(V=V, C=C, D=D, S=cfg["S"], u=u, v=v, d=d, sizes=sizes,
                         digest=sk.digest(), forest=fr.forest_edges(),
                         counts=(fr.n_links, fr.n_cuts, fr.n_rounds))
    return _REF[key]


def _run(cupk, R, serial, timed, mode, bad=None):
    import torch
    sm = cupk.SCATTER_ATOMIC if mode == "atomic" else cupk.SCATTER_STAGED
    # (overlap_min_batch 1: these small batches overlap too)
    ctx = cupk.Context(R["V"], R["C"], R["D"], R["S"], scatter_mode=sm,
                       max_batch=max(R["sizes"]), time_kernels=timed, serial_rounds=serial,
                       overlap_min_batch=1)
    packed = torch.from_numpy(cupk.pack_updates(R["u"], R["v"], R["d"]).view(np.int64)).cuda()
    off = 0
    for i, s in enumerate(R["sizes"]):
        b = packed[off:off + s]
        if i == bad:
            b = b.clone()
            b[s // 2] = 5 | (5 << 32)  # u == v: the whole batch is rejected
        ctx.apply_updates_device(b)
        off += s
        if i == bad:
            # the next call completes the rejected batch and reports it
            nxt = packed[off:off + R["sizes"][i + 1]]
            with pytest.raises(cupk.CupkError) as ei:
                ctx.apply_updates_device(nxt)
            assert ei.value.code == cupk.EINVAL
    ctx.sync()
    torch.cuda.synchronize()
    return ctx


@pytest.mark.parametrize("name", list(WORKLOADS))
@pytest.mark.parametrize("timed", [False, True])
def test_overlapped_batches_match_oracle_and_serial(cupk, name, timed):
    R = _reference(name)
    print(f"overlap {name} n={len(R['u'])} batches={len(R['sizes'])} timed={timed}", flush=True)
    ctxs = {}
    for serial in (False, True):
        ctx = _run(cupk, R, serial, timed, "staged")
        assert ctx.digest() == R["digest"], serial
        assert ctx.forest_edges() == R["forest"], serial
        ctr = ctx.counters()
        assert (ctr["links"], ctr["cuts"], ctr["rounds"]) == R["counts"], serial
        ctxs[serial] = (ctx, ctr)
    a, b = ctxs[False][1], ctxs[True][1]
    assert {k: a[k] for k in SAME} == {k: b[k] for k in SAME}
    # a batch after a walk that left broken trees unsplit, or fewer than two
    # dirty trees, takes the serial order; the fixed-forest stream has no
    # cut at all, so nothing for the rounds to hide
    want = sum(1 for s in R["sizes"][1:] if s > SMALL_MAX)
    if name == "fixed":
        assert a["overlapped"] == 0
    else:
        assert 0 < a["overlapped"] <= want
    assert b["overlapped"] == 0
    if timed:
        assert a["timed_launches"] > 0 and a["scatter_ms"] > 0 and a["bin_ms"] > 0
    assert np.array_equal(ctxs[False][0].component_labels(), ctxs[True][0].component_labels())
    for ctx, _ in ctxs.values():
        ctx.close()


def test_overlapped_batches_plain_scatter(cupk):
    R = _reference("clusters")
    print(f"overlap clusters atomic n={len(R['u'])}", flush=True)
    ctx = _run(cupk, R, False, False, "atomic")
    assert ctx.digest() == R["digest"]
    assert ctx.forest_edges() == R["forest"]
    ctr = ctx.counters()
    assert (ctr["links"], ctr["cuts"], ctr["rounds"]) == R["counts"]
    assert 0 < ctr["overlapped"] <= sum(1 for s in R["sizes"][1:] if s > SMALL_MAX)
    ctx.close()


@pytest.mark.parametrize("serial", [False, True])
def test_invalid_batch_between_overlapped_batches(cupk, serial):
    bad = 3
    R = _reference("clusters", skip=bad)
    print(f"overlap invalid batch {bad} serial={serial}", flush=True)
    ctx = _run(cupk, R, serial, False, "staged", bad=bad)
    assert ctx.digest() == R["digest"]
    assert ctx.forest_edges() == R["forest"]
    ctr = ctx.counters()
    assert (ctr["links"], ctr["cuts"], ctr["rounds"]) == R["counts"]
    ctx.close()


def test_small_batches_take_the_serial_order_by_default(cupk):
    # below overlap_min_batch (default 4,194,304 updates) no batch overlaps
    import torch
    R = _reference("clusters")
    ctx = cupk.Context(R["V"], R["C"], R["D"], R["S"], max_batch=max(R["sizes"]))
    packed = torch.from_numpy(cupk.pack_updates(R["u"], R["v"], R["d"]).view(np.int64)).cuda()
    off = 0
    for s in R["sizes"]:
        ctx.apply_updates_device(packed[off:off + s])
        off += s
    ctx.sync()
    assert ctx.counters()["overlapped"] == 0
    assert ctx.digest() == R["digest"]
    assert ctx.forest_edges() == R["forest"]
    ctx.close()
