"""The allocation-free entry point cupk_component_sketch_batch_noalloc
against cupk_component_sketch_batch, through the C ABI: the same aggregate
sketches bit for bit, on two calls in a row (the second smaller, so that a
leftover of the first in the shared scratch would show), and the limits."""
import ctypes

import numpy as np
import pytest

import streamgen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cupk():
    import torch
    assert torch.cuda.is_available(), "GPU test on a machine without a GPU"
    import paper_2509_14433_amd as m
    return m


def _csr(sets):
    offs = np.zeros(len(sets) + 1, np.uint64)
    offs[1:] = np.cumsum([len(s) for s in sets])
    verts = (np.concatenate([np.asarray(s, np.uint32) for s in sets]) if offs[-1]
             else np.zeros(1, np.uint32))
    return offs, np.ascontiguousarray(verts, np.uint32)


def _noalloc(cupk, ctx, sets, out=None):
    import torch
    offs, verts = _csr(sets)
    k = len(sets)
    if out is None:
        out = torch.full((max(1, k) * ctx.C * ctx.D * 2,), -1, dtype=torch.int64, device="cuda")
    rc = cupk.lib.cupk_component_sketch_batch_noalloc(
        ctx._h, ctypes.c_void_p(offs.ctypes.data), k, ctypes.c_void_p(verts.ctypes.data),
        ctypes.c_void_p(out.data_ptr()))
    return rc, out


def _as_arrays(ctx, out, k):
    b = out.cpu().numpy().view(np.uint64)[: k * ctx.C * ctx.D * 2].reshape(k, ctx.C, ctx.D, 2)
    return b[..., 0], b[..., 1]


def test_noalloc_matches_the_allocating_entry_point(cupk):
    V, C, D, S = 5000, 13, 26, 0x5EEDA110
    u, v, d = streamgen.er_standard(V, 0.004, 0.3, 91)
    ctx = cupk.Context(V, C, D, S)
    ctx.apply_updates(u, v, d)
    rng = np.random.default_rng(7)
    sizes1 = [int(s) for s in rng.integers(0, 60, 300)]
    sizes1[5] = sizes1[17] = 0          # empty sets
    sizes1[40] = 4000                    # one set spanning many work chunks
    sets1 = [rng.choice(V, size=s, replace=False).tolist() for s in sizes1]
    sets2 = [rng.choice(V, size=s, replace=False).tolist() for s in (3, 0, 40, 1, 500)]
    for call, sets in enumerate((sets1, sets2)):
        print(f"noalloc call {call}: k={len(sets)} members={sum(map(len, sets))}", flush=True)
        rc, out = _noalloc(cupk, ctx, sets)
        assert rc == cupk.OK, cupk.lib.cupk_last_error(ctx._h)
        ga, gg = _as_arrays(ctx, out, len(sets))
        wa, wg = ctx.component_sketch_batch(sets)
        assert np.array_equal(ga, wa) and np.array_equal(gg, wg), call
        assert ga.any()
    ctx.close()


def test_noalloc_limits_and_pending_batch(cupk):
    import torch
    V, C, D, S = 3000, 12, 24, 0x5EEDA111
    ctx = cupk.Context(V, C, D, S)
    u, v, d = streamgen.er_standard(V, 0.01, 0.0, 5)
    one = [[1, 2, 3]]
    # more sets than the scratch holds
    rc, _ = _noalloc(cupk, ctx, [[0]] * 4097)
    assert rc == cupk.EINVAL
    # more members than the scratch holds
    rc, _ = _noalloc(cupk, ctx, [list(range(V))] * 350)
    assert rc == cupk.EINVAL
    # host memory as the output
    offs, verts = _csr(one)
    host = np.zeros(C * D * 2, np.uint64)
    rc = cupk.lib.cupk_component_sketch_batch_noalloc(
        ctx._h, ctypes.c_void_p(offs.ctypes.data), 1, ctypes.c_void_p(verts.ctypes.data),
        ctypes.c_void_p(host.ctypes.data))
    assert rc == cupk.EINVAL
    # a device batch whose host part is pending
    packed = torch.from_numpy(cupk.pack_updates(u, v, d).view(np.int64)).cuda()
    ctx.apply_updates_device(packed)
    rc, _ = _noalloc(cupk, ctx, one)
    assert rc == cupk.EINVAL
    ctx.sync()
    rc, out = _noalloc(cupk, ctx, one)
    assert rc == cupk.OK
    ga, gg = _as_arrays(ctx, out, 1)
    wa, wg = ctx.component_sketch_batch(one)
    assert np.array_equal(ga, wa) and np.array_equal(gg, wg)
    ctx.close()
