"""ctypes binding of ``libcupk.so`` (argument marshalling only).

Every step of the hot path runs in the library's HIP kernels and its C++
runtime; this module only converts numpy arrays / torch tensors to pointers
and sizes.  PyTorch provides the device memory of the sketch and the stream
the library launches on.  If the shared library is missing the import
fails loudly: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

# torch first: its HIP runtime (loaded by name "libamdhip64.so") then
# satisfies this library's dependency on soname "libamdhip64.so.7", so the
# process holds one HIP runtime.  Loading ours first would load a second
# copy, and the two would compete for the device.
try:
    import torch as _torch_mod  # noqa: F401
except Exception:  # pragma: no cover - torch is part of the image
    _torch_mod = None

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcupk.so")

OK, EMPTY, SAMPLE_FAILED = 0, 1, 2
EINVAL, ENOMEM, EDEVICE, EBUSY = -1, -2, -3, -4
SCATTER_ATOMIC, SCATTER_STAGED = 0, 1
LAYOUT_RECORD, LAYOUT_PAIR = 1, 2

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is not built: run `python -c 'import __graft_entry__ as g; g.build()'` "
        "(hipcc --offload-arch=gfx950).  There is no CPU fallback.")


class cupk_bucket(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_uint64), ("gamma", ctypes.c_uint64)]


class cupk_opts(ctypes.Structure):
    _fields_ = [
        ("scatter_mode", ctypes.c_uint32),
        ("max_batch", ctypes.c_uint32),
        ("stream", ctypes.c_void_p),
        ("use_given_stream", ctypes.c_uint32),
        ("sketch_device_ptr", ctypes.c_void_p),
        ("time_kernels", ctypes.c_uint32),
        ("tile_vertices", ctypes.c_uint32),
        ("lds_rows", ctypes.c_uint32),
        ("chunk_records", ctypes.c_uint32),
        ("tile_grid", ctypes.c_uint32),
        ("use_graph", ctypes.c_uint32),
        ("exact", ctypes.c_uint32),
        ("levels", ctypes.c_uint32),
        ("walk_plain", ctypes.c_uint32),
        ("split_rounds", ctypes.c_uint32),
        ("fill_reserve", ctypes.c_uint32),
        ("tile_layout", ctypes.c_uint32),
        ("serial_rounds", ctypes.c_uint32),
        ("coarse_tiles", ctypes.c_uint32),
        ("overlap_min_batch", ctypes.c_uint32),
    ]


class cupk_counters_t(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in (
        "updates", "batches", "flagged", "links", "cuts", "rounds", "sets_reduced",
        "slabs_reduced", "sample_failed", "scatter_launches")] + [
        ("scatter_ms", ctypes.c_double), ("bin_ms", ctypes.c_double),
        ("host_wait_ms", ctypes.c_double), ("host_flags_ms", ctypes.c_double),
        ("host_rounds_ms", ctypes.c_double), ("reverts", ctypes.c_uint64),
        ("level_passes", ctypes.c_uint64), ("level_repairs", ctypes.c_uint64),
        ("level_failed", ctypes.c_uint64),
        ("walks_contracted", ctypes.c_uint64),
        ("walks_fallback", ctypes.c_uint64),
        ("timed_launches", ctypes.c_uint64),
        ("timed_updates", ctypes.c_uint64),
        ("pieces_sketchless", ctypes.c_uint64),
        ("sets_complemented", ctypes.c_uint64),
        ("timed_buckets", ctypes.c_uint64),
        ("overlapped", ctypes.c_uint64)]


class cupk_serve_opts(ctypes.Structure):
    _fields_ = [("max_batch", ctypes.c_uint32), ("nonblocking", ctypes.c_uint32),
                ("mem_budget_bytes", ctypes.c_size_t)]


class cupk_serve_stats_t(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in (
        "update_requests", "queries", "batches", "updates", "admission_waits")] + [
        (n, ctypes.c_double) for n in ("query_p50_us", "query_p99_us", "query_max_us")]


class cupk_tune_result(ctypes.Structure):
    _fields_ = [("tile_vertices", ctypes.c_uint32), ("lds_rows", ctypes.c_uint32),
                ("chunk_records", ctypes.c_uint32), ("candidates", ctypes.c_uint32),
                ("best_ms", ctypes.c_double), ("before_ms", ctypes.c_double),
                ("batch_target", ctypes.c_uint32), ("batch_ms", ctypes.c_double * 8),
                ("batch_sizes", ctypes.c_uint32 * 8), ("host_ms_per_batch", ctypes.c_double),
                ("tile_layout", ctypes.c_uint32), ("coarse_tiles", ctypes.c_uint32)]


class cupk_static_info(ctypes.Structure):
    _fields_ = [("n_components", ctypes.c_uint32), ("rounds", ctypes.c_uint32),
                ("sample_failed", ctypes.c_uint32), ("n_edges", ctypes.c_uint32)]


def _load():
    L = ctypes.CDLL(LIB_PATH)
    p, u32, u64, sz, i32 = (ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64,
                            ctypes.c_size_t, ctypes.c_int32)
    sig = {
        "cupk_sketch_bytes": (sz, [u32, u32, u32]),
        "cupk_sketch_init": (ctypes.c_int, [ctypes.POINTER(p), u32, u32, u32, u64,
                                            ctypes.POINTER(cupk_opts)]),
        "cupk_free": (None, [p]),
        "cupk_apply_updates": (ctypes.c_int, [p, p, p, p, sz]),
        "cupk_apply_updates_device": (ctypes.c_int, [p, p, sz, p]),
        "cupk_component_sketch": (ctypes.c_int, [p, p, sz, p]),
        "cupk_component_sketch_batch": (ctypes.c_int, [p, p, sz, p, p]),
        "cupk_component_sketch_batch_noalloc": (ctypes.c_int, [p, p, sz, p, p]),
        "cupk_sample_cut_edge": (ctypes.c_int, [p, p, ctypes.POINTER(u32), ctypes.POINTER(u32)]),
        "cupk_sample_cut_edge_batch": (ctypes.c_int, [p, p, sz, p, p, p]),
        "cupk_connected": (ctypes.c_int, [p, u32, u32]),
        "cupk_get_sketch": (ctypes.c_int, [p, u32, u32, p]),
        "cupk_digest": (ctypes.c_int, [p, ctypes.POINTER(u64)]),
        "cupk_num_components": (ctypes.c_int, [p, ctypes.POINTER(u64)]),
        "cupk_forest_edges": (ctypes.c_int, [p, p, p, sz, ctypes.POINTER(sz)]),
        "cupk_component_labels": (ctypes.c_int, [p, p]),
        "cupk_level_forest_edges": (ctypes.c_int, [p, u32, p, p, sz, ctypes.POINTER(sz)]),
        "cupk_counters": (ctypes.c_int, [p, ctypes.POINTER(cupk_counters_t)]),
        "cupk_sync": (ctypes.c_int, [p]),
        "cupk_autotune": (ctypes.c_int, [p, p, sz, ctypes.POINTER(cupk_tune_result)]),
        "cupk_static_components": (ctypes.c_int, [p, p, p, p, ctypes.POINTER(cupk_static_info)]),
        "cupk_serve_start": (ctypes.c_int, [p, ctypes.POINTER(cupk_serve_opts)]),
        "cupk_submit_updates": (ctypes.c_int, [p, p, p, p, sz, ctypes.POINTER(u64)]),
        "cupk_submit_query": (ctypes.c_int, [p, u32, u32, ctypes.POINTER(u64)]),
        "cupk_submit_queries": (ctypes.c_int, [p, p, p, sz, p, ctypes.POINTER(u64)]),
        "cupk_wait": (ctypes.c_int, [p, u64, ctypes.POINTER(i32)]),
        "cupk_serve_stats": (ctypes.c_int, [p, ctypes.POINTER(cupk_serve_stats_t)]),
        "cupk_serve_reset_stats": (ctypes.c_int, [p]),
        "cupk_serve_stop": (ctypes.c_int, [p]),
        "cupk_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "cupk_last_error": (ctypes.c_char_p, [p]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    return L


lib = _load()


class CupkError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"cupk error {code}: {msg}")
        self.code = code


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def pack_updates(u, v, is_delete) -> np.ndarray:
    """Device update format: lo32 = u, bits 32..62 = v, bit 63 = delete."""
    u = np.asarray(u, dtype=np.uint64)
    v = np.asarray(v, dtype=np.uint64)
    d = np.asarray(is_delete, dtype=np.uint64)
    return (u | (v << np.uint64(32)) | (d << np.uint64(63))).astype(np.uint64)


def _torch():
    try:
        import torch
    except Exception:  # pragma: no cover - torch is part of the image
        return None
    return torch


class Context:
    """One resident sketch + host forest (``cupk_sketch_init``)."""

    def __init__(self, V, C=0, D=0, seed=0, scatter_mode=SCATTER_STAGED, max_batch=0,
                 stream=None, use_torch_memory=True, time_kernels=False, tile_vertices=0,
                 lds_rows=0, chunk_records=0, tile_grid=0, use_graph=False, exact=False,
                 levels=False, walk_plain=False, split_rounds=False, fill_reserve=False,
                 tile_layout=0, serial_rounds=False, coarse_tiles=0, overlap_min_batch=0):
        self._h = None
        self._sk_tensor = None
        self._keep = {}
        opts = cupk_opts()
        opts.scatter_mode = scatter_mode
        opts.max_batch = max_batch
        # True = every launch; an int k = every k-th launch
        opts.time_kernels = int(time_kernels)
        opts.tile_vertices = tile_vertices
        opts.lds_rows = lds_rows
        opts.chunk_records = chunk_records
        opts.tile_grid = tile_grid
        opts.use_graph = 1 if use_graph else 0
        opts.exact = 1 if exact else 0
        opts.levels = 1 if levels else 0
        opts.walk_plain = 1 if walk_plain else 0
        opts.split_rounds = 1 if split_rounds else 0
        opts.fill_reserve = 1 if fill_reserve else 0
        opts.tile_layout = tile_layout
        opts.serial_rounds = 1 if serial_rounds else 0
        opts.coarse_tiles = coarse_tiles
        opts.overlap_min_batch = overlap_min_batch
        torch = _torch()
        if stream is None and torch is not None and torch.cuda.is_available():
            # launch on torch's current stream so that torch-produced device
            # batches are ordered before the library's kernels
            stream = torch.cuda.current_stream().cuda_stream
        if stream is not None:
            opts.stream = stream
            opts.use_given_stream = 1
        L = 1
        while (1 << L) < V:
            L += 1
        self.V = V
        self.C = C or L
        self.D = D or 2 * L
        self.seed = seed
        if use_torch_memory and torch is not None and torch.cuda.is_available():
            nbytes = lib.cupk_sketch_bytes(V, self.C, self.D)
            self._sk_tensor = torch.empty(nbytes // 8, dtype=torch.int64, device="cuda")
            opts.sketch_device_ptr = self._sk_tensor.data_ptr()
        h = ctypes.c_void_p()
        rc = lib.cupk_sketch_init(ctypes.byref(h), V, C, D, seed, ctypes.byref(opts))
        if rc != OK:
            raise CupkError(rc, lib.cupk_strerror(rc).decode() + ": " +
                            lib.cupk_last_error(None).decode())
        self._h = h

    def close(self):
        if self._h:
            lib.cupk_free(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def _check(self, rc):
        if rc < 0:
            raise CupkError(rc, lib.cupk_last_error(self._h).decode() or
                            lib.cupk_strerror(rc).decode())
        return rc

    @property
    def sketch_tensor(self):
        """The torch tensor holding the device sketch (when torch memory is used)."""
        return self._sk_tensor

    # -- hot path -------------------------------------------------------------
    def apply_updates(self, u, v, is_delete):
        u = np.ascontiguousarray(u, dtype=np.uint32)
        v = np.ascontiguousarray(v, dtype=np.uint32)
        d = np.ascontiguousarray(is_delete, dtype=np.uint8)
        n = u.shape[0]
        if v.shape[0] != n or d.shape[0] != n:
            raise ValueError("u, v, is_delete must have equal length")
        return self._check(lib.cupk_apply_updates(self._h, _ptr(u), _ptr(v), _ptr(d), n))

    def apply_updates_device(self, packed, n=None, stream=None):
        """packed: a cuda int64/uint64 tensor (or a raw device address with n).
        stream: the hipStream_t (int) that produced it; default torch's
        current stream.  Returns once the device work is queued; the host
        part runs at the next call that needs it (see cupk.h)."""
        if isinstance(packed, int):
            ptr = packed
            assert n is not None
        else:
            assert packed.is_cuda and packed.element_size() == 8 and packed.is_contiguous()
            ptr = packed.data_ptr()
            n = packed.numel() if n is None else n
        if stream is None:
            torch = _torch()
            stream = torch.cuda.current_stream().cuda_stream if torch is not None else 0
        return self._check(lib.cupk_apply_updates_device(self._h, ctypes.c_void_p(ptr), n,
                                                         ctypes.c_void_p(stream or None)))

    def component_sketch(self, verts, out=None):
        """(alpha, gamma) as C x D arrays; with out (a cuda tensor of
        C*D*2 int64), the canonical buckets are written there instead."""
        if out is not None:
            return self.component_sketch_batch([verts], out=out)
        verts = np.ascontiguousarray(verts, dtype=np.uint32)
        buf = np.zeros(self.C * self.D * 2, dtype=np.uint64)
        self._check(lib.cupk_component_sketch(self._h, _ptr(verts), verts.shape[0], _ptr(buf)))
        buf = buf.reshape(self.C, self.D, 2)
        return buf[..., 0].copy(), buf[..., 1].copy()

    def component_sketch_batch(self, sets, out=None):
        """(alpha, gamma) as k x C x D arrays; with out (a cuda tensor of
        k*C*D*2 int64), the canonical buckets are written there instead
        and out is returned."""
        sizes = [len(s) for s in sets]
        offs = np.zeros(len(sets) + 1, dtype=np.uint64)
        offs[1:] = np.cumsum(sizes)
        verts = (np.ascontiguousarray(np.concatenate([np.asarray(s, np.uint32) for s in sets]))
                 if sets and offs[-1] else np.zeros(1, np.uint32))
        k = len(sets)
        if out is not None:
            assert out.is_cuda and out.element_size() == 8 and out.is_contiguous()
            assert out.numel() >= k * self.C * self.D * 2
            self._check(lib.cupk_component_sketch_batch(self._h, _ptr(offs), k, _ptr(verts),
                                                         ctypes.c_void_p(out.data_ptr())))
            return out
        buf = np.zeros(max(1, k) * self.C * self.D * 2, dtype=np.uint64)
        self._check(lib.cupk_component_sketch_batch(self._h, _ptr(offs), k, _ptr(verts),
                                                     _ptr(buf)))
        buf = buf[: k * self.C * self.D * 2].reshape(k, self.C, self.D, 2)
        return buf[..., 0].copy(), buf[..., 1].copy()

    def sample_cut_edge(self, alpha, gamma):
        buf = np.empty((self.C, self.D, 2), dtype=np.uint64)
        buf[..., 0] = np.asarray(alpha, np.uint64).reshape(self.C, self.D)
        buf[..., 1] = np.asarray(gamma, np.uint64).reshape(self.C, self.D)
        uu, vv = ctypes.c_uint32(0), ctypes.c_uint32(0)
        st = self._check(lib.cupk_sample_cut_edge(self._h, _ptr(buf), ctypes.byref(uu),
                                                  ctypes.byref(vv)))
        return (st, uu.value, vv.value) if st == OK else (st, 0, 0)

    def sample_cut_edge_batch(self, alpha, gamma):
        alpha = np.asarray(alpha, np.uint64).reshape(-1, self.C, self.D)
        k = alpha.shape[0]
        buf = np.empty((k, self.C, self.D, 2), dtype=np.uint64)
        buf[..., 0] = alpha
        buf[..., 1] = np.asarray(gamma, np.uint64).reshape(k, self.C, self.D)
        st = np.zeros(max(1, k), np.int32)
        u = np.zeros(max(1, k), np.uint32)
        v = np.zeros(max(1, k), np.uint32)
        self._check(lib.cupk_sample_cut_edge_batch(self._h, _ptr(buf), k, _ptr(st), _ptr(u),
                                                   _ptr(v)))
        return st[:k], u[:k], v[:k]

    def connected(self, u, v) -> bool:
        return bool(self._check(lib.cupk_connected(self._h, u, v)))

    # -- introspection ------------------------------------------------------------
    def get_sketch(self, w0=0, nv=None):
        nv = self.V - w0 if nv is None else nv
        out = np.zeros(max(1, nv) * self.C * self.D * 2, dtype=np.uint64)
        self._check(lib.cupk_get_sketch(self._h, w0, nv, _ptr(out)))
        out = out[: nv * self.C * self.D * 2].reshape(nv, self.C, self.D, 2)
        return out[..., 0].copy(), out[..., 1].copy()

    def digest(self) -> int:
        o = ctypes.c_uint64(0)
        self._check(lib.cupk_digest(self._h, ctypes.byref(o)))
        return o.value

    def num_components(self) -> int:
        o = ctypes.c_uint64(0)
        self._check(lib.cupk_num_components(self._h, ctypes.byref(o)))
        return o.value

    def forest_edge_arrays(self):
        """Forest edges as two uint32 arrays (u < v), in the library's order."""
        n = ctypes.c_size_t(0)
        cap = self.V
        u = np.zeros(cap, np.uint32)
        v = np.zeros(cap, np.uint32)
        self._check(lib.cupk_forest_edges(self._h, _ptr(u), _ptr(v), cap, ctypes.byref(n)))
        return u[: n.value].copy(), v[: n.value].copy()

    def forest_edges(self):
        u, v = self.forest_edge_arrays()
        return sorted(zip(u.tolist(), v.tolist()))

    def level_forest_edges(self, level):
        """Levels mode: edges of the forest of `level` (1..C)."""
        n = ctypes.c_size_t(0)
        u = np.zeros(self.V, np.uint32)
        v = np.zeros(self.V, np.uint32)
        self._check(lib.cupk_level_forest_edges(self._h, level, _ptr(u), _ptr(v), self.V,
                                                ctypes.byref(n)))
        return sorted(zip(u[: n.value].tolist(), v[: n.value].tolist()))

    def component_labels(self):
        out = np.zeros(self.V, np.uint32)
        self._check(lib.cupk_component_labels(self._h, _ptr(out)))
        return out

    def static_components(self):
        """Components from the sketches alone (``cupk_static_components``):
        (labels = smallest vertex per component, merge edges in merge order,
        info dict)."""
        labels = np.zeros(self.V, np.uint32)
        eu = np.zeros(max(1, self.V - 1), np.uint32)
        ev = np.zeros(max(1, self.V - 1), np.uint32)
        info = cupk_static_info()
        self._check(lib.cupk_static_components(self._h, _ptr(labels), _ptr(eu), _ptr(ev),
                                               ctypes.byref(info)))
        n = info.n_edges
        edges = list(zip(eu[:n].tolist(), ev[:n].tolist()))
        return labels, edges, {f: getattr(info, f) for f, _ in cupk_static_info._fields_}

    def counters(self) -> dict:
        c = cupk_counters_t()
        self._check(lib.cupk_counters(self._h, ctypes.byref(c)))
        return {f: getattr(c, f) for f, _ in cupk_counters_t._fields_}

    def sync(self):
        self._check(lib.cupk_sync(self._h))

    def autotune(self, sample) -> dict:
        """Tune the staged scatter on a device sample batch (cuda tensor of
        packed updates); the sketch is left unchanged."""
        assert sample.is_cuda and sample.element_size() == 8 and sample.is_contiguous()
        r = cupk_tune_result()
        self._check(lib.cupk_autotune(self._h, ctypes.c_void_p(sample.data_ptr()),
                                      sample.numel(), ctypes.byref(r)))
        out = {f: getattr(r, f) for f, _ in cupk_tune_result._fields_}
        out["batch_ms"] = list(r.batch_ms)
        out["batch_sizes"] = list(r.batch_sizes)
        return out

    # -- serving loop ---------------------------------------------------------------
    def serve_start(self, max_batch=0, mem_budget_bytes=0, nonblocking=False):
        o = cupk_serve_opts(max_batch, 1 if nonblocking else 0, mem_budget_bytes)
        self._check(lib.cupk_serve_start(self._h, ctypes.byref(o)))

    def submit_updates(self, u, v, is_delete) -> int:
        u = np.ascontiguousarray(u, dtype=np.uint32)
        v = np.ascontiguousarray(v, dtype=np.uint32)
        d = np.ascontiguousarray(is_delete, dtype=np.uint8)
        t = ctypes.c_uint64(0)
        self._check(lib.cupk_submit_updates(self._h, _ptr(u), _ptr(v), _ptr(d), u.shape[0],
                                            ctypes.byref(t)))
        return t.value

    def submit_query(self, u, v) -> int:
        t = ctypes.c_uint64(0)
        self._check(lib.cupk_submit_query(self._h, u, v, ctypes.byref(t)))
        return t.value

    def submit_queries(self, u, v):
        """Submit a burst of queries; returns (ticket, answers array).  The
        answers are valid after wait(ticket)."""
        u = np.ascontiguousarray(u, dtype=np.uint32)
        v = np.ascontiguousarray(v, dtype=np.uint32)
        assert u.shape == v.shape
        out = np.full(u.shape[0], -1, np.int32)
        t = ctypes.c_uint64(0)
        self._check(lib.cupk_submit_queries(self._h, _ptr(u), _ptr(v), u.shape[0], _ptr(out),
                                            ctypes.byref(t)))
        # the library writes into these arrays until the burst is answered
        self._keep[t.value] = (u, v, out)
        return t.value, out

    def wait(self, ticket) -> int:
        r = ctypes.c_int32(0)
        self._check(lib.cupk_wait(self._h, ticket, ctypes.byref(r)))
        self._keep.pop(ticket, None)
        return r.value

    def serve_stats(self) -> dict:
        st = cupk_serve_stats_t()
        self._check(lib.cupk_serve_stats(self._h, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in cupk_serve_stats_t._fields_}

    def serve_reset_stats(self):
        self._check(lib.cupk_serve_reset_stats(self._h))

    def serve_stop(self):
        self._check(lib.cupk_serve_stop(self._h))
        self._keep.clear()
