"""Oracle for sketch-based dynamic connectivity (test infrastructure only).

A plain CPU implementation of what the GPU hot path computes, used by the
tests, the smoke check and the CPU-baseline leg of the benchmark, and by
nothing else.  It shares no code with the product library: the sketch
arithmetic lives in ``oracle.c`` (built with gcc into ``liboracle.so``), the
forest replay and the connectivity truth are plain Python below.

Paper: "Fast and Compact Sketch-Based Dynamic Connectivity" (arXiv
2509.14433).  See ``oracle.c`` for the sketch definition and the readings of
the points the paper leaves open.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_LIB names another build of oracle.c to load instead (the mutation
# test uses it to check that the pins catch planted mistakes).
_BUILT = os.path.join(_HERE, "liboracle.so")
_SO = os.environ.get("ORACLE_LIB") or _BUILT
_SRC = os.path.join(_HERE, "oracle.c")

OK, EMPTY, FAILED = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` with gcc into ``liboracle.so`` (in place)."""
    if force or not os.path.exists(_BUILT):
        tmp = _BUILT + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-shared", "-fPIC",
                               "-o", tmp, _SRC])
        os.replace(tmp, _BUILT)
    return _BUILT


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        L = ctypes.CDLL(_SO)
        u64, u32, sz, p = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_size_t, ctypes.c_void_p
        L.orc_mix.restype = u64; L.orc_mix.argtypes = [u64]
        L.orc_seed.restype = u64; L.orc_seed.argtypes = [u64, u32]
        L.orc_hash.restype = u64; L.orc_hash.argtypes = [u64, u32, u64]
        L.orc_depth_of_hash.restype = u32; L.orc_depth_of_hash.argtypes = [u64, u32]
        L.orc_edge_index.restype = u64; L.orc_edge_index.argtypes = [u32, u32, u32]
        L.orc_valid_index.restype = ctypes.c_int; L.orc_valid_index.argtypes = [u32, u64]
        L.orc_new.restype = p; L.orc_new.argtypes = [u32, u32, u32, u64]
        L.orc_free.restype = None; L.orc_free.argtypes = [p]
        L.orc_clear.restype = None; L.orc_clear.argtypes = [p]
        L.orc_alpha.restype = p; L.orc_alpha.argtypes = [p]
        L.orc_gamma.restype = p; L.orc_gamma.argtypes = [p]
        L.orc_toggle.restype = None; L.orc_toggle.argtypes = [p, u32, u32]
        L.orc_apply.restype = None; L.orc_apply.argtypes = [p, p, p, sz]
        if hasattr(L, "orc_apply_threads"):
            L.orc_apply_threads.restype = ctypes.c_int
            L.orc_apply_threads.argtypes = [p, p, p, sz, ctypes.c_int]
        L.orc_vertex_from_stream.restype = None
        L.orc_vertex_from_stream.argtypes = [u32, u32, u32, u64, u32, p, p, sz, p, p]
        L.orc_set_sketch.restype = None; L.orc_set_sketch.argtypes = [p, p, sz, p, p]
        L.orc_sample.restype = ctypes.c_int
        L.orc_sample.argtypes = [u32, u32, u32, u64, p, p, p, p]
        L.orc_sample_col.restype = ctypes.c_int
        L.orc_sample_col.argtypes = [u32, u32, u32, u64, u32, p, p, p, p]
        L.orc_digest.restype = u64; L.orc_digest.argtypes = [p]
        if hasattr(L, "orc_uf_new"):
            L.orc_uf_new.restype = p; L.orc_uf_new.argtypes = [u32]
            L.orc_uf_free.restype = None; L.orc_uf_free.argtypes = [p]
            L.orc_uf_add.restype = u64; L.orc_uf_add.argtypes = [p, p, p, sz]
            L.orc_uf_same.restype = ctypes.c_int; L.orc_uf_same.argtypes = [p, u32, u32]
        if hasattr(L, "orc_uf_components"):
            L.orc_uf_components.restype = u64
            L.orc_uf_components.argtypes = [u32, p, p, sz, p]
        L.orc_digest_arrays.restype = u64
        L.orc_digest_arrays.argtypes = [u32, u32, u64, u32, u32, p, p]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


# ---- scalar hash functions ------------------------------------------------

def mix(z: int) -> int:
    return lib().orc_mix(z & 0xFFFFFFFFFFFFFFFF)


def seed(S: int, c: int) -> int:
    return lib().orc_seed(S, c)


def hash_c(S: int, c: int, x: int) -> int:
    return lib().orc_hash(S, c, x)


def depth_of_hash(h: int, D: int) -> int:
    return lib().orc_depth_of_hash(h, D)


def edge_index(V: int, a: int, b: int) -> int:
    return lib().orc_edge_index(V, a, b)


# ---- sketch state -----------------------------------------------------------

class Sketch:
    """All vertex sketches of a graph on V vertices: C columns x D depth
    buckets of (alpha, gamma) per vertex, canonical order [w][c][d]."""

    def __init__(self, V: int, C: int, D: int, S: int):
        self.V, self.C, self.D, self.S = V, C, D, S
        self._h = lib().orc_new(V, C, D, S)
        if not self._h:
            raise MemoryError("oracle sketch allocation failed")

    def __del__(self):
        if getattr(self, "_h", None):
            lib().orc_free(self._h)
            self._h = None

    def clear(self):
        lib().orc_clear(self._h)

    def apply(self, u, v):
        u = np.ascontiguousarray(u, dtype=np.uint32)
        v = np.ascontiguousarray(v, dtype=np.uint32)
        assert u.shape == v.shape
        lib().orc_apply(self._h, _ptr(u), _ptr(v), u.shape[0])

    def apply_threads(self, u, v, nthreads: int) -> int:
        """``apply`` with the vertex range split over host threads (each
        thread writes only the buckets of its own vertices, in stream order:
        the same result).  Returns the number of threads used."""
        u = np.ascontiguousarray(u, dtype=np.uint32)
        v = np.ascontiguousarray(v, dtype=np.uint32)
        assert u.shape == v.shape
        return lib().orc_apply_threads(self._h, _ptr(u), _ptr(v), u.shape[0], int(nthreads))

    def toggle(self, a: int, b: int):
        lib().orc_toggle(self._h, a, b)

    def _view(self, fn):
        n = self.V * self.C * self.D
        buf = (ctypes.c_uint64 * n).from_address(fn(self._h))
        return np.frombuffer(buf, dtype=np.uint64).reshape(self.V, self.C, self.D)

    @property
    def alpha(self) -> np.ndarray:
        return self._view(lib().orc_alpha)

    @property
    def gamma(self) -> np.ndarray:
        return self._view(lib().orc_gamma)

    def set_sketch(self, verts):
        verts = np.ascontiguousarray(verts, dtype=np.uint32)
        a = np.zeros(self.C * self.D, np.uint64)
        g = np.zeros(self.C * self.D, np.uint64)
        lib().orc_set_sketch(self._h, _ptr(verts), verts.shape[0], _ptr(a), _ptr(g))
        return a.reshape(self.C, self.D), g.reshape(self.C, self.D)

    def sample(self, alpha, gamma):
        return sample(self.V, self.C, self.D, self.S, alpha, gamma)

    def digest(self) -> int:
        return lib().orc_digest(self._h)


def sample(V, C, D, S, alpha, gamma):
    """(status, u, v) of the query on one aggregate sketch."""
    a = np.ascontiguousarray(alpha, dtype=np.uint64).reshape(-1)
    g = np.ascontiguousarray(gamma, dtype=np.uint64).reshape(-1)
    assert a.shape[0] == C * D and g.shape[0] == C * D
    ou, ov = ctypes.c_uint32(0), ctypes.c_uint32(0)
    st = lib().orc_sample(V, C, D, S, _ptr(a), _ptr(g), ctypes.byref(ou), ctypes.byref(ov))
    if st != OK:
        return st, 0, 0
    return st, ou.value, ov.value


def sample_col(V, C, D, S, c, alpha, gamma):
    """(status, u, v) of the query of column c alone on one aggregate
    sketch (C x D arrays): the sampler of level c of the hierarchy."""
    a = np.ascontiguousarray(alpha, dtype=np.uint64).reshape(-1)
    g = np.ascontiguousarray(gamma, dtype=np.uint64).reshape(-1)
    assert a.shape[0] == C * D and g.shape[0] == C * D and 0 <= c < C
    ou, ov = ctypes.c_uint32(0), ctypes.c_uint32(0)
    st = lib().orc_sample_col(V, C, D, S, c, _ptr(a), _ptr(g), ctypes.byref(ou), ctypes.byref(ov))
    if st != OK:
        return st, 0, 0
    return st, ou.value, ov.value


def uf_components(V, u, v):
    """(number of components, label array: smallest vertex of each vertex's
    component) of the graph with edge list (u, v), by union-find in C."""
    u = np.ascontiguousarray(u, dtype=np.uint32)
    v = np.ascontiguousarray(v, dtype=np.uint32)
    lab = np.zeros(V, np.uint32)
    k = lib().orc_uf_components(V, _ptr(u), _ptr(v), u.shape[0], _ptr(lab))
    if k == 0 and V > 0:
        raise MemoryError("union-find allocation failed")
    return int(k), lab


class UnionFind:
    """Connectivity truth along a growing edge set (union-find in C)."""

    def __init__(self, V: int):
        self._h = lib().orc_uf_new(V)
        if not self._h:
            raise MemoryError("union-find allocation failed")
        self.n_components = V

    def __del__(self):
        if getattr(self, "_h", None):
            lib().orc_uf_free(self._h)
            self._h = None

    def add(self, u, v) -> int:
        u = np.ascontiguousarray(u, dtype=np.uint32)
        v = np.ascontiguousarray(v, dtype=np.uint32)
        self.n_components = int(lib().orc_uf_add(self._h, _ptr(u), _ptr(v), u.shape[0]))
        return self.n_components

    def same(self, a: int, b: int) -> bool:
        return bool(lib().orc_uf_same(self._h, a, b))


def vertex_from_stream(V, C, D, S, w, u, v):
    """Sketch of vertex w from the updates that touch it (C x D arrays)."""
    u = np.ascontiguousarray(u, dtype=np.uint32)
    v = np.ascontiguousarray(v, dtype=np.uint32)
    a = np.zeros(C * D, np.uint64)
    g = np.zeros(C * D, np.uint64)
    lib().orc_vertex_from_stream(V, C, D, S, w, _ptr(u), _ptr(v), u.shape[0], _ptr(a), _ptr(g))
    return a.reshape(C, D), g.reshape(C, D)


def digest_arrays(C, D, S, w0, alpha, gamma) -> int:
    """Digest contribution of vertices w0 .. w0+len-1 given as (n, C, D)
    alpha / gamma arrays in canonical order."""
    a = np.ascontiguousarray(alpha, dtype=np.uint64)
    g = np.ascontiguousarray(gamma, dtype=np.uint64)
    nv = a.shape[0]
    assert a.shape == (nv, C, D) and g.shape == a.shape
    return lib().orc_digest_arrays(C, D, S, w0, nv, _ptr(a), _ptr(g))


from .forest import ForestReplay, components_truth, check_spanning_forest  # noqa: E402
from .static_cc import static_components  # noqa: E402
from .levels import LevelsReplay  # noqa: E402

__all__ = [
    "OK", "EMPTY", "FAILED", "build", "lib", "mix", "seed", "hash_c",
    "depth_of_hash", "edge_index", "Sketch", "sample", "sample_col", "vertex_from_stream",
    "digest_arrays", "uf_components", "UnionFind", "ForestReplay", "components_truth", "check_spanning_forest",
    "static_components", "LevelsReplay",
]
