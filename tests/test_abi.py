"""The C-ABI library loads and exports every symbol the header declares
(no compute calls: these run without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cupk.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cupk_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_symbols()
    for want in ("cupk_sketch_init", "cupk_apply_updates", "cupk_apply_updates_device",
                 "cupk_component_sketch", "cupk_component_sketch_batch",
                 "cupk_sample_cut_edge", "cupk_sample_cut_edge_batch", "cupk_connected",
                 "cupk_free", "cupk_digest", "cupk_get_sketch"):
        assert want in names


def _prototype(name):
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    m = re.search(r"\b" + name + r"\s*\(([^)]*)\)", text)
    assert m, name
    return [a.strip() for a in m.group(1).split(",")]


def test_device_apply_takes_a_stream():
    # (ctx, device batch, count, hipStream_t the batch was produced on)
    args = _prototype("cupk_apply_updates_device")
    assert len(args) == 4
    assert args[1].startswith("const uint64_t *") and args[2].startswith("size_t")
    assert args[3].replace(" ", "") == "void*hip_stream"
    import paper_2509_14433_amd as cupk
    assert len(cupk.lib.cupk_apply_updates_device.argtypes) == 4


def test_library_exports_every_declared_symbol():
    import paper_2509_14433_amd as cupk
    lib = ctypes.CDLL(cupk.LIB_PATH)
    missing = [n for n in declared_symbols() if not hasattr(lib, n)]
    assert not missing, missing


def test_host_only_calls_without_gpu():
    import paper_2509_14433_amd as cupk
    assert cupk.lib.cupk_sketch_bytes(16384, 14, 28) == 16384 * 14 * 28 * 16
    assert cupk.lib.cupk_strerror(-1) == b"invalid argument"
    assert cupk.lib.cupk_strerror(2).startswith(b"sample failed")
    # argument checks that return before touching the device
    h = ctypes.c_void_p()
    assert cupk.lib.cupk_sketch_init(ctypes.byref(h), 1, 0, 0, 0, None) == cupk.EINVAL
    assert cupk.lib.cupk_sketch_init(ctypes.byref(h), 16, 65, 0, 0, None) == cupk.EINVAL
    assert cupk.lib.cupk_sketch_init(ctypes.byref(h), 16, 4, 1, 0, None) == cupk.EINVAL
    assert cupk.lib.cupk_connected(None, 0, 1) == cupk.EINVAL
    assert cupk.lib.cupk_static_components(None, None, None, None, None) == cupk.EINVAL
    assert cupk.lib.cupk_level_forest_edges(None, 1, None, None, 0, None) == cupk.EINVAL


def test_packing_format():
    import numpy as np
    import paper_2509_14433_amd as cupk
    p = cupk.pack_updates(np.array([3, 7]), np.array([5, 2]), np.array([0, 1]))
    assert p[0] == 3 | (5 << 32)
    assert int(p[1]) == 7 | (2 << 32) | (1 << 63)


@pytest.mark.gpu
def test_context_roundtrip_on_gpu():
    import paper_2509_14433_amd as cupk
    ctx = cupk.Context(64, 4, 8, 1)
    assert ctx.num_components() == 64
    assert ctx.digest() == ctx.digest()
    ctx.close()


def test_binding_structs_match_the_header(tmp_path):
    # every field of every struct the binding mirrors: offset and size as a C
    # compiler lays out the header's definition
    import shutil
    import subprocess
    import paper_2509_14433_amd._binding as b
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    structs = [b.cupk_bucket, b.cupk_opts, b.cupk_counters_t, b.cupk_static_info,
               b.cupk_tune_result, b.cupk_serve_opts, b.cupk_serve_stats_t]
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "cupk.h"', "int main(void) {"]
    for st in structs:
        lines.append(f'printf("{st.__name__} %zu\\n", sizeof({st.__name__}));')
        for f, _ in st._fields_:
            lines.append(f'printf("{st.__name__}.{f} %zu\\n", offsetof({st.__name__}, {f}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = dict(ln.split() for ln in subprocess.run([str(exe)], check=True, capture_output=True,
                                                   text=True).stdout.splitlines())
    for st in structs:
        assert int(got[st.__name__]) == ctypes.sizeof(st), st.__name__
        for f, _ in st._fields_:
            assert int(got[f"{st.__name__}.{f}"]) == getattr(st, f).offset, (st.__name__, f)
