"""cupk: sketch-based dynamic connectivity hot path on one MI355X (gfx950).

The data-parallel part of the CUPCaKE method (arXiv 2509.14433): resident
per-vertex l0-sketches, batched XOR scatter of edge updates, component
XOR-reduction and bucket verify/sample run as hand-written HIP kernels
behind a C ABI (``include/cupk.h``); the spanning forest lives in the
library's C++ host runtime.  This package is the thin Python binding.
"""
from ._binding import (  # noqa: F401
    Context, CupkError, pack_updates, lib, LIB_PATH,
    OK, EMPTY, SAMPLE_FAILED, EINVAL, ENOMEM, EDEVICE, EBUSY,
    SCATTER_ATOMIC, SCATTER_STAGED, LAYOUT_RECORD, LAYOUT_PAIR,
)

sketch_init = Context
