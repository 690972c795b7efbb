"""The oracle's pins catch plausible mistakes.

Each case plants one mistake in a copy of oracle.c (on the CPU only),
builds it, and runs the pin suite against it in a subprocess; the suite
must fail.  The unmodified copy must pass.
"""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

MUTANTS = {
    "depth_depends_on_endpoint": (
        "size_t iv = ((size_t)b * s->C + c) * s->D + d;",
        "size_t iv = ((size_t)b * s->C + c) * s->D + (d + 1) % s->D;"),
    "checksum_not_verified": ("if (h != g) continue;", ""),
    "decode_swapped": ("*out_u = (uint32_t)(a / V);\n            *out_v = (uint32_t)(a % V);",
                       "*out_u = (uint32_t)(a % V);\n            *out_v = (uint32_t)(a / V);"),
    "depth_scan_ascending": ("uint32_t d = D - 1 - k;", "uint32_t d = k;"),
    "depth_cap_off_by_one": ("return z < D - 1 ? z : D - 1;", "return z < D - 2 ? z : D - 2;"),
    "seed_increment_wrong": ("state += 0x9E3779B97F4A7C15ULL;", "state += 0x9E3779B97F4A7C17ULL;"),
    "gamma_missing_at_one_endpoint": ("s->alpha[iv] ^= x; s->gamma[iv] ^= h;",
                                      "s->alpha[iv] ^= x;"),
    "index_transposed": ("return (uint64_t)u * V + v;", "return (uint64_t)v * V + u;"),
    # the one-column sampler (level c of the hierarchy)
    "column_scan_ascending": (
        "for (int32_t d = (int32_t)D - 1; d >= 0; d--) { /* deepest first */",
        "for (int32_t d = 0; d < (int32_t)D; d++) {"),
    "column_checksum_dropped": (
        "if (hc != g || orc_depth_of_hash(hc, D) != (uint32_t)d) continue;",
        "if (orc_depth_of_hash(hc, D) != (uint32_t)d) continue;"),
    "column_seed_of_column_zero": ("const uint64_t seed_c = orc_seed(S, c);",
                                   "const uint64_t seed_c = orc_seed(S, 0);"),
    "column_failed_reported_empty": ("return nonzero ? ORC_FAILED : ORC_EMPTY;",
                                     "return ORC_EMPTY;"),
}


def _run_pins(lib_path):
    env = dict(os.environ, ORACLE_LIB=lib_path)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return r.returncode, r.stdout[-2000:]


def _build(src_text, d):
    c = os.path.join(d, "oracle.c")
    so = os.path.join(d, "liboracle.so")
    with open(c, "w") as f:
        f.write(src_text)
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-shared", "-fPIC", "-o", so, c])
    return so


def test_unmodified_copy_passes():
    with tempfile.TemporaryDirectory() as d:
        rc, out = _run_pins(_build(open(SRC).read(), d))
        assert rc == 0, out


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name):
    old, new = MUTANTS[name]
    text = open(SRC).read()
    assert old in text, f"mutation site of {name} not found"
    with tempfile.TemporaryDirectory() as d:
        rc, out = _run_pins(_build(text.replace(old, new), d))
        assert rc != 0, f"pins did not catch mutant {name}"
