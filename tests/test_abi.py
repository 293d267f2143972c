"""The C-ABI library loads and exports every entry point include/quadamg.h declares (no GPU needed)."""
import ctypes as C
import os
import re

import pytest

from paper_1209_5421_amd import amg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "quadamg.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(amg.LIB_PATH):
        from paper_1209_5421_amd import build
        build.build()
    return amg.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(amg_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("amg_setup", "amg_solve", "amg_free", "amg_solve_batch", "amg_estimate_bytes",
                     "amg_num_levels", "amg_export_level", "amg_status_string"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(amg.EXPORTED) == names


def test_host_only_entry_points(lib):
    o = amg.default_options()
    assert (o.precision, o.coarse_max, o.inner_iters, o.sweeps, o.outer_mmax, o.max_iters, o.engine, o.batch,
            o.smoother) == (0, 64, 2, 1, 1, 1000, 1, 1, 0)
    assert not o.alloc and not o.dealloc and not o.ctx
    # the options struct of the binding has the size of the C one (alloc / dealloc / ctx at its end)
    assert C.sizeof(amg.Options) == 4 * 9 + 4 + 8 * 5
    assert lib.amg_status_string(0) == b"AMG_OK"
    assert lib.amg_status_string(4) == b"AMG_ERR_NOT_SPD"
    small = amg.estimate_bytes(3969, 27281)
    big = amg.estimate_bytes(1_044_484, 7_300_000)
    assert 0 < small < big
    assert big < 2 * 1024 ** 3
    # the exact-block smoother's factors (at most 16.5 values of 12 bytes per unknown) raise the bound
    blk = amg.estimate_bytes(1_044_484, 7_300_000, smoother=1)
    assert big < blk <= big + 1_044_484 * 33 * 6 + 4 ** 9 * 16 + (64 << 20)
    # invalid arguments are rejected before any device work
    h = C.c_void_p()
    assert lib.amg_setup(0, None, None, None, None, 0, None, C.byref(h)) == amg.INVALID
    assert lib.amg_solve(None, None, None, 1e-8, None) == amg.INVALID
    lib.amg_free(None)
    # values update and device assembly: rejected without a handle or buffers, before any device work
    assert lib.amg_update_values(None, None, None, None, 0) == amg.INVALID
    m = C.c_void_p()
    assert lib.amg_p1_mesh_create(0, None, 0, None, None, 0, None, C.byref(m)) == amg.INVALID and not m.value
    assert lib.amg_p1_mesh_create(10, None, 4, None, None, 11, None, C.byref(m)) == amg.INVALID  # ndof > nv
    n = C.c_int64()
    assert lib.amg_p1_mesh_pattern(None, C.byref(n), None, None) == amg.INVALID
    assert lib.amg_p1_assemble(None, None, None) == amg.INVALID
    lib.amg_p1_mesh_free(None)


def test_product_path_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_1209_5421_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle\b|liboracle|\borc_[a-z]|oracle\.h", src, re.M), f
