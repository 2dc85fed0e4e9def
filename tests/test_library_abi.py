"""The C-ABI library loads and exports every function that include/nks.h
declares; the Python binding declares exactly those names.  No compute
calls (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nks.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nks_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("nks_create", "nks_lattice_create", "nks_lattice_set_params", "nks_apply_op",
                     "nks_sign_apply", "nks_sign_apply_batch", "nks_workspace_size", "nks_outer_basis",
                     "nks_nested_step", "nks_last_error", "nks_status_str"):
        assert required in names


def test_library_exports_every_declared_symbol():
    import paper_0912_4457_amd as nks
    if not os.path.exists(nks.LIB_PATH):
        from paper_0912_4457_amd import build
        build.build()
    lib = ctypes.CDLL(nks.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), f"{name} declared in nks.h but not exported"
    assert set(nks.SIGNATURES) == set(declared_functions())


def test_status_strings_and_defaults_without_gpu():
    import paper_0912_4457_amd as nks
    lib = nks.lib()
    assert lib.nks_status_str(0) == b"ok"
    assert lib.nks_status_str(5).startswith(b"serious")
    o = nks.Opts()
    lib.nks_opts_default(ctypes.byref(o))
    assert o.size == ctypes.sizeof(nks.Opts)
    assert (o.k, o.ell, o.precision, o.max_rhi_iter) == (200, 50, 0, 50)
    assert o.rhi_tol == pytest.approx(1e-14)


def test_invalid_device_rejected_without_gpu():
    import paper_0912_4457_amd as nks
    h = ctypes.c_void_p()
    assert nks.lib().nks_create(-1, ctypes.byref(h)) != 0
