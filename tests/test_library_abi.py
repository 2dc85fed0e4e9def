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
    assert o.levels == 1 and list(o.ell_deep) == [0] * (nks.MAX_LEVELS - 1)


def test_struct_layouts_match_the_header(tmp_path):
    # the ctypes mirrors have the C sizes and field offsets (gcc on the header)
    import shutil
    import subprocess
    import paper_0912_4457_amd as nks
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    fields = {"nks_opts": nks.Opts, "nks_stats": nks.Stats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void) {"]
    for cname, cls in fields.items():
        lines.append(f'printf("%zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("%zu\\n", offsetof({cname}, {f}));')
    lines.append('printf("%d\\n", NKS_MAX_LEVELS); return 0; }')
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-o", str(exe), str(src)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    want = []
    for cls in fields.values():
        want.append(ctypes.sizeof(cls))
        want.extend(getattr(cls, f).offset for f, _ in cls._fields_)
    want.append(nks.MAX_LEVELS)
    assert got == want


def test_invalid_device_rejected_without_gpu():
    import paper_0912_4457_amd as nks
    h = ctypes.c_void_p()
    assert nks.lib().nks_create(-1, ctypes.byref(h)) != 0
