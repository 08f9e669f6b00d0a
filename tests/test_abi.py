"""The C-ABI library loads and exports every entry point include/stp.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names += re.findall(r"\b(stp_[a-z_]+)\s*\(", src)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    import paper_1802_08126_amd as stp
    lib = stp.load()
    names = declared_functions()
    assert "stp_create" in names and "stp_uzawa_solve" in names
    for name in names:
        assert hasattr(lib, name), name
        assert ctypes.cast(getattr(lib, name), ctypes.c_void_p).value


def test_host_only_entry_points():
    import paper_1802_08126_amd as stp
    from paper_1802_08126_amd import binding as b
    lib = stp.load()
    o = b.stp_options()
    lib.stp_default_options(ctypes.byref(o))
    assert o.precision == 0 and o.nu_A == 1 and o.tol == pytest.approx(1e-8) and o.omega == pytest.approx(0.8)
    assert lib.stp_status_string(-4) == b"not converged"
    # workspace grows with the problem and shrinks with the storage precision
    w64 = stp.stp_workspace_bytes(2, 255, 256, 2, precision="f64")
    w32 = stp.stp_workspace_bytes(2, 255, 256, 2, precision="f32")
    w16 = stp.stp_workspace_bytes(2, 255, 256, 2, precision="bf16")
    assert w64 > w32 > w16 > 2 * 256 * 255 * 255 * 2
    assert stp.stp_workspace_bytes(2, 10, 4, 1, spatial="mg") == 0       # multigrid needs 2^L - 1
    assert stp.stp_workspace_bytes(2, 10, 4, 1, spatial="none") > 0
    assert stp.stp_workspace_bytes(4, 7, 4, 1) == 0


def test_no_cpu_fallback_in_binding():
    """The binding marshals arguments only: it never imports the oracle."""
    import paper_1802_08126_amd.binding as b
    src = open(b.__file__).read()
    assert "oracle" not in src.replace("never imports the oracle", "")
