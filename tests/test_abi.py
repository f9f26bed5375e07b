"""CPU checks of the C-ABI library: it loads, exports what include/dpcg.h declares,
and the Python binding has no silent fallback.  No kernel is launched here."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dpcg.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*[A-Za-z_][\w\s\*]*?\b(dpcg_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("dpcg_setup", "dpcg_solve", "dpcg_solve_adjoint", "dpcg_destroy", "dpcg_status_string"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2111_09294_amd import _binding as B
    L = B.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
        assert name in B.SIGNATURES, f"binding lacks a signature for {name}"


def test_status_strings():
    from paper_2111_09294_amd import status_string
    assert status_string(0) == "converged"
    for code in (1, -1, -2, -3, -4, -5, -6, -7, -8):
        s = status_string(code)
        assert s and s != "unknown status"
    assert status_string(42) == "unknown status"


def test_missing_library_raises(monkeypatch, tmp_path):
    from paper_2111_09294_amd import _binding as B
    monkeypatch.setattr(B, "_lib", None)
    monkeypatch.setattr(B, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(RuntimeError, match="no fallback"):
        B.lib()


def test_binding_has_no_oracle_import():
    """The product package never reaches the CPU oracle."""
    pkg = os.path.join(ROOT, "paper_2111_09294_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in src.lower(), f


def test_setup_host_contract_checks_arguments_on_the_host():
    """dpcg_setup takes device arrays, dpcg_setup_host host arrays (both documented in
    include/dpcg.h); the host variant reads k_rowptr[n] and z_rowptr[n] on the host and
    rejects malformed row pointers before any device work."""
    import ctypes as C

    import numpy as np

    from paper_2111_09294_amd import _binding as B
    text = open(HEADER).read()
    assert "dpcg_setup_host" in text and "HOST memory" in text
    assert "device arrays here (dpcg_setup_host takes host arrays)" in text
    L = B.lib()
    h = C.c_void_p()
    info = B.Info()
    kp = np.array([1, 2, 3, 4], np.int64)            # does not start at 0
    kc = np.zeros(4, np.int32)
    kv = np.ones(4)
    bp = np.array([0, 3], np.int32)
    ptr = lambda a: a.ctypes.data_as(C.c_void_p)  # noqa: E731
    st = L.dpcg_setup_host(C.byref(h), 3, ptr(kp), ptr(kc), ptr(kv), 0, None, None, None, 1, ptr(bp), None,
                           C.byref(info))
    assert st == B.EINVAL and not h.value and info.status == B.EINVAL
    st = L.dpcg_setup_host(C.byref(h), 0, ptr(kp), ptr(kc), ptr(kv), 0, None, None, None, 1, ptr(bp), None, None)
    assert st == B.EINVAL
    kp0 = np.array([0, 1, 2, 3], np.int64)
    st = L.dpcg_setup_host(C.byref(h), 3, ptr(kp0), ptr(kc), ptr(kv), 2, None, None, None, 1, ptr(bp), None, None)
    assert st == B.EINVAL                             # k > 0 without Z
