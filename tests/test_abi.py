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
    for code in (1, -1, -2, -3, -4, -5, -6, -7):
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
