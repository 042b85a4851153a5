"""Host-side checks of the C ABI library (no GPU): it loads, exports every
function include/cfd.h declares, and the binding covers all of them."""
import ctypes
import os
import re

import pytest

from paper_2203_13760_amd import cfd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "cfd.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cfd_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_abi():
    names = _declared()
    for required in ("cfd_state_init", "cfd_rhs", "cfd_rk3_step", "cfd_advance", "cfd_rhs_adjoint"):
        assert required in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(cfd.LIB_PATH):
        pytest.skip("libcfd.so not built")
    lib = ctypes.CDLL(cfd.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(_declared()) == set(cfd.EXPORTS)


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(cfd, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(cfd, "_lib", None)
    with pytest.raises(RuntimeError):
        cfd.load()
