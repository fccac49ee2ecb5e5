"""Host-side checks of the C ABI (no GPU needed): the built library loads
and exports every function that include/schur.h declares."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "schur.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|double)\s+(schur_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_boundary():
    names = _declared()
    for f in ("schur_reduce", "schur_reduce_async", "schur_reduce_batched", "schur_create",
              "schur_destroy"):
        assert f in names


def test_library_exports_every_declared_symbol():
    from paper_1905_04975_amd import schur

    if not os.path.exists(schur.LIB_PATH):
        pytest.skip("library not built")
    import ctypes

    lib = ctypes.CDLL(schur.LIB_PATH)
    missing = [f for f in _declared() if not hasattr(lib, f)]
    assert missing == []
    assert set(schur.EXPORTS) == set(_declared())


def test_binding_refuses_missing_library(tmp_path, monkeypatch):
    from paper_1905_04975_amd import schur

    monkeypatch.setattr(schur, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(schur, "_lib", None)
    with pytest.raises(RuntimeError):
        schur.load()
