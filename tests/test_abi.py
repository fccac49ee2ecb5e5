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


def _struct_fields(name):
    """(C type, field name) pairs of `typedef struct name { ... }` in the
    header, arrays expanded as (type, name, count)."""
    src = open(os.path.join(ROOT, "include", "schur.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    body = re.search(r"typedef struct %s \{(.*?)\}" % name, src, flags=re.S).group(1)
    out = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        ctype, rest = decl.split(None, 1)
        for item in rest.split(","):
            item = item.strip()
            m = re.match(r"(\w+)\s*\[(\d+)\]$", item)
            out.append((ctype, m.group(1), int(m.group(2))) if m else (ctype, item, 1))
    return out


@pytest.mark.parametrize("cname,pyname", [("schur_opts", "SchurOpts"),
                                          ("schur_stats", "SchurStats"),
                                          ("schur_server_stats", "ServerStats")])
def test_binding_structs_match_the_header(cname, pyname):
    """The ctypes mirrors carry the header's fields in the header's order
    and types, so the library and the binding agree on every offset."""
    import ctypes

    from paper_1905_04975_amd import schur

    ctypes_of = {"int": ctypes.c_int, "int64_t": ctypes.c_int64, "double": ctypes.c_double}
    want = _struct_fields(cname)
    got = getattr(schur, pyname)._fields_
    assert [f[1] for f in want] == [g[0] for g in got]
    for (ctype, name, count), (gname, gtype) in zip(want, got):
        exp = ctypes_of[ctype] if count == 1 else ctypes_of[ctype] * count
        assert ctypes.sizeof(gtype) == ctypes.sizeof(exp) and (
            gtype is exp or getattr(gtype, "_type_", None) is getattr(exp, "_type_", None)), name
