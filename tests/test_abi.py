"""The C-ABI library builds for gfx950, loads, and exports every entry point
that include/ep.h declares (no compute calls: this runs without a GPU)."""
import os
import re

import pytest

from paper_1805_04155_amd import _ep

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "ep.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ep_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_ep.LIB_PATH):
        from paper_1805_04155_amd import build
        build.build()
    return _ep.lib()


def test_every_declared_symbol_is_exported(lib):
    syms = declared_symbols()
    assert len(syms) >= 20
    for s in syms:
        assert hasattr(lib, s), s
    assert sorted(_ep.EXPORTED) == syms


def test_struct_layouts_match_header():
    """ctypes structures mirror the header field by field."""
    text = open(os.path.join(ROOT, "include", "ep.h")).read()
    for st in ("ep_mesh", "ep_material", "ep_options", "ep_sizes", "ep_newton_info",
               "ep_quadrature", "ep_warm_info"):
        m = re.search(r"typedef struct \{([^{}]*)\}\s*" + st + ";", text)
        assert m, st
        body = re.sub(r"/\*.*?\*/", "", m.group(1), flags=re.S)
        names = []
        for decl in body.split(";"):
            decl = decl.strip()
            if not decl:
                continue
            parts = decl.replace("*", " ").split()
            rest = " ".join(parts[1:]) if parts[0] != "const" else " ".join(parts[2:])
            names += [n.strip() for n in rest.split(",")]
        fields = [f for f, _ in getattr(_ep, st)._fields_]
        assert fields == names, (st, fields, names)


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(_ep, "LIB_PATH", str(tmp_path / "libep.so"))
    monkeypatch.setattr(_ep, "_lib", None)
    with pytest.raises(ImportError):
        _ep.lib()


def test_mlp_constants_match_header():
    text = open(os.path.join(ROOT, "include", "ep.h")).read()
    for name, val in (("IN", _ep.MLP_IN), ("HID", _ep.MLP_HID), ("OUT", _ep.MLP_OUT),
                      ("XS", _ep.MLP_XS), ("YS", _ep.MLP_YS), ("NPARAM", _ep.MLP_NPARAM)):
        m = re.search(r"#define EP_MLP_" + name + r"\s+(\d+)", text)
        assert m and int(m.group(1)) == val, name
    assert _ep.MLP_NPARAM == (_ep.MLP_IN * _ep.MLP_HID + _ep.MLP_HID + _ep.MLP_HID ** 2
                              + _ep.MLP_HID + _ep.MLP_OUT * _ep.MLP_HID + _ep.MLP_OUT)
