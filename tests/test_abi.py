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


def _setup_error(mesh, free, mat, options=None):
    import ctypes as C
    with pytest.raises(_ep.EpError) as ei:
        _ep.ep_setup(mesh, free, mat, options, stream=C.c_void_p(0))
    return ei.value


@pytest.mark.parametrize("what", ["node_range", "repeated_node", "nu", "yield", "local_prec",
                                  "tangent_prec", "operator_form", "split_local_prec"])
def test_setup_rejects_invalid_input(lib, what):
    """Invalid meshes, materials and options are refused at setup with
    EP_EINVAL and a message, before any device work (runs without a GPU)."""
    import numpy as np
    from paper_1805_04155_amd import workloads as W
    mesh = W.mesh_q1_3d(2, 2, 2, 1.0, 1.0, 1.0)
    free = np.ones(mesh.n_dof, np.uint8)
    mat = W.VM_MATERIAL
    opts = None
    if what == "node_range":
        elem = mesh.elem.copy()
        elem[3, 2] = mesh.n_nodes
        mesh = W.Mesh(mesh.etype, mesh.coord, elem)
    elif what == "repeated_node":
        elem = mesh.elem.copy()
        elem[5, 1] = elem[5, 6]
        mesh = W.Mesh(mesh.etype, mesh.coord, elem)
    elif what == "nu":
        mat = W.Material("VM", E=1000.0, nu=0.5, Y=1.0, a=0.0)
    elif what == "yield":
        mat = W.Material("DP", E=1000.0, nu=0.3, eta=0.0, c=1.0)
    elif what == "local_prec":
        opts = {"local_prec": _ep.EP_BF16}   # matrix-core products: Q2-27 / P2 only
    elif what == "operator_form":
        opts = {"operator_form": 5}
    elif what == "split_local_prec":
        mesh = W.mesh_q2_3d(2, 2, 2, 1.0, 1.0, 1.0)
        free = np.ones(mesh.n_dof, np.uint8)
        opts = {"operator_form": _ep.EP_OPERATOR_SPLIT, "local_prec": _ep.EP_BF16}
    else:
        opts = {"tangent_prec": _ep.EP_BF16}
    err = _setup_error(mesh, free, mat, opts)
    assert err.status == _ep.EP_EINVAL
    assert str(err)


@pytest.mark.parametrize("what", ["nodes", "position_map"])
def test_setup_rejects_meshes_beyond_32bit_indices(lib, what):
    """Meshes whose node dofs or element position map exceed 32-bit indices
    are refused with EP_EINVAL before any array is read (the arrays passed
    here are one element long)."""
    import ctypes as C
    import numpy as np
    from paper_1805_04155_amd import workloads as W
    coord = np.zeros(3)
    elem = np.zeros(8, np.int32)
    free = np.ones(3, np.uint8)
    n_nodes, n_elems = (2 ** 30, 1) if what == "nodes" else (8, 2 ** 25)
    m = _ep.ep_mesh(3, _ep.EP_Q1, n_nodes, n_elems, coord.ctypes.data, elem.ctypes.data,
                    free.ctypes.data)
    mat = _ep._material(W.VM_MATERIAL)
    h = C.c_void_p()
    st = lib.ep_setup(C.byref(m), None, C.byref(mat), None, C.c_void_p(0), C.byref(h))
    assert st == _ep.EP_EINVAL and not h.value
    assert b"32-bit" in _ep.lib().ep_last_error(None)
