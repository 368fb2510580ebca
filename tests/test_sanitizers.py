"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU):
the library's mesh graph (pattern, position maps, colouring;
csrc/ep_mesh_graph.cpp) and every entry point of the C oracle, each built
with -fsanitize=address,undefined into a small driver (tests/native/) and
run on the small cases of every element kind.  A sanitizer report fails the
run; the outputs are checked against the oracle (mesh graph) and against
the regular oracle build (oracle), bit for bit."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import oracle as O
from tests.gpu_cases import CASES, make_case

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NATIVE = os.path.join(ROOT, "tests", "native")
CSRC = os.path.join(ROOT, "paper_1805_04155_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


@pytest.fixture(scope="module")
def exes(tmp_path_factory):
    if shutil.which("g++") is None or shutil.which("gcc") is None:
        pytest.skip("no host compiler")
    d = tmp_path_factory.mktemp("san")
    mg = str(d / "mesh_graph_check")
    oc = str(d / "oracle_check")
    subprocess.run(["g++", "-std=c++17", *SAN, "-I", CSRC,
                    os.path.join(CSRC, "ep_mesh_graph.cpp"),
                    os.path.join(NATIVE, "mesh_graph_check.cpp"), "-o", mg, "-pthread"],
                   check=True)
    subprocess.run(["gcc", "-std=c99", *SAN, "-ffp-contract=off",
                    os.path.join(ROOT, "oracle", "ep_oracle.c"),
                    os.path.join(NATIVE, "oracle_check.c"), "-o", oc, "-lm"], check=True)
    return d, mg, oc


def _run(exe, inp, out):
    r = subprocess.run([exe, inp, out], capture_output=True, text=True, env=ENV, timeout=300)
    assert "Sanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-3000:]
    assert r.returncode == 0, r.stderr[-3000:]
    return r


class _Reader:
    def __init__(self, path):
        self.b = open(path, "rb").read()
        self.o = 0

    def take(self, dtype, n):
        a = np.frombuffer(self.b, dtype=dtype, count=n, offset=self.o)
        self.o += a.nbytes
        return a

    def arr32(self):
        n = int(self.take(np.int64, 1)[0])
        return self.take(np.int32, n)


def _mesh_graph(exes, mesh, sorted_cols, tag, elem=None):
    d, mg, _ = exes
    elem = mesh.elem if elem is None else elem
    inp, out = str(d / f"mg_{tag}.in"), str(d / f"mg_{tag}.out")
    with open(inp, "wb") as f:
        f.write(np.array([mesh.n_nodes, elem.shape[0]], np.int64).tobytes())
        f.write(np.array([mesh.n_p, mesh.dim, int(sorted_cols)], np.int32).tobytes())
        f.write(np.ascontiguousarray(elem, np.int32).tobytes())
    r = _run(mg, inp, out)
    return _Reader(out), r


@pytest.mark.parametrize("name", list(CASES))
def test_mesh_graph_under_sanitizers(exes, name):
    mesh = make_case(name)[0]
    rd, _ = _mesh_graph(exes, mesh, True, name)
    assert rd.take(np.int32, 1)[0] == 0
    nnzb, n_col = (int(v) for v in rd.take(np.int64, 2))
    bptr, bcol, bdiag, bpos, bposs, colour, n2e_ptr, fslot, slot_elem, perm = \
        (rd.arr32() for _ in range(10))
    d, n_p, n_n, n_e = mesh.dim, mesh.n_p, mesh.n_nodes, mesh.n_elems
    # scalar CSR and position map expanded from the node blocks equal the
    # oracle's independent sort-unique and binary search
    rp, ci = O.pattern(mesh)
    deg = np.diff(bptr)
    row_len = np.repeat(deg * d, d)
    assert np.array_equal(rp, np.concatenate([[0], np.cumsum(row_len)]))
    cols = []
    for m in range(n_n):
        blk = bcol[bptr[m]:bptr[m + 1]]
        cols.append((d * blk[:, None] + np.arange(d)).ravel())
    cols_row = [c for c in cols for _ in range(d)]
    assert np.array_equal(ci, np.concatenate(cols_row))
    assert np.array_equal(bcol[bdiag], np.arange(n_n))
    pos_o = O.position_map(mesh, rp, ci)
    bp = bpos.reshape(n_e, n_p, n_p)
    # block (p, p') of element e -> scalar entry (d p + i, d p' + j)
    node = mesh.elem
    for e in range(0, n_e, max(1, n_e // 50)):
        for p in range(n_p):
            m = node[e, p]
            for i in range(d):
                r = d * m + i
                k = bp[e, p] - bptr[m]
                want = rp[r] + (d * k[:, None] + np.arange(d)).ravel()
                assert np.array_equal(pos_o[e, d * p + i], want)
    # sorted columns: the same blocks, ascending node order per row
    bs = bposs.reshape(n_e, n_p, n_p)
    assert np.array_equal(np.sort(bs, axis=2), np.sort(bp, axis=2))
    assert np.all(np.diff(bcol[bs], axis=2) > 0)
    # colouring: elements of one colour share no node; colour-major order
    assert colour.min() == 0 and colour.max() == n_col - 1
    for c in range(n_col):
        nodes = node[colour == c].ravel()
        assert len(np.unique(nodes)) == len(nodes)
    listed = perm[perm >= 0]
    assert np.array_equal(np.sort(listed), np.arange(n_e))
    assert np.all(np.diff(colour[listed]) >= 0)
    # node -> slot map
    assert n2e_ptr[-1] == n_e * n_p
    assert np.array_equal(slot_elem[fslot], np.repeat(np.arange(n_e), n_p))
    assert nnzb == len(bcol)


@pytest.mark.parametrize("what", ["out_of_range", "repeated"])
def test_mesh_graph_refuses_bad_connectivity_under_sanitizers(exes, what):
    mesh = make_case("q1_3d_vm")[0]
    elem = mesh.elem.copy()
    if what == "out_of_range":
        elem[4, 3] = mesh.n_nodes
    else:
        elem[4, 3] = elem[4, 0]
    rd, r = _mesh_graph(exes, mesh, True, what, elem)
    assert rd.take(np.int32, 1)[0] == 1
    assert "refused" in r.stderr


@pytest.mark.parametrize("name", list(CASES))
def test_oracle_under_sanitizers(exes, name):
    d_, _, oc = exes
    mesh, free, mat, u, (ep, beta, kappa) = make_case(name)
    d, n_int = mesh.dim, mesh.n_int
    ep6, beta6 = O.state_to_ip6(ep, d), O.state_to_ip6(beta, d)
    rows = np.array([0, 1, mesh.n_dof // 2, mesh.n_dof - 1], np.int64)
    inp, out = str(d_ / f"or_{name}.in"), str(d_ / f"or_{name}.out")
    with open(inp, "wb") as f:
        f.write(np.array([O.ETYPE[mesh.etype], 1 if mat.model == "VM" else 2], np.int32).tobytes())
        f.write(np.array([mesh.n_nodes, mesh.n_elems, len(rows)], np.int64).tobytes())
        f.write(np.array([mat.shear, mat.bulk, mat.a, mat.Y, mat.eta, mat.c]).tobytes())
        for a in (mesh.coord, mesh.elem.astype(np.int32), u, free.astype(np.uint8), ep6, beta6,
                  kappa, rows):
            f.write(np.ascontiguousarray(a).tobytes())
    _run(oc, inp, out)
    rd = _Reader(out)
    n_p = mesh.n_p
    assert rd.take(np.int64, 1)[0] == 0
    dphi, w = O.geometry(mesh)
    assert np.array_equal(rd.take(np.float64, n_int * n_p * d), dphi.ravel())
    assert np.array_equal(rd.take(np.float64, n_int), w)
    eps = O.strain(mesh, dphi, u)
    assert np.array_equal(rd.take(np.float64, 6 * n_int), eps.ravel())
    ref = O.constitutive(mat, eps, ep6, beta6, kappa, crit=True)
    for key, dt, k in (("sig", np.float64, 6), ("D", np.float64, 36), ("flag", np.uint8, 1),
                       ("ep", np.float64, 6), ("beta", np.float64, 6), ("kappa", np.float64, 1),
                       ("crit", np.float64, 2)):
        assert np.array_equal(rd.take(dt, k * n_int), ref[key].ravel()), key
    F = O.internal_force(mesh, dphi, w, ref["sig"])
    assert np.array_equal(rd.take(np.float64, mesh.n_dof), F)
    rp, ci = O.pattern(mesh)
    assert rd.take(np.int64, 1)[0] == len(ci)
    assert np.array_equal(rd.take(np.int32, mesh.n_dof + 1), rp)
    assert np.array_equal(rd.take(np.int32, len(ci)), ci)
    nl = d * n_p
    assert np.array_equal(rd.take(np.int32, mesh.n_elems * nl * nl),
                          O.position_map(mesh, rp, ci).ravel())
    assert rd.take(np.int32, 1)[0] == 0
    _, _, K = O.assemble(mesh, dphi, w, ref["D"], rp, ci)
    assert np.array_equal(rd.take(np.float64, len(ci)), K)
    assert rd.take(np.int32, 1)[0] == 0
    mc = 3 * 125 * 2
    cnt = rd.take(np.int32, len(rows))
    cols = rd.take(np.int32, len(rows) * mc).reshape(len(rows), mc)
    vals = rd.take(np.float64, len(rows) * mc).reshape(len(rows), mc)
    for i, (oc_, ov) in enumerate(O.K_rows(mesh, dphi, w, ref["D"], rows, max_cols=mc)):
        assert np.array_equal(cols[i, :cnt[i]], oc_) and np.array_equal(vals[i, :cnt[i]], ov)
    x, it, rel = O.pcg(rp, ci, K, free, F, 1e-10, 100000)
    assert rd.take(np.int32, 1)[0] == it
    # (a tangent with apex points may be singular: NaN results must agree too)
    assert np.array_equal(rd.take(np.float64, 1), np.array([rel]), equal_nan=True)
    assert np.array_equal(rd.take(np.float64, mesh.n_dof), x, equal_nan=True)
