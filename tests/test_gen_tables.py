"""Host logic of the general-mesh path, on the CPU: the tables that the
library's mesh analysis builds for a general tetrahedral FEM box (node
ranges, sliced ELL adjacency, edge contribution lists, lumped masses, the
gradient contraction tables) against an independent numpy assembly of the P1
stiffness and lumped mass matrices (Sec. 7.2), and the conformity checks of
the overlap (Sec. 3).  The analysis source is compiled with g++ into a small
shim; no GPU is involved."""
import ctypes as ct
import os
import subprocess

import numpy as np
import pytest
import scipy.sparse as sp

from paper_1509_01399_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
N, C, O = 16, 8, 4
H = 1.0 / N


class Grid(ct.Structure):
    _fields_ = [("n_cells", ct.c_int32 * 3), ("h", ct.c_double), ("origin", ct.c_double * 3),
                ("face", ct.c_int32 * 6)]


class Mesh(ct.Structure):
    _fields_ = [("n_nodes", ct.c_int64), ("xyz", ct.POINTER(ct.c_double)), ("n_tets", ct.c_int64),
                ("tet4", ct.POINTER(ct.c_int32))]


@pytest.fixture(scope="module")
def shim(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("shim") / "gen_shim.so")
    subprocess.run(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", "-D__HIP_PLATFORM_AMD__",
                    "-I/opt/rocm/include", os.path.join(ROOT, "tests", "gen_tables_shim.cpp"),
                    os.path.join(ROOT, "paper_1509_01399_amd", "csrc", "hyb_gen_mesh.cpp"), "-o", out],
                   check=True)
    lib = ct.CDLL(out)
    lib.gen_error.restype = ct.c_char_p
    return lib


def analyse(lib, xyz, tet):
    g = Grid()
    g.n_cells[:] = (N, N, N)
    g.h = H
    xyz = np.ascontiguousarray(xyz, np.float64)
    tet = np.ascontiguousarray(tet, np.int32)
    m = Mesh(len(xyz), xyz.ctypes.data_as(ct.POINTER(ct.c_double)), len(tet),
             tet.ctypes.data_as(ct.POINTER(ct.c_int32)))
    o = (ct.c_int * 3)(O, O, O)
    c = (ct.c_int * 3)(C, C, C)
    sz = (ct.c_longlong * 12)()
    st = lib.gen_analyse(ct.byref(g), ct.byref(m), o, c, sz)
    if st:
        return st, lib.gen_error().decode()
    keys = ("fn", "nA", "nH", "nR", "ntet", "nslice", "nslice_h", "nnz", "nE", "nedge", "ncontrib", "all_grid")
    s = dict(zip(keys, list(sz)))
    shapes = {"orig_of_dev": (s["fn"], np.int32), "grid_lin": (s["fn"], np.int64), "gq": (3 * s["fn"], np.int32),
              "soff": (s["nslice"] + 1, np.int32), "eoff": (s["nslice_h"] + 1, np.int32),
              "col": (s["nnz"], np.int32), "eid": (s["nnz"], np.int32), "cptr": (s["nedge"] + 1, np.int32),
              "ctet": (s["ncontrib"], np.int32), "cw": (s["ncontrib"], np.float64),
              "minv": (s["fn"], np.float64), "tetE": (6 * s["ntet"], np.int32),
              "ke6": (6 * s["ntet"], np.float64), "pvol": (s["ntet"], np.float64)}
    for k, (n, dt) in shapes.items():
        a = np.zeros(max(n, 1), dt)
        assert lib.gen_table(k.encode(), a.ctypes.data_as(ct.c_void_p)) == 0
        s[k] = a[:n]
    return 0, s


def p1(xyz, tet):
    """Element matrices and volumes of P1 tetrahedra."""
    X = xyz[tet]
    E = np.transpose(X[:, 1:] - X[:, :1], (0, 2, 1))
    inv = np.linalg.inv(E)
    G = np.concatenate([-inv.sum(1, keepdims=True), inv], 1)
    vol = np.abs(np.linalg.det(E)) / 6
    return vol[:, None, None] * G @ np.transpose(G, (0, 2, 1)), vol


MESHES = {
    "kuhn": lambda: synth.kuhn_box_mesh(O, C, H),
    "perturbed": lambda: synth.perturbed_box_mesh(O, C, H, seed=21, amp=0.15),
}


@pytest.mark.parametrize("kind", list(MESHES))
def test_tables_match_assembly(shim, kind):
    xyz, tet = MESHES[kind]()
    rng = np.random.default_rng(5)
    # shuffle the caller's numbering: the device numbering must not depend on it
    pn = rng.permutation(len(xyz))
    inv = np.empty_like(pn)
    inv[pn] = np.arange(len(pn))
    xyz, tet = xyz[pn], inv[tet].astype(np.int32)
    st, t = analyse(shim, xyz, tet)
    assert st == 0, t
    fn, nA, nH, nR = t["fn"], t["nA"], t["nH"], t["nR"]
    orig = t["orig_of_dev"]
    assert sorted(orig) == list(range(len(xyz)))
    dev = np.empty(fn, np.int64)
    dev[orig] = np.arange(fn)
    q = xyz[orig] / H - O
    qi = np.rint(q)
    grid = np.all(np.abs(q - qi) < 1e-7, axis=1)
    surf = np.any((np.abs(q) < 1e-7) | (np.abs(q - C) < 1e-7), axis=1)
    inner = np.all((q > 2 - 1e-7) & (q < C - 2 + 1e-7), axis=1)
    onD = grid & inner & np.any((np.abs(q - 2) < 1e-7) | (np.abs(q - (C - 2)) < 1e-7), axis=1)
    idx = np.arange(fn)
    assert np.array_equal(idx < nA, onD)
    assert np.array_equal(idx < nH, inner)
    assert np.array_equal(idx >= nR, surf)
    assert t["all_grid"] == (1 if grid.all() else 0)
    assert np.array_equal(t["grid_lin"] >= 0, grid)
    g3 = t["gq"].reshape(-1, 3)
    assert np.array_equal(g3[grid], (qi[grid] + O).astype(int))
    assert np.array_equal(t["grid_lin"][grid], g3[grid, 0] + (N + 1) * (g3[grid, 1] + (N + 1) * g3[grid, 2]))
    # assembled stiffness K(a) and lumped masses, device numbering
    ke, vol = p1(xyz, tet)
    td = dev[tet]
    free = np.all(td < nH, axis=1)
    a = np.ones(len(tet))
    a[free] += rng.uniform(0, 3, free.sum())
    r = np.repeat(td, 4, axis=1).ravel()
    c = np.tile(td, (1, 4)).ravel()
    Ka = sp.coo_matrix(((a[:, None, None] * ke).ravel(), (r, c)), shape=(fn, fn)).tocsr()
    mass = np.zeros(fn)
    np.add.at(mass, td.ravel(), np.repeat(vol / 4, 4))
    assert np.allclose(t["minv"][:nR], 1 / mass[:nR], rtol=1e-13) and np.all(t["minv"][nR:] == 0)
    # sliced ELL rows: neighbour sets, kappa(a) from the contribution lists, ordering
    soff, col, eid, cptr, ctet, cw = t["soff"], t["col"], t["eid"], t["cptr"], t["ctet"], t["cw"]
    kap = np.zeros(len(col))
    for p in np.nonzero(eid >= 0)[0]:
        e = eid[p]
        kap[p] = -(a[ctet[cptr[e]:cptr[e + 1]]] * cw[cptr[e]:cptr[e + 1]]).sum()
    scale = np.abs(Ka.data).max()
    # mesh edges (element connectivity; on the 6-tetrahedra split the diagonal
    # edges carry an exactly zero stiffness but are still neighbours)
    pattern = sp.coo_matrix((np.ones(len(r)), (r, c)), shape=(fn, fn)).tocsr().tolil()
    for n in range(fn):
        s_, l_ = n // 64, n % 64
        w = (soff[s_ + 1] - soff[s_]) // 64
        pos = soff[s_] + 64 * np.arange(w) + l_
        real = eid[pos] >= 0
        assert np.all(col[pos][~real] == n)
        cols = col[pos][real]
        nb = set(pattern.rows[n]) - {n}
        assert set(cols) == nb and len(cols) == len(nb)
        ref = -Ka[n, cols].toarray().ravel()
        assert np.abs(kap[pos][real] - ref).max() <= 1e-13 * scale
        if n < nH:  # the upper neighbours inside [0, nH) come first, ascending
            up = sorted(m for m in nb if n < m < nH)
            assert list(cols[:len(up)]) == up
    # gradient contraction tables of the free tetrahedra
    eoff, tetE, ke6, pvol = t["eoff"], t["tetE"], t["ke6"], t["pvol"]
    assert np.allclose(pvol[free], vol[free], rtol=1e-13) and np.all(pvol[~free] == 0)
    pairs = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
    for tt in np.nonzero(free)[0][::7]:
        for u, (qq, ww) in enumerate(pairs):
            va, vb = sorted((td[tt, qq], td[tt, ww]))
            pe = tetE[6 * tt + u]
            s_, l_ = va // 64, va % 64
            j = (pe - eoff[s_] - l_) // 64
            assert (pe - eoff[s_] - l_) % 64 == 0 and 0 <= j < (eoff[s_ + 1] - eoff[s_]) // 64
            assert col[soff[s_] + 64 * j + l_] == vb
            assert ke6[6 * tt + u] == pytest.approx(ke[tt, qq, ww], rel=1e-12, abs=1e-14 * H)
    assert t["nE"] == eoff[-1] and t["nnz"] == soff[-1]


def test_nonconforming_meshes_rejected(shim):
    xyz, tet = synth.kuhn_box_mesh(O, C, H)
    q = np.rint(xyz / H).astype(int) - O
    E_ARG, E_MESH = -1, -2

    def at(i, j, k):
        return int(np.nonzero((q[:, 0] == i) & (q[:, 1] == j) & (q[:, 2] == k))[0][0])

    bad = xyz.copy()
    bad[at(0, C // 2, C // 2), 1] += 0.1 * H  # box-surface node off the grid
    assert analyse(shim, bad, tet)[0] == E_MESH
    bad = xyz.copy()
    bad[at(2, C // 2, C // 2), 1] += 0.1 * H  # inner-box surface grid node missing
    assert analyse(shim, bad, tet)[0] == E_MESH
    bad = xyz.copy()
    bad[at(3, 3, 3)] = bad[at(3, 3, 4)]  # two nodes at one grid point
    assert analyse(shim, bad, tet)[0] == E_MESH
    t2 = tet.copy()
    t2[5, 1] = t2[5, 0]  # repeated vertex
    assert analyse(shim, xyz, t2)[0] == E_MESH
    t2 = tet.copy()
    t2[7, 2] = len(xyz)  # node id out of range
    assert analyse(shim, xyz, t2)[0] == E_ARG
    assert analyse(shim, xyz, np.delete(tet, 100, axis=0))[0] == E_MESH  # a hole
    assert analyse(shim, xyz, np.concatenate([tet, tet[100:101]]))[0] == E_MESH  # an overlap
    t2 = tet.copy()
    t2[100] = t2[101]  # one cube loses a tetrahedron, another is doubled: equal volume
    assert analyse(shim, xyz, t2)[0] == E_MESH
    # a perturbed mesh (nodes off the grid inside the inner box) is accepted
    xp, tp = synth.perturbed_box_mesh(O, C, H, seed=2)
    st, tab = analyse(shim, xp, tp)
    assert st == 0 and tab["all_grid"] == 0
