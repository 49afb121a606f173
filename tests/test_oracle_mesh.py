"""Pins of the oracle's explicit-mesh mode (a general tetrahedral mesh of the
FEM box, one conductivity per tetrahedron; P1 elements of Sec. 7.2 with
lumped masses, Algorithm 2 unchanged).

- The 6-tetrahedra split passed as an explicit mesh reproduces the built-in
  lattice mode (trace, per-cube gradient as the sum over its tetrahedra, J).
- Renumbering the nodes and reordering the tetrahedra changes nothing.
- On a perturbed (unstructured) mesh: the adjoint passes a dot test, the
  gradient matches central differences, and the trace moves linearly with
  the size of the perturbation.
- Meshes that do not meet the grid on the overlap are rejected.
"""
import numpy as np
import pytest

from paper_1509_01399_amd import synth

N, C, O = 16, 8, 4
H = 1.0 / N


def rel(a, b):
    a, b = np.asarray(a, float).ravel(), np.asarray(b, float).ravel()
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _geom(orc, mesh=None, bc=(0, 0, 0, 0, 0, 2)):
    return orc.Geometry(N, bc=bc, fem_o=O, fem_c=C, mesh=mesh)


def _sigma_cube(seed):
    rng = np.random.default_rng(seed)
    s = np.zeros((C, C, C))
    s[2:C - 2, 2:C - 2, 2:C - 2] = rng.uniform(0, 3, (C - 4,) * 3)
    return s


def _volumes(xyz, tet):
    X = xyz[tet]
    E = X[:, 1:] - X[:, :1]
    return np.abs(np.linalg.det(E)) / 6.0


def test_explicit_kuhn_mesh_equals_lattice(orc):
    sc = _sigma_cube(1)
    xyz, tet = synth.kuhn_box_mesh(O, C, H)
    st = np.repeat(sc.ravel(), 6)  # the mesh is cube-major, 6 tetrahedra per cube
    gl, gm = _geom(orc), _geom(orc, (xyz, tet))
    assert gm.sizes()["fem_cubes"] == 6 * gl.sizes()["fem_cubes"]
    assert gm.sizes()["fem_updated"] == gl.sizes()["fem_updated"]
    nt, dt = 60, 0.25 * H
    a = orc.forward(gl, sc.ravel(), nt, dt, omega=30.0)
    b = orc.forward(gm, st, nt, dt, omega=30.0)
    assert np.abs(a).max() > 1e-3
    assert rel(b, a) <= 1e-13
    rng = np.random.default_rng(2)
    seed = rng.standard_normal(a.shape)
    da = orc.adjoint(gl, sc.ravel(), nt, dt, seed, omega=30.0)
    db = orc.adjoint(gm, st, nt, dt, seed, omega=30.0)
    assert rel(db.reshape(-1, 6).sum(1), da) <= 1e-12
    data = a + 0.01 * rng.standard_normal(a.shape)
    ga, Ja = orc.gradient(gl, sc.ravel(), nt, dt, data, omega=30.0)
    gb, Jb = orc.gradient(gm, st, nt, dt, data, omega=30.0)
    # L2 densities: the cube value is the mean over its 6 equal-volume tetrahedra
    assert rel(gb.reshape(-1, 6).mean(1), ga) <= 1e-12
    assert abs(Jb - Ja) <= 1e-13 * abs(Ja)


def test_renumbering_invariance(orc):
    xyz, tet = synth.perturbed_box_mesh(O, C, H, seed=3)
    st = synth.tet_sigma(xyz, tet, _sigma_cube(4), O, C, H)
    rng = np.random.default_rng(5)
    pn = rng.permutation(len(xyz))        # new id of old node i: inv[i]
    inv = np.empty_like(pn)
    inv[pn] = np.arange(len(pn))
    pt = rng.permutation(len(tet))
    xyz2, tet2, st2 = xyz[pn], inv[tet][pt].astype(np.int32), st[pt]
    nt, dt = 50, 0.25 * H
    a = orc.forward(_geom(orc, (xyz, tet)), st, nt, dt, omega=30.0)
    b = orc.forward(_geom(orc, (xyz2, tet2)), st2, nt, dt, omega=30.0)
    assert rel(b, a) <= 1e-13
    seed = rng.standard_normal(a.shape)
    da = orc.adjoint(_geom(orc, (xyz, tet)), st, nt, dt, seed, omega=30.0)
    db = orc.adjoint(_geom(orc, (xyz2, tet2)), st2, nt, dt, seed, omega=30.0)
    assert rel(db, da[pt]) <= 1e-12


def test_perturbed_mesh_dot_test(orc):
    """<seed, T(flux)> = <T^T(seed), flux> for the linear map from the source
    flux table to the trace, on an unstructured mesh."""
    xyz, tet = synth.perturbed_box_mesh(O, C, H, seed=6)
    st = synth.tet_sigma(xyz, tet, _sigma_cube(7), O, C, H)
    g = _geom(orc, (xyz, tet))
    nt, dt = 40, 0.25 * H
    rng = np.random.default_rng(8)
    flux = rng.standard_normal((nt, N + 1, N + 1))
    tr = orc.forward(g, st, nt, dt, flux=flux, k_on=nt)
    seed = rng.standard_normal(tr.shape)
    _, dflux = orc.adjoint(g, st, nt, dt, seed, flux=flux, k_on=nt, want_dflux=True)
    lhs, rhs = float((seed * tr).sum()), float((dflux.ravel() * flux.ravel()).sum())
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_perturbed_mesh_gradient_central_differences(orc):
    xyz, tet = synth.perturbed_box_mesh(O, C, H, seed=9)
    st = synth.tet_sigma(xyz, tet, _sigma_cube(10), O, C, H)
    g = _geom(orc, (xyz, tet))
    nt, dt = 60, 0.25 * H
    data = orc.forward(g, 1.3 * st, nt, dt, omega=30.0)
    grad, J = orc.gradient(g, st, nt, dt, data, omega=30.0)
    vol = _volumes(xyz, tet)
    free = grad != 0
    assert free.sum() > 100
    rng = np.random.default_rng(11)
    for _ in range(3):
        v = rng.standard_normal(len(st)) * free
        v /= np.linalg.norm(v)
        eps = 1e-4
        _, Jp = orc.gradient(g, st + eps * v, nt, dt, data, omega=30.0)
        _, Jm = orc.gradient(g, st - eps * v, nt, dt, data, omega=30.0)
        fd = (Jp - Jm) / (2 * eps)
        an = float((vol * grad * v).sum())
        assert abs(fd - an) <= 1e-6 * abs(an)


def test_trace_linear_in_perturbation(orc):
    """Moving the inner nodes by amp*h changes the trace by O(amp): halving
    the perturbation halves the change."""
    sc = _sigma_cube(12)
    nt, dt = 60, 0.25 * H
    x0, t0 = synth.kuhn_box_mesh(O, C, H)
    base = orc.forward(_geom(orc, (x0, t0)), np.repeat(sc.ravel(), 6), nt, dt, omega=30.0)
    d = []
    for amp in (0.02, 0.01, 0.005):
        xyz, tet = synth.perturbed_box_mesh(O, C, H, seed=13, amp=amp)
        st = synth.tet_sigma(xyz, tet, sc, O, C, H)
        d.append(rel(orc.forward(_geom(orc, (xyz, tet)), st, nt, dt, omega=30.0), base))
    assert d[0] > 1e-8
    assert 1.8 < d[0] / d[1] < 2.2 and 1.8 < d[1] / d[2] < 2.2


def test_nonconforming_meshes_rejected(orc):
    xyz, tet = synth.kuhn_box_mesh(O, C, H)
    q = np.rint(xyz / H).astype(int) - O
    bad = xyz.copy()
    face = np.where((q[:, 0] == 0) & (q[:, 1] == C // 2) & (q[:, 2] == C // 2))[0][0]
    bad[face, 1] += 0.1 * H  # a box-surface node off the grid
    with pytest.raises(ValueError):
        orc.forward(_geom(orc, (bad, tet)), None, 5, 0.25 * H)
    bad = xyz.copy()
    inner = np.where((q[:, 0] == 2) & (q[:, 1] == C // 2) & (q[:, 2] == C // 2))[0][0]
    bad[inner, 1] += 0.1 * H  # an inner-box surface node off the grid
    with pytest.raises(ValueError):
        orc.forward(_geom(orc, (bad, tet)), None, 5, 0.25 * H)
