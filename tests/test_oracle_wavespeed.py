"""Pins of the oracle's variable wave speed: the coefficient 1/c^2 of the
time derivative in eq. (modelhyb), one value per free FEM cube (c = 1 near
and outside the FEM box, condition (coefic)), which weights the element mass
matrices and hence the lumped masses of Sec. 7.2.

- 1/c^2 = 1 gives the plain scheme bitwise;
- the hybrid sweep equals the independent merged whole-grid formulation
  (tests/assembled_ref.py) whose lumped masses take the 1/c^2-weighted Kuhn
  mass shares computed by brute force from the tetrahedra;
- the discrete energy with those masses is conserved with reflecting walls;
- the exact discrete derivative dJ/d(1/c^2) matches central differences,
  alone and together with Model Problem 1 data.
"""
import numpy as np

from tests.assembled_ref import Merged, kuhn_cube_lumped_share

ABC, NEUMANN, SOURCE = 0, 1, 2


def _free(C, rng, lo, hi):
    s = np.zeros((C, C, C))
    s[2:C - 2, 2:C - 2, 2:C - 2] = rng.uniform(lo, hi, (C - 4,) * 3)
    return s.ravel()


def _eps(C, rng, lo=0.25, hi=1.0):
    e = np.ones((C, C, C))
    e[2:C - 2, 2:C - 2, 2:C - 2] = rng.uniform(lo, hi, (C - 4,) * 3)
    return e.ravel()


def test_kuhn_lumped_shares():
    """The diagonal ends of the cube lie in all 6 tetrahedra (share 1/4),
    the other corners in 2 (share 1/12)."""
    sh = kuhn_cube_lumped_share()
    assert abs(sh.sum() - 1.0) < 1e-15
    assert np.allclose(sh[[0, 7]], 0.25, atol=1e-15)
    assert np.allclose(sh[1:7], 1.0 / 12.0, atol=1e-15)


def test_unit_coefficient_is_plain_scheme(orc):
    rng = np.random.default_rng(20)
    n, o, C = 16, 4, 8
    h = 1.0 / n
    dt, nt, om = 0.25 * h, 80, 30.0
    sig = _free(C, rng, 0, 3)
    g = orc.Geometry(n, fem_o=o, fem_c=C)
    a = orc.forward(g, sig, nt, dt, omega=om)
    b = orc.forward(g, sig, nt, dt, omega=om, eps=np.ones(C ** 3))
    assert np.array_equal(a, b)
    r = rng.standard_normal(a.shape)
    da = orc.adjoint(g, sig, nt, dt, r, omega=om)
    db, de = orc.adjoint(g, sig, nt, dt, r, omega=om, eps=np.ones(C ** 3), want_deps=True)
    assert np.array_equal(da, db)
    assert np.any(de != 0)


def test_hybrid_equals_merged_reference_with_wave_speed(orc):
    rng = np.random.default_rng(21)
    n, o, C = 16, 4, 8
    h = 1.0 / n
    bc = (NEUMANN, ABC, ABC, NEUMANN, ABC, SOURCE)
    sig = _free(C, rng, 0, 3)
    eps = _eps(C, rng)
    dt, nt, om = 0.2 * h, 90, 30.0
    g = orc.Geometry(n, bc=bc, fem_o=o, fem_c=C)
    a = orc.forward(g, sig, nt, dt, omega=om, eps=eps)
    M = Merged((n,) * 3, h, bc, (o,) * 3, (C,) * 3, sig, eps=eps)
    t1 = 2 * np.pi / om
    k_on = max(k + 1 for k in range(nt) if k * dt < t1)
    b = M.run(nt, dt, lambda k: np.sin(om * k * dt), k_on)
    assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(b)
    # and differs from the constant wave speed
    c = orc.forward(g, sig, nt, dt, omega=om)
    assert np.linalg.norm(a - c) > 1e-4 * np.linalg.norm(c)


def test_energy_conserved_with_wave_speed(orc):
    rng = np.random.default_rng(22)
    n, o, C = 16, 4, 8
    h = 1.0 / n
    dt = 0.2 * h
    sig = _free(C, rng, 0, 3)
    eps = _eps(C, rng)
    g = orc.Geometry(n, bc=(NEUMANN,) * 6, fem_o=o, fem_c=C)
    x = np.arange(n + 1) * h - 0.5
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    u0 = np.exp(-(X ** 2 + Y ** 2 + Z ** 2) / 0.02)
    M = Merged((n,) * 3, h, (NEUMANN,) * 6, (o,) * 3, (C,) * 3, sig, eps=eps)

    def merged(nt):
        _, vh, uf = orc.forward(g, sig, nt, dt, u0=u0, um1=u0, want_vhist=True, want_ufinal=True, eps=eps)
        u = uf.reshape((n + 1,) * 3).copy()
        v = vh[nt].reshape((C + 1,) * 3)
        u[o + 1:o + C, o + 1:o + C, o + 1:o + C] = v[1:-1, 1:-1, 1:-1]
        return u

    E = [M.energy(merged(k + 1), merged(k), dt) for k in (0, 41, 160)]
    assert E[0] > 0
    assert max(abs(e - E[0]) for e in E) <= 1e-12 * E[0]
    # the energy with the unit masses is not conserved
    M1 = Merged((n,) * 3, h, (NEUMANN,) * 6, (o,) * 3, (C,) * 3, sig)
    E1 = [M1.energy(merged(k + 1), merged(k), dt) for k in (0, 160)]
    assert abs(E1[1] - E1[0]) > 1e-8 * E1[0]


def _fd_check(orc, taylor):
    rng = np.random.default_rng(23 + taylor)
    n, o, C = 12, 3, 6
    h = 1.0 / n
    bc = (ABC, NEUMANN, ABC, ABC, ABC, SOURCE)
    sig = _free(C, rng, 0.5, 2.5)
    eps = _eps(C, rng, 0.4, 1.0)
    # long enough for the waves scattered in the free cubes to reach the trace
    dt, nt, om = 0.15 * h, 110, 30.0
    g = orc.Geometry(n, bc=bc, fem_o=o, fem_c=C)
    kw = dict(omega=om)
    if taylor:
        z, y, x = np.meshgrid(*(np.arange(n + 1) * h,) * 3, indexing="ij")
        kw.update(taylor=True, f0=np.exp(-(x ** 2 + y ** 2 + z ** 2)).ravel(),
                  f1=(np.sin(2 * x) * np.cos(3 * y) * z).ravel())
    r = rng.standard_normal((nt + 1, (n + 1) ** 2))
    dsig, deps = orc.adjoint(g, sig, nt, dt, r, eps=eps, want_deps=True, **kw)
    free = np.flatnonzero(eps != 1.0)
    step = 1e-4
    fd = []
    for c in free:
        ep, em = eps.copy(), eps.copy()
        ep[c] += step
        em[c] -= step
        Lp = np.sum(r * orc.forward(g, sig, nt, dt, eps=ep, **kw).reshape(r.shape))
        Lm = np.sum(r * orc.forward(g, sig, nt, dt, eps=em, **kw).reshape(r.shape))
        fd.append((Lp - Lm) / (2 * step))
    fd = np.array(fd)
    assert np.linalg.norm(deps[free] - fd) <= 1e-7 * np.linalg.norm(fd)
    assert np.all(deps[eps == 1.0] == 0)
    # the conductivity gradient with the wave speed also matches
    c = int(np.flatnonzero(sig)[0])
    sp, sm = sig.copy(), sig.copy()
    sp[c] += step
    sm[c] -= step
    Lp = np.sum(r * orc.forward(g, sp, nt, dt, eps=eps, **kw).reshape(r.shape))
    Lm = np.sum(r * orc.forward(g, sm, nt, dt, eps=eps, **kw).reshape(r.shape))
    assert abs(dsig[c] - (Lp - Lm) / (2 * step)) <= 1e-6 * abs(dsig[c])


def test_wave_speed_gradient_central_differences(orc):
    _fd_check(orc, False)


def test_wave_speed_gradient_with_model_problem_1(orc):
    _fd_check(orc, True)


def test_l2_gradient_density(orc):
    """orc.gradient's geps is (1/h^3) dJ_misfit/d(1/c^2) on free cubes."""
    rng = np.random.default_rng(25)
    n, o, C = 12, 3, 6
    h = 1.0 / n
    sig = _free(C, rng, 0.5, 2.5)
    eps = _eps(C, rng, 0.4, 1.0)
    dt, nt = 0.15 * h, 40
    g = orc.Geometry(n, fem_o=o, fem_c=C)
    data = orc.forward(g, 0.5 * sig, nt, dt, omega=30.0)
    _, _, geps, obs = orc.gradient(g, sig, nt, dt, data, omega=30.0, eps=eps, want_geps=True, want_obs=True)
    _, seed = orc.misfit(g, nt, dt, obs, data)
    _, deps = orc.adjoint(g, sig, nt, dt, seed, omega=30.0, eps=eps, want_deps=True)
    assert np.allclose(geps, deps / h ** 3, rtol=1e-13, atol=0)
