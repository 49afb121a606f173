"""Pins of the oracle's Model Problem 1 form (eq. (model1), Sec. 5): initial
data u(x,0) = f0, u_t(x,0) = f1 and the second-order Taylor start
u^1 = u^0 + tau f1 + (tau^2/2) A(u^0).

- exactness: a solution quadratic in t and x (u = (x-x0)^2/2 + t^2/2 +
  t (y-y0) + c z) is reproduced to rounding on every node the boundary rows
  cannot have reached yet; the plain leapfrog start from u^{-1} = f0 - tau f1
  is not (it misses the tau^2/2 term), so the test sees the weight 1/2;
- second-order convergence of a travelling pulse with non-zero initial
  velocity against its closed form (the plain start converges at first
  order);
- dot test of the adjoint with respect to (f0, f1) through the Taylor start;
- gradient with respect to the conductivity against central differences
  (the first step's weight 1/2 enters the gradient's k = 0 term);
- zero data reduce to Model Problem 2 (IP2 from IP1 with f0 = f1 = 0, Sec. 6).
"""
import numpy as np

ABC, NEUMANN, SOURCE = 0, 1, 2


def _grid_xyz(n, h):
    nx, ny, nz = (n, n, n) if np.isscalar(n) else n
    z, y, x = np.meshgrid(np.arange(nz + 1) * h, np.arange(ny + 1) * h, np.arange(nx + 1) * h, indexing="ij")
    return x, y, z


def _quadratic(x, y, z, t):
    return 0.5 * (x - 0.5) ** 2 + 0.5 * t * t + t * (y - 0.45) + 0.3 * z


def _fem_field(vh_level, C):
    return vh_level.reshape(C + 1, C + 1, C + 1)


def test_taylor_start_exact_for_quadratic_solution(orc):
    n, C, o = 24, 10, 7
    h = 1.0 / n
    dt, nt = 0.25 * h, 6
    g = orc.Geometry(n, bc=(ABC,) * 6, fem_o=o, fem_c=C)
    x, y, z = _grid_xyz(n, h)
    f0 = _quadratic(x, y, z, 0.0)
    f1 = (y - 0.45)
    exact = _quadratic(x, y, z, nt * dt)
    _, vh, uf = orc.forward(g, None, nt, dt, taylor=True, f0=f0, f1=f1, want_vhist=True, want_ufinal=True)
    uf = uf.reshape(n + 1, n + 1, n + 1)
    # nodes at index distance > nt from the outer boundary; the hole interior
    # (o+2, o+C-2)^3 belongs to no grid row, its values are in the FEM field
    lo, hi = nt + 1, n - nt - 1
    m = np.zeros_like(uf, bool)
    m[lo:hi + 1, lo:hi + 1, lo:hi + 1] = True
    m[o + 3:o + C - 2, o + 3:o + C - 2, o + 3:o + C - 2] = False
    scale = np.abs(exact).max()
    assert np.abs(uf - exact)[m].max() <= 1e-12 * scale
    # FEM rows (a = 1) in the same region
    V = _fem_field(vh[nt], C)
    ex_f = exact[o:o + C + 1, o:o + C + 1, o:o + C + 1]
    mf = m[o:o + C + 1, o:o + C + 1, o:o + C + 1].copy()
    mf[3:C - 2, 3:C - 2, 3:C - 2] = True
    assert np.abs(V - ex_f)[mf].max() <= 1e-12 * scale
    # the plain start u^{-1} = f0 - tau f1 misses tau^2/2 (error ~ tau^2 nt / 2)
    uf2 = orc.forward(g, None, nt, dt, u0=f0, um1=f0 - dt * f1, want_ufinal=True)[1].reshape(uf.shape)
    err2 = np.abs(uf2 - exact)[m].max()
    assert err2 >= 0.25 * dt * dt * nt


def _pulse_errors(orc, N, taylor):
    w, zc, T = 0.08, 0.6, 0.3
    n = (8, 8, N)
    h = 1.0 / N
    dt = 0.25 * h
    nt = int(round(T / dt))
    g = orc.Geometry(n, h=h, bc=(NEUMANN, NEUMANN, NEUMANN, NEUMANN, ABC, NEUMANN),
                     fem_o=(1, 1, N // 2 - 3), fem_c=(6, 6, 6))
    x, y, z = _grid_xyz(n, h)
    s = z - zc
    f0 = np.exp(-(s / w) ** 2)
    f1 = -2.0 * s / (w * w) * f0          # u = G(z - zc + t): u_t = G'
    sT = z - zc + nt * dt
    exact = np.exp(-(sT / w) ** 2)
    if taylor:
        uf = orc.forward(g, None, nt, dt, taylor=True, f0=f0, f1=f1, want_ufinal=True)[1]
    else:
        uf = orc.forward(g, None, nt, dt, u0=f0, um1=f0 - dt * f1, want_ufinal=True)[1]
    uf = uf.reshape(exact.shape)
    # exclude the hole interior of the FEM box (no grid row there)
    m = np.ones_like(uf, bool)
    oz = N // 2 - 3
    m[oz + 3, 4, 4] = False
    return np.abs(uf - exact)[m].max()


def test_taylor_start_second_order_travelling_pulse(orc):
    # at N = 40 the O(h^2) error of the scheme still hides the O(h) error of
    # the plain start, so the refinement runs over 80, 160, 320
    e = [_pulse_errors(orc, N, True) for N in (80, 160, 320)]
    orders = [np.log2(e[i] / e[i + 1]) for i in range(2)]
    assert min(orders) > 1.9, (e, orders)
    p = [_pulse_errors(orc, N, False) for N in (80, 160, 320)]
    porders = [np.log2(p[i] / p[i + 1]) for i in range(2)]
    assert max(porders) < 1.2, (p, porders)
    assert e[-1] < 0.5 * p[-1]


def _small_case(rng):
    n, C, o = 12, 6, 3
    h = 1.0 / n
    bc = (ABC, NEUMANN, ABC, ABC, NEUMANN, ABC)
    sig = np.zeros((C, C, C))
    sig[2:C - 2, 2:C - 2, 2:C - 2] = rng.uniform(0.5, 3.0, (C - 4,) * 3)
    return n, C, o, h, bc, sig.ravel()


def test_taylor_adjoint_dot_test(orc):
    rng = np.random.default_rng(11)
    n, C, o, h, bc, sig = _small_case(rng)
    g = orc.Geometry(n, bc=bc, fem_o=o, fem_c=C)
    dt, nt = 0.2 * h, 25
    nn = (n + 1) ** 3
    f0, f1 = rng.standard_normal(nn), rng.standard_normal(nn)
    r = rng.standard_normal((nt + 1, (n + 1) ** 2))
    obs = orc.forward(g, sig, nt, dt, taylor=True, f0=f0, f1=f1)
    _, df0, df1 = orc.adjoint(g, sig, nt, dt, r, taylor=True, f0=f0, f1=f1, want_ddata=True)
    lhs = np.sum(r * obs.reshape(r.shape))
    rhs = df0 @ f0 + df1 @ f1
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + np.abs(r).sum() * np.abs(obs).max())
    # df0 and df1 separately: perturb one at a time
    d0 = rng.standard_normal(nn)
    obs_a = orc.forward(g, sig, nt, dt, taylor=True, f0=d0, f1=None)
    assert abs(np.sum(r * obs_a.reshape(r.shape)) - df0 @ d0) <= 1e-11 * np.abs(df0 @ d0 + 1.0)
    obs_b = orc.forward(g, sig, nt, dt, taylor=True, f0=None, f1=d0)
    assert abs(np.sum(r * obs_b.reshape(r.shape)) - df1 @ d0) <= 1e-11 * np.abs(df1 @ d0 + 1.0)


def test_taylor_gradient_central_differences(orc):
    rng = np.random.default_rng(12)
    n, C, o, h, bc, sig = _small_case(rng)
    bc = (ABC, ABC, NEUMANN, ABC, ABC, SOURCE)
    g = orc.Geometry(n, bc=bc, fem_o=o, fem_c=C)
    dt, nt = 0.2 * h, 40
    x, y, z = _grid_xyz(n, h)
    f0 = np.exp(-((x - 0.5) ** 2 + (y - 0.5) ** 2 + (z - 0.5) ** 2) / 0.02).ravel()
    f1 = (np.sin(3 * x) * np.cos(2 * z)).ravel()
    r = rng.standard_normal((nt + 1, (n + 1) ** 2))
    dsig = orc.adjoint(g, sig, nt, dt, r, omega=30.0, taylor=True, f0=f0, f1=f1)
    el = np.flatnonzero(sig)
    eps = 1e-5
    fd = []
    for c in el:
        sp, sm = sig.copy(), sig.copy()
        sp[c] += eps
        sm[c] -= eps
        Lp = np.sum(r * orc.forward(g, sp, nt, dt, omega=30.0, taylor=True, f0=f0, f1=f1).reshape(r.shape))
        Lm = np.sum(r * orc.forward(g, sm, nt, dt, omega=30.0, taylor=True, f0=f0, f1=f1).reshape(r.shape))
        fd.append((Lp - Lm) / (2 * eps))
    fd = np.array(fd)
    assert np.linalg.norm(dsig[el] - fd) <= 1e-7 * np.linalg.norm(fd)
    # the k = 0 weight matters: the leapfrog start from the same levels gives
    # a different gradient
    ds2 = orc.adjoint(g, sig, nt, dt, r, omega=30.0, u0=f0, um1=f0 - dt * f1)
    assert np.linalg.norm(ds2[el] - fd) > 1e-5 * np.linalg.norm(fd)


def test_taylor_zero_data_is_model_problem_2(orc):
    n, C, o = 16, 8, 4
    h = 1.0 / n
    g = orc.Geometry(n, fem_o=o, fem_c=C)
    sig = np.zeros((C, C, C))
    sig[2:C - 2, 2:C - 2, 2:C - 2] = 1.5
    dt, nt = 0.25 * h, 60
    a = orc.forward(g, sig.ravel(), nt, dt, omega=30.0)
    b = orc.forward(g, sig.ravel(), nt, dt, omega=30.0, taylor=True)
    assert np.array_equal(a, b)
