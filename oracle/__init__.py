"""ctypes wrapper around the plain FP64 CPU oracle (``hyb_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, by the smoke check and
by the CPU-baseline leg of the benchmark.  The product package never imports
it, and it imports nothing from the product package.

Geometry convention (shared by the whole project, stated in the paper's
terms): the outer box has ``n[d]`` cells of size ``h`` per axis (``n[d]+1``
nodes, x fastest); the FEM box covers cells ``[o, o+C)`` per axis; faces are
ordered x-, x+, y-, y+, z-, z+; the backscattered trace is recorded on z+.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

from .build import build, lib_path

ABC, NEUMANN, SOURCE = 0, 1, 2


class _Geom(ct.Structure):
    _fields_ = [("n", ct.c_int32 * 3), ("h", ct.c_double), ("bc", ct.c_int32 * 6),
                ("fem_o", ct.c_int32 * 3), ("fem_c", ct.c_int32 * 3)]


class _Mesh(ct.Structure):
    _fields_ = [("n_nodes", ct.c_int64), ("xyz", ct.POINTER(ct.c_double)), ("n_tets", ct.c_int64),
                ("tet4", ct.POINTER(ct.c_int32))]


class _Source(ct.Structure):
    _fields_ = [("kind", ct.c_int32), ("omega", ct.c_double),
                ("flux", ct.POINTER(ct.c_double)), ("k_on", ct.c_int32)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(lib_path()):
            build()
        lib = ct.CDLL(lib_path())
        dp = ct.POINTER(ct.c_double)
        G, M, S = ct.POINTER(_Geom), ct.POINTER(_Mesh), ct.POINTER(_Source)
        lib.orc_sizes_m.argtypes = [G, M, ct.POINTER(ct.c_int64)]
        ci, cd = ct.c_int, ct.c_double
        lib.orc_forward_x.argtypes = [G, M, dp, dp, S, ci, cd, dp, dp, ci, dp, dp, dp]
        lib.orc_adjoint_x.argtypes = [G, M, dp, dp, S, ci, cd, dp, dp, ci, dp, dp, dp, dp, dp, dp, dp, dp]
        lib.orc_threads.argtypes = [ci]
        lib.orc_threads.restype = ci
        lib.orc_misfit.argtypes = [G, ci, cd, dp, dp, dp]
        lib.orc_misfit.restype = ct.c_double
        lib.orc_gradient_x.argtypes = [G, M, dp, dp, S, ci, cd, dp, dp, ci, dp, cd, dp, dp, ct.POINTER(cd), dp]
        lib.orc_cg_x.argtypes = [G, M, dp, dp, S, ci, cd, dp, dp, ci, dp, cd, cd, ci, ci, dp]
        lib.orc_cg_x.restype = ci
        _lib = lib
    return _lib


def threads(n=0):
    """Threads of the oracle's FDM rows (n > 0 sets them); returns the number
    in use.  Results are the same for every thread count."""
    return _load().orc_threads(int(n))


class Geometry:
    """Outer grid, face boundary conditions and FEM box (cells).  mesh: an
    explicit tetrahedral mesh (xyz [nodes, 3], tets [n, 4]) of the FEM box;
    then sigma and the gradients hold one value per tetrahedron.  Without it
    the box is split into the 6 tetrahedra of each cube."""

    def __init__(self, n, h=None, bc=(ABC, ABC, ABC, ABC, ABC, SOURCE), fem_o=(0, 0, 0),
                 fem_c=(0, 0, 0), mesh=None):
        n = (n, n, n) if np.isscalar(n) else tuple(int(v) for v in n)
        self.n = n
        self.h = float(h if h is not None else 1.0 / n[2])
        self.bc = tuple(int(b) for b in bc)
        self.fem_o = (fem_o,) * 3 if np.isscalar(fem_o) else tuple(int(v) for v in fem_o)
        self.fem_c = (fem_c,) * 3 if np.isscalar(fem_c) else tuple(int(v) for v in fem_c)
        self.mesh = None
        if mesh is not None:
            xyz = np.ascontiguousarray(mesh[0], dtype=np.float64)
            tet = np.ascontiguousarray(mesh[1], dtype=np.int32)
            self._keep = (xyz, tet)
            m = _Mesh()
            m.n_nodes, m.n_tets = xyz.shape[0], tet.shape[0]
            m.xyz = xyz.ctypes.data_as(ct.POINTER(ct.c_double))
            m.tet4 = tet.ctypes.data_as(ct.POINTER(ct.c_int32))
            self.mesh = m

    def _m(self):
        return ct.byref(self.mesh) if self.mesh is not None else None

    def _c(self):
        g = _Geom()
        g.n[:] = self.n
        g.h = self.h
        g.bc[:] = self.bc
        g.fem_o[:] = self.fem_o
        g.fem_c[:] = self.fem_c
        return g

    @property
    def nodes(self):
        return tuple(v + 1 for v in self.n)

    @property
    def nface(self):
        return (self.n[0] + 1) * (self.n[1] + 1)

    @property
    def ncube(self):
        return int(np.prod(self.fem_c))

    def sizes(self):
        out = (ct.c_int64 * 8)()
        if _load().orc_sizes_m(ct.byref(self._c()), self._m(), out):
            raise ValueError("invalid geometry")
        keys = ("grid_nodes", "face_nodes", "fem_nodes", "fem_cubes", "fem_updated",
                "fdm_updated", "omega_o", "omega_diamond")
        return dict(zip(keys, list(out)))


def _src(kind=0, omega=40.0, flux=None, k_on=0):
    s = _Source()
    s.kind = kind
    s.omega = omega
    s.k_on = k_on
    if flux is not None:
        s.flux = flux.ctypes.data_as(ct.POINTER(ct.c_double))
    return s


def _p(a):
    return None if a is None else a.ctypes.data_as(ct.POINTER(ct.c_double))


def _f64(a, shape=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _init(u0, um1, taylor, f0, f1):
    """(u0, u1, taylor) of the oracle's _x calls: levels (u0, um1), or the
    Model Problem 1 data (f0, f1) when taylor."""
    if taylor:
        return _f64(f0), _f64(f1), 1
    return _f64(u0), _f64(um1), 0


def forward(geom, sigma, nt, dt, omega=40.0, flux=None, k_on=0, u0=None, um1=None,
            want_vhist=False, want_ufinal=False, taylor=False, f0=None, f1=None, eps=None):
    """Forward sweep of Algorithm 2.  Returns obs [nt+1, ny+1, nx+1] and,
    optionally, the FEM history [nt+1, fz, fy, fx] and the final grid level.
    Initial data: levels u0, um1 (leapfrog start), or with taylor=True the
    Model Problem 1 data f0 = u(x,0), f1 = u_t(x,0) with the Taylor start.
    eps: 1/c^2 per FEM cube (None = 1)."""
    lib = _load()
    g = geom._c()
    sz = geom.sizes()
    sigma, eps = _f64(sigma), _f64(eps)
    flux = _f64(flux)
    a0, a1, tay = _init(u0, um1, taylor, f0, f1)
    obs = np.zeros((nt + 1, geom.n[1] + 1, geom.n[0] + 1))
    vh = np.zeros((nt + 1, sz["fem_nodes"])) if want_vhist and sz["fem_nodes"] else None
    uf = np.zeros(sz["grid_nodes"]) if want_ufinal else None
    s = _src(1 if flux is not None else 0, omega, flux, k_on)
    rc = lib.orc_forward_x(ct.byref(g), geom._m(), _p(sigma), _p(eps), ct.byref(s), nt, dt, _p(a0), _p(a1), tay,
                           _p(obs), _p(vh), _p(uf))
    if rc:
        raise RuntimeError(f"orc_forward failed ({rc})")
    out = [obs]
    if want_vhist:
        out.append(vh)
    if want_ufinal:
        out.append(uf)
    return out[0] if len(out) == 1 else tuple(out)


def adjoint(geom, sigma, nt, dt, seed, omega=40.0, flux=None, k_on=0, u0=None, um1=None,
            want_dflux=False, want_dinit=False, taylor=False, f0=None, f1=None, want_ddata=False,
            eps=None, want_deps=False):
    """Exact discrete adjoint: seed [nt+1, face] is the cotangent of the
    trace.  Returns dJ/dsigma per cell (Euclidean) and optionally, in this
    order: dJ/d(1/c^2) per cube (want_deps), the source cotangent [nt, face],
    the cotangents of u^0, u^{-1} (want_dinit) and, with taylor=True (Model
    Problem 1 data f0, f1), those of f0 and f1 (want_ddata)."""
    lib = _load()
    g = geom._c()
    sz = geom.sizes()
    sigma, eps = _f64(sigma), _f64(eps)
    flux = _f64(flux)
    seed = _f64(seed)
    a0, a1, tay = _init(u0, um1, taylor, f0, f1)
    dsig = np.zeros(max(sz["fem_cubes"], 1))
    deps = np.zeros(max(sz["fem_cubes"], 1)) if want_deps else None
    dflux = np.zeros((nt, geom.nface)) if want_dflux else None
    du0 = np.zeros(sz["grid_nodes"]) if want_dinit else None
    dum1 = np.zeros(sz["grid_nodes"]) if want_dinit else None
    df0 = np.zeros(sz["grid_nodes"]) if want_ddata else None
    df1 = np.zeros(sz["grid_nodes"]) if want_ddata else None
    s = _src(1 if flux is not None else 0, omega, flux, k_on)
    rc = lib.orc_adjoint_x(ct.byref(g), geom._m(), _p(sigma), _p(eps), ct.byref(s), nt, dt, _p(a0), _p(a1), tay,
                           _p(seed), _p(dsig), _p(deps), _p(dflux), _p(du0), _p(dum1), _p(df0), _p(df1))
    if rc:
        raise RuntimeError(f"orc_adjoint failed ({rc})")
    out = [dsig[:sz["fem_cubes"]]]
    if want_deps:
        out.append(deps[:sz["fem_cubes"]])
    if want_dflux:
        out.append(dflux)
    if want_dinit:
        out += [du0, dum1]
    if want_ddata:
        out += [df0, df1]
    return out[0] if len(out) == 1 else tuple(out)


def misfit(geom, nt, dt, obs, data):
    """J_misfit and its trace cotangent seed (eq. (functional))."""
    lib = _load()
    obs, data = _f64(obs), _f64(data)
    seed = np.zeros_like(obs)
    J = lib.orc_misfit(ct.byref(geom._c()), nt, dt, _p(obs), _p(data), _p(seed))
    return J, seed


def gradient(geom, sigma, nt, dt, data, gamma=0.01, omega=40.0, want_obs=False, f0=None, f1=None,
             taylor=False, eps=None, want_geps=False):
    """L2 gradient g_c (eq. (gradient1), discrete) and J at sigma; with
    taylor=True the sweeps start from Model Problem 1 data (f0, f1); eps:
    1/c^2 per cube.  Returns (grad, J[, geps][, obs]); geps is the L2
    density of dJ_misfit/d(1/c^2)."""
    lib = _load()
    sz = geom.sizes()
    sigma, eps = _f64(sigma), _f64(eps)
    data = _f64(data)
    grad = np.zeros(sz["fem_cubes"])
    geps = np.zeros(sz["fem_cubes"]) if want_geps else None
    J = ct.c_double()
    obs = np.zeros_like(data) if want_obs else None
    a0, a1, tay = _init(None, None, taylor, f0, f1)
    s = _src(0, omega)
    rc = lib.orc_gradient_x(ct.byref(geom._c()), geom._m(), _p(sigma), _p(eps), ct.byref(s), nt, dt, _p(a0),
                            _p(a1), tay, _p(data), gamma, _p(grad), _p(geps), ct.byref(J), _p(obs))
    if rc:
        raise RuntimeError(f"orc_gradient failed ({rc})")
    out = [grad, J.value]
    if want_geps:
        out.append(geps)
    if want_obs:
        out.append(obs)
    return tuple(out)


def cg(geom, sigma, nt, dt, data, iters, gamma=0.01, alpha_rel=0.25, omega=40.0, f0=None, f1=None,
       taylor=False, eps=None, max_trials=8):
    """Algorithm 3 with the backtracking step rule: returns (sigma after the
    iterations run, log [iterations run, 8] with columns J^m, |g^m|_L2,
    beta^m, alpha taken (0: none), max|d^m|, trials, restart, J(sigma^{m+1})).
    The run ends early when no trial step lowers J.  taylor=True: IP1, every
    sweep starts from Model Problem 1 data (f0, f1); eps: a known 1/c^2 per
    cube."""
    lib = _load()
    sig = np.array(sigma, dtype=np.float64, copy=True)
    data = _f64(data)
    log = np.zeros((iters, 8))
    a0, a1, tay = _init(None, None, taylor, f0, f1)
    s = _src(0, omega)
    rc = lib.orc_cg_x(ct.byref(geom._c()), geom._m(), _p(sig), _p(_f64(eps)), ct.byref(s), nt, dt, _p(a0), _p(a1),
                      tay, _p(data), gamma, alpha_rel, max_trials, iters, _p(log))
    if rc < 0:
        raise RuntimeError(f"orc_cg failed ({rc})")
    return sig, log[:rc]
