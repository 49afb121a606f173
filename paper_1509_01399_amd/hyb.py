"""ctypes binding of libhyb (include/hyb.h): argument marshalling only.

Every function of the C ABI is exposed under the same name and takes torch
CUDA tensors where the C call takes device pointers.  All computation runs in
the HIP kernels of ``libhyb.so``; this module never computes a step of the
method.  If the library is missing the first call raises RuntimeError.

``Solver`` is a small convenience wrapper holding one ``hyb_ctx``.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhyb.so")

HYB_OK, HYB_E_ARG, HYB_E_MESH, HYB_E_CFL, HYB_E_STATE = 0, -1, -2, -3, -4
HYB_E_OOM, HYB_E_DEVICE, HYB_E_NONFINITE, HYB_E_UNSUPPORTED = -5, -6, -7, -8
STATUS_NAMES = {0: "HYB_OK", -1: "HYB_E_ARG", -2: "HYB_E_MESH", -3: "HYB_E_CFL", -4: "HYB_E_STATE",
                -5: "HYB_E_OOM", -6: "HYB_E_DEVICE", -7: "HYB_E_NONFINITE", -8: "HYB_E_UNSUPPORTED"}
BC_ABC, BC_NEUMANN, BC_SOURCE = 0, 1, 2

EXPORTS = ("hyb_create", "hyb_destroy", "hyb_forward", "hyb_set_initial", "hyb_adjoint",
           "hyb_gradient", "hyb_cg_step", "hyb_footprint", "hyb_sync", "hyb_last_error",
           "hyb_counts", "hyb_time_interior", "hyb_get_wavefield", "hyb_batch_create",
           "hyb_batch_destroy", "hyb_batch_submit", "hyb_batch_tick", "hyb_batch_poll",
           "hyb_batch_release", "hyb_batch_last_error", "hyb_batch_poll_all", "hyb_fem_info",
           "hyb_time_fem", "hyb_set_initial_taylor", "hyb_set_wave_speed", "hyb_gradient_eps",
           "hyb_gradient_noalloc")


class hyb_fd_grid(ct.Structure):
    _fields_ = [("n_cells", ct.c_int32 * 3), ("h", ct.c_double), ("origin", ct.c_double * 3),
                ("face", ct.c_int32 * 6)]


class hyb_fem_mesh(ct.Structure):
    _fields_ = [("n_nodes", ct.c_int64), ("xyz", ct.POINTER(ct.c_double)), ("n_tets", ct.c_int64),
                ("tet4", ct.POINTER(ct.c_int32))]


class hyb_overlap(ct.Structure):
    _fields_ = [("width_cells", ct.c_int32)]


class hyb_opts(ct.Structure):
    _fields_ = [("field_f32", ct.c_int32), ("store_mode", ct.c_int32), ("gamma", ct.c_double),
                ("alpha_rel", ct.c_double), ("hip_stream", ct.c_void_p), ("fem_general", ct.c_int32),
                ("cg_max_trials", ct.c_int32)]


class hyb_source(ct.Structure):
    _fields_ = [("kind", ct.c_int32), ("omega", ct.c_double), ("flux_dev", ct.c_void_p),
                ("k_on", ct.c_int32)]


class hyb_cg_state(ct.Structure):
    _fields_ = [("iter", ct.c_int32), ("gnorm2_prev", ct.c_double), ("beta", ct.c_double),
                ("dmax", ct.c_double), ("alpha", ct.c_double), ("J_next", ct.c_double),
                ("trials", ct.c_int32), ("restart", ct.c_int32), ("stalled", ct.c_int32),
                ("forwards", ct.c_int32)]


class HybError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load():
    """Load libhyb.so (built in-tree by paper_1509_01399_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_1509_01399_amd.build` (HIP path required)")
    lib = ct.CDLL(LIB_PATH)
    P = ct.POINTER
    vp, dp = ct.c_void_p, ct.c_double
    lib.hyb_create.argtypes = [P(hyb_fd_grid), P(hyb_fem_mesh), P(hyb_overlap), P(hyb_opts), P(vp)]
    lib.hyb_destroy.argtypes = [vp]
    lib.hyb_destroy.restype = None
    lib.hyb_forward.argtypes = [vp, vp, P(hyb_source), ct.c_int32, dp, vp]
    lib.hyb_set_initial.argtypes = [vp, vp, vp]
    lib.hyb_set_initial_taylor.argtypes = [vp, vp, vp]
    lib.hyb_set_wave_speed.argtypes = [vp, vp]
    lib.hyb_gradient_eps.argtypes = [vp, vp]
    lib.hyb_adjoint.argtypes = [vp, vp, ct.c_int32]
    lib.hyb_gradient.argtypes = [vp, vp, P(dp)]
    lib.hyb_gradient_noalloc.argtypes = [vp, vp, vp]
    lib.hyb_cg_step.argtypes = [vp, vp, vp, P(hyb_source), ct.c_int32, dp, P(hyb_cg_state), P(dp),
                                P(dp)]
    lib.hyb_footprint.argtypes = [P(hyb_fd_grid), P(hyb_fem_mesh), P(hyb_overlap), P(hyb_opts),
                                  ct.c_int32, P(ct.c_size_t)]
    lib.hyb_sync.argtypes = [vp]
    lib.hyb_last_error.argtypes = [vp]
    lib.hyb_last_error.restype = ct.c_char_p
    lib.hyb_counts.argtypes = [vp, P(ct.c_int64), P(ct.c_int64)]
    lib.hyb_time_interior.argtypes = [vp, vp, dp, ct.c_int32, P(dp)]
    lib.hyb_get_wavefield.argtypes = [vp, ct.c_int32, vp, vp]
    lib.hyb_fem_info.argtypes = [vp, P(ct.c_int64), P(ct.c_int32), P(ct.c_int64)]
    lib.hyb_time_fem.argtypes = [vp, ct.c_int32, ct.c_int32, P(dp)]
    lib.hyb_batch_create.argtypes = [ct.c_int32, vp, P(vp)]
    lib.hyb_batch_destroy.argtypes = [vp]
    lib.hyb_batch_destroy.restype = None
    lib.hyb_batch_submit.argtypes = [vp, vp, vp, dp, P(hyb_source), ct.c_int32, dp, vp, vp, vp,
                                     P(ct.c_int32)]
    lib.hyb_batch_tick.argtypes = [vp, ct.c_int32, P(ct.c_int32)]
    lib.hyb_batch_poll_all.argtypes = [vp, P(ct.c_int32), P(dp)]
    lib.hyb_batch_poll.argtypes = [vp, ct.c_int32, P(ct.c_int32), P(dp)]
    lib.hyb_batch_release.argtypes = [vp, ct.c_int32]
    lib.hyb_batch_last_error.argtypes = [vp]
    lib.hyb_batch_last_error.restype = ct.c_char_p
    for name in EXPORTS:
        if name not in ("hyb_destroy", "hyb_last_error", "hyb_batch_destroy", "hyb_batch_last_error"):
            getattr(lib, name).restype = ct.c_int
    _lib = lib
    return lib


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    return ct.c_void_p(t.data_ptr())


def _check(status, ctx=None):
    if status != HYB_OK:
        msg = load().hyb_last_error(ctx)
        raise HybError(status, msg.decode() if msg else "")


def make_grid(n, h=None, bc=(0, 0, 0, 0, 0, 2), origin=(0.0, 0.0, 0.0)):
    n = (n, n, n) if np.isscalar(n) else tuple(int(v) for v in n)
    g = hyb_fd_grid()
    g.n_cells[:] = n
    g.h = float(h if h is not None else 1.0 / n[2])
    g.origin[:] = origin
    g.face[:] = bc
    return g


def make_mesh(xyz, tet4):
    """Host mesh struct; keeps references to the numpy arrays alive."""
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    tet4 = np.ascontiguousarray(tet4, dtype=np.int32)
    m = hyb_fem_mesh()
    m.n_nodes = xyz.shape[0]
    m.xyz = xyz.ctypes.data_as(ct.POINTER(ct.c_double))
    m.n_tets = tet4.shape[0]
    m.tet4 = tet4.ctypes.data_as(ct.POINTER(ct.c_int32))
    m._keep = (xyz, tet4)
    return m


def make_opts(f32=False, store_mode=0, gamma=0.01, alpha_rel=0.25, stream=None, general=False,
              cg_max_trials=0):
    o = hyb_opts()
    o.cg_max_trials = int(cg_max_trials)
    o.fem_general = int(bool(general))
    o.field_f32 = int(bool(f32))
    o.store_mode = int(store_mode)
    o.gamma = gamma
    o.alpha_rel = alpha_rel
    o.hip_stream = stream
    return o


def make_source(omega=40.0, flux=None, k_on=0):
    s = hyb_source()
    if flux is None:
        s.kind, s.omega = 0, float(omega)
    else:
        s.kind, s.flux_dev, s.k_on = 1, flux.data_ptr(), int(k_on)
    return s


# ---- the C ABI under its own names ----

def hyb_create(grid, fem=None, overlap=2, opts=None):
    lib = load()
    ctx = ct.c_void_p()
    ov = hyb_overlap(overlap)
    st = lib.hyb_create(ct.byref(grid), ct.byref(fem) if fem is not None else None, ct.byref(ov),
                        ct.byref(opts) if opts is not None else None, ct.byref(ctx))
    _check(st)
    return ctx


def hyb_destroy(ctx):
    load().hyb_destroy(ctx)


def hyb_forward(ctx, sigma, src, nt, dt, obs):
    _check(load().hyb_forward(ctx, _ptr(sigma), ct.byref(src), int(nt), float(dt), _ptr(obs)), ctx)


def hyb_set_initial(ctx, u0, um1):
    _check(load().hyb_set_initial(ctx, _ptr(u0), _ptr(um1)), ctx)


def hyb_set_initial_taylor(ctx, f0, f1):
    _check(load().hyb_set_initial_taylor(ctx, _ptr(f0), _ptr(f1)), ctx)


def hyb_set_wave_speed(ctx, eps):
    _check(load().hyb_set_wave_speed(ctx, _ptr(eps)), ctx)


def hyb_gradient_eps(ctx, geps):
    _check(load().hyb_gradient_eps(ctx, _ptr(geps)), ctx)


def hyb_adjoint(ctx, residual, mode):
    _check(load().hyb_adjoint(ctx, _ptr(residual), int(mode)), ctx)


def hyb_gradient(ctx, grad, want_J=False):
    J = ct.c_double(0.0)
    _check(load().hyb_gradient(ctx, _ptr(grad), ct.byref(J) if want_J else None), ctx)
    return J.value if want_J else None


def hyb_gradient_noalloc(ctx, grad, J=None):
    """hyb_gradient without allocation: grad and J (device FP64 [1] or None)
    are device tensors; nothing is synchronised."""
    _check(load().hyb_gradient_noalloc(ctx, _ptr(grad), _ptr(J)), ctx)


def hyb_cg_step(ctx, data, sigma, src, nt, dt, state, want_norms=True):
    gn, J = ct.c_double(0.0), ct.c_double(0.0)
    _check(load().hyb_cg_step(ctx, _ptr(data), _ptr(sigma), ct.byref(src), int(nt), float(dt),
                              ct.byref(state), ct.byref(gn) if want_norms else None,
                              ct.byref(J) if want_norms else None), ctx)
    return (gn.value, J.value) if want_norms else None


def hyb_footprint(grid, fem=None, overlap=2, opts=None, nt=1):
    b = ct.c_size_t(0)
    ov = hyb_overlap(overlap)
    _check(load().hyb_footprint(ct.byref(grid), ct.byref(fem) if fem is not None else None,
                                ct.byref(ov), ct.byref(opts) if opts is not None else None, int(nt),
                                ct.byref(b)))
    return b.value


def hyb_sync(ctx):
    _check(load().hyb_sync(ctx), ctx)


def hyb_last_error(ctx=None):
    m = load().hyb_last_error(ctx)
    return m.decode() if m else ""


def hyb_counts(ctx):
    a, b = ct.c_int64(), ct.c_int64()
    _check(load().hyb_counts(ctx, ct.byref(a), ct.byref(b)), ctx)
    return a.value, b.value


def hyb_time_interior(ctx, sigma, dt, reps):
    ms = ct.c_double()
    _check(load().hyb_time_interior(ctx, _ptr(sigma), float(dt), int(reps), ct.byref(ms)), ctx)
    return ms.value


def hyb_get_wavefield(ctx, which, u, v=None):
    _check(load().hyb_get_wavefield(ctx, int(which), _ptr(u), _ptr(v)), ctx)


def hyb_fem_info(ctx):
    """(number of conductivity values, general mesh?, FEM nodes)."""
    a, b, c = ct.c_int64(), ct.c_int32(), ct.c_int64()
    _check(load().hyb_fem_info(ctx, ct.byref(a), ct.byref(b), ct.byref(c)), ctx)
    return a.value, bool(b.value), c.value


def hyb_time_fem(ctx, which, reps):
    ms = ct.c_double()
    _check(load().hyb_time_fem(ctx, int(which), int(reps), ct.byref(ms)), ctx)
    return ms.value


def _bcheck(status, b):
    if status != HYB_OK:
        msg = load().hyb_batch_last_error(b)
        raise HybError(status, msg.decode() if msg else "")


def hyb_batch_create(max_slots, stream=None):
    b = ct.c_void_p()
    _check(load().hyb_batch_create(int(max_slots), stream, ct.byref(b)))
    return b


def hyb_batch_destroy(b):
    load().hyb_batch_destroy(b)


def hyb_batch_submit(b, ctx, sigma, sigma_max, src, nt, dt, data, obs, grad):
    slot = ct.c_int32(-1)
    _bcheck(load().hyb_batch_submit(b, ctx, _ptr(sigma), float(sigma_max), ct.byref(src), int(nt),
                                    float(dt), _ptr(data), _ptr(obs), _ptr(grad), ct.byref(slot)), b)
    return slot.value


def hyb_batch_tick(b, steps=1):
    n = ct.c_int32(0)
    _bcheck(load().hyb_batch_tick(b, int(steps), ct.byref(n)), b)
    return n.value


def hyb_batch_poll_all(b, max_slots):
    st = (ct.c_int32 * max_slots)()
    J = (ct.c_double * max_slots)()
    _bcheck(load().hyb_batch_poll_all(b, st, J), b)
    return list(st), list(J)


def hyb_batch_poll(b, slot):
    st, J = ct.c_int32(0), ct.c_double(0.0)
    _bcheck(load().hyb_batch_poll(b, int(slot), ct.byref(st), ct.byref(J)), b)
    return st.value, J.value


def hyb_batch_release(b, slot):
    _bcheck(load().hyb_batch_release(b, int(slot)), b)


def hyb_batch_last_error(b):
    m = load().hyb_batch_last_error(b)
    return m.decode() if m else ""


# ---- convenience wrapper ----

class Solver:
    """One problem on one GPU: outer grid n^3 cells (h = 1/n by default), FEM
    box of C cells at cell offset o (C = 0: pure finite differences).  mesh:
    (xyz, tets) of the FEM box (default: the 6-tetrahedra split of its cubes);
    general=True runs even that split on the general-mesh path."""

    def __init__(self, n, C=0, o=None, h=None, bc=(0, 0, 0, 0, 0, 2), f32=False, store_mode=0,
                 gamma=0.01, alpha_rel=0.25, stream=None, mesh=None, general=False):
        import torch
        from . import synth
        self.torch = torch
        self.n = (n, n, n) if np.isscalar(n) else tuple(n)
        self.h = float(h if h is not None else 1.0 / self.n[2])
        self.C = C
        self.o = o if o is not None else (self.n[0] - C) // 2
        self.f32 = f32
        self.grid = make_grid(self.n, self.h, bc)
        if mesh is None and C:
            mesh = synth.kuhn_box_mesh(self.o, C, self.h)
        self.mesh = make_mesh(*mesh) if mesh is not None else None
        self.stream = stream if stream is not None else torch.cuda.current_stream().cuda_stream
        self.opts = make_opts(f32, store_mode, gamma, alpha_rel, self.stream, general)
        self.ctx = hyb_create(self.grid, self.mesh, 2, self.opts)
        self.n_params, self.general, self.n_fem_nodes = hyb_fem_info(self.ctx)
        self.nface = (self.n[0] + 1) * (self.n[1] + 1)
        self.nt = None
        self.generation = 0  # counts forward sweeps (the adjoint uses the last one)

    def close(self):
        if self.ctx is not None:
            hyb_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dev(self):
        return self.torch.device("cuda")

    def trace_buffer(self, nt):
        return self.torch.zeros((nt + 1, self.n[1] + 1, self.n[0] + 1), dtype=self.torch.float64,
                                device=self._dev())

    def forward(self, sigma, nt, dt, omega=40.0, flux=None, k_on=0, obs=None):
        if obs is None:
            obs = self.trace_buffer(nt)
        hyb_forward(self.ctx, sigma, make_source(omega, flux, k_on), nt, dt, obs)
        self.nt = nt
        self.generation += 1
        return obs

    def set_initial(self, u0=None, um1=None):
        self._ic = (u0, um1)
        hyb_set_initial(self.ctx, u0, um1)

    def set_initial_taylor(self, f0=None, f1=None):
        """Model Problem 1 data u(x,0) = f0, u_t(x,0) = f1 for every later
        forward sweep (None, None: back to zero data)."""
        hyb_set_initial_taylor(self.ctx, f0, f1)

    def set_wave_speed(self, eps=None):
        """1/c^2 per FEM cube for every later sweep (None: c = 1)."""
        hyb_set_wave_speed(self.ctx, eps)

    def gradient_eps(self, out=None):
        """dJ/d(1/c^2) per cube after an adjoint (L2 density in mode 0,
        Euclidean in mode 1)."""
        if out is None:
            out = self.torch.zeros((self.C, self.C, self.C), dtype=self.torch.float64, device=self._dev())
        hyb_gradient_eps(self.ctx, out)
        return out

    def adjoint(self, residual, mode=0):
        hyb_adjoint(self.ctx, residual, mode)

    def gradient(self, grad=None, want_J=True):
        if grad is None:
            shape = (self.n_params,) if self.general else (self.C, self.C, self.C)
            grad = self.torch.zeros(shape, dtype=self.torch.float64, device=self._dev())
        J = hyb_gradient(self.ctx, grad, want_J)
        return grad, J

    def cg_step(self, data, sigma, nt, dt, state, omega=40.0):
        """One iteration of Algorithm 3 (sigma updated in place); returns
        (|g^m|, J^m); state reports beta, the step, trials, restart and
        whether the run stalled."""
        self.generation += 1  # runs forward sweeps
        return hyb_cg_step(self.ctx, data, sigma, make_source(omega), nt, dt, state)

    def wavefield(self, which=0):
        """Newest level of the last sweep as (grid [nz,ny,nx], FEM part or None):
        [C+1]^3 on the structured path, [nodes] in mesh order on a general mesh."""
        t = self.torch
        u = t.zeros((self.n[2] + 1, self.n[1] + 1, self.n[0] + 1), dtype=t.float64, device=self._dev())
        shape = (self.n_fem_nodes,) if self.general else (self.C + 1,) * 3
        v = (t.zeros(shape, dtype=t.float64, device=self._dev()) if self.C else None)
        hyb_get_wavefield(self.ctx, which, u, v)
        return u, v

    def counts(self):
        return hyb_counts(self.ctx)

    def time_fem(self, which=0, reps=20):
        return hyb_time_fem(self.ctx, which, reps)

    def sync(self):
        hyb_sync(self.ctx)
