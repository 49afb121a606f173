"""Seeded synthetic inputs: grids, FEM box meshes, conductivity inclusions,
observation noise and request streams.

This module holds none of the method's arithmetic.  It only draws seeded
random inputs (numpy ``default_rng``) with the shapes and value ranges of the
paper's experiments (Sec. 9: plane-wave source on the front face, small
inclusions of high conductivity inside the FEM box, additive noise on the
backscattered data) and of the benchmark workloads.  It imports nothing from
the rest of the package, so the CPU oracle's tests and the HIP path can both
use it.

Conventions: ``n`` cells per axis (``n+1`` nodes), ``h = 1/n``, FEM box of
``C`` cells starting at cell ``o = (n - C)//2``; per-cube arrays are indexed
``[z, y, x]`` over the C^3 FEM cubes (x fastest when flattened).  Cubes within
two cells of the FEM boundary are never given a non-zero sigma (a = 1 there).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

ABC, NEUMANN, SOURCE = 0, 1, 2
DEFAULT_BC = (ABC, ABC, ABC, ABC, ABC, SOURCE)


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    n: int           # cells per axis of the outer grid
    C: int           # cells per axis of the FEM box
    nt: int          # time steps
    omega: float     # plane-wave angular frequency
    inclusions: str  # generator name
    noise: float     # relative additive noise level
    cg_iters: int
    precision: str   # "f64" or "f32"

    @property
    def o(self):
        return (self.n - self.C) // 2

    @property
    def h(self):
        return 1.0 / self.n


# The five benchmark workloads (sizes from the project's configuration list).
WORKLOADS = {
    "tiny40": Workload("tiny40", 40, 16, 300, 40.0, "symmetric_pair", 0.0, 3, "f64"),
    "cg256": Workload("cg256", 256, 96, 1200, 40.0, "cubes", 0.03, 10, "f64"),
    "diff384": Workload("diff384", 384, 128, 2000, 40.0, "bumps", 0.0, 0, "f32"),
    "scale512": Workload("scale512", 512, 160, 2500, 40.0, "cubes", 0.03, 0, "f32"),
}
SERVE_SIZES = (64, 96, 128, 192, 256)


def dt_rule(h, sigma_max):
    """Time step used for a workload: 0.4 h when the medium is homogeneous
    enough for it, else 0.25 h (stable for every a = 1 + sigma <= 5 under the
    paper's CFL bound tau <= h / sqrt(3 a))."""
    return 0.4 * h if 1.0 + sigma_max <= 1.0 / (3 * 0.4 ** 2) else 0.25 * h


def eligible_mask(C):
    m = np.zeros((C, C, C), bool)
    m[2:C - 2, 2:C - 2, 2:C - 2] = True
    return m


def symmetric_pair(C, seed, edge=3, value=2.0):
    """Two edge^3-cell cubes of sigma = value, mirror images about the box's
    mid-plane x = const, at seed-chosen offsets inside the free cubes."""
    rng = np.random.default_rng(seed)
    s = np.zeros((C, C, C))
    lo, hi = 2, C - 2
    half = C // 2
    x0 = int(rng.integers(lo, max(lo + 1, half - edge)))  # gap >= 1 cell
    y0 = int(rng.integers(lo, hi - edge + 1))
    z0 = int(rng.integers(lo, hi - edge + 1))
    x1 = C - x0 - edge
    s[z0:z0 + edge, y0:y0 + edge, x0:x0 + edge] = value
    s[z0:z0 + edge, y0:y0 + edge, x1:x1 + edge] = value
    return s


def cubes(C, seed, count=(1, 4), edge=(4, 12), value=(1.0, 4.0)):
    """1-4 cubic inclusions with edges 4-12 cells and sigma ~ U(1,4), placed
    uniformly inside the free cubes; overlaps keep the larger value."""
    rng = np.random.default_rng(seed)
    s = np.zeros((C, C, C))
    lo, hi = 2, C - 2
    k = int(rng.integers(count[0], count[1] + 1))
    for _ in range(k):
        e = int(rng.integers(edge[0], edge[1] + 1))
        e = min(e, hi - lo)
        v = float(rng.uniform(*value))
        p = [int(rng.integers(lo, hi - e + 1)) for _ in range(3)]
        blk = s[p[2]:p[2] + e, p[1]:p[1] + e, p[0]:p[0] + e]
        np.maximum(blk, v, out=blk)
    return s


def bumps(C, h, seed, count=(1, 4), amp=(0.0, 2.0), width=(2.0, 6.0)):
    """Sum of Gaussian bumps (amplitude ~U(0,2), width ~U(2h,6h)) sampled at
    cube centres on the free cubes, clipped to [0, 4]."""
    rng = np.random.default_rng(seed)
    k = int(rng.integers(count[0], count[1] + 1))
    c = (np.arange(C) + 0.5) * h
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    s = np.zeros((C, C, C))
    for _ in range(k):
        a = rng.uniform(*amp)
        w = rng.uniform(*width) * h
        ctr = rng.uniform(2 * h, (C - 2) * h, 3)
        s += a * np.exp(-((X - ctr[0]) ** 2 + (Y - ctr[1]) ** 2 + (Z - ctr[2]) ** 2) / (2 * w * w))
    s = np.clip(s, 0.0, 4.0)
    s[~eligible_mask(C)] = 0.0
    return s


def wave_speed(C, seed, count=(1, 4), edge=(4, 12), speed=(1.0, 2.0)):
    """1/c^2 per FEM cube: 1-4 cubic regions (edges 4-12 cells) with wave
    speed c ~ U(1, 2) inside the free cubes, c = 1 elsewhere (the coefficient
    range c in [1, d2] of condition (coefic) with d2 = 2); overlapping regions
    keep the faster speed."""
    rng = np.random.default_rng(seed)
    c = np.ones((C, C, C))
    lo, hi = 2, C - 2
    k = int(rng.integers(count[0], count[1] + 1))
    for _ in range(k):
        e = min(int(rng.integers(edge[0], edge[1] + 1)), hi - lo)
        v = float(rng.uniform(*speed))
        p = [int(rng.integers(lo, hi - e + 1)) for _ in range(3)]
        blk = c[p[2]:p[2] + e, p[1]:p[1] + e, p[0]:p[0] + e]
        np.maximum(blk, v, out=blk)
    return 1.0 / (c * c)


def gaussian_initial(n, h=None):
    """The initial condition of the paper's Test 1, read with x3^2:
    u(x, 0) = exp(-(x1^2 + x2^2 + x3^2)) on the (n+1)^3 grid, at rest."""
    h = 1.0 / n if h is None else h
    x = np.arange(n + 1) * h
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    return np.exp(-(X ** 2 + Y ** 2 + Z ** 2))


def face_gaussian(n, omega, width=0.25, h=None):
    """Initial condition of the reconstruction study's Model Problem 1 test:
    a Gaussian bump of the given width at the centre of the backscattered
    face z = 1, scaled by 1/omega (the amplitude of the plane wave the source
    sends), at rest.  The paper places exp(-|x|^2) at the backscattered side
    of a domain whose size it does not give, and notes that it changes the
    data little; at unit amplitude and width on the unit cube it would
    dominate the trace and its noise."""
    h = 1.0 / n if h is None else h
    x = np.arange(n + 1) * h
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    r2 = (X - 0.5) ** 2 + (Y - 0.5) ** 2 + (Z - 1.0) ** 2
    return np.exp(-r2 / (width * width)) / omega


def sigma_for(wl: Workload, seed=0):
    if wl.inclusions == "symmetric_pair":
        return symmetric_pair(wl.C, seed)
    if wl.inclusions == "cubes":
        return cubes(wl.C, seed)
    if wl.inclusions == "bumps":
        return bumps(wl.C, wl.h, seed)
    raise ValueError(wl.inclusions)


def add_noise(obs, level, seed, kind="additive"):
    """Gaussian noise, xi ~ N(0,1) i.i.d.: additive and scaled by the largest
    absolute datum, data = obs + level * max|obs| * xi (the workloads), or
    relative to each datum, data = obs * (1 + level * xi)."""
    if level == 0:
        return np.array(obs, dtype=np.float64, copy=True)
    rng = np.random.default_rng(seed)
    obs = np.asarray(obs, dtype=np.float64)
    if kind == "relative":
        return obs * (1.0 + level * rng.standard_normal(obs.shape))
    if kind != "additive":
        raise ValueError(f"noise kind {kind!r}")
    return obs + level * np.max(np.abs(obs)) * rng.standard_normal(obs.shape)


def kuhn_box_mesh(o, C, h, origin=(0.0, 0.0, 0.0)):
    """Tetrahedral mesh of the FEM box [o, o+C]^3 (cells of size h): node
    coordinates [(C+1)^3, 3] (x fastest) and [6 C^3, 4] node ids, each cube
    split into the 6 tetrahedra v0 -> v0+e_p -> v0+e_p+e_q -> v0+1 along the
    cube diagonal, one per ordering (p, q, r) of the axes."""
    o = (o,) * 3 if np.isscalar(o) else tuple(o)
    C = (C,) * 3 if np.isscalar(C) else tuple(C)
    fx, fy, fz = C[0] + 1, C[1] + 1, C[2] + 1
    k, j, i = np.meshgrid(np.arange(fz), np.arange(fy), np.arange(fx), indexing="ij")
    xyz = np.stack([(o[0] + i) * h + origin[0], (o[1] + j) * h + origin[1],
                    (o[2] + k) * h + origin[2]], -1).reshape(-1, 3)
    cz, cy, cx = np.meshgrid(np.arange(C[2]), np.arange(C[1]), np.arange(C[0]), indexing="ij")
    base = np.stack([cx.ravel(), cy.ravel(), cz.ravel()], -1)
    perms = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]
    tets = []
    for p in perms:
        v = base.copy()
        ids = [v[:, 0] + fx * (v[:, 1] + fy * v[:, 2])]
        for ax in p:
            v = v.copy()
            v[:, ax] += 1
            ids.append(v[:, 0] + fx * (v[:, 1] + fy * v[:, 2]))
        tets.append(np.stack(ids, -1))
    tet = np.stack(tets, 1).reshape(-1, 4).astype(np.int32)  # cube-major, 6 per cube
    return xyz.astype(np.float64), tet


def perturbed_box_mesh(o, C, h, seed, amp=0.15):
    """Unstructured mesh of the FEM box: the 6-tetrahedra split of every cube,
    with each node strictly inside the inner box (o+2, o+C-2)^3 moved by an
    offset ~U(-amp h, amp h) per axis.  The two-cell overlap layer and the
    inner box surface keep their grid nodes (the coupling to the grid needs
    them); inside, element shapes, volumes and lumped masses vary and every
    element matrix couples all 4 vertices.  amp <= 0.2 keeps every element
    positively oriented."""
    xyz, tet = kuhn_box_mesh(o, C, h)
    rng = np.random.default_rng(seed)
    q = np.rint(xyz / h).astype(np.int64) - np.asarray((o,) * 3 if np.isscalar(o) else o)
    inner = np.all((q > 2) & (q < C - 2), axis=1)
    xyz = xyz.copy()
    xyz[inner] += rng.uniform(-amp * h, amp * h, (int(inner.sum()), 3))
    return xyz, tet


def tet_sigma(xyz, tet, sigma_cube, o, C, h):
    """Per-tetrahedron conductivity sampling a per-cube field at each
    element's centroid (cube cells of the FEM box)."""
    cen = xyz[tet].mean(axis=1) / h - np.asarray((o,) * 3 if np.isscalar(o) else o)
    idx = np.clip(np.floor(cen).astype(np.int64), 0, C - 1)
    return np.asarray(sigma_cube)[idx[:, 2], idx[:, 1], idx[:, 0]]


def poisson_arrivals(n_req, rate, seed):
    """Arrival times (seconds) of a Poisson stream with the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, n_req))


def serve_requests(n_req, seed, sizes=SERVE_SIZES):
    """Request mix: grid size uniform over `sizes`, FEM box 3/8 of the edge,
    1-4 cubic inclusions, nt = 5 n steps (dt = 0.25 h)."""
    rng = np.random.default_rng(seed)
    out = []
    for r in range(n_req):
        n = int(rng.choice(sizes))
        C = 3 * n // 8
        out.append(dict(id=r, n=n, C=C, o=(n - C) // 2, nt=5 * n, omega=40.0,
                        sigma_seed=int(rng.integers(0, 2 ** 31 - 1))))
    return out


def cfl_limit(h, a_max):
    """The paper's bound tau <= h / sqrt(3 a) for a uniform grid."""
    return h / math.sqrt(3.0 * a_max)
