"""Independent whole-grid reference for tiny problems (test helper).

A second CPU formulation of the same discrete method, written without the
oracle's FDM/FEM split: one merged nodal field on the whole grid, a lumped
mass W_i = h^3 2^{-(number of boundary axes of i)}, and a symmetric
edge-conductance stiffness S u = sum_e kappa_e (u_i - u_j) over the axis
edges of the grid.  kappa_e is the sum, over the (up to 4) cubes that contain
the edge, of a_c * w_{c,e}, where w_{c,e} is the entry of the P1 stiffness of
the cube's 6 Kuhn tetrahedra (computed here by brute force from vertex
coordinates), when all 4 cubes around the edge belong to the FEM box; every
other edge joins two finite-difference rows and has kappa_e = h/4 times the
number of its cubes that lie in the domain.
Because the Kuhn cube stiffness couples only along the 12 axis edges, P1 FEM
on such cubes and the seven-point FDM are both special cases of this one
stencil; the hybrid scheme of Algorithm 2 must reproduce it to rounding.
The leapfrog update is u^{k+1} = 2u^k - u^{k-1} - tau^2 W^{-1}(S u^k - b^k),
with b^k the Neumann flux load p(t_k) times the trapezoid face weight on the
source face while the source is on.  Absorbing boundary rows (eq. (eq:abs2))
then overwrite the boundary nodes that have at least one absorbing axis,
faces first, edges next, corners last, each averaging over its absorbing
axes.
"""
from __future__ import annotations

import itertools

import numpy as np

ABC, NEUMANN, SOURCE = 0, 1, 2


def kuhn_cube_stiffness(h):
    """8x8 P1 stiffness (a = 1) of a cube of edge h split into the 6 Kuhn
    tetrahedra along the (0,0,0)-(1,1,1) diagonal; local node l = x + 2y + 4z."""
    K = np.zeros((8, 8))
    for perm in itertools.permutations(range(3)):
        p = np.zeros(3, int)
        verts = [p.copy()]
        for ax in perm:
            p[ax] += 1
            verts.append(p.copy())
        X = np.array(verts, float) * h
        E = (X[1:] - X[0]).T
        vol = abs(np.linalg.det(E)) / 6.0
        Ginv = np.linalg.inv(E)
        G = np.vstack([-Ginv.sum(0), Ginv])
        ids = [int(v[0] + 2 * v[1] + 4 * v[2]) for v in verts]
        Ke = vol * G @ G.T
        for a in range(4):
            for b in range(4):
                K[ids[a], ids[b]] += Ke[a, b]
    return K


def kuhn_cube_lumped_share():
    """Row sums of the P1 mass of the 6 Kuhn tetrahedra of a unit cube,
    lumped: share[l] = sum over the tetrahedra containing local node l of
    |K| / 4 (brute force from the vertex coordinates; they sum to 1)."""
    share = np.zeros(8)
    for perm in itertools.permutations(range(3)):
        p = np.zeros(3, int)
        verts = [p.copy()]
        for ax in perm:
            p[ax] += 1
            verts.append(p.copy())
        X = np.array(verts, float)
        vol = abs(np.linalg.det((X[1:] - X[0]).T)) / 6.0
        for v in verts:
            share[int(v[0] + 2 * v[1] + 4 * v[2])] += vol / 4.0
    return share


class Merged:
    def __init__(self, n, h, bc, fem_o=None, fem_c=None, sigma=None, eps=None):
        self.n = tuple(n)
        self.h = h
        self.bc = tuple(bc)
        nx, ny, nz = (v + 1 for v in n)
        self.shape = (nz, ny, nx)  # arrays indexed [z, y, x]
        # per-cube conductivity a (cells), NaN marks finite-difference cubes
        acell = np.full((n[2], n[1], n[0]), np.nan)
        if fem_c is not None and fem_c[0] > 0:
            o, C = fem_o, fem_c
            a = np.ones((C[2], C[1], C[0]))
            if sigma is not None:
                s = np.asarray(sigma, float).reshape(C[2], C[1], C[0])
                a[2:C[2] - 2, 2:C[1] - 2, 2:C[0] - 2] += s[2:C[2] - 2, 2:C[1] - 2, 2:C[0] - 2]
            acell[o[2]:o[2] + C[2], o[1]:o[1] + C[1], o[0]:o[0] + C[0]] = a
        Kc = kuhn_cube_stiffness(h)
        # kappa for edges along axis d: array of node-pair lower ends
        self.kappa = []
        for d in range(3):
            shp = list(self.shape)
            shp[2 - d] -= 1
            kfem = np.zeros(shp)
            nfem = np.zeros(shp, int)
            ndom = np.zeros(shp, int)
            # the 4 cubes around an edge along d are offset in the two other axes
            others = [e for e in range(3) if e != d]
            for s0 in (0, 1):
                for s1 in (0, 1):
                    # cube index = edge lower node - (1 - s) along the other axes
                    # local position of the edge in that cube: coordinate s along others
                    sl_edge = [slice(None)] * 3
                    sl_cube = [slice(None)] * 3
                    for e, s in zip(others, (s0, s1)):
                        ne = n[e] + 1
                        # edge nodes along e: 0..ne-1 ; cube index c = i - s must be in [0, n[e])
                        lo = s
                        hi = ne - 1 + s  # exclusive end for i such that i - s < n[e]
                        sl_edge[2 - e] = slice(lo, min(hi, ne))
                        sl_cube[2 - e] = slice(lo - s, min(hi, ne) - s)
                    sl_cube[2 - d] = slice(None)
                    sl_edge[2 - d] = slice(None)
                    cubes = acell[tuple(sl_cube)]
                    loc0 = [0, 0, 0]
                    for e, s in zip(others, (s0, s1)):
                        loc0[e] = s
                    loc1 = list(loc0)
                    loc1[d] = 1
                    l0 = loc0[0] + 2 * loc0[1] + 4 * loc0[2]
                    l1 = loc1[0] + 2 * loc1[1] + 4 * loc1[2]
                    w = -Kc[l0, l1]
                    isfem = ~np.isnan(cubes)
                    kfem[tuple(sl_edge)] += np.where(isfem, cubes * w, 0.0)
                    nfem[tuple(sl_edge)] += isfem
                    ndom[tuple(sl_edge)] += 1
            # an edge inside the FEM box (all 4 cubes FEM) takes the FEM
            # conductance; any other edge joins FDM rows and takes h per
            # quarter of its cubes that lie in the domain
            self.kappa.append(np.where(nfem == 4, kfem, h * ndom / 4.0))
        # lumped mass
        W = np.full(self.shape, h ** 3)
        for d in range(3):
            sl = [slice(None)] * 3
            sl[2 - d] = 0
            W[tuple(sl)] *= 0.5
            sl[2 - d] = -1
            W[tuple(sl)] *= 0.5
        if eps is not None:
            # the coefficient 1/c^2 of the free cubes weights their lumped
            # Kuhn mass shares (every other cube keeps 1/c^2 = 1)
            o, C = fem_o, fem_c
            e = np.asarray(eps, float).reshape(C[2], C[1], C[0])
            share = kuhn_cube_lumped_share()
            for kz in range(2, C[2] - 2):
                for ky in range(2, C[1] - 2):
                    for kx in range(2, C[0] - 2):
                        for l in range(8):
                            x, y, z = o[0] + kx + (l & 1), o[1] + ky + ((l >> 1) & 1), o[2] + kz + (l >> 2)
                            W[z, y, x] += h ** 3 * (e[kz, ky, kx] - 1.0) * share[l]
        self.W = W
        # face trapezoid weights on z+
        fw = np.full((ny, nx), h * h)
        fw[0, :] *= 0.5
        fw[-1, :] *= 0.5
        fw[:, 0] *= 0.5
        fw[:, -1] *= 0.5
        self.face_w = fw
        # boundary nodes grouped by codimension
        self.bnd = {1: [], 2: [], 3: []}
        for z in range(nz):
            for y in range(ny):
                for x in range(nx):
                    p = (x, y, z)
                    cd = sum(1 for d in range(3) if p[d] in (0, n[d]))
                    if cd:
                        self.bnd[cd].append(p)

    def stiff(self, u):
        out = np.zeros_like(u)
        for d in range(3):
            ax = 2 - d
            du = np.diff(u, axis=ax) * self.kappa[d]
            sl_lo = [slice(None)] * 3
            sl_hi = [slice(None)] * 3
            sl_lo[ax] = slice(0, -1)
            sl_hi[ax] = slice(1, None)
            out[tuple(sl_lo)] -= du
            out[tuple(sl_hi)] += du
        return out

    def energy(self, u_next, u_cur, dt):
        """E^{k+1/2} = 1/2 |(u^{k+1}-u^k)/tau|_W^2 + 1/2 (u^{k+1})^T S u^k."""
        v = (u_next - u_cur) / dt
        return 0.5 * np.sum(self.W * v * v) + 0.5 * np.sum(u_next * self.stiff(u_cur))

    def run(self, nt, dt, pflux, k_on, u0=None, um1=None, keep=False):
        """pflux(k) -> flux array [ny, nx] on the z+ face at step k."""
        h = self.h
        r = (h - dt) / (h + dt)
        u = np.zeros(self.shape) if u0 is None else np.asarray(u0, float).reshape(self.shape).copy()
        um = np.zeros(self.shape) if um1 is None else np.asarray(um1, float).reshape(self.shape).copy()
        obs = [u[-1].copy()]
        hist = [u.copy()] if keep else None
        for k in range(nt):
            src_on = k < k_on
            b = np.zeros(self.shape)
            if self.bc[5] == SOURCE and src_on:
                b[-1] = pflux(k) * self.face_w
            up = 2 * u - um - dt * dt * (self.stiff(u) - b) / self.W
            for cd in (1, 2, 3):
                for (x, y, z) in self.bnd[cd]:
                    p = (x, y, z)
                    axes = []
                    for d in range(3):
                        if p[d] == 0:
                            f, di = 2 * d, 1
                        elif p[d] == self.n[d]:
                            f, di = 2 * d + 1, -1
                        else:
                            continue
                        t = self.bc[f]
                        absorbing = t == ABC or (t == SOURCE and not src_on)
                        if absorbing:
                            axes.append((d, di))
                    if not axes:
                        continue
                    acc = 0.0
                    for d, di in axes:
                        q = list(p)
                        q[d] += di
                        acc += u[q[2], q[1], q[0]] + r * (u[z, y, x] - up[q[2], q[1], q[0]])
                    up[z, y, x] = acc / len(axes)
            um, u = u, up
            obs.append(u[-1].copy())
            if keep:
                hist.append(u.copy())
        return (np.array(obs), hist) if keep else np.array(obs)
