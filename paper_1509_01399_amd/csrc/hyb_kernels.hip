// HIP kernels (gfx950) of the domain-decomposition FEM/FDM time stepping of
// arXiv 1509.01399 (Algorithm 2, Sec. 7.5) and its exact discrete adjoint.
//
// Per forward step k -> k+1 one launch, and a second one while a face has
// reflecting rows:
//   k_interior<T,false>: the seven-point leapfrog of eq. (fdmschemeforward)
//     on every FDM-owned interior node (blocks of 8 grid rows of 16 bytes of
//     columns per lane, 64 x 8 in FP64 and 128 x 8 in FP32, streaming along
//     z, each plane staged in LDS; the hole [o+2, o+C-2]^3 is skipped) and,
//     in the same launch, the lumped-mass P1 update of eq. (fem) on the open
//     FEM box (32 x 8 columns).  On the 6-tetrahedra cube split the P1
//     stiffness couples only along the 12 axis edges of each cube, so the
//     element gather over the 8 cubes around a node reduces to six edge
//     conductances kappa_e = sum over the 4 cubes of the edge of a_c * w_{c,e}
//     (w from the element matrices computed on the host); no atomics.  The
//     rows of absorbing faces, eq. (eq:abs2), away from the edges, the copy
//     of Algorithm 2 step 3 (FEM values into the grid on omega_diamond) and
//     the trace on an absorbing z+ face are computed here too.  Step 4 (grid
//     values into the FEM level on omega_o) needs no copy: the FEM rows read
//     those neighbours from the grid level.  Its first blocks compute the
//     edge and corner rows of the previous step (no row of this step reads
//     them).
//   k_bnd_fwd: the rows of reflecting faces (the ghost-node Neumann/source
//     rows of eq. (f)), with their part of the trace; the edges and corners
//     run there too when they are not carried by the next interior launch.
//     An edge or corner thread recomputes the values of the boundary
//     neighbours it depends on (a corner's edges, a reflecting face node),
//     so its threads need no ordering (three rotating buffers keep level
//     k-1 intact).
// Per adjoint step (computing the multipliers of level k) the reverse:
//   k_bnd_adj_ecf: multipliers of the corner and edge rows, and beside them
//     the FEM rows of the adjoint with the FP64 gradient time-integral of
//     eq. (gradient1) and the omega_o couplings of the FDM rows;
//   k_bnd_adj_face: multipliers of the face rows, including the trace seed;
//   k_interior<T,true>: the FDM stencil applied to the multipliers plus the
//     transposed boundary and exchange couplings.
#include "hyb_gen_rows.h"
#include "hyb_internal.h"

#include <cmath>
#include <mutex>

namespace hyb {

__device__ __forceinline__ long long gidx(const Geo &g, int x, int y, int z)
{
    return (long long)x + (long long)y * g.px + (long long)z * g.plane;
}

__device__ __forceinline__ long long fidx(const Geo &g, int i, int j, int k)
{
    return (long long)i + (long long)j * g.fpx + (long long)k * g.fplane;
}

__device__ __forceinline__ int ftype(int types, int f) { return (types >> (2 * f)) & 3; }

__device__ __forceinline__ bool on_bnd(const Geo &g, int x, int y, int z)
{
    return x == 0 || y == 0 || z == 0 || x == g.nx - 1 || y == g.ny - 1 || z == g.nz - 1;
}

// Boundary axes of a node and the condition of each at one step; kind[d] is
// -1 when d is not a boundary axis, dir[d] the inward direction.  Fixed-size
// per-axis arrays indexed by unrolled loop constants stay in registers.
struct BInfo {
    int kind[3], dir[3];
    int nabc;
};

__device__ __forceinline__ BInfo classify(const Geo &g, int x, int y, int z, int types)
{
    BInfo B;
    B.nabc = 0;
    const int c[3] = {x, y, z};
    const int m[3] = {g.nx - 1, g.ny - 1, g.nz - 1};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        B.kind[d] = -1;
        B.dir[d] = 0;
        if (c[d] == 0) { B.kind[d] = ftype(types, 2 * d); B.dir[d] = 1; }
        else if (c[d] == m[d]) { B.kind[d] = ftype(types, 2 * d + 1); B.dir[d] = -1; }
        if (B.kind[d] == F_ABC) B.nabc++;
    }
    return B;
}

// Index of a boundary node in the compact per-face arrays (the node is
// stored once, on its first boundary face in the order x, y, z).
__device__ __forceinline__ long long cidx(const Geo &g, int x, int y, int z)
{
    if (x == 0) return g.foff[0] + y + (long long)g.ny * z;
    if (x == g.nx - 1) return g.foff[1] + y + (long long)g.ny * z;
    if (y == 0) return g.foff[2] + x + (long long)g.nx * z;
    if (y == g.ny - 1) return g.foff[3] + x + (long long)g.nx * z;
    if (z == 0) return g.foff[4] + x + (long long)g.nx * y;
    return g.foff[5] + x + (long long)g.nx * y;
}

// Boundary threads: face-interior nodes first (z faces, then y, then x; f is
// the face), then the 12 edges, then the 8 corners.  The coordinates are
// formed with selects: assigning them in branches that depend on the thread
// makes the compiler keep them in scratch memory.
__device__ __forceinline__ void face_node(const Geo &g, long long t, int &x, int &y, int &z, int &f)
{
    const long long ax = g.nx - 2, ay = g.ny - 2, az = g.nz - 2;
    const long long A45 = ax * ay, A23 = ax * az, A01 = ay * az;
    long long r, a1;
    if (t < 2 * A45) {
        f = t < A45 ? 4 : 5;
        r = t % A45;
        a1 = ax;
    } else if (t - 2 * A45 < 2 * A23) {
        t -= 2 * A45;
        f = t < A23 ? 2 : 3;
        r = t % A23;
        a1 = ax;
    } else {
        t -= 2 * A45 + 2 * A23;
        f = t < A01 ? 0 : 1;
        r = t % A01;
        a1 = ay;
    }
    // tangential positions in storage order, the normal coordinate fixed
    const int p = 1 + (int)(r % a1), q = 1 + (int)(r / a1);
    const int d = f >> 1;
    const bool hi = f & 1;
    x = d == 0 ? (hi ? g.nx - 1 : 0) : p;
    y = d == 1 ? (hi ? g.ny - 1 : 0) : (d == 0 ? p : q);
    z = d == 2 ? (hi ? g.nz - 1 : 0) : q;
}

// Absorbing x faces: their adjoint rows away from the face's edges (y in
// [2, ny-3], z in [2, nz-3]) run in the adjoint interior launch (fdm_tile),
// whose x = 0 lane and x = nx-2 lane already hold the inward neighbour's
// multiplier; the face launch covers the ring next to the edges (it reads
// the edge multipliers of the same level) and every row of a reflecting x
// face.  A face qualifies when it is absorbing in the rows of steps k and
// k+1 (types1, types2), the two rows its level-k multiplier enters, and, for
// x = nx-1, when that column lies inside the last tile rather than in its
// halo (a halo column would need a store instruction of its own per row:
// measured +2 us per FP64 adjoint step at 257^3, more than the face launch
// saves on that face).
__host__ __device__ __forceinline__ long long x_fast_rows(const Geo &g)
{
    return (g.ny >= 5 && g.nz >= 5) ? (long long)(g.ny - 4) * (g.nz - 4) : 0;
}
__host__ __device__ __forceinline__ bool x_face_in_tile(const Geo &g, int types1, int types2, int f)
{
    return x_fast_rows(g) > 0 && ((types1 >> (2 * f)) & 3) == F_ABC && ((types2 >> (2 * f)) & 3) == F_ABC &&
           (f == 0 || (g.nx - 2) % TX_FDM != TX_FDM - 1);
}
// face-launch rows of x face f
__host__ __device__ __forceinline__ long long x_face_launch_rows(const Geo &g, int types1, int types2, int f)
{
    const long long A01 = (long long)(g.ny - 2) * (g.nz - 2);
    return x_face_in_tile(g, types1, types2, f) ? A01 - x_fast_rows(g) : A01;
}
__host__ __device__ __forceinline__ long long adj_face_rows(const Geo &g, int types1, int types2)
{
    const long long A01 = (long long)(g.ny - 2) * (g.nz - 2);
    return g.n_fi - 2 * A01 + x_face_launch_rows(g, types1, types2, 0) + x_face_launch_rows(g, types1, types2, 1);
}

// Face-interior node t of the adjoint face launch: the z and y faces as in
// face_node, then per x face all its rows, or only its ring next to the
// edges (the rows z = 1 and z = nz-2, then the columns y = 1 and y = ny-2)
// when its other rows run in the interior launch.
__device__ __forceinline__ void adj_face_node(const Geo &g, int types1, int types2, long long t, int &x, int &y,
                                              int &z, int &f)
{
    const long long A01 = (long long)(g.ny - 2) * (g.nz - 2);
    const long long zy = g.n_fi - 2 * A01;
    if (t < zy) {
        face_node(g, t, x, y, z, f);
        return;
    }
    t -= zy;
    const long long c0 = x_face_launch_rows(g, types1, types2, 0);
    f = t < c0 ? 0 : 1;
    const long long r = f ? t - c0 : t;
    x = f ? g.nx - 1 : 0;
    const long long a = g.ny - 2;
    if (!x_face_in_tile(g, types1, types2, f)) {
        y = 1 + (int)(r % a);
        z = 1 + (int)(r / a);
    } else if (r < 2 * a) {
        y = 1 + (int)(r % a);
        z = r < a ? 1 : g.nz - 2;
    } else {
        const long long r2 = r - 2 * a, b = g.nz - 4;
        y = r2 < b ? 1 : g.ny - 2;
        z = 2 + (int)(r2 % b);
    }
}

__device__ __forceinline__ void edge_corner_node(const Geo &g, long long t, int &x, int &y, int &z)
{
    const long long ex = g.nx - 2, ey = g.ny - 2, ez = g.nz - 2;
    // a: axis of the edge (3 for corners); e: edge number on that axis (or
    // the corner number); p: position along the edge
    int a;
    long long e, p = 0;
    if (t < 4 * ex) {
        a = 0; e = t / ex; p = 1 + t % ex;
    } else if (t - 4 * ex < 4 * ey) {
        t -= 4 * ex;
        a = 1; e = t / ey; p = 1 + t % ey;
    } else if (t - 4 * ex - 4 * ey < 4 * ez) {
        t -= 4 * ex + 4 * ey;
        a = 2; e = t / ez; p = 1 + t % ez;
    } else {
        a = 3; e = t - 4 * (ex + ey + ez);
    }
    const bool bx = e & 1, by = a == 0 ? (e & 1) : (e & 2), bz = a == 3 ? (e & 4) : (e & 2);
    x = a == 0 ? (int)p : (bx ? g.nx - 1 : 0);
    y = a == 1 ? (int)p : (by ? g.ny - 1 : 0);
    z = a == 2 ? (int)p : (bz ? g.nz - 1 : 0);
}

template <typename T>
__device__ __forceinline__ T src_flux(const Step<T> &s, int x, int y)
{
    return s.flux ? (T)(s.fluxscale * s.flux[x + (long long)s.g.nx * y]) : s.srcterm;
}

// A face-interior node whose face is absorbing at this step: its new value
// comes from the interior launch.
__device__ __forceinline__ bool fwd_face_in_tile(const Geo &g, int types, int x, int y, int z)
{
    const bool bx = x == 0 || x == g.nx - 1, by = y == 0 || y == g.ny - 1, bz = z == 0 || z == g.nz - 1;
    if ((int)bx + (int)by + (int)bz != 1) return false;
    const int f = bx ? (x == 0 ? 0 : 1) : (by ? (y == 0 ? 2 : 3) : (z == 0 ? 4 : 5));
    return ftype(types, f) == F_ABC;
}

// Level k+1 value of boundary node (x,y,z), any codimension.  Ghost-node
// leapfrog when every boundary axis reflects (Neumann, or the source face
// while the pulse is on: each such axis contributes 2(u_in - u)/h^2, the
// source adds 2 p/h); otherwise the absorbing row of eq. (eq:abs2) averaged
// over the absorbing axes.  The absorbing row needs the new value of the
// inward neighbour: read from the level, unless that neighbour is itself a
// boundary node the interior launch does not compute (an edge of a corner, or
// a ghost-row face node), which is then recomputed here (D bounds the depth:
// corner -> edge -> face).
template <typename T, int D>
__device__ __forceinline__ T bnd_fwd(const Step<T> &s, int x, int y, int z)
{
    const Geo &g = s.g;
    const BInfo B = classify(g, x, y, z, s.types1);
    const long long id = gidx(g, x, y, z);
    const long long st[3] = {1, g.px, g.plane};
    const T u = s.Ub[id];
    if (B.nabc == 0) {
        T lap = 0;
        bool src = false;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            if (B.kind[d] < 0) lap += (s.Ub[id + st[d]] - u) + (s.Ub[id - st[d]] - u);
            else lap += (T)2 * (s.Ub[id + B.dir[d] * st[d]] - u);
            if (B.kind[d] == F_SOURCE) src = true;
        }
        if constexpr (incr_form<T>()) {
            T d = s.Da[id] + s.c2 * lap;
            if (src) d += src_flux(s, x, y);
            return u + d;
        } else {
            T v = (T)2 * u - s.Ua[id] + s.c2 * lap;
            if (src) v += src_flux(s, x, y);
            return v;
        }
    }
    T acc = 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (B.kind[d] != F_ABC) continue;
        const int cx = x + (d == 0 ? B.dir[d] : 0), cy = y + (d == 1 ? B.dir[d] : 0),
                  cz = z + (d == 2 ? B.dir[d] : 0);
        const long long in = gidx(g, cx, cy, cz);
        T up;
        if constexpr (D > 1)
            up = (on_bnd(g, cx, cy, cz) && !fwd_face_in_tile(g, s.types1, cx, cy, cz)) ? bnd_fwd<T, D - 1>(s, cx, cy, cz)
                                                                                   : s.Uc[in];
        else up = s.Uc[in];
        acc += s.Ub[in] + s.r * (u - up);
    }
    return acc / (T)B.nabc;
}

// Surface node t of a box with L+1 nodes per axis (L >= 1): local coords.
__device__ __forceinline__ void box_surface(long long t, int L, int &a, int &b, int &c)
{
    const long long n1 = L + 1, f = n1 * n1;
    if (t < 2 * f) {
        c = t < f ? 0 : L;
        const long long r = t % f;
        a = (int)(r % n1);
        b = (int)(r / n1);
        return;
    }
    t -= 2 * f;
    const long long fy = n1 * (L - 1);
    if (t < 2 * fy) {
        b = t < fy ? 0 : L;
        const long long r = t % fy;
        a = (int)(r % n1);
        c = 1 + (int)(r / n1);
        return;
    }
    t -= 2 * fy;
    const long long fx = (long long)(L - 1) * (L - 1);
    a = t < fx ? 0 : L;
    const long long r = t % fx;
    b = 1 + (int)(r % (L - 1));
    c = 1 + (int)(r / (L - 1));
}

// Face-interior rows of the forward step on an absorbing face are computed
// by the interior launch (fdm_tile_cols), as is the overlap copy; the
// boundary launch takes the faces whose rows are not absorbing at this step
// (ghost-node Neumann or source rows), then the edges and corners.
__host__ __device__ __forceinline__ long long face_area(const Geo &g, int f)
{
    const int d = f >> 1;
    return d == 2 ? (long long)(g.nx - 2) * (g.ny - 2)
                  : (d == 1 ? (long long)(g.nx - 2) * (g.nz - 2) : (long long)(g.ny - 2) * (g.nz - 2));
}
__host__ __device__ __forceinline__ long long fwd_face_rows(const Geo &g, int types)
{
    long long n = 0;
    for (int f = 0; f < 6; ++f)
        if (((types >> (2 * f)) & 3) != F_ABC) n += face_area(g, f);
    return n;
}

// Node t of the forward launch's face rows: the non-absorbing faces in the
// order z, y, x (low side first), tangential positions as in face_node.
__device__ __forceinline__ void fwd_face_node(const Geo &g, int types, long long t, int &x, int &y, int &z, int &f)
{
    f = 5;
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        const int ff = q < 2 ? 4 + q : (q < 4 ? q : q - 4);
        if (ftype(types, ff) == F_ABC) continue;
        const long long A = face_area(g, ff);
        if (t < A) {
            f = ff;
            break;
        }
        t -= A;
    }
    const int d = f >> 1;
    const bool hi = f & 1;
    const long long a1 = d == 0 ? g.ny - 2 : g.nx - 2;
    const int p = 1 + (int)(t % a1), q2 = 1 + (int)(t / a1);
    x = d == 0 ? (hi ? g.nx - 1 : 0) : p;
    y = d == 1 ? (hi ? g.ny - 1 : 0) : (d == 0 ? p : q2);
    z = d == 2 ? (hi ? g.nz - 1 : 0) : q2;
}

// Edge or corner node t of the forward step s (t >= n_ec: nothing).
template <typename T>
__device__ __forceinline__ void edge_row(const Step<T> &s, long long t)
{
    const Geo &g = s.g;
    if (t < 0 || t >= g.n_ec) return;
    int x, y, z;
    edge_corner_node(g, t, x, y, z);
    const T v = bnd_fwd<T, 3>(s, x, y, z);
    const long long id = gidx(g, x, y, z);
    s.Uc[id] = v;
    if constexpr (incr_form<T>()) s.Dc[id] = v - s.Ub[id];
    if (s.obs && z == g.nz - 1) s.obs[x + (long long)g.nx * y] = (double)v;
}

// The edge rows of the step described by ea, with the invariant arguments
// (geometry, r) of the step s that carries them.
template <typename T>
__device__ __forceinline__ void edge_row_of(const Step<T> &s, const EdgeArgs<T> &ea, long long t)
{
    Step<T> e = s;
    e.Ua = ea.Ua; e.Ub = ea.Ub; e.Da = ea.Da; e.Uc = ea.Uc; e.Dc = ea.Dc;
    e.obs = ea.obs; e.flux = ea.flux; e.fluxscale = ea.fluxscale;
    e.srcterm = ea.srcterm; e.c2 = ea.c2; e.types1 = ea.types1;
    edge_row<T>(e, t);
}

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_bnd_fwd_edges(Step<T> s)
{
    edge_row<T>(s, (long long)blockIdx.x * BLOCK + threadIdx.x);
}

template <typename T>
__device__ __forceinline__ void bnd_fwd_body(const Step<T> &s, long long t)
{
    const Geo &g = s.g;
    const long long nfr = fwd_face_rows(g, s.types1);
    if (t < nfr) {
        // ghost-node row of a reflecting face (Neumann, or the source face
        // while the source is on), eq. (f)
        int x, y, z, f;
        fwd_face_node(g, s.types1, t, x, y, z, f);
        const int d = f >> 1, dir = (f & 1) ? -1 : 1;
        const long long sd = d == 0 ? 1 : (d == 1 ? g.px : g.plane);     // inward axis stride
        const long long sa = d == 0 ? g.px : 1, sb = d == 2 ? g.px : g.plane;  // tangential strides
        const long long id = gidx(g, x, y, z), in = id + dir * sd;
        const int kind = ftype(s.types1, f);
        const T u = s.Ub[id];
        T v;
        const T lap = (T)2 * (s.Ub[in] - u) + ((s.Ub[id + sa] - u) + (s.Ub[id - sa] - u)) +
                      ((s.Ub[id + sb] - u) + (s.Ub[id - sb] - u));
        if constexpr (incr_form<T>()) {
            T dd = s.Da[id] + s.c2 * lap;
            if (kind == F_SOURCE) dd += src_flux(s, x, y);
            s.Dc[id] = dd;
            v = u + dd;
        } else {
            v = (T)2 * u - s.Ua[id] + s.c2 * lap;
            if (kind == F_SOURCE) v += src_flux(s, x, y);
        }
        s.Uc[id] = v;
        if (s.obs && f == 5) s.obs[x + (long long)g.nx * y] = (double)v;
        return;
    }
    edge_row<T>(s, t - nfr);
}

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_bnd_fwd(Step<T> s)
{
    bnd_fwd_body<T>(s, (long long)blockIdx.x * BLOCK + threadIdx.x);
}

// ---------------------------------------------------------------- adjoint
//
// Multipliers of the boundary rows live in compact per-face arrays (Fa, Fb,
// Fc = levels k+2, k+1, k).  The grid array of level k+1 carries, at each
// face node, the value the seven-point stencil of the interior neighbour has
// to see ("proxy": (wB1 mu^{k+1}_b + wB0 mu^k_b) / c2), so the interior
// adjoint update is the plain stencil.

template <typename T>
__device__ __forceinline__ T seed_at(const Step<T> &s, int x, int y)
{
    const Geo &g = s.g;
    double rv = s.res[x + (long long)g.nx * y];
    if (s.seed_mode == 0) {
        double w = s.h2;
        if (x == 0 || x == g.nx - 1) w *= 0.5;
        if (y == 0 || y == g.ny - 1) w *= 0.5;
        rv *= s.dt * w;
    }
    return (T)rv;
}

// Multiplier of boundary node b at level k: the sum, over every row that
// reads u^k_b, of (its coefficient) x (its multiplier):
//   own row at level k+1 (ghost: 2 - 6 c2, absorbing: r) and at level k+2
//   (ghost: -1); the interior FDM row of the inward neighbour (c2); ghost
//   rows of boundary neighbours at level k+1 (c2, or 2 c2 when b is their
//   inward neighbour); absorbing rows at level k+1 whose inward neighbour is
//   b (1/|S|) and absorbing rows of the same level k whose inward neighbour
//   is b (-r/|S|); the trace seed on z+.  The last kind comes from nodes of
//   higher codimension, whose level-k multipliers are already in Fc:
//   corners are computed first, then edges, then faces.
template <typename T>
__device__ __forceinline__ T bnd_adj(const Step<T> &s, int x, int y, int z)
{
    const Geo &g = s.g;
    const T c2 = s.c2;
    const long long cb = cidx(g, x, y, z);
    const BInfo B1 = classify(g, x, y, z, s.types1);
    const BInfo B2 = classify(g, x, y, z, s.types2);
    // Every term's operand address and weight first (a term that does not
    // apply reads the node's own entry with weight 0), then all the loads,
    // then the sum in the order of the terms: the loads are in flight
    // together instead of one dependent round trip per neighbour.
    const T *p1[6], *p0[6];
    T w1[6], w0[6];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int i = 2 * d + q, sg = 2 * q - 1;
            const int cx = x + (d == 0 ? sg : 0), cy = y + (d == 1 ? sg : 0), cz = z + (d == 2 ? sg : 0);
            const int cd = d == 0 ? cx : (d == 1 ? cy : cz);
            const int md = d == 0 ? g.nx : (d == 1 ? g.ny : g.nz);
            p1[i] = p0[i] = s.Fb + cb;
            w1[i] = w0[i] = (T)0;
            if (cd >= 0 && cd < md) {
                if (!on_bnd(g, cx, cy, cz)) {
                    p1[i] = s.Ub + gidx(g, cx, cy, cz);
                    w1[i] = c2;
                } else {
                    const long long cn = cidx(g, cx, cy, cz);
                    const BInfo N1 = classify(g, cx, cy, cz, s.types1);
                    p1[i] = s.Fb + cn;
                    if (N1.nabc == 0) w1[i] = N1.kind[d] >= 0 ? (T)2 * c2 : c2;
                    else if (N1.kind[d] == F_ABC) w1[i] = (T)1 / (T)N1.nabc;
                    if (s.level_rows) {
                        const BInfo N0 = classify(g, cx, cy, cz, s.types0);
                        if (N0.nabc > 0 && N0.kind[d] == F_ABC) {
                            p0[i] = s.Fc + cn;
                            w0[i] = s.r / (T)N0.nabc;
                        }
                    }
                }
            }
        }
    }
    const T fb = s.Fb[cb], fa = s.Fa[cb];
    T v1[6], v0[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        v1[i] = *p1[i];
        v0[i] = *p0[i];
    }
    T mu = (B1.nabc == 0 ? ((T)2 - (T)6 * c2) : s.r) * fb;
    if (B2.nabc == 0) mu -= fa;
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        mu += w1[i] * v1[i];
        mu -= w0[i] * v0[i];
    }
    if (s.res && z == g.nz - 1) mu += seed_at(s, x, y);
    return mu;
}

// Edge node number p (1..L) of edge e (0-3 along x, 4-7 along y, 8-11 along z;
// bit 0 / bit 1 of e pick the low or high side of the other two axes).
__device__ __forceinline__ void edge_node(const Geo &g, int e, int p, int &x, int &y, int &z)
{
    // plain selects: assigning the outputs in branches that depend on e
    // makes the compiler keep them in scratch memory
    const int a = e >> 2, b0 = e & 1, b1 = (e >> 1) & 1;
    x = a == 0 ? p : (b0 ? g.nx - 1 : 0);
    y = a == 1 ? p : ((a == 0 ? b0 : b1) ? g.ny - 1 : 0);
    z = a == 2 ? p : (b1 ? g.nz - 1 : 0);
}

// Corners and edges of level k.  Only the two end nodes of each edge read a
// corner of the same level: block 0 computes the 8 corners, then (after a
// barrier) the 24 end nodes; all other edge nodes are independent.
__host__ __device__ __forceinline__ int ec_blocks(const Geo &g)
{
    long long inner = 0;
    for (int n : {g.nx, g.ny, g.nz}) inner += 4 * (long long)(n - 2 > 2 ? n - 4 : 0);
    return (int)(1 + (inner + BLOCK - 1) / BLOCK);
}

template <typename T>
__device__ __forceinline__ void bnd_adj_ec_body(const Step<T> &s, int bid)
{
    const Geo &g = s.g;
    const int L[3] = {g.nx - 2, g.ny - 2, g.nz - 2};
    if (bid == 0) {
        if (threadIdx.x < 8) {
            const int t = threadIdx.x;
            const int x = (t & 1) ? g.nx - 1 : 0, y = (t & 2) ? g.ny - 1 : 0, z = (t & 4) ? g.nz - 1 : 0;
            s.Fc[cidx(g, x, y, z)] = bnd_adj(s, x, y, z);
        }
        __syncthreads();
        if (threadIdx.x < 24) {
            const int e = threadIdx.x >> 1, end = threadIdx.x & 1;
            // select, not a runtime index into the local array (which would
            // put it in scratch memory)
            const int Le = (e >> 2) == 0 ? L[0] : ((e >> 2) == 1 ? L[1] : L[2]);
            int x, y, z;
            edge_node(g, e, end ? Le : 1, x, y, z);
            const T mu = bnd_adj(s, x, y, z);
            if (!(end && Le == 1)) s.Fc[cidx(g, x, y, z)] = mu;  // a 1-node edge is written once
        }
        return;
    }
    // inner edge nodes (positions 2..L-1)
    long long t = (long long)(bid - 1) * BLOCK + threadIdx.x;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const long long m = L[a] > 2 ? L[a] - 2 : 0;
        if (t < 4 * m) {
            int x, y, z;
            edge_node(g, 4 * a + (int)(t / m), 2 + (int)(t % m), x, y, z);
            s.Fc[cidx(g, x, y, z)] = bnd_adj(s, x, y, z);
            return;
        }
        t -= 4 * m;
    }
}

template <typename T, bool ADJ, bool VM>
__device__ __forceinline__ void fem_tile(const Step<T> &s, int bid);
template <typename T>
__device__ __forceinline__ void omega_o_fill(const Step<T> &s, long long t);

// Corner and edge blocks, rounded up to a multiple of 8 so that the FEM
// blocks after them keep their XCD placement (the extra blocks do nothing).
__host__ __device__ __forceinline__ int ec_blocks8(const Geo &g) { return (ec_blocks(g) + 7) / 8 * 8; }

// First adjoint launch of a step: the corners and edges of level k (their
// blocks first: a short chain of dependent loads that the rest of the launch
// hides), and the work of level k that needs no boundary multiplier of
// level k: the FEM rows of the adjoint with the gradient integral, and the
// omega_o couplings of the FDM rows of level k, left in the level-k array for
// the interior launch to add.  Measured at 257^3 against the FEM rows in
// the face launch: adjoint step 106.2 -> 101.0 us (FP64), 94.5 -> 88.3 us
// (FP32).
template <typename T, bool VM>
__device__ __forceinline__ void bnd_adj_ecf_body(const Step<T> &s, int bid)
{
    const Geo &g = s.g;
    const int nec = ec_blocks8(g);
    if (bid < nec) {
        bnd_adj_ec_body<T>(s, bid);
        return;
    }
    bid -= nec;
    if (bid < g.n_fem_blocks) {
        fem_tile<T, true, VM>(s, bid);
        return;
    }
    const long long t = (long long)(bid - g.n_fem_blocks) * BLOCK + threadIdx.x;
    if (t < g.nwo) omega_o_fill(s, t);
}

template <typename T, bool VM>
__global__ __launch_bounds__(BLOCK) void k_bnd_adj_ecf(Step<T> s)
{
    bnd_adj_ecf_body<T, VM>(s, blockIdx.x);
}

// On a general mesh, the same launch with the omega_o couplings of its FEM
// rows in the last blocks (they need only the nu of level k+1).
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_bnd_adj_ecf_gen(Step<T> s, GenStep<T> gs, int nw)
{
    const int nb = (int)gridDim.x - nw;
    if ((int)blockIdx.x < nb) bnd_adj_ecf_body<T, false>(s, blockIdx.x);
    else gen_wo_row<T>(gs, gs.nR + (long long)((int)blockIdx.x - nb) * BLOCK + threadIdx.x);
}

// Second adjoint launch: the face-interior nodes (they read the corner and
// edge multipliers of level k).
template <typename T>
__device__ __forceinline__ void bnd_adj_face_body(const Step<T> &s, int bid)
{
    const Geo &g = s.g;
    const long long t = (long long)bid * BLOCK + threadIdx.x;
    if (t >= adj_face_rows(g, s.types1, s.types2)) return;
    int x, y, z, f;
    adj_face_node(g, s.types1, s.types2, t, x, y, z, f);
    const int d = f >> 1, dir = (f & 1) ? -1 : 1;
    const long long sd = d == 0 ? 1 : (d == 1 ? g.px : g.plane);
    const long long id = gidx(g, x, y, z), in = id + dir * sd;
    const long long cb = cidx(g, x, y, z);
    // position on the face along its two tangential axes
    const int pa = d == 0 ? y : x, pb = d == 2 ? y : z;
    const int na = d == 0 ? g.ny : g.nx, nb = d == 2 ? g.ny : g.nz;
    const T fb = s.Fb[cb];
    T mu;
    if (pa >= 2 && pa <= na - 3 && pb >= 2 && pb <= nb - 3) {
        // away from edges: the neighbours on the face are face nodes of the
        // same kind; the only other neighbour is the interior one
        const int k1 = ftype(s.types1, f), k2 = ftype(s.types2, f);
        const long long sb = d == 0 ? g.ny : g.nx;  // strides in the face array: 1 and sb
        mu = (k1 != F_ABC ? ((T)2 - (T)6 * s.c2) : s.r) * fb + s.c2 * s.Ub[in];
        if (k2 != F_ABC) mu -= s.Fa[cb];
        if (k1 != F_ABC) mu += s.c2 * ((s.Fb[cb - 1] + s.Fb[cb + 1]) + (s.Fb[cb - sb] + s.Fb[cb + sb]));
        if (s.res && f == 5) mu += seed_at(s, x, y);
    } else {
        mu = bnd_adj(s, x, y, z);
    }
    // proxy weights of face f: its level-(k+1) row reads the interior
    // neighbour with 2 c2 (ghost) or 1 (absorbing); an absorbing row of level
    // k reads it with -r (computed from the packed face conditions: a runtime
    // index into the by-value argument would force a private copy of it)
    const T w1 = ftype(s.types1, f) == F_ABC ? (T)1 : (T)2 * s.c2;
    const T w0 = (s.level_rows && ftype(s.types0, f) == F_ABC) ? -s.r : (T)0;
    s.Fc[cb] = mu;
    s.Pw[id] = (w1 * fb + w0 * mu) * s.ic2;  // what the interior stencil reads
}

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_bnd_adj_face(Step<T> s)
{
    bnd_adj_face_body<T>(s, blockIdx.x);
}

// ---------------------------------------------------------------- interior

// a of FEM-local cube (i,j,k) and kappa_e / h of the FEM-local x/y/z edge
// starting at node (i,j,k): the sum over the 4 cubes of the edge of a_c * w.
template <typename T>
__device__ __forceinline__ T acub(const Step<T> &s, int i, int j, int k)
{
    return s.acube[i + (long long)s.g.C[0] * (j + (long long)s.g.C[1] * k)];
}

template <typename T>
__device__ __forceinline__ T kappa_edge(const Step<T> &s, int d, int i, int j, int k)
{
    T kap = 0;
#pragma unroll
    for (int s1 = 0; s1 < 2; ++s1)
#pragma unroll
        for (int s0 = 0; s0 < 2; ++s0) {
            T a;
            if (d == 0) a = acub(s, i, j - s0, k - s1);
            else if (d == 1) a = acub(s, i - s0, j, k - s1);
            else a = acub(s, i - s0, j - s1, k);
            kap += a * s.w[4 * d + s0 + 2 * s1];
        }
    return kap;
}

// Adjoint only, on omega_o (the FEM boundary, FDM interior): the FEM rows
// that read the copied value V[omega_o] = U[omega_o] contribute
// c2 kappa_e lambda_V^{k+1} of the FEM node next to it.  Only face-interior
// nodes of the FEM box surface have such a neighbour.  ax: 0/1/2 for a node
// on an x/y/z face of the surface; (i,j,k) FEM-local coordinates.
template <typename T>
__device__ __forceinline__ T omega_o_term(const Step<T> &s, int ax, int i, int j, int k)
{
    const Geo &g = s.g;
    if (ax == 0) {
        const int ie = i == 0 ? 0 : g.C[0] - 1, im = i == 0 ? 1 : g.C[0] - 1;
        return s.c2 * kappa_edge(s, 0, ie, j, k) * s.Vb[fidx(g, im, j, k)];
    }
    if (ax == 1) {
        const int je = j == 0 ? 0 : g.C[1] - 1, jm = j == 0 ? 1 : g.C[1] - 1;
        return s.c2 * kappa_edge(s, 1, i, je, k) * s.Vb[fidx(g, i, jm, k)];
    }
    const int ke = k == 0 ? 0 : g.C[2] - 1, km = k == 0 ? 1 : g.C[2] - 1;
    return s.c2 * kappa_edge(s, 2, i, j, ke) * s.Vb[fidx(g, i, j, km)];
}

// Loads and stores of data touched once per launch (u^{k-1}, u^{k+1}, the
// FEM history).  With NT they carry the non-temporal hint, so that they do
// not evict the reused level-k field from the caches; the host selects NT
// when the three field levels do not fit in the last-level cache.
template <typename T, bool NT>
__device__ __forceinline__ T ld_once(const T *p)
{
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

template <typename T, bool NT>
__device__ __forceinline__ void st_once(T *p, T v)
{
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// Adjoint coupling of an FDM row on omega_o (zero elsewhere); (i, j, k) are
// FEM-local coordinates of the node.
template <typename T>
__device__ __forceinline__ T omega_o_adj(const Step<T> &s, int i, int j, int k)
{
    const Geo &g = s.g;
    const bool ii = i > 0 && i < g.C[0], jj = j > 0 && j < g.C[1], kk = k > 0 && k < g.C[2];
    if (jj && kk && (i == 0 || i == g.C[0])) return omega_o_term(s, 0, i, j, k);
    if (ii && kk && (j == 0 || j == g.C[1])) return omega_o_term(s, 1, i, j, k);
    if (ii && jj && (k == 0 || k == g.C[2])) return omega_o_term(s, 2, i, j, k);
    return (T)0;
}

// Node t of omega_o (FEM box surface, enumerated like the forward copy):
// its adjoint coupling, written to the level-k array where the FDM row of the
// node adds it (zero on the edges of the box surface).
template <typename T>
__device__ __forceinline__ void omega_o_fill(const Step<T> &s, long long t)
{
    const Geo &g = s.g;
    int i, j, k;
    box_surface(t, g.C[0], i, j, k);
    s.Uc[gidx(g, g.o[0] + i, g.o[1] + j, g.o[2] + k)] = omega_o_adj(s, i, j, k);
}

// Workgroups are dealt round-robin to the 8 XCDs, each with its own L2.
// Remap so that every XCD gets a contiguous range of tiles: neighbouring
// tiles (which read each other's rows as halo) then share an L2.
__device__ __forceinline__ int xcd_remap(int b, int nblk)
{
    const int per = (nblk + 7) / 8;
    return (b % 8) * per + b / 8;
}

// Adjoint FDM tile: the seven-point stencil of eq. (fdmschemeadjoint) on
// 64 x-lanes starting at a multiple of 64 (rows of the padded field start on
// a 128-byte line, so a wave's row access covers whole cache lines; the lane
// on the x = 0 boundary has no stencil row) by 4 thread rows of 2 grid rows each,
// streaming z over the block's chunk.  Each plane of the tile and its
// one-node halo (66 x 10 values) is loaded once from memory into one of two
// LDS buffers; the x and y neighbours are read from LDS and the z neighbours
// kept in registers, so a node costs one load of its next-plane value (plus
// its share of the halo and its old level).  Reading the x and y neighbours
// with vector loads instead (five loads per node, served by L1) measured
// 11% slower: the stencil was bound by the rate of vector memory
// instructions, not by HBM.  One barrier per plane: with two buffers a
// plane's buffer is rewritten only after every thread has passed the
// barrier that follows its last read.  Every thread of the block reaches
// every barrier; threads without a row to update still load their part.
// Rows inside the closed hole [o+2, o+C-2]^3 are skipped; in the adjoint
// (ADJ) the rows on omega_o add the coupling the boundary launch left in
// their level-k entry.
template <typename T, bool ADJ, bool NT>
__device__ __forceinline__ void fdm_tile(const Step<T> &s, int bid)
{
    static_assert(ADJ, "the forward step runs on fdm_tile_cols");
    constexpr int R = RY_FDM, TX = TX_FDM, TY = TY_FDM, LX = TX + 2, LY = TY + 2;
    constexpr bool INC = incr_form<T>();
    __shared__ T buf[2][LY][LX];
    const Geo &g = s.g;
    bid = xcd_remap(bid, g.n_fdm_blocks[ADJ]);
    if (bid >= g.n_fdm_blocks[ADJ]) return;
    const int bx = bid % g.fdm_tx[1];
    const int tt = bid / g.fdm_tx[1];
    const int by = tt % g.fdm_ty;
    const int bz = tt / g.fdm_ty;
    const int x0 = bx * TX, y0 = 1 + by * TY;
    const int z0 = 1 + bz * g.zc_fdm[ADJ];
    const int z1 = min(z0 + g.zc_fdm[ADJ], g.nz - 1);
    // the whole tile inside the closed hole: nothing to do (uniform exit)
    {
        const int xa = max(x0, 1), xb = min(x0 + TX - 1, g.nx - 2), yb = min(y0 + TY - 1, g.ny - 2);
        if (g.has_fem && xa >= g.hlo[0] && xb <= g.hhi[0] && y0 >= g.hlo[1] && yb <= g.hhi[1] &&
            z0 >= g.hlo[2] && z1 - 1 <= g.hhi[2])
            return;
    }
    const int lx = (int)(threadIdx.x % TX), ty = (int)(threadIdx.x / TX);
    const int x = x0 + lx, y = y0 + R * ty;
    const long long py = g.px, pz = g.plane;
    const T c2 = s.c2;
    const T *__restrict__ Ub = s.Ub;
    const T *__restrict__ Ua = INC ? s.Da : s.Ua;
    T *__restrict__ Uc = s.Uc;
    T *__restrict__ Dc = s.Dc;
    const bool xval = x <= g.nx - 1;                 // a grid node (loads)
    const bool xcmp = x >= 1 && x <= g.nx - 2;       // an interior column (updates)
    // halo columns: wave 1, lanes 0..LY-1 the left one, LY..2LY-1 the right one
    const bool hcol = ty == 1 && lx < 2 * LY;
    const int hly = lx < LY ? lx : lx - LY;          // halo row in the tile
    const int hx = lx < LY ? x0 - 1 : x0 + TX, hy = y0 - 1 + hly;
    const bool hval = hcol && hx >= 0 && hx <= g.nx - 1 && hy <= g.ny - 1;
    // halo rows: wave 0 the row below the tile, the last wave the row above
    const int nw = TY / R;
    const bool hrow = (ty == 0 || ty == nw - 1) && xval;
    const int hry = ty == 0 ? y0 - 1 : y0 + TY;
    const bool hrval = hrow && hry <= g.ny - 1;
    // rows of this thread: present (a grid row), updated (interior, not in the hole)
    bool rval[R], rcmp[R], side[R], top[R];
    const int i = x - g.o[0], C0 = g.C[0], C1 = g.C[1], C2 = g.C[2];
    const bool ib = ADJ && g.has_fem && i >= 0 && i <= C0, ii = i > 0 && i < C0;
    const bool xin = g.has_fem && x >= g.hlo[0] && x <= g.hhi[0];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int yr = y + r, j = yr - g.o[1];
        rval[r] = xval && yr <= g.ny - 1;
        rcmp[r] = xcmp && yr <= g.ny - 2;
        side[r] = ib && j >= 0 && j <= C1 && !(ii && j > 0 && j < C1);
        top[r] = ib && ii && j > 0 && j < C1;
    }
    // rows inside the hole's x-y range skip the planes of the hole
    unsigned hmask = 0;
#pragma unroll
    for (int r = 0; r < R; ++r)
        if (xin && y + r >= g.hlo[1] && y + r <= g.hhi[1]) hmask |= 1u << r;
    // Absorbing x faces of the adjoint, away from the face's edges (rows y
    // in [2, ny-3] of planes z in [2, nz-3]; the face launch takes the
    // ring next to the edges, which reads the edge multipliers of the same
    // level, the rows of reflecting x faces and those of x = nx-1 when that
    // column is the last tile's halo, see x_face_in_tile): the face node's
    // multiplier is kept in the grid array itself, so the staged plane holds
    // mu^{k+1} of the face node beside its inward neighbour's.  The face
    // node's lane writes mu^k = r mu^{k+1} + c2 mu^{k+1}_in with the row's
    // store, and the inward neighbour's stencil reads the face row's proxy
    // (mu^{k+1} + w0 mu^k) / c2 in its place, w0 = -r when level k has
    // rows and the face absorbed in step k-1.  In the face launch these rows
    // read and wrote one value per 128-byte line.
    const bool xq0 = ADJ && x0 == 0 && x_face_in_tile(g, s.types1, s.types2, 0);                        // uniform
    const bool xq1 = ADJ && x0 <= g.nx - 2 && g.nx - 1 <= x0 + TX - 1 && x_face_in_tile(g, s.types1, s.types2, 1);
    const T xw0 = (ADJ && s.level_rows) ? -s.r : (T)0;  // the x faces absorb in every step here
    unsigned xfy = 0;  // rows y + r in [2, ny-3]
#pragma unroll
    for (int r = 0; r < R; ++r)
        if (y + r >= 2 && y + r <= g.ny - 3) xfy |= 1u << r;
    // prologue: plane z0 into buffer 0, plane z0-1 of the own rows in registers
    T cm[R], c0[R];
    long long id = gidx(g, min(x, g.nx - 1), y, z0);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        c0[r] = rval[r] ? Ub[id + r * py] : (T)0;
        cm[r] = rval[r] ? Ub[id + r * py - pz] : (T)0;
        buf[0][1 + R * ty + r][1 + lx] = c0[r];
    }
    if (hval) buf[0][hly][lx < LY ? 0 : LX - 1] = Ub[gidx(g, hx, hy, z0)];
    if (hrval) buf[0][ty == 0 ? 0 : LY - 1][1 + lx] = Ub[gidx(g, x, hry, z0)];
    __syncthreads();
    int cur = 0;
    for (int z = z0; z < z1; ++z, id += pz) {
        const int nxt = cur ^ 1;
        // loads: the next plane (own rows, halo), the old level of this plane
        T cp[R], ua[R], w[R];
        bool dor[R];
        const bool inh = z >= g.hlo[2] && z <= g.hhi[2];
        const bool xfz = ADJ && z >= 2 && z <= g.nz - 3;  // plane of absorbing x-face rows (see xq0)
        const int kz = z - g.o[2];
        const bool zs = kz >= 0 && kz <= C2, zt = kz == 0 || kz == C2;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const long long ir = id + r * py;
            cp[r] = rval[r] ? Ub[ir + pz] : (T)0;
            dor[r] = rcmp[r] && !(((hmask >> r) & 1u) && inh);
            ua[r] = dor[r] ? ld_once<T, NT>(Ua + ir) : (T)0;
            w[r] = (ADJ && dor[r] && ((side[r] && zs) || (top[r] && zt))) ? Uc[ir] : (T)0;
        }
        const T hv = hval ? Ub[gidx(g, hx, hy, z + 1)] : (T)0;
        const T hr = hrval ? Ub[gidx(g, x, hry, z + 1)] : (T)0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const long long ir = id + r * py;
            const int ly = 1 + R * ty + r;
            const T xp = buf[cur][ly][lx + 2];
            const bool xfr = xfz && ((xfy >> r) & 1u);  // an absorbing x-face row at this (y, z)
            T d = (T)0, v = (T)0;
            if (dor[r]) {
                T xm = buf[cur][ly][lx], xpr = xp;
                if constexpr (ADJ) {
                    // the face row's proxy in place of the face node's mu^{k+1}
                    if (xq0 && x == 1 && xfr) xm = (xm + xw0 * (s.r * xm + c2 * c0[r])) * s.ic2;
                    if (xq1 && x == g.nx - 2 && xfr) xpr = (xp + xw0 * (s.r * xp + c2 * c0[r])) * s.ic2;
                }
                const T ym = buf[cur][ly - 1][1 + lx], yp = buf[cur][ly + 1][1 + lx];
                // FP32 (increment form): the Laplacian as a sum of neighbour
                // differences, each exact in FP32 while the neighbours are
                // within a factor 2 of the node (Sterbenz), so a smooth field
                // does not lose its second difference to cancellation.  With
                // the sum-then-subtract form a plane wave on a 512-cell axis
                // over 2500 steps kept 1.5e-5 trace error, with this one
                // 4.6e-7 (FP64 reference, x-y uniform field).
                T L;
                if constexpr (INC)
                    L = ((xm - c0[r]) + (xpr - c0[r])) + ((ym - c0[r]) + (yp - c0[r])) +
                        ((cm[r] - c0[r]) + (cp[r] - c0[r]));
                else
                    L = ((xm + xpr) + (ym + yp)) + (cm[r] + cp[r]) - (T)6 * c0[r];
                if constexpr (INC) {
                    d = ua[r] + c2 * L + w[r];
                    v = c0[r] + d;
                } else {
                    v = (T)2 * c0[r] - ua[r] + c2 * L + w[r];
                }
            }
            bool st = dor[r];
            {
                // mu^k of the face node into the grid array (see xq0), with
                // the row's own store (the increment array gets 0 there, which
                // no row reads)
                if (xq0 && x == 0 && xfr) {
                    v = s.r * c0[r] + c2 * xp;
                    st = true;
                }
                if (xq1 && xfr && x == g.nx - 1) {
                    v = s.r * c0[r] + c2 * buf[cur][ly][lx];
                    st = true;
                }
            }
            if (st) {
                if constexpr (INC) st_once<T, NT>(Dc + ir, d);
                st_once<T, NT>(Uc + ir, v);
            }
        }
        // the next plane into the other buffer
#pragma unroll
        for (int r = 0; r < R; ++r) buf[nxt][1 + R * ty + r][1 + lx] = cp[r];
        if (hval) buf[nxt][hly][lx < LY ? 0 : LX - 1] = hv;
        if (hrval) buf[nxt][ty == 0 ? 0 : LY - 1][1 + lx] = hr;
        __syncthreads();
#pragma unroll
        for (int r = 0; r < R; ++r) {
            cm[r] = c0[r];
            c0[r] = cp[r];
        }
        cur = nxt;
    }
}

// W neighbouring x columns of one lane, moved by one 16-byte access (FP64
// pairs, FP32 quads) instead of W.
template <typename T, int W> struct ColsV {
    typedef T type __attribute__((ext_vector_type(W)));
};

template <typename T, int W, bool NT>
__device__ __forceinline__ typename ColsV<T, W>::type ld_cols(const T *p)
{
    using P = typename ColsV<T, W>::type;
    if constexpr (NT) return __builtin_nontemporal_load(reinterpret_cast<const P *>(p));
    else return *reinterpret_cast<const P *>(p);
}

template <typename T, int W, bool NT>
__device__ __forceinline__ void st_cols(T *p, typename ColsV<T, W>::type v)
{
    using P = typename ColsV<T, W>::type;
    if constexpr (NT) __builtin_nontemporal_store(v, reinterpret_cast<P *>(p));
    else *reinterpret_cast<P *>(p) = v;
}

// Values a[0..W) stored at p: one vector store when every column has a row
// (ok), else one store per column that has.
template <typename T, int W, bool NT>
__device__ __forceinline__ void st_cols_masked(T *p, const T a[W], const bool ok[W])
{
    using P = typename ColsV<T, W>::type;
    bool all = true;
#pragma unroll
    for (int e = 0; e < W; ++e) all = all && ok[e];
    if (all) {
        P v;
#pragma unroll
        for (int e = 0; e < W; ++e) v[e] = a[e];
        st_cols<T, W, NT>(p, v);
    } else {
#pragma unroll
        for (int e = 0; e < W; ++e)
            if (ok[e]) st_once<T, NT>(p + e, a[e]);
    }
}

// Absorbing face rows, eq. (eq:abs2), beside W interior rows:
// u^{k+1}_b = u^k_in + r (u^k_b - u^{k+1}_in) for the columns with a row
// (ok), stored at `at` (the face node of the first column), with the
// increment in FP32 and the trace when obs is given.
template <typename T, int W, bool NT>
__device__ __forceinline__ void face_cols(T *Uc, T *Dc, long long at, const T ub[W], const T uin[W], const T vin[W],
                                          const bool ok[W], double *obs, T r)
{
    T vf[W], df[W];
#pragma unroll
    for (int e = 0; e < W; ++e) {
        vf[e] = uin[e] + r * (ub[e] - vin[e]);
        df[e] = vf[e] - ub[e];
        if (obs && ok[e]) obs[e] = (double)vf[e];
    }
    if constexpr (incr_form<T>()) st_cols_masked<T, W, NT>(Dc + at, df, ok);
    st_cols_masked<T, W, NT>(Uc + at, vf, ok);
}

// Columns per lane of the forward FDM tile: 16 bytes.
template <typename T>
constexpr int fwd_cols() { return 16 / (int)sizeof(T); }

// Forward FDM tile with W columns per lane: a block of 8 thread rows of 32
// lanes covers 8 grid rows of 32 W columns (fwd_tile_x(sizeof(T)), a 64 x 8 tile
// in FP64 and 128 x 8 in FP32), streaming along z through the chunk of
// zc_fdm[0] planes, each plane staged in LDS; the FEM hole is skipped (the
// tile when it lies inside, else the rows).  Every field access of the z
// loop moves W values per lane.  Rows start on 128-byte lines, so the W
// columns at a lane's x (a multiple of W) stay inside its row; values past
// nx - 1 are padding, never stored, and enter only rows that are not
// computed (a column's row reads its own column and its x neighbours, and
// the right neighbour of a computed row, x <= nx-2, is a grid node), so
// they are used as loaded: a masking select right after a load would make
// the wave wait for it before issuing the next one.  LDS rows hold the
// tile's columns at offset W (16-byte aligned), the left halo column at
// W - 1 and the right one at TX + W.  The tile also takes the rows of the
// absorbing faces next to its rows (x faces in the lane of the inward
// neighbour; y and z faces by the row beside them) and the trace on an
// absorbing z+ face.
template <typename T, bool NT, int W>
__device__ __forceinline__ void fdm_tile_cols(const Step<T> &s, int bid)
{
    using P = typename ColsV<T, W>::type;
    constexpr int HL = 32, TX = HL * W, TY = BLOCK / HL, LX = TX + 2 * W, LY = TY + 2;
    static_assert(TX == fwd_tile_x(sizeof(T)) && TY == TY_FDM, "forward tile shape");
    constexpr bool INC = incr_form<T>();
    __shared__ __align__(16) T buf[2][LY][LX];
    const Geo &g = s.g;
    bid = xcd_remap(bid, g.n_fdm_blocks[0]);
    if (bid >= g.n_fdm_blocks[0]) return;
    const int bx = bid % g.fdm_tx[0];
    const int tt = bid / g.fdm_tx[0];
    const int by = tt % g.fdm_ty;
    const int bz = tt / g.fdm_ty;
    const int x0 = bx * TX, y0 = 1 + by * TY;
    const int z0 = 1 + bz * g.zc_fdm[0];
    const int z1 = min(z0 + g.zc_fdm[0], g.nz - 1);
    {
        const int xa = max(x0, 1), xb = min(x0 + TX - 1, g.nx - 2), yb = min(y0 + TY - 1, g.ny - 2);
        if (g.has_fem && xa >= g.hlo[0] && xb <= g.hhi[0] && y0 >= g.hlo[1] && yb <= g.hhi[1] &&
            z0 >= g.hlo[2] && z1 - 1 <= g.hhi[2])
            return;
    }
    const int lx = (int)(threadIdx.x % HL), ty = (int)(threadIdx.x / HL);
    const int x = x0 + W * lx, y = y0 + ty, ly = 1 + ty, lc = W + W * lx;
    const long long pz = g.plane;
    const T c2 = s.c2;
    const T *__restrict__ Ub = s.Ub;
    const T *__restrict__ Ua = INC ? s.Da : s.Ua;
    T *__restrict__ Uc = s.Uc;
    T *__restrict__ Dc = s.Dc;
    const bool rval = x <= g.nx - 1 && y <= g.ny - 1;  // column loads of this row
    // halo columns: lanes 0..2LY-1 of thread row 2 (the second wave)
    const bool hcol = ty == 2 && lx < 2 * LY;
    const int hly = lx < LY ? lx : lx - LY;
    const int hx = lx < LY ? x0 - 1 : x0 + TX, hy = y0 - 1 + hly;
    const bool hval = hcol && hx >= 0 && hx <= g.nx - 1 && hy <= g.ny - 1;
    const int hcl = lx < LY ? W - 1 : TX + W;
    // halo rows: thread row 0 the row below the tile, the last the row above
    const bool hrow = (ty == 0 || ty == TY - 1) && x <= g.nx - 1;
    const int hry = ty == 0 ? y0 - 1 : y0 + TY, hrl = ty == 0 ? 0 : LY - 1;
    const bool hrval = hrow && hry <= g.ny - 1;
    const bool yin = y >= g.hlo[1] && y <= g.hhi[1];
    bool rcmp[W], hole[W], fx1[W];
    const bool a0 = ftype(s.types1, 0) == F_ABC, a1 = ftype(s.types1, 1) == F_ABC;
#pragma unroll
    for (int e = 0; e < W; ++e) {
        const int xe = x + e;
        rcmp[e] = xe >= 1 && xe <= g.nx - 2 && y <= g.ny - 2;
        hole[e] = g.has_fem && xe >= g.hlo[0] && xe <= g.hhi[0] && yin;
        fx1[e] = a1 && xe == g.nx - 2 && rcmp[e];
    }
    // absorbing x faces: the x = 0 row takes the new value of x = 1 from the
    // same lane; the row of x = nx-1 joins the lane's store when nx-2 is not
    // its last column, else it is a store of its own
    const bool fx0 = a0 && x == 0 && y <= g.ny - 2;
    // absorbing y and z faces: the row of a node next to the face has the
    // face node's old value (staged row, or the z neighbour in registers) and
    // its own old and new values, so it adds the face row, eq. (eq:abs2),
    // with a store of its own (rows y = 1 and y = ny-2, planes z = 1 and
    // z = nz-2; the trace takes the z+ face)
    const bool fy0 = y == 1 && ftype(s.types1, 2) == F_ABC;
    const bool fy1 = y == g.ny - 2 && ftype(s.types1, 3) == F_ABC;
    const bool az0 = ftype(s.types1, 4) == F_ABC, az1 = ftype(s.types1, 5) == F_ABC;
    // prologue: plane z0 into buffer 0, plane z0-1 of the own columns in registers
    long long id = gidx(g, min(x, g.nx - 1), y, z0);
    P c0 = (T)0, cm = (T)0;
    if (rval) {
        c0 = ld_cols<T, W, false>(Ub + id);
        cm = ld_cols<T, W, false>(Ub + id - pz);
    }
    *reinterpret_cast<P *>(&buf[0][ly][lc]) = c0;
    if (hval) buf[0][hly][hcl] = Ub[gidx(g, hx, hy, z0)];
    if (hrow) {
        P hr = (T)0;
        if (hrval) hr = ld_cols<T, W, false>(Ub + gidx(g, x, hry, z0));
        *reinterpret_cast<P *>(&buf[0][hrl][lc]) = hr;
    }
    __syncthreads();
    int cur = 0;
    for (int z = z0; z < z1; ++z, id += pz) {
        const int nxt = cur ^ 1;
        const bool inh = z >= g.hlo[2] && z <= g.hhi[2];
        bool dor[W], any = false;
#pragma unroll
        for (int e = 0; e < W; ++e) {
            dor[e] = rcmp[e] && !(hole[e] && inh);
            any = any || dor[e];
        }
        P cp = (T)0, ua = (T)0;
        if (rval) cp = ld_cols<T, W, false>(Ub + id + pz);
        if (any) ua = ld_cols<T, W, NT>(Ua + id);
        const T hv = hval ? Ub[gidx(g, hx, hy, z + 1)] : (T)0;
        P hr = (T)0;
        if (hrval) hr = ld_cols<T, W, false>(Ub + gidx(g, x, hry, z + 1));
        const P ym = *reinterpret_cast<const P *>(&buf[cur][ly - 1][lc]);
        const P yp = *reinterpret_cast<const P *>(&buf[cur][ly + 1][lc]);
        const T xl = buf[cur][ly][lc - 1], xr = buf[cur][ly][lc + W];
        T cc[W], cmv[W], cpv[W], ymv[W], ypv[W], d[W], v[W];
        bool st[W];
#pragma unroll
        for (int e = 0; e < W; ++e) {
            cc[e] = c0[e]; cmv[e] = cm[e]; cpv[e] = cp[e]; ymv[e] = ym[e]; ypv[e] = yp[e];
            d[e] = v[e] = (T)0;
        }
#pragma unroll
        for (int e = 0; e < W; ++e) {
            st[e] = dor[e];
            if (!dor[e]) continue;
            // the old x neighbours of the column
            const T xm = e == 0 ? xl : cc[e - 1], xpr = e == W - 1 ? xr : cc[e + 1];
            T L;
            if constexpr (INC)
                L = ((xm - cc[e]) + (xpr - cc[e])) + ((ymv[e] - cc[e]) + (ypv[e] - cc[e])) +
                    ((cmv[e] - cc[e]) + (cpv[e] - cc[e]));
            else
                L = ((xm + xpr) + (ymv[e] + ypv[e])) + (cmv[e] + cpv[e]) - (T)6 * cc[e];
            if constexpr (INC) {
                d[e] = ua[e] + c2 * L;
                v[e] = cc[e] + d[e];
            } else {
                v[e] = (T)2 * cc[e] - ua[e] + c2 * L;
            }
        }
        // face rows next to this row (see fy0)
        if (fy0) face_cols<T, W, NT>(Uc, Dc, id - g.px, ymv, cc, v, dor, nullptr, s.r);
        if (fy1) face_cols<T, W, NT>(Uc, Dc, id + g.px, ypv, cc, v, dor, nullptr, s.r);
        if (az0 && z == 1) face_cols<T, W, NT>(Uc, Dc, id - pz, cmv, cc, v, dor, nullptr, s.r);
        if (az1 && z == g.nz - 2)
            face_cols<T, W, NT>(Uc, Dc, id + pz, cpv, cc, v, dor, s.obs ? s.obs + x + (long long)g.nx * y : nullptr,
                                s.r);
        if (fx0) {
            v[0] = cc[1] + s.r * (cc[0] - v[1]);
            if constexpr (INC) d[0] = v[0] - cc[0];
            st[0] = true;
        }
#pragma unroll
        for (int e = 0; e + 1 < W; ++e)
            if (fx1[e]) {  // x = nx-2 is column e: the face is column e+1
                v[e + 1] = cc[e] + s.r * (cc[e + 1] - v[e]);
                if constexpr (INC) d[e + 1] = v[e + 1] - cc[e + 1];
                st[e + 1] = true;
            }
        if (fx1[W - 1]) {
            const T vf = cc[W - 1] + s.r * (xr - v[W - 1]);
            if constexpr (INC) st_once<T, NT>(Dc + id + W, vf - xr);
            st_once<T, NT>(Uc + id + W, vf);
        }
        if constexpr (INC) st_cols_masked<T, W, NT>(Dc + id, d, st);
        st_cols_masked<T, W, NT>(Uc + id, v, st);
        // the next plane into the other buffer
        *reinterpret_cast<P *>(&buf[nxt][ly][lc]) = cp;
        if (hval) buf[nxt][hly][hcl] = hv;
        if (hrow) *reinterpret_cast<P *>(&buf[nxt][hrl][lc]) = hr;
        __syncthreads();
        cm = c0;
        c0 = cp;
        cur = nxt;
    }
}

// FEM rows of one tile (forward, or with ADJ the adjoint rows and the
// gradient integral).  Variable wave speed: the forward row divides by its
// own lumped mass (s.minv = 1/m per node, h^3 units; uniform when null); the
// adjoint rows (VM) apply the transposed stencil to nu = minv * mu, pair nu
// with u^k in the conductivity gradient, and accumulate dJ/dm per node.
template <typename T, bool ADJ, bool VM>
__device__ __forceinline__ void fem_tile(const Step<T> &s, int bid)
{
    const Geo &g = s.g;
    const int Cx = g.C[0], Cy = g.C[1], Cz = g.C[2];
    // contiguous tile ranges per XCD, as for the FDM tiles
    bid = xcd_remap(bid, g.n_fem_blocks);
    if (bid >= g.n_fem_tiles) return;
    const int bx = bid % g.fem_tiles[0];
    const int t = bid / g.fem_tiles[0];
    const int by = t % g.fem_tiles[1];
    const int bz = t / g.fem_tiles[1];
    const int i = 1 + bx * TX_FEM + (int)(threadIdx.x % TX_FEM);
    const int j = 1 + by * TY_FEM + (int)(threadIdx.x / TX_FEM);
    if (i > Cx - 1 || j > Cy - 1) return;
    const int k0 = 1 + bz * g.zc_fem;
    const int k1 = min(k0 + g.zc_fem, Cz);
    const long long cpy = Cx, cpz = (long long)Cx * Cy;
    const long long cb = (i - 1) + (long long)(j - 1) * cpy;
    const T *A = s.acube;
    // a of the 8 cubes around the node: index dx + 2 dy, lo = dz 0, hi = dz 1
    T alo[4], ahi[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) alo[q] = A[cb + (q & 1) + (q >> 1) * cpy + (long long)(k0 - 1) * cpz];
    const T *w = s.w;
    const T c2 = s.c2;
    const long long fy = g.fpx, fz = g.fplane;
    long long id = fidx(g, i, j, k0);
    // Forward: the neighbours on omega_o (the box surface, FDM rows) are read
    // from the grid level, which holds them (Algorithm 2 step 4 makes the
    // FEM copy equal to it); the adjoint multipliers of the FEM level are 0
    // there.  gq: grid index of the node.
    const T *__restrict__ Gb = s.Ub;
    long long gq = gidx(g, g.o[0] + i, g.o[1] + j, g.o[2] + k0);
    const bool sxm = !ADJ && i == 1, sxp = !ADJ && i == Cx - 1, sym = !ADJ && j == 1, syp = !ADJ && j == Cy - 1;
    T vm = (!ADJ && k0 == 1) ? Gb[gq - g.plane] : s.Vb[id - fz], v0 = s.Vb[id];
    constexpr bool AV = ADJ && VM;
    const T *__restrict__ Mi = s.minv;
    T mm = 1, m0 = 1;  // minv of the planes k-1, k (AV)
    if constexpr (AV) {
        mm = Mi[id - fz];
        m0 = Mi[id];
    }
    // adjoint gradient: multipliers and history on the 4 corners (x,y)+{0,1}
    const bool gcol = ADJ && i >= 2 && i <= Cx - 3 && j >= 2 && j <= Cy - 3;
    const bool hcol = i >= 2 && i <= Cx - 2 && j >= 2 && j <= Cy - 2;
    const int hn0 = g.hn[0], hn1 = g.hn[1];
    const long long hpz = (long long)hn0 * hn1;
    double ql[4] = {0, 0, 0, 0}, hl[4] = {0, 0, 0, 0};  // plane k of the gradient corners
    for (int k = k0; k < k1; ++k, id += fz, gq += g.plane) {
#pragma unroll
        for (int q = 0; q < 4; ++q) ahi[q] = A[cb + (q & 1) + (q >> 1) * cpy + (long long)k * cpz];
        const T vp = (!ADJ && k + 1 == Cz) ? Gb[gq + g.plane] : s.Vb[id + fz];
        const T xm = sxm ? Gb[gq - 1] : s.Vb[id - 1], xp = sxp ? Gb[gq + 1] : s.Vb[id + 1];
        const T ym = sym ? Gb[gq - g.px] : s.Vb[id - fy], yp = syp ? Gb[gq + g.px] : s.Vb[id + fy];
        // operand of the stencil: the level itself, or nu = minv * mu (AV)
        T mp = 1, nxm = xm, nxp = xp, nym = ym, nyp = yp;
        if constexpr (AV) {
            mp = Mi[id + fz];
            nxm = Mi[id - 1] * xm;
            nxp = Mi[id + 1] * xp;
            nym = Mi[id - fy] * ym;
            nyp = Mi[id + fy] * yp;
        }
        const T n0 = AV ? m0 * v0 : v0, nzm = AV ? mm * vm : vm, nzp = AV ? mp * vp : vp;
        if constexpr (ADJ) {
            // gradient of eq. (gradient1): cube with lower corner (i,j,k),
            // sum over its 12 edges of w_e (D_e lambda^{k+1}) (D_e u^k) in
            // FP64.  The corners of plane k come from the previous
            // iteration's plane k+1 (register queue), so each plane's
            // multipliers and history values are loaded once per column.
            // Every thread runs it on every plane, with history addresses
            // clamped into the history box and weight 0 where the cube has
            // no gradient (gcol, k in [2, Cz-3]; it then adds an exact zero to
            // its own cube, which no other thread touches), so these loads
            // are issued with the stencil's instead of after them.  Plain
            // loads for the history: the four columns around a corner re-read
            // it from L2.
            const bool gq = gcol && k >= 2 && k <= Cz - 3;
            const T *H = s.hist;
            const int hi0 = min(max(i - 2, 0), hn0 - 2), hj0 = min(max(j - 2, 0), hn1 - 2);
            const long long hcol0 = hi0 + (long long)hj0 * hn0;
            const int hn2 = Cz - 3;
            const long long hk = min(max(k - 2, 0), hn2 - 1), hk1 = min(max(k - 1, 0), hn2 - 1);
            if (k == k0) {
                ql[0] = (double)n0;
                ql[1] = (double)nxp;
                ql[2] = (double)nyp;
                ql[3] = AV ? (double)(Mi[id + 1 + fy] * s.Vb[id + 1 + fy]) : (double)s.Vb[id + 1 + fy];
#pragma unroll
                for (int c = 0; c < 4; ++c) hl[c] = (double)H[hcol0 + hk * hpz + (c & 1) + (c >> 1) * hn0];
            }
            double q[8], hv[8], qh[4], hh[4];
            qh[0] = (double)nzp;
            if constexpr (AV) {
                qh[1] = (double)(Mi[id + fz + 1] * s.Vb[id + fz + 1]);
                qh[2] = (double)(Mi[id + fz + fy] * s.Vb[id + fz + fy]);
                qh[3] = (double)(Mi[id + fz + fy + 1] * s.Vb[id + fz + fy + 1]);
            } else {
                qh[1] = (double)s.Vb[id + fz + 1];
                qh[2] = (double)s.Vb[id + fz + fy];
                qh[3] = (double)s.Vb[id + fz + fy + 1];
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) hh[c] = (double)H[hcol0 + hk1 * hpz + (c & 1) + (c >> 1) * hn0];
            double *gp = s.G + (i + cpy * j + cpz * k);
            const double gv = *gp;
            // corner c = dx + 2 dy + 4 dz
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                q[c] = ql[c];
                q[c + 4] = qh[c];
                hv[c] = hl[c];
                hv[c + 4] = hh[c];
                ql[c] = qh[c];
                hl[c] = hh[c];
            }
            double acc = 0.0;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int s0 = e & 1, s1 = e >> 1;
                const int ax0 = 0 + 2 * s0 + 4 * s1, ax1 = ax0 + 1;          // x-edge (y=s0,z=s1)
                const int ay0 = s0 + 4 * s1, ay1 = ay0 + 2;                  // y-edge (x=s0,z=s1)
                const int az0 = s0 + 2 * s1, az1 = az0 + 4;                  // z-edge (x=s0,y=s1)
                acc += (double)w[e] * (q[ax1] - q[ax0]) * (hv[ax1] - hv[ax0]);
                acc += (double)w[4 + e] * (q[ay1] - q[ay0]) * (hv[ay1] - hv[ay0]);
                acc += (double)w[8 + e] * (q[az1] - q[az0]) * (hv[az1] - hv[az0]);
            }
            *gp = __builtin_fma(gq ? s.w2 : 0.0, acc, gv);
        }
        // a(dx,dy,dz): dz = 0 -> alo, 1 -> ahi
#define AC(dx, dy, dz) ((dz) ? ahi[(dx) + 2 * (dy)] : alo[(dx) + 2 * (dy)])
        const T kxp = w[0] * AC(1, 1, 1) + w[1] * AC(1, 0, 1) + w[2] * AC(1, 1, 0) + w[3] * AC(1, 0, 0);
        const T kxm = w[0] * AC(0, 1, 1) + w[1] * AC(0, 0, 1) + w[2] * AC(0, 1, 0) + w[3] * AC(0, 0, 0);
        const T kyp = w[4] * AC(1, 1, 1) + w[5] * AC(0, 1, 1) + w[6] * AC(1, 1, 0) + w[7] * AC(0, 1, 0);
        const T kym = w[4] * AC(1, 0, 1) + w[5] * AC(0, 0, 1) + w[6] * AC(1, 0, 0) + w[7] * AC(0, 0, 0);
        const T kzp = w[8] * AC(1, 1, 1) + w[9] * AC(0, 1, 1) + w[10] * AC(1, 0, 1) + w[11] * AC(0, 0, 1);
        const T kzm = w[8] * AC(1, 1, 0) + w[9] * AC(0, 1, 0) + w[10] * AC(1, 0, 0) + w[11] * AC(0, 0, 0);
#undef AC
        const T Ku = kxp * (n0 - nxp) + kxm * (n0 - nxm) + kyp * (n0 - nyp) + kym * (n0 - nym) +
                     kzp * (n0 - nzp) + kzm * (n0 - nzm);
        // leapfrog part: v = 2 v0 - v_prev - c2 Ku, or in increment form
        // dv = dv_prev - c2 Ku (v = v0 + dv once the couplings are in dv);
        // a forward row with variable mass scales c2 by its own minv
        T cm = c2;
        if constexpr (!ADJ)
            if (Mi) cm = c2 * Mi[id];
        T dv = 0, v = 0;
        if constexpr (incr_form<T>()) dv = s.VDa[id] - cm * Ku;
        else v = (T)2 * v0 - s.Va[id] - cm * Ku;
        const bool hin = hcol && k >= 2 && k <= Cz - 2;
        if constexpr (ADJ) {
            // omega_diamond: the FDM rows around read the copied value
            if (hin && (i == 2 || i == Cx - 2 || j == 2 || j == Cy - 2 || k == 2 || k == Cz - 2)) {
                const long long gg = gidx(g, g.o[0] + i, g.o[1] + j, g.o[2] + k);
                const T cw = c2 * (((s.Ub[gg - 1] + s.Ub[gg + 1]) + (s.Ub[gg - g.px] + s.Ub[gg + g.px])) +
                                   (s.Ub[gg - g.plane] + s.Ub[gg + g.plane]));
                if constexpr (incr_form<T>()) dv += cw;
                else v += cw;
            }
            // wave speed: row n reads u^{k+1}_n = ... - c2 (K u^k)_n / m_n, so
            // d u^{k+1}_n / d m_n = -(u^{k+1} - 2 u^k + u^{k-1})_n / m_n and
            // dJ/dm_n gains mu_n^{k+1} times that (FP64); the history levels
            // k+1, k, k-1 of the node give the second difference
            if constexpr (AV)
                if (hin && s.Gm && s.hnext) {
                    const long long hb0 = (i - 2) + (long long)(j - 2) * hn0 + (long long)(k - 2) * hpz;
                    const double d2 = ((double)s.hnext[hb0] - 2.0 * (double)s.hist[hb0]) + (double)s.hprev[hb0];
                    s.Gm[id] -= (double)v0 * d2 * (double)m0;
                }
        }
        if constexpr (incr_form<T>()) {
            s.VDc[id] = dv;
            v = v0 + dv;
        }
        // Algorithm 2 step 3: the new FEM values on omega_diamond (surface of
        // the inner box) into the grid level
        if constexpr (!ADJ)
            if (hin && (i == 2 || i == Cx - 2 || j == 2 || j == Cy - 2 || k == 2 || k == Cz - 2))
                s.Uc[gidx(g, g.o[0] + i, g.o[1] + j, g.o[2] + k)] = v;
        if constexpr (!ADJ)
            if (hin && s.hist)
                st_once<T, true>(s.hist + (i - 2) + (long long)(j - 2) * hn0 + (long long)(k - 2) * hpz, v);
        s.Vc[id] = v;
        vm = v0;
        v0 = vp;
        if constexpr (AV) {
            mm = m0;
            m0 = mp;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) alo[q] = ahi[q];
    }
}

// Block order of the interior launch: in the forward sweep the previous
// step's edge and corner rows (when given), then the rows of a general FEM
// mesh (when given, in both sweeps), then the FDM tiles, then the FEM tiles
// of the structured box; each range is rounded up to a multiple of 8 for the
// XCD remap.  The structured FEM rows of the adjoint run in the boundary
// launch.
//
// Occupancy bounds: the FP32 adjoint at most 64 VGPRs (8 waves per SIMD);
// the forward kernels unbounded (FP64 79 VGPRs, set by the FEM tile; FP32
// 100, set by the four-column tile, which bounded to 6 waves spills 16 VGPRs
// and measured 83.4 against 69.7 us per step at 257^3; FP64 bounded to 7
// waves spills 2 in the FEM tile, 78.2 against 75.8 us); the FP64 adjoint
// unbounded (56 VGPRs).
template <typename T, bool ADJ>
constexpr int interior_waves() { return sizeof(T) == 4 ? (ADJ ? 8 : 1) : 1; }

// Forward FDM tiles take 16 bytes of columns per lane (fdm_tile_cols),
// adjoint tiles one column per lane (fdm_tile).  Per step at 257^3, pairs
// against single columns (same run, same box, before the forward tile took
// the y and z faces): FP64 forward 85.3 / 86.7 us, adjoint 101.1 / 97.4 us;
// FP32 forward 77.1 / 76.4 us, adjoint 86.0 / 81.5 us.  With the face rows in
// the tile and the edge rows one launch later, the forward step over 1200
// steps went from 85.3 to 83.1 us (FP64) and from 75.9 to 74.9 us (FP32): the
// interior launch grew by ~4 us, the boundary launch (9 us, the latency of
// the edge rows) is gone while every face absorbs.

// Blocks of the interior launch (kernels k_interior and, on a general FEM
// mesh, k_interior_gen); with GEN, gs and ngb give the mesh's FEM rows in ngb
// blocks (forward: the rows of step k; adjoint: the rows of level k, which
// read only levels k+1 and k+2, as the grid tiles do).
template <typename T, bool ADJ, bool NT, bool GEN>
__device__ __forceinline__ void interior_block(const Step<T> &s, const EdgeArgs<T> &ea, int ne,
                                               const GenStep<T> &gs, int ngb)
{
    int b = blockIdx.x;
    if constexpr (!ADJ) {
        // the previous step's edge and corner rows first
        if (b < ne) {
            edge_row_of<T>(s, ea, (long long)b * BLOCK + threadIdx.x);
            return;
        }
        b -= ne;
    }
    if constexpr (GEN) {
        // the rows of a general FEM mesh next: their gathers take longer per
        // block than a tile, so they start before the tiles (adjoint step
        // 197.1 -> 189.1 us on a 256^3-cell grid with a 96^3-cell general
        // box, against placing them last)
        if (b < ngb) {
            const long long n = gen_row(b, ngb);
            if constexpr (ADJ) gen_adj_row<T>(gs, n);
            else gen_fwd_row<T>(gs, n);
            return;
        }
        b -= ngb;
    }
    const int nf = (s.g.n_fdm_blocks[ADJ] + 7) / 8 * 8;
    if (b < nf) {
        if constexpr (ADJ) fdm_tile<T, true, NT>(s, b);
        else fdm_tile_cols<T, NT, fwd_cols<T>()>(s, b);
        return;
    }
    if constexpr (!ADJ) fem_tile<T, false, false>(s, b - nf);
}

template <typename T, bool ADJ, bool NT>
__global__ __launch_bounds__(BLOCK, (interior_waves<T, ADJ>())) void k_interior(Step<T> s, EdgeArgs<T> ea, int ne)
{
    interior_block<T, ADJ, NT, false>(s, ea, ne, GenStep<T>{}, 0);
}

// A separate kernel, so that the structured launch carries neither the
// general rows' code nor their arguments (both cost the structured steps
// ~0.6 us in FP64 and ~0.8 us in FP32).
template <typename T, bool ADJ, bool NT>
__global__ __launch_bounds__(BLOCK, (interior_waves<T, ADJ>())) void k_interior_gen(Step<T> s, EdgeArgs<T> ea,
                                                                                   int ne, GenStep<T> gs, int ngb)
{
    interior_block<T, ADJ, NT, true>(s, ea, ne, gs, ngb);
}

// Non-temporal hints pay when the field arrays a step streams (three levels,
// or level pair + increment pair in the FP32 increment form) of all slots of
// a launch exceed what the 256 MB last-level cache keeps (measured: they slow
// a cache-resident 257^3 sweep of three FP32 arrays by a third and speed up
// larger ones).
static bool stream_nt(const Geo &g, size_t esz, int slots)
{
    const double arrays = esz == 4 ? 4.0 : 3.0;
    return arrays * (double)g.plane * g.nz * esz * slots > 224.0 * (1 << 20);
}

// blocks of the edge and corner rows carried by a forward interior launch, a
// multiple of 8 so that the tile numbering after them keeps its XCD mapping
static int edge_blocks8(const Geo &g) { return (int)((g.n_ec + 8 * BLOCK - 1) / (8 * BLOCK) * 8); }

template <typename T>
void launch_interior(const Step<T> &s, bool adjoint, hipStream_t st, const EdgeArgs<T> *edges,
                     const GenStep<T> *gen)
{
    const int nf = (s.g.n_fdm_blocks[adjoint ? 1 : 0] + 7) / 8 * 8;
    const bool nt = stream_nt(s.g, sizeof(T), 1);
    EdgeArgs<T> ea{};
    int ne = 0;
    if (edges && !adjoint) {
        ea = *edges;
        ne = edge_blocks8(s.g);
    }
    if (gen) {
        const int ngb = gen_row_blocks(gen->nR);
        const dim3 grid((adjoint ? 0 : ne) + ngb + nf + (adjoint ? 0 : s.g.n_fem_blocks));
        if (adjoint) {
            if (nt) hipLaunchKernelGGL((k_interior_gen<T, true, true>), grid, dim3(BLOCK), 0, st, s, ea, 0, *gen, ngb);
            else hipLaunchKernelGGL((k_interior_gen<T, true, false>), grid, dim3(BLOCK), 0, st, s, ea, 0, *gen, ngb);
        } else {
            if (nt) hipLaunchKernelGGL((k_interior_gen<T, false, true>), grid, dim3(BLOCK), 0, st, s, ea, ne, *gen, ngb);
            else hipLaunchKernelGGL((k_interior_gen<T, false, false>), grid, dim3(BLOCK), 0, st, s, ea, ne, *gen, ngb);
        }
        return;
    }
    if (adjoint) {
        if (nt) hipLaunchKernelGGL((k_interior<T, true, true>), dim3(nf), dim3(BLOCK), 0, st, s, ea, 0);
        else hipLaunchKernelGGL((k_interior<T, true, false>), dim3(nf), dim3(BLOCK), 0, st, s, ea, 0);
    } else {
        const dim3 grid(ne + nf + s.g.n_fem_blocks);
        if (nt) hipLaunchKernelGGL((k_interior<T, false, true>), grid, dim3(BLOCK), 0, st, s, ea, ne);
        else hipLaunchKernelGGL((k_interior<T, false, false>), grid, dim3(BLOCK), 0, st, s, ea, ne);
    }
}

template <typename T>
void launch_bnd_fwd(const Step<T> &s, hipStream_t st)
{
    const long long n = fwd_face_rows(s.g, s.types1) + s.g.n_ec;
    hipLaunchKernelGGL((k_bnd_fwd<T>), dim3((unsigned)((n + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, st, s);
}

template <typename T>
void launch_bnd_fwd_faces(const Step<T> &s, hipStream_t st)
{
    const long long n = fwd_face_rows(s.g, s.types1);
    if (n > 0) hipLaunchKernelGGL((k_bnd_fwd<T>), dim3((unsigned)((n + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, st, s);
}

template <typename T>
void launch_bnd_fwd_edges(const Step<T> &s, hipStream_t st)
{
    if (s.g.n_ec > 0)
        hipLaunchKernelGGL((k_bnd_fwd_edges<T>), dim3((unsigned)((s.g.n_ec + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, st, s);
}

static long long ecf_blocks(const Geo &g)
{
    return ec_blocks8(g) + g.n_fem_blocks + (g.nwo + BLOCK - 1) / BLOCK;
}

template <typename T>
void launch_bnd_adj(const Step<T> &s, hipStream_t st, const GenStep<T> *gen)
{
    if (gen) {
        // a variable wave speed (minv) is not carried by general meshes
        const int nw = (int)((gen->fn - gen->nR + BLOCK - 1) / BLOCK);
        hipLaunchKernelGGL((k_bnd_adj_ecf_gen<T>), dim3((unsigned)(ecf_blocks(s.g) + nw)), dim3(BLOCK), 0, st, s,
                           *gen, nw);
    } else {
        const dim3 na((unsigned)ecf_blocks(s.g));
        if (s.minv) hipLaunchKernelGGL((k_bnd_adj_ecf<T, true>), na, dim3(BLOCK), 0, st, s);
        else hipLaunchKernelGGL((k_bnd_adj_ecf<T, false>), na, dim3(BLOCK), 0, st, s);
    }
    const long long nf = (adj_face_rows(s.g, s.types1, s.types2) + BLOCK - 1) / BLOCK;
    if (nf > 0) hipLaunchKernelGGL((k_bnd_adj_face<T>), dim3((unsigned)nf), dim3(BLOCK), 0, st, s);
}
// ---------------------------------------------------------------- batches
//
// Batched launches for the request server: blockIdx.y selects a slot whose
// step arguments sit in a device array.  Every slot of one launch has the
// same geometry (same grid and FEM box) but its own fields, time step and
// phase; the per-slot work is exactly that of the single-context kernels.

template <typename T, bool ADJ, bool NT>
__global__ __launch_bounds__(BLOCK, (interior_waves<T, ADJ>())) void k_interior_b(
    const Step<T> *__restrict__ steps, const EdgeArgs<T> *__restrict__ edges, int ne)
{
    const Step<T> &s = steps[blockIdx.y];
    int b = blockIdx.x;
    if constexpr (!ADJ) {
        // the slot's previous step's edge and corner rows first
        if (b < ne) {
            if (edges[blockIdx.y].Uc) edge_row_of<T>(s, edges[blockIdx.y], (long long)b * BLOCK + threadIdx.x);
            return;
        }
        b -= ne;
    }
    const int nf = (s.g.n_fdm_blocks[ADJ] + 7) / 8 * 8;
    if (b < nf) {
        if constexpr (ADJ) fdm_tile<T, true, NT>(s, b);
        else fdm_tile_cols<T, NT, fwd_cols<T>()>(s, b);
    }
    else if constexpr (!ADJ) fem_tile<T, false, false>(s, b - nf);
}

// faces_only: the slot's reflecting face rows (its edge rows run lagged in
// the next interior launch), else those and its edge and corner rows
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_bnd_fwd_b(const Step<T> *__restrict__ steps, int faces_only)
{
    const Step<T> &s = steps[blockIdx.y];
    const long long t = (long long)blockIdx.x * BLOCK + threadIdx.x;
    if (faces_only && t >= fwd_face_rows(s.g, s.types1)) return;
    bnd_fwd_body<T>(s, t);
}

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_bnd_adj_ecf_b(const Step<T> *__restrict__ steps)
{
    bnd_adj_ecf_body<T, false>(steps[blockIdx.y], blockIdx.x);
}

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_bnd_adj_face_b(const Step<T> *__restrict__ steps)
{
    bnd_adj_face_body<T>(steps[blockIdx.y], blockIdx.x);
}

long long fwd_face_row_count(const Geo &g, int types) { return fwd_face_rows(g, types); }

// With edges_dev the edge rows of each slot's previous step ride in the
// interior launch and the boundary launch takes the reflecting face rows
// alone; without it the boundary launch takes every slot's face, edge and
// corner rows.
template <typename T>
void launch_batch_fwd(const Geo &g, const Step<T> *steps_dev, const EdgeArgs<T> *edges_dev, int n,
                      long long face_rows, hipStream_t st)
{
    const int nf = (g.n_fdm_blocks[0] + 7) / 8 * 8;
    const int ne = edges_dev ? edge_blocks8(g) : 0;
    const dim3 grid(ne + nf + g.n_fem_blocks, n);
    if (stream_nt(g, sizeof(T), n))
        hipLaunchKernelGGL((k_interior_b<T, false, true>), grid, dim3(BLOCK), 0, st, steps_dev, edges_dev, ne);
    else
        hipLaunchKernelGGL((k_interior_b<T, false, false>), grid, dim3(BLOCK), 0, st, steps_dev, edges_dev, ne);
    const long long m = edges_dev ? face_rows : face_rows + g.n_ec;
    if (m > 0)
        hipLaunchKernelGGL((k_bnd_fwd_b<T>), dim3((unsigned)((m + BLOCK - 1) / BLOCK), n), dim3(BLOCK), 0, st,
                           steps_dev, edges_dev ? 1 : 0);
}

template <typename T>
void launch_batch_adj(const Geo &g, const Step<T> *steps_dev, int n, hipStream_t st)
{
    hipLaunchKernelGGL((k_bnd_adj_ecf_b<T>), dim3((unsigned)ecf_blocks(g), n), dim3(BLOCK), 0, st, steps_dev);
    // every slot's own face rows (its face conditions decide which x-face
    // rows its interior launch takes); the largest count is that of n_fi
    const long long nfb = (g.n_fi + BLOCK - 1) / BLOCK;
    if (nfb > 0) hipLaunchKernelGGL((k_bnd_adj_face_b<T>), dim3((unsigned)nfb, n), dim3(BLOCK), 0, st, steps_dev);
    const int nf = (g.n_fdm_blocks[1] + 7) / 8 * 8;
    if (stream_nt(g, sizeof(T), n))
        hipLaunchKernelGGL((k_interior_b<T, true, true>), dim3(nf, n), dim3(BLOCK), 0, st, steps_dev,
                           (const EdgeArgs<T> *)nullptr, 0);
    else
        hipLaunchKernelGGL((k_interior_b<T, true, false>), dim3(nf, n), dim3(BLOCK), 0, st, steps_dev,
                           (const EdgeArgs<T> *)nullptr, 0);
}

// ---------------------------------------------------------------- helpers

__device__ __forceinline__ bool cube_free(const Geo &g, long long c)
{
    const int i = (int)(c % g.C[0]);
    const int j = (int)((c / g.C[0]) % g.C[1]);
    const int k = (int)(c / ((long long)g.C[0] * g.C[1]));
    return i >= 2 && i < g.C[0] - 2 && j >= 2 && j < g.C[1] - 2 && k >= 2 && k < g.C[2] - 2;
}

// block-wide sum / max of a double (wave64 shuffles + LDS), thread 0 gets it
__device__ double block_reduce(double v, bool is_max)
{
    __shared__ double sh[BLOCK / 64];
    for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_down(v, off, 64);
        v = is_max ? fmax(v, o) : v + o;
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        v = sh[0];
        for (int q = 1; q < BLOCK / 64; ++q) v = is_max ? fmax(v, sh[q]) : v + sh[q];
    }
    return v;
}

// Second pass of a deterministic reduction: one block folds the partials in
// a fixed order; result scaled by `scale` into scal[slot].
__global__ __launch_bounds__(BLOCK) void k_final(const double *part, int n, int is_max, double scale,
                                                 double *scal, int slot)
{
    double v = is_max ? 0.0 : 0.0;
    for (int q = threadIdx.x; q < n; q += BLOCK) v = is_max ? fmax(v, part[q]) : v + part[q];
    v = block_reduce(v, is_max != 0);
    if (threadIdx.x == 0) scal[slot] = v * scale;
}

static int nparts(long long n) { return (int)std::min<long long>(MAX_PARTIALS, (n + BLOCK - 1) / BLOCK); }

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_acube(Geo g, const double *sigma, T *acube, double *part_max,
                                                 double *part_bad)
{
    const long long n = (long long)g.C[0] * g.C[1] * g.C[2];
    double mx = 0.0, bad = 0.0;
    for (long long c = (long long)blockIdx.x * BLOCK + threadIdx.x; c < n; c += (long long)gridDim.x * BLOCK) {
        double sv = 0.0;
        if (sigma && cube_free(g, c)) {
            sv = sigma[c];
            if (!isfinite(sv)) { bad = 1.0; sv = 0.0; }
            mx = fmax(mx, sv);
        }
        acube[c] = (T)(1.0 + sv);
    }
    mx = block_reduce(mx, true);
    __syncthreads();
    bad = block_reduce(bad, true);
    if (threadIdx.x == 0) { part_max[blockIdx.x] = mx; part_bad[blockIdx.x] = bad; }
}

template <typename T>
void launch_acube(const Geo &g, const double *sigma, T *acube, double *partials, double *scal,
                  hipStream_t st)
{
    const long long n = (long long)g.C[0] * g.C[1] * g.C[2];
    const int nb = std::min(nparts(n), MAX_PARTIALS / 2);
    hipLaunchKernelGGL((k_acube<T>), dim3(nb), dim3(BLOCK), 0, st, g, sigma, acube, partials,
                       partials + MAX_PARTIALS / 2);
    hipLaunchKernelGGL(k_final, dim3(1), dim3(BLOCK), 0, st, partials, nb, 1, 1.0, scal, (int)S_SMAX);
    hipLaunchKernelGGL(k_final, dim3(1), dim3(BLOCK), 0, st, partials + MAX_PARTIALS / 2, nb, 1, 1.0,
                       scal, (int)S_BAD);
}

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_load_level(Geo g, const double *src, T *U, T *V)
{
    const long long n = (long long)g.nx * g.ny * g.nz;
    for (long long t = (long long)blockIdx.x * BLOCK + threadIdx.x; t < n; t += (long long)gridDim.x * BLOCK) {
        const int x = (int)(t % g.nx), y = (int)((t / g.nx) % g.ny), z = (int)(t / ((long long)g.nx * g.ny));
        const T v = src ? (T)src[t] : (T)0;
        U[gidx(g, x, y, z)] = v;
        if (g.has_fem) {
            const int i = x - g.o[0], j = y - g.o[1], k = z - g.o[2];
            if (i >= 0 && i <= g.C[0] && j >= 0 && j <= g.C[1] && k >= 0 && k <= g.C[2]) V[fidx(g, i, j, k)] = v;
        }
    }
}

template <typename T>
void launch_load_level(const Geo &g, const double *src, T *U, T *V, hipStream_t st)
{
    hipLaunchKernelGGL((k_load_level<T>), dim3(2048), dim3(BLOCK), 0, st, g, src, U, V);
}

// eps of FEM-local cube (a, b, c): 1/c^2 on free cubes, 1 elsewhere
__device__ __forceinline__ double eps_at(const Geo &g, const double *eps, int a, int b, int c)
{
    if (a < 2 || b < 2 || c < 2 || a > g.C[0] - 3 || b > g.C[1] - 3 || c > g.C[2] - 3) return 1.0;
    return eps[a + (long long)g.C[0] * (b + (long long)g.C[1] * c)];
}

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_minv(Geo g, const double *eps, T *minv)
{
    const long long n = g.fem_n;
    for (long long t = (long long)blockIdx.x * BLOCK + threadIdx.x; t < n; t += (long long)gridDim.x * BLOCK) {
        const int i = (int)(t % g.fpx), j = (int)((t / g.fpx) % (g.fplane / g.fpx)), k = (int)(t / g.fplane);
        // the node is corner (dx,dy,dz) of cube (i-dx, j-dy, k-dz); the Kuhn
        // diagonal joins corners (0,0,0) and (1,1,1)
        double ends = eps_at(g, eps, i, j, k) + eps_at(g, eps, i - 1, j - 1, k - 1);
        double others = 0.0;
#pragma unroll
        for (int q = 1; q < 7; ++q)
            others += eps_at(g, eps, i - (q & 1), j - ((q >> 1) & 1), k - (q >> 2));
        minv[t] = (T)(12.0 / (3.0 * ends + others));
    }
}

template <typename T>
void launch_minv(const Geo &g, const double *eps, T *minv, hipStream_t st)
{
    hipLaunchKernelGGL((k_minv<T>), dim3(1024), dim3(BLOCK), 0, st, g, eps, minv);
}

__global__ __launch_bounds__(BLOCK) void k_eps_grad(Geo g, const double *Gm, double scale, double *geps)
{
    const long long n = (long long)g.C[0] * g.C[1] * g.C[2];
    for (long long c = (long long)blockIdx.x * BLOCK + threadIdx.x; c < n; c += (long long)gridDim.x * BLOCK) {
        const int a = (int)(c % g.C[0]), b = (int)((c / g.C[0]) % g.C[1]), z = (int)(c / ((long long)g.C[0] * g.C[1]));
        double v = 0.0;
        if (a >= 2 && b >= 2 && z >= 2 && a <= g.C[0] - 3 && b <= g.C[1] - 3 && z <= g.C[2] - 3) {
            const long long n0 = fidx(g, a, b, z);
            double ends = Gm[n0] + Gm[n0 + 1 + g.fpx + g.fplane], others = 0.0;
#pragma unroll
            for (int q = 1; q < 7; ++q) others += Gm[n0 + (q & 1) + ((q >> 1) & 1) * g.fpx + (q >> 2) * g.fplane];
            v = scale * (3.0 * ends + others) / 12.0;
        }
        geps[c] = v;
    }
}

void launch_eps_grad(const Geo &g, const double *Gm, double scale, double *geps, hipStream_t st)
{
    hipLaunchKernelGGL(k_eps_grad, dim3(1024), dim3(BLOCK), 0, st, g, Gm, scale, geps);
}

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_hist_diff(Geo g, const T *a, const T *b, T *hist)
{
    const long long n = g.hlevel;
    for (long long t = (long long)blockIdx.x * BLOCK + threadIdx.x; t < n; t += (long long)gridDim.x * BLOCK) {
        const int p = (int)(t % g.hn[0]), q = (int)((t / g.hn[0]) % g.hn[1]), r = (int)(t / ((long long)g.hn[0] * g.hn[1]));
        const long long f = fidx(g, 2 + p, 2 + q, 2 + r);
        hist[t] = b ? a[f] - b[f] : a[f];
    }
}

template <typename T>
void launch_hist_diff(const Geo &g, const T *a, const T *b, T *hist, hipStream_t st)
{
    hipLaunchKernelGGL((k_hist_diff<T>), dim3(1024), dim3(BLOCK), 0, st, g, a, b, hist);
}

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_load_combo(Geo g, const double *a, const double *b, double cb, T *U,
                                                      T *V)
{
    const long long n = (long long)g.nx * g.ny * g.nz;
    for (long long t = (long long)blockIdx.x * BLOCK + threadIdx.x; t < n; t += (long long)gridDim.x * BLOCK) {
        const int x = (int)(t % g.nx), y = (int)((t / g.nx) % g.ny), z = (int)(t / ((long long)g.nx * g.ny));
        const T v = (T)((a ? a[t] : 0.0) + (b ? cb * b[t] : 0.0));
        U[gidx(g, x, y, z)] = v;
        if (g.has_fem) {
            const int i = x - g.o[0], j = y - g.o[1], k = z - g.o[2];
            if (i >= 0 && i <= g.C[0] && j >= 0 && j <= g.C[1] && k >= 0 && k <= g.C[2]) V[fidx(g, i, j, k)] = v;
        }
    }
}

template <typename T>
void launch_load_combo(const Geo &g, const double *a, const double *b, double cb, T *U, T *V, hipStream_t st)
{
    hipLaunchKernelGGL((k_load_combo<T>), dim3(2048), dim3(BLOCK), 0, st, g, a, b, cb, U, V);
}

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_load_incr(Geo g, const double *u0, const double *um1, T *D, T *VD)
{
    const long long n = (long long)g.nx * g.ny * g.nz;
    for (long long t = (long long)blockIdx.x * BLOCK + threadIdx.x; t < n; t += (long long)gridDim.x * BLOCK) {
        const int x = (int)(t % g.nx), y = (int)((t / g.nx) % g.ny), z = (int)(t / ((long long)g.nx * g.ny));
        const T d = (T)((u0 ? u0[t] : 0.0) - (um1 ? um1[t] : 0.0));
        D[gidx(g, x, y, z)] = d;
        if (g.has_fem) {
            const int i = x - g.o[0], j = y - g.o[1], k = z - g.o[2];
            if (i >= 0 && i <= g.C[0] && j >= 0 && j <= g.C[1] && k >= 0 && k <= g.C[2]) VD[fidx(g, i, j, k)] = d;
        }
    }
}

template <typename T>
void launch_load_incr(const Geo &g, const double *u0, const double *um1, T *D, T *VD, hipStream_t st)
{
    hipLaunchKernelGGL((k_load_incr<T>), dim3(2048), dim3(BLOCK), 0, st, g, u0, um1, D, VD);
}

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_hist_level(Geo g, const T *V, T *hist)
{
    const long long n = g.hlevel;
    for (long long t = (long long)blockIdx.x * BLOCK + threadIdx.x; t < n; t += (long long)gridDim.x * BLOCK) {
        const int a = (int)(t % g.hn[0]), b = (int)((t / g.hn[0]) % g.hn[1]),
                  c = (int)(t / ((long long)g.hn[0] * g.hn[1]));
        hist[t] = V[fidx(g, 2 + a, 2 + b, 2 + c)];
    }
}

template <typename T>
void launch_hist_level(const Geo &g, const T *V, T *hist, hipStream_t st)
{
    hipLaunchKernelGGL((k_hist_level<T>), dim3(1024), dim3(BLOCK), 0, st, g, V, hist);
}

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_record_face(Geo g, const T *U, double *row)
{
    const long long n = (long long)g.nx * g.ny;
    for (long long t = (long long)blockIdx.x * BLOCK + threadIdx.x; t < n; t += (long long)gridDim.x * BLOCK)
        row[t] = (double)U[gidx(g, (int)(t % g.nx), (int)(t / g.nx), g.nz - 1)];
}

template <typename T>
void launch_record_face(const Geo &g, const T *U, double *obs_row, hipStream_t st)
{
    hipLaunchKernelGGL((k_record_face<T>), dim3(256), dim3(BLOCK), 0, st, g, U, obs_row);
}

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_export_level(Geo g, const T *U, const T *V, const T *F, double *u,
                                                       double *v, int types)
{
    const long long n = (long long)g.nx * g.ny * g.nz;
    for (long long t = (long long)blockIdx.x * BLOCK + threadIdx.x; t < n; t += (long long)gridDim.x * BLOCK) {
        const int x = (int)(t % g.nx), y = (int)((t / g.nx) % g.ny), z = (int)(t / ((long long)g.nx * g.ny));
        // nodes strictly inside the hole belong to no grid row: no value
        const bool hole = g.has_fem && x > g.hlo[0] && x < g.hhi[0] && y > g.hlo[1] && y < g.hhi[1] &&
                          z > g.hlo[2] && z < g.hhi[2];
        // boundary multipliers live in the face arrays, except the rows of
        // absorbing x faces away from the edges (kept in the grid array)
        const bool xin = (x == 0 || x == g.nx - 1) && x_face_in_tile(g, types, types, x == 0 ? 0 : 1) &&
                         y >= 2 && y <= g.ny - 3 && z >= 2 && z <= g.nz - 3;
        if (u)
            u[t] = hole ? 0.0
                        : (double)((F && on_bnd(g, x, y, z) && !xin) ? F[cidx(g, x, y, z)] : U[gidx(g, x, y, z)]);
    }
    if (!v || !g.has_fem) return;
    const long long nf = (long long)(g.C[0] + 1) * (g.C[1] + 1) * (g.C[2] + 1);
    for (long long t = (long long)blockIdx.x * BLOCK + threadIdx.x; t < nf; t += (long long)gridDim.x * BLOCK) {
        // the forward level's box surface (omega_o) is the grid's
        const int i = (int)(t % (g.C[0] + 1)), j = (int)((t / (g.C[0] + 1)) % (g.C[1] + 1));
        const int k = (int)(t / ((long long)(g.C[0] + 1) * (g.C[1] + 1)));
        const bool surf = i == 0 || i == g.C[0] || j == 0 || j == g.C[1] || k == 0 || k == g.C[2];
        v[t] = (double)((!F && surf) ? U[gidx(g, g.o[0] + i, g.o[1] + j, g.o[2] + k)] : V[t]);
    }
}

template <typename T>
void launch_export_level(const Geo &g, const T *U, const T *V, const T *F, double *u, double *v,
                         hipStream_t st, int types)
{
    hipLaunchKernelGGL((k_export_level<T>), dim3(1024), dim3(BLOCK), 0, st, g, U, V, F, u, v, types);
}

__device__ __forceinline__ uint16_t f32_to_bf16(float x)
{
    const uint32_t u = __float_as_uint(x);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);  // round to nearest even
}

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__global__ __launch_bounds__(BLOCK) void k_pack_bf16(const float *a, uint16_t *half, long long n)
{
    for (long long i = (long long)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (long long)gridDim.x * BLOCK)
        half[i] = f32_to_bf16(a[i]);
}

__global__ __launch_bounds__(BLOCK) void k_unpack_bf16(const uint16_t *half, float *b, long long n)
{
    for (long long i = (long long)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (long long)gridDim.x * BLOCK)
        b[i] = bf16_to_f32(half[i]);
}

void launch_pack_bf16(const void *a, uint16_t *half, long long n, hipStream_t st)
{
    hipLaunchKernelGGL(k_pack_bf16, dim3(4096), dim3(BLOCK), 0, st, (const float *)a, half, n);
}

void launch_unpack_bf16(const uint16_t *half, void *b, long long n, hipStream_t st)
{
    hipLaunchKernelGGL(k_unpack_bf16, dim3(4096), dim3(BLOCK), 0, st, half, (float *)b, n);
}

// 16-bit block-scaled checkpoint increments: each group of 64 consecutive
// values (one wavefront) shares the scale m / 32767, m the group's largest
// magnitude, and stores round(a / scale) as int16, so every value is kept to
// m / 65534 -- 128 times finer than BF16's relative 2^-9 for the group's
// large values, which set the state's perturbation.
__global__ __launch_bounds__(BLOCK) void k_pack_q16(const float *a, int16_t *q, float *scale, long long n)
{
    const int lane = (int)(threadIdx.x & 63);
    const long long ng = (n + 63) / 64;
    const long long w0 = ((long long)blockIdx.x * BLOCK + threadIdx.x) >> 6, nw = (long long)gridDim.x * BLOCK / 64;
    for (long long grp = w0; grp < ng; grp += nw) {
        const long long i = grp * 64 + lane;
        const float v = i < n ? a[i] : 0.0f;
        float m = fabsf(v);
        for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
        const float sc = m / 32767.0f;
        int qv = 0;
        if (sc > 0.0f) qv = max(-32767, min(32767, (int)rintf(v / sc)));
        if (i < n) q[i] = (int16_t)qv;
        if (lane == 0) scale[grp] = sc;
    }
}

__global__ __launch_bounds__(BLOCK) void k_unpack_q16(const int16_t *q, const float *scale, float *b, long long n)
{
    for (long long i = (long long)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (long long)gridDim.x * BLOCK)
        b[i] = (float)q[i] * scale[i >> 6];
}

void launch_pack_q16(const void *a, int16_t *q, float *scale, long long n, hipStream_t st)
{
    hipLaunchKernelGGL(k_pack_q16, dim3(4096), dim3(BLOCK), 0, st, (const float *)a, q, scale, n);
}

void launch_unpack_q16(const int16_t *q, const float *scale, void *b, long long n, hipStream_t st)
{
    hipLaunchKernelGGL(k_unpack_q16, dim3(4096), dim3(BLOCK), 0, st, q, scale, (float *)b, n);
}

__global__ __launch_bounds__(BLOCK) void k_misfit(Geo g, const double *res, int nt, double wscale,
                                                  double *part)
{
    const long long nf = (long long)g.nx * g.ny, n = nf * nt;
    double acc = 0.0;
    for (long long t = (long long)blockIdx.x * BLOCK + threadIdx.x; t < n; t += (long long)gridDim.x * BLOCK) {
        const long long q = t % nf;
        const int x = (int)(q % g.nx), y = (int)(q / g.nx);
        double w = 1.0;
        if (x == 0 || x == g.nx - 1) w *= 0.5;
        if (y == 0 || y == g.ny - 1) w *= 0.5;
        const double r = res[nf + t];  // levels 1..nt
        acc += w * r * r;
    }
    acc = block_reduce(acc, false);
    if (threadIdx.x == 0) part[blockIdx.x] = acc * wscale;
}

void launch_misfit(const Geo &g, const double *res, int nt, double dt, double h, double *partials,
                   double *scal, int slot, hipStream_t st)
{
    const long long n = (long long)g.nx * g.ny * nt;
    const int nb = nparts(n);
    hipLaunchKernelGGL(k_misfit, dim3(nb), dim3(BLOCK), 0, st, g, res, nt, 0.5 * dt * h * h, partials);
    hipLaunchKernelGGL(k_final, dim3(1), dim3(BLOCK), 0, st, partials, nb, 0, 1.0, scal, slot);
}

__global__ __launch_bounds__(BLOCK) void k_grad_final(Geo g, const double *G, const double *sigma, double coefG,
                                                      double gamma, int mode, double *grad, double *part)
{
    const long long n = (long long)g.C[0] * g.C[1] * g.C[2];
    double reg = 0.0;
    for (long long c = (long long)blockIdx.x * BLOCK + threadIdx.x; c < n; c += (long long)gridDim.x * BLOCK) {
        double v = 0.0;
        if (cube_free(g, c)) {
            const double sv = sigma ? sigma[c] : 0.0;
            v = coefG * G[c];
            if (mode == 0) {
                v += gamma * sv;
                reg += sv * sv;
            }
        }
        grad[c] = v;
    }
    reg = block_reduce(reg, false);
    if (threadIdx.x == 0) part[blockIdx.x] = reg;
}

void launch_grad_final(const Geo &g, const double *G, const double *sigma, double coefG, double gamma,
                       int mode, double h3, double *grad, double *partials, double *scal, int slot,
                       hipStream_t st, int blocks)
{
    const long long n = (long long)g.C[0] * g.C[1] * g.C[2];
    const int nb = blocks > 0 ? blocks : nparts(n);
    hipLaunchKernelGGL(k_grad_final, dim3(nb), dim3(BLOCK), 0, st, g, G, sigma, coefG, gamma, mode, grad,
                       partials);
    hipLaunchKernelGGL(k_final, dim3(1), dim3(BLOCK), 0, st, partials, nb, 0, 0.5 * gamma * h3, scal, slot);
}

// ---------------------------------------------------------------- CG
//
// Algorithm 3 on the conductivity parameters: cubes of a structured box or
// tetrahedra of a general mesh, each with its L2 weight (cell volume) when
// it is free and weight 0 otherwise (those cells never move).

__device__ __forceinline__ double pweight(const Params &p, long long c)
{
    if (p.pvol) return p.pvol[c];
    const int i = (int)(c % p.C[0]);
    const int j = (int)((c / p.C[0]) % p.C[1]);
    const int k = (int)(c / ((long long)p.C[0] * p.C[1]));
    return (i >= 2 && i < p.C[0] - 2 && j >= 2 && j < p.C[1] - 2 && k >= 2 && k < p.C[2] - 2) ? p.h3 : 0.0;
}

// partial sums of w v^2 (L2 norm with the cell volumes)
__global__ __launch_bounds__(BLOCK) void k_wsumsq(Params p, const double *v, double *part)
{
    double acc = 0.0;
    for (long long c = (long long)blockIdx.x * BLOCK + threadIdx.x; c < p.n; c += (long long)gridDim.x * BLOCK)
        acc += pweight(p, c) * v[c] * v[c];
    acc = block_reduce(acc, false);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

void launch_cg_norm2(const Params &p, const double *v, double *partials, double *scal, int slot, hipStream_t st)
{
    const int nb = nparts(p.n);
    hipLaunchKernelGGL(k_wsumsq, dim3(nb), dim3(BLOCK), 0, st, p, v, partials);
    hipLaunchKernelGGL(k_final, dim3(1), dim3(BLOCK), 0, st, partials, nb, 0, 1.0, scal, slot);
}

// Fletcher-Reeves direction d = -g + beta d^{m-1} on free cells (beta^0 = 0)
// and per block: max|d|, max|g| and the slope sum w g d over the cells free
// to move (a cell held by a bound, sigma = 0 moving down or sigma = 4 moving
// up, does not move under the projection).
constexpr int DIR_PARTS = MAX_PARTIALS / 4;

__global__ __launch_bounds__(BLOCK) void k_cg_dir(Params p, const double *grad, double *dir, const double *sigma,
                                                  int first, const double *scal, double *part)
{
    const double beta = first ? 0.0 : scal[S_GN2] / scal[S_GN2P];
    double dm = 0.0, gm = 0.0, slope = 0.0;
    for (long long c = (long long)blockIdx.x * BLOCK + threadIdx.x; c < p.n; c += (long long)gridDim.x * BLOCK) {
        const double w = pweight(p, c);
        double d = 0.0;
        if (w > 0.0) {
            const double g = grad[c], sv = sigma[c];
            d = first ? -g : -g + beta * dir[c];
            const bool held = (sv <= 0.0 && d < 0.0) || (sv >= 4.0 && d > 0.0);
            if (!held) slope += w * g * d;
            gm = fmax(gm, fabs(g));
        }
        dir[c] = d;
        dm = fmax(dm, fabs(d));
    }
    dm = block_reduce(dm, true);
    __syncthreads();
    gm = block_reduce(gm, true);
    __syncthreads();
    slope = block_reduce(slope, false);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = dm;
        part[DIR_PARTS + blockIdx.x] = gm;
        part[2 * DIR_PARTS + blockIdx.x] = slope;
    }
}

// Folds the direction partials (fixed order) and decides the iteration:
// beta, restart when m > 0 and the slope is >= 0 (then d = -g), and max|d|
// of the direction searched.
__global__ __launch_bounds__(BLOCK) void k_cg_decide(const double *part, int nb, int first, double *scal)
{
    double dm = 0.0, gm = 0.0, slope = 0.0;
    for (int q = threadIdx.x; q < nb; q += BLOCK) {
        dm = fmax(dm, part[q]);
        gm = fmax(gm, part[DIR_PARTS + q]);
        slope += part[2 * DIR_PARTS + q];
    }
    dm = block_reduce(dm, true);
    __syncthreads();
    gm = block_reduce(gm, true);
    __syncthreads();
    slope = block_reduce(slope, false);
    if (threadIdx.x == 0) {
        const bool restart = !first && slope >= 0.0;
        scal[S_BETA] = first ? 0.0 : scal[S_GN2] / scal[S_GN2P];
        scal[S_SLOPE] = slope;
        scal[S_RESTART] = restart ? 1.0 : 0.0;
        scal[S_DMAX] = restart ? gm : dm;
    }
}

__global__ __launch_bounds__(BLOCK) void k_cg_restart(Params p, const double *grad, double *dir, const double *scal)
{
    if (scal[S_RESTART] == 0.0) return;
    for (long long c = (long long)blockIdx.x * BLOCK + threadIdx.x; c < p.n; c += (long long)gridDim.x * BLOCK)
        dir[c] = pweight(p, c) > 0.0 ? -grad[c] : 0.0;
}

void launch_cg_dir(const Params &p, const double *grad, double *dir, const double *sigma, int first,
                   double *partials, double *scal, hipStream_t st)
{
    const int nb = std::min(nparts(p.n), DIR_PARTS);
    hipLaunchKernelGGL(k_cg_dir, dim3(nb), dim3(BLOCK), 0, st, p, grad, dir, sigma, first, scal, partials);
    hipLaunchKernelGGL(k_cg_decide, dim3(1), dim3(BLOCK), 0, st, partials, nb, first, scal);
    hipLaunchKernelGGL(k_cg_restart, dim3(nparts(p.n)), dim3(BLOCK), 0, st, p, grad, dir, scal);
}

// Trial point t of the step search: sigma_t = clip(sigma + alpha_t d, 0, 4)
// on free cells (the others copy sigma), alpha_t = 2^{-t} alpha_rel / max|d|;
// partials of w sigma_t^2 for the Tikhonov term of J(sigma_t).
__global__ __launch_bounds__(BLOCK) void k_cg_trial(Params p, const double *dir, const double *sigma, double *trial,
                                                    double alpha_rel, int t, double *scal, double *part)
{
    const double dmax = scal[S_DMAX];
    const double alpha = dmax > 0.0 ? ldexp(alpha_rel / dmax, -t) : 0.0;
    double reg = 0.0;
    for (long long c = (long long)blockIdx.x * BLOCK + threadIdx.x; c < p.n; c += (long long)gridDim.x * BLOCK) {
        const double w = pweight(p, c);
        double sv = sigma[c];
        if (w > 0.0) {
            sv += alpha * dir[c];
            sv = sv < 0.0 ? 0.0 : (sv > 4.0 ? 4.0 : sv);
            reg += w * sv * sv;
        }
        trial[c] = sv;
    }
    reg = block_reduce(reg, false);
    if (threadIdx.x == 0) part[blockIdx.x] = reg;
    if (blockIdx.x == 0 && threadIdx.x == 0) scal[S_ALPHA] = alpha;
}

void launch_cg_trial(const Params &p, const double *dir, const double *sigma, double *trial, double alpha_rel,
                     int t, double gamma, double *partials, double *scal, hipStream_t st)
{
    const int nb = nparts(p.n);
    hipLaunchKernelGGL(k_cg_trial, dim3(nb), dim3(BLOCK), 0, st, p, dir, sigma, trial, alpha_rel, t, scal,
                       partials);
    hipLaunchKernelGGL(k_final, dim3(1), dim3(BLOCK), 0, st, partials, nb, 0, 0.5 * gamma, scal, (int)S_JREGT);
}

__global__ void k_roll_gn2(double *scal)
{
    if (threadIdx.x == 0) scal[S_GN2P] = scal[S_GN2];
}

void launch_cg_roll(double *scal, hipStream_t st)
{
    hipLaunchKernelGGL(k_roll_gn2, dim3(1), dim3(64), 0, st, scal);
}

// 1 when two FP64 arrays differ anywhere (bitwise, NaN-safe)
__global__ __launch_bounds__(BLOCK) void k_differ(const double *a, const double *b, long long n, double *part)
{
    double diff = 0.0;
    for (long long c = (long long)blockIdx.x * BLOCK + threadIdx.x; c < n; c += (long long)gridDim.x * BLOCK)
        if (__double_as_longlong(a[c]) != __double_as_longlong(b[c])) diff = 1.0;
    diff = block_reduce(diff, true);
    if (threadIdx.x == 0) part[blockIdx.x] = diff;
}

void launch_differ(const double *a, const double *b, long long n, double *partials, double *scal, int slot,
                   hipStream_t st)
{
    const int nb = nparts(n);
    hipLaunchKernelGGL(k_differ, dim3(nb), dim3(BLOCK), 0, st, a, b, n, partials);
    hipLaunchKernelGGL(k_final, dim3(1), dim3(BLOCK), 0, st, partials, nb, 1, 1.0, scal, slot);
}

__global__ __launch_bounds__(BLOCK) void k_residual(const double *obs, const double *data, double *res,
                                                    long long n)
{
    for (long long t = (long long)blockIdx.x * BLOCK + threadIdx.x; t < n; t += (long long)gridDim.x * BLOCK)
        res[t] = obs[t] - data[t];
}

void launch_residual(const double *obs, const double *data, double *res, long long n, hipStream_t st)
{
    hipLaunchKernelGGL(k_residual, dim3(nparts(n)), dim3(BLOCK), 0, st, obs, data, res, n);
}

// ------------------------------------------------------- no-allocation scratch
//
// Scratch of hyb_gradient_noalloc, for callers that cannot allocate device
// memory: the reduction partials (one per block of 256 parameters) and the
// scalars, in a file-scope device array.  Each GPU the library runs on holds
// its own copy until the process ends; every call on that GPU shares it.
// Host code must not pass the array's name to a kernel (on the host it is a
// stand-in, not a device address): noalloc_scratch resolves the address once
// per device with hipGetSymbolAddress and the kernels take that pointer.
static __device__ __align__(256) double scratch[NOALLOC_PARTS + NOALLOC_SCAL];

hipError_t noalloc_scratch(double **out)
{
    static std::mutex mu;
    static double *addr[NOALLOC_MAX_DEVICES] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = (double *)p;
    }
    *out = addr[dev];
    return hipSuccess;
}

// J = misfit (from the adjoint, in the context's scalars) + regularisation
// (from the scratch scalars), or 0 for a cotangent adjoint (mode 1).
__global__ void k_sum_J(const double *jmis, const double *jreg, int mode, double *J)
{
    if (threadIdx.x == 0) J[0] = mode == 0 ? jmis[0] + jreg[0] : 0.0;
}

void launch_sum_J(const double *jmis, const double *jreg, int mode, double *J, hipStream_t st)
{
    hipLaunchKernelGGL(k_sum_J, dim3(1), dim3(64), 0, st, jmis, jreg, mode, J);
}

// explicit instantiations
#define HYB_INST(T)                                                                               \
    template void launch_interior<T>(const Step<T> &, bool, hipStream_t, const EdgeArgs<T> *,       \
                                     const GenStep<T> *);                                         \
    template void launch_bnd_fwd<T>(const Step<T> &, hipStream_t);                                \
    template void launch_bnd_fwd_faces<T>(const Step<T> &, hipStream_t);                          \
    template void launch_bnd_fwd_edges<T>(const Step<T> &, hipStream_t);                          \
    template void launch_bnd_adj<T>(const Step<T> &, hipStream_t, const GenStep<T> *);            \
    template void launch_batch_fwd<T>(const Geo &, const Step<T> *, const EdgeArgs<T> *, int,     \
                                       long long, hipStream_t);                                 \
    template void launch_batch_adj<T>(const Geo &, const Step<T> *, int, hipStream_t);                                \
    template void launch_acube<T>(const Geo &, const double *, T *, double *, double *, hipStream_t); \
    template void launch_load_level<T>(const Geo &, const double *, T *, T *, hipStream_t);        \
    template void launch_load_combo<T>(const Geo &, const double *, const double *, double, T *, T *, \
                                       hipStream_t);                                              \
    template void launch_minv<T>(const Geo &, const double *, T *, hipStream_t);                   \
    template void launch_hist_diff<T>(const Geo &, const T *, const T *, T *, hipStream_t);         \
    template void launch_load_incr<T>(const Geo &, const double *, const double *, T *, T *, hipStream_t); \
    template void launch_hist_level<T>(const Geo &, const T *, T *, hipStream_t);                  \
    template void launch_record_face<T>(const Geo &, const T *, double *, hipStream_t);            \
    template void launch_export_level<T>(const Geo &, const T *, const T *, const T *, double *, double *,     \
                                         hipStream_t, int);
HYB_INST(double)
HYB_INST(float)

}  // namespace hyb
