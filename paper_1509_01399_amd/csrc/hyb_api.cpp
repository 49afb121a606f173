// Host side of libhyb: the C ABI of include/hyb.h.  Validates inputs, turns
// the tetrahedral FEM mesh into per-cube P1 element weights, owns the device
// memory of one problem and drives the time loops of Algorithm 2 (forward and
// exact adjoint) and the conjugate-gradient iteration of Algorithm 3.  All
// arithmetic on fields runs in the kernels of hyb_kernels.hip.
#include "../../include/hyb.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "hyb_gen.h"
#include "hyb_internal.h"

using namespace hyb;

namespace {

thread_local std::string g_create_err;

struct Mesh {
    int o[3] = {0, 0, 0}, C[3] = {0, 0, 0};
    double w[12] = {0};  // cube edge weights / h
};

}  // namespace

struct hyb_ctx {
    Geo g{};
    int n[3]{};
    double h = 0;
    int bc[6]{};
    int f32 = 0, store_mode = 0;
    double gamma = 0.01, alpha_rel = 0.25;
    int max_trials = 8;          // CG trial steps per iteration
    hipStream_t stream = nullptr;
    Mesh mesh;
    size_t esz = 8;  // field element size
    // device memory
    void *U[3]{}, *V[3]{}, *P[3]{}, *Q[3]{}, *F[3]{};
    void *D[2]{}, *VD[2]{};  // FP32: forward increments, d^k in slot k & 1
    void *E[2]{}, *QE[2]{};  // FP32: adjoint increments (level k in slot k & 1)
    void *acube = nullptr;
    void *hist = nullptr;
    size_t hist_levels = 0;
    double *sig = nullptr, *G = nullptr, *dir = nullptr, *grad = nullptr, *trial = nullptr;
    // CG: the last forward sweep ran at the accepted trial point that the
    // previous hyb_cg_step wrote to cg_sigma (with these data), so the next
    // iteration can start from it
    bool cg_ready = false;
    const double *cg_sigma = nullptr, *cg_data = nullptr;
    double *obsbuf = nullptr, *resbuf = nullptr;
    size_t tracebuf_levels = 0;
    double *partials = nullptr, *scal = nullptr;
    const double *ic_u0 = nullptr, *ic_um1 = nullptr;
    bool ic_set = false;
    // Model Problem 1 data (hyb_set_initial_taylor): f0, f1 copied into the
    // context (full unpadded FP64 grid levels), used by every forward sweep
    bool taylor = false;
    double *tf0 = nullptr, *tf1 = nullptr;
    bool sweep_taylor = false;   // the last forward sweep started with the Taylor step
    // variable wave speed (hyb_set_wave_speed): 1/c^2 per cube, per-node
    // 1/m (field precision), per-node dJ/dm (FP64), history box of u^{-1}
    bool vm = false;
    double eps_min = 1.0;
    double *epsc = nullptr, *Gm = nullptr;
    void *minv = nullptr, *hm1 = nullptr;
    // state of the last forward / adjoint
    bool have_forward = false, have_adjoint = false;
    int nt = 0, k_on = 0, adj_mode = 0;
    int last_u = 1, last_p = 1;  // buffer index of the newest level
    bool u_valid = false;        // U buffers still hold the last forward level
    hyb_source src{};            // source of the last forward (recompute)
    void *ckpt = nullptr;        // checkpoints (store modes 1, 2)
    size_t ckpt_bytes = 0;
    int ckK = 1, cur_seg = 0;    // segment length and the segment in the history
    bool in_batch = false;       // owned by a batch slot (single calls refused)
    double dt = 0;
    // general tetrahedral mesh: per-tetrahedron sigma, FEM rows in hyb_gen.hip
    bool gen = false;
    bool gen_all_grid = true;    // every FEM node is a grid node (initial levels allowed)
    long long npar = 0;          // conductivity parameters: cubes, or tetrahedra
    GenDev gd{};
    std::string err;
};

namespace {

hyb_status fail(hyb_ctx *c, hyb_status s, const std::string &msg)
{
    if (c) c->err = msg;
    else g_create_err = msg;
    return s;
}

#define HIPCHK(ctx, call)                                                                     \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(ctx, HYB_E_DEVICE, std::string(#call ": ") + hipGetErrorString(e_)); \
    } while (0)

long long ceil_div(long long a, long long b) { return (a + b - 1) / b; }

// Gradients of the barycentric coordinates of a tetrahedron (P1 element,
// Sec. 7.2) and its volume from the vertex coordinates.
double tet_grads(const double X[4][3], double Gr[4][3])
{
    double E[3][3];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) E[r][c] = X[c + 1][r] - X[0][r];
    const double det = E[0][0] * (E[1][1] * E[2][2] - E[1][2] * E[2][1]) -
                       E[0][1] * (E[1][0] * E[2][2] - E[1][2] * E[2][0]) +
                       E[0][2] * (E[1][0] * E[2][1] - E[1][1] * E[2][0]);
    double I[3][3];  // rows: gradients of barycentric coordinates 1..3
    I[0][0] = (E[1][1] * E[2][2] - E[1][2] * E[2][1]) / det;
    I[0][1] = (E[0][2] * E[2][1] - E[0][1] * E[2][2]) / det;
    I[0][2] = (E[0][1] * E[1][2] - E[0][2] * E[1][1]) / det;
    I[1][0] = (E[1][2] * E[2][0] - E[1][0] * E[2][2]) / det;
    I[1][1] = (E[0][0] * E[2][2] - E[0][2] * E[2][0]) / det;
    I[1][2] = (E[0][2] * E[1][0] - E[0][0] * E[1][2]) / det;
    I[2][0] = (E[1][0] * E[2][1] - E[1][1] * E[2][0]) / det;
    I[2][1] = (E[0][1] * E[2][0] - E[0][0] * E[2][1]) / det;
    I[2][2] = (E[0][0] * E[1][1] - E[0][1] * E[1][0]) / det;
    for (int c = 0; c < 3; ++c) {
        Gr[0][c] = -(I[0][c] + I[1][c] + I[2][c]);
        for (int r = 0; r < 3; ++r) Gr[r + 1][c] = I[r][c];
    }
    return std::fabs(det) / 6.0;
}

// The FEM box [o, o+C] of a mesh: its bounding box, whose corners must be
// grid nodes, cubic, >= 5 cells wide and >= 1 cell from the outer boundary.
hyb_status find_box(const hyb_fd_grid *gr, const hyb_fem_mesh *m, Mesh *out, hyb_ctx *c)
{
    const double h = gr->h;
    if (m->n_nodes < 8 || m->n_tets < 6 || !m->xyz || !m->tet4)
        return fail(c, HYB_E_ARG, "fem mesh: empty or null arrays");
    double lo[3], hi[3];
    for (int d = 0; d < 3; ++d) { lo[d] = 1e300; hi[d] = -1e300; }
    for (int64_t i = 0; i < m->n_nodes; ++i)
        for (int d = 0; d < 3; ++d) {
            const double v = m->xyz[3 * i + d];
            if (!std::isfinite(v)) return fail(c, HYB_E_NONFINITE, "fem mesh: non-finite coordinate");
            lo[d] = std::min(lo[d], v);
            hi[d] = std::max(hi[d], v);
        }
    const double tol = 1e-7 * h;
    for (int d = 0; d < 3; ++d) {
        const double fo = (lo[d] - gr->origin[d]) / h, fc = (hi[d] - lo[d]) / h;
        out->o[d] = (int)std::lround(fo);
        out->C[d] = (int)std::lround(fc);
        if (std::fabs(fo - out->o[d]) * h > tol || std::fabs(fc - out->C[d]) * h > tol)
            return fail(c, HYB_E_MESH, "fem mesh: box corners are not grid nodes");
        if (out->C[d] < 5) return fail(c, HYB_E_MESH, "fem mesh: box must be at least 5 cells wide");
        if (out->o[d] < 1 || out->o[d] + out->C[d] > gr->n_cells[d] - 1)
            return fail(c, HYB_E_MESH, "fem mesh: box must keep at least one cell to the outer boundary");
    }
    if (out->C[0] != out->C[1] || out->C[1] != out->C[2])
        return fail(c, HYB_E_UNSUPPORTED, "fem mesh: only cubic FEM boxes are supported");
    return HYB_OK;
}

// Check that the mesh (of the box found by find_box) is the 6-tetrahedra
// split of its cubes and extract the per-cube P1 stiffness (a = 1), which
// must be the same for every cube and couple only along the 12 axis edges
// (then the FEM update is exactly an edge-conductance stencil, which the
// structured kernels use).
hyb_status analyse_kuhn(const hyb_fd_grid *gr, const hyb_fem_mesh *m, Mesh *out, hyb_ctx *c)
{
    const double h = gr->h, tol = 1e-7 * h;
    double lo[3];
    for (int d = 0; d < 3; ++d) lo[d] = gr->origin[d] + out->o[d] * h;
    const long long fx = out->C[0] + 1, fy = out->C[1] + 1, fz = out->C[2] + 1;
    const long long ncube = (long long)out->C[0] * out->C[1] * out->C[2];
    if (m->n_nodes != fx * fy * fz || m->n_tets != 6 * ncube)
        return fail(c, HYB_E_UNSUPPORTED, "fem mesh: not a 6-tetrahedra split of its box (node/tet count)");
    // lattice position of every node, must be a bijection onto the box nodes
    std::vector<int64_t> lat(m->n_nodes);
    std::vector<int64_t> owner(m->n_nodes, -1);
    for (int64_t i = 0; i < m->n_nodes; ++i) {
        long long q[3];
        for (int d = 0; d < 3; ++d) {
            const double f = (m->xyz[3 * i + d] - lo[d]) / h;
            q[d] = std::llround(f);
            if (std::fabs(f - q[d]) * h > tol) return fail(c, HYB_E_MESH, "fem mesh: node off the grid");
        }
        const int64_t L = q[0] + fx * (q[1] + fy * q[2]);
        if (owner[L] >= 0) return fail(c, HYB_E_MESH, "fem mesh: duplicate node");
        owner[L] = i;
        lat[i] = L;
    }
    // every tetrahedron: one of the 6 diagonal tetrahedra of one cube
    std::vector<uint8_t> seen(ncube, 0);
    std::vector<int64_t> tet_of(6 * ncube, -1);
    for (int64_t t = 0; t < m->n_tets; ++t) {
        long long v[4][3], s[4];
        for (int q = 0; q < 4; ++q) {
            const int32_t id = m->tet4[4 * t + q];
            if (id < 0 || id >= m->n_nodes) return fail(c, HYB_E_ARG, "fem mesh: node id out of range");
            const int64_t L = lat[id];
            v[q][0] = L % fx;
            v[q][1] = (L / fx) % fy;
            v[q][2] = L / (fx * fy);
            s[q] = v[q][0] + v[q][1] + v[q][2];
        }
        int ord[4] = {0, 1, 2, 3};
        std::sort(ord, ord + 4, [&](int a, int b) { return s[a] < s[b]; });
        int perm_code = 0, used = 0;
        bool ok = true;
        for (int q = 1; q < 4 && ok; ++q) {
            int ax = -1, nd = 0;
            for (int d = 0; d < 3; ++d) {
                const long long df = v[ord[q]][d] - v[ord[q - 1]][d];
                if (df == 1) { ax = d; ++nd; }
                else if (df != 0) ok = false;
            }
            if (nd != 1 || (used >> ax & 1)) ok = false;
            else { used |= 1 << ax; perm_code = perm_code * 3 + ax; }
        }
        if (!ok) return fail(c, HYB_E_UNSUPPORTED, "fem mesh: tetrahedron is not a cube-diagonal tetrahedron");
        static const int codes[6] = {0 * 9 + 1 * 3 + 2, 0 * 9 + 2 * 3 + 1, 1 * 9 + 0 * 3 + 2,
                                     1 * 9 + 2 * 3 + 0, 2 * 9 + 0 * 3 + 1, 2 * 9 + 1 * 3 + 0};
        int p = -1;
        for (int q = 0; q < 6; ++q)
            if (codes[q] == perm_code) p = q;
        const long long *b = v[ord[0]];
        if (b[0] >= out->C[0] || b[1] >= out->C[1] || b[2] >= out->C[2])
            return fail(c, HYB_E_MESH, "fem mesh: tetrahedron outside the box");
        const long long cube = b[0] + out->C[0] * (b[1] + (long long)out->C[1] * b[2]);
        if (seen[cube] >> p & 1) return fail(c, HYB_E_MESH, "fem mesh: duplicate tetrahedron");
        seen[cube] |= (uint8_t)(1 << p);
        tet_of[6 * cube + p] = t;
    }
    // per-cube stiffness from the element matrices; all cubes must agree
    double Kref[8][8];
    std::vector<double> mass(m->n_nodes, 0.0);
    for (long long cube = 0; cube < ncube; ++cube) {
        if (seen[cube] != 63) return fail(c, HYB_E_MESH, "fem mesh: cube not covered by its 6 tetrahedra");
        const long long ci = cube % out->C[0], cj = (cube / out->C[0]) % out->C[1],
                        ck = cube / ((long long)out->C[0] * out->C[1]);
        double K[8][8];
        std::memset(K, 0, sizeof K);
        for (int p = 0; p < 6; ++p) {
            const int64_t t = tet_of[6 * cube + p];
            double X[4][3], Gr[4][3];
            int loc[4];
            for (int q = 0; q < 4; ++q) {
                const int32_t id = m->tet4[4 * t + q];
                for (int d = 0; d < 3; ++d) X[q][d] = m->xyz[3 * id + d];
                const int64_t L = lat[id];
                const long long a = L % fx - ci, b = (L / fx) % fy - cj, cc = L / (fx * fy) - ck;
                loc[q] = (int)(a + 2 * b + 4 * cc);
            }
            const double vol = tet_grads(X, Gr);
            for (int q = 0; q < 4; ++q) {
                mass[m->tet4[4 * t + q]] += vol / 4.0;
                for (int r = 0; r < 4; ++r)
                    K[loc[q]][loc[r]] += vol * (Gr[q][0] * Gr[r][0] + Gr[q][1] * Gr[r][1] + Gr[q][2] * Gr[r][2]);
            }
        }
        if (cube == 0) std::memcpy(Kref, K, sizeof K);
        else
            for (int a = 0; a < 8; ++a)
                for (int b = 0; b < 8; ++b)
                    if (std::fabs(K[a][b] - Kref[a][b]) > 1e-9 * h)
                        return fail(c, HYB_E_UNSUPPORTED, "fem mesh: cubes with different element matrices");
    }
    for (int a = 0; a < 8; ++a)
        for (int b = 0; b < 8; ++b)
            if (a != b && __builtin_popcount(a ^ b) != 1 && std::fabs(Kref[a][b]) > 1e-9 * h)
                return fail(c, HYB_E_UNSUPPORTED, "fem mesh: element matrices couple across cube diagonals");
    // lumped mass of the FEM interior nodes must be h^3 (uniform cells)
    const double h3 = h * h * h;
    for (int64_t i = 0; i < m->n_nodes; ++i) {
        const int64_t L = lat[i];
        const long long a = L % fx, b = (L / fx) % fy, cc = L / (fx * fy);
        if (a > 0 && a < fx - 1 && b > 0 && b < fy - 1 && cc > 0 && cc < fz - 1 &&
            std::fabs(mass[i] - h3) > 1e-9 * h3)
            return fail(c, HYB_E_UNSUPPORTED, "fem mesh: non-uniform lumped mass");
    }
    for (int s1 = 0; s1 < 2; ++s1)
        for (int s0 = 0; s0 < 2; ++s0) {
            const int e = s0 + 2 * s1;
            out->w[e] = -Kref[2 * s0 + 4 * s1][1 + 2 * s0 + 4 * s1] / h;      // x-edge (y=s0, z=s1)
            out->w[4 + e] = -Kref[s0 + 4 * s1][s0 + 2 + 4 * s1] / h;          // y-edge (x=s0, z=s1)
            out->w[8 + e] = -Kref[s0 + 2 * s1][s0 + 2 * s1 + 4] / h;          // z-edge (x=s0, y=s1)
        }
    return HYB_OK;
}

// The FEM mesh: the structured path when it is the 6-tetrahedra split of its
// box (one sigma per cube), unless `general` asks for the general path; the
// general path (one sigma per tetrahedron) otherwise.
hyb_status analyse_fem(const hyb_fd_grid *gr, const hyb_fem_mesh *m, bool general, Mesh *mesh, GenHost *gh,
                       bool *gen, hyb_ctx *c)
{
    hyb_status s = find_box(gr, m, mesh, c);
    if (s) return s;
    if (!general) {
        s = analyse_kuhn(gr, m, mesh, c);
        if (s == HYB_OK) {
            *gen = false;
            return HYB_OK;
        }
        if (s == HYB_E_ARG) return s;
    }
    std::string err;
    s = analyse_general(gr, m, mesh->o, mesh->C, *gh, err);
    if (s) return fail(c, s, err);
    *gen = true;
    return HYB_OK;
}

hyb_status check_grid(const hyb_fd_grid *gr, hyb_ctx *c)
{
    if (!gr) return fail(c, HYB_E_ARG, "grid is null");
    if (!(gr->h > 0) || !std::isfinite(gr->h)) return fail(c, HYB_E_ARG, "grid: h must be positive");
    for (int d = 0; d < 3; ++d)
        if (gr->n_cells[d] < 2) return fail(c, HYB_E_ARG, "grid: need at least 2 cells per axis");
    for (int f = 0; f < 6; ++f) {
        if (gr->face[f] < 0 || gr->face[f] > 2) return fail(c, HYB_E_ARG, "grid: bad face condition");
        if (gr->face[f] == HYB_BC_SOURCE && f != 5)
            return fail(c, HYB_E_UNSUPPORTED, "grid: the source must be on the z+ face");
    }
    const double nodes = (double)(gr->n_cells[0] + 1) * (gr->n_cells[1] + 1) * (gr->n_cells[2] + 1);
    if (nodes > 4.0e9) return fail(c, HYB_E_UNSUPPORTED, "grid: too many nodes");
    return HYB_OK;
}

void setup_geo(Geo &g, const int n[3], const Mesh &m, bool has_fem, size_t esz)
{
    g.nx = n[0] + 1;
    g.ny = n[1] + 1;
    g.nz = n[2] + 1;
    const long long align = 128 / (long long)esz;  // rows start on 128-byte lines
    g.px = ceil_div(g.nx, align) * align;
    g.plane = g.px * g.ny;
    g.has_fem = has_fem ? 1 : 0;
    for (int d = 0; d < 3; ++d) {
        g.o[d] = has_fem ? m.o[d] : 0;
        g.C[d] = has_fem ? m.C[d] : 0;
        g.hlo[d] = g.o[d] + 2;
        g.hhi[d] = g.o[d] + g.C[d] - 2;
        g.hn[d] = has_fem ? g.C[d] - 3 : 0;
    }
    g.fpx = g.C[0] + 1;
    g.fplane = g.fpx * (g.C[1] + 1);
    g.hlevel = (long long)g.hn[0] * g.hn[1] * g.hn[2];
    g.nbnd = (long long)g.nx * g.ny * g.nz - (long long)(g.nx - 2) * (g.ny - 2) * (g.nz - 2);
    g.n_fi = 2 * ((long long)(g.nx - 2) * (g.ny - 2) + (long long)(g.nx - 2) * (g.nz - 2) +
                  (long long)(g.ny - 2) * (g.nz - 2));
    g.n_ec = g.nbnd - g.n_fi;
    const long long fxx = (long long)g.ny * g.nz, fyy = (long long)g.nx * g.nz, fzz = (long long)g.nx * g.ny;
    g.foff[0] = 0;
    g.foff[1] = fxx;
    g.foff[2] = 2 * fxx;
    g.foff[3] = 2 * fxx + fyy;
    g.foff[4] = 2 * fxx + 2 * fyy;
    g.foff[5] = 2 * fxx + 2 * fyy + fzz;
    g.ftot = 2 * (fxx + fyy + fzz);
    if (has_fem) {
        const long long L1 = g.C[0] - 4 + 1, L2 = g.C[0] + 1;
        g.nwd = L1 * L1 * L1 - (L1 - 2) * (L1 - 2) * (L1 - 2);
        g.nwo = L2 * L2 * L2 - (L2 - 2) * (L2 - 2) * (L2 - 2);
    } else {
        g.nwd = g.nwo = 0;
    }
    // x tiles start at multiples of the tile width (x = 0 included: no stencil
    // row), so that they cover the interior [1, nx-2]
    g.fdm_tx[0] = (int)ceil_div(g.nx - 1, fwd_tile_x(esz));
    g.fdm_tx[1] = (int)ceil_div(g.nx - 1, TX_FDM);
    g.fdm_ty = (int)ceil_div(g.ny - 2, TY_FDM);
    // Planes per z chunk, measured per precision and sweep on 257^3 grids
    // (us per step).  Adjoint, chunks of 4 / 6 / 8 / 12 / 16: FP64 110.9 /
    // 112.7 / 106.5 / 119.3 / 106.1; FP32 (6 / 8 / 12) 94.3 / 95.8 / 100.6.
    // Forward with the column-pair tile and its face rows, chunks of 3 / 4 /
    // 6 / 8 / 10 / 12 / 16: FP64 82.9 / 79.9 / 80.8 / 78.3 / 85.0 / 79.9 /
    // 87.9; FP32 (4 / 6 / 8) 75.0 / 73.6 / 80.3, with the tile of four FP32
    // columns per lane 73.1 / 69.7 / 75.0.  Chunk counts that divide into
    // whole rounds of resident blocks balance best; small grids keep 4 planes
    // for parallelism.
    const bool big = g.nz > 200;
    const int zc[2] = {big ? (esz == 4 ? 6 : 8) : 4, big ? (esz == 4 ? 6 : 8) : 4};
    for (int a = 0; a < 2; ++a) {
        g.zc_fdm[a] = zc[a];
        g.fdm_zt[a] = (int)ceil_div(g.nz - 2, zc[a]);
        g.n_fdm_blocks[a] = (int)((long long)g.fdm_tx[a] * g.fdm_ty * g.fdm_zt[a]);
    }
    if (has_fem) {
        g.fem_tiles[0] = (int)ceil_div(g.C[0] - 1, TX_FEM);
        g.fem_tiles[1] = (int)ceil_div(g.C[1] - 1, TY_FEM);
        const long long fxy = (long long)g.fem_tiles[0] * g.fem_tiles[1];
        const int zf = 4;  // as for the FDM tiles: measured best
        g.zc_fem = zf;
        g.fem_tiles[2] = (int)ceil_div(g.C[2] - 1, zf);
        g.n_fem_tiles = (int)(fxy * g.fem_tiles[2]);
        // a multiple of 8 for the XCD remap (the extra blocks exit at once)
        g.n_fem_blocks = (g.n_fem_tiles + 7) / 8 * 8;
    } else {
        g.fem_tiles[0] = g.fem_tiles[1] = g.fem_tiles[2] = 0;
        g.zc_fem = 1;
        g.n_fem_blocks = g.n_fem_tiles = 0;
    }
    g.bnd_blocks = (int)ceil_div(g.nbnd + g.nwd + g.nwo, BLOCK);  // informational
    g.fem_n = has_fem ? (long long)(g.C[0] + 1) * (g.C[1] + 1) * (g.C[2] + 1) : 0;
    g.gen = 0;
}

// A general mesh of the same box: no structured FEM tiles, exchanges or
// history box; the history holds the nodes [0, nH) of the device numbering.
void setup_geo_gen(Geo &g, const GenHost &gh)
{
    g.gen = 1;
    g.n_fem_blocks = g.n_fem_tiles = 0;
    g.fem_tiles[0] = g.fem_tiles[1] = g.fem_tiles[2] = 0;
    g.nwd = g.nwo = 0;
    g.hn[0] = g.hn[1] = g.hn[2] = 0;
    g.hlevel = gh.nH;
    g.fem_n = gh.fn;
    g.bnd_blocks = (int)ceil_div(g.nbnd, BLOCK);
}

size_t field_bytes(const Geo &g, size_t esz) { return (size_t)g.plane * g.nz * esz; }
size_t fem_bytes(const Geo &g, size_t esz) { return g.has_fem ? (size_t)g.fem_n * esz : 0; }
size_t cube_count(const Geo &g) { return (size_t)g.C[0] * g.C[1] * g.C[2]; }

int face_types(const hyb_ctx *c, int step)
{
    int t = 0;
    for (int f = 0; f < 6; ++f) {
        int v;
        if (c->bc[f] == HYB_BC_NEUMANN) v = F_NEUMANN;
        else if (c->bc[f] == HYB_BC_SOURCE) v = (step >= 0 && step < c->k_on) ? F_SOURCE : F_ABC;
        else v = F_ABC;
        t |= v << (2 * f);
    }
    return t;
}

hyb_status dmalloc(hyb_ctx *c, void **p, size_t bytes)
{
    if (*p) return HYB_OK;
    if (hipMalloc(p, bytes ? bytes : 8) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(c, HYB_E_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    }
    return HYB_OK;
}

void dfree(void *&p)
{
    if (p) (void)hipFree(p);
    p = nullptr;
}

template <typename V>
hyb_status upload(hyb_ctx *c, V *&dst, const std::vector<V> &src)
{
    hyb_status s = dmalloc(c, (void **)&dst, std::max<size_t>(src.size(), 1) * sizeof(V));
    if (s) return s;
    if (!src.empty()) HIPCHK(c, hipMemcpy(dst, src.data(), src.size() * sizeof(V), hipMemcpyHostToDevice));
    return HYB_OK;
}

// Device tables of a general mesh (hyb_gen.h); the omega_diamond / omega_o
// nodes get their padded grid indices here.
hyb_status upload_gen(hyb_ctx *c, const GenHost &gh)
{
    GenDev &d = c->gd;
    d.fn = gh.fn; d.nA = gh.nA; d.nH = gh.nH; d.nR = gh.nR; d.ntet = gh.ntet;
    d.nslice = gh.nslice; d.nnz = gh.nnz; d.nE = gh.nE;
    c->gen_all_grid = gh.all_grid;
    const Geo &g = c->g;
    std::vector<int64_t> wdg(gh.nA), wog(gh.fn - gh.nR);
    auto pad = [&](long long n) {
        return gh.gq[3 * n] + g.px * gh.gq[3 * n + 1] + g.plane * (long long)gh.gq[3 * n + 2];
    };
    for (long long n = 0; n < gh.nA; ++n) wdg[n] = pad(n);
    for (long long n = gh.nR; n < gh.fn; ++n) wog[n - gh.nR] = pad(n);
    hyb_status s = HYB_OK;
    if (!s) s = upload(c, d.soff, gh.soff);
    if (!s) s = upload(c, d.eoff, gh.eoff);
    if (!s) s = upload(c, d.col, gh.col);
    if (!s) s = upload(c, d.eid, gh.eid);
    if (!s) s = upload(c, d.cptr, gh.cptr);
    if (!s) s = upload(c, d.ctet, gh.ctet);
    if (!s) s = upload(c, d.cw, gh.cw);
    if (!s) s = upload(c, d.minv, gh.minv);
    if (!s) s = upload(c, d.ke6, gh.ke6);
    if (!s) s = upload(c, d.pvol, gh.pvol);
    if (!s) s = upload(c, d.tetE, gh.tetE);
    if (!s) s = upload(c, d.orig_of_dev, gh.orig_of_dev);
    if (!s) s = upload(c, d.grid_lin, gh.grid_lin);
    if (!s) s = upload(c, d.wdg, wdg);
    if (!s) s = upload(c, d.wog, wog);
    if (!s) s = dmalloc(c, &d.kap, (size_t)std::max<long long>(gh.nnz, 1) * c->esz);
    if (!s) s = dmalloc(c, &d.cn, (size_t)gh.fn * c->esz);
    if (!s) s = dmalloc(c, &d.nu[0], (size_t)gh.fn * c->esz);
    if (!s) s = dmalloc(c, &d.nu[1], (size_t)gh.fn * c->esz);
    if (!s) s = dmalloc(c, (void **)&d.E, (size_t)std::max<long long>(gh.nE, 1) * sizeof(double));
    return s;
}

void free_gen(GenDev &d)
{
    dfree((void *&)d.soff); dfree((void *&)d.eoff); dfree((void *&)d.col); dfree((void *&)d.eid);
    dfree((void *&)d.cptr); dfree((void *&)d.ctet); dfree((void *&)d.cw); dfree((void *&)d.minv);
    dfree((void *&)d.ke6); dfree((void *&)d.pvol); dfree((void *&)d.E); dfree((void *&)d.tetE);
    dfree((void *&)d.orig_of_dev); dfree((void *&)d.grid_lin); dfree((void *&)d.wdg);
    dfree((void *&)d.wog); dfree(d.kap); dfree(d.cn); dfree(d.nu[0]); dfree(d.nu[1]);
}

template <typename T>
Step<T> make_step(const hyb_ctx *c)
{
    Step<T> s;
    std::memset(&s, 0, sizeof s);
    s.g = c->g;
    s.acube = (const T *)c->acube;
    s.c2 = (T)((c->dt / c->h) * (c->dt / c->h));
    s.ic2 = (T)1 / s.c2;
    s.w2 = 1.0;
    s.minv = c->vm ? (const T *)c->minv : nullptr;
    s.r = (T)((c->h - c->dt) / (c->h + c->dt));
    for (int q = 0; q < 12; ++q) s.w[q] = (T)c->mesh.w[q];
    s.dt = c->dt;
    s.h2 = c->h * c->h;
    return s;
}

// History pointer of FEM level L (null when not kept).  Store mode 0 keeps
// every level; the checkpoint modes keep the levels of one segment
// [seg*K, seg*K + K - 1] of the sqrt(nt) segmentation.
template <typename T>
T *hist_ptr(hyb_ctx *c, int L)
{
    if (!c->g.has_fem) return nullptr;
    if (c->store_mode == 0) return (T *)c->hist + (long long)L * c->g.hlevel;
    const int lo = c->cur_seg * c->ckK;
    if (L < lo || L >= lo + c->ckK) return nullptr;
    return (T *)c->hist + (long long)(L - lo) * c->g.hlevel;
}

// Bytes of the 16-bit block-scaled form of n FP32 values: int16 values and
// one FP32 scale per 64, each part rounded up to 256 bytes.
size_t q16_values_bytes(size_t n) { return (2 * n + 255) / 256 * 256; }
size_t q16_bytes(size_t n) { return q16_values_bytes(n) + (4 * ((n + 63) / 64) + 255) / 256 * 256; }

// One checkpoint: u^L in field precision plus the second level (mode 1:
// u^{L-1}, or the FP32 increment d^L, in field precision; mode 2: d^L in
// BF16; mode 3: d^L in the 16-bit block-scaled form), grid then FEM part.
size_t ckpt_slot_bytes(const Geo &g, size_t esz, int mode)
{
    const size_t fb = field_bytes(g, esz), vb = fem_bytes(g, esz);
    if (mode == 2) return (fb + vb) + (fb + vb) / 2;
    if (mode == 3) return (fb + vb) + q16_bytes(fb / 4) + q16_bytes(vb / 4);
    return 2 * (fb + vb);
}

// Save the state at level L (u^L in buffer ib; u^{L-1} in ia, or in FP32 the
// increment d^L in slot L & 1) as checkpoint number q.  Store mode 1 copies
// both parts in field precision; mode 2 (FP32 only) keeps d^L in BF16, mode 3
// (FP32 only) in the 16-bit block-scaled form.
template <typename T>
hyb_status save_ckpt(hyb_ctx *c, int q, int L, int ia, int ib)
{
    const Geo &g = c->g;
    const size_t fb = field_bytes(g, sizeof(T)), vb = fem_bytes(g, sizeof(T));
    char *base = (char *)c->ckpt + (size_t)q * ckpt_slot_bytes(g, sizeof(T), c->store_mode);
    const hipStream_t st = c->stream;
    const bool inc = incr_form<T>();
    void *u1 = inc ? c->D[L & 1] : c->U[ia], *v1 = inc ? c->VD[L & 1] : c->V[ia];
    HIPCHK(c, hipMemcpyAsync(base, c->U[ib], fb, hipMemcpyDeviceToDevice, st));
    if (vb) HIPCHK(c, hipMemcpyAsync(base + fb, c->V[ib], vb, hipMemcpyDeviceToDevice, st));
    if (c->store_mode == 1) {
        HIPCHK(c, hipMemcpyAsync(base + fb + vb, u1, fb, hipMemcpyDeviceToDevice, st));
        if (vb) HIPCHK(c, hipMemcpyAsync(base + 2 * fb + vb, v1, vb, hipMemcpyDeviceToDevice, st));
    } else if (c->store_mode == 3) {
        char *p = base + fb + vb;
        const size_t nf = fb / 4, nv = vb / 4;
        launch_pack_q16(u1, (int16_t *)p, (float *)(p + q16_values_bytes(nf)), (long long)nf, st);
        p += q16_bytes(nf);
        if (vb) launch_pack_q16(v1, (int16_t *)p, (float *)(p + q16_values_bytes(nv)), (long long)nv, st);
    } else {
        uint16_t *half = (uint16_t *)(base + fb + vb);
        launch_pack_bf16(u1, half, (long long)(fb / sizeof(float)), st);
        if (vb) launch_pack_bf16(v1, half + fb / sizeof(float), (long long)(vb / sizeof(float)), st);
    }
    return HYB_OK;
}

// Restore checkpoint q (level L = q K) into buffer 1 (u^L) and buffer 0
// (u^{L-1}), or in FP32 the increment slot L & 1.
template <typename T>
hyb_status load_ckpt(hyb_ctx *c, int q)
{
    const Geo &g = c->g;
    const size_t fb = field_bytes(g, sizeof(T)), vb = fem_bytes(g, sizeof(T));
    const char *base = (const char *)c->ckpt + (size_t)q * ckpt_slot_bytes(g, sizeof(T), c->store_mode);
    const hipStream_t st = c->stream;
    const int L = q * c->ckK;
    const bool inc = incr_form<T>();
    void *u1 = inc ? c->D[L & 1] : c->U[0], *v1 = inc ? c->VD[L & 1] : c->V[0];
    HIPCHK(c, hipMemcpyAsync(c->U[1], base, fb, hipMemcpyDeviceToDevice, st));
    if (vb) HIPCHK(c, hipMemcpyAsync(c->V[1], base + fb, vb, hipMemcpyDeviceToDevice, st));
    if (c->store_mode == 1) {
        HIPCHK(c, hipMemcpyAsync(u1, base + fb + vb, fb, hipMemcpyDeviceToDevice, st));
        if (vb) HIPCHK(c, hipMemcpyAsync(v1, base + 2 * fb + vb, vb, hipMemcpyDeviceToDevice, st));
    } else if (c->store_mode == 3) {
        const char *p = base + fb + vb;
        const size_t nf = fb / 4, nv = vb / 4;
        launch_unpack_q16((const int16_t *)p, (const float *)(p + q16_values_bytes(nf)), u1, (long long)nf, st);
        p += q16_bytes(nf);
        if (vb)
            launch_unpack_q16((const int16_t *)p, (const float *)(p + q16_values_bytes(nv)), v1, (long long)nv, st);
    } else {
        const uint16_t *half = (const uint16_t *)(base + fb + vb);
        launch_unpack_bf16(half, u1, (long long)(fb / sizeof(float)), st);
        if (vb) launch_unpack_bf16(half + fb / sizeof(float), v1, (long long)(vb / sizeof(float)), st);
    }
    return HYB_OK;
}

// Arguments of forward step k (levels k-1, k, k+1 in buffers ia, ib, ic).
template <typename T>
Step<T> fwd_step_args(hyb_ctx *c, int k, int ia, int ib, int ic, double *obs)
{
    const long long nface = (long long)c->g.nx * c->g.ny;
    Step<T> s = make_step<T>(c);
    s.Ua = (const T *)c->U[ia]; s.Ub = (const T *)c->U[ib]; s.Uc = (T *)c->U[ic];
    s.Va = (const T *)c->V[ia]; s.Vb = (const T *)c->V[ib]; s.Vc = (T *)c->V[ic];
    if (incr_form<T>()) {
        s.Da = (const T *)c->D[k & 1]; s.Dc = (T *)c->D[(k + 1) & 1];
        s.VDa = (const T *)c->VD[k & 1]; s.VDc = (T *)c->VD[(k + 1) & 1];
    }
    s.types1 = face_types(c, k);
    // Taylor start: the first step weights dt^2 by 1/2 in the leapfrog rows
    // (grid, FEM and ghost rows, the source flux included); the absorbing
    // rows do not contain dt^2 and are unchanged
    s.w2 = (c->sweep_taylor && k == 0) ? 0.5 : 1.0;
    s.c2 = (T)(s.w2 * (c->dt / c->h) * (c->dt / c->h));
    s.ic2 = (T)1 / s.c2;
    const double fluxscale = s.w2 * 2.0 * c->dt * c->dt / c->h;
    if (c->src.kind == 0) {
        s.flux = nullptr;
        s.srcterm = (T)(fluxscale * std::sin(c->src.omega * ((double)k * c->dt)));
    } else {
        s.flux = k < c->k_on ? c->src.flux_dev + (long long)k * nface : nullptr;
        s.fluxscale = fluxscale;
        s.srcterm = 0;
    }
    s.obs = obs ? obs + (long long)(k + 1) * nface : nullptr;
    s.hist = hist_ptr<T>(c, k + 1);
    return s;
}

// Arguments of the adjoint step that computes level k (multipliers of levels
// k+2, k+1, k in buffers ia, ib, ic).
template <typename T>
Step<T> adj_step_args(hyb_ctx *c, int k, int ia, int ib, int ic, const double *res, int mode)
{
    const long long nface = (long long)c->g.nx * c->g.ny;
    Step<T> s = make_step<T>(c);
    s.seed_mode = mode;
    s.G = c->G;
    s.Ua = (const T *)c->P[ia]; s.Ub = (const T *)c->P[ib]; s.Uc = (T *)c->P[ic];
    s.Va = (const T *)c->Q[ia]; s.Vb = (const T *)c->Q[ib]; s.Vc = (T *)c->Q[ic];
    s.Fa = (const T *)c->F[ia]; s.Fb = (const T *)c->F[ib]; s.Fc = (T *)c->F[ic];
    s.Pw = (T *)c->P[ib];
    if (incr_form<T>()) {
        s.Da = (const T *)c->E[(k + 1) & 1]; s.Dc = (T *)c->E[k & 1];
        s.VDa = (const T *)c->QE[(k + 1) & 1]; s.VDc = (T *)c->QE[k & 1];
    }
    s.types0 = face_types(c, k - 1);
    s.types1 = face_types(c, k);
    s.types2 = face_types(c, k + 1);
    s.level_rows = k >= 1;
    // level 0 is read by the rows of step 0 only: with the Taylor start their
    // dt^2 weight 1/2 enters the transposed rows and the gradient term
    s.w2 = (c->sweep_taylor && k == 0) ? 0.5 : 1.0;
    s.c2 = (T)(s.w2 * (c->dt / c->h) * (c->dt / c->h));
    s.ic2 = (T)1 / s.c2;
    s.res = (mode == 0 && k == 0) ? nullptr : res + (long long)k * nface;
    s.hist = hist_ptr<T>(c, k);
    if (c->vm && c->store_mode == 0 && c->g.has_fem) {
        // dJ/dm needs the history levels k+1, k, k-1 of the node (full history)
        s.Gm = c->Gm;
        s.hnext = k < c->nt ? hist_ptr<T>(c, k + 1) : nullptr;
        s.hprev = k >= 1 ? hist_ptr<T>(c, k - 1) : (const T *)c->hm1;
    }
    return s;
}

// The general FEM step that goes with a grid step: the same buffers (see
// GenStep), the device tables of the mesh.
template <typename T>
GenStep<T> gen_args(const hyb_ctx *c, const Step<T> &s)
{
    GenStep<T> q;
    std::memset(&q, 0, sizeof q);
    const GenDev &d = c->gd;
    q.fn = d.fn; q.nA = d.nA; q.nH = d.nH; q.nR = d.nR;
    q.px = c->g.px; q.plane = c->g.plane;
    q.soff = d.soff; q.eoff = d.eoff; q.col = d.col;
    q.kap = (const T *)d.kap; q.cn = (const T *)d.cn;
    q.wdg = d.wdg; q.wog = d.wog;
    q.Ub = s.Ub; q.Uc = s.Uc;
    q.Va = s.Va; q.Vb = s.Vb; q.Vc = s.Vc;
    q.VDa = s.VDa; q.VDc = s.VDc;
    q.hist = s.hist;
    q.E = d.E;
    q.c2 = s.c2;
    q.cs = (T)s.w2;
    return q;
}

// The adjoint general FEM step computing level k: nu^{k+1} from the launch
// of level k+1 (parity buffers), nu^k for the launch of level k-1 with the
// weight of step k-1.
template <typename T>
GenStep<T> gen_adj_args(const hyb_ctx *c, const Step<T> &s, int k)
{
    GenStep<T> q = gen_args<T>(c, s);
    q.nu_in = (const T *)c->gd.nu[(k + 1) & 1];
    q.nu_out = (T *)c->gd.nu[k & 1];
    q.cs_prev = (T)((c->sweep_taylor && k - 1 == 0) ? 0.5 : 1.0);
    return q;
}

// History level L of the FEM nodes [0, nH) from a FEM level (general mesh).
template <typename T>
hyb_status gen_hist_level(hyb_ctx *c, const void *V, T *h)
{
    HIPCHK(c, hipMemcpyAsync(h, V, (size_t)c->gd.nH * sizeof(T), hipMemcpyDeviceToDevice, c->stream));
    return HYB_OK;
}

// Zero the multipliers and the gradient accumulator; the misfit J of mode 0.
template <typename T>
hyb_status adj_setup(hyb_ctx *c, const double *res, int mode)
{
    const Geo &g = c->g;
    const hipStream_t st = c->stream;
    const size_t fb = field_bytes(g, sizeof(T)), vb = fem_bytes(g, sizeof(T));
    for (int q = 0; q < 3; ++q) {
        HIPCHK(c, hipMemsetAsync(c->P[q], 0, fb, st));
        HIPCHK(c, hipMemsetAsync(c->F[q], 0, (size_t)g.ftot * sizeof(T), st));
        if (g.has_fem) HIPCHK(c, hipMemsetAsync(c->Q[q], 0, vb, st));
    }
    if (incr_form<T>())
        for (int q = 0; q < 2; ++q) {
            HIPCHK(c, hipMemsetAsync(c->E[q], 0, fb, st));
            if (g.has_fem) HIPCHK(c, hipMemsetAsync(c->QE[q], 0, vb, st));
        }
    if (c->gen) {
        HIPCHK(c, hipMemsetAsync(c->gd.E, 0, std::max<long long>(c->gd.nE, 1) * sizeof(double), st));
        // nu^{nt+1} = 0 (no rows at level nt+1); omega_o entries stay 0
        for (int q = 0; q < 2; ++q) HIPCHK(c, hipMemsetAsync(c->gd.nu[q], 0, (size_t)c->gd.fn * sizeof(T), st));
    }
    else if (g.has_fem) HIPCHK(c, hipMemsetAsync(c->G, 0, cube_count(g) * sizeof(double), st));
    if (c->vm && c->store_mode == 0) HIPCHK(c, hipMemsetAsync(c->Gm, 0, g.fem_n * sizeof(double), st));
    if (mode == 0) launch_misfit(g, res, c->nt, c->dt, c->h, c->partials, c->scal, S_JMIS, st);
    else HIPCHK(c, hipMemsetAsync(c->scal + S_JMIS, 0, sizeof(double), st));
    return HYB_OK;
}

// Zero the wavefields, load initial levels, record level 0.
template <typename T>
hyb_status fwd_setup(hyb_ctx *c, double *obs)
{
    const Geo &g = c->g;
    const hipStream_t st = c->stream;
    const size_t fb = field_bytes(g, sizeof(T)), vb = fem_bytes(g, sizeof(T));
    for (int q = 0; q < 3; ++q) {
        HIPCHK(c, hipMemsetAsync(c->U[q], 0, fb, st));
        if (g.has_fem) HIPCHK(c, hipMemsetAsync(c->V[q], 0, vb, st));
    }
    if (incr_form<T>())
        for (int q = 0; q < 2; ++q) {
            HIPCHK(c, hipMemsetAsync(c->D[q], 0, fb, st));
            if (g.has_fem) HIPCHK(c, hipMemsetAsync(c->VD[q], 0, vb, st));
        }
    c->sweep_taylor = false;
    if (c->taylor) {
        // u^0 = f0 and the virtual level u^{-1} = f0 - dt f1 (FP64 fields), or
        // the increment d^0 = u^0 - u^{-1} = dt f1 (FP32 increment form)
        Geo gg = g;
        if (c->gen) gg.has_fem = 0;
        launch_load_level<T>(gg, c->tf0, (T *)c->U[1], (T *)c->V[1], st);
        if (c->gen) launch_gen_load<T>(c->gd, c->tf0, (T *)c->V[1], st);
        if (incr_form<T>()) {
            launch_load_combo<T>(gg, nullptr, c->tf1, c->dt, (T *)c->D[0], (T *)c->VD[0], st);
            if (c->gen) launch_gen_load_combo<T>(c->gd, nullptr, c->tf1, c->dt, (T *)c->VD[0], st);
        } else {
            launch_load_combo<T>(gg, c->tf0, c->tf1, -c->dt, (T *)c->U[0], (T *)c->V[0], st);
            if (c->gen) launch_gen_load_combo<T>(c->gd, c->tf0, c->tf1, -c->dt, (T *)c->V[0], st);
        }
        c->sweep_taylor = true;
    } else if (c->ic_set) {
        // a general mesh loads its FEM part through its node -> grid map
        Geo gg = g;
        if (c->gen) gg.has_fem = 0;
        if (c->ic_u0) {
            launch_load_level<T>(gg, c->ic_u0, (T *)c->U[1], (T *)c->V[1], st);
            if (c->gen) launch_gen_load<T>(c->gd, c->ic_u0, (T *)c->V[1], st);
        }
        if (incr_form<T>()) {
            launch_load_incr<T>(gg, c->ic_u0, c->ic_um1, (T *)c->D[0], (T *)c->VD[0], st);
            if (c->gen) launch_gen_load_incr<T>(c->gd, c->ic_u0, c->ic_um1, (T *)c->VD[0], st);
        } else if (c->ic_um1) {
            launch_load_level<T>(gg, c->ic_um1, (T *)c->U[0], (T *)c->V[0], st);
            if (c->gen) launch_gen_load<T>(c->gd, c->ic_um1, (T *)c->V[0], st);
        }
        c->ic_set = false;
        c->ic_u0 = c->ic_um1 = nullptr;
    }
    c->cur_seg = c->store_mode ? c->nt / c->ckK : 0;
    if (c->vm && c->store_mode == 0) {
        // history box of the level u^{-1}: the second difference of step 0
        if (incr_form<T>()) launch_hist_diff<T>(g, (const T *)c->V[1], (const T *)c->VD[0], (T *)c->hm1, st);
        else launch_hist_diff<T>(g, (const T *)c->V[0], nullptr, (T *)c->hm1, st);
    }
    if (obs) launch_record_face<T>(g, (const T *)c->U[1], obs, st);
    if (T *h0 = hist_ptr<T>(c, 0)) {
        if (c->gen) return gen_hist_level<T>(c, c->V[1], h0);
        launch_hist_level<T>(g, (const T *)c->V[1], h0, st);
    }
    return HYB_OK;
}

// Forward steps k in [k0, k1) on buffers (ia, ib, ic) (levels k-1, k, k+1);
// records the trace when obs is given and the FEM history where kept; saves
// a checkpoint at every multiple of K when `save` is set.
template <typename T>
hyb_status fwd_steps(hyb_ctx *c, int k0, int k1, int &ia, int &ib, int &ic, double *obs, bool save)
{
    const hipStream_t st = c->stream;
    // The edge and corner rows of step k run as extra blocks of the interior
    // launch of step k+1 (nothing in that launch reads them), so the
    // boundary launch of a step remains only while some face has reflecting
    // rows.  They run in a launch of their own before a checkpoint, at the
    // end, and when the face conditions of the two steps differ (the edge
    // rows recompute reflecting face rows from the levels of their own step,
    // which the next launch overwrites on faces that absorb there).
    Step<T> prev{};
    bool lag = false;
    for (int k = k0; k < k1; ++k) {
        const Step<T> s = fwd_step_args<T>(c, k, ia, ib, ic, obs);
        if (lag && prev.types1 != s.types1) {
            launch_bnd_fwd_edges<T>(prev, st);
            lag = false;
        }
        const EdgeArgs<T> pe = edge_args(prev);
        if (c->gen) {
            const GenStep<T> gs = gen_args<T>(c, s);
            launch_interior<T>(s, false, st, lag ? &pe : nullptr, &gs);
        } else {
            launch_interior<T>(s, false, st, lag ? &pe : nullptr);
        }
        launch_bnd_fwd_faces<T>(s, st);
        prev = s;
        lag = true;
        const int t = ia; ia = ib; ib = ic; ic = t;
        if (save && (k + 1) % c->ckK == 0) {
            launch_bnd_fwd_edges<T>(prev, st);
            lag = false;
            hyb_status r = save_ckpt<T>(c, (k + 1) / c->ckK, k + 1, ia, ib);
            if (r) return r;
        }
    }
    if (lag) launch_bnd_fwd_edges<T>(prev, st);
    return HYB_OK;
}

template <typename T>
hyb_status run_forward(hyb_ctx *c, double *obs)
{
    // the forward sweep ends in the last segment, whose history it keeps
    const bool ck = c->store_mode != 0;
    hyb_status r0 = fwd_setup<T>(c, obs);
    if (r0) return r0;
    int ia = 0, ib = 1, ic = 2;
    if (ck) {
        hyb_status r = save_ckpt<T>(c, 0, 0, ia, ib);
        if (r) return r;
    }
    hyb_status r = fwd_steps<T>(c, 0, c->nt, ia, ib, ic, obs, ck);
    if (r) return r;
    c->last_u = ib;
    c->u_valid = true;
    HIPCHK(c, hipGetLastError());
    return HYB_OK;
}

// Make the history hold the segment of level L (checkpoint modes): restore
// its checkpoint and recompute its levels.
template <typename T>
hyb_status load_segment(hyb_ctx *c, int L)
{
    const int seg = L / c->ckK;
    if (seg == c->cur_seg) return HYB_OK;
    hyb_status r = load_ckpt<T>(c, seg);
    if (r) return r;
    c->cur_seg = seg;
    c->u_valid = false;
    const int lo = seg * c->ckK, hi = std::min(lo + c->ckK - 1, c->nt);
    if (T *h0 = hist_ptr<T>(c, lo)) {
        if (c->gen) {
            hyb_status r2 = gen_hist_level<T>(c, c->V[1], h0);
            if (r2) return r2;
        } else {
            launch_hist_level<T>(c->g, (const T *)c->V[1], h0, c->stream);
        }
    }
    int ia = 0, ib = 1, ic = 2;
    return fwd_steps<T>(c, lo, hi, ia, ib, ic, nullptr, false);
}

template <typename T>
hyb_status run_adjoint(hyb_ctx *c, const double *res, int mode)
{
    const Geo &g = c->g;
    const hipStream_t st = c->stream;
    hyb_status r0 = adj_setup<T>(c, res, mode);
    if (r0) return r0;
    int ia = 0, ib = 1, ic = 2;
    for (int k = c->nt; k >= 0; --k) {
        if (c->store_mode != 0 && g.has_fem) {
            hyb_status r = load_segment<T>(c, k);
            if (r) return r;
        }
        const Step<T> s = adj_step_args<T>(c, k, ia, ib, ic, res, mode);
        if (c->gen) {
            const GenStep<T> gs = gen_adj_args<T>(c, s, k);
            launch_bnd_adj<T>(s, st, &gs);
            launch_interior<T>(s, true, st, nullptr, &gs);
        } else {
            launch_bnd_adj<T>(s, st);
            launch_interior<T>(s, true, st);
        }
        const int t = ia; ia = ib; ib = ic; ic = t;
    }
    c->last_p = ib;
    HIPCHK(c, hipGetLastError());
    return HYB_OK;
}

hyb_status ensure_trace_bufs(hyb_ctx *c, int nt)
{
    if ((size_t)nt + 1 > c->tracebuf_levels) {
        dfree((void *&)c->obsbuf);
        dfree((void *&)c->resbuf);
        c->tracebuf_levels = 0;
        const size_t b = (size_t)(nt + 1) * c->g.nx * c->g.ny * sizeof(double);
        hyb_status s = dmalloc(c, (void **)&c->obsbuf, b);
        if (s) return s;
        s = dmalloc(c, (void **)&c->resbuf, b);
        if (s) return s;
        c->tracebuf_levels = (size_t)nt + 1;
    }
    return HYB_OK;
}

}  // namespace

extern "C" {

hyb_status hyb_create(const hyb_fd_grid *grid, const hyb_fem_mesh *fem, const hyb_overlap *overlap,
                      const hyb_opts *opts, hyb_ctx **out)
{
    if (!out) return fail(nullptr, HYB_E_ARG, "out is null");
    *out = nullptr;
    hyb_status s = check_grid(grid, nullptr);
    if (s) return s;
    Mesh mesh;
    GenHost gh;
    bool gen = false;
    if (fem) {
        if (!overlap || overlap->width_cells != 2)
            return fail(nullptr, HYB_E_UNSUPPORTED, "overlap: the method uses a two-element overlap");
        s = analyse_fem(grid, fem, opts && opts->fem_general, &mesh, &gh, &gen, nullptr);
        if (s) return s;
    }
    hyb_ctx *c = new hyb_ctx();
    for (int d = 0; d < 3; ++d) c->n[d] = grid->n_cells[d];
    c->h = grid->h;
    for (int f = 0; f < 6; ++f) c->bc[f] = grid->face[f];
    if (opts) {
        if (opts->field_f32 < 0 || opts->field_f32 > 1 || opts->store_mode < 0 || opts->store_mode > 3 ||
            !std::isfinite(opts->gamma) || opts->gamma < 0 || !(opts->alpha_rel > 0)) {
            delete c;
            return fail(nullptr, HYB_E_ARG, "opts: invalid options");
        }
        if (opts->store_mode >= 2 && !opts->field_f32) {
            delete c;
            return fail(nullptr, HYB_E_UNSUPPORTED, "opts: 16-bit checkpoint increments need FP32 wavefields");
        }
        c->f32 = opts->field_f32;
        c->store_mode = opts->store_mode;
        c->gamma = opts->gamma;
        c->alpha_rel = opts->alpha_rel;
        c->stream = (hipStream_t)opts->hip_stream;
        if (opts->cg_max_trials < 0 || opts->cg_max_trials > 60) {
            delete c;
            return fail(nullptr, HYB_E_ARG, "opts: cg_max_trials must be in [0, 60]");
        }
        if (opts->cg_max_trials > 0) c->max_trials = opts->cg_max_trials;
    }
    c->esz = c->f32 ? 4 : 8;
    c->mesh = mesh;
    setup_geo(c->g, c->n, mesh, fem != nullptr, c->esz);
    c->gen = gen;
    if (gen) setup_geo_gen(c->g, gh);
    c->npar = gen ? gh.ntet : (long long)cube_count(c->g);
    const size_t fb = field_bytes(c->g, c->esz), vb = fem_bytes(c->g, c->esz);
    const size_t nc = (size_t)c->npar;
    s = HYB_OK;
    for (int q = 0; q < 3 && !s; ++q) s = dmalloc(c, &c->U[q], fb);
    if (!s && c->g.has_fem)
        for (int q = 0; q < 3 && !s; ++q) s = dmalloc(c, &c->V[q], vb);
    if (c->f32) {
        for (int q = 0; q < 2 && !s; ++q) s = dmalloc(c, &c->D[q], fb);
        if (!s && c->g.has_fem)
            for (int q = 0; q < 2 && !s; ++q) s = dmalloc(c, &c->VD[q], vb);
    }
    if (!s && c->g.has_fem && !gen) s = dmalloc(c, &c->acube, nc * c->esz);
    if (!s && c->g.has_fem) s = dmalloc(c, (void **)&c->sig, nc * sizeof(double));
    if (!s && gen) s = upload_gen(c, gh);
    if (!s) s = dmalloc(c, (void **)&c->partials, MAX_PARTIALS * sizeof(double));
    if (!s) s = dmalloc(c, (void **)&c->scal, S_NSCAL * sizeof(double));
    if (s) {
        g_create_err = c->err;
        hyb_destroy(c);
        return s;
    }
    if (hipMemsetAsync(c->scal, 0, S_NSCAL * sizeof(double), c->stream) != hipSuccess) {
        hyb_destroy(c);
        return fail(nullptr, HYB_E_DEVICE, "hipMemset failed");
    }
    *out = c;
    return HYB_OK;
}

void hyb_destroy(hyb_ctx *c)
{
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    for (int q = 0; q < 3; ++q) {
        dfree(c->U[q]); dfree(c->V[q]); dfree(c->P[q]); dfree(c->Q[q]); dfree(c->F[q]);
    }
    for (int q = 0; q < 2; ++q) {
        dfree(c->D[q]);
        dfree(c->VD[q]);
        dfree(c->E[q]);
        dfree(c->QE[q]);
    }
    dfree(c->acube);
    free_gen(c->gd);
    dfree(c->hist);
    dfree(c->ckpt);
    dfree((void *&)c->sig);
    dfree((void *&)c->G);
    dfree((void *&)c->dir);
    dfree((void *&)c->grad);
    dfree((void *&)c->trial);
    dfree((void *&)c->obsbuf);
    dfree((void *&)c->resbuf);
    dfree((void *&)c->partials);
    dfree((void *&)c->scal);
    dfree((void *&)c->tf0);
    dfree((void *&)c->tf1);
    dfree((void *&)c->epsc);
    dfree((void *&)c->Gm);
    dfree(c->minv);
    dfree(c->hm1);
    delete c;
}

hyb_status hyb_set_initial(hyb_ctx *c, const double *u0, const double *um1)
{
    if (!c) return HYB_E_ARG;
    if (c->gen && !c->gen_all_grid && (u0 || um1))
        return fail(c, HYB_E_UNSUPPORTED, "initial levels need every FEM node on the grid");
    c->ic_u0 = u0;
    c->ic_um1 = um1;
    c->ic_set = u0 || um1;
    c->taylor = false;
    return HYB_OK;
}

hyb_status hyb_set_wave_speed(hyb_ctx *c, const double *eps)
{
    if (!c) return HYB_E_ARG;
    if (c->in_batch) return fail(c, HYB_E_STATE, "context is owned by a batch slot");
    if (!c->g.has_fem) return fail(c, HYB_E_ARG, "a wave speed needs a FEM box");
    if (c->gen) return fail(c, HYB_E_UNSUPPORTED, "variable wave speed on a general mesh");
    const Geo &g = c->g;
    const hipStream_t st = c->stream;
    if (!eps) {
        if (c->vm) c->have_forward = c->have_adjoint = c->u_valid = false;
        c->vm = false;
        return HYB_OK;
    }
    // validate on the host (a one-off call): finite and positive on the
    // free cubes, and the smallest value for the CFL bound
    const long long nc = cube_count(g);
    std::vector<double> h(nc);
    HIPCHK(c, hipMemcpyAsync(h.data(), eps, nc * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    double emin = 1.0;
    for (int z = 2; z < g.C[2] - 2; ++z)
        for (int y = 2; y < g.C[1] - 2; ++y)
            for (int x = 2; x < g.C[0] - 2; ++x) {
                const double e = h[x + (long long)g.C[0] * (y + (long long)g.C[1] * z)];
                if (!std::isfinite(e) || !(e > 0.0)) return fail(c, HYB_E_ARG, "1/c^2 must be finite and > 0");
                emin = std::min(emin, e);
            }
    if (!c->epsc) {
        hyb_status r = dmalloc(c, (void **)&c->epsc, nc * sizeof(double));
        if (!r) r = dmalloc(c, (void **)&c->Gm, g.fem_n * sizeof(double));
        if (!r) r = dmalloc(c, &c->minv, g.fem_n * c->esz);
        if (!r) r = dmalloc(c, &c->hm1, std::max<long long>(g.hlevel, 1) * c->esz);
        if (r) {
            dfree((void *&)c->epsc);
            dfree((void *&)c->Gm);
            dfree(c->minv);
            dfree(c->hm1);
            return r;
        }
    }
    HIPCHK(c, hipMemcpyAsync(c->epsc, eps, nc * sizeof(double), hipMemcpyDeviceToDevice, st));
    if (c->f32) launch_minv<float>(g, c->epsc, (float *)c->minv, st);
    else launch_minv<double>(g, c->epsc, (double *)c->minv, st);
    HIPCHK(c, hipGetLastError());
    c->eps_min = emin;
    c->vm = true;
    c->have_forward = c->have_adjoint = c->u_valid = false;
    return HYB_OK;
}

hyb_status hyb_gradient_eps(hyb_ctx *c, double *geps)
{
    if (!c || !geps) return HYB_E_ARG;
    if (!c->vm) return fail(c, HYB_E_STATE, "no wave speed set (hyb_set_wave_speed)");
    if (!c->have_adjoint) return fail(c, HYB_E_STATE, "hyb_gradient_eps needs a previous hyb_adjoint");
    if (c->store_mode != 0)
        return fail(c, HYB_E_UNSUPPORTED, "dJ/d(1/c^2) needs the full FEM history (store mode 0)");
    const double h3 = c->h * c->h * c->h;
    launch_eps_grad(c->g, c->Gm, c->adj_mode == 0 ? 1.0 / h3 : 1.0, geps, c->stream);
    HIPCHK(c, hipGetLastError());
    return HYB_OK;
}

hyb_status hyb_set_initial_taylor(hyb_ctx *c, const double *f0, const double *f1)
{
    if (!c) return HYB_E_ARG;
    if (c->in_batch) return fail(c, HYB_E_STATE, "context is owned by a batch slot");
    c->ic_set = false;
    c->ic_u0 = c->ic_um1 = nullptr;
    if (!f0 && !f1) {
        c->taylor = false;
        return HYB_OK;
    }
    if (c->gen && !c->gen_all_grid)
        return fail(c, HYB_E_UNSUPPORTED, "initial data need every FEM node on the grid");
    const size_t b = (size_t)c->g.nx * c->g.ny * c->g.nz * sizeof(double);
    for (double **p : {&c->tf0, &c->tf1})
        if (!*p) {
            hyb_status s = dmalloc(c, (void **)p, b);
            if (s) return s;
        }
    if (f0) HIPCHK(c, hipMemcpyAsync(c->tf0, f0, b, hipMemcpyDeviceToDevice, c->stream));
    else HIPCHK(c, hipMemsetAsync(c->tf0, 0, b, c->stream));
    if (f1) HIPCHK(c, hipMemcpyAsync(c->tf1, f1, b, hipMemcpyDeviceToDevice, c->stream));
    else HIPCHK(c, hipMemsetAsync(c->tf1, 0, b, c->stream));
    c->taylor = true;
    return HYB_OK;
}

}  // extern "C"

namespace {

// Validation and set-up shared by hyb_forward and the batch submission:
// source, CFL (with the largest a, from the device unless the caller passes
// sigma_max), storage for history/checkpoints, sigma copy, step counts.
hyb_status prepare_forward(hyb_ctx *c, const double *sigma, const hyb_source *src, int32_t nt, double dt,
                           const double *sigma_max_host)
{
    if (!src) return fail(c, HYB_E_ARG, "source is null");
    if (nt < 1 || !(dt > 0) || !std::isfinite(dt)) return fail(c, HYB_E_ARG, "need nt >= 1 and dt > 0");
    if (src->kind == 0) {
        if (!(src->omega > 0) || !std::isfinite(src->omega)) return fail(c, HYB_E_ARG, "source: omega must be > 0");
    } else if (src->kind == 1) {
        if (src->k_on < 0 || (src->k_on > 0 && !src->flux_dev)) return fail(c, HYB_E_ARG, "source: flux table");
    } else {
        return fail(c, HYB_E_ARG, "source: unknown kind");
    }
    if (!c->g.has_fem && sigma) return fail(c, HYB_E_ARG, "sigma given without a FEM box");
    if (sigma_max_host && !std::isfinite(*sigma_max_host))
        return fail(c, HYB_E_NONFINITE, "sigma_max is not finite");
    if (c->gen && sigma_max_host) return fail(c, HYB_E_UNSUPPORTED, "general meshes take sigma_max from the device");
    const hipStream_t st = c->stream;
    // From here on the device conductivity of the context is replaced: a
    // refused step below also invalidates the previous sweeps.
    auto refuse = [&](hyb_status e, const char *msg) {
        c->have_forward = c->have_adjoint = c->u_valid = false;
        return fail(c, e, msg);
    };
    double smax = 0.0, gersh = 0.0;
    if (c->g.has_fem && c->gen) {
        if (c->f32) launch_gen_prepare<float>(c->gd, sigma, dt * dt, c->partials, c->scal, st);
        else launch_gen_prepare<double>(c->gd, sigma, dt * dt, c->partials, c->scal, st);
        double hs[S_NSCAL];
        HIPCHK(c, hipMemcpyAsync(hs, c->scal, S_NSCAL * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipStreamSynchronize(st));
        if (hs[S_BAD] != 0.0) return refuse(HYB_E_NONFINITE, "sigma has non-finite entries");
        smax = hs[S_SMAX];
        gersh = hs[S_GERSH];
    } else if (c->g.has_fem) {
        if (c->f32) launch_acube<float>(c->g, sigma, (float *)c->acube, c->partials, c->scal, st);
        else launch_acube<double>(c->g, sigma, (double *)c->acube, c->partials, c->scal, st);
        if (sigma_max_host) {
            smax = *sigma_max_host;
        } else {
            double hs[2];
            HIPCHK(c, hipMemcpyAsync(hs, c->scal + S_SMAX, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
            HIPCHK(c, hipStreamSynchronize(st));
            if (hs[1] != 0.0) return refuse(HYB_E_NONFINITE, "sigma has non-finite entries");
            smax = hs[0];
        }
    }
    if (c->gen) {
        // grid rows (a = 1): tau <= h / sqrt(3); FEM rows on a general mesh:
        // tau^2 times the Gershgorin bound of M^{-1} K(a) at most 4
        if (dt > c->h / std::sqrt(3.0) * (1.0 + 1e-12))
            return refuse(HYB_E_CFL, "dt violates the CFL bound h/sqrt(3) of the grid");
        if (dt * dt * gersh > 4.0 * (1.0 + 1e-12))
            return refuse(HYB_E_CFL, "dt violates the bound dt^2 max_n (|K_nn| + sum_m |K_nm|) / m_n <= 4 "
                                     "of the FEM mesh");
    } else {
        // CFL condition, eq. (CFL): tau <= h / sqrt(3 a) with the largest a;
        // with a variable wave speed tau <= h sqrt(eps_min / (3 a_max))
        // (eps = 1/c^2; the lumped mass of a node is at least eps_min h^3)
        const double amax = 1.0 + std::max(0.0, smax);
        const double emin = c->vm ? std::min(1.0, c->eps_min) : 1.0;
        if (dt > c->h * std::sqrt(emin / (3.0 * amax)) * (1.0 + 1e-12))
            return refuse(HYB_E_CFL, c->vm ? "dt violates the CFL bound h sqrt(eps_min / (3 a_max))"
                                           : "dt violates the CFL bound h/sqrt(3 a_max)");
    }
    // sqrt(nt) segmentation of the levels 0..nt (checkpoint modes)
    c->ckK = c->store_mode ? (int)std::ceil(std::sqrt((double)nt + 1.0)) : nt + 1;
    if (c->store_mode) {
        const size_t nck = (size_t)(nt / c->ckK + 1);
        const size_t need = nck * ckpt_slot_bytes(c->g, c->esz, c->store_mode);
        if (need > c->ckpt_bytes) {
            dfree(c->ckpt);
            c->ckpt_bytes = 0;
            hyb_status s = dmalloc(c, &c->ckpt, need);
            if (s) return s;
            c->ckpt_bytes = need;
        }
    }
    if (c->g.has_fem) {
        const size_t need = (size_t)(c->store_mode ? c->ckK : nt + 1);
        if (need > c->hist_levels) {
            dfree(c->hist);
            c->hist_levels = 0;
            hyb_status s = dmalloc(c, &c->hist, need * (size_t)c->g.hlevel * c->esz);
            if (s) return s;
            c->hist_levels = need;
        }
        if (sigma) HIPCHK(c, hipMemcpyAsync(c->sig, sigma, (size_t)c->npar * sizeof(double),
                                           hipMemcpyDeviceToDevice, st));
        else HIPCHK(c, hipMemsetAsync(c->sig, 0, (size_t)c->npar * sizeof(double), st));
    }
    c->nt = nt;
    c->dt = dt;
    if (src->kind == 0) {
        const double t1 = 2.0 * M_PI / src->omega;
        int kon = 0;
        for (int k = 0; k < nt; ++k)
            if ((double)k * dt < t1) kon = k + 1;
        c->k_on = kon;
    } else {
        c->k_on = std::min(src->k_on, nt);
    }
    c->have_forward = false;
    c->have_adjoint = false;
    c->cg_ready = false;
    c->src = *src;
    return HYB_OK;
}

hyb_status alloc_adjoint(hyb_ctx *c)
{
    const size_t fb = field_bytes(c->g, c->esz), vb = fem_bytes(c->g, c->esz);
    hyb_status s = HYB_OK;
    for (int q = 0; q < 3 && !s; ++q) s = dmalloc(c, &c->P[q], fb);
    for (int q = 0; q < 3 && !s; ++q) s = dmalloc(c, &c->F[q], (size_t)c->g.ftot * c->esz);
    if (!s && c->g.has_fem)
        for (int q = 0; q < 3 && !s; ++q) s = dmalloc(c, &c->Q[q], vb);
    if (!s && c->g.has_fem && !c->gen) s = dmalloc(c, (void **)&c->G, cube_count(c->g) * sizeof(double));
    if (c->f32) {
        for (int q = 0; q < 2 && !s; ++q) s = dmalloc(c, &c->E[q], fb);
        if (!s && c->g.has_fem)
            for (int q = 0; q < 2 && !s; ++q) s = dmalloc(c, &c->QE[q], vb);
    }
    return s;
}

}  // namespace

namespace {

bool same_source(const hyb_source &a, const hyb_source &b)
{
    return a.kind == b.kind && a.omega == b.omega && a.flux_dev == b.flux_dev && a.k_on == b.k_on;
}

Params cg_params(const hyb_ctx *c)
{
    Params p;
    p.n = c->npar;
    for (int d = 0; d < 3; ++d) p.C[d] = c->g.C[d];
    p.pvol = c->gen ? c->gd.pvol : nullptr;
    p.h3 = c->h * c->h * c->h;
    return p;
}

// Forward sweep at sigma into the context's trace buffer, then the residual
// obs - data and its misfit J -> scal[slot].
hyb_status cg_forward(hyb_ctx *c, const double *sigma, const hyb_source *src, int32_t nt, double dt,
                      const double *data, int slot)
{
    hyb_status s = hyb_forward(c, sigma, src, nt, dt, c->obsbuf);
    if (s) return s;
    const long long ntr = (long long)(nt + 1) * c->g.nx * c->g.ny;
    launch_residual(c->obsbuf, data, c->resbuf, ntr, c->stream);
    launch_misfit(c->g, c->resbuf, nt, dt, c->h, c->partials, c->scal, slot, c->stream);
    HIPCHK(c, hipGetLastError());
    return HYB_OK;
}

hyb_status read_scal(hyb_ctx *c, double *hs)
{
    HIPCHK(c, hipMemcpyAsync(hs, c->scal, S_NSCAL * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return HYB_OK;
}

}  // namespace

extern "C" {

hyb_status hyb_forward(hyb_ctx *c, const double *sigma, const hyb_source *src, int32_t nt, double dt,
                       double *obs)
{
    if (!c) return HYB_E_ARG;
    if (c->in_batch) return fail(c, HYB_E_STATE, "context is busy in a batch");
    hyb_status s = prepare_forward(c, sigma, src, nt, dt, nullptr);
    if (s) return s;
    s = c->f32 ? run_forward<float>(c, obs) : run_forward<double>(c, obs);
    if (s) return s;
    c->have_forward = true;
    return HYB_OK;
}

hyb_status hyb_adjoint(hyb_ctx *c, const double *res, int32_t mode)
{
    if (!c) return HYB_E_ARG;
    if (!res || (mode != 0 && mode != 1)) return fail(c, HYB_E_ARG, "adjoint: residual and mode 0/1");
    if (!c->have_forward) return fail(c, HYB_E_STATE, "adjoint before forward");
    if (c->in_batch) return fail(c, HYB_E_STATE, "context is busy in a batch");
    hyb_status s = alloc_adjoint(c);
    if (s) return s;
    s = c->f32 ? run_adjoint<float>(c, res, mode) : run_adjoint<double>(c, res, mode);
    if (s) return s;
    c->have_adjoint = true;
    c->adj_mode = mode;
    return HYB_OK;
}

hyb_status hyb_gradient(hyb_ctx *c, double *grad, double *J)
{
    if (!c) return HYB_E_ARG;
    if (!grad) return fail(c, HYB_E_ARG, "grad is null");
    if (!c->g.has_fem) return fail(c, HYB_E_STATE, "gradient needs a FEM box");
    if (!c->have_adjoint) return fail(c, HYB_E_STATE, "gradient before adjoint");
    const double h = c->h, h3 = h * h * h;
    // dJ/dsigma_c = -(dt^2/h^2) G_c (G = sum_k sum_e w_e D_e lambda^{k+1} D_e u^k)
    const double dJ = -(c->dt * c->dt) / (h * h);
    const int mode = c->adj_mode;
    if (c->gen)
        launch_gen_grad_final(c->gd, c->sig, c->gamma, mode, grad, c->partials, c->scal, S_JREG, c->stream);
    else
        launch_grad_final(c->g, c->G, c->sig, mode == 0 ? dJ / h3 : dJ, c->gamma, mode, h3, grad, c->partials,
                          c->scal, S_JREG, c->stream);
    HIPCHK(c, hipGetLastError());
    if (J) {
        double hs[2];
        HIPCHK(c, hipMemcpyAsync(hs, c->scal + S_JMIS, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        *J = mode == 0 ? hs[0] + hs[1] : 0.0;
    }
    return HYB_OK;
}

hyb_status hyb_gradient_noalloc(hyb_ctx *c, double *grad, double *J_dev)
{
    if (!c) return HYB_E_ARG;
    if (!grad) return fail(c, HYB_E_ARG, "grad is null");
    if (!c->g.has_fem) return fail(c, HYB_E_STATE, "gradient needs a FEM box");
    // one partial sum per block of 256 parameters, all in the scratch array
    const long long nb = ceil_div(c->npar, BLOCK);
    if (nb > NOALLOC_PARTS)
        return fail(c, HYB_E_UNSUPPORTED, "hyb_gradient_noalloc: " + std::to_string(c->npar) +
                                              " parameters, the scratch holds partials for at most " +
                                              std::to_string((long long)NOALLOC_PARTS * BLOCK));
    if (!c->have_adjoint) return fail(c, HYB_E_STATE, "gradient before adjoint");
    double *scr = nullptr;
    HIPCHK(c, noalloc_scratch(&scr));
    double *part = scr, *sc = scr + NOALLOC_PARTS;
    const double h = c->h, h3 = h * h * h;
    const double dJ = -(c->dt * c->dt) / (h * h);
    const int mode = c->adj_mode;
    if (c->gen)
        launch_gen_grad_final(c->gd, c->sig, c->gamma, mode, grad, part, sc, 0, c->stream, (int)nb);
    else
        launch_grad_final(c->g, c->G, c->sig, mode == 0 ? dJ / h3 : dJ, c->gamma, mode, h3, grad, part, sc, 0,
                          c->stream, (int)nb);
    if (J_dev) launch_sum_J(c->scal + S_JMIS, sc, mode, J_dev, c->stream);
    HIPCHK(c, hipGetLastError());
    return HYB_OK;
}

hyb_status hyb_cg_step(hyb_ctx *c, const double *data, double *sigma, const hyb_source *src, int32_t nt,
                       double dt, hyb_cg_state *state, double *gnorm, double *J)
{
    if (!c) return HYB_E_ARG;
    if (!data || !sigma || !state || !src) return fail(c, HYB_E_ARG, "cg_step: null argument");
    if (!c->g.has_fem) return fail(c, HYB_E_STATE, "cg_step needs a FEM box");
    if (c->in_batch) return fail(c, HYB_E_STATE, "context is busy in a batch");
    if (state->iter < 0) return fail(c, HYB_E_ARG, "cg_step: state->iter < 0");
    hyb_status s = ensure_trace_bufs(c, nt);
    if (!s) s = dmalloc(c, (void **)&c->dir, (size_t)c->npar * sizeof(double));
    if (!s) s = dmalloc(c, (void **)&c->grad, (size_t)c->npar * sizeof(double));
    if (!s) s = dmalloc(c, (void **)&c->trial, (size_t)c->npar * sizeof(double));
    if (s) return s;
    const hipStream_t st = c->stream;
    const Params p = cg_params(c);
    double hs[S_NSCAL];
    // 1. the forward sweep at sigma^m, unless the accepted trial of the
    // previous iteration left it (then sigma must still hold that point)
    bool reuse = state->iter > 0 && c->cg_ready && c->have_forward && c->cg_sigma == sigma &&
                 c->cg_data == data && c->nt == nt && c->dt == dt && same_source(c->src, *src);
    if (reuse) {
        launch_differ(sigma, c->sig, c->npar, c->partials, c->scal, S_DIFF, st);
        s = read_scal(c, hs);
        if (s) return s;
        reuse = hs[S_DIFF] == 0.0;
    }
    c->cg_ready = false;
    int forwards = 0;
    if (!reuse) {
        s = cg_forward(c, sigma, src, nt, dt, data, S_JMIST);
        if (s) return s;
        ++forwards;
    }
    s = hyb_adjoint(c, c->resbuf, 0);
    if (s) return s;
    s = hyb_gradient(c, c->grad, nullptr);
    if (s) return s;
    // 2. direction (beta, restart) and its max norm
    const int first = state->iter == 0;
    launch_cg_norm2(p, c->grad, c->partials, c->scal, S_GN2, st);
    launch_cg_dir(p, c->grad, c->dir, sigma, first, c->partials, c->scal, st);
    HIPCHK(c, hipGetLastError());
    s = read_scal(c, hs);
    if (s) return s;
    const double Jm = hs[S_JMIS] + hs[S_JREG], gn2 = hs[S_GN2], dmax = hs[S_DMAX];
    const double beta = hs[S_BETA];
    const bool restart = hs[S_RESTART] != 0.0;
    // 3. trial steps 2^-t rho / max|d| until J falls below J^m; rho is the
    // first relative step (largest change of sigma): alpha_rel, and after the
    // first iteration twice the previous accepted one, at most alpha_rel (a
    // call after a stalled one, which took no step, starts from alpha_rel)
    const double prev = state->alpha * state->dmax;
    const double rho = (first || !(prev > 0.0)) ? c->alpha_rel : std::fmin(c->alpha_rel, 2.0 * prev);
    bool taken = false;
    int t = 0;
    double alpha = 0.0, Jn = Jm;
    while (dmax > 0.0 && t < c->max_trials && !taken) {
        launch_cg_trial(p, c->dir, sigma, c->trial, rho, t, c->gamma, c->partials, c->scal, st);
        HIPCHK(c, hipGetLastError());
        s = cg_forward(c, c->trial, src, nt, dt, data, S_JMIST);
        if (s) return s;
        ++forwards;
        ++t;
        s = read_scal(c, hs);
        if (s) return s;
        const double Jt = hs[S_JMIST] + hs[S_JREGT];
        if (Jt < Jm) {
            taken = true;
            alpha = hs[S_ALPHA];
            Jn = Jt;
            HIPCHK(c, hipMemcpyAsync(sigma, c->trial, (size_t)c->npar * sizeof(double), hipMemcpyDeviceToDevice,
                                     st));
        }
    }
    launch_cg_roll(c->scal, st);
    HIPCHK(c, hipGetLastError());
    if (taken) {
        c->cg_ready = true;
        c->cg_sigma = sigma;
        c->cg_data = data;
    }
    state->iter += 1;
    state->gnorm2_prev = gn2;
    state->beta = beta;
    state->dmax = dmax;
    state->restart = restart ? 1 : 0;
    state->alpha = alpha;
    state->J_next = Jn;
    state->trials = t;
    state->stalled = taken ? 0 : 1;
    state->forwards = forwards;
    if (gnorm) *gnorm = std::sqrt(gn2);
    if (J) *J = Jm;
    return HYB_OK;
}

hyb_status hyb_footprint(const hyb_fd_grid *grid, const hyb_fem_mesh *fem, const hyb_overlap *overlap,
                         const hyb_opts *opts, int32_t nt, size_t *bytes)
{
    if (!bytes || nt < 1) return fail(nullptr, HYB_E_ARG, "footprint: bytes null or nt < 1");
    hyb_status s = check_grid(grid, nullptr);
    if (s) return s;
    Mesh mesh;
    GenHost gh;
    bool gen = false;
    if (fem) {
        if (!overlap || overlap->width_cells != 2)
            return fail(nullptr, HYB_E_UNSUPPORTED, "overlap: the method uses a two-element overlap");
        s = analyse_fem(grid, fem, opts && opts->fem_general, &mesh, &gh, &gen, nullptr);
        if (s) return s;
    }
    const size_t esz = (opts && opts->field_f32) ? 4 : 8;
    Geo g{};
    int n[3] = {grid->n_cells[0], grid->n_cells[1], grid->n_cells[2]};
    setup_geo(g, n, mesh, fem != nullptr, esz);
    if (gen) setup_geo_gen(g, gh);
    const size_t nc = gen ? (size_t)gh.ntet : cube_count(g), ntr = (size_t)(nt + 1) * g.nx * g.ny * sizeof(double);
    const int nlev = esz == 4 ? 10 : 6;  // three U and P levels (+ two increments each in FP32)
    size_t b = nlev * field_bytes(g, esz) + nlev * fem_bytes(g, esz) + nc * (esz + 4 * sizeof(double));
    if (gen)  // tables of hyb_gen.h
        b += (size_t)gh.nnz * (8 + esz) + gh.cw.size() * 12 + (size_t)gh.fn * (8 + esz + 4 + 8) +
             (size_t)gh.nE * 8 + (size_t)gh.ntet * (6 * 12 + 8) + (size_t)(gh.nA + gh.fn - gh.nR) * 8 +
             (gh.soff.size() + gh.eoff.size()) * 4 - nc * esz;
    b += (size_t)(nt + 1) * g.hlevel * esz + 2 * ntr + (MAX_PARTIALS + S_NSCAL) * sizeof(double);
    b += 3 * (size_t)g.ftot * esz;
    const int sm = opts ? opts->store_mode : 0;
    if (sm) {
        const int K = (int)std::ceil(std::sqrt((double)nt + 1.0));
        b -= (size_t)(nt + 1 - K) * g.hlevel * esz;
        b += (size_t)(nt / K + 1) * ckpt_slot_bytes(g, esz, sm);
    }
    *bytes = b;
    return HYB_OK;
}

hyb_status hyb_sync(hyb_ctx *c)
{
    if (!c) return HYB_E_ARG;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipGetLastError());
    return HYB_OK;
}

const char *hyb_last_error(const hyb_ctx *c)
{
    return c ? c->err.c_str() : g_create_err.c_str();
}

hyb_status hyb_counts(const hyb_ctx *c, int64_t *fdm, int64_t *fem)
{
    if (!c || !fdm || !fem) return HYB_E_ARG;
    const Geo &g = c->g;
    const long long nn = (long long)g.nx * g.ny * g.nz;
    const long long hole = g.has_fem ? (long long)(g.C[0] - 3) * (g.C[1] - 3) * (g.C[2] - 3) : 0;
    *fdm = nn - hole;
    *fem = c->gen ? c->gd.nR : (g.has_fem ? (long long)(g.C[0] - 1) * (g.C[1] - 1) * (g.C[2] - 1) : 0);
    return HYB_OK;
}

hyb_status hyb_fem_info(const hyb_ctx *c, int64_t *n_params, int32_t *general, int64_t *n_fem_nodes)
{
    if (!c) return HYB_E_ARG;
    if (n_params) *n_params = c->g.has_fem ? c->npar : 0;
    if (general) *general = c->gen ? 1 : 0;
    if (n_fem_nodes) *n_fem_nodes = c->g.has_fem ? c->g.fem_n : 0;
    return HYB_OK;
}

hyb_status hyb_get_wavefield(hyb_ctx *c, int32_t which, double *u, double *v)
{
    if (!c || (which != 0 && which != 1)) return HYB_E_ARG;
    if ((which == 0 && !(c->have_forward && c->u_valid)) || (which == 1 && !c->have_adjoint))
        return fail(c, HYB_E_STATE, "get_wavefield: no such sweep yet (or overwritten by a recompute)");
    void *const *A = which == 0 ? c->U : c->P;
    void *const *B = which == 0 ? c->V : c->Q;
    const int q = which == 0 ? c->last_u : c->last_p;
    const void *Fq = which == 1 ? c->F[q] : nullptr;  // true boundary multipliers
    double *vs = c->gen ? nullptr : v;  // a general mesh exports in the caller's node numbering
    // x faces never change condition during a sweep (only z+ carries the source)
    const int types = face_types(c, 0);
    if (c->f32)
        launch_export_level<float>(c->g, (const float *)A[q], (const float *)B[q], (const float *)Fq, u, vs,
                                   c->stream, types);
    else
        launch_export_level<double>(c->g, (const double *)A[q], (const double *)B[q], (const double *)Fq, u,
                                    vs, c->stream, types);
    if (c->gen && v) {
        // the forward level's omega_o nodes hold grid values, read from the grid level
        const void *Ug = which == 0 ? A[q] : nullptr;
        if (c->f32) launch_gen_export<float>(c->gd, (const float *)B[q], (const float *)Ug, v, c->stream);
        else launch_gen_export<double>(c->gd, (const double *)B[q], (const double *)Ug, v, c->stream);
    }
    HIPCHK(c, hipGetLastError());
    return HYB_OK;
}

hyb_status hyb_time_fem(hyb_ctx *c, int32_t which, int32_t reps, double *ms)
{
    if (!c || !ms || reps < 1 || (which != 0 && which != 1)) return HYB_E_ARG;
    if (!c->gen) return fail(c, HYB_E_STATE, "time_fem: the FEM box is not a general mesh");
    if (!c->have_forward || !c->hist) return fail(c, HYB_E_STATE, "time_fem needs a previous forward");
    if (which == 1 && !c->have_adjoint) return fail(c, HYB_E_STATE, "time_fem (adjoint) needs a previous adjoint");
    const hipStream_t st = c->stream;
    // the launches overwrite the wavefields, multipliers and accumulators
    c->have_forward = false;
    c->u_valid = false;
    c->have_adjoint = false;
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    auto body = [&](auto tag) -> hyb_status {
        using T = decltype(tag);
        Step<T> s = make_step<T>(c);
        void *const *A = which == 0 ? c->U : c->P;
        void *const *B = which == 0 ? c->V : c->Q;
        void *const *I = which == 0 ? c->VD : c->QE;
        int ia = 0, ib = 1, ic = 2;
        HIPCHK(c, hipEventRecord(e0, st));
        for (int r = 0; r < reps; ++r) {
            s.Ub = (const T *)A[ib]; s.Uc = (T *)A[ic];
            s.Va = (const T *)B[ia]; s.Vb = (const T *)B[ib]; s.Vc = (T *)B[ic];
            if (incr_form<T>()) { s.VDa = (const T *)I[r & 1]; s.VDc = (T *)I[(r + 1) & 1]; }
            s.hist = (T *)c->hist;
            if (which == 0) launch_gen_fwd<T>(gen_args<T>(c, s), st);
            else launch_gen_adj<T>(gen_adj_args<T>(c, s, r), st);
            const int t = ia; ia = ib; ib = ic; ic = t;
        }
        HIPCHK(c, hipEventRecord(e1, st));
        return HYB_OK;
    };
    hyb_status s = c->f32 ? body(0.0f) : body(0.0);
    if (s) return s;
    HIPCHK(c, hipEventSynchronize(e1));
    float t = 0;
    HIPCHK(c, hipEventElapsedTime(&t, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = (double)t / reps;
    return HYB_OK;
}

hyb_status hyb_time_interior(hyb_ctx *c, const double *sigma, double dt, int32_t reps, double *ms)
{
    if (!c || !ms || reps < 1 || !(dt > 0)) return HYB_E_ARG;
    const hipStream_t st = c->stream;
    if (c->g.has_fem) {
        if (!c->hist) return fail(c, HYB_E_STATE, "time_interior needs a previous forward (history)");
        if (!c->gen) {
            if (c->f32) launch_acube<float>(c->g, sigma, (float *)c->acube, c->partials, c->scal, st);
            else launch_acube<double>(c->g, sigma, (double *)c->acube, c->partials, c->scal, st);
        }
    }
    // the launches overwrite the wavefields and the first history level
    c->have_forward = false;
    c->u_valid = false;
    c->have_adjoint = false;
    const double save_dt = c->dt;
    c->dt = dt;
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    auto body = [&](auto tag) -> hyb_status {
        using T = decltype(tag);
        Step<T> s = make_step<T>(c);
        s.types1 = face_types(c, -1);
        int ia = 0, ib = 1, ic = 2;
        HIPCHK(c, hipEventRecord(e0, st));
        for (int r = 0; r < reps; ++r) {
            s.Ua = (const T *)c->U[ia]; s.Ub = (const T *)c->U[ib]; s.Uc = (T *)c->U[ic];
            s.Va = (const T *)c->V[ia]; s.Vb = (const T *)c->V[ib]; s.Vc = (T *)c->V[ic];
            if (incr_form<T>()) {
                s.Da = (const T *)c->D[r & 1]; s.Dc = (T *)c->D[(r + 1) & 1];
                s.VDa = (const T *)c->VD[r & 1]; s.VDc = (T *)c->VD[(r + 1) & 1];
            }
            s.hist = c->g.has_fem ? (T *)c->hist : nullptr;
            launch_interior<T>(s, false, st);
            const int t = ia; ia = ib; ib = ic; ic = t;
        }
        HIPCHK(c, hipEventRecord(e1, st));
        return HYB_OK;
    };
    hyb_status s = c->f32 ? body(0.0f) : body(0.0);
    c->dt = save_dt;
    if (s) return s;
    HIPCHK(c, hipEventSynchronize(e1));
    float t = 0;
    HIPCHK(c, hipEventElapsedTime(&t, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = (double)t / reps;
    return HYB_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ batch

struct hyb_batch {
    struct Slot {
        hyb_ctx *c = nullptr;
        int state = 0;  // 0 free, 1 forward, 2 adjoint, 3 finished (event pending), 4 failed
        int k = 0, ia = 0, ib = 1, ic = 2;
        const double *data = nullptr;
        double *obs = nullptr, *grad = nullptr;
        hipEvent_t done = nullptr;
        double *J_host = nullptr;  // pinned quadruple: device max sigma, non-finite flag, misfit,
                                   // regularisation
        double sigma_max = 0.0;    // the caller's max sigma, used for the CFL check
        int lane = 0;
        // the slot's last planned forward step, whose edge and corner rows
        // its next forward launch runs (lag set) or a launch of their own
        Step<float> prevf{};
        Step<double> prevd{};
        bool lag = false;
    };
    // one lane per stream: slots of different lanes run concurrently on the
    // device; each lane has its own ring of step-argument staging buffers
    struct Lane {
        hipStream_t st = nullptr;
        char *h_stage = nullptr, *d_stage = nullptr;
        int cur = 0;
        std::vector<hipEvent_t> ev;
    };
    int max_slots = 0;
    std::vector<Slot> slots;
    std::vector<Lane> lanes;
    size_t entry = 0;
    int ring = 0;
    double *h_J = nullptr;
    std::string err;
};

namespace {

constexpr int STAGE_RING = 16;
constexpr int TICKS_PER_PLAN = 32;

hyb_status bfail(hyb_batch *b, hyb_status s, const std::string &m)
{
    if (b) b->err = m;
    return s;
}

void free_lane(hyb_batch::Lane &L)
{
    for (auto e : L.ev)
        if (e) (void)hipEventDestroy(e);
    L.ev.clear();
    if (L.h_stage) (void)hipHostFree(L.h_stage);
    if (L.d_stage) (void)hipFree(L.d_stage);
    L.h_stage = L.d_stage = nullptr;
}

// index of the lane of stream st (created on first use)
int lane_of(hyb_batch *b, hipStream_t st)
{
    for (size_t q = 0; q < b->lanes.size(); ++q)
        if (b->lanes[q].st == st) return (int)q;
    hyb_batch::Lane L;
    L.st = st;
    bool ok = hipHostMalloc((void **)&L.h_stage, b->entry * b->ring) == hipSuccess &&
              hipMalloc((void **)&L.d_stage, b->entry * b->ring) == hipSuccess;
    L.ev.resize(b->ring, nullptr);
    for (int q = 0; ok && q < b->ring; ++q) ok = hipEventCreateWithFlags(&L.ev[q], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        free_lane(L);
        return -1;
    }
    b->lanes.push_back(L);
    return (int)b->lanes.size() - 1;
}

// Advance the host-side state of a slot by one step; returns 1 when its
// forward sweep has just ended, 2 when its adjoint sweep has just ended.
int advance_slot(hyb_batch::Slot &sl)
{
    hyb_ctx *c = sl.c;
    const int t = sl.ia; sl.ia = sl.ib; sl.ib = sl.ic; sl.ic = t;
    if (sl.state == 1) {
        if (++sl.k == c->nt) {
            c->last_u = sl.ib;
            sl.state = 2;
            sl.k = c->nt;
            sl.ia = 0; sl.ib = 1; sl.ic = 2;
            return 1;
        }
    } else if (sl.state == 2) {
        if (--sl.k < 0) {
            c->last_p = sl.ib;
            sl.state = 3;
            return 2;
        }
    }
    return 0;
}

// Work between the sweeps of a slot: residual against the data, adjoint set-up.
template <typename T>
void finish_forward(hyb_batch::Slot &sl)
{
    hyb_ctx *c = sl.c;
    c->u_valid = true;
    c->have_forward = true;
    const long long ntr = (long long)(c->nt + 1) * c->g.nx * c->g.ny;
    launch_residual(sl.obs, sl.data, c->resbuf, ntr, c->stream);
    adj_setup<T>(c, c->resbuf, 0);
}

// Gradient of the slot, its J and the completion event.
void finish_adjoint(hyb_batch::Slot &sl)
{
    hyb_ctx *c = sl.c;
    c->have_adjoint = true;
    c->adj_mode = 0;
    const double h = c->h, h3 = h * h * h, dJ = -(c->dt * c->dt) / (h * h);
    launch_grad_final(c->g, c->G, c->sig, dJ / h3, c->gamma, 0, h3, sl.grad, c->partials, c->scal, S_JREG,
                      c->stream);
    // device max sigma, non-finite flag of sigma, misfit, regularisation
    static_assert(S_SMAX == 0 && S_BAD == 1 && S_JMIS == 2 && S_JREG == 3, "slot quadruple layout");
    (void)hipMemcpyAsync(sl.J_host, c->scal + S_SMAX, 4 * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    (void)hipEventRecord(sl.done, c->stream);
}

// One planned launch group, edge launch or slot transition, in stream order.
struct Action {
    int kind;        // 0 launch group, 1 forward ended, 2 adjoint ended, 3 edge rows of a step
    int lane, slot;  // lane of the work; slot for transitions / first slot of a group
    int adjoint, n, f32;
    size_t offset;   // byte offset of the group's step array in the lane buffer (kind 3: of the
                     // step in the host-only buffer)
    int edges = 0;   // forward group: the lane buffer holds its edge arguments at eoff
    size_t eoff = 0;
    long long face_rows = 0;  // forward group: largest count of reflecting face rows
};

template <typename T> Step<T> &slot_prev(hyb_batch::Slot &sl);
template <> Step<float> &slot_prev<float>(hyb_batch::Slot &sl) { return sl.prevf; }
template <> Step<double> &slot_prev<double>(hyb_batch::Slot &sl) { return sl.prevd; }

// append n objects to a staging buffer at a 256-byte boundary; returns their offset
size_t stage_put(std::vector<char> &B, const void *p, size_t bytes)
{
    const size_t off = (B.size() + 255) / 256 * 256;
    B.resize(off + bytes);
    std::memcpy(B.data() + off, p, bytes);
    return off;
}

// Plan one launch group of slots ids (one phase, one geometry, lane `lane`).
// A forward group carries the edge and corner rows of each slot's previous
// step in its interior launch (as the single-context sweep does); a slot
// whose face conditions change between the two steps gets them in a launch
// of their own first (they recompute reflecting face rows from their own
// step's levels, which the interior launch overwrites on faces that absorb).
template <typename T>
void plan_group(hyb_batch *b, const std::vector<int> &ids, bool adj, int lane, std::vector<char> &B,
                std::vector<char> &H, std::vector<Action> &acts)
{
    const size_t n = ids.size();
    const int f32 = sizeof(T) == 4 ? 1 : 0;
    std::vector<Step<T>> steps(n);
    std::vector<EdgeArgs<T>> edges(n, EdgeArgs<T>{});
    bool any = false;
    long long frows = 0;
    for (size_t j = 0; j < n; ++j) {
        hyb_batch::Slot &sl = b->slots[ids[j]];
        if (adj) {
            steps[j] = adj_step_args<T>(sl.c, sl.k, sl.ia, sl.ib, sl.ic, sl.c->resbuf, 0);
            continue;
        }
        steps[j] = fwd_step_args<T>(sl.c, sl.k, sl.ia, sl.ib, sl.ic, sl.obs);
        Step<T> &prev = slot_prev<T>(sl);
        if (sl.lag && prev.types1 != steps[j].types1) {
            acts.push_back(Action{3, lane, ids[j], 0, 1, f32, stage_put(H, &prev, sizeof prev)});
            sl.lag = false;
        }
        if (sl.lag) {
            edges[j] = edge_args(prev);
            any = true;
        }
        frows = std::max(frows, fwd_face_row_count(sl.c->g, steps[j].types1));
        prev = steps[j];
        sl.lag = true;
    }
    Action a{0, lane, ids[0], adj ? 1 : 0, (int)n, f32, stage_put(B, steps.data(), n * sizeof(Step<T>))};
    if (any) {
        a.edges = 1;
        a.eoff = stage_put(B, edges.data(), n * sizeof(EdgeArgs<T>));
    }
    a.face_rows = frows;
    acts.push_back(a);
}

// the edge and corner rows of a slot's last forward step, once its sweep ends
template <typename T>
void plan_flush(hyb_batch::Slot &sl, int id, std::vector<char> &H, std::vector<Action> &acts)
{
    if (!sl.lag) return;
    const Step<T> &prev = slot_prev<T>(sl);
    acts.push_back(Action{3, sl.lane, id, 0, 1, sizeof(T) == 4 ? 1 : 0, stage_put(H, &prev, sizeof prev)});
    sl.lag = false;
}

bool same_geometry(const hyb_ctx *a, const hyb_ctx *b)
{
    return a->f32 == b->f32 && a->stream == b->stream && std::memcmp(&a->g, &b->g, sizeof(Geo)) == 0 &&
           std::memcmp(a->mesh.w, b->mesh.w, sizeof a->mesh.w) == 0 && a->dt == b->dt && a->h == b->h;
}

}  // namespace

namespace {

// Plan up to `ticks` ticks: the host advances every running slot one step per
// tick and records the step arguments of each launch group (per lane, in one
// buffer) and the slot transitions; then one copy per lane ships all step
// arguments and the launches and transitions are issued in the planned order.
hyb_status batch_plan_run(hyb_batch *b, int ticks, int32_t *n_first)
{
    std::vector<std::vector<char>> buf(b->lanes.size());
    std::vector<char> hbuf;  // steps of the edge launches, read on the host only
    std::vector<Action> acts;
    int first = -1;
    for (int t = 0; t < ticks; ++t) {
        std::vector<std::vector<int>> groups;
        std::vector<int> gphase;
        for (int i = 0; i < b->max_slots; ++i) {
            const auto &sl = b->slots[i];
            if (sl.state != 1 && sl.state != 2) continue;
            int gi = -1;
            for (size_t q = 0; q < groups.size(); ++q)
                if (gphase[q] == sl.state && same_geometry(b->slots[groups[q][0]].c, sl.c)) { gi = (int)q; break; }
            if (gi < 0) { groups.emplace_back(); gphase.push_back(sl.state); gi = (int)groups.size() - 1; }
            groups[gi].push_back(i);
        }
        if (first < 0) {
            first = 0;
            for (auto &gr : groups) first += (int)gr.size();
        }
        if (groups.empty()) break;
        std::vector<Action> trans;
        for (size_t q = 0; q < groups.size(); ++q) {
            const auto &ids = groups[q];
            const hyb_batch::Slot &s0 = b->slots[ids[0]];
            const bool adj = gphase[q] == 2, f32 = s0.c->f32;
            if (f32) plan_group<float>(b, ids, adj, s0.lane, buf[s0.lane], hbuf, acts);
            else plan_group<double>(b, ids, adj, s0.lane, buf[s0.lane], hbuf, acts);
            for (int id : ids) {
                hyb_batch::Slot &sl = b->slots[id];
                const int ev = advance_slot(sl);
                if (ev == 1) {
                    if (sl.c->f32) plan_flush<float>(sl, id, hbuf, trans);
                    else plan_flush<double>(sl, id, hbuf, trans);
                }
                if (ev) trans.push_back(Action{ev, sl.lane, id, 0, 0, sl.c->f32 ? 1 : 0, 0});
            }
        }
        acts.insert(acts.end(), trans.begin(), trans.end());
    }
    // ship the step arguments, one copy per lane
    std::vector<char *> dbase(b->lanes.size(), nullptr);
    std::vector<int> used(b->lanes.size(), -1);
    for (size_t li = 0; li < b->lanes.size(); ++li) {
        if (buf[li].empty()) continue;
        hyb_batch::Lane &L = b->lanes[li];
        if (buf[li].size() > b->entry) return bfail(b, HYB_E_ARG, "batch: staging entry too small");
        const int e = L.cur;
        L.cur = (L.cur + 1) % b->ring;
        if (hipEventSynchronize(L.ev[e]) != hipSuccess) return bfail(b, HYB_E_DEVICE, "staging event");
        char *h = L.h_stage + (size_t)e * b->entry;
        dbase[li] = L.d_stage + (size_t)e * b->entry;
        std::memcpy(h, buf[li].data(), buf[li].size());
        if (hipMemcpyAsync(dbase[li], h, buf[li].size(), hipMemcpyHostToDevice, L.st) != hipSuccess)
            return bfail(b, HYB_E_DEVICE, "staging copy failed");
        used[li] = e;
    }
    // launches and transitions in planned order
    for (const Action &a : acts) {
        hyb_batch::Slot &sl = b->slots[a.slot];
        if (a.kind == 0 && a.n == 1) {
            // a group of one: the plain kernels with the arguments by value
            const hipStream_t st = b->lanes[a.lane].st;
            const char *hp = buf[a.lane].data() + a.offset;
            auto one = [&](auto tag) {
                using T = decltype(tag);
                Step<T> s1;
                std::memcpy(&s1, hp, sizeof s1);
                if (a.adjoint) {
                    launch_bnd_adj<T>(s1, st);
                    launch_interior<T>(s1, true, st);
                } else {
                    EdgeArgs<T> e1{};
                    if (a.edges) std::memcpy(&e1, buf[a.lane].data() + a.eoff, sizeof e1);
                    launch_interior<T>(s1, false, st, a.edges ? &e1 : nullptr);
                    launch_bnd_fwd_faces<T>(s1, st);
                }
            };
            if (a.f32) one(0.0f);
            else one(0.0);
        } else if (a.kind == 0) {
            const Geo &g = sl.c->g;
            const hipStream_t st = b->lanes[a.lane].st;
            auto group = [&](auto tag) {
                using T = decltype(tag);
                const Step<T> *d = (const Step<T> *)(dbase[a.lane] + a.offset);
                if (a.adjoint) launch_batch_adj<T>(g, d, a.n, st);
                else
                    launch_batch_fwd<T>(g, d, a.edges ? (const EdgeArgs<T> *)(dbase[a.lane] + a.eoff) : nullptr,
                                        a.n, a.face_rows, st);
            };
            if (a.f32) group(0.0f);
            else group(0.0);
        } else if (a.kind == 3) {
            const hipStream_t st = b->lanes[a.lane].st;
            auto flush = [&](auto tag) {
                using T = decltype(tag);
                Step<T> p;
                std::memcpy(&p, hbuf.data() + a.offset, sizeof p);
                launch_bnd_fwd_edges<T>(p, st);
            };
            if (a.f32) flush(0.0f);
            else flush(0.0);
        } else if (a.kind == 1) {
            if (a.f32) finish_forward<float>(sl); else finish_forward<double>(sl);
        } else {
            finish_adjoint(sl);
        }
    }
    for (size_t li = 0; li < b->lanes.size(); ++li)
        if (used[li] >= 0 && hipEventRecord(b->lanes[li].ev[used[li]], b->lanes[li].st) != hipSuccess)
            return bfail(b, HYB_E_DEVICE, "staging event");
    if (hipGetLastError() != hipSuccess) return bfail(b, HYB_E_DEVICE, "kernel launch failed");
    if (n_first) *n_first = first < 0 ? 0 : first;
    return HYB_OK;
}

}  // namespace

extern "C" {

hyb_status hyb_batch_create(int32_t max_slots, void *hip_stream, hyb_batch **out)
{
    if (!out || max_slots < 1 || max_slots > 4096) return HYB_E_ARG;
    *out = nullptr;
    hyb_batch *b = new hyb_batch();
    b->max_slots = max_slots;
    b->slots.resize(max_slots);
    b->ring = STAGE_RING;
    // per plan and lane: TICKS_PER_PLAN ticks of at most max_slots step
    // structs in at most max_slots groups, each group aligned to 256 bytes
    // per slot and tick: its step and its edge arguments, each group's two
    // arrays at 256-byte boundaries
    b->entry = (size_t)TICKS_PER_PLAN * (size_t)max_slots * (sizeof(Step<double>) + sizeof(EdgeArgs<double>) + 512);
    bool ok = hipHostMalloc((void **)&b->h_J, 4 * sizeof(double) * max_slots) == hipSuccess &&
              lane_of(b, (hipStream_t)hip_stream) == 0;
    for (int q = 0; ok && q < max_slots; ++q) {
        ok = hipEventCreateWithFlags(&b->slots[q].done, hipEventDisableTiming) == hipSuccess;
        b->slots[q].J_host = b->h_J + 4 * q;
    }
    if (!ok) {
        hyb_batch_destroy(b);
        return fail(nullptr, HYB_E_OOM, "batch: allocation failed");
    }
    *out = b;
    return HYB_OK;
}

void hyb_batch_destroy(hyb_batch *b)
{
    if (!b) return;
    for (auto &L : b->lanes) (void)hipStreamSynchronize(L.st);
    for (auto &sl : b->slots) {
        if (sl.c) sl.c->in_batch = false;
        if (sl.done) (void)hipEventDestroy(sl.done);
    }
    for (auto &L : b->lanes) free_lane(L);
    if (b->h_J) (void)hipHostFree(b->h_J);
    delete b;
}

hyb_status hyb_batch_submit(hyb_batch *b, hyb_ctx *c, const double *sigma, double sigma_max, const hyb_source *src,
                            int32_t nt, double dt, const double *data, double *obs, double *grad, int32_t *slot)
{
    if (!b || !c || !slot) return HYB_E_ARG;
    *slot = -1;
    if (c->in_batch) return bfail(b, HYB_E_STATE, "context already in a batch slot");
    if (!c->g.has_fem || !data || !obs || !grad) return bfail(b, HYB_E_ARG, "batch: needs a FEM box, data, obs, grad");
    if (c->store_mode != 0) return bfail(b, HYB_E_UNSUPPORTED, "batch: contexts must keep the full history");
    if (c->gen) return bfail(b, HYB_E_UNSUPPORTED, "batch: general FEM meshes are not batched");
    if (c->taylor || c->ic_set)
        return bfail(b, HYB_E_UNSUPPORTED, "batch: contexts start from zero initial data");
    if (c->vm) return bfail(b, HYB_E_UNSUPPORTED, "batch: contexts have a constant wave speed");
    int q = -1;
    for (int i = 0; i < b->max_slots; ++i)
        if (b->slots[i].state == 0) { q = i; break; }
    if (q < 0) return bfail(b, HYB_E_STATE, "batch: no free slot");
    const int lane = lane_of(b, c->stream);
    if (lane < 0) return bfail(b, HYB_E_OOM, "batch: staging allocation failed");
    hyb_status s = prepare_forward(c, sigma, src, nt, dt, &sigma_max);
    if (!s) s = alloc_adjoint(c);
    if (!s) s = ensure_trace_bufs(c, nt);
    if (s) return bfail(b, s, c->err);
    s = c->f32 ? fwd_setup<float>(c, obs) : fwd_setup<double>(c, obs);
    if (s) return bfail(b, s, c->err);
    hyb_batch::Slot &sl = b->slots[q];
    sl.c = c;
    sl.state = 1;
    sl.k = 0; sl.ia = 0; sl.ib = 1; sl.ic = 2;
    sl.data = data; sl.obs = obs; sl.grad = grad;
    sl.sigma_max = sigma_max;
    sl.lane = lane;
    sl.lag = false;
    c->in_batch = true;
    *slot = q;
    return HYB_OK;
}

hyb_status hyb_batch_tick(hyb_batch *b, int32_t steps, int32_t *n_active)
{
    if (!b || steps < 1) return HYB_E_ARG;
    int32_t first = -1;
    while (steps > 0) {
        const int m = std::min(steps, (int32_t)TICKS_PER_PLAN);
        int32_t act = 0;
        hyb_status s = batch_plan_run(b, m, &act);
        if (s) return s;
        if (first < 0) first = act;
        if (act == 0) break;
        steps -= m;
    }
    if (n_active) *n_active = first < 0 ? 0 : first;
    return HYB_OK;
}

hyb_status hyb_batch_poll_all(hyb_batch *b, int32_t *state, double *J)
{
    if (!b || !state) return HYB_E_ARG;
    for (int q = 0; q < b->max_slots; ++q) {
        hyb_status s = hyb_batch_poll(b, q, state + q, J ? J + q : nullptr);
        if (s) return s;
    }
    return HYB_OK;
}

}  // extern "C"


extern "C" {

hyb_status hyb_batch_poll(hyb_batch *b, int32_t slot, int32_t *state, double *J)
{
    if (!b || slot < 0 || slot >= b->max_slots || !state) return HYB_E_ARG;
    hyb_batch::Slot &sl = b->slots[slot];
    int st = sl.state;
    if (st == 3) {
        const hipError_t e = hipEventQuery(sl.done);
        if (e == hipSuccess) {
            // failed: non-finite sigma, or a larger max sigma on the device
            // than the caller's (the CFL check of the submission used the
            // caller's value); finished otherwise
            const bool bad = sl.J_host[1] != 0.0;
            const bool cfl = sl.J_host[0] > std::max(0.0, sl.sigma_max) * (1.0 + 1e-12) + 1e-300;
            st = (bad || cfl) ? 4 : 5;
            if (bad) b->err = "batch: slot " + std::to_string(slot) + ": sigma has non-finite entries";
            else if (cfl)
                b->err = "batch: slot " + std::to_string(slot) + ": max sigma on the device " +
                         std::to_string(sl.J_host[0]) + " exceeds the submitted sigma_max (CFL check)";
            if (J) *J = sl.J_host[2] + sl.J_host[3];
        } else if (e != hipErrorNotReady) {
            return bfail(b, HYB_E_DEVICE, "batch: device error");
        }
    }
    *state = st == 5 ? 2 : (st == 0 ? -1 : (st == 3 ? 1 : (st == 4 ? 3 : 0)));
    return HYB_OK;
}

hyb_status hyb_batch_release(hyb_batch *b, int32_t slot)
{
    if (!b || slot < 0 || slot >= b->max_slots) return HYB_E_ARG;
    hyb_batch::Slot &sl = b->slots[slot];
    if (sl.state == 1 || sl.state == 2) return bfail(b, HYB_E_STATE, "batch: slot still running");
    if (sl.state == 3 && hipEventSynchronize(sl.done) != hipSuccess) return bfail(b, HYB_E_DEVICE, "batch: device error");
    if (sl.c) sl.c->in_batch = false;
    sl.c = nullptr;
    sl.state = 0;
    sl.k = 0; sl.ia = 0; sl.ib = 1; sl.ic = 2;
    sl.data = nullptr; sl.obs = nullptr; sl.grad = nullptr;
    return HYB_OK;
}

const char *hyb_batch_last_error(const hyb_batch *b) { return b ? b->err.c_str() : ""; }

}  // extern "C"
