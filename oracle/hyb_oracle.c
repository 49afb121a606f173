/*
 * Plain FP64 CPU oracle for the domain-decomposition FEM/FDM method of
 * L. Beilina, "Domain decomposition finite element/finite difference method
 * for the conductivity reconstruction in a hyperbolic equation"
 * (arXiv 1509.01399).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled into liboracle.so and is
 * called from the test suite, from the smoke check and from the CPU-baseline
 * leg of the benchmark.  The HIP product library never links, loads or calls
 * it, and it includes nothing from the product.
 *
 * What it computes, in the paper's order (Algorithm 2, Sec. 7.5):
 *   (i)   FDM rows on the structured outer grid, eq. (fdmschemeforward) with
 *         the seven-point Laplacian of Sec. 7.3;
 *   (ii)  FEM rows on the P1-tetrahedral inner mesh, eq. (fem) first line:
 *         lumped mass M^L, element stiffness K^K = (a grad phi_i, grad phi_j)_K
 *         (Sec. 7.2).  The boundary matrix G only touches rows on the FEM
 *         boundary, which step 4 of Algorithm 2 overwrites, so it is omitted;
 *   (iii) the outer boundary: first-order absorbing rows eq. (eq:abs2) and the
 *         Neumann plane-wave source p(t) of eq. (f) on the front face,
 *         discretised with a ghost node;
 *   (iv)  the two overlap copies of Algorithm 2 steps 3-4 (Algorithm 1);
 *   (v)   recording of the backscattered trace on the front face (S_T, Sec. 5).
 * The adjoint is the exact transpose of this discrete sweep (each sub-step
 * transposed literally, in reverse order).  In the interior it coincides with
 * eq. (fdmschemeadjoint) and the second line of eq. (fem).  The gradient with
 * respect to the per-cube conductivity is the discrete form of eq.
 * (gradient1); Algorithm 3 (Sec. 8) is the conjugate-gradient loop.
 *
 * Readings of the paper fixed here (the paper is silent or ambiguous):
 *   - a = 1 + sigma; sigma is piecewise constant per FEM cube, shared by the 6
 *     Kuhn tetrahedra of the cube (a subspace of C_h, eq. (p0)); cubes within
 *     two cells of the FEM boundary keep a = 1 (condition (2.3));
 *   - node sets: omega_o = surface of the FEM box [o, o+C]^3 (FEM boundary,
 *     FDM interior), omega_diamond = surface of [o+2, o+C-2]^3 (FDM inner
 *     boundary, FEM interior) -- a two-element overlap (Sec. 3);
 *   - boundary nodes on edges/corners: a node whose boundary axes are all
 *     reflecting (Neumann, or the source face while the source is on) takes
 *     the ghost-node leapfrog; otherwise it averages the absorbing update of
 *     eq. (eq:abs2) over its absorbing axes.  Faces are done before edges,
 *     edges before corners, so every inward neighbour is final first;
 *   - misfit quadrature: trapezoid weights on the observed face, rectangle
 *     rule in time, cut-off z_delta = 1;
 *   - gradient time pairing: u^k is paired with the multiplier of the update
 *     that consumes it (level k+1), which makes the gradient the exact
 *     derivative of the discrete functional;
 *   - CG step length (cited to another work by the paper): backtracking
 *     from alpha_rel / max|d^m| by halving until the projected point lowers
 *     J, projection onto the admissible set 1 <= a <= 5 of eq. (admpar); a
 *     Fletcher-Reeves direction that is no descent direction restarts as
 *     -g^m (orc_cg_x);
 *   - variable wave speed (eq. (modelhyb)): the coefficient 1/c^2 of the
 *     time derivative is piecewise constant per free cube like a, and 1
 *     elsewhere (condition (coefic)); it weights the element mass matrices,
 *     so each lumped mass is sum_K (1/c^2)_K |K| / 4 (prob_init);
 *   - Model Problem 1 (eq. (model1)): the first level follows from the data
 *     u(x,0) = f0, u_t(x,0) = f1 by the second-order Taylor start
 *     u^1 = u^0 + tau f1 + (tau^2/2) A(u^0) (orc_ic); the paper names the data
 *     but not the start.
 *
 * Parity pins (all in the CPU test suite): the FEM rows equal the seven-point
 * rows when a = 1 (the schemes coincide on structured meshes); hybrid with
 * sigma = 0 equals pure FDM; hybrid equals a whole-grid variable-coefficient
 * stencil assembled independently; discrete energy is conserved with
 * reflecting walls; the plane wave matches its closed form and converges at
 * second order; the adjoint passes a dot test; the gradient matches central
 * finite differences.  The Taylor start reproduces a solution quadratic in
 * time exactly, converges at second order for a travelling pulse with
 * non-zero initial velocity, and its adjoint passes a dot test in (f0, f1).
 * With 1/c^2 the sweep equals an independent whole-grid formulation whose
 * masses come from brute-force Kuhn mass shares, conserves the discrete
 * energy with those masses, and dJ/d(1/c^2) matches central differences.
 * The CG driver (orc_cg) is pinned by rebuilding its iterates from
 * independent gradient evaluations with the formulas of Algorithm 3
 * (beta^m, d^m, the trial steps and the acceptance test), by the first
 * trial being the fixed step alpha_rel / max|d|, and by J decreasing.
 */
#include <math.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

#define ORC_ABC 0
#define ORC_NEUMANN 1
#define ORC_SOURCE 2

/* ------------------------------------------------------------------ types */

typedef struct {
    int32_t n[3];     /* cells per axis; the grid has n+1 nodes per axis      */
    double h;         /* mesh size, the same on every axis                    */
    int32_t bc[6];    /* per face x-,x+,y-,y+,z-,z+: ORC_ABC/NEUMANN/SOURCE     */
    int32_t fem_o[3]; /* lower corner of the FEM box, in cells                */
    int32_t fem_c[3]; /* FEM box size in cells; all zero = no FEM subdomain   */
} orc_geom;

typedef struct {
    int32_t kind;        /* 0: plane wave p(t)=sin(omega t), t < 2 pi/omega  */
    double omega;        /* angular frequency (kind 0)                        */
    const double *flux;  /* kind 1: [nt][(n0+1)(n1+1)] flux per step and node  */
    int32_t k_on;        /* kind 1: the source face is a flux face for k<k_on */
} orc_source;

/* An explicit tetrahedral mesh of the FEM box (node coordinates in the
 * grid's units, x = i h; tetrahedra as 4 node ids).  Nodes on the box
 * surface and on the surface of the inner box [o+2, o+C-2]^3 must be grid
 * nodes; the conductivity is then one value per tetrahedron. */
typedef struct {
    int64_t n_nodes;
    const double *xyz;    /* [n_nodes][3] */
    int64_t n_tets;
    const int32_t *tet4;  /* [n_tets][4] */
} orc_mesh;

typedef struct {
    orc_geom g;
    int nx, ny, nz;        /* grid node counts                                 */
    int64_t nn;            /* grid nodes                                       */
    int nface;             /* nodes on the observed face z = n2                */
    int has_fem;
    int fx, fy, fz;        /* FEM node counts                                  */
    int64_t fn;            /* FEM nodes                                        */
    int64_t ncube;         /* FEM cubes                                        */
    int64_t ntet;
    int32_t *tet;          /* [ntet][4] FEM-local node ids                      */
    int32_t *tcube;        /* [ntet] FEM-local cube id                          */
    double *ke;            /* [ntet][16] element stiffness for a = 1            */
    double *mass;          /* [fn] lumped mass                                  */
    double *acube;         /* [ncube] conductivity a per cube                   */
    uint8_t *eligible;     /* [ncube] 1 if the cube's a is a free parameter     */
    uint8_t *fdm_row;      /* [nn] 1 for FDM-updated interior nodes             */
    uint8_t *fem_row;      /* [fn] 1 for FEM-updated nodes (open box)           */
    int64_t nwo, nwd;      /* sizes of omega_o and omega_diamond                */
    int64_t *wo_g, *wo_f;  /* omega_o as grid / FEM-local indices               */
    int64_t *wd_g, *wd_f;  /* omega_diamond as grid / FEM-local indices         */
    int64_t nb[4];         /* boundary node counts by codimension 1..3          */
    int64_t *bnd[4];       /* boundary nodes by codimension                     */
    double *pvol;          /* [ncube] volume of each parameter cell (cube/tet)   */
    double *ecube;         /* [ncube] wave-speed coefficient 1/c^2 per cube      */
                           /* (lattice mode; 1 on non-free cubes), or NULL       */
    double *tvol;          /* [ntet] tetrahedron volumes (lattice mode)          */
    int64_t *fgrid;        /* [fn] grid index of an FEM node on a grid point, -1 */
} orc_prob;

/* ---------------------------------------------------------------- helpers */

static int64_t gidx(const orc_prob *P, int i, int j, int k)
{
    return (int64_t)i + (int64_t)P->nx * ((int64_t)j + (int64_t)P->ny * k);
}

static int64_t fidx(const orc_prob *P, int a, int b, int c)
{
    return (int64_t)a + (int64_t)P->fx * ((int64_t)b + (int64_t)P->fy * c);
}

static void gcoord(const orc_prob *P, int64_t id, int *x)
{
    x[0] = (int)(id % P->nx);
    x[1] = (int)((id / P->nx) % P->ny);
    x[2] = (int)(id / ((int64_t)P->nx * P->ny));
}

static void prob_free(orc_prob *P)
{
    free(P->tet); free(P->tcube); free(P->ke); free(P->mass); free(P->acube);
    free(P->eligible); free(P->fdm_row); free(P->fem_row);
    free(P->wo_g); free(P->wo_f); free(P->wd_g); free(P->wd_f);
    free(P->pvol); free(P->fgrid); free(P->ecube); free(P->tvol);
    for (int c = 1; c <= 3; ++c) free(P->bnd[c]);
    memset(P, 0, sizeof(*P));
}

/* Validate the geometry: every axis needs at least 2 cells; the FEM box must
 * leave at least one cell to the outer boundary and be at least 5 cells wide
 * so that the two-element overlap leaves an FEM interior.  Returns 0 or -1. */
static int geom_check(const orc_geom *g)
{
    if (!(g->h > 0)) return -1;
    int any = 0, all = 1;
    for (int d = 0; d < 3; ++d) {
        if (g->n[d] < 2) return -1;
        if (g->fem_c[d] != 0) any = 1; else all = 0;
    }
    for (int f = 0; f < 6; ++f) {
        if (g->bc[f] < 0 || g->bc[f] > 2) return -1;
        if (g->bc[f] == ORC_SOURCE && f != 5) return -1;
    }
    if (any && !all) return -1;
    if (any)
        for (int d = 0; d < 3; ++d) {
            if (g->fem_c[d] < 5 || g->fem_o[d] < 1) return -1;
            if (g->fem_o[d] + g->fem_c[d] > g->n[d] - 1) return -1;
        }
    return 0;
}

/* Gradients of the four barycentric coordinates of a tetrahedron and its
 * volume, from the vertex coordinates (standard P1 element, Sec. 7.2). */
static double tet_grads(const double X[4][3], double G[4][3])
{
    double E[3][3];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) E[r][c] = X[c + 1][r] - X[0][r];
    double det = E[0][0] * (E[1][1] * E[2][2] - E[1][2] * E[2][1])
               - E[0][1] * (E[1][0] * E[2][2] - E[1][2] * E[2][0])
               + E[0][2] * (E[1][0] * E[2][1] - E[1][1] * E[2][0]);
    /* inverse of E: row r of E^{-1} is grad of barycentric coordinate r+1 */
    double I[3][3];
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
        G[0][c] = -(I[0][c] + I[1][c] + I[2][c]);
        for (int r = 0; r < 3; ++r) G[r + 1][c] = I[r][c];
    }
    return fabs(det) / 6.0;
}

static int prob_init_mesh(orc_prob *P, const orc_mesh *m, const double *sigma);

/* Build the problem: grid node classes, the FEM mesh (each cube of the FEM box
 * split into the 6 Kuhn tetrahedra sharing the cube diagonal, or the given
 * mesh), element stiffness matrices from the vertex coordinates, lumped
 * masses, and the overlap node sets of Sec. 3.  sigma may be NULL (a = 1
 * everywhere); it holds one value per cube, or per tetrahedron of a given
 * mesh.  eps (lattice mode only; NULL = 1): the coefficient 1/c^2 of the
 * time derivative in eq. (modelhyb), one value per cube, used on the free
 * cubes (c = 1 near and outside the FEM box, condition (coefic)); it weights
 * the element mass matrices, so the lumped mass of node i is
 * sum_{K containing i} eps_K |K| / 4. */
static int prob_init(orc_prob *P, const orc_geom *g, const orc_mesh *m, const double *sigma,
                     const double *eps)
{
    memset(P, 0, sizeof(*P));
    if (geom_check(g)) return -1;
    P->g = *g;
    P->nx = g->n[0] + 1; P->ny = g->n[1] + 1; P->nz = g->n[2] + 1;
    P->nn = (int64_t)P->nx * P->ny * P->nz;
    P->nface = P->nx * P->ny;
    P->has_fem = g->fem_c[0] > 0;
    const int *o = g->fem_o, *C = g->fem_c;

    P->fdm_row = (uint8_t *)calloc((size_t)P->nn, 1);
    for (int k = 1; k < P->nz - 1; ++k)
        for (int j = 1; j < P->ny - 1; ++j)
            for (int i = 1; i < P->nx - 1; ++i) {
                int in_hole = P->has_fem &&
                    i >= o[0] + 2 && i <= o[0] + C[0] - 2 &&
                    j >= o[1] + 2 && j <= o[1] + C[1] - 2 &&
                    k >= o[2] + 2 && k <= o[2] + C[2] - 2;
                P->fdm_row[gidx(P, i, j, k)] = !in_hole;
            }

    /* boundary nodes sorted by codimension */
    int64_t cnt[4] = {0, 0, 0, 0};
    for (int64_t id = 0; id < P->nn; ++id) {
        int x[3]; gcoord(P, id, x);
        int cd = 0;
        for (int d = 0; d < 3; ++d) cd += (x[d] == 0 || x[d] == g->n[d]);
        cnt[cd]++;
    }
    for (int c = 1; c <= 3; ++c) {
        P->bnd[c] = (int64_t *)malloc(sizeof(int64_t) * (size_t)(cnt[c] ? cnt[c] : 1));
        P->nb[c] = 0;
    }
    for (int64_t id = 0; id < P->nn; ++id) {
        int x[3]; gcoord(P, id, x);
        int cd = 0;
        for (int d = 0; d < 3; ++d) cd += (x[d] == 0 || x[d] == g->n[d]);
        if (cd) P->bnd[cd][P->nb[cd]++] = id;
    }

    if (!P->has_fem) return m ? -1 : 0;
    if (m) return eps ? -1 : prob_init_mesh(P, m, sigma);

    P->fx = C[0] + 1; P->fy = C[1] + 1; P->fz = C[2] + 1;
    P->fn = (int64_t)P->fx * P->fy * P->fz;
    P->ncube = (int64_t)C[0] * C[1] * C[2];
    P->ntet = 6 * P->ncube;
    P->tet = (int32_t *)malloc(sizeof(int32_t) * 4 * (size_t)P->ntet);
    P->tcube = (int32_t *)malloc(sizeof(int32_t) * (size_t)P->ntet);
    P->ke = (double *)malloc(sizeof(double) * 16 * (size_t)P->ntet);
    P->mass = (double *)calloc((size_t)P->fn, sizeof(double));
    P->acube = (double *)malloc(sizeof(double) * (size_t)P->ncube);
    P->eligible = (uint8_t *)calloc((size_t)P->ncube, 1);
    P->fem_row = (uint8_t *)calloc((size_t)P->fn, 1);
    P->pvol = (double *)malloc(sizeof(double) * (size_t)P->ncube);
    P->fgrid = (int64_t *)malloc(sizeof(int64_t) * (size_t)P->fn);
    P->ecube = (double *)malloc(sizeof(double) * (size_t)P->ncube);
    P->tvol = (double *)malloc(sizeof(double) * (size_t)P->ntet);
    for (int64_t c = 0; c < P->ncube; ++c) P->pvol[c] = g->h * g->h * g->h;
    for (int c = 0; c < P->fz; ++c)
        for (int b = 0; b < P->fy; ++b)
            for (int a = 0; a < P->fx; ++a) P->fgrid[fidx(P, a, b, c)] = gidx(P, o[0] + a, o[1] + b, o[2] + c);

    static const int perm[6][3] = {{0,1,2},{0,2,1},{1,0,2},{1,2,0},{2,0,1},{2,1,0}};
    int64_t t = 0;
    for (int c = 0; c < C[2]; ++c)
        for (int b = 0; b < C[1]; ++b)
            for (int a = 0; a < C[0]; ++a) {
                int64_t cube = a + (int64_t)C[0] * (b + (int64_t)C[1] * c);
                int elig = a >= 2 && a < C[0] - 2 && b >= 2 && b < C[1] - 2 &&
                           c >= 2 && c < C[2] - 2;
                P->eligible[cube] = (uint8_t)elig;
                P->acube[cube] = 1.0 + ((elig && sigma) ? sigma[cube] : 0.0);
                P->ecube[cube] = (elig && eps) ? eps[cube] : 1.0;
                for (int p = 0; p < 6; ++p, ++t) {
                    int v[3] = {a, b, c};
                    double X[4][3];
                    for (int q = 0; q < 4; ++q) {
                        if (q > 0) v[perm[p][q - 1]] += 1;
                        P->tet[4 * t + q] = (int32_t)fidx(P, v[0], v[1], v[2]);
                        for (int d = 0; d < 3; ++d) X[q][d] = (o[d] + v[d]) * g->h;
                    }
                    double Gr[4][3];
                    double vol = tet_grads(X, Gr);
                    for (int r = 0; r < 4; ++r)
                        for (int s = 0; s < 4; ++s)
                            P->ke[16 * t + 4 * r + s] =
                                vol * (Gr[r][0] * Gr[s][0] + Gr[r][1] * Gr[s][1] +
                                       Gr[r][2] * Gr[s][2]);
                    for (int q = 0; q < 4; ++q) P->mass[P->tet[4 * t + q]] += P->ecube[cube] * vol / 4.0;
                    P->tvol[t] = vol;
                    P->tcube[t] = (int32_t)cube;
                }
            }

    int64_t nwo = 0, nwd = 0;
    for (int c = 0; c < P->fz; ++c)
        for (int b = 0; b < P->fy; ++b)
            for (int a = 0; a < P->fx; ++a) {
                int onb = a == 0 || a == C[0] || b == 0 || b == C[1] || c == 0 || c == C[2];
                int inD = a >= 2 && a <= C[0] - 2 && b >= 2 && b <= C[1] - 2 &&
                          c >= 2 && c <= C[2] - 2;
                int onD = inD && (a == 2 || a == C[0] - 2 || b == 2 || b == C[1] - 2 ||
                                  c == 2 || c == C[2] - 2);
                P->fem_row[fidx(P, a, b, c)] = (uint8_t)!onb;
                nwo += onb; nwd += onD;
            }
    P->nwo = nwo; P->nwd = nwd;
    P->wo_g = (int64_t *)malloc(sizeof(int64_t) * (size_t)nwo);
    P->wo_f = (int64_t *)malloc(sizeof(int64_t) * (size_t)nwo);
    P->wd_g = (int64_t *)malloc(sizeof(int64_t) * (size_t)nwd);
    P->wd_f = (int64_t *)malloc(sizeof(int64_t) * (size_t)nwd);
    nwo = nwd = 0;
    for (int c = 0; c < P->fz; ++c)
        for (int b = 0; b < P->fy; ++b)
            for (int a = 0; a < P->fx; ++a) {
                int onb = a == 0 || a == C[0] || b == 0 || b == C[1] || c == 0 || c == C[2];
                int inD = a >= 2 && a <= C[0] - 2 && b >= 2 && b <= C[1] - 2 &&
                          c >= 2 && c <= C[2] - 2;
                int onD = inD && (a == 2 || a == C[0] - 2 || b == 2 || b == C[1] - 2 ||
                                  c == 2 || c == C[2] - 2);
                int64_t gi = gidx(P, o[0] + a, o[1] + b, o[2] + c), fi = fidx(P, a, b, c);
                if (onb) { P->wo_g[nwo] = gi; P->wo_f[nwo] = fi; ++nwo; }
                if (onD) { P->wd_g[nwd] = gi; P->wd_f[nwd] = fi; ++nwd; }
            }
    return 0;
}

/* FEM part of the problem from an explicit mesh (the grid part is set up).
 * The parameter cells are the tetrahedra; a tetrahedron is a free parameter
 * when all its vertices lie in the closed inner box [o+2, o+C-2]^3 (a = 1 on
 * the two-element overlap, condition (2.3)).  FEM rows: the nodes inside the
 * open box; omega_o: the mesh nodes on the box surface (grid nodes);
 * omega_diamond: the grid nodes on the inner box surface, each of which must
 * be a mesh node.  Returns 0 or -1 (mesh not conforming to the grid). */
static int prob_init_mesh(orc_prob *P, const orc_mesh *m, const double *sigma)
{
    const orc_geom *g = &P->g;
    const int *o = g->fem_o, *C = g->fem_c;
    const double h = g->h, tol = 1e-9;
    if (m->n_nodes < 4 || m->n_tets < 1) return -1;
    P->fn = m->n_nodes;
    P->ntet = m->n_tets;
    P->ncube = m->n_tets;
    P->tet = (int32_t *)malloc(sizeof(int32_t) * 4 * (size_t)P->ntet);
    P->tcube = (int32_t *)malloc(sizeof(int32_t) * (size_t)P->ntet);
    P->ke = (double *)malloc(sizeof(double) * 16 * (size_t)P->ntet);
    P->mass = (double *)calloc((size_t)P->fn, sizeof(double));
    P->acube = (double *)malloc(sizeof(double) * (size_t)P->ncube);
    P->eligible = (uint8_t *)calloc((size_t)P->ncube, 1);
    P->fem_row = (uint8_t *)calloc((size_t)P->fn, 1);
    P->pvol = (double *)malloc(sizeof(double) * (size_t)P->ncube);
    P->fgrid = (int64_t *)malloc(sizeof(int64_t) * (size_t)P->fn);
    uint8_t *inner = (uint8_t *)calloc((size_t)P->fn, 1);
    /* node positions in cells: grid points, box surface, inner box */
    int64_t nwo = 0;
    for (int64_t n = 0; n < P->fn; ++n) {
        double q[3];
        int grid = 1, inside = 1, surf = 0, in_inner = 1;
        long long qi[3];
        for (int d = 0; d < 3; ++d) {
            q[d] = m->xyz[3 * n + d] / h;
            qi[d] = llround(q[d]);
            if (fabs(q[d] - (double)qi[d]) > tol) grid = 0;
            if (q[d] < o[d] - tol || q[d] > o[d] + C[d] + tol) inside = 0;
            if (fabs(q[d] - o[d]) <= tol || fabs(q[d] - (o[d] + C[d])) <= tol) surf = 1;
            if (q[d] < o[d] + 2 - tol || q[d] > o[d] + C[d] - 2 + tol) in_inner = 0;
        }
        if (!inside || (surf && !grid)) { free(inner); return -1; }
        P->fgrid[n] = grid ? gidx(P, (int)qi[0], (int)qi[1], (int)qi[2]) : -1;
        P->fem_row[n] = (uint8_t)!surf;
        inner[n] = (uint8_t)in_inner;
        nwo += surf;
    }
    /* elements */
    for (int64_t t = 0; t < P->ntet; ++t) {
        double X[4][3], Gr[4][3];
        int all_inner = 1;
        for (int q = 0; q < 4; ++q) {
            int32_t v = m->tet4[4 * t + q];
            if (v < 0 || v >= P->fn) { free(inner); return -1; }
            P->tet[4 * t + q] = v;
            for (int d = 0; d < 3; ++d) X[q][d] = m->xyz[3 * v + d];
            all_inner &= inner[v];
        }
        double vol = tet_grads(X, Gr);
        if (!(vol > 1e-12 * h * h * h)) { free(inner); return -1; }
        for (int r = 0; r < 4; ++r)
            for (int c = 0; c < 4; ++c)
                P->ke[16 * t + 4 * r + c] = vol * (Gr[r][0] * Gr[c][0] + Gr[r][1] * Gr[c][1] + Gr[r][2] * Gr[c][2]);
        for (int q = 0; q < 4; ++q) P->mass[P->tet[4 * t + q]] += vol / 4.0;
        P->tcube[t] = (int32_t)t;
        P->pvol[t] = vol;
        P->eligible[t] = (uint8_t)all_inner;
        P->acube[t] = 1.0 + ((all_inner && sigma) ? sigma[t] : 0.0);
    }
    free(inner);
    /* omega_o: the box-surface nodes; they must be all grid nodes of the surface */
    int64_t want = (int64_t)(C[0] + 1) * (C[1] + 1) * (C[2] + 1) - (int64_t)(C[0] - 1) * (C[1] - 1) * (C[2] - 1);
    if (nwo != want) return -1;
    P->nwo = nwo;
    P->wo_g = (int64_t *)malloc(sizeof(int64_t) * (size_t)nwo);
    P->wo_f = (int64_t *)malloc(sizeof(int64_t) * (size_t)nwo);
    nwo = 0;
    for (int64_t n = 0; n < P->fn; ++n)
        if (!P->fem_row[n]) { P->wo_g[nwo] = P->fgrid[n]; P->wo_f[nwo] = n; ++nwo; }
    /* omega_diamond: grid nodes on the inner box surface, matched to mesh nodes */
    int64_t *node_at = (int64_t *)malloc(sizeof(int64_t) * (size_t)P->nn);
    for (int64_t i = 0; i < P->nn; ++i) node_at[i] = -1;
    for (int64_t n = 0; n < P->fn; ++n)
        if (P->fgrid[n] >= 0) node_at[P->fgrid[n]] = n;
    const int L = C[0] - 4;
    int64_t nwd = 0;
    P->wd_g = (int64_t *)malloc(sizeof(int64_t) * (size_t)(6 * (L + 1) * (L + 1)));
    P->wd_f = (int64_t *)malloc(sizeof(int64_t) * (size_t)(6 * (L + 1) * (L + 1)));
    for (int c = 0; c <= C[2] - 4; ++c)
        for (int b = 0; b <= C[1] - 4; ++b)
            for (int a = 0; a <= C[0] - 4; ++a) {
                if (!(a == 0 || a == C[0] - 4 || b == 0 || b == C[1] - 4 || c == 0 || c == C[2] - 4)) continue;
                int64_t gi = gidx(P, o[0] + 2 + a, o[1] + 2 + b, o[2] + 2 + c);
                if (node_at[gi] < 0) { free(node_at); return -1; }
                P->wd_g[nwd] = gi; P->wd_f[nwd] = node_at[gi]; ++nwd;
            }
    P->nwd = nwd;
    free(node_at);
    return 0;
}

/* Number of steps k whose time t_k = k*dt lies before the end 2 pi/omega of
 * the plane-wave pulse of eq. (f); for a flux table, the caller's k_on. */
static int source_k_on(const orc_source *S, int nt, double dt)
{
    if (!S) return 0;
    if (S->kind == 1) return S->k_on;
    int kon = 0;
    double t1 = 2.0 * M_PI / S->omega;
    for (int k = 0; k < nt; ++k)
        if ((double)k * dt < t1) kon = k + 1;
    return kon;
}

/* p(t_k) at face node (i,j) of the front face, eq. (f). */
static double source_flux(const orc_prob *P, const orc_source *S, int k, double dt, int i, int j)
{
    if (S->kind == 1) return S->flux[(int64_t)k * P->nface + i + (int64_t)P->nx * j];
    return sin(S->omega * ((double)k * dt));
}

/* Classification of a boundary node for the update at step k (k -> k+1).
 * nb: number of boundary axes; ax/dir: boundary axis and inward direction;
 * kind[m]: 0 absorbing, 1 reflecting (Neumann ghost), 2 source flux. */
typedef struct { int nb; int ax[3]; int dir[3]; int kind[3]; int ghost_row; int nabc; } bclass;

static bclass classify(const orc_prob *P, const int *x, int src_on)
{
    bclass B; memset(&B, 0, sizeof(B));
    for (int d = 0; d < 3; ++d) {
        int f = -1, dir = 0;
        if (x[d] == 0) { f = 2 * d; dir = 1; }
        else if (x[d] == P->g.n[d]) { f = 2 * d + 1; dir = -1; }
        if (f < 0) continue;
        int bc = P->g.bc[f], kind;
        if (bc == ORC_NEUMANN) kind = 1;
        else if (bc == ORC_SOURCE) kind = src_on ? 2 : 0;
        else kind = 0;
        B.ax[B.nb] = d; B.dir[B.nb] = dir; B.kind[B.nb] = kind; B.nb++;
        if (kind == 0) B.nabc++;
    }
    B.ghost_row = (B.nabc == 0);
    return B;
}

/* ---------------------------------------------------------------- forward */

/* One time step of Algorithm 2 (Sec. 7.5): levels (Um,U) -> Up, (Vm,V) -> Vp.
 * r is FEM scratch of size fn.  w2 weights tau^2 in the rows that take the
 * leapfrog (1; 1/2 in the first step of the Taylor start, see
 * forward_sweep); the absorbing rows do not depend on it. */
static void step_forward(const orc_prob *P, int k, double dt, double w2, const orc_source *S, int k_on,
                         const double *Um, const double *U, double *Up,
                         const double *Vm, const double *V, double *Vp, double *r)
{
    const double h = P->g.h, h2 = h * h, tau2 = w2 * dt * dt;
    const double rr = (h - dt) / (h + dt);  /* coefficient of eq. (eq:abs2) */
    memset(Up, 0, sizeof(double) * (size_t)P->nn);

    /* (i) FDM rows: u^{k+1} = tau^2 Lap u^k + 2 u^k - u^{k-1},
     *     eq. (fdmschemeforward) with the seven-point Laplacian.  Every row
     *     writes only its own node, so the z planes run on parallel threads
     *     with the same result as one thread. */
#pragma omp parallel for schedule(static)
    for (int kk = 1; kk < P->nz - 1; ++kk)
        for (int j = 1; j < P->ny - 1; ++j)
            for (int i = 1; i < P->nx - 1; ++i) {
                int64_t id = gidx(P, i, j, kk);
                if (!P->fdm_row[id]) continue;
                double u = U[id];
                double lap = (U[id + 1] - 2.0 * u + U[id - 1]) / h2
                           + (U[id + P->nx] - 2.0 * u + U[id - P->nx]) / h2
                           + (U[id + (int64_t)P->nx * P->ny] - 2.0 * u +
                              U[id - (int64_t)P->nx * P->ny]) / h2;
                Up[id] = tau2 * lap + 2.0 * u - Um[id];
            }

    /* (ii) FEM rows: u^{k+1} = 2u^k - tau^2 (M^L)^{-1} K u^k - u^{k-1},
     *      eq. (fem), with K = sum over tetrahedra of a_K K^K. */
    if (P->has_fem) {
        memset(Vp, 0, sizeof(double) * (size_t)P->fn);
        memset(r, 0, sizeof(double) * (size_t)P->fn);
        for (int64_t t = 0; t < P->ntet; ++t) {
            const int32_t *v = P->tet + 4 * t;
            const double *ke = P->ke + 16 * t;
            double a = P->acube[P->tcube[t]];
            for (int q = 0; q < 4; ++q) {
                double s = 0.0;
                for (int w = 0; w < 4; ++w) s += ke[4 * q + w] * V[v[w]];
                r[v[q]] += a * s;
            }
        }
        for (int64_t n = 0; n < P->fn; ++n)
            if (P->fem_row[n]) Vp[n] = 2.0 * V[n] - tau2 * r[n] / P->mass[n] - Vm[n];
    }

    /* (iii) outer boundary, faces then edges then corners. */
    int src_on = k < k_on;
    for (int cd = 1; cd <= 3; ++cd)
        for (int64_t m = 0; m < P->nb[cd]; ++m) {
            int64_t id = P->bnd[cd][m];
            int x[3]; gcoord(P, id, x);
            bclass B = classify(P, x, src_on);
            if (B.ghost_row) {
                /* ghost-node leapfrog: each reflecting axis contributes
                 * 2(u_in - u)/h^2, the source axis adds 2 p(t_k)/h. */
                double u = U[id], lap = 0.0, src = 0.0;
                for (int d = 0; d < 3; ++d) {
                    int m2 = -1;
                    for (int q = 0; q < B.nb; ++q) if (B.ax[q] == d) m2 = q;
                    int64_t st = d == 0 ? 1 : (d == 1 ? P->nx : (int64_t)P->nx * P->ny);
                    if (m2 < 0) {
                        lap += (U[id + st] - 2.0 * u + U[id - st]) / h2;
                    } else {
                        lap += 2.0 * (U[id + B.dir[m2] * st] - u) / h2;
                        if (B.kind[m2] == 2) src += 2.0 * source_flux(P, S, k, dt, x[0], x[1]) / h;
                    }
                }
                Up[id] = tau2 * (lap + src) + 2.0 * u - Um[id];
            } else {
                /* absorbing row, eq. (eq:abs2), averaged over absorbing axes */
                double acc = 0.0;
                for (int q = 0; q < B.nb; ++q) {
                    if (B.kind[q] != 0) continue;
                    int d = B.ax[q];
                    int64_t st = d == 0 ? 1 : (d == 1 ? P->nx : (int64_t)P->nx * P->ny);
                    int64_t in = id + B.dir[q] * st;
                    acc += U[in] + rr * (U[id] - Up[in]);
                }
                Up[id] = acc / B.nabc;
            }
        }

    /* (iv) exchange, Algorithm 2 steps 3 and 4. */
    if (P->has_fem) {
        for (int64_t m = 0; m < P->nwd; ++m) Up[P->wd_g[m]] = Vp[P->wd_f[m]];
        for (int64_t m = 0; m < P->nwo; ++m) Vp[P->wo_f[m]] = Up[P->wo_g[m]];
    }
}

static void record_face(const orc_prob *P, const double *U, double *row)
{
    int64_t base = gidx(P, 0, 0, P->nz - 1);
    memcpy(row, U + base, sizeof(double) * (size_t)P->nface);
}

/* Initial data of a sweep (on the whole grid; NULL arrays are zero).
 * taylor = 0: the leapfrog starts from the given levels u^0 = u0 and
 *   u^{-1} = um1 (zero for Model Problem 2).
 * taylor = 1: Model Problem 1, eq. (model1): u(x,0) = u0 (f_0) and
 *   u_t(x,0) = f1 (f_1).  The first level is the second-order Taylor
 *   expansion u^1 = u^0 + tau f_1 + (tau^2/2) A(u^0), A(u^0) the acceleration
 *   the scheme assigns to level 0 (its leapfrog rows with the source at
 *   t_0).  Written as a leapfrog step it is the step from the virtual level
 *   u^{-1} = u^0 - tau f_1 with tau^2 weighted by 1/2:
 *   2u^0 - (u^0 - tau f_1) + (tau^2/2) A(u^0).  The absorbing rows of
 *   eq. (eq:abs2) use levels 0 and 1 only and are unchanged. */
typedef struct {
    const double *u0, *um1, *f1;
    int taylor;
} orc_ic;

/* tau^2 weight of step k. */
static double step_w2(const orc_ic *ic, int k) { return (ic->taylor && k == 0) ? 0.5 : 1.0; }

/* Full forward sweep from the initial data ic.  obs: [nt+1][nface].
 * vhist (optional): [nt+1][fn] FEM levels.  ufin (optional): u^{nt}. */
static int forward_sweep(const orc_prob *P, const orc_source *S, int nt, double dt,
                         const orc_ic *ic, double *obs, double *vhist, double *ufin)
{
    int k_on = source_k_on(S, nt, dt);
    size_t gb = sizeof(double) * (size_t)P->nn, fb = sizeof(double) * (size_t)(P->fn ? P->fn : 1);
    double *Ua = (double *)calloc(1, gb), *Ub = (double *)calloc(1, gb), *Uc = (double *)calloc(1, gb);
    double *Va = (double *)calloc(1, fb), *Vb = (double *)calloc(1, fb), *Vc = (double *)calloc(1, fb);
    double *r = (double *)calloc(1, fb);
    if (!Ua || !Ub || !Uc || !Va || !Vb || !Vc || !r) return -2;
    const double *u0 = ic->u0, *um1 = ic->taylor ? NULL : ic->um1;
    if (u0) memcpy(Ub, u0, gb);
    if (um1) memcpy(Ua, um1, gb);
    if (ic->taylor) {
        /* virtual level u^{-1} = u^0 - tau f_1 */
        for (int64_t i = 0; i < P->nn; ++i)
            Ua[i] = (u0 ? u0[i] : 0.0) - (ic->f1 ? dt * ic->f1[i] : 0.0);
        um1 = Ua;
    }
    if (P->has_fem)
        for (int64_t f = 0; f < P->fn; ++f) {
            /* FEM copies of the initial levels: defined on grid points only */
            if (P->fgrid[f] >= 0) { Vb[f] = Ub[P->fgrid[f]]; Va[f] = Ua[P->fgrid[f]]; }
            else if (u0 || um1) { free(Ua); free(Ub); free(Uc); free(Va); free(Vb); free(Vc); free(r); return -1; }
        }
    double *Um = Ua, *U = Ub, *Up = Uc, *Vm = Va, *V = Vb, *Vp = Vc;
    if (obs) record_face(P, U, obs);
    if (vhist && P->has_fem) memcpy(vhist, V, fb);
    for (int k = 0; k < nt; ++k) {
        step_forward(P, k, dt, step_w2(ic, k), S, k_on, Um, U, Up, Vm, V, Vp, r);
        double *t1 = Um; Um = U; U = Up; Up = t1;          /* swap, Alg. 2 step 5 */
        double *t2 = Vm; Vm = V; V = Vp; Vp = t2;
        if (obs) record_face(P, U, obs + (int64_t)(k + 1) * P->nface);
        if (vhist && P->has_fem) memcpy(vhist + (int64_t)(k + 1) * P->fn, V, fb);
    }
    if (ufin) memcpy(ufin, U, gb);
    free(Ua); free(Ub); free(Uc); free(Va); free(Vb); free(Vc); free(r);
    return 0;
}

/* ---------------------------------------------------------------- adjoint */

/* Exact transpose of step_forward(k): cotangents of level k+1 (aUp, aVp) are
 * consumed and pushed to levels k (aU, aV) and k-1 (aUm, aVm).  V is the
 * forward FEM level k (for the conductivity derivative); dsig accumulates
 * dJ/da per cube; dflux (optional) accumulates the source cotangent. */
static void step_adjoint(const orc_prob *P, int k, double dt, double w2, const orc_source *S, int k_on,
                         double *aUm, double *aU, double *aUp,
                         double *aVm, double *aV, double *aVp,
                         const double *V, double *dsig, double *dflux, double *gsave,
                         double *deps, double *rsave)
{
    const double h = P->g.h, h2 = h * h, tau2 = w2 * dt * dt;
    const double rr = (h - dt) / (h + dt);

    /* (iv)^T: V[omega_o] = U[omega_o] was done last, so it is undone first. */
    if (P->has_fem) {
        for (int64_t m = 0; m < P->nwo; ++m) {
            aUp[P->wo_g[m]] += aVp[P->wo_f[m]];
            aVp[P->wo_f[m]] = 0.0;
        }
        for (int64_t m = 0; m < P->nwd; ++m) {
            aVp[P->wd_f[m]] += aUp[P->wd_g[m]];
            aUp[P->wd_g[m]] = 0.0;
        }
    }

    /* (iii)^T: corners, then edges, then faces. */
    int src_on = k < k_on;
    for (int cd = 3; cd >= 1; --cd)
        for (int64_t m = 0; m < P->nb[cd]; ++m) {
            int64_t id = P->bnd[cd][m];
            int x[3]; gcoord(P, id, x);
            bclass B = classify(P, x, src_on);
            double gb = aUp[id];
            aUp[id] = 0.0;
            if (B.ghost_row) {
                for (int d = 0; d < 3; ++d) {
                    int m2 = -1;
                    for (int q = 0; q < B.nb; ++q) if (B.ax[q] == d) m2 = q;
                    int64_t st = d == 0 ? 1 : (d == 1 ? P->nx : (int64_t)P->nx * P->ny);
                    if (m2 < 0) {
                        aU[id + st] += tau2 / h2 * gb;
                        aU[id - st] += tau2 / h2 * gb;
                        aU[id] -= 2.0 * tau2 / h2 * gb;
                    } else {
                        aU[id + B.dir[m2] * st] += 2.0 * tau2 / h2 * gb;
                        aU[id] -= 2.0 * tau2 / h2 * gb;
                        if (B.kind[m2] == 2 && dflux)
                            dflux[(int64_t)k * P->nface + x[0] + (int64_t)P->nx * x[1]] +=
                                2.0 * tau2 / h * gb;
                    }
                }
                aU[id] += 2.0 * gb;
                aUm[id] -= gb;
            } else {
                for (int q = 0; q < B.nb; ++q) {
                    if (B.kind[q] != 0) continue;
                    int d = B.ax[q];
                    int64_t st = d == 0 ? 1 : (d == 1 ? P->nx : (int64_t)P->nx * P->ny);
                    int64_t in = id + B.dir[q] * st;
                    aU[in] += gb / B.nabc;
                    aU[id] += rr * gb / B.nabc;
                    aUp[in] -= rr * gb / B.nabc;
                }
            }
        }

    /* (ii)^T: FEM rows. */
    if (P->has_fem) {
        for (int64_t n = 0; n < P->fn; ++n) {
            gsave[n] = 0.0;
            if (!P->fem_row[n]) continue;
            double gv = aVp[n];
            aVp[n] = 0.0;
            aV[n] += 2.0 * gv;
            aVm[n] -= gv;
            gsave[n] = -tau2 * gv / P->mass[n];   /* cotangent of (K u^k)_n */
        }
        for (int64_t t = 0; t < P->ntet; ++t) {
            const int32_t *v = P->tet + 4 * t;
            const double *ke = P->ke + 16 * t;
            int64_t cube = P->tcube[t];
            double a = P->acube[cube];
            for (int q = 0; q < 4; ++q) {
                double gq = gsave[v[q]];
                if (gq == 0.0) continue;
                double s = 0.0;
                for (int w = 0; w < 4; ++w) {
                    aV[v[w]] += gq * a * ke[4 * q + w];
                    s += ke[4 * q + w] * V[v[w]];
                }
                if (P->eligible[cube]) dsig[cube] += gq * s;
            }
        }
        /* wave-speed coefficient: the FEM row n divides by its lumped mass
         * m_n, so dJ/dm_n = (cotangent of v_n^{k+1}) tau^2 (K u^k)_n / m_n^2
         * = -gsave_n (K u^k)_n / m_n, and m_n = sum_{K containing n}
         * eps_K |K| / 4 passes it to the cubes. */
        if (deps && P->ecube) {
            memset(rsave, 0, sizeof(double) * (size_t)P->fn);
            for (int64_t t = 0; t < P->ntet; ++t) {
                const int32_t *v = P->tet + 4 * t;
                const double *ke = P->ke + 16 * t;
                double a = P->acube[P->tcube[t]];
                for (int q = 0; q < 4; ++q) {
                    double s = 0.0;
                    for (int w = 0; w < 4; ++w) s += ke[4 * q + w] * V[v[w]];
                    rsave[v[q]] += a * s;
                }
            }
            for (int64_t n = 0; n < P->fn; ++n)
                rsave[n] = P->fem_row[n] ? -gsave[n] * rsave[n] / P->mass[n] : 0.0;
            for (int64_t t = 0; t < P->ntet; ++t) {
                int64_t cube = P->tcube[t];
                if (!P->eligible[cube]) continue;
                const int32_t *v = P->tet + 4 * t;
                for (int q = 0; q < 4; ++q) deps[cube] += P->tvol[t] / 4.0 * rsave[v[q]];
            }
        }
    }

    /* (i)^T: FDM rows.  The row of node m reads u^k at m and its six
     * neighbours and u^{k-1} at m, so its cotangent g_m = aUp[m] goes to
     * aU[m] with weight 2 - 6 tau^2/h^2, to aU of each neighbour with
     * tau^2/h^2 and to aUm[m] with -1.  Gathered per receiving node (its own
     * row first, then the neighbours' rows in a fixed order), every node is
     * written by one thread only: the z planes run in parallel with the same
     * result as one thread.  aUp is read in a first pass and cleared in a
     * second. */
    {
        const double c = tau2 / h2;
        const int64_t st[3] = {1, P->nx, (int64_t)P->nx * P->ny};
        const int n3[3] = {P->nx, P->ny, P->nz};
#pragma omp parallel for schedule(static)
        for (int kk = 0; kk < P->nz; ++kk)
            for (int j = 0; j < P->ny; ++j)
                for (int i = 0; i < P->nx; ++i) {
                    int64_t id = gidx(P, i, j, kk);
                    const int x[3] = {i, j, kk};
                    double acc = aU[id];
                    if (P->fdm_row[id]) {
                        double g = aUp[id];
                        acc += (2.0 - 6.0 * c) * g;
                        aUm[id] -= g;
                    }
                    for (int d = 0; d < 3; ++d) {
                        if (x[d] > 0 && P->fdm_row[id - st[d]]) acc += c * aUp[id - st[d]];
                        if (x[d] < n3[d] - 1 && P->fdm_row[id + st[d]]) acc += c * aUp[id + st[d]];
                    }
                    aU[id] = acc;
                }
#pragma omp parallel for schedule(static)
        for (int64_t id = 0; id < P->nn; ++id)
            if (P->fdm_row[id]) aUp[id] = 0.0;
    }
}

/* Reverse sweep.  seed: [nt+1][nface] cotangent of the recorded trace.
 * vhist: forward FEM levels [nt+1][fn].  Outputs (each optional): dsig
 * [ncube] dJ/da_c (Euclidean), dflux [nt][nface], du0 and dum1 [nn]
 * cotangents of the initial levels. */
static int adjoint_sweep(const orc_prob *P, const orc_source *S, int nt, double dt, const orc_ic *ic,
                         const double *seed, const double *vhist, double *dsig, double *deps,
                         double *dflux, double *du0, double *dum1)
{
    int k_on = source_k_on(S, nt, dt);
    size_t gb = sizeof(double) * (size_t)P->nn, fb = sizeof(double) * (size_t)(P->fn ? P->fn : 1);
    double *A0 = (double *)calloc(1, gb), *A1 = (double *)calloc(1, gb), *A2 = (double *)calloc(1, gb);
    double *B0 = (double *)calloc(1, fb), *B1 = (double *)calloc(1, fb), *B2 = (double *)calloc(1, fb);
    double *gs = (double *)calloc(1, fb), *rs = (double *)calloc(1, fb);
    if (!A0 || !A1 || !A2 || !B0 || !B1 || !B2 || !gs || !rs) return -2;
    double *aUm = A0, *aU = A1, *aUp = A2, *aVm = B0, *aV = B1, *aVp = B2;
    int64_t base = gidx(P, 0, 0, P->nz - 1);
    if (dsig && P->has_fem) memset(dsig, 0, sizeof(double) * (size_t)P->ncube);
    if (deps && P->has_fem) memset(deps, 0, sizeof(double) * (size_t)P->ncube);
    for (int k = nt - 1; k >= 0; --k) {
        /* (v)^T: the trace of level k+1 */
        const double *sd = seed + (int64_t)(k + 1) * P->nface;
        for (int q = 0; q < P->nface; ++q) aUp[base + q] += sd[q];
        step_adjoint(P, k, dt, step_w2(ic, k), S, k_on, aUm, aU, aUp, aVm, aV, aVp,
                     P->has_fem ? vhist + (int64_t)k * P->fn : NULL, dsig, dflux, gs, deps, rs);
        /* aUp is fully consumed; rotate: level k becomes the newest */
        double *t1 = aUp; aUp = aU; aU = aUm; aUm = t1;
        memset(aUm, 0, gb);
        double *t2 = aVp; aVp = aV; aV = aVm; aVm = t2;
        memset(aVm, 0, fb);
    }
    /* level 0 trace, then fold the FEM copies of the initial levels back. */
    for (int q = 0; q < P->nface; ++q) aUp[base + q] += seed[q];
    if (P->has_fem)
        for (int64_t f = 0; f < P->fn; ++f)
            if (P->fgrid[f] >= 0) {
                aUp[P->fgrid[f]] += aVp[f];
                aU[P->fgrid[f]] += aV[f];
            }
    if (du0) memcpy(du0, aUp, gb);
    if (dum1) memcpy(dum1, aU, gb);
    free(A0); free(A1); free(A2); free(B0); free(B1); free(B2); free(gs); free(rs);
    return 0;
}

/* Trapezoid weight of face node (i,j) on the observed face. */
static double face_weight(const orc_prob *P, int i, int j)
{
    double w = P->g.h * P->g.h;
    if (i == 0 || i == P->nx - 1) w *= 0.5;
    if (j == 0 || j == P->ny - 1) w *= 0.5;
    return w;
}

/* ---------------------------------------------------------- exported API */

/* Threads of the FDM rows (OpenMP over z planes; n <= 0 leaves the setting);
 * returns the number now in use.  Results do not depend on it. */
int orc_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* Every entry point takes an optional explicit mesh m (NULL: the 6-tetrahedra
 * split of the FEM box); with a mesh, sigma, dsig and grad hold one value per
 * tetrahedron.  The _x calls take every option:
 *   eps:  1/c^2 per cube (lattice mode only; NULL = 1), see prob_init;
 *   u0, u1, taylor: initial data, see orc_ic (taylor = 0: levels u^0 = u0,
 *         u^{-1} = u1; taylor = 1: Model Problem 1 data f0 = u0, f1 = u1).
 * The names without _x are the same calls with eps = NULL and the given
 * levels (or zero data); without _m also without a mesh. */

/* Sizes: out[0] grid nodes, out[1] face nodes, out[2] FEM nodes,
 * out[3] parameter cells (cubes, or tetrahedra of a given mesh),
 * out[4] FEM-updated nodes, out[5] FDM-updated nodes (interior + boundary),
 * out[6] |omega_o|, out[7] |omega_diamond|. */
int orc_sizes_m(const orc_geom *g, const orc_mesh *m, int64_t *out)
{
    orc_prob P;
    if (prob_init(&P, g, m, NULL, NULL)) return -1;
    int64_t nfdm = 0, nfem = 0;
    for (int64_t i = 0; i < P.nn; ++i) nfdm += P.fdm_row[i];
    nfdm += P.nb[1] + P.nb[2] + P.nb[3];
    for (int64_t i = 0; i < P.fn; ++i) nfem += P.fem_row[i];
    out[0] = P.nn; out[1] = P.nface; out[2] = P.fn; out[3] = P.ncube;
    out[4] = nfem; out[5] = nfdm; out[6] = P.nwo; out[7] = P.nwd;
    prob_free(&P);
    return 0;
}

int orc_sizes(const orc_geom *g, int64_t *out) { return orc_sizes_m(g, NULL, out); }

/* Forward solve: obs [nt+1][nface]; vhist [nt+1][fn], ufin [nn] optional
 * (initial data need every FEM node on a grid point). */
int orc_forward_x(const orc_geom *g, const orc_mesh *m, const double *sigma, const double *eps,
                  const orc_source *S, int nt, double dt, const double *u0, const double *u1, int taylor,
                  double *obs, double *vhist, double *ufin)
{
    orc_prob P;
    if (nt < 0 || !(dt > 0) || prob_init(&P, g, m, sigma, eps)) return -1;
    const orc_ic ic = {u0, taylor ? NULL : u1, taylor ? u1 : NULL, taylor};
    int rc = forward_sweep(&P, S, nt, dt, &ic, obs, vhist, ufin);
    prob_free(&P);
    return rc;
}

int orc_forward_m(const orc_geom *g, const orc_mesh *m, const double *sigma, const orc_source *S, int nt,
                  double dt, const double *u0, const double *um1, double *obs, double *vhist, double *ufin)
{
    return orc_forward_x(g, m, sigma, NULL, S, nt, dt, u0, um1, 0, obs, vhist, ufin);
}

int orc_forward(const orc_geom *g, const double *sigma, const orc_source *S, int nt, double dt,
                const double *u0, const double *um1, double *obs, double *vhist, double *ufin)
{
    return orc_forward_x(g, NULL, sigma, NULL, S, nt, dt, u0, um1, 0, obs, vhist, ufin);
}

/* Linear adjoint: given the cotangent seed [nt+1][nface] of the trace,
 * returns dsig [cells] = dJ/da per parameter cell (Euclidean, zero on
 * non-eligible cells) and, each optional: deps [cubes] = dJ/d(1/c^2) per
 * cube (Euclidean, zero on non-eligible cubes; lattice mode), dflux
 * [nt][nface], du0 and dum1 [nn] the cotangents of the levels u^0 and u^{-1}
 * (with the FEM copies folded back), and with taylor df0, df1 [nn] those of
 * the Model Problem 1 data: u^{-1} = f0 - tau f1, so df0 = du0 + dum1 and
 * df1 = -tau dum1. */
int orc_adjoint_x(const orc_geom *g, const orc_mesh *m, const double *sigma, const double *eps,
                  const orc_source *S, int nt, double dt, const double *u0, const double *u1, int taylor,
                  const double *seed, double *dsig, double *deps, double *dflux, double *du0, double *dum1,
                  double *df0, double *df1)
{
    orc_prob P;
    if (nt < 0 || !(dt > 0) || prob_init(&P, g, m, sigma, eps)) return -1;
    const orc_ic ic = {u0, taylor ? NULL : u1, taylor ? u1 : NULL, taylor};
    size_t gb = sizeof(double) * (size_t)P.nn;
    double *vh = NULL, *a0 = (double *)malloc(gb), *a1 = (double *)malloc(gb);
    if (!a0 || !a1) { free(a0); free(a1); prob_free(&P); return -2; }
    if (P.has_fem) {
        vh = (double *)malloc(sizeof(double) * (size_t)P.fn * (size_t)(nt + 1));
        if (!vh) { free(a0); free(a1); prob_free(&P); return -2; }
        if (forward_sweep(&P, S, nt, dt, &ic, NULL, vh, NULL)) {
            free(vh); free(a0); free(a1); prob_free(&P);
            return -1;
        }
    }
    if (dflux) memset(dflux, 0, sizeof(double) * (size_t)nt * (size_t)P.nface);
    int rc = adjoint_sweep(&P, S, nt, dt, &ic, seed, vh, dsig, deps, dflux, a0, a1);
    if (!rc)
        for (int64_t i = 0; i < P.nn; ++i) {
            if (du0) du0[i] = a0[i];
            if (dum1) dum1[i] = a1[i];
            if (df0) df0[i] = a0[i] + a1[i];
            if (df1) df1[i] = -dt * a1[i];
        }
    free(vh); free(a0); free(a1);
    prob_free(&P);
    return rc;
}

int orc_adjoint_m(const orc_geom *g, const orc_mesh *m, const double *sigma, const orc_source *S, int nt,
                  double dt, const double *u0, const double *um1, const double *seed, double *dsig,
                  double *dflux, double *du0, double *dum1)
{
    return orc_adjoint_x(g, m, sigma, NULL, S, nt, dt, u0, um1, 0, seed, dsig, NULL, dflux, du0, dum1, NULL,
                         NULL);
}

int orc_adjoint(const orc_geom *g, const double *sigma, const orc_source *S, int nt, double dt,
                const double *u0, const double *um1, const double *seed,
                double *dsig, double *dflux, double *du0, double *dum1)
{
    return orc_adjoint_m(g, NULL, sigma, S, nt, dt, u0, um1, seed, dsig, dflux, du0, dum1);
}

/* Misfit part of the Tikhonov functional, eq. (functional), and its trace
 * cotangent: J = 1/2 sum_{k=1}^{nt} tau sum_i w_i (obs - data)^2 and
 * seed^k_i = tau w_i (obs^k_i - data^k_i) (seed^0 = 0). */
double orc_misfit(const orc_geom *g, int nt, double dt, const double *obs, const double *data,
                  double *seed)
{
    orc_prob P;
    if (prob_init(&P, g, NULL, NULL, NULL)) return NAN;
    double J = 0.0;
    if (seed) memset(seed, 0, sizeof(double) * (size_t)P.nface);
    for (int k = 1; k <= nt; ++k)
        for (int j = 0; j < P.ny; ++j)
            for (int i = 0; i < P.nx; ++i) {
                int64_t q = (int64_t)k * P.nface + i + (int64_t)P.nx * j;
                double w = face_weight(&P, i, j), d = obs[q] - data[q];
                J += 0.5 * dt * w * d * d;
                if (seed) seed[q] = dt * w * d;
            }
    prob_free(&P);
    return J;
}

/* Gradient of the Tikhonov functional with respect to the per-cell sigma as
 * an L2 density, the discrete form of eq. (gradient1):
 *   g_c = (1/|c|) dJ_misfit/da_c + gamma (sigma_c - sigma0_c)  (eligible c),
 *   g_c = 0 elsewhere, |c| the cell volume (h^3 for a cube, |K| for a
 *   tetrahedron).  Returns J (misfit + regularisation) in *J.  geps
 *   (optional, lattice mode): the L2 density (1/h^3) dJ_misfit/d(1/c^2) per
 *   free cube (the functional regularises a only), 0 elsewhere. */
int orc_gradient_x(const orc_geom *g, const orc_mesh *m, const double *sigma, const double *eps,
                   const orc_source *S, int nt, double dt, const double *u0, const double *u1, int taylor,
                   const double *data, double gamma, double *grad, double *geps, double *J, double *obs_out)
{
    orc_prob P;
    if (nt < 0 || !(dt > 0) || prob_init(&P, g, m, sigma, eps) || !P.has_fem) return -1;
    const orc_ic ic = {u0, taylor ? NULL : u1, taylor ? u1 : NULL, taylor};
    double *obs = (double *)malloc(sizeof(double) * (size_t)P.nface * (size_t)(nt + 1));
    double *seed = (double *)malloc(sizeof(double) * (size_t)P.nface * (size_t)(nt + 1));
    double *vh = (double *)malloc(sizeof(double) * (size_t)P.fn * (size_t)(nt + 1));
    if (!obs || !seed || !vh) { free(obs); free(seed); free(vh); prob_free(&P); return -2; }
    if (forward_sweep(&P, S, nt, dt, &ic, obs, vh, NULL)) {
        free(obs); free(seed); free(vh); prob_free(&P);
        return -1;
    }
    double Jm = orc_misfit(g, nt, dt, obs, data, seed);
    adjoint_sweep(&P, S, nt, dt, &ic, seed, vh, grad, geps, NULL, NULL, NULL);
    double reg = 0.0;
    for (int64_t c = 0; c < P.ncube; ++c) {
        if (!P.eligible[c]) {
            grad[c] = 0.0;
            if (geps) geps[c] = 0.0;
            continue;
        }
        double s = sigma ? sigma[c] : 0.0;
        grad[c] = grad[c] / P.pvol[c] + gamma * s;
        if (geps) geps[c] /= P.pvol[c];
        reg += 0.5 * gamma * P.pvol[c] * s * s;
    }
    if (J) *J = Jm + reg;
    if (obs_out) memcpy(obs_out, obs, sizeof(double) * (size_t)P.nface * (size_t)(nt + 1));
    free(obs); free(seed); free(vh);
    prob_free(&P);
    return 0;
}

int orc_gradient_m(const orc_geom *g, const orc_mesh *m, const double *sigma, const orc_source *S, int nt,
                   double dt, const double *data, double gamma, double *grad, double *J, double *obs_out)
{
    return orc_gradient_x(g, m, sigma, NULL, S, nt, dt, NULL, NULL, 0, data, gamma, grad, NULL, J, obs_out);
}

int orc_gradient(const orc_geom *g, const double *sigma, const orc_source *S, int nt, double dt,
                 const double *data, double gamma, double *grad, double *J, double *obs_out)
{
    return orc_gradient_m(g, NULL, sigma, S, nt, dt, data, gamma, grad, J, obs_out);
}

/* J of eq. (functional) at sigma (a_0 = 1): one forward sweep, the misfit
 * of orc_misfit and the Tikhonov term 1/2 gamma sum_c |c| sigma_c^2 over the
 * eligible cells. */
static int functional_at(const orc_geom *g, const orc_mesh *m, const double *sigma, const double *eps,
                         const orc_source *S, int nt, double dt, const double *u0, const double *u1, int taylor,
                         const double *data, double gamma, double *J)
{
    orc_prob P;
    if (prob_init(&P, g, m, sigma, eps) || !P.has_fem) return -1;
    const orc_ic ic = {u0, taylor ? NULL : u1, taylor ? u1 : NULL, taylor};
    double *obs = (double *)malloc(sizeof(double) * (size_t)P.nface * (size_t)(nt + 1));
    if (!obs) { prob_free(&P); return -2; }
    if (forward_sweep(&P, S, nt, dt, &ic, obs, NULL, NULL)) { free(obs); prob_free(&P); return -1; }
    double reg = 0.0;
    for (int64_t c = 0; c < P.ncube; ++c)
        if (P.eligible[c]) reg += 0.5 * gamma * P.pvol[c] * sigma[c] * sigma[c];
    *J = orc_misfit(g, nt, dt, obs, data, NULL) + reg;
    free(obs);
    prob_free(&P);
    return 0;
}

#define ORC_CG_LOGW 8

/* Algorithm 3 (Sec. 8), at most `iters` iterations from sigma (in/out).
 * Iteration m:
 *   g^m and J^m = J(sigma^m) from orc_gradient_x (eq. (gradient1));
 *   beta^m = |g^m|^2 / |g^{m-1}|^2, beta^0 = 0 (Fletcher-Reeves; L2 norms
 *   weighted by the cell volumes);
 *   d^m = -g^m + beta^m d^{m-1} on eligible cells; when m > 0 and the
 *   slope sum_c |c| g^m_c d^m_c over the cells that can move (not held by a
 *   bound: sigma_c = 0 with d_c < 0, or sigma_c = 4 with d_c > 0) is >= 0,
 *   the projected direction does not descend and it restarts as d^m = -g^m;
 *   step length (the paper refers to another work for it; reading R9):
 *   trial steps alpha_t = 2^{-t} rho^m / max|d^m| for t = 0, 1, ...,
 *   max_trials - 1, where the first relative step (largest change of sigma)
 *   is rho^0 = alpha_rel and rho^m = min(alpha_rel, 2 alpha^{m-1}
 *   max|d^{m-1}|), twice the previous accepted one; the first trial whose
 *   projected point
 *   sigma_t = clip(sigma^m + alpha_t d^m, 0, 4) on eligible cells (a in
 *   [1, 5], eq. (admpar)) has J(sigma_t) < J^m becomes sigma^{m+1}.  When
 *   no trial lowers J, sigma stays and the iteration ends the run (the norms
 *   have stabilised, Step 3).
 * Every sweep uses the same eps and initial data (IP1 when taylor).
 * log[ORC_CG_LOGW*m + {0..7}] = J^m, |g^m|_{L2}, beta^m (as computed, before
 * a restart), alpha taken (0 if none), max|d^m|, trials run, restart (1/0),
 * J(sigma^{m+1}).
 * Returns the number of iterations run (a stalled one included), negative
 * on error. */
int orc_cg_x(const orc_geom *g, const orc_mesh *msh, double *sigma, const double *eps, const orc_source *S,
             int nt, double dt, const double *u0, const double *u1, int taylor, const double *data, double gamma,
             double alpha_rel, int max_trials, int iters, double *log)
{
    orc_prob P;
    if (max_trials < 1 || prob_init(&P, g, msh, NULL, NULL) || !P.has_fem) return -1;
    int64_t nc = P.ncube;
    double *gr = (double *)calloc((size_t)nc, sizeof(double));
    double *d = (double *)calloc((size_t)nc, sizeof(double));
    double *trial = (double *)calloc((size_t)nc, sizeof(double));
    double gn2_prev = 0.0, rho_prev = 0.0;
    int m = 0, rc = 0;
    if (!gr || !d || !trial) rc = -2;
    for (; m < iters && rc == 0; ++m) {
        double J = 0.0;
        if (orc_gradient_x(g, msh, sigma, eps, S, nt, dt, u0, u1, taylor, data, gamma, gr, NULL, &J, NULL)) {
            rc = -1;
            break;
        }
        double gn2 = 0.0;
        for (int64_t c = 0; c < nc; ++c) gn2 += P.pvol[c] * gr[c] * gr[c];
        double beta = m == 0 ? 0.0 : gn2 / gn2_prev;
        /* slope of J(clip(sigma + alpha d)) at alpha = 0+: cells held by a
         * bound (sigma = 0 moving down, sigma = 4 moving up) do not move */
        double gd = 0.0;
        for (int64_t c = 0; c < nc; ++c) {
            d[c] = P.eligible[c] ? -gr[c] + beta * d[c] : 0.0;
            int held = (sigma[c] <= 0.0 && d[c] < 0.0) || (sigma[c] >= 4.0 && d[c] > 0.0);
            if (!held) gd += P.pvol[c] * gr[c] * d[c];
        }
        int restart = m > 0 && gd >= 0.0;
        if (restart)
            for (int64_t c = 0; c < nc; ++c) d[c] = P.eligible[c] ? -gr[c] : 0.0;
        double dmax = 0.0;
        for (int64_t c = 0; c < nc; ++c)
            if (fabs(d[c]) > dmax) dmax = fabs(d[c]);
        double alpha = 0.0, Jnext = J;
        double rho = m == 0 ? alpha_rel : fmin(alpha_rel, 2.0 * rho_prev);
        int t = 0, taken = 0;
        while (dmax > 0.0 && t < max_trials && !taken) {
            double at = ldexp(rho / dmax, -t);
            for (int64_t c = 0; c < nc; ++c) {
                if (!P.eligible[c]) { trial[c] = sigma[c]; continue; }
                double s = sigma[c] + at * d[c];
                trial[c] = s < 0.0 ? 0.0 : (s > 4.0 ? 4.0 : s);
            }
            double Jt = 0.0;
            if (functional_at(g, msh, trial, eps, S, nt, dt, u0, u1, taylor, data, gamma, &Jt)) {
                rc = -1;
                break;
            }
            ++t;
            if (Jt < J) {
                taken = 1;
                alpha = at;
                Jnext = Jt;
                memcpy(sigma, trial, sizeof(double) * (size_t)nc);
            }
        }
        gn2_prev = gn2;
        rho_prev = alpha * dmax;
        if (log) {
            double *r = log + ORC_CG_LOGW * m;
            r[0] = J; r[1] = sqrt(gn2); r[2] = beta; r[3] = alpha;
            r[4] = dmax; r[5] = t; r[6] = restart; r[7] = Jnext;
        }
        if (!taken && rc == 0) { ++m; break; }
    }
    free(gr); free(d); free(trial);
    prob_free(&P);
    return rc ? rc : m;
}

int orc_cg_m(const orc_geom *g, const orc_mesh *msh, double *sigma, const orc_source *S, int nt, double dt,
             const double *data, double gamma, double alpha_rel, int max_trials, int iters, double *log)
{
    return orc_cg_x(g, msh, sigma, NULL, S, nt, dt, NULL, NULL, 0, data, gamma, alpha_rel, max_trials, iters,
                    log);
}

int orc_cg(const orc_geom *g, double *sigma, const orc_source *S, int nt, double dt,
           const double *data, double gamma, double alpha_rel, int max_trials, int iters, double *log)
{
    return orc_cg_m(g, NULL, sigma, S, nt, dt, data, gamma, alpha_rel, max_trials, iters, log);
}
