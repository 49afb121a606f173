// General (unstructured) tetrahedral meshes of the FEM box: host analysis
// (hyb_gen_mesh.cpp) and kernels (hyb_gen.hip).  Internal, not part of the
// public ABI.
//
// Device numbering of the FEM nodes, in four contiguous ranges:
//   [0, nA)   omega_diamond: grid nodes on the surface of the inner box
//             [o+2, o+C-2]^3, whose values the grid reads (Sec. 3);
//   [nA, nH)  the other nodes of the closed inner box;
//   [nH, nR)  the other FEM rows (the two-element overlap layer);
//   [nR, fn)  omega_o: the box surface, grid nodes whose values are the grid
//             values (the rows read them from the grid level).
// [0, nR) are the rows of the lumped-mass scheme eq. (fem); [0, nH) are the
// nodes of the free tetrahedra (those with every vertex in the closed inner
// box), whose history the gradient integral reads.  Within a range the nodes
// follow the grid's z, y, x order of the cell that holds them.
//
// Stiffness: K(a) = sum_t a_t K^t with P1 element matrices K^t from the vertex
// coordinates (Sec. 7.2).  Its rows sum to zero, so (K v)_n =
// sum_m kappa_nm (v_n - v_m) with kappa_nm = -K_nm over the mesh neighbours m
// of n.  kappa is stored in a sliced ELL layout: slices of 64 rows (one
// wavefront), entry j of row n at soff[n/64] + 64 j + n%64; a slice is as
// wide as its longest row, padding entries point at the row itself with
// kappa = 0.  Each row lists first its neighbours m > n inside [0, nH) (for
// n < nH), in increasing order, then the others.  Per-edge FP64 gradient
// accumulators E use the same layout for those first entries, with their own
// slice offsets eoff.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/hyb.h"

namespace hyb {

struct GenHost {
    int o[3] = {0, 0, 0}, C[3] = {0, 0, 0};
    long long fn = 0, nA = 0, nH = 0, nR = 0, ntet = 0;
    long long nslice = 0, nslice_h = 0, nnz = 0, nE = 0, nedge = 0;
    bool all_grid = true;                  // every FEM node is a grid node
    std::vector<int32_t> orig_of_dev;      // [fn] caller's node id of device node n
    std::vector<int64_t> grid_lin;         // [fn] unpadded grid index x + nx (y + ny z), or -1
    std::vector<int32_t> gq;               // [fn][3] grid coordinates (grid nodes only)
    std::vector<int32_t> soff, eoff;       // slice offsets (entries)
    std::vector<int32_t> col, eid;         // [nnz] column; edge id (-1: padding)
    std::vector<int32_t> cptr, ctet;       // per edge: contributions (tetrahedron, K^t entry)
    std::vector<double> cw;
    std::vector<double> minv;              // [fn] 1 / lumped mass (0 on omega_o)
    std::vector<int32_t> tetE;             // [ntet][6] E position of each vertex pair (free tets)
    std::vector<double> ke6;               // [ntet][6] K^t entry of each vertex pair (free tets)
    std::vector<double> pvol;              // [ntet] volume of free tetrahedra, 0 for the others
};

// Validate a general mesh of the box [o, o+C] (o, C from its bounding box,
// already checked) against the grid and build the device tables.  Errors:
// HYB_E_ARG (ids out of range), HYB_E_MESH (not conforming: box-surface node
// off the grid, missing omega_o / omega_diamond grid node, two nodes at one
// grid point, degenerate tetrahedron, node in no tetrahedron),
// HYB_E_UNSUPPORTED (too large for 32-bit tables).
hyb_status analyse_general(const hyb_fd_grid *gr, const hyb_fem_mesh *m, const int o[3], const int C[3],
                           GenHost &out, std::string &err);

// Device copies of the tables (owned by the context).
struct GenDev {
    long long fn, nA, nH, nR, ntet, nslice, nnz, nE;
    int32_t *soff, *eoff, *col, *eid, *cptr, *ctet;
    double *cw, *minv, *ke6, *pvol, *E;
    int32_t *tetE, *orig_of_dev;
    int64_t *grid_lin, *wdg, *wog;  // wdg/wog: padded grid index of omega_diamond / omega_o nodes
    void *kap, *cn;                 // [nnz], [fn] in field precision
    void *nu[2];                    // [fn] adjoint: nu = cs dt^2/m mu of the levels, by parity
};

// Arguments of one general FEM step.  Forward: V levels k-1, k, k+1 (or the
// increments VDa = d^k, VDc = d^{k+1}), Ub the grid level k (the rows read
// their omega_o neighbours there), Uc the grid level k+1 (omega_diamond
// receives the new FEM values), hist the history level k+1 (nodes [0, nH)).  Adjoint (computing level k): V levels
// k+2, k+1, k of the FEM multipliers, Ub the grid multipliers of level k+1
// (read by the omega_diamond rows), Uc the grid level k (receives the
// omega_o couplings), hist the history level k, E the gradient accumulators.
template <typename T>
struct GenStep {
    long long fn, nA, nH, nR;
    long long px, plane;
    const int32_t *soff, *eoff, *col;
    const T *kap, *cn;
    const int64_t *wdg, *wog;
    const T *Ub;
    T *Uc;
    const T *Va, *Vb;
    T *Vc;
    const T *VDa;
    T *VDc;
    T *hist;
    double *E;
    T c2;  // (dt/h)^2 of the grid rows that read omega_diamond (times the step weight)
    T cs;  // weight of dt^2 in this step (1; 1/2 in the first step of the Taylor
           // start): multiplies cn in the rows and in the gradient pairs
    // adjoint: nu^{k+1} = cs cn mu^{k+1} of every node (written by the launch
    // that computed level k+1; 0 on omega_o), and the array that receives
    // nu^k = cs_prev cn mu^k for the next launch (cs_prev: weight of step k-1)
    const T *nu_in;
    T *nu_out;
    T cs_prev;
};

// The rows in launches of their own (timing; the sweeps run them inside the
// grid's launches, launch_interior and launch_bnd_adj): forward rows, and
// adjoint rows with the omega_o couplings.
template <typename T> void launch_gen_fwd(const GenStep<T> &s, hipStream_t st);
template <typename T> void launch_gen_adj(const GenStep<T> &s, hipStream_t st);

// kappa from the per-tetrahedron a = 1 + sigma (free tetrahedra, 1 elsewhere)
// in FP64, stored in field precision; cn = dt^2 / m on the rows (0 on
// omega_o).  scal[S_SMAX] = max sigma over free tetrahedra, scal[S_BAD] = 1
// if sigma has a non-finite entry there, scal[S_GERSH] = the Gershgorin
// bound max_n (|K_nn| + sum_m |K_nm|) / m_n of the rows (a spectral bound of
// M^{-1} K(a); the leapfrog is stable when dt^2 times it is <= 4).
template <typename T>
void launch_gen_prepare(const GenDev &d, const double *sigma, double dt2, double *partials, double *scal,
                        hipStream_t st);

// FEM level from a full unpadded FP64 grid level (every FEM node is a grid
// node); increments d = u0 - um1 (either may be null).
template <typename T>
void launch_gen_load(const GenDev &d, const double *src, T *V, hipStream_t st);
// V = a + cb * b at the grid points of the FEM nodes (either may be null = 0)
template <typename T>
void launch_gen_load_combo(const GenDev &d, const double *a, const double *b, double cb, T *V, hipStream_t st);
template <typename T>
void launch_gen_load_incr(const GenDev &d, const double *u0, const double *um1, T *VD, hipStream_t st);
// v[orig_of_dev[n]] = V[n] (FP64, caller's numbering); with U (the grid
// level of a forward sweep) the omega_o nodes take their grid values, which
// the time steps do not copy into the FEM level
template <typename T>
void launch_gen_export(const GenDev &d, const T *V, const T *U, double *v, hipStream_t st);

// Gradient from the edge accumulators: dJ/da_t = sum over the 6 vertex pairs
// of K^t_pair E_pair (free t).  mode 0: g_t = dJ/da_t / |t| + gamma sigma_t,
// scal[slot] = 0.5 gamma sum_t |t| sigma_t^2; mode 1: g_t = dJ/da_t.
void launch_gen_grad_final(const GenDev &d, const double *sigma, double gamma, int mode, double *grad,
                           double *partials, double *scal, int slot, hipStream_t st, int blocks = 0);

}  // namespace hyb
