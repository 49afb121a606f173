// Internal declarations shared by the host library (hyb_api.cpp) and the
// kernels (hyb_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace hyb {

// Block shapes (64-wide wavefronts): the adjoint FDM tile is 64 x TY_FDM
// columns (each thread takes RY_FDM neighbouring rows); the forward FDM tile
// is fwd_tile_x(element size) x TY_FDM columns (32 lanes of 16 bytes of
// columns per grid row); the FEM tile 32 x TY_FEM columns; all stream along z.
constexpr int TX_FDM = 64, RY_FDM = 2, TY_FDM = 4 * RY_FDM;
constexpr int TX_FEM = 32, TY_FEM = 8;
constexpr int BLOCK = 256;
static_assert(BLOCK / TX_FDM * RY_FDM == TY_FDM, "FDM tile: BLOCK / TX_FDM thread rows of RY_FDM grid rows");
constexpr int fwd_tile_x(size_t esz) { return 32 * (16 / (int)esz); }

// Face condition of one face at one step, 2 bits per face in a packed int.
enum : int { F_ABC = 0, F_NEUMANN = 1, F_SOURCE = 2 };

struct Geo {
    int nx, ny, nz;           // grid nodes per axis
    long long px, plane;      // row pitch and plane pitch (elements)
    int has_fem;
    int o[3], C[3];           // FEM box: cells [o, o+C)
    long long fpx, fplane;    // FEM node array pitches ((C+1) per axis)
    int hlo[3], hhi[3];       // closed hole [o+2, o+C-2] (grid coords)
    int hn[3];                // history sub-box node counts (C-3 per axis)
    long long hlevel;         // history elements per level
    long long nbnd;           // outer boundary nodes (= n_fi + n_ec)
    long long n_fi, n_ec;     // face-interior nodes; edge and corner nodes
    long long foff[6], ftot;  // compact per-face arrays of boundary values
    long long nwd, nwo;       // |omega_diamond|, |omega_o|
    int fdm_tx[2], fdm_ty;    // FDM tiles along x (forward [0], adjoint [1]) and y
    int fem_tiles[3];         // FEM tiles along x, y, z
    // FDM z chunks per tile column, planes per chunk and blocks launched, for
    // the forward [0] and the adjoint [1] sweep
    int fdm_zt[2], zc_fdm[2], n_fdm_blocks[2];
    int zc_fem;               // FEM planes per chunk
    int n_fem_blocks;         // FEM blocks launched: n_fem_tiles rounded up to 8
    int n_fem_tiles;
    int bnd_blocks;           // blocks of the boundary kernels
    long long fem_n;          // FEM nodes ((C+1)^3, or the nodes of a general mesh)
    int gen;                  // general tetrahedral mesh: the FEM rows run in the
                              // kernels of hyb_gen.hip (n_fem_blocks = nwd = nwo = 0)
};

// Arguments of one time step.  In the forward sweep the U/V fields are the
// wavefields (a = level k-1, b = level k, c = level k+1).  In the adjoint
// sweep they are the multipliers of the U/V rows (a = level k+2, b = level
// k+1, c = level k, computed).
template <typename T>
struct Step {
    Geo g;
    const T *Ua, *Ub;
    T *Uc;
    const T *Va, *Vb;
    T *Vc;
    // FP32 sweeps (increment form): the forward state is (u^k, d^k) with
    // d^k = u^k - u^{k-1} instead of (u^k, u^{k-1}); Da/VDa hold d^k and
    // Dc/VDc receive d^{k+1} (grid and FEM parts; unused in FP64).  The
    // adjoint uses them the same way for the multipliers of levels k+1, k.
    const T *Da, *VDa;
    T *Dc, *VDc;
    const T *acube;          // conductivity a per FEM cube [C^3]
    T c2;                    // (dt/h)^2 (times w2)
    T ic2;                   // 1 / c2 (adjoint x-face proxies in the interior tile)
    double w2;               // weight of dt^2 in the leapfrog rows of this step: 1, or
                             // 1/2 in the first step of the Taylor start (Model
                             // Problem 1); the adjoint's gradient term of that step
                             // carries the same weight
    T r;                     // (h - dt)/(h + dt), eq. (eq:abs2)
    T w[12];                 // cube edge weights / h: x-edges [y+2z], y [x+2z], z [x+2y]
    int types0, types1, types2;  // face conditions of steps k-1, k, k+1
    // forward
    T srcterm;               // 2 dt^2 p(t_k) / h (plane wave)
    const double *flux;      // flux row of step k (table source) or null
    double fluxscale;        // 2 dt^2 / h
    double *obs;             // trace row k+1 (or null)
    T *hist;                 // forward: history level k+1; adjoint: level k
    // adjoint
    int level_rows;          // level k has rows (k >= 1)
    const double *res;       // residual row of level k (or null)
    int seed_mode;           // 0: tau * w_i * res; 1: res
    double dt, h2;
    double *G;               // FP64 gradient accumulator [C^3]
    const T *Fa, *Fb;        // boundary multipliers of levels k+2, k+1 (face arrays)
    T *Fc;                   // boundary multipliers of level k
    T *Pw;                   // level k+1 grid array: receives the boundary proxies
    // variable wave speed (null: 1/c^2 = 1)
    const T *minv;           // [(C+1)^3] h^3 / (lumped mass) per FEM node
    double *Gm;              // adjoint: FP64 dJ/dm per FEM node (h^3 units), or null
    const T *hnext, *hprev;  // adjoint: history levels k+1 (null at k = nt) and k-1
};

// FP32 wavefields advance in increment form (d^{k+1} = d^k + tau^2 L u^k,
// u^{k+1} = u^k + d^{k+1}), algebraically the leapfrog of the three-level
// scheme: rounding u^{k+1} then perturbs the position only, not the implied
// velocity u^{k+1} - u^k, so FP32 errors grow like sqrt(nt) instead of nt^1.5.
template <typename T> constexpr bool incr_form() { return sizeof(T) == 4; }

// The edge and corner rows of one forward step (its levels, source term,
// face conditions and dt^2 weight), run as extra blocks of the next step's
// interior launch: no interior or absorbing-face row reads an edge value.
template <typename T>
struct EdgeArgs {
    const T *Ua, *Ub, *Da;
    T *Uc, *Dc;
    double *obs;
    const double *flux;
    double fluxscale;
    T srcterm, c2;
    int types1;
};

template <typename T>
inline EdgeArgs<T> edge_args(const Step<T> &s)
{
    EdgeArgs<T> e;
    e.Ua = s.Ua; e.Ub = s.Ub; e.Da = s.Da; e.Uc = s.Uc; e.Dc = s.Dc;
    e.obs = s.obs; e.flux = s.flux; e.fluxscale = s.fluxscale;
    e.srcterm = s.srcterm; e.c2 = s.c2; e.types1 = s.types1;
    return e;
}

template <typename T> struct GenStep;

// ---- launchers (hyb_kernels.hip) ----
// edges: the step whose edge and corner rows the forward launch also runs
// (null: none); gen: the FEM rows of a general mesh that go with the step
// (null: none)
template <typename T>
void launch_interior(const Step<T> &s, bool adjoint, hipStream_t st, const EdgeArgs<T> *edges = nullptr,
                     const GenStep<T> *gen = nullptr);
// boundary launch of a forward step: reflecting face rows, edges and corners
template <typename T> void launch_bnd_fwd(const Step<T> &s, hipStream_t st);
// the same split in two: the reflecting face rows (no launch when every face
// absorbs), and the edge and corner rows
template <typename T> void launch_bnd_fwd_faces(const Step<T> &s, hipStream_t st);
template <typename T> void launch_bnd_fwd_edges(const Step<T> &s, hipStream_t st);
// gen: the omega_o couplings of a general mesh's FEM rows (null: none)
template <typename T> void launch_bnd_adj(const Step<T> &s, hipStream_t st, const GenStep<T> *gen = nullptr);

// rows of the forward boundary launch that face conditions `types` give
long long fwd_face_row_count(const Geo &g, int types);

// batched steps: steps_dev[n] device array, all of geometry g.  Forward:
// edges_dev[n] (or null) holds, per slot, the step whose edge and corner rows
// the interior launch also runs (Uc null: none); face_rows is the largest
// count of reflecting face rows over the slots (0: no boundary launch).
template <typename T>
void launch_batch_fwd(const Geo &g, const Step<T> *steps_dev, const EdgeArgs<T> *edges_dev, int n,
                      long long face_rows, hipStream_t st);
template <typename T> void launch_batch_adj(const Geo &g, const Step<T> *steps_dev, int n, hipStream_t st);

// a = 1 + sigma on free cubes (1 elsewhere); scal[0] = max sigma over free
// cubes, scal[1] = 1 if sigma has a non-finite entry.
template <typename T>
void launch_acube(const Geo &g, const double *sigma, T *acube, double *partials, double *scal,
                  hipStream_t st);
// copy a full grid level (unpadded FP64) into a padded field, and its FEM part
template <typename T>
void launch_load_level(const Geo &g, const double *src, T *U, T *V, hipStream_t st);
// the same for the combination a + cb * b of two full levels (either may be
// null = 0)
template <typename T>
void launch_load_combo(const Geo &g, const double *a, const double *b, double cb, T *U, T *V, hipStream_t st);
// increments d^0 = u^0 - u^{-1} of given initial levels (either may be null = 0)
template <typename T>
void launch_load_incr(const Geo &g, const double *u0, const double *um1, T *D, T *VD, hipStream_t st);
template <typename T>
void launch_hist_level(const Geo &g, const T *V, T *hist, hipStream_t st);
template <typename T>
void launch_record_face(const Geo &g, const T *U, double *obs_row, hipStream_t st);

// types: the face conditions of the level's adjoint rows (which multipliers
// of absorbing x faces the grid array holds); unused when F is null
template <typename T>
void launch_export_level(const Geo &g, const T *U, const T *V, const T *F, double *u, double *v,
                         hipStream_t st, int types = 0);

// BF16 checkpoint increments: half[i] = bf16(a[i]) (round to nearest even);
// unpack: b[i] = float(half[i]).  a, b are FP32 arrays.
void launch_pack_bf16(const void *a, uint16_t *half, long long n, hipStream_t st);
void launch_unpack_bf16(const uint16_t *half, void *b, long long n, hipStream_t st);
// 16-bit block-scaled checkpoint increments: per group of 64 values
// scale[g] = max|a| / 32767 and q[i] = round(a[i] / scale); unpack b[i] =
// q[i] * scale[i / 64].  a, b are FP32 arrays of n values.
void launch_pack_q16(const void *a, int16_t *q, float *scale, long long n, hipStream_t st);
void launch_unpack_q16(const int16_t *q, const float *scale, void *b, long long n, hipStream_t st);

// J_misfit = 1/2 sum_{k=1..nt} dt sum_i w_i res^2 -> scal[slot]
void launch_misfit(const Geo &g, const double *res, int nt, double dt, double h, double *partials,
                   double *scal, int slot, hipStream_t st);
// gradient finalisation (see hyb_gradient); reg -> scal[slot] (0.5 gamma h^3 sum sigma^2)
void launch_grad_final(const Geo &g, const double *G, const double *sigma, double coefG,
                       double gamma, int mode, double h3, double *grad, double *partials,
                       double *scal, int slot, hipStream_t st, int blocks = 0);
// Conductivity parameters for the CG kernels: the C^3 cubes of a structured
// box (weight h^3 on free cubes) or the tetrahedra of a general mesh
// (weight = volume on free tetrahedra); weight 0 = not free.
struct Params {
    long long n;
    int C[3];
    const double *pvol;  // general mesh: weight per tetrahedron; null = structured cubes
    double h3;
};
// Algorithm 3.  norm2: scal[slot] = sum w v^2.  dir: d = -g + beta d with
// beta = scal[GN2]/scal[GN2P] (0 when first); restart d = -g when not first
// and the slope over the cells free to move is >= 0; scal[BETA, SLOPE,
// RESTART, DMAX].  trial: trial = clip(sigma + 2^{-t} alpha_rel / DMAX d) on
// free cells, scal[ALPHA], scal[JREGT] = gamma/2 sum w trial^2.  roll:
// GN2P <- GN2.  differ: scal[slot] = 1 when a and b differ anywhere.
void launch_cg_norm2(const Params &p, const double *v, double *partials, double *scal, int slot, hipStream_t st);
void launch_cg_dir(const Params &p, const double *grad, double *dir, const double *sigma, int first,
                   double *partials, double *scal, hipStream_t st);
void launch_cg_trial(const Params &p, const double *dir, const double *sigma, double *trial, double alpha_rel,
                     int t, double gamma, double *partials, double *scal, hipStream_t st);
void launch_cg_roll(double *scal, hipStream_t st);
void launch_differ(const double *a, const double *b, long long n, double *partials, double *scal, int slot,
                   hipStream_t st);
void launch_residual(const double *obs, const double *data, double *res, long long n,
                     hipStream_t st);

// Variable wave speed: minv[n] = 1 / m_n of each FEM node from 1/c^2 per
// cube (1 outside the free cubes): m_n = (3 (e_a + e_b) + sum of the other 6
// incident cubes) / 12, e_a, e_b the two cubes whose Kuhn diagonal ends at n.
template <typename T>
void launch_minv(const Geo &g, const double *eps, T *minv, hipStream_t st);
// dJ/d(1/c^2) per cube from the per-node dJ/dm: the same shares (1/4 at the
// diagonal ends, 1/12 elsewhere); mode 0 divides by h^3 (L2 density), 0 on
// cubes that are not free.
void launch_eps_grad(const Geo &g, const double *Gm, double scale, double *geps, hipStream_t st);
// history box of a - b (b may be null) for the level u^{-1}
template <typename T>
void launch_hist_diff(const Geo &g, const T *a, const T *b, T *hist, hipStream_t st);

// hyb_gradient_noalloc: a file-scope device array of NOALLOC_PARTS partial
// sums and NOALLOC_SCAL scalars (131 200 bytes per GPU); *out = its address
// on the current device (resolved once per device).
constexpr int NOALLOC_PARTS = 16384, NOALLOC_SCAL = 16, NOALLOC_MAX_DEVICES = 64;
hipError_t noalloc_scratch(double **out);
// J[0] = mode 0 ? jmis[0] + jreg[0] : 0
void launch_sum_J(const double *jmis, const double *jreg, int mode, double *J, hipStream_t st);

// device scalar slots
enum : int { S_SMAX = 0, S_BAD = 1, S_JMIS = 2, S_JREG = 3, S_GN2 = 4, S_GN2P = 5, S_BETA = 6,
             S_DMAX = 7, S_ALPHA = 8, S_GERSH = 9, S_SLOPE = 10, S_RESTART = 11, S_JMIST = 12, S_JREGT = 13,
             S_DIFF = 14, S_NSCAL = 16 };
constexpr int MAX_PARTIALS = 4096;

}  // namespace hyb
