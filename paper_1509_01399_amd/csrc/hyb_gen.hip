// HIP kernels (gfx950) of the FEM box on a general tetrahedral mesh: the
// coefficient preparation, loads and exports of FEM levels, the gradient
// from the edge accumulators, and the rows of hyb_gen_rows.h in launches of
// their own (the time steps run them inside the grid's launches).
#include <algorithm>

#include "hyb_gen.h"
#include "hyb_gen_rows.h"
#include "hyb_internal.h"

namespace hyb {

namespace {

// The forward rows alone.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_gen_fwd(GenStep<T> s, int nblk)
{
    gen_fwd_row<T>(s, gen_row((int)blockIdx.x, nblk));
}

// The adjoint rows and the omega_o couplings alone.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_gen_adj(GenStep<T> s, int nblk)
{
    const long long n = gen_row((int)blockIdx.x, nblk);
    if (n < s.nR) gen_adj_row<T>(s, n);
    else gen_wo_row<T>(s, n);
}

__device__ double block_reduce_g(double v, bool is_max)
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

// Fold the partials of a reduction in a fixed order into scal[slot].
__global__ __launch_bounds__(BLOCK) void k_final_g(const double *part, int n, int is_max, double scale,
                                                   double *scal, int slot)
{
    double v = 0.0;
    for (int q = threadIdx.x; q < n; q += BLOCK) v = is_max ? fmax(v, part[q]) : v + part[q];
    v = block_reduce_g(v, is_max != 0);
    if (threadIdx.x == 0) scal[slot] = v * scale;
}

int nparts_g(long long n) { return (int)std::min<long long>(MAX_PARTIALS / 2, (n + BLOCK - 1) / BLOCK); }

__global__ __launch_bounds__(BLOCK) void k_gen_sigma(long long nt, const double *pvol, const double *sigma,
                                                     double *part_max, double *part_bad)
{
    double mx = 0.0, bad = 0.0;
    if (sigma)
        for (long long t = (long long)blockIdx.x * BLOCK + threadIdx.x; t < nt; t += (long long)gridDim.x * BLOCK) {
            if (!(pvol[t] > 0.0)) continue;
            const double sv = sigma[t];
            if (!isfinite(sv)) bad = 1.0;
            else mx = fmax(mx, sv);
        }
    mx = block_reduce_g(mx, true);
    __syncthreads();
    bad = block_reduce_g(bad, true);
    if (threadIdx.x == 0) { part_max[blockIdx.x] = mx; part_bad[blockIdx.x] = bad; }
}

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_gen_prepare(GenDev d, const double *sigma, double dt2, double *part)
{
    double R = 0.0;
    T *kap = (T *)d.kap, *cn = (T *)d.cn;
    for (long long n = (long long)blockIdx.x * BLOCK + threadIdx.x; n < d.fn; n += (long long)gridDim.x * BLOCK) {
        const int sl = (int)(n >> 6), ln = (int)(n & 63);
        const int b = d.soff[sl], w = (d.soff[sl + 1] - b) >> 6;
        double s1 = 0.0, s2 = 0.0;
        for (int j = 0; j < w; ++j) {
            const int p = b + 64 * j + ln;
            const int e = d.eid[p];
            double k = 0.0;
            if (e >= 0)
                for (int c = d.cptr[e]; c < d.cptr[e + 1]; ++c) {
                    const int t = d.ctet[c];
                    const double a = (sigma && d.pvol[t] > 0.0) ? 1.0 + sigma[t] : 1.0;
                    k -= a * d.cw[c];
                }
            kap[p] = (T)k;
            s1 += k;
            s2 += fabs(k);
        }
        const bool row = n < d.nR;
        cn[n] = row ? (T)(dt2 * d.minv[n]) : (T)0;
        if (row) R = fmax(R, (fabs(s1) + s2) * d.minv[n]);
    }
    R = block_reduce_g(R, true);
    if (threadIdx.x == 0) part[blockIdx.x] = R;
}

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_gen_load(long long fn, const int64_t *lin, const double *src, T *V)
{
    for (long long n = (long long)blockIdx.x * BLOCK + threadIdx.x; n < fn; n += (long long)gridDim.x * BLOCK)
        V[n] = lin[n] >= 0 ? (T)src[lin[n]] : (T)0;
}

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_gen_load_combo(long long fn, const int64_t *lin, const double *a,
                                                          const double *b, double cb, T *V)
{
    for (long long n = (long long)blockIdx.x * BLOCK + threadIdx.x; n < fn; n += (long long)gridDim.x * BLOCK) {
        const long long g = lin[n];
        V[n] = g >= 0 ? (T)((a ? a[g] : 0.0) + (b ? cb * b[g] : 0.0)) : (T)0;
    }
}

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_gen_load_incr(long long fn, const int64_t *lin, const double *u0,
                                                         const double *um1, T *VD)
{
    for (long long n = (long long)blockIdx.x * BLOCK + threadIdx.x; n < fn; n += (long long)gridDim.x * BLOCK) {
        const long long g = lin[n];
        VD[n] = g >= 0 ? (T)((u0 ? u0[g] : 0.0) - (um1 ? um1[g] : 0.0)) : (T)0;
    }
}

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_gen_export(long long fn, long long nR, const int32_t *orig, const T *V,
                                                      const T *U, const int64_t *wog, double *v)
{
    for (long long n = (long long)blockIdx.x * BLOCK + threadIdx.x; n < fn; n += (long long)gridDim.x * BLOCK)
        v[orig[n]] = (double)((U && n >= nR) ? U[wog[n - nR]] : V[n]);
}

__global__ __launch_bounds__(BLOCK) void k_gen_grad_final(long long nt, const int32_t *tetE, const double *ke6,
                                                          const double *E, const double *pvol,
                                                          const double *sigma, double gamma, int mode,
                                                          double *grad, double *part)
{
    double reg = 0.0;
    for (long long t = (long long)blockIdx.x * BLOCK + threadIdx.x; t < nt; t += (long long)gridDim.x * BLOCK) {
        double v = 0.0;
        const double vol = pvol[t];
        if (vol > 0.0) {
            double ds = 0.0;
#pragma unroll
            for (int u = 0; u < 6; ++u) ds += ke6[6 * t + u] * E[tetE[6 * t + u]];
            if (mode == 0) {
                const double sv = sigma ? sigma[t] : 0.0;
                v = ds / vol + gamma * sv;
                reg += vol * sv * sv;
            } else {
                v = ds;
            }
        }
        grad[t] = v;
    }
    reg = block_reduce_g(reg, false);
    if (threadIdx.x == 0) part[blockIdx.x] = reg;
}

}  // namespace

template <typename T>
void launch_gen_fwd(const GenStep<T> &s, hipStream_t st)
{
    const int nb = gen_row_blocks(s.nR);
    hipLaunchKernelGGL((k_gen_fwd<T>), dim3(nb), dim3(BLOCK), 0, st, s, nb);
}

template <typename T>
void launch_gen_adj(const GenStep<T> &s, hipStream_t st)
{
    const int nb = gen_row_blocks(s.fn);
    hipLaunchKernelGGL((k_gen_adj<T>), dim3(nb), dim3(BLOCK), 0, st, s, nb);
}

template <typename T>
void launch_gen_prepare(const GenDev &d, const double *sigma, double dt2, double *partials, double *scal,
                        hipStream_t st)
{
    const int n1 = nparts_g(d.ntet);
    hipLaunchKernelGGL(k_gen_sigma, dim3(n1), dim3(BLOCK), 0, st, d.ntet, d.pvol, sigma, partials,
                       partials + MAX_PARTIALS / 2);
    hipLaunchKernelGGL(k_final_g, dim3(1), dim3(BLOCK), 0, st, partials, n1, 1, 1.0, scal, (int)S_SMAX);
    hipLaunchKernelGGL(k_final_g, dim3(1), dim3(BLOCK), 0, st, partials + MAX_PARTIALS / 2, n1, 1, 1.0, scal,
                       (int)S_BAD);
    const int n2 = nparts_g(d.fn);
    hipLaunchKernelGGL((k_gen_prepare<T>), dim3(n2), dim3(BLOCK), 0, st, d, sigma, dt2, partials);
    hipLaunchKernelGGL(k_final_g, dim3(1), dim3(BLOCK), 0, st, partials, n2, 1, 1.0, scal, (int)S_GERSH);
}

template <typename T>
void launch_gen_load(const GenDev &d, const double *src, T *V, hipStream_t st)
{
    hipLaunchKernelGGL((k_gen_load<T>), dim3(nparts_g(d.fn)), dim3(BLOCK), 0, st, d.fn, d.grid_lin, src, V);
}

template <typename T>
void launch_gen_load_combo(const GenDev &d, const double *a, const double *b, double cb, T *V, hipStream_t st)
{
    hipLaunchKernelGGL((k_gen_load_combo<T>), dim3(nparts_g(d.fn)), dim3(BLOCK), 0, st, d.fn, d.grid_lin, a, b,
                       cb, V);
}

template <typename T>
void launch_gen_load_incr(const GenDev &d, const double *u0, const double *um1, T *VD, hipStream_t st)
{
    hipLaunchKernelGGL((k_gen_load_incr<T>), dim3(nparts_g(d.fn)), dim3(BLOCK), 0, st, d.fn, d.grid_lin, u0,
                       um1, VD);
}

template <typename T>
void launch_gen_export(const GenDev &d, const T *V, const T *U, double *v, hipStream_t st)
{
    hipLaunchKernelGGL((k_gen_export<T>), dim3(nparts_g(d.fn)), dim3(BLOCK), 0, st, d.fn, d.nR, d.orig_of_dev, V,
                       U, d.wog, v);
}

void launch_gen_grad_final(const GenDev &d, const double *sigma, double gamma, int mode, double *grad,
                           double *partials, double *scal, int slot, hipStream_t st, int blocks)
{
    const int nb = blocks > 0 ? blocks : nparts_g(d.ntet);
    hipLaunchKernelGGL(k_gen_grad_final, dim3(nb), dim3(BLOCK), 0, st, d.ntet, d.tetE, d.ke6, d.E, d.pvol,
                       sigma, gamma, mode, grad, partials);
    hipLaunchKernelGGL(k_final_g, dim3(1), dim3(BLOCK), 0, st, partials, nb, 0, 0.5 * gamma, scal, slot);
}

#define HYB_GEN_INST(T)                                                                            \
    template void launch_gen_fwd<T>(const GenStep<T> &, hipStream_t);                              \
    template void launch_gen_adj<T>(const GenStep<T> &, hipStream_t);                              \
    template void launch_gen_prepare<T>(const GenDev &, const double *, double, double *, double *, \
                                        hipStream_t);                                              \
    template void launch_gen_load<T>(const GenDev &, const double *, T *, hipStream_t);            \
    template void launch_gen_load_combo<T>(const GenDev &, const double *, const double *, double, T *, \
                                           hipStream_t);                                           \
    template void launch_gen_load_incr<T>(const GenDev &, const double *, const double *, T *,     \
                                          hipStream_t);                                            \
    template void launch_gen_export<T>(const GenDev &, const T *, const T *, double *, hipStream_t);
HYB_GEN_INST(double)
HYB_GEN_INST(float)

}  // namespace hyb
