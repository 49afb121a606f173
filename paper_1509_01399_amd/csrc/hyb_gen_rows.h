// Row bodies of the FEM box on a general tetrahedral mesh (device code
// shared by hyb_gen.hip and hyb_kernels.hip): the lumped-mass P1 update of
// eq. (fem), its exact adjoint with the FP64 gradient integral of
// eq. (gradient1), and the omega_o couplings of the adjoint, on the sliced
// ELL tables described in hyb_gen.h.  One thread per row; a wavefront owns
// one 64-row slice, so its column and kappa loads are contiguous, and the
// neighbour values are gathered (the node numbering follows the grid order
// of the cells, so the gathers stay within a few z planes of the box and hit
// the caches).
#pragma once

#include "hyb_gen.h"
#include "hyb_internal.h"

namespace hyb {

// Row of thread threadIdx.x in block b of a range of nblk row blocks (nblk a
// multiple of 8, the range starting at a multiple of 8 of its launch):
// blocks are dealt round-robin to the 8 XCDs, so each XCD gets a contiguous
// range of rows and the rows of a neighbourhood share an L2.
__device__ __forceinline__ long long gen_row(int b, int nblk)
{
    const int per = nblk / 8;
    return (long long)((b % 8) * per + b / 8) * BLOCK + threadIdx.x;
}

// Forward row n < nR (level k -> k+1):
//   v^{k+1}_n = 2 v^k_n - v^{k-1}_n - (dt^2 / m_n) sum_m kappa_nm (v^k_n - v^k_m),
// or in increment form d^{k+1}_n = d^k_n - (dt^2/m_n) (...), v^{k+1} = v^k + d^{k+1}.
// A neighbour on omega_o (m >= nR) is a grid node whose FEM value is the
// grid value (Algorithm 2, step 4): the row reads it from the grid level k,
// so the FEM level is not copied there.  Rows on omega_diamond also write
// their new value into the grid level (step 3).
template <typename T>
__device__ __forceinline__ void gen_fwd_row(const GenStep<T> &s, long long n)
{
    if (n >= s.nR) return;
    const int sl = (int)(n >> 6), ln = (int)(n & 63);
    const int b = s.soff[sl], w = (s.soff[sl + 1] - b) >> 6;
    const T *__restrict__ Vb = s.Vb;
    const T *__restrict__ kap = s.kap;
    const int32_t *__restrict__ col = s.col;
    const T v0 = Vb[n];
    T acc = 0;
#pragma unroll 2
    for (int j = 0; j < w; ++j) {
        const int p = b + 64 * j + ln;
        const int m = col[p];
        const T vm = m < s.nR ? Vb[m] : s.Ub[s.wog[m - s.nR]];
        acc += kap[p] * (v0 - vm);
    }
    const T c = s.cs * s.cn[n];
    T v;
    if constexpr (incr_form<T>()) {
        const T d = s.VDa[n] - c * acc;
        s.VDc[n] = d;
        v = v0 + d;
    } else {
        v = (T)2 * v0 - s.Va[n] - c * acc;
    }
    s.Vc[n] = v;
    if (n < s.nA) s.Uc[s.wdg[n]] = v;
    if (n < s.nH && s.hist) __builtin_nontemporal_store(v, s.hist + n);
}

// Adjoint row n < nR, computing the multipliers of level k from those of
// levels k+1 and k+2 (the transpose of the forward rows):
//   mu^k_n = 2 mu^{k+1}_n - mu^{k+2}_n - sum_m kappa_nm (nu_n - nu_m)
//            [+ (dt/h)^2 sum of the 6 grid multipliers around n, on omega_diamond]
// with nu_m = (dt^2 / m_m) mu^{k+1}_m (0 off the rows).  The gradient
// integral pairs u^k with nu: every edge (n, m), n < m, of the inner box
// accumulates (nu_n - nu_m)(u^k_n - u^k_m) in FP64.
template <typename T>
__device__ __forceinline__ void gen_adj_row(const GenStep<T> &s, long long n)
{
    if (n >= s.nR) return;
    const int sl = (int)(n >> 6), ln = (int)(n & 63);
    const int b = s.soff[sl], w = (s.soff[sl + 1] - b) >> 6;
    const T *__restrict__ Vb = s.Vb;
    const T *__restrict__ nu = s.nu_in;
    const T *__restrict__ kap = s.kap;
    const int32_t *__restrict__ col = s.col;
    const T mu1 = Vb[n];
    const T nu0 = nu[n];
    const bool hrow = n < s.nH;
    const T *__restrict__ H = s.hist;
    // the slice's first we entries carry the E slots (upper inner edges
    // first in each row of [0, nH)); the rest only the stencil
    int eb = 0, we = 0;
    double u0 = 0.0;
    if ((long long)sl * 64 < s.nH) {
        eb = s.eoff[sl];
        we = (s.eoff[sl + 1] - eb) >> 6;
    }
    T acc = 0;
    int j0 = 0;
    if constexpr (sizeof(T) == 4) {
        // FP32 fields: every access of the E loop is unconditional, so the
        // loads of several slots are in flight together; a slot that is not
        // an upper inner edge pairs the row's history with itself (factor
        // u0 - u0 = 0) and writes its E entry, which no tetrahedron reads,
        // back.  Adjoint step on a 256^3-cell grid with a 96^3-cell general
        // box 141.8 -> 137.3 us; with FP64 fields the extra E writes cost
        // more than the wait they save (189.4 -> 194.5 us), so those keep
        // the conditional update.
        if (hrow) {
            u0 = (double)H[n];
#pragma unroll 4
            for (int j = 0; j < we; ++j) {
                const int p = b + 64 * j + ln;
                const int m = col[p];
                const T num = nu[m];
                acc += kap[p] * (nu0 - num);
                const bool up = m > n && m < s.nH;
                double *e = s.E + eb + 64 * j + ln;
                *e += ((double)nu0 - (double)num) * (u0 - (double)H[up ? m : n]);
            }
            j0 = we;
        }
    } else {
        if (hrow) u0 = (double)H[n];
#pragma unroll 4
        for (int j = 0; j < we; ++j) {
            const int p = b + 64 * j + ln;
            const int m = col[p];
            const T num = nu[m];
            acc += kap[p] * (nu0 - num);
            if (hrow && m > n && m < s.nH) {
                double *e = s.E + eb + 64 * j + ln;
                *e += ((double)nu0 - (double)num) * (u0 - (double)H[m]);
            }
        }
        j0 = we;
    }
#pragma unroll 2
    for (int j = j0; j < w; ++j) {
        const int p = b + 64 * j + ln;
        acc += kap[p] * (nu0 - nu[col[p]]);
    }
    T cw = 0;
    if (n < s.nA) {
        const long long gg = s.wdg[n];
        const T *Ub = s.Ub;
        cw = s.c2 * (((Ub[gg - 1] + Ub[gg + 1]) + (Ub[gg - s.px] + Ub[gg + s.px])) +
                     (Ub[gg - s.plane] + Ub[gg + s.plane]));
    }
    T mu0;
    if constexpr (incr_form<T>()) {
        const T d = s.VDa[n] - acc + cw;
        s.VDc[n] = d;
        mu0 = mu1 + d;
    } else {
        mu0 = (T)2 * mu1 - s.Va[n] - acc + cw;
    }
    s.Vc[n] = mu0;
    s.nu_out[n] = (s.cs_prev * s.cn[n]) * mu0;
}

// Adjoint coupling of omega_o node n >= nR (not a row): sum_m kappa_nm nu_m,
// what the FEM rows that read the node contribute to its multiplier, left in
// the grid level k for the grid row of the node to add.  It needs only the
// nu of level k+1.
template <typename T>
__device__ __forceinline__ void gen_wo_row(const GenStep<T> &s, long long n)
{
    if (n < s.nR || n >= s.fn) return;
    const int sl = (int)(n >> 6), ln = (int)(n & 63);
    const int b = s.soff[sl], w = (s.soff[sl + 1] - b) >> 6;
    const T *__restrict__ nu = s.nu_in;
    const T *__restrict__ kap = s.kap;
    const int32_t *__restrict__ col = s.col;
    T acc = 0;
#pragma unroll 2
    for (int j = 0; j < w; ++j) {
        const int p = b + 64 * j + ln;
        acc += kap[p] * nu[col[p]];
    }
    s.Uc[s.wog[n - s.nR]] = acc;
}

// Row blocks of rows [0, n), a multiple of 8 (the extra blocks exit at once).
__host__ __device__ __forceinline__ int gen_row_blocks(long long n)
{
    const long long nb = (n + BLOCK - 1) / BLOCK;
    return (int)((nb + 7) / 8 * 8);
}

}  // namespace hyb
