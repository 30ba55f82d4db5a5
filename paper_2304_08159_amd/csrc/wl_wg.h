// Whole-workgroup multigrid pieces: every thread of a workgroup calls them
// together, they loop over the cells of one level with the workgroup's stride
// and end with a barrier.  Used where one workgroup owns a whole (small)
// hierarchy (the batched solver).  The
// per-cell arithmetic is apply_row's, as in the tiled multigrid kernels.
#pragma once

#include "wl_cg.h"
#include "wl_device.h"

namespace wl {

template <typename T>
struct WgLevel {
    Grid g;
    T* x[2];
    T* b;
    T* L[3];
    T Lc;
    int uniform;  // all faces Lc, fully periodic
};

__device__ __forceinline__ void wg_coords(const Grid& g, int c, int& i, int& j, int& k) {
    i = c % g.n0;
    const int q = c / g.n0;
    j = q % g.n1;
    k = q / g.n1;
}

// Fixed-order sum over the workgroup, returned to every thread.
__device__ inline double wg_sum(double v, double* red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < int(blockDim.x + 63) / 64; ++w) s += red[w];
    __syncthreads();
    return s;
}

template <typename T>
__device__ __forceinline__ Coeffs<T> wg_coeffs(const WgLevel<T>& L) {
    return Coeffs<T>{L.L[0], L.L[1], L.L[2], L.Lc};
}

// xout = x - w (b - A x) / D on active cells, 0 elsewhere; returns
// sum (b - A x)^2 when norm (0 otherwise).
template <typename T, int XM, bool UNIF>
__device__ double wg_sweep_u(const WgLevel<T>& L, const XAccess<T, XM>& X, const T* b, T w,
                             T* xout, bool norm, double* red) {
    const Coeffs<T> C = wg_coeffs(L);
    const int N = int(cells(L.g));
    double r2 = 0.0;
    for (int c = threadIdx.x; c < N; c += blockDim.x) {
        int i, j, k;
        wg_coords(L.g, c, i, j, k);
        T xI, Ax, D;
        apply_row<T, XM, UNIF>(L.g, X, C, i, j, k, xI, Ax, D);
        const T r = b[c] - Ax;
        xout[c] = D > T(0) ? xI - w * r / D : T(0);
        r2 += double(r) * double(r);
    }
    __syncthreads();
    return norm ? wg_sum(r2, red) : 0.0;
}

template <typename T, int XM>
__device__ double wg_sweep(const WgLevel<T>& L, const XAccess<T, XM>& X, const T* b, T w, T* xout,
                           bool norm, double* red) {
    return L.uniform ? wg_sweep_u<T, XM, true>(L, X, b, w, xout, norm, red)
                     : wg_sweep_u<T, XM, false>(L, X, b, w, xout, norm, red);
}

// Coarse right-hand side = sum of the child residuals b - A x.
template <typename T, bool UNIF>
__device__ void wg_restrict_u(const WgLevel<T>& F, const T* x, const T* b, const WgLevel<T>& Cl) {
    const Coeffs<T> C = wg_coeffs(F);
    const XAccess<T, XM_PLAIN> X{x};
    const int Nc = int(cells(Cl.g));
    const int fz = F.g.n2 > Cl.g.n2 ? 2 : 1;
    for (int c = threadIdx.x; c < Nc; c += blockDim.x) {
        int ic, jc, kc;
        wg_coords(Cl.g, c, ic, jc, kc);
        T sum = T(0);
        for (int dz = 0; dz < fz; ++dz)
            for (int dy = 0; dy < 2; ++dy)
                for (int dx = 0; dx < 2; ++dx) {
                    const int i = 2 * ic + dx, j = 2 * jc + dy, k = fz * kc + dz;
                    T xI, Ax, D;
                    apply_row<T, XM_PLAIN, UNIF>(F.g, X, C, i, j, k, xI, Ax, D);
                    sum += b[cid(F.g, i, j, k)] - Ax;
                }
        Cl.b[c] = sum;
    }
    __syncthreads();
}

template <typename T>
__device__ void wg_restrict(const WgLevel<T>& F, const T* x, const T* b, const WgLevel<T>& Cl) {
    if (F.uniform)
        wg_restrict_u<T, true>(F, x, b, Cl);
    else
        wg_restrict_u<T, false>(F, x, b, Cl);
}

// x += P xc on every cell of L: the coarse correction xc of level C,
// interpolated linearly (prolong_at).
template <typename T>
__device__ void wg_prolong(const WgLevel<T>& L, const WgLevel<T>& C, const T* xc, T* x) {
    const int N = int(cells(L.g));
    for (int c = threadIdx.x; c < N; c += blockDim.x) {
        int i, j, k;
        wg_coords(L.g, c, i, j, k);
        x[c] += prolong_at<T>(L.g, C.g, xc, i, j, k);
    }
    __syncthreads();
}

// Coarse coefficient = 1/2 the sum of the fine faces it covers.
template <typename T>
__device__ void wg_coarsen(const WgLevel<T>& F, const WgLevel<T>& Cl) {
    const int Nc = int(cells(Cl.g));
    const int fz = F.g.n2 > Cl.g.n2 ? 2 : 1;
    for (int c = threadIdx.x; c < Nc; c += blockDim.x) {
        int i, j, k;
        wg_coords(Cl.g, c, i, j, k);
        const int I = 2 * i, J = 2 * j, K = fz * k;
        T s0 = T(0), s1 = T(0), s2 = T(0);
        for (int dz = 0; dz < fz; ++dz)
            for (int dy = 0; dy < 2; ++dy) s0 += F.L[0][cid(F.g, I, J + dy, K + dz)];
        for (int dz = 0; dz < fz; ++dz)
            for (int dx = 0; dx < 2; ++dx) s1 += F.L[1][cid(F.g, I + dx, J, K + dz)];
        Cl.L[0][c] = T(0.5) * s0;
        Cl.L[1][c] = T(0.5) * s1;
        if (F.g.ndim == 3) {
            for (int dy = 0; dy < 2; ++dy)
                for (int dx = 0; dx < 2; ++dx) s2 += F.L[2][cid(F.g, I + dx, J + dy, K)];
            Cl.L[2][c] = T(0.5) * s2;
        }
    }
    __syncthreads();
}

// The rest of a V-cycle from level lev[0] (its right-hand side in place)
// down to the coarsest lev[n - 1] and back up, leaving the corrected iterate
// in lev[0].x[1]: per level a zero-start and a plain sweep, restriction,
// the minimum-norm coarsest solve, then the prolongation and two plain
// sweeps.
template <typename T>
__device__ void wg_vcycle_tail(const WgLevel<T>* lev, int n, T w, double coarse_tol, CoarseLds& S) {
    for (int l = 0; l < n - 1; ++l) {
        const WgLevel<T>& L = lev[l];
        wg_sweep<T, XM_ZERO>(L, XAccess<T, XM_ZERO>{nullptr}, L.b, w, L.x[0], false,
                             S.red);
        wg_sweep<T, XM_PLAIN>(L, XAccess<T, XM_PLAIN>{L.x[0]}, L.b, w, L.x[1], false, S.red);
        wg_restrict<T>(L, L.x[1], L.b, lev[l + 1]);
    }
    const WgLevel<T>& Cst = lev[n - 1];
    coarse_cg_block<T>(Cst.g, wg_coeffs(Cst), Cst.uniform, Cst.b, Cst.x[1], coarse_tol,
                       int(cells(Cst.g)) + 64, S);
    for (int l = n - 2; l >= 0; --l) {
        const WgLevel<T>& L = lev[l];
        const WgLevel<T>& C = lev[l + 1];
        wg_prolong<T>(L, C, C.x[1], L.x[1]);
        wg_sweep<T, XM_PLAIN>(L, XAccess<T, XM_PLAIN>{L.x[1]}, L.b, w, L.x[0], false, S.red);
        wg_sweep<T, XM_PLAIN>(L, XAccess<T, XM_PLAIN>{L.x[0]}, L.b, w, L.x[1], false, S.red);
    }
}

}  // namespace wl
