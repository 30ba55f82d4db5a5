// One workgroup's mixed-precision GMG solve (FP32 V-cycles with an FP64
// defect correction around them), shared by the batched Poisson solver and
// the batched Navier-Stokes steps.  Every thread of the workgroup calls these
// together; each ends with a barrier.
#pragma once

#include "wl_wg.h"

namespace wl {

constexpr int kWgMixedInner = 3;   // FP32 V-cycles per outer iteration

// b_in projected onto the active cells of F (mean removed there) into F.b;
// returns ||F.b||^2 (every thread).
__device__ inline double wg_project_rhs(const WgLevel<double>& F, const double* b_in, double* red) {
    const int N = int(cells(F.g));
    const XAccess<double, XM_ZERO> Z{nullptr};
    const Coeffs<double> C = wg_coeffs(F);
    double sb = 0.0, cnt = 0.0;
    for (int c = threadIdx.x; c < N; c += blockDim.x) {
        int i, j, k;
        wg_coords(F.g, c, i, j, k);
        double xI, Ax, D;
        apply_row<double, XM_ZERO, false>(F.g, Z, C, i, j, k, xI, Ax, D);
        if (D > 0.0) {
            sb += b_in[c];
            cnt += 1.0;
        }
    }
    sb = wg_sum(sb, red);
    cnt = wg_sum(cnt, red);
    const double mean = cnt > 0.0 ? sb / cnt : 0.0;
    double b2 = 0.0;
    for (int c = threadIdx.x; c < N; c += blockDim.x) {
        int i, j, k;
        wg_coords(F.g, c, i, j, k);
        double xI, Ax, D;
        apply_row<double, XM_ZERO, false>(F.g, Z, C, i, j, k, xI, Ax, D);
        const double bv = D > 0.0 ? b_in[c] - mean : 0.0;
        F.b[c] = bv;
        b2 += bv * bv;
    }
    __syncthreads();
    return wg_sum(b2, red);
}

// FP32 coefficients of lev[0] from F's FP64 ones, then the coarse levels
// (half the covered fine faces).
__device__ inline void wg_coeffs32(const WgLevel<double>& F, const WgLevel<float>* lev, int nlev) {
    const int N = int(cells(F.g));
    for (int c = threadIdx.x; c < N; c += blockDim.x)
        for (int d = 0; d < F.g.ndim; ++d) lev[0].L[d][c] = float(F.L[d][c]);
    __syncthreads();
    for (int l = 1; l < nlev; ++l) wg_coarsen<float>(lev[l - 1], lev[l]);
}

// One FP32 V-cycle on lev[0..n) for A e = lev[0].b from the iterate in
// lev[0].x[1] (zero: from e = 0), result in lev[0].x[1].
__device__ inline void wg_vcycle32(const WgLevel<float>* lev, int n, float w, bool zero,
                                   CoarseLds& S) {
    const WgLevel<float>& L0 = lev[0];
    if (n == 1) {
        coarse_cg_block<float>(L0.g, wg_coeffs(L0), L0.uniform, L0.b, L0.x[1], 1e-6,
                               int(cells(L0.g)) + 64, S);
        return;
    }
    if (zero) {
        wg_vcycle_tail<float>(lev, n, w, 1e-6, S);
        return;
    }
    wg_sweep<float, XM_PLAIN>(L0, XAccess<float, XM_PLAIN>{L0.x[1]}, L0.b, w, L0.x[0], false, S.red);
    wg_sweep<float, XM_PLAIN>(L0, XAccess<float, XM_PLAIN>{L0.x[0]}, L0.b, w, L0.x[1], false, S.red);
    wg_restrict<float>(L0, L0.x[1], L0.b, lev[1]);
    wg_vcycle_tail<float>(&lev[1], n - 1, w, 1e-6, S);
    wg_prolong<float>(L0, lev[1], lev[1].x[1], L0.x[1]);
    wg_sweep<float, XM_PLAIN>(L0, XAccess<float, XM_PLAIN>{L0.x[1]}, L0.b, w, L0.x[0], false, S.red);
    wg_sweep<float, XM_PLAIN>(L0, XAccess<float, XM_PLAIN>{L0.x[0]}, L0.b, w, L0.x[1], false, S.red);
}

// Defect correction on F (FP64: solution F.x[0], projected right-hand side
// F.b, coefficients F.L): r = b - A x rounded into lev[0].b, kWgMixedInner
// FP32 V-cycles from zero on A e = r, x += e, until ||r||^2 <= tol2 or
// ||r||^2 <= abs_r2 or max_vcycles inner V-cycles.  Returns the status;
// *vcycles gets the inner V-cycles run, *r2 the last ||r||^2.
__device__ inline int wg_solve_mixed(const WgLevel<double>& F, const WgLevel<float>* lev, int nlev,
                                     float w, double tol2, double abs_r2, int max_vcycles,
                                     CoarseLds& S, int* vcycles, double* r2_out) {
    double* x = F.x[0];
    const int N = int(cells(F.g));
    const Coeffs<double> C = wg_coeffs(F);
    const XAccess<double, XM_PLAIN> X{x};
    int k = 0;
    int status = WL_OK;
    double r2 = 0.0;
    for (;;) {
        double s = 0.0;
        for (int c = threadIdx.x; c < N; c += blockDim.x) {
            int i, j, kk;
            wg_coords(F.g, c, i, j, kk);
            double xI, Ax, D;
            apply_row<double, XM_PLAIN, false>(F.g, X, C, i, j, kk, xI, Ax, D);
            const double r = D > 0.0 ? F.b[c] - Ax : 0.0;
            lev[0].b[c] = float(r);
            s += r * r;
        }
        __syncthreads();
        r2 = wg_sum(s, S.red);
        if (!isfinite(r2)) {
            status = WL_ERR_NONFINITE;
            break;
        }
        if (r2 <= tol2 || r2 <= abs_r2 || k >= max_vcycles) break;
        const int m = min(kWgMixedInner, max_vcycles - k);
        for (int v = 0; v < m; ++v) wg_vcycle32(lev, nlev, w, v == 0, S);
        for (int c = threadIdx.x; c < N; c += blockDim.x) x[c] += double(lev[0].x[1][c]);
        __syncthreads();
        k += m;
    }
    if (status == WL_OK && !(r2 <= tol2 || r2 <= abs_r2)) status = WL_ERR_NOT_CONVERGED;
    *vcycles = k;
    *r2_out = r2;
    return status;
}

}  // namespace wl
