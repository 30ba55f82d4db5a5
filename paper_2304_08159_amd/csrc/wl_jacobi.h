// The damped-Jacobi update of one cell, shared by the single-sweep and the
// fused two-sweep multigrid kernels so that both evaluate it with the same
// operations in the same order (their iterates are then bitwise equal).
#pragma once

#include <hip/hip_runtime.h>

namespace wl {

// A x and the diagonal magnitude D of one row,
//   A x = sum_d Lu_d (x_up - x) - Ll_d (x - x_lo),   D = sum_d (Ll_d + Lu_d),
// from the cell value, its lower / upper neighbours per direction and the
// face coefficients; the z terms are left out in 2D.
template <typename T>
__device__ __forceinline__ void jacobi_terms(T xI, T xxl, T xxu, T xyl, T xyu, T xzl, T xzu,
                                             T Lxl, T Lxu, T Lyl, T Lyu, T Lzl, T Lzu, bool d3,
                                             T& Ax, T& D) {
    Ax = T(0);
    D = T(0);
    Ax += Lxu * (xxu - xI) - Lxl * (xI - xxl);
    D += Lxl + Lxu;
    Ax += Lyu * (xyu - xI) - Lyl * (xI - xyl);
    D += Lyl + Lyu;
    if (d3) {
        Ax += Lzu * (xzu - xI) - Lzl * (xI - xzl);
        D += Lzl + Lzu;
    }
}

// Residual b - A x of one row as the restriction forms it, with every
// rounding fixed: per direction one product and one fused multiply-add, the
// directions summed x, y, z.  A kernel that walks column pairs shares the
// product of the face between the two cells, which would otherwise let the
// compiler fuse the other product of the lower cell's term; written out,
// the pair kernel and one that forms single cells agree bit for bit.
template <typename T>
__device__ __forceinline__ T resid_row(T bv, T xI, T xxl, T xxu, T xyl, T xyu, T xzl, T xzu,
                                       T Lxl, T Lxu, T Lyl, T Lyu, T Lzl, T Lzu, bool d3) {
#pragma clang fp contract(off)
    T Ax = fma(Lxu, xxu - xI, -(Lxl * (xI - xxl)));
    Ax = Ax + fma(Lyu, xyu - xI, -(Lyl * (xI - xyl)));
    if (d3) Ax = Ax + fma(Lzu, xzu - xI, -(Lzl * (xI - xzl)));
    return bv - Ax;
}

// A x of a row on a level with one coefficient Lc: the second differences
// of the directions summed, then one multiply.
template <typename T>
__device__ __forceinline__ T jacobi_ax_uniform(T xI, T xxl, T xxu, T xyl, T xyu, T xzl, T xzu,
                                               T Lc, bool d3) {
    T s = (xxu - xI) - (xI - xxl);
    s += (xyu - xI) - (xI - xyl);
    if (d3) s += (xzu - xI) - (xI - xzl);
    return Lc * s;
}

// Right-hand side seen by the sweep: with a mean to remove, b - mean on
// active cells and 0 on inactive ones.
template <typename T>
__device__ __forceinline__ T jacobi_rhs(T bv, bool act, bool shift, T mean) {
    if (shift) bv = act ? bv - mean : T(0);
    return bv;
}

// x - (w / D) r on active cells (D > 0), 0 elsewhere.  The factor is one
// correctly rounded division of w by D, so a kernel that knows D from the
// cell's position may take it from a table formed by the same division.
template <typename T>
__device__ __forceinline__ T jacobi_new(T xI, T r, T D, T omega) {
    return D > T(0) ? xI - (omega / D) * r : T(0);
}

// The same with the factor w / D given: levels with one coefficient
// everywhere have one D, and the factor is formed once per level.
template <typename T>
__device__ __forceinline__ T jacobi_new_scaled(T xI, T r, bool act, T wD) {
    return act ? xI - wD * r : T(0);
}

}  // namespace wl
