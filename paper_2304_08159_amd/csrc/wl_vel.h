// Velocity ghost rules and the exact median shared by the forward and the
// adjoint Navier-Stokes kernels.
#pragma once

#include "wl_device.h"
#include "wl_ns.h"

namespace wl {

// --------------------------------------------------------- velocity ghosts

// Value of velocity component c at (i, j, k), where at most one coordinate
// lies outside the grid (by up to two cells).  Ghost rules: periodic wrap;
// INFLOW ghosts = U; free-slip WALL: normal component odd about the wall
// face (boundary face 0), tangential components even; OUTFLOW (upper x): the
// boundary face is the plane uout, ghosts beyond it zero-gradient.
template <typename T, bool ALLPER>
__device__ __forceinline__ T vget(const VelField<T>& V, int c, int i, int j, int k) {
    const Grid& g = V.g;
    if (ALLPER) {
        i = i < 0 ? i + g.n0 : (i >= g.n0 ? i - g.n0 : i);
        j = j < 0 ? j + g.n1 : (j >= g.n1 ? j - g.n1 : j);
        if (g.ndim == 3) k = k < 0 ? k + g.n2 : (k >= g.n2 ? k - g.n2 : k);
        return V.u[c][cid(g, i, j, k)];
    }
    int q[3] = {i, j, k};
    const int n[3] = {g.n0, g.n1, g.n2};
    const int per[3] = {g.per0, g.per1, g.per2};
#pragma unroll
    for (int d = 0; d < 3; ++d)
        if (per[d]) q[d] = q[d] < 0 ? q[d] + n[d] : (q[d] >= n[d] ? q[d] - n[d] : q[d]);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int m = n[d], kk = q[d];
        if (kk >= 0 && kk < m) continue;
        // (the other coordinates are in range for every evaluation the kernels
        // make; clamping keeps any other request inside the array)
        auto at = [&](int idx) -> T {
            int r[3] = {q[0], q[1], q[2]};
            r[d] = idx;
#pragma unroll
            for (int e = 0; e < 3; ++e) r[e] = r[e] < 0 ? 0 : (r[e] >= n[e] ? n[e] - 1 : r[e]);
            return V.u[c][cid(g, r[0], r[1], r[2])];
        };
        if (kk < 0) {
            if (V.bclo[d] == WL_BC_INFLOW) return V.U[c];
            if (c == d) {
                const int mir = -kk;
                return -at(mir < m ? mir : 0);
            }
            const int mir = -1 - kk;
            return at(mir < m - 1 ? mir : m - 1);
        }
        if (c == d) {
            if (V.bchi[d] == WL_BC_OUTFLOW) {
                const int a = q[1] < 0 ? 0 : (q[1] >= g.n1 ? g.n1 - 1 : q[1]);
                const int b = q[2] < 0 ? 0 : (q[2] >= g.n2 ? g.n2 - 1 : q[2]);
                return V.uout[a + size_t(g.n1) * b];
            }
            if (kk == m) return T(0);
            return -at(m - 1 > 0 ? m - 1 : 0);
        }
        if (V.bchi[d] == WL_BC_OUTFLOW) return at(m - 1);
        if (kk == m) return at(m - 1);
        return at(m - 2 > 0 ? m - 2 : 0);
    }
    return V.u[c][cid(g, q[0], q[1], q[2])];
}

// Pressure-gradient update of one face: u - cl (p_here - p_lower) with
// cl = c dt L, one rounding (shared by the projection kernel and the
// momentum kernel that applies the predictor projection on the fly).
__device__ __forceinline__ float proj_face(float u, float cl, float ph, float pl) {
    return fmaf(-cl, ph - pl, u);
}
__device__ __forceinline__ double proj_face(double u, double cl, double ph, double pl) {
    return fma(-cl, ph - pl, u);
}

__device__ __forceinline__ float med3(float a, float b, float c) {
    return __builtin_amdgcn_fmed3f(a, b, c);
}
__device__ __forceinline__ double med3(double a, double b, double c) {
    return fmax(fmin(a, b), fmin(fmax(a, b), c));
}

}  // namespace wl
