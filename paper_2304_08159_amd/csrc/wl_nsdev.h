// Per-face geometry and BDIM arithmetic shared by the tiled Navier-Stokes
// kernels and the one-workgroup batched steps, so that both evaluate them
// with the same operations.
#pragma once

#include "wl_ns.h"
#include "wl_vel.h"

namespace wl {

// Flux of u_c through the lower d-face of the c-momentum control volume at J:
// ubar * phi - nu (u_c(J) - u_c(J - delta_d)), phi the limited third-order
// upwind-biased face value.
template <typename T, bool ALLPER>
__device__ __forceinline__ T face_flux(const VelField<T>& V, int c, int d, int i, int j, int k,
                                       T nu) {
    const int di = d == 0, dj = d == 1, dk = d == 2;
    const int ci = c == 0, cj = c == 1, ck = c == 2;
    const T um2 = vget<T, ALLPER>(V, c, i - 2 * di, j - 2 * dj, k - 2 * dk);
    const T um1 = vget<T, ALLPER>(V, c, i - di, j - dj, k - dk);
    const T u0 = vget<T, ALLPER>(V, c, i, j, k);
    const T up1 = vget<T, ALLPER>(V, c, i + di, j + dj, k + dk);
    const T ubar = T(0.5) * (vget<T, ALLPER>(V, d, i, j, k) +
                             vget<T, ALLPER>(V, d, i - ci, j - cj, k - ck));
    const bool pos = ubar >= T(0);
    const T cu = pos ? um1 : u0;
    const T bd = pos ? u0 : um1;
    const T au = pos ? um2 : up1;
    const T phik = (T(5) * cu + T(2) * bd - au) / T(6);
    const T phi = med3(phik, cu, med3(T(2) * cu - au, cu, bd));
    return ubar * phi - nu * (u0 - um1);
}

// BDIM moments of the lower c-face of cell (i, j, k) (c >= ndim: none):
// signed distance d of the body at the face centre, r = d / eps,
//   mu0 = (1 + r + sin(pi r)/pi) / 2,
//   mu1 = eps [(1 - r^2)/4 - r sin(pi r)/(2 pi) - (1 + cos(pi r))/(2 pi^2)]
// for |r| < 1 (1 / 0 outside), and the unit normal n = grad d.  Sphere /
// circle (kind 1) or torus about the x axis (kind 2); kind 0: mu0 = 1.
__device__ __forceinline__ void measure_face(const Grid& g, const BodyDev& body, int c, int i,
                                             int j, int k, double& m0, double& m1,
                                             double nrm[3]) {
    m0 = 1.0;
    m1 = 0.0;
    nrm[0] = nrm[1] = nrm[2] = 0.0;
    if (body.kind == 0 || c >= g.ndim) return;
    double x[3] = {i + 0.5, j + 0.5, k + 0.5};
    x[c] -= 0.5;
    double rel[3] = {0.0, 0.0, 0.0}, sd;
    for (int d = 0; d < g.ndim; ++d) rel[d] = x[d] - body.centre[d];
    if (body.kind == 1) {
        double r2 = 0.0;
        for (int d = 0; d < g.ndim; ++d) r2 += rel[d] * rel[d];
        const double dist = sqrt(r2);
        sd = dist - body.radius;
        if (dist > 0.0)
            for (int d = 0; d < g.ndim; ++d) nrm[d] = rel[d] / dist;
    } else {
        // torus about the x axis: distance to the tube's centre circle (in
        // the plane through x and the axis) minus the tube radius
        const double rho = sqrt(rel[1] * rel[1] + rel[2] * rel[2]);
        const double qr = rho - body.radius;
        const double q = sqrt(rel[0] * rel[0] + qr * qr);
        sd = q - body.radius2;
        if (q > 0.0) {
            nrm[0] = rel[0] / q;
            if (rho > 0.0) {
                nrm[1] = qr / q * rel[1] / rho;
                nrm[2] = qr / q * rel[2] / rho;
            }
        }
    }
    const double r = sd / body.eps;
    if (r >= 1.0) {
        m0 = 1.0;
    } else if (r <= -1.0) {
        m0 = 0.0;
    } else {
        const double pi = 3.14159265358979323846;
        const double sn = sin(pi * r), cs = cos(pi * r);
        m0 = 0.5 * (1.0 + r + sn / pi);
        m1 = body.eps * ((1.0 - r * r) / 4.0 - r * sn / (2.0 * pi) - (1.0 + cs) / (2.0 * pi * pi));
    }
}

// Poisson coefficient of the lower c-face: mu0, 0 on a non-periodic lower
// domain face and on the z faces in 2D.
__device__ __forceinline__ double face_coeff(const Grid& g, const int bclo[3], int c, int i, int j,
                                             int k, double m0) {
    const int coord[3] = {i, j, k};
    double L = (c < g.ndim) ? m0 : 0.0;
    if (bclo[c] != WL_BC_PERIODIC && coord[c] == 0) L = 0.0;
    return L;
}

// First-order BDIM blend of the lower c-face of cell (i, j, k):
//   u*_c = mu0_c f_c + (1 - mu0_c) V_b,c
//          + sum_d (mu1 n)_cd [(f_c(I+delta_d) - f_c(I-delta_d)) / 2 - dV_b,c/dx_d],
// V_b the body velocity at the face (zero for a body at rest); boundary faces
// keep f.  EAGER loads the neighbours of every direction before testing
// (mu1 n)_cd, so that the loads do not wait on it (same result).
template <typename T, bool EAGER = false>
__device__ __forceinline__ T bdim_face(const VelField<T>& F, const BdimFields<T>& B,
                                       const BodyMotionDev& mo, int c, int i, int j, int k) {
    const Grid& g = F.g;
    const size_t id = cid(g, i, j, k);
    const int coord[3] = {i, j, k};
    const int per[3] = {g.per0, g.per1, g.per2};
    const T f = F.u[c][id];
    if (!per[c] && coord[c] == 0) return f;
    const T m0 = B.mu0[c][id];
    T v = m0 * f;
    // body velocity at the face centre and its gradient row c
    double gw[3] = {0.0, 0.0, 0.0};
    if (mo.on) {
        double x[3] = {i + 0.5 - mo.X[0], j + 0.5 - mo.X[1], k + 0.5 - mo.X[2]};
        x[c] -= 0.5;
        if (g.ndim == 2) x[2] = 0.0;
        const double cr[3] = {mo.w[1] * x[2] - mo.w[2] * x[1], mo.w[2] * x[0] - mo.w[0] * x[2],
                              mo.w[0] * x[1] - mo.w[1] * x[0]};
        v += (T(1) - m0) * T(mo.xdot[c] + cr[c]);
        // dV_b,c/dx_d = eps_{c k d} w_k
        const double G[3][3] = {{0.0, -mo.w[2], mo.w[1]},
                                {mo.w[2], 0.0, -mo.w[0]},
                                {-mo.w[1], mo.w[0], 0.0}};
        for (int d = 0; d < 3; ++d) gw[d] = G[c][d];
    }
    if constexpr (EAGER) {
        T m[3], fp[3], fm[3];
        for (int d = 0; d < g.ndim; ++d) {
            m[d] = B.mu1n[3 * c + d][id];
            fp[d] = vget<T, false>(F, c, i + (d == 0), j + (d == 1), k + (d == 2));
            fm[d] = vget<T, false>(F, c, i - (d == 0), j - (d == 1), k - (d == 2));
        }
        for (int d = 0; d < g.ndim; ++d)
            if (m[d] != T(0)) v += m[d] * (T(0.5) * (fp[d] - fm[d]) - T(gw[d]));
        return v;
    }
    for (int d = 0; d < g.ndim; ++d) {
        const T m = B.mu1n[3 * c + d][id];
        if (m != T(0)) {
            const T fp = vget<T, false>(F, c, i + (d == 0), j + (d == 1), k + (d == 2));
            const T fm = vget<T, false>(F, c, i - (d == 0), j - (d == 1), k - (d == 2));
            v += m * (T(0.5) * (fp - fm) - T(gw[d]));
        }
    }
    return v;
}

}  // namespace wl
