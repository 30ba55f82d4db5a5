// Conjugate-gradient smoothing on the multigrid levels.  Sec. 2 notes that
// relaxations that visit points in order cannot be written as kernels and
// that the levels are therefore smoothed with conjugate gradients.  Each
// smoothing step here is a fresh run of Jacobi-preconditioned CG on the
// level's system, written for the positive semi-definite M = -A and c = -b:
//
//   r = P(c - M x), z = r / D, p = z;  per iteration
//   q = M p, alpha = (r.z)/(p.q), x += alpha p, r = P(r - alpha q),
//   z = r / D, beta = (r.z)/(r.z)_old, p = z + beta p,
//
// with D = -diag(A) (the sum of a cell's face coefficients; 0 on inactive
// cells, which stay at zero) and P the removal of the mean over the active
// cells, which keeps the residual in the range of M (a no-op in exact
// arithmetic that keeps the iteration stable once it reaches the rounding
// floor of the singular system).  P is folded into the sums: with n active
// cells and the unprojected r, m = sum r / n and
//   (r - m).(r - m)/D = sum r^2/D - 2 m sum r/D + m^2 sum 1/D,
// so one deterministic reduction per half-iteration gives m, r.z and beta
// (or alpha), and the next sweep applies r - m as it reads r.
//
// Kernels: init (residual, 1/D, sums), dir (projection, z, new direction),
// apply (q = M p and p.q), update (x, r and the sums); the reductions are
// one workgroup, fixed order.  Scalars (m, r.z, alpha, beta) live in the
// level's device scalars: nothing returns to the host.
#include "wl_device.h"

namespace wl {
namespace {

enum { CG_M = 0, CG_RZ = 1, CG_ALPHA = 2, CG_BETA = 3 };
constexpr int kSums = 5;  // sum r, r^2/D, r/D, 1/D, count over active cells

// Five per-block sums of one thread's values, written to partial[5 * block].
__device__ __forceinline__ void block_sums5(double (&v)[kSums], double* partial) {
    __shared__ double lds[4 * kSums];
#pragma unroll
    for (int k = 0; k < kSums; ++k)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
    const int t = threadIdx.x;
    if ((t & 63) == 0)
#pragma unroll
        for (int k = 0; k < kSums; ++k) lds[(t >> 6) * kSums + k] = v[k];
    __syncthreads();
    if (t == 0)
#pragma unroll
        for (int k = 0; k < kSums; ++k) {
            double s = 0.0;
            for (int w = 0; w < (kBlock >> 6); ++w) s += lds[w * kSums + k];
            partial[kSums * block_linear() + k] = s;
        }
}

// r = A x - (b - mean) on active cells (= c - M x), 0 elsewhere; 1/D into
// dinv (non-uniform levels); with XM_ZERO, x is written as zero.
template <typename T, int XM, bool UNIF>
__global__ __launch_bounds__(kBlock) void k_cg_init(TileDev TL, Grid g, XAccess<T, XM> X,
                                                    Coeffs<T> C, const T* __restrict__ b,
                                                    const double* __restrict__ bshift,
                                                    T* __restrict__ xzero, T* __restrict__ r,
                                                    T* __restrict__ dinv,
                                                    double* __restrict__ partial) {
    const Span sp = tile_span(TL, g.n0, g.n1, g.n2);
    double v[kSums] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (sp.i < g.n0 && sp.j < g.n1) {
        const T mean = bshift ? T(*bshift) : T(0);
        for (int k = sp.z0; k < sp.z1; ++k) {
            const size_t id = cid(g, sp.i, sp.j, k);
            T xI, Ax, D;
            apply_row<T, XM, UNIF>(g, X, C, sp.i, sp.j, k, xI, Ax, D);
            const bool act = D > T(0);
            T bv = b[id];
            if (bshift) bv = act ? bv - mean : T(0);
            const T rv = act ? Ax - bv : T(0);
            const T di = act ? T(1) / D : T(0);
            r[id] = rv;
            if (!UNIF) dinv[id] = di;
            if (XM == XM_ZERO) xzero[id] = T(0);
            if (act) {
                const double rd = double(rv), dd = double(di);
                v[0] += rd;
                v[1] += rd * rd * dd;
                v[2] += rd * dd;
                v[3] += dd;
                v[4] += 1.0;
            }
        }
    }
    block_sums5(v, partial);
}

// m, the projected r.z and beta from the five sums (first: beta = 0).
__global__ __launch_bounds__(1024) void k_cg_reduce_rz(const double* __restrict__ partial,
                                                       size_t nslots, double* __restrict__ cgs,
                                                       int first) {
    __shared__ double lds[16 * kSums];
    double S[kSums];
    wg_slot_reduce<kSums, false>(partial, nslots, S, lds);
    if (threadIdx.x == 0) {
        const double m = S[4] > 0.0 ? S[0] / S[4] : 0.0;
        const double rz = fmax(S[1] - 2.0 * m * S[2] + m * m * S[3], 0.0);
        const double old = cgs[CG_RZ];
        cgs[CG_BETA] = (first || !(old > 0.0)) ? 0.0 : rz / old;
        cgs[CG_M] = m;
        cgs[CG_RZ] = rz;
    }
}

// r <- r - m (active cells), z = r / D, p <- z + beta p (first: p = z).
template <typename T, bool UNIF>
__global__ __launch_bounds__(kBlock) void k_cg_dir(TileDev TL, Grid g, T* __restrict__ r,
                                                   const T* __restrict__ dinv, T dinv_u,
                                                   T* __restrict__ p,
                                                   const double* __restrict__ cgs, int first) {
    const Span sp = tile_span(TL, g.n0, g.n1, g.n2);
    if (sp.i >= g.n0 || sp.j >= g.n1) return;
    const T m = T(cgs[CG_M]), beta = T(cgs[CG_BETA]);
    for (int k = sp.z0; k < sp.z1; ++k) {
        const size_t id = cid(g, sp.i, sp.j, k);
        const T di = UNIF ? dinv_u : dinv[id];
        const T rv = di > T(0) ? r[id] - m : T(0);
        r[id] = rv;
        const T z = rv * di;
        p[id] = first ? z : fma(beta, p[id], z);
    }
}

// q = M p = -A p on active cells (0 elsewhere) and the block sums of p.q.
template <typename T, bool UNIF>
__global__ __launch_bounds__(kBlock) void k_cg_apply(TileDev TL, Grid g, const T* __restrict__ p,
                                                     Coeffs<T> C, T* __restrict__ q,
                                                     double* __restrict__ partial) {
    __shared__ double lds[4];
    const Span sp = tile_span(TL, g.n0, g.n1, g.n2);
    double pq = 0.0;
    if (sp.i < g.n0 && sp.j < g.n1) {
        const XAccess<T, XM_PLAIN> P{p};
        for (int k = sp.z0; k < sp.z1; ++k) {
            const size_t id = cid(g, sp.i, sp.j, k);
            T pI, Ap, D;
            apply_row<T, XM_PLAIN, UNIF>(g, P, C, sp.i, sp.j, k, pI, Ap, D);
            const T qv = D > T(0) ? -Ap : T(0);
            q[id] = qv;
            pq += double(pI) * double(qv);
        }
    }
    const double s = block_sum(pq, lds);
    if (threadIdx.x == 0) partial[block_linear()] = s;
}

// alpha = (r.z) / (p.q), 0 when either is not positive (nothing to do).
__global__ __launch_bounds__(1024) void k_cg_reduce_alpha(const double* __restrict__ partial,
                                                          size_t nslots, double* __restrict__ cgs) {
    __shared__ double lds[16];
    double S[1];
    wg_slot_reduce<1, false>(partial, nslots, S, lds);
    if (threadIdx.x == 0) {
        const double rz = cgs[CG_RZ];
        cgs[CG_ALPHA] = (S[0] > 0.0 && rz > 0.0) ? rz / S[0] : 0.0;
    }
}

// x += alpha p, r -= alpha q; with sums, the five sums of the new r.
template <typename T, bool UNIF>
__global__ __launch_bounds__(kBlock) void k_cg_update(TileDev TL, Grid g, T* __restrict__ x,
                                                      const T* __restrict__ p, T* __restrict__ r,
                                                      const T* __restrict__ q,
                                                      const T* __restrict__ dinv, T dinv_u,
                                                      const double* __restrict__ cgs,
                                                      double* __restrict__ partial, int sums) {
    const Span sp = tile_span(TL, g.n0, g.n1, g.n2);
    double v[kSums] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (sp.i < g.n0 && sp.j < g.n1) {
        const T alpha = T(cgs[CG_ALPHA]);
        for (int k = sp.z0; k < sp.z1; ++k) {
            const size_t id = cid(g, sp.i, sp.j, k);
            x[id] = fma(alpha, p[id], x[id]);
            const T rv = fma(-alpha, q[id], r[id]);
            r[id] = rv;
            const T di = UNIF ? dinv_u : dinv[id];
            if (sums && di > T(0)) {
                const double rd = double(rv), dd = double(di);
                v[0] += rd;
                v[1] += rd * rd * dd;
                v[2] += rd * dd;
                v[3] += dd;
                v[4] += 1.0;
            }
        }
    }
    if (sums) block_sums5(v, partial);
}

}  // namespace

template <typename T>
wl_status cg_smooth(const Hierarchy<T>& h, const Level<T>& L, T* x, bool zero, const T* b,
                    const double* bshift, int iters, hipStream_t s) {
    if (!L.cr || !L.cp || !L.cq || !L.cgs || !h.cgpart) {
        set_error("internal: conjugate-gradient smoothing on a hierarchy laid out without it");
        return WL_ERR_INVALID_ARG;
    }
    const Launch ln = launch_for(L.g.n0, L.g.n1, L.g.n2);
    const Coeffs<T> C{L.L[0], L.L[1], L.L[2], L.Lc};
    const bool u = L.uniform != 0;
    // uniform levels (fully periodic, one coefficient): every cell is active
    // with D = 2 d Lc
    const T Du = T(2 * L.g.ndim) * L.Lc;
    const T dinv_u = Du > T(0) ? T(1) / Du : T(0);
    double* part = h.cgpart;
    const unsigned nb = ln.nblocks();
#define WL_CG_INIT(XM, U)                                                                        \
    k_cg_init<T, XM, U><<<ln.grid, ln.block, 0, s>>>(ln.td, L.g, XAccess<T, XM>{x}, C, b, bshift, \
                                                     x, L.cr, L.cd, part)
    if (zero) {
        if (u) WL_CG_INIT(XM_ZERO, true); else WL_CG_INIT(XM_ZERO, false);
    } else {
        if (u) WL_CG_INIT(XM_PLAIN, true); else WL_CG_INIT(XM_PLAIN, false);
    }
#undef WL_CG_INIT
    WL_CHECK_LAUNCH();
    k_cg_reduce_rz<<<1, 1024, 0, s>>>(part, nb, L.cgs, 1);
    WL_CHECK_LAUNCH();
    for (int it = 0; it < iters; ++it) {
        const int first = it == 0 ? 1 : 0;
        const bool more = it + 1 < iters;
        if (u) {
            k_cg_dir<T, true><<<ln.grid, ln.block, 0, s>>>(ln.td, L.g, L.cr, L.cd, dinv_u, L.cp,
                                                           L.cgs, first);
            WL_CHECK_LAUNCH();
            k_cg_apply<T, true><<<ln.grid, ln.block, 0, s>>>(ln.td, L.g, L.cp, C, L.cq, part);
        } else {
            k_cg_dir<T, false><<<ln.grid, ln.block, 0, s>>>(ln.td, L.g, L.cr, L.cd, dinv_u, L.cp,
                                                            L.cgs, first);
            WL_CHECK_LAUNCH();
            k_cg_apply<T, false><<<ln.grid, ln.block, 0, s>>>(ln.td, L.g, L.cp, C, L.cq, part);
        }
        WL_CHECK_LAUNCH();
        k_cg_reduce_alpha<<<1, 1024, 0, s>>>(part, nb, L.cgs);
        WL_CHECK_LAUNCH();
        if (u)
            k_cg_update<T, true><<<ln.grid, ln.block, 0, s>>>(ln.td, L.g, x, L.cp, L.cr, L.cq, L.cd,
                                                              dinv_u, L.cgs, part, more ? 1 : 0);
        else
            k_cg_update<T, false><<<ln.grid, ln.block, 0, s>>>(ln.td, L.g, x, L.cp, L.cr, L.cq,
                                                               L.cd, dinv_u, L.cgs, part,
                                                               more ? 1 : 0);
        WL_CHECK_LAUNCH();
        if (more) {
            k_cg_reduce_rz<<<1, 1024, 0, s>>>(part, nb, L.cgs, 0);
            WL_CHECK_LAUNCH();
        }
    }
    return WL_OK;
}

template wl_status cg_smooth<float>(const Hierarchy<float>&, const Level<float>&, float*, bool,
                                    const float*, const double*, int, hipStream_t);
template wl_status cg_smooth<double>(const Hierarchy<double>&, const Level<double>&, double*, bool,
                                     const double*, const double*, int, hipStream_t);

}  // namespace wl
