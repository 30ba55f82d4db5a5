// Coarsest-level solve shared by the multigrid kernels and the batched
// one-workgroup solver.
#pragma once

#include "wl_device.h"

namespace wl {

struct CoarseLds {
    double L[3][kCoarseMax];
    double x[kCoarseMax], r[kCoarseMax], p[kCoarseMax], q[kCoarseMax];
    double red[16];
};

// Coarsest level: CG on -A (SPD on the active set) with the right-hand side
// restricted to the active cells and made mean-free there; FP64 internally,
// minimum-norm (mean-free) result.  Run by one whole workgroup (any size up to
// 1024 threads), everything in LDS; ends with a barrier.
template <typename T>
__device__ void coarse_cg_block(const Grid& g, const Coeffs<T>& C, int uniform,
                                const T* __restrict__ b, T* __restrict__ xout, double tol,
                                int maxit, CoarseLds& S) {
    double (&sL)[3][kCoarseMax] = S.L;
    double* sx = S.x;
    double* sr = S.r;
    double* sp = S.p;
    double* sq = S.q;
    double* red = S.red;
    const int N = int(cells(g));
    const int t = threadIdx.x, nt = blockDim.x;
    auto dot_all = [&](double v) -> double {  // fixed-order block sum broadcast to all
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if ((t & 63) == 0) red[t >> 6] = v;
        __syncthreads();
        double s = 0.0;
        for (int w = 0; w < (nt + 63) / 64; ++w) s += red[w];
        __syncthreads();
        return s;
    };
    for (int c = t; c < N; c += nt) {
        sL[0][c] = uniform ? double(C.Lc) : double(C.L0[c]);
        sL[1][c] = uniform ? double(C.Lc) : double(C.L1[c]);
        sL[2][c] = (g.ndim == 3) ? (uniform ? double(C.Lc) : double(C.L2[c])) : 0.0;
    }
    __syncthreads();
    auto coords = [&](int c, int& i, int& j, int& k) {
        i = c % g.n0;
        j = (c / g.n0) % g.n1;
        k = c / (g.n0 * g.n1);
    };
    auto lup = [&](int d, int i, int j, int k) -> double {  // coefficient of the upper d-face
        int n = d == 0 ? g.n0 : (d == 1 ? g.n1 : g.n2);
        int per = d == 0 ? g.per0 : (d == 1 ? g.per1 : g.per2);
        int c = d == 0 ? i : (d == 1 ? j : k);
        if (c < n - 1 || per) {
            int cu = (c < n - 1) ? c + 1 : 0;
            int ii = d == 0 ? cu : i, jj = d == 1 ? cu : j, kk = d == 2 ? cu : k;
            return sL[d][ii + g.n0 * (jj + g.n1 * kk)];
        }
        return 0.0;
    };
    auto diag = [&](int c) -> double {  // sum of the 2d face coefficients of cell c
        int i, j, k;
        coords(c, i, j, k);
        double D = 0.0;
        for (int d = 0; d < g.ndim; ++d) D += sL[d][c] + lup(d, i, j, k);
        return D;
    };
    // sq holds D during set-up and A p during the iteration
    double sumb = 0.0, cnt = 0.0;
    for (int c = t; c < N; c += nt) {
        const double D = diag(c);
        sq[c] = D;
        if (D > 0.0) {
            sumb += double(b[c]);
            cnt += 1.0;
        }
    }
    sumb = dot_all(sumb);
    cnt = dot_all(cnt);
    const double mean = cnt > 0.0 ? sumb / cnt : 0.0;
    // solve M x = B with M = -A, B = -(b - mean) on active cells
    double rr = 0.0;
    for (int c = t; c < N; c += nt) {
        const double B = sq[c] > 0.0 ? -(double(b[c]) - mean) : 0.0;
        sx[c] = 0.0;
        sr[c] = B;
        sp[c] = B;
        rr += B * B;
    }
    rr = dot_all(rr);
    const double rr0 = rr;
    if (rr0 > 0.0) {
        for (int it = 0; it < maxit; ++it) {
            double pq = 0.0;
            for (int c = t; c < N; c += nt) {
                int i, j, k;
                coords(c, i, j, k);
                double Mp = 0.0;
                const double D = diag(c);
                if (D > 0.0) {
                    const double pc = sp[c];
                    Mp = D * pc;
                    // neighbours
                    {
                        int il = nb_lo(i, g.n0, g.per0), iu = nb_up(i, g.n0, g.per0);
                        Mp -= sL[0][c] * sp[il + g.n0 * (j + g.n1 * k)];
                        Mp -= lup(0, i, j, k) * sp[iu + g.n0 * (j + g.n1 * k)];
                    }
                    {
                        int jl = nb_lo(j, g.n1, g.per1), ju = nb_up(j, g.n1, g.per1);
                        Mp -= sL[1][c] * sp[i + g.n0 * (jl + g.n1 * k)];
                        Mp -= lup(1, i, j, k) * sp[i + g.n0 * (ju + g.n1 * k)];
                    }
                    if (g.ndim == 3) {
                        int kl = nb_lo(k, g.n2, g.per2), ku = nb_up(k, g.n2, g.per2);
                        Mp -= sL[2][c] * sp[i + g.n0 * (j + g.n1 * kl)];
                        Mp -= lup(2, i, j, k) * sp[i + g.n0 * (j + g.n1 * ku)];
                    }
                }
                sq[c] = Mp;
                pq += sp[c] * Mp;
            }
            pq = dot_all(pq);
            if (!(pq > 0.0)) break;
            const double alpha = rr / pq;
            double rn = 0.0;
            for (int c = t; c < N; c += nt) {
                sx[c] += alpha * sp[c];
                sr[c] -= alpha * sq[c];
                rn += sr[c] * sr[c];
            }
            rn = dot_all(rn);
            if (rn <= tol * tol * rr0) break;
            const double beta = rn / rr;
            rr = rn;
            for (int c = t; c < N; c += nt) sp[c] = sr[c] + beta * sp[c];
            __syncthreads();
        }
    }
    // mean-free result on the active cells
    double sx_sum = 0.0;
    for (int c = t; c < N; c += nt)
        if (diag(c) > 0.0) sx_sum += sx[c];
    sx_sum = dot_all(sx_sum);
    const double xm = cnt > 0.0 ? sx_sum / cnt : 0.0;
    for (int c = t; c < N; c += nt) xout[c] = diag(c) > 0.0 ? T(sx[c] - xm) : T(0);
    __syncthreads();
}

}  // namespace wl
