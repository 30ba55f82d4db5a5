// Reverse-mode (adjoint) kernels of one Navier-Stokes step and of the
// pressure-drag functional.  The paper (Sec. 2) notes that the whole solver is
// differentiable; this is a hand-written discrete adjoint of the forward
// kernels in ns.hip under these readings: dt is frozen from the forward run,
// every pressure solve is treated as exact (p = A^+ sigma, so its adjoint is
// the same symmetric GMG solve), and the limiter / upwind branches are frozen
// at the forward values.
//
// Every adjoint is written as a gather (each output sums the contributions of
// the forward terms that read it, in a fixed order), so results are bitwise
// reproducible without atomics.  Reads through ghost cells are first gathered
// onto a padded array (two ghost layers) and then folded back onto the stored
// faces by the inverse of the ghost rules.
#include <cmath>

#include "wl_adj.h"
#include "wl_device.h"
#include "wl_vel.h"

namespace wl {

PadGrid pad_grid(const Grid& g) {
    PadGrid p;
    p.P0 = g.n0 + 4;
    p.P1 = g.n1 + 4;
    p.o2 = g.ndim == 3 ? 2 : 0;
    p.P2 = g.n2 + 2 * p.o2;
    return p;
}

__device__ __forceinline__ size_t pid(const PadGrid& p, int i, int j, int k) {
    return size_t(i + 2) + size_t(p.P0) * (size_t(j + 2) + size_t(p.P1) * size_t(k + p.o2));
}

__device__ __forceinline__ bool in_grid(const Grid& g, int i, int j, int k) {
    return i >= 0 && i < g.n0 && j >= 0 && j < g.n1 && k >= 0 && k < g.n2;
}

// interior face of component c: not the lower boundary face of a
// non-periodic direction c
__device__ __forceinline__ bool interior(const Grid& g, int c, int i, int j, int k) {
    const int per = c == 0 ? g.per0 : (c == 1 ? g.per1 : g.per2);
    const int q = c == 0 ? i : (c == 1 ? j : k);
    return per || q != 0;
}

template <typename T>
__device__ __forceinline__ T sixth(T v);
template <>
__device__ __forceinline__ float sixth<float>(float v) { return v * (1.f / 6.f); }
template <>
__device__ __forceinline__ double sixth<double>(double v) { return v / 6.0; }

// Adjoint weights of one face flux F_cd(J) = ubar phi(a, c, b) - nu (u_c(J) -
// u_c(J - delta_d)): with Fbar the adjoint of F, w[s] receives Fbar dF/du_c at
// J + s delta_d for s = -2..1 (w[0..3]) and wphi = Fbar phi (the adjoint of
// ubar).  Fbar = Rbar_c(J) - Rbar_c(J - delta_d) over the stored faces (R_c(I)
// = -(F(I + delta_d) - F(I)) sums into the stage).  Returns false when the face
// is not one the forward evaluates or Fbar is zero.
template <typename T, bool ALLPER>
__device__ bool face_adj(const VelField<T>& E, T* const* Rb, int c, int d, int i, int j, int k, T nu,
                         T w[4], T& wphi) {
    const Grid& g = E.g;
    const int J[3] = {i, j, k};
    const int n[3] = {g.n0, g.n1, g.n2};
    for (int e = 0; e < 3; ++e) {
        if (e == d) continue;
        if (J[e] < 0 || J[e] >= n[e]) return false;
    }
    if (J[d] < 0 || J[d] > n[d]) return false;
    T Fb = T(0);
    if (J[d] < n[d]) Fb += Rb[c][cid(g, i, j, k)];
    if (J[d] >= 1) Fb -= Rb[c][cid(g, i - (d == 0), j - (d == 1), k - (d == 2))];
    if (Fb == T(0)) return false;
    const int di = d == 0, dj = d == 1, dk = d == 2;
    const int ci = c == 0, cj = c == 1, ck = c == 2;
    const T um2 = vget<T, ALLPER>(E, c, i - 2 * di, j - 2 * dj, k - 2 * dk);
    const T um1 = vget<T, ALLPER>(E, c, i - di, j - dj, k - dk);
    const T u0 = vget<T, ALLPER>(E, c, i, j, k);
    const T up1 = vget<T, ALLPER>(E, c, i + di, j + dj, k + dk);
    const T ubar = T(0.5) * (vget<T, ALLPER>(E, d, i, j, k) +
                             vget<T, ALLPER>(E, d, i - ci, j - cj, k - ck));
    const bool pos = ubar >= T(0);
    const T cu = pos ? um1 : u0;
    const T bd = pos ? u0 : um1;
    const T au = pos ? um2 : up1;
    const T phik = sixth<T>(T(5) * cu + T(2) * bd - au);
    const T bnd = T(2) * cu - au;
    const T m1 = med3(bnd, cu, bd);
    const T phi = med3(phik, cu, m1);
    // d phi / d(au, cu, bd) on the active branch (ties take the first match)
    T pa, pc, pb;
    if (phi == phik) {
        pa = T(-1) / T(6);
        pc = T(5) / T(6);
        pb = T(2) / T(6);
    } else if (phi == cu) {
        pa = T(0);
        pc = T(1);
        pb = T(0);
    } else if (m1 == bnd) {
        pa = T(-1);
        pc = T(2);
        pb = T(0);
    } else {
        pa = T(0);
        pc = T(0);
        pb = T(1);
    }
    w[0] = w[1] = w[2] = w[3] = T(0);
    const T s = Fb * ubar;
    if (pos) {  // au = J-2d, cu = J-d, bd = J
        w[0] += s * pa;
        w[1] += s * pc;
        w[2] += s * pb;
    } else {    // au = J+d, cu = J, bd = J-d
        w[3] += s * pa;
        w[2] += s * pc;
        w[1] += s * pb;
    }
    w[2] -= nu * Fb;
    w[1] += nu * Fb;
    wphi = Fb * phi;
    return true;
}

// Gather of R'(e)^T Rbar on the padded grid: the padded value of component c
// at V receives every face flux that read u_c at V, as the transported
// variable (F_cd at J = V + 2d, V + d, V, V - d) or as half of an advecting
// velocity (F_{c2,c} at J = V and J = V + delta_c2).
template <typename T, bool ALLPER>
__global__ __launch_bounds__(kBlock) void k_adj_flux(TileDev TL, VelField<T> E, AdjPtrs<T> R, T nu,
                                                     PadField<T> out) {
    const Grid& g = E.g;
    const PadGrid& pg = out.pg;
    const Span sp = tile_span(TL, pg.P0, pg.P1, pg.P2);
    if (sp.i >= pg.P0 || sp.j >= pg.P1) return;
    const int i = sp.i - 2, j = sp.j - 2;
    for (int kk = sp.z0; kk < sp.z1; ++kk) {
        const int k = kk - pg.o2;
        for (int c = 0; c < g.ndim; ++c) {
            T acc = T(0);
            T w[4], wphi;
            for (int d = 0; d < g.ndim; ++d) {
                const int di = d == 0, dj = d == 1, dk = d == 2;
                // J = V - s d reads u_c at J + s d = V for slot s
                for (int sl = -2; sl <= 1; ++sl)
                    if (face_adj<T, ALLPER>(E, R.p, c, d, i - sl * di, j - sl * dj, k - sl * dk, nu,
                                            w, wphi))
                        acc += w[sl + 2];
            }
            for (int c2 = 0; c2 < g.ndim; ++c2) {
                const int ei = c2 == 0, ej = c2 == 1, ek = c2 == 2;
                if (face_adj<T, ALLPER>(E, R.p, c2, c, i, j, k, nu, w, wphi)) acc += T(0.5) * wphi;
                if (face_adj<T, ALLPER>(E, R.p, c2, c, i + ei, j + ej, k + ek, nu, w, wphi))
                    acc += T(0.5) * wphi;
            }
            out.a[c][pid(pg, i, j, k)] = acc;
        }
    }
}

// Gather of BDIM^T gbar on the padded grid:
//   f_bar(V) = mu0(V) gbar(V) + sum_j [mu1n_cj(V-dj) gbar(V-dj) - mu1n_cj(V+dj) gbar(V+dj)] / 2
// over stored interior faces.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_adj_bdim(TileDev TL, Grid g, AdjPtrs<T> gb, AdjPtrs<T> m0,
                                                     AdjPtrs9<T> m1, PadField<T> out) {
    const PadGrid& pg = out.pg;
    const Span sp = tile_span(TL, pg.P0, pg.P1, pg.P2);
    if (sp.i >= pg.P0 || sp.j >= pg.P1) return;
    const int i = sp.i - 2, j = sp.j - 2;
    for (int kk = sp.z0; kk < sp.z1; ++kk) {
        const int k = kk - pg.o2;
        for (int c = 0; c < g.ndim; ++c) {
            T acc = T(0);
            if (in_grid(g, i, j, k) && interior(g, c, i, j, k)) {
                const size_t id = cid(g, i, j, k);
                acc += m0.p[c][id] * gb.p[c][id];
            }
            for (int d = 0; d < g.ndim; ++d) {
                const int di = d == 0, dj = d == 1, dk = d == 2;
                const int a0 = i - di, a1 = j - dj, a2 = k - dk;
                if (in_grid(g, a0, a1, a2) && interior(g, c, a0, a1, a2)) {
                    const size_t id = cid(g, a0, a1, a2);
                    acc += T(0.5) * (m1.p[3 * c + d][id] * gb.p[c][id]);
                }
                const int b0 = i + di, b1 = j + dj, b2 = k + dk;
                if (in_grid(g, b0, b1, b2) && interior(g, c, b0, b1, b2)) {
                    const size_t id = cid(g, b0, b1, b2);
                    acc -= T(0.5) * (m1.p[3 * c + d][id] * gb.p[c][id]);
                }
            }
            out.a[c][pid(pg, i, j, k)] = acc;
        }
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_adj_bdim_param(TileDev TL, VelField<T> F, AdjPtrs<T> gb,
                                                           AdjPtrs<T> m0b, AdjPtrs9<T> m1b) {
    const Grid& g = F.g;
    const Span sp = tile_span(TL, g.n0, g.n1, g.n2);
    const int i = sp.i, j = sp.j;
    if (i >= g.n0 || j >= g.n1) return;
    for (int k = sp.z0; k < sp.z1; ++k) {
        const size_t id = cid(g, i, j, k);
        for (int c = 0; c < g.ndim; ++c) {
            if (!interior(g, c, i, j, k)) continue;
            const T gv = gb.p[c][id];
            m0b.p[c][id] += F.u[c][id] * gv;
            for (int d = 0; d < g.ndim; ++d) {
                const T fp = vget<T, false>(F, c, i + (d == 0), j + (d == 1), k + (d == 2));
                const T fm = vget<T, false>(F, c, i - (d == 0), j - (d == 1), k - (d == 2));
                m1b.p[3 * c + d][id] += T(0.5) * (fp - fm) * gv;
            }
        }
    }
}

// Preimages under the ghost rules of vget: the padded coordinates along
// direction d (with their factors) whose value is component c's stored value
// at coordinate q.  At most three entries.
struct Pre {
    int n;
    int q[3];
    signed char f[3];
};

__device__ __forceinline__ Pre preimages(const Grid& g, int c, int d, int q, int bclo, int bchi) {
    Pre P;
    P.n = 1;
    P.q[0] = q;
    P.f[0] = 1;
    const int m = d == 0 ? g.n0 : (d == 1 ? g.n1 : g.n2);
    const int per = d == 0 ? g.per0 : (d == 1 ? g.per1 : g.per2);
    auto add = [&](int v, int f) {
        P.q[P.n] = v;
        P.f[P.n] = static_cast<signed char>(f);
        ++P.n;
    };
    if (per) {
        if (q < 2) add(q + m, 1);
        if (q >= m - 2) add(q - m, 1);
        return P;
    }
    if (bclo == WL_BC_WALL) {
        if (c == d) {
            if (q == (1 < m ? 1 : 0)) add(-1, -1);
            if (q == (2 < m ? 2 : 0)) add(-2, -1);
        } else {
            if (q == 0) add(-1, 1);
            if (q == (1 < m - 1 ? 1 : m - 1)) add(-2, 1);
        }
    }
    if (bchi == WL_BC_WALL) {
        if (c == d) {
            if (q == (m - 1 > 0 ? m - 1 : 0)) add(m + 1, -1);
        } else {
            if (q == m - 1) add(m, 1);
            if (q == (m - 2 > 0 ? m - 2 : 0)) add(m + 1, 1);
        }
    } else if (bchi == WL_BC_OUTFLOW && c != d) {
        if (q == m - 1) {
            add(m, 1);
            add(m + 1, 1);
        }
    }
    return P;
}

// Fold of a padded adjoint onto the stored faces: the inverse of the ghost
// rules of vget (periodic wrap; wall: normal odd / tangential even
// reflections; outflow: zero-gradient tangential ghosts onto the last face,
// normal ghosts onto the outflow plane; inflow ghosts are constants).  Ghost
// positions outside the grid in several directions at once (reads of an
// advecting velocity at J - delta_c for J on an upper face) are the product
// of the per-direction rules, as in the forward's direction-by-direction fill.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_adj_fold(TileDev TL, VelField<T> G, PadField<T> pad,
                                                     AdjPtrs<T> acc, T* accout) {
    const Grid& g = G.g;
    const PadGrid& pg = pad.pg;
    const Span sp = tile_span(TL, g.n0, g.n1, g.n2);
    const int i = sp.i, j = sp.j;
    if (i >= g.n0 || j >= g.n1) return;
    for (int k = sp.z0; k < sp.z1; ++k) {
        const int K[3] = {i, j, k};
        for (int c = 0; c < g.ndim; ++c) {
            if (!interior(g, c, i, j, k)) continue;
            const T* P = pad.a[c];
            Pre pr[3];
            for (int d = 0; d < 3; ++d) {
                if (d < g.ndim) {
                    pr[d] = preimages(g, c, d, K[d], G.bclo[d], G.bchi[d]);
                } else {
                    pr[d].n = 1;
                    pr[d].q[0] = K[d];
                    pr[d].f[0] = 1;
                }
            }
            T v = T(0);
            for (int a = 0; a < pr[0].n; ++a)
                for (int b = 0; b < pr[1].n; ++b)
                    for (int e = 0; e < pr[2].n; ++e) {
                        const int f = pr[0].f[a] * pr[1].f[b] * pr[2].f[e];
                        const T x = P[pid(pg, pr[0].q[a], pr[1].q[b], pr[2].q[e])];
                        v += f > 0 ? x : -x;
                    }
            acc.p[c][cid(g, i, j, k)] += v;
        }
        if (accout && G.bchi[0] == WL_BC_OUTFLOW && i == g.n0 - 1) {
            // the outflow plane: x ghosts n0, n0+1 of component 0, times the
            // tangential preimages of (j, k)
            const T* P = pad.a[0];
            const Pre py = preimages(g, 0, 1, j, G.bclo[1], G.bchi[1]);
            Pre pz;
            if (g.ndim == 3) {
                pz = preimages(g, 0, 2, k, G.bclo[2], G.bchi[2]);
            } else {
                pz.n = 1;
                pz.q[0] = k;
                pz.f[0] = 1;
            }
            T v = T(0);
            for (int xg = g.n0; xg <= g.n0 + 1; ++xg)
                for (int b = 0; b < py.n; ++b)
                    for (int e = 0; e < pz.n; ++e) {
                        const T x = P[pid(pg, xg, py.q[b], pz.q[e])];
                        v += (py.f[b] * pz.f[e]) > 0 ? x : -x;
                    }
            accout[j + size_t(g.n1) * k] += v;
        }
    }
}

// rhs = pbar + coef * div(L ubar): the adjoint of u = g - coef L G p with
// respect to p is coef * div(L ubar) (G^T = -div on these faces).
template <typename T, bool UNIF>
__global__ __launch_bounds__(kBlock) void k_adj_proj_rhs(TileDev TL, Grid g, const T* __restrict__ pbar,
                                                         AdjPtrs<T> ub, AdjPtrs<T> L, T Lc, T coef,
                                                         T* __restrict__ rhs) {
    const Span sp = tile_span(TL, g.n0, g.n1, g.n2);
    const int i = sp.i, j = sp.j;
    if (i >= g.n0 || j >= g.n1) return;
    const int n[3] = {g.n0, g.n1, g.n2};
    const int per[3] = {g.per0, g.per1, g.per2};
    for (int k = sp.z0; k < sp.z1; ++k) {
        const int K[3] = {i, j, k};
        const size_t id = cid(g, i, j, k);
        T div = T(0);
        for (int d = 0; d < g.ndim; ++d) {
            const T lo = (UNIF ? Lc : L.p[d][id]) * ub.p[d][id];
            T up = T(0);
            if (K[d] + 1 < n[d] || per[d]) {
                int r[3] = {i, j, k};
                r[d] = K[d] + 1 < n[d] ? K[d] + 1 : 0;
                const size_t iu = cid(g, r[0], r[1], r[2]);
                up = (UNIF ? Lc : L.p[d][iu]) * ub.p[d][iu];
            }
            div += up - lo;
        }
        rhs[id] = (pbar ? pbar[id] : T(0)) + coef * div;
    }
}

// gbar_d(K) = ubar_d(K) + (sbar(K - d) - sbar(K)) / coef on interior faces,
// Lbar_d(K) += (G p)_d(K) ((G sbar)_d(K) - coef ubar_d(K)).
template <typename T, bool UNIF>
__global__ __launch_bounds__(kBlock) void k_adj_proj_update(TileDev TL, Grid g, AdjPtrs<T> ub,
                                                            const T* __restrict__ sb,
                                                            const T* __restrict__ p, AdjPtrs<T> L,
                                                            T Lc, T coef, AdjPtrs<T> gb,
                                                            AdjPtrs<T> Lb) {
    const Span sp = tile_span(TL, g.n0, g.n1, g.n2);
    const int i = sp.i, j = sp.j;
    if (i >= g.n0 || j >= g.n1) return;
    const int n[3] = {g.n0, g.n1, g.n2};
    for (int k = sp.z0; k < sp.z1; ++k) {
        const int K[3] = {i, j, k};
        const size_t id = cid(g, i, j, k);
        for (int d = 0; d < g.ndim; ++d) {
            if (!interior(g, d, i, j, k)) {
                gb.p[d][id] = T(0);
                continue;
            }
            int r[3] = {i, j, k};
            r[d] = K[d] > 0 ? K[d] - 1 : n[d] - 1;
            const size_t il = cid(g, r[0], r[1], r[2]);
            const T u = ub.p[d][id];
            gb.p[d][id] = u + (sb[il] - sb[id]) / coef;
            if (!UNIF) Lb.p[d][id] += (p[id] - p[il]) * ((sb[id] - sb[il]) - coef * u);
        }
    }
}

// Outflow plane of the projection adjoint and the exit-flux balance: gout =
// fout_bar + uout_bar + sbar(n0-1)/coef (fout_bar on entry holds what BDIM
// read from the balanced plane), then fout_bar = gout - mean(gout).  One
// workgroup.
template <typename T>
__global__ __launch_bounds__(1024) void k_adj_plane_proj(Grid g, const T* __restrict__ uoutb,
                                                         const T* __restrict__ sb, T coef,
                                                         T* __restrict__ foutb) {
    __shared__ double lds[32];
    const int P = g.n1 * g.n2;
    double s = 0.0;
    for (int q = threadIdx.x; q < P; q += blockDim.x) {
        const int j = q % g.n1, k = q / g.n1;
        const T v = foutb[q] + uoutb[q] + sb[cid(g, g.n0 - 1, j, k)] / coef;
        foutb[q] = v;
        s += double(v);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = s;
    __syncthreads();
    double tot = 0.0;
    for (int w = 0; w < int(blockDim.x + 63) / 64; ++w) tot += lds[w];
    const T mean = T(tot / double(P));
    for (int q = threadIdx.x; q < P; q += blockDim.x) foutb[q] -= mean;
}

template <typename T>
__global__ __launch_bounds__(1024) void k_adj_plane_stage(Grid g, const T* __restrict__ foutb, T wb,
                                                          T adt, T Ux, T* baseb, T* eoutb,
                                                          T* __restrict__ ebx) {
    // baseb and eoutb may be the same array (the predictor's base and
    // evaluation planes are both u^n), so they carry no restrict qualifier.
    const int P = g.n1 * g.n2;
    for (int q = threadIdx.x; q < P; q += blockDim.x) {
        const int j = q % g.n1, k = q / g.n1;
        const T fb = foutb[q];
        baseb[q] += wb * fb;
        const T Rb = adt * fb;         // R_out = -Ux (e_out - e_x(n0-1))
        eoutb[q] += -Ux * Rb;
        ebx[cid(g, g.n0 - 1, j, k)] += Ux * Rb;
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_adj_axpy(TileDev TL, Grid g, AdjPtrs<T> x, T alpha,
                                                     AdjPtrs<T> y, int accumulate) {
    const Span sp = tile_span(TL, g.n0, g.n1, g.n2);
    const int i = sp.i, j = sp.j;
    if (i >= g.n0 || j >= g.n1) return;
    for (int k = sp.z0; k < sp.z1; ++k) {
        const size_t id = cid(g, i, j, k);
        for (int c = 0; c < g.ndim; ++c) {
            if (!interior(g, c, i, j, k)) {
                y.p[c][id] = T(0);
                continue;
            }
            const T v = alpha * x.p[c][id];
            y.p[c][id] = accumulate ? y.p[c][id] + v : v;
        }
    }
}

// y += x over n cells (grid-stride).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_cells_add(size_t n, const T* __restrict__ x,
                                                      T* __restrict__ y) {
    for (size_t q = size_t(blockIdx.x) * kBlock + threadIdx.x; q < n; q += size_t(gridDim.x) * kBlock)
        y[q] += x[q];
}

// Face geometry for the parameter chain rule: signed distance d, unit normal
// n and distance rho to the centre, at the centre of the lower c-face of cell
// (i, j, k) (c < 0: the cell centre).
__device__ __forceinline__ void face_geom(const Grid& g, const BodyDev& b, int c, int i, int j, int k,
                                          double& d, double n[3], double& rho) {
    double x[3] = {i + 0.5, j + 0.5, k + 0.5};
    if (c >= 0) x[c] -= 0.5;
    double r2 = 0.0;
    double rel[3] = {0.0, 0.0, 0.0};
    for (int e = 0; e < g.ndim; ++e) {
        rel[e] = x[e] - b.centre[e];
        r2 += rel[e] * rel[e];
    }
    rho = sqrt(r2);
    d = rho - b.radius;
    for (int e = 0; e < 3; ++e) n[e] = (rho > 0.0 && e < g.ndim) ? rel[e] / rho : 0.0;
}

__device__ __forceinline__ double kern(double d, double eps) {
    const double r = d / eps;
    return fabs(r) < 1.0 ? (1.0 + cos(3.14159265358979323846 * r)) / (2.0 * eps) : 0.0;
}
__device__ __forceinline__ double kern_d(double d, double eps) {
    const double pi = 3.14159265358979323846;
    const double r = d / eps;
    return fabs(r) < 1.0 ? -pi * sin(pi * r) / (2.0 * eps * eps) : 0.0;
}
__device__ __forceinline__ double mu1_of(double d, double eps) {
    const double pi = 3.14159265358979323846;
    const double r = d / eps;
    if (fabs(r) >= 1.0) return 0.0;
    return eps * ((1.0 - r * r) / 4.0 - r * sin(pi * r) / (2.0 * pi) - (1.0 + cos(pi * r)) / (2.0 * pi * pi));
}

// theta = (R, c_x, c_y, c_z): d = rho - R, n = (x - c)/rho,
// dd/dR = -1, dd/dc_k = -n_k, dn_j/dc_k = -(delta_jk - n_j n_k)/rho,
// mu0' = K(d), mu1' = -d K(d); L = mu0 on interior faces.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_adj_params(TileDev TL, Grid g, BodyDev body, AdjPtrs<T> Lb,
                                                       AdjPtrs<T> m0b, AdjPtrs9<T> m1b,
                                                       double* __restrict__ partial) {
    __shared__ double lds[4][8];
    const Span sp = tile_span(TL, g.n0, g.n1, g.n2);
    const int i = sp.i, j = sp.j;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (i < g.n0 && j < g.n1) {
        for (int k = sp.z0; k < sp.z1; ++k) {
            const size_t id = cid(g, i, j, k);
            for (int c = 0; c < g.ndim; ++c) {
                double a0 = double(m0b.p[c][id]);
                if (interior(g, c, i, j, k)) a0 += double(Lb.p[c][id]);
                double a1[3] = {0.0, 0.0, 0.0};
                for (int e = 0; e < g.ndim; ++e) a1[e] = double(m1b.p[3 * c + e][id]);
                Lb.p[c][id] = T(0);
                m0b.p[c][id] = T(0);
                for (int e = 0; e < 3; ++e) m1b.p[3 * c + e][id] = T(0);
                if (a0 == 0.0 && a1[0] == 0.0 && a1[1] == 0.0 && a1[2] == 0.0) continue;
                double d, n[3], rho;
                face_geom(g, body, c, i, j, k, d, n, rho);
                const double K = kern(d, body.eps);
                const double m1 = mu1_of(d, body.eps);
                const double m1p = -d * K;
                double an = 0.0;  // sum_j a1_j n_j
                for (int e = 0; e < g.ndim; ++e) an += a1[e] * n[e];
                // dR
                acc[0] += -(a0 * K + an * m1p);
                // dc_k
                for (int kk = 0; kk < g.ndim; ++kk) {
                    double v = -(a0 * K + an * m1p) * n[kk];
                    if (rho > 0.0) v += -m1 * (a1[kk] - an * n[kk]) / rho;
                    acc[1 + kk] += v;
                }
            }
        }
    }
    // four deterministic block sums
    for (int q = 0; q < 4; ++q) {
        double v = acc[q];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if ((threadIdx.x & 63) == 0) lds[q][threadIdx.x >> 6] = v;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        double s = 0.0;
        for (int w = 0; w < (kBlock >> 6); ++w) s += lds[threadIdx.x][w];
        partial[4 * block_linear() + threadIdx.x] = s;
    }
}

template <typename T>
__device__ __forceinline__ bool active_cell(const Grid& g, T* const* L, int i, int j, int k) {
    const int n[3] = {g.n0, g.n1, g.n2};
    const int per[3] = {g.per0, g.per1, g.per2};
    const int K[3] = {i, j, k};
    const size_t id = cid(g, i, j, k);
    T D = T(0);
    for (int d = 0; d < g.ndim; ++d) {
        D += L[d][id];
        if (K[d] + 1 < n[d] || per[d]) {
            int r[3] = {i, j, k};
            r[d] = K[d] + 1 < n[d] ? K[d] + 1 : 0;
            D += L[d][cid(g, r[0], r[1], r[2])];
        }
    }
    return D > T(0);
}

// Partial sums of (w, p, p w, 1) over active cells, w = n_x K(d) at the cell centre.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_drag_sums(TileDev TL, Grid g, BodyDev body,
                                                      const T* __restrict__ p, AdjPtrs<T> L,
                                                      double* __restrict__ partial) {
    __shared__ double lds[4][8];
    const Span sp = tile_span(TL, g.n0, g.n1, g.n2);
    const int i = sp.i, j = sp.j;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (i < g.n0 && j < g.n1) {
        for (int k = sp.z0; k < sp.z1; ++k) {
            if (!active_cell<T>(g, L.p, i, j, k)) continue;
            double d, n[3], rho;
            face_geom(g, body, -1, i, j, k, d, n, rho);
            const double w = n[0] * kern(d, body.eps);
            const double pv = double(p[cid(g, i, j, k)]);
            acc[0] += w;
            acc[1] += pv;
            acc[2] += pv * w;
            acc[3] += 1.0;
        }
    }
    for (int q = 0; q < 4; ++q) {
        double v = acc[q];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if ((threadIdx.x & 63) == 0) lds[q][threadIdx.x >> 6] = v;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        double s = 0.0;
        for (int w = 0; w < (kBlock >> 6); ++w) s += lds[threadIdx.x][w];
        partial[4 * block_linear() + threadIdx.x] = s;
    }
}

// Drag F = -sum_active (p - pmean)(w - wmean) = -sum_active p (w - wmean).
// pbar = -weight (w - wmean) on active cells; theta-gradient partial sums of
// -weight sum_active (p - pmean) dw/dtheta with dw/dR = -n_x K'(d),
// dw/dc_k = dn_x/dc_k K(d) - n_x K'(d) n_k.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_drag_adj(TileDev TL, Grid g, BodyDev body,
                                                     const T* __restrict__ p, AdjPtrs<T> L,
                                                     double weight, const double* __restrict__ means,
                                                     T* __restrict__ pbar,
                                                     double* __restrict__ partial) {
    __shared__ double lds[4][8];
    const Span sp = tile_span(TL, g.n0, g.n1, g.n2);
    const int i = sp.i, j = sp.j;
    const double wmean = means[0], pmean = means[1];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (i < g.n0 && j < g.n1) {
        for (int k = sp.z0; k < sp.z1; ++k) {
            const size_t id = cid(g, i, j, k);
            if (!active_cell<T>(g, L.p, i, j, k)) {
                pbar[id] = T(0);
                continue;
            }
            double d, n[3], rho;
            face_geom(g, body, -1, i, j, k, d, n, rho);
            const double K = kern(d, body.eps), Kp = kern_d(d, body.eps);
            pbar[id] = T(-weight * (n[0] * K - wmean));
            const double q = -weight * (double(p[id]) - pmean);
            acc[0] += q * (-n[0] * Kp);
            for (int kk = 0; kk < g.ndim; ++kk) {
                const double dn = rho > 0.0 ? -((kk == 0 ? 1.0 : 0.0) - n[0] * n[kk]) / rho : 0.0;
                acc[1 + kk] += q * (dn * K - n[0] * Kp * n[kk]);
            }
        }
    }
    for (int qq = 0; qq < 4; ++qq) {
        double v = acc[qq];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if ((threadIdx.x & 63) == 0) lds[qq][threadIdx.x >> 6] = v;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        double s = 0.0;
        for (int w = 0; w < (kBlock >> 6); ++w) s += lds[threadIdx.x][w];
        partial[4 * block_linear() + threadIdx.x] = s;
    }
}

// out[c] = sum over slots of partial[slot*ncomp + c] (slot order).  One block.
__global__ __launch_bounds__(1024) void k_reduce_cols(const double* __restrict__ partial,
                                                      size_t nslots, int ncomp,
                                                      double* __restrict__ out) {
    __shared__ double lds[1024];
    for (int c = 0; c < ncomp; ++c) {
        double s = 0.0;
        for (size_t q = threadIdx.x; q < nslots; q += blockDim.x) s += partial[q * ncomp + c];
        lds[threadIdx.x] = s;
        __syncthreads();
        for (int w = blockDim.x / 2; w > 0; w >>= 1) {
            if (threadIdx.x < w) lds[threadIdx.x] += lds[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[c] = lds[0];
        __syncthreads();
    }
}

// ------------------------------------------------------------- launchers

template <typename T>
wl_status adj_flux(const VelField<T>& E, T* const Rbar[3], T nu, const PadField<T>& out, bool allper,
                   hipStream_t s) {
    const Launch ln = launch_for(out.pg.P0, out.pg.P1, out.pg.P2);
    AdjPtrs<T> R{{Rbar[0], Rbar[1], Rbar[2]}};
    if (allper)
        k_adj_flux<T, true><<<ln.grid, ln.block, 0, s>>>(ln.td, E, R, nu, out);
    else
        k_adj_flux<T, false><<<ln.grid, ln.block, 0, s>>>(ln.td, E, R, nu, out);
    WL_CHECK_LAUNCH();
    return WL_OK;
}

template <typename T>
wl_status adj_bdim(const Grid& g, T* const gbar[3], T* const mu0[3], T* const mu1n[9],
                   const PadField<T>& out, hipStream_t s) {
    const Launch ln = launch_for(out.pg.P0, out.pg.P1, out.pg.P2);
    AdjPtrs<T> gb{{gbar[0], gbar[1], gbar[2]}}, m0{{mu0[0], mu0[1], mu0[2]}};
    AdjPtrs9<T> m1;
    for (int q = 0; q < 9; ++q) m1.p[q] = mu1n[q];
    k_adj_bdim<T><<<ln.grid, ln.block, 0, s>>>(ln.td, g, gb, m0, m1, out);
    WL_CHECK_LAUNCH();
    return WL_OK;
}

template <typename T>
wl_status adj_bdim_param(const VelField<T>& F, T* const gbar[3], T* const mu0b[3], T* const mu1nb[9],
                         hipStream_t s) {
    const Launch ln = launch_for(F.g.n0, F.g.n1, F.g.n2);
    AdjPtrs<T> gb{{gbar[0], gbar[1], gbar[2]}}, m0{{mu0b[0], mu0b[1], mu0b[2]}};
    AdjPtrs9<T> m1;
    for (int q = 0; q < 9; ++q) m1.p[q] = mu1nb[q];
    k_adj_bdim_param<T><<<ln.grid, ln.block, 0, s>>>(ln.td, F, gb, m0, m1);
    WL_CHECK_LAUNCH();
    return WL_OK;
}

template <typename T>
wl_status adj_fold(const VelField<T>& geom, const PadField<T>& pad, T* const acc[3], T* acc_out,
                   hipStream_t s) {
    const Launch ln = launch_for(geom.g.n0, geom.g.n1, geom.g.n2);
    AdjPtrs<T> a{{acc[0], acc[1], acc[2]}};
    k_adj_fold<T><<<ln.grid, ln.block, 0, s>>>(ln.td, geom, pad, a, acc_out);
    WL_CHECK_LAUNCH();
    return WL_OK;
}

template <typename T>
wl_status adj_proj_rhs(const Grid& g, const T* pbar, T* const ubar[3], T* const L[3], T Lc, bool unif,
                       double coef, T* rhs, hipStream_t s) {
    const Launch ln = launch_for(g.n0, g.n1, g.n2);
    AdjPtrs<T> ub{{ubar[0], ubar[1], ubar[2]}}, LL{{L[0], L[1], L[2]}};
    if (unif)
        k_adj_proj_rhs<T, true><<<ln.grid, ln.block, 0, s>>>(ln.td, g, pbar, ub, LL, Lc, T(coef), rhs);
    else
        k_adj_proj_rhs<T, false><<<ln.grid, ln.block, 0, s>>>(ln.td, g, pbar, ub, LL, Lc, T(coef), rhs);
    WL_CHECK_LAUNCH();
    return WL_OK;
}

template <typename T>
wl_status adj_proj_update(const Grid& g, T* const ubar[3], const T* sbar, const T* p, T* const L[3],
                          T Lc, bool unif, double coef, T* const gbar[3], T* const Lbar[3],
                          hipStream_t s) {
    const Launch ln = launch_for(g.n0, g.n1, g.n2);
    AdjPtrs<T> ub{{ubar[0], ubar[1], ubar[2]}}, LL{{L[0], L[1], L[2]}}, gb{{gbar[0], gbar[1], gbar[2]}},
        Lb{{Lbar[0], Lbar[1], Lbar[2]}};
    if (unif)
        k_adj_proj_update<T, true><<<ln.grid, ln.block, 0, s>>>(ln.td, g, ub, sbar, p, LL, Lc, T(coef),
                                                               gb, Lb);
    else
        k_adj_proj_update<T, false><<<ln.grid, ln.block, 0, s>>>(ln.td, g, ub, sbar, p, LL, Lc,
                                                                T(coef), gb, Lb);
    WL_CHECK_LAUNCH();
    return WL_OK;
}

template <typename T>
wl_status adj_plane_proj(const Grid& g, const T* uoutb, const T* sbar, double coef, T* foutb,
                         hipStream_t s) {
    k_adj_plane_proj<T><<<1, 1024, 0, s>>>(g, uoutb, sbar, T(coef), foutb);
    WL_CHECK_LAUNCH();
    return WL_OK;
}

template <typename T>
wl_status adj_plane_stage(const Grid& g, const T* foutb, double wb, double adt, T Ux, T* baseb,
                          T* eoutb, T* ebx, hipStream_t s) {
    k_adj_plane_stage<T><<<1, 1024, 0, s>>>(g, foutb, T(wb), T(adt), Ux, baseb, eoutb, ebx);
    WL_CHECK_LAUNCH();
    return WL_OK;
}

template <typename T>
wl_status adj_faces_axpy(const Grid& g, T* const x[3], double alpha, T* const y[3], bool accumulate,
                         hipStream_t s) {
    const Launch ln = launch_for(g.n0, g.n1, g.n2);
    AdjPtrs<T> xx{{x[0], x[1], x[2]}}, yy{{y[0], y[1], y[2]}};
    k_adj_axpy<T><<<ln.grid, ln.block, 0, s>>>(ln.td, g, xx, T(alpha), yy, accumulate ? 1 : 0);
    WL_CHECK_LAUNCH();
    return WL_OK;
}

template <typename T>
wl_status adj_cells_add(size_t n, const T* x, T* y, hipStream_t s) {
    if (n == 0) return WL_OK;
    const size_t want = (n + kBlock - 1) / kBlock;
    const unsigned blocks = unsigned(want < 4096 ? want : 4096);
    k_cells_add<T><<<blocks, kBlock, 0, s>>>(n, x, y);
    WL_CHECK_LAUNCH();
    return WL_OK;
}

template <typename T>
wl_status adj_params(const Grid& g, const BodyDev& body, T* const Lb[3], T* const mu0b[3],
                     T* const mu1nb[9], double* partial, hipStream_t s) {
    const Launch ln = launch_for(g.n0, g.n1, g.n2);
    AdjPtrs<T> L{{Lb[0], Lb[1], Lb[2]}}, m0{{mu0b[0], mu0b[1], mu0b[2]}};
    AdjPtrs9<T> m1;
    for (int q = 0; q < 9; ++q) m1.p[q] = mu1nb[q];
    k_adj_params<T><<<ln.grid, ln.block, 0, s>>>(ln.td, g, body, L, m0, m1, partial);
    WL_CHECK_LAUNCH();
    return WL_OK;
}

template <typename T>
wl_status drag_sums(const Grid& g, const BodyDev& body, const T* p, T* const L[3], double* partial,
                    hipStream_t s) {
    const Launch ln = launch_for(g.n0, g.n1, g.n2);
    AdjPtrs<T> LL{{L[0], L[1], L[2]}};
    k_drag_sums<T><<<ln.grid, ln.block, 0, s>>>(ln.td, g, body, p, LL, partial);
    WL_CHECK_LAUNCH();
    return WL_OK;
}

template <typename T>
wl_status drag_adj(const Grid& g, const BodyDev& body, const T* p, T* const L[3], double weight,
                   const double* means, T* pbar, double* partial, hipStream_t s) {
    const Launch ln = launch_for(g.n0, g.n1, g.n2);
    AdjPtrs<T> LL{{L[0], L[1], L[2]}};
    k_drag_adj<T><<<ln.grid, ln.block, 0, s>>>(ln.td, g, body, p, LL, weight, means, pbar, partial);
    WL_CHECK_LAUNCH();
    return WL_OK;
}

wl_status reduce_cols(const double* partial, size_t nslots, int ncomp, double* out, hipStream_t s) {
    k_reduce_cols<<<1, 1024, 0, s>>>(partial, nslots, ncomp, out);
    WL_CHECK_LAUNCH();
    return WL_OK;
}

#define WL_INST(T)                                                                                  \
    template wl_status adj_flux<T>(const VelField<T>&, T* const*, T, const PadField<T>&, bool,      \
                                   hipStream_t);                                                    \
    template wl_status adj_bdim<T>(const Grid&, T* const*, T* const*, T* const*, const PadField<T>&, \
                                   hipStream_t);                                                    \
    template wl_status adj_bdim_param<T>(const VelField<T>&, T* const*, T* const*, T* const*,        \
                                         hipStream_t);                                              \
    template wl_status adj_fold<T>(const VelField<T>&, const PadField<T>&, T* const*, T*,            \
                                   hipStream_t);                                                    \
    template wl_status adj_proj_rhs<T>(const Grid&, const T*, T* const*, T* const*, T, bool, double, \
                                       T*, hipStream_t);                                            \
    template wl_status adj_proj_update<T>(const Grid&, T* const*, const T*, const T*, T* const*, T,  \
                                          bool, double, T* const*, T* const*, hipStream_t);         \
    template wl_status adj_plane_proj<T>(const Grid&, const T*, const T*, double, T*, hipStream_t);  \
    template wl_status adj_plane_stage<T>(const Grid&, const T*, double, double, T, T*, T*, T*,     \
                                          hipStream_t);                                             \
    template wl_status adj_faces_axpy<T>(const Grid&, T* const*, double, T* const*, bool,            \
                                         hipStream_t);                                              \
    template wl_status adj_cells_add<T>(size_t, const T*, T*, hipStream_t);                          \
    template wl_status adj_params<T>(const Grid&, const BodyDev&, T* const*, T* const*, T* const*,   \
                                     double*, hipStream_t);                                         \
    template wl_status drag_sums<T>(const Grid&, const BodyDev&, const T*, T* const*, double*,       \
                                    hipStream_t);                                                   \
    template wl_status drag_adj<T>(const Grid&, const BodyDev&, const T*, T* const*, double,         \
                                   const double*, T*, double*, hipStream_t);
WL_INST(float)
WL_INST(double)
#undef WL_INST

}  // namespace wl
