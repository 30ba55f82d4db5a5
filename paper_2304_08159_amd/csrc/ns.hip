// Navier-Stokes step kernels: geometry measure (BDIM moments and Poisson
// coefficients), CFL time step, third-order limited convection-diffusion with
// the Heun stage update, BDIM blend, outflow plane with exit-flux balance,
// divergence and the pressure-gradient projection.
//
// Paper Sec. 2 fixes the method (third-order finite volume, explicit adaptive
// time stepping, implicit LES, BDIM on velocity and pressure matrix, the
// gradient loop u[I,i] -= coeff[I,i]*(p[I]-p[I-del(i)]) fused over i);
// Sec. 3 / Table 2 name the routines convdiff!, BDIM!, BC!, project!, CFL!.
// Constants the paper leaves open follow the readings stated in the headers:
// kappa = 1/3 interpolant bounded by the Koren limiter (median form), cosine
// BDIM kernel of half-width eps, Heun stages with projection factor c = 1 and
// c = 1/2, CFL from the per-cell outflow velocity plus 2 d nu.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <type_traits>

#include "wl_device.h"
#include "wl_jacobi.h"
#include "wl_ns.h"
#include "wl_vel.h"
#include "wl_nsdev.h"

namespace wl {

// Stage update of every interior face of cell (i,j,k):
//   PRED: f = u_e + dt R(u_e)          CORR: f = (u_n + u_e + dt R(u_e)) / 2
// with R_c = -sum_d [F_cd(I + delta_d) - F_cd(I)].  Domain-boundary faces take
// their boundary value (U_c at an inflow, 0 at a wall).
template <typename T, bool ALLPER, bool CORR>
__global__ __launch_bounds__(kBlock) void k_momentum(TileDev TL, VelField<T> E, const T* __restrict__ un0,
                                                     const T* __restrict__ un1,
                                                     const T* __restrict__ un2,
                                                     T* __restrict__ f0, T* __restrict__ f1,
                                                     T* __restrict__ f2, T nu,
                                                     const double* __restrict__ dt_dev) {
    const Grid& g = E.g;
    const Span sp = tile_span(TL, g.n0, g.n1, g.n2);
    const int i = sp.i, j = sp.j;
    if (i >= g.n0 || j >= g.n1) return;
    for (int k = sp.z0; k < sp.z1; ++k) {
    const size_t id = cid(g, i, j, k);
    const T dt = T(*dt_dev);
    const int coord[3] = {i, j, k};
    const int per[3] = {g.per0, g.per1, g.per2};
    const T* un[3] = {un0, un1, un2};
    T* fo[3] = {f0, f1, f2};
    for (int c = 0; c < g.ndim; ++c) {
        if (!per[c] && coord[c] == 0) {
            fo[c][id] = (E.bclo[c] == WL_BC_INFLOW) ? E.U[c] : T(0);
            continue;
        }
        T R = T(0);
        for (int d = 0; d < g.ndim; ++d) {
            const T Flo = face_flux<T, ALLPER>(E, c, d, i, j, k, nu);
            const T Fhi = face_flux<T, ALLPER>(E, c, d, i + (d == 0), j + (d == 1), k + (d == 2), nu);
            R -= Fhi - Flo;
        }
        const T ue = E.u[c][id];
        fo[c][id] = CORR ? T(0.5) * (un[c][id] + ue + dt * R) : ue + dt * R;
    }
    }
}

// ---------------------------------------------------------------------------
// LDS-tiled convection-diffusion for FP32 3D grids.  A block of 512 threads
// owns a 64 x 8 column of cells and marches through a chunk of z planes.  Planes z-1, z,
// z+1 of all three components (with a two-cell x/y halo) sit in a 3-plane LDS
// ring; the thread's own column of planes z-2 .. z+2 is kept in registers for
// the z stencil.  Fetched planes sit in three register sets indexed by plane
// modulo 3, the loop unrolled three times so that no copy waits on a load;
// the non-projecting kernels fetch two planes ahead, the projecting corrector
// one.  Every face flux
// is evaluated once: a thread computes the lower x, y and z faces of its cell;
// the tile's extra x column goes to wave 1 and its extra y row to wave 2, and
// the upper x / y fluxes a cell needs are read from LDS, the upper z flux is
// kept for the next plane.  Fluxes are evaluated doubled (sum of the two
// advecting velocities instead of their mean, 2 nu) and the step uses dt/2:
// scaling by two is exact, so this changes no bit of the result.  Block ids
// are remapped so that each XCD (blocks are dealt round-robin to the 8 XCDs)
// walks a contiguous range of tiles and shares halo rows through its L2.
namespace {
constexpr int MT_X = 64, MT_Y = 8, MT_T = MT_X * MT_Y;  // MT_T threads per block
constexpr int MT_LX = MT_X + 4, MT_LY = MT_Y + 4, MT_PL = MT_LX * MT_LY;
constexpr int MT_NP = 3;
constexpr int MT_HALO = MT_PL - MT_X * MT_Y;
constexpr int MT_LOADS = 1 + (MT_HALO + MT_T - 1) / MT_T;
}  // namespace

__device__ __forceinline__ int wrapi(int a, int n) {
    int r = a % n;
    return r < 0 ? r + n : r;
}

// LDS position (Y * MT_LX + X) of load slot k of thread t, -1 if unused.
// Slot 0 is the thread's own cell; the halo (rows 0, 1 and MT_LY-2, MT_LY-1
// in full, then columns 0, 1, MT_LX-2, MT_LX-1 of the tile rows) is dealt
// out over the following slots in that order, so consecutive threads read
// consecutive x.
__device__ __forceinline__ int mt_pos(int t, int k) {
    if (k == 0) return ((t >> 6) + 2) * MT_LX + (t & 63) + 2;
    const int h = t + (k - 1) * MT_T;
    if (h >= MT_HALO) return -1;
    if (h < 4 * MT_LX) {
        const int r = h / MT_LX, x = h - r * MT_LX;
        return (r < 2 ? r : r + MT_Y) * MT_LX + x;
    }
    const int q = h - 4 * MT_LX, r = q >> 2, c = q & 3;
    return (r + 2) * MT_LX + (c < 2 ? c : MT_X + c);
}

// The velocity ghost rule (vget) evaluated inline for the halo of a tile at a
// domain face:
// the first coordinate outside the grid (x, then y, then z, after the
// periodic wraps) picks the branch of the rule, the others are clamped, and
// only that branch runs, so a tile at a face pays a few instructions per
// ghost slot instead of a call.
__device__ __forceinline__ float ghost_inl(const VelField<float>& V, int c, int px, int py, int pz) {
    // the grid and boundary fields pass through readfirstlane (they are
    // uniform): a per-lane choice between fields loaded from the kernel
    // argument would otherwise become a per-lane load from a private copy
    auto u_ = [](int v) { return __builtin_amdgcn_readfirstlane(v); };
    const int n0 = u_(V.g.n0), n1 = u_(V.g.n1), n2 = u_(V.g.n2);
    if (V.g.per0) px = px < 0 ? px + n0 : (px >= n0 ? px - n0 : px);
    if (V.g.per1) py = py < 0 ? py + n1 : (py >= n1 ? py - n1 : py);
    if (V.g.per2) pz = pz < 0 ? pz + n2 : (pz >= n2 ? pz - n2 : pz);
    const bool ox_ = px < 0 || px >= n0, oy_ = py < 0 || py >= n1;
    const int d = ox_ ? 0 : (oy_ ? 1 : 2);
    const int kk = d == 0 ? px : (d == 1 ? py : pz);
    const int m = d == 0 ? n0 : (d == 1 ? n1 : n2);
    const int cx = min(max(px, 0), n0 - 1), cy = min(max(py, 0), n1 - 1);
    const int cz = min(max(pz, 0), n2 - 1);
    auto at = [&](int idx) -> float {
        idx = min(max(idx, 0), m - 1);
        const int x = d == 0 ? idx : cx, y = d == 1 ? idx : cy, z = d == 2 ? idx : cz;
        return V.u[c][size_t(x) + size_t(n0) * (size_t(y) + size_t(n1) * size_t(z))];
    };
    const int l0 = u_(V.bclo[0]), l1 = u_(V.bclo[1]), l2 = u_(V.bclo[2]);
    const int h0 = u_(V.bchi[0]), h1 = u_(V.bchi[1]), h2 = u_(V.bchi[2]);
    const int blo = d == 0 ? l0 : (d == 1 ? l1 : l2);
    const int bhi = d == 0 ? h0 : (d == 1 ? h1 : h2);
    if (kk < 0) {
        if (blo == WL_BC_INFLOW) return V.U[c];
        if (c == d) {
            const int mir = -kk;
            return -at(mir < m ? mir : 0);
        }
        const int mir = -1 - kk;
        return at(mir < m - 1 ? mir : m - 1);
    }
    if (c == d) {
        if (bhi == WL_BC_OUTFLOW) return V.uout[cy + size_t(n1) * cz];
        if (kk == m) return 0.f;
        return -at(m - 1 > 0 ? m - 1 : 0);
    }
    if (bhi == WL_BC_OUTFLOW) return at(m - 1);
    if (kk == m) return at(m - 1);
    return at(m - 2 > 0 ? m - 2 : 0);
}

template <bool ALLPER>
__device__ __forceinline__ float tile_fetch(const VelField<float>& V, int c, int gx, int gy, int gz) {
    const Grid& g = V.g;
    if (ALLPER) return V.u[c][cid(g, wrapi(gx, g.n0), wrapi(gy, g.n1), wrapi(gz, g.n2))];
    if (gx >= 0 && gx < g.n0 && gy >= 0 && gy < g.n1 && gz >= 0 && gz < g.n2)
        return V.u[c][cid(g, gx, gy, gz)];
    return ghost_inl(V, c, gx, gy, gz);
}

// Twice the flux through a face of a momentum control volume: s is the sum of
// the two advecting velocities on the face, nu2 = 2 nu; the face value is the
// kappa = 1/3 upwind-biased interpolant bounded by the median-form limiter.
__device__ __forceinline__ float flux2(float um2, float um1, float u0, float up1, float s,
                                       float nu2) {
    const bool pos = s >= 0.f;
    const float cu = pos ? um1 : u0;
    const float bd = pos ? u0 : um1;
    const float au = pos ? um2 : up1;
    const float phik = fmaf(5.f, cu, fmaf(2.f, bd, -au)) * (1.f / 6.f);
    const float phi = med3(phik, cu, med3(fmaf(2.f, cu, -au), cu, bd));
    return fmaf(s, phi, -(nu2 * (u0 - um1)));
}

// A fetched plane: the velocity at the thread's load slots and, with PROJ,
// the pressure there and at the slots' x-1 and y-1 neighbours.
struct MtPlane {
    float u[3][MT_LOADS];
    float p[MT_LOADS], pxm[MT_LOADS], pym[MT_LOADS];
};

// PROJ (periodic, uniform coefficients): E holds the predictor's stage field
// u* and pp its pressure; the kernel evaluates the projected field
// u1 = u* - dt Lc grad(pp) as it fills its tile (the predictor's projection is
// then never stored), with the same rounding as k_project.
template <bool ALLPER, bool CORR, bool PROJ, bool BUF>
__device__ __forceinline__ void momentum_tile(const VelField<float>& E, const float* __restrict__ un0,
                                              const float* __restrict__ un1,
                                              const float* __restrict__ un2, float* __restrict__ f0,
                                              float* __restrict__ f1, float* __restrict__ f2,
                                              float nu, const double* __restrict__ dt_dev, TileMap tm,
                                              const float* __restrict__ pp, float Lc) {
    static_assert(!PROJ || ALLPER, "the fused projection assumes periodic wrap");
    static_assert(!BUF || ALLPER, "buffer addressing assumes periodic wrap");
    __shared__ float sU[3][MT_NP][MT_PL];
    __shared__ float sFx[3][MT_Y][MT_X + 1];
    __shared__ float sFy[3][MT_Y + 1][MT_X];
    const Grid& g = E.g;
    unsigned b = blockIdx.x;
    if (tm.remap) b = (b & 7u) * (tm.nblocks >> 3) + (b >> 3);
    const int tix = int(b % unsigned(tm.tiles_x));
    b /= unsigned(tm.tiles_x);
    const int tiy = int(b % unsigned(tm.tiles_y));
    const int ch = int(b / unsigned(tm.tiles_y));
    const int x0 = tix * MT_X, y0 = tiy * MT_Y, z0 = ch * tm.zc;
    const int z1 = min(z0 + tm.zc, g.n2);
    const int t = threadIdx.x, tx = t & 63, ty = t >> 6;
    const int lx = tx + 2, ly = ty + 2, own = ly * MT_LX + lx;
    const float hdt = 0.5f * float(*dt_dev);
    const float cl = float(*dt_dev) * Lc;  // c dt L of the predictor projection (c = 1)
    const float nu2 = 2.f * nu;
    const int gx = x0 + tx, gy = y0 + ty;
    const bool inside = gx < g.n0 && gy < g.n1;
    const float* un[3] = {un0, un1, un2};
    float* fo[3] = {f0, f1, f2};
    // extra flux items: the tile's upper x column (wave 1) and upper y row (wave 2)
    const bool xtra_x = t >= 64 && t < 64 + MT_Y;
    const bool xtra_y = t >= 128 && t < 192;
    const int xx_pos = (t - 64 + 2) * MT_LX + MT_X + 2;  // (X = 66, Y = row + 2)
    const int xy_pos = (MT_Y + 2) * MT_LX + (t - 128) + 2;
    // load slots; with periodic wrap the x/y part of each global offset is
    // fixed for the whole column and computed once
    int lpos[MT_LOADS];
    unsigned offxy[MT_LOADS], offxm[MT_LOADS], offym[MT_LOADS];
    int pxs[MT_LOADS], pys[MT_LOADS];
    bool inxy[MT_LOADS];  // x/y position inside the grid (no ghost rule needed)
#pragma unroll
    for (int k = 0; k < MT_LOADS; ++k) {
        lpos[k] = mt_pos(t, k);
        const int p = lpos[k] < 0 ? 0 : lpos[k];
        const int Y = p / MT_LX;
        pxs[k] = x0 - 2 + (p - Y * MT_LX);
        pys[k] = y0 - 2 + Y;
        inxy[k] = pxs[k] >= 0 && pxs[k] < g.n0 && pys[k] >= 0 && pys[k] < g.n1;
        offxy[k] = ALLPER ? unsigned(wrapi(pxs[k], g.n0)) + unsigned(g.n0) * unsigned(wrapi(pys[k], g.n1))
                          : (inxy[k] ? unsigned(pxs[k]) + unsigned(g.n0) * unsigned(pys[k]) : 0u);
        offxm[k] = PROJ ? unsigned(wrapi(pxs[k] - 1, g.n0)) + unsigned(g.n0) * unsigned(wrapi(pys[k], g.n1))
                        : 0u;
        offym[k] = PROJ ? unsigned(wrapi(pxs[k], g.n0)) + unsigned(g.n0) * unsigned(wrapi(pys[k] - 1, g.n1))
                        : 0u;
    }
    const unsigned plane = unsigned(g.n0) * unsigned(g.n1);
    // BUF (periodic, arrays below 4 GiB): loads and stores go through buffer
    // descriptors with the plane's byte offset in a scalar register and the
    // thread's fixed column offset in a vector register, so that no per-plane
    // address arithmetic is repeated on the vector ALU
    const int nbytes = BUF ? int(unsigned(size_t(plane) * unsigned(g.n2) * 4u)) : 0;
    auto rsrc = [&](const float* q) {
        return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(q), 0, nbytes, 0x00020000);
    };
    const auto dU0 = rsrc(E.u[0]), dU1 = rsrc(E.u[1]), dU2 = rsrc(E.u[2]);
    const auto dN0 = rsrc(un0), dN1 = rsrc(un1), dN2 = rsrc(un2);
    const auto dF0 = rsrc(f0), dF1 = rsrc(f1), dF2 = rsrc(f2);
    const auto dP = rsrc(pp);
    // the plane offsets are uniform over the block; readfirstlane says so to
    // the compiler, which otherwise may loop over "distinct" lanes' values
    auto uni = [](unsigned v) { return int(__builtin_amdgcn_readfirstlane(int(v))); };
    auto bld = [&](const __amdgpu_buffer_rsrc_t& rs, unsigned voff, unsigned soff) -> float {
        return __builtin_bit_cast(float,
                                  __builtin_amdgcn_raw_buffer_load_b32(rs, int(voff), uni(soff), 0));
    };
    auto ldu = [&](int c, unsigned col, unsigned pl) -> float {
        if constexpr (BUF)
            return bld(c == 0 ? dU0 : (c == 1 ? dU1 : dU2), col * 4u, pl * 4u);
        else
            return E.u[c][pl + col];
    };
    auto ldn = [&](int c, unsigned col, unsigned pl) -> float {
        if constexpr (BUF)
            return bld(c == 0 ? dN0 : (c == 1 ? dN1 : dN2), col * 4u, pl * 4u);
        else
            return un[c][pl + col];
    };
    auto ldp = [&](unsigned col, unsigned pl) -> float {
        if constexpr (BUF)
            return bld(dP, col * 4u, pl * 4u);
        else
            return pp[pl + col];
    };
    auto stf = [&](int c, unsigned col, unsigned pl, float v) {
        if constexpr (BUF)
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v),
                                                  c == 0 ? dF0 : (c == 1 ? dF1 : dF2),
                                                  int(col * 4u), uni(pl * 4u), 0);
        else
            fo[c][pl + col] = v;
    };
    auto fetch = [&](int zz, MtPlane& P) {
        float (&r)[3][MT_LOADS] = P.u;
        if (ALLPER) {
            const int gz = zz < 0 ? zz + g.n2 : (zz >= g.n2 ? zz - g.n2 : zz);
            const unsigned base = unsigned(gz) * plane;
            // without PROJ the loads are unconditional: an unused slot
            // (lpos < 0) reads the tile's corner, a valid address; no branch
            // around the loads keeps the wait counts exact, so waiting for
            // one plane never waits for the planes fetched after it
#pragma unroll
            for (int k = 0; k < MT_LOADS; ++k) {
                if (PROJ && lpos[k] < 0) continue;
#pragma unroll
                for (int c = 0; c < 3; ++c) r[c][k] = ldu(c, offxy[k], base);
                if (PROJ) {
                    P.p[k] = ldp(offxy[k], base);
                    P.pxm[k] = ldp(offxm[k], base);
                    P.pym[k] = ldp(offym[k], base);
                }
            }
        } else {
            // every slot first loads an address inside the grid (the plane
            // clamped in z, offset 0 for a position outside it), with no branch
            // around the loads; the slots outside the grid then take the ghost
            // rule, a branch no lane of an interior tile enters
            const bool zin = zz >= 0 && zz < g.n2;
            const unsigned base = unsigned(min(max(zz, 0), g.n2 - 1)) * plane;
#pragma unroll
            for (int k = 0; k < MT_LOADS; ++k) {
#pragma unroll
                for (int c = 0; c < 3; ++c) r[c][k] = E.u[c][base + offxy[k]];
            }
#pragma unroll
            for (int k = 0; k < MT_LOADS; ++k) {
                if (lpos[k] >= 0 && !(zin && inxy[k])) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) r[c][k] = ghost_inl(E, c, pxs[k], pys[k], zz);
                }
            }
        }
    };
    // LDS ring slot of plane z: (z - z0 + 1) mod 3 (plane z0 - 1 in slot 0);
    // register set of a fetched plane q: (q - z0) mod 3.  The plane loop is
    // unrolled three times, so both are constants inside it.
    // u* -> u1 on a fetched plane; pb: the pressure of the plane below at
    // the same slots
    auto project = [&](MtPlane& P, const float (&pb)[MT_LOADS]) {
#pragma unroll
        for (int k = 0; k < MT_LOADS; ++k)
            if (lpos[k] >= 0) {
                P.u[0][k] = proj_face(P.u[0][k], cl, P.p[k], P.pxm[k]);
                P.u[1][k] = proj_face(P.u[1][k], cl, P.p[k], P.pym[k]);
                P.u[2][k] = proj_face(P.u[2][k], cl, P.p[k], pb[k]);
            }
    };
    auto store = [&](int sl, const MtPlane& P) {
        const float (&r)[3][MT_LOADS] = P.u;
#pragma unroll
        for (int k = 0; k < MT_LOADS; ++k)
            if (lpos[k] >= 0)
#pragma unroll
                for (int c = 0; c < 3; ++c) sU[c][sl][lpos[k]] = r[c][k];
    };
    auto U = [&](int c, int sl, int p) -> float { return sU[c][sl][p]; };

    MtPlane PR[3];
    MtPlane& PA = PR[2];  // plane z0 - 1
    MtPlane& PB = PR[0];  // plane z0
    float wm2[3];
    fetch(z0 - 1, PA);
    fetch(z0, PB);
#pragma unroll
    for (int c = 0; c < 3; ++c) wm2[c] = tile_fetch<ALLPER>(E, c, gx, gy, z0 - 2);
    if (PROJ) {
        // plane z0 - 2: pressure at the slots (for plane z0 - 1) and the
        // projected own-column value
        const Grid& G = g;
        auto pat = [&](int x, int y, int z) {
            return pp[cid(G, wrapi(x, G.n0), wrapi(y, G.n1), wrapi(z, G.n2))];
        };
        const int gzm2 = wrapi(z0 - 2, g.n2);
        float pm2[MT_LOADS];
#pragma unroll
        for (int k = 0; k < MT_LOADS; ++k)
            pm2[k] = lpos[k] >= 0 ? pp[unsigned(gzm2) * plane + offxy[k]] : 0.f;
        const float po = pat(gx, gy, z0 - 2);
        wm2[0] = proj_face(wm2[0], cl, po, pat(gx - 1, gy, z0 - 2));
        wm2[1] = proj_face(wm2[1], cl, po, pat(gx, gy - 1, z0 - 2));
        wm2[2] = proj_face(wm2[2], cl, po, pat(gx, gy, z0 - 3));
        project(PA, pm2);
        project(PB, PA.p);
    }
    store(0, PA);
    store(1, PB);
    fetch(z0 + 1, PR[1]);
    if (PROJ) project(PR[1], PB.p);
    // Without PROJ, loads run two planes ahead and the corrector's u^n of the
    // own cell one plane ahead, issued before that plane's prefetch so that
    // waiting for it never waits for the prefetch.  Loads are unconditional
    // (a thread outside a ragged tile reads the nearest cell, a chunk's last
    // planes repeat its last fetch), so that the compiler's wait counts stay
    // exact.  With PROJ (whose planes carry three times the loads, under
    // per-slot conditions) one plane of lookahead measured faster.
    const unsigned idl = unsigned(min(gx, g.n0 - 1)) + unsigned(g.n0) * unsigned(min(gy, g.n1 - 1));
    float ubn[3] = {0.f, 0.f, 0.f};
    if (CORR && !PROJ) {
#pragma unroll
        for (int c = 0; c < 3; ++c) ubn[c] = ldn(c, idl, plane * unsigned(z0));
    }
    fetch(z0 + 2, PR[2]);  // projected when its plane is first used
    if (!PROJ) fetch(min(z0 + 3, z1 + 1), PR[0]);
    store(2, PR[1]);
    __syncthreads();
    // own-column window W[q][c]: planes z-1, z, z+1 in the LDS ring's slots
    // (plane z+2 is slot 0 of the register set that holds it); lower z-face
    // fluxes Fz[q][c] of planes z and z+1 in slots (z - z0) mod 3
    float W[3][3];
    float Fz[3][3];
    {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            W[0][c] = U(c, 0, own);
            W[1][c] = U(c, 1, own);
            W[2][c] = U(c, 2, own);
        }
        const float wb[3] = {U(2, 1, own - 1), U(2, 1, own - MT_LX), W[0][2]};
#pragma unroll
        for (int c = 0; c < 3; ++c)
            Fz[0][c] = flux2(wm2[c], W[0][c], W[1][c], W[2][c], W[1][2] + wb[c], nu2);
    }

    // One plane, rc = (z - z0) mod 3.  Register set (r + 2) mod 3 holds
    // plane z + 2.  Without PROJ: set r holds plane z + 3 (in flight since
    // the previous plane) and set (r + 1) mod 3 (plane z + 1, already in LDS)
    // receives plane z + 4.  With PROJ: set r (plane z, already in LDS)
    // receives plane z + 3, and set (r + 1) mod 3 holds plane z + 1, whose
    // pressure projects plane z + 2.
    auto do_plane = [&](auto rc, int z) {
        constexpr int r = decltype(rc)::value;
        constexpr int sm1 = r, s0 = (r + 1) % 3, sp1 = (r + 2) % 3;
        constexpr int flo = r, fhi = (r + 1) % 3;
        MtPlane& curP = PR[(r + 2) % 3];
        MtPlane& below = PR[(r + 1) % 3];
        float (&wm1)[3] = W[sm1];
        float (&w0)[3] = W[s0];
        float (&wp1)[3] = W[sp1];
        float (&Fzlo)[3] = Fz[flo];
        float (&Fzhi)[3] = Fz[fhi];
        const bool more = z + 1 < z1;
        const unsigned col = unsigned(gx) + unsigned(g.n0) * unsigned(gy);
        const unsigned zpl = plane * unsigned(z);
        float ubase[3] = {0.f, 0.f, 0.f};
        if constexpr (PROJ) {
            if (more) fetch(z + 3, PR[r]);
            project(curP, below.p);
            if (CORR && inside) {
#pragma unroll
                for (int c = 0; c < 3; ++c) ubase[c] = ldn(c, col, zpl);
            }
        } else {
#pragma unroll
            for (int c = 0; c < 3; ++c) ubase[c] = ubn[c];
            if (CORR) {
                const unsigned zn = unsigned(min(z + 1, z1 - 1));
#pragma unroll
                for (int c = 0; c < 3; ++c) ubn[c] = ldn(c, idl, plane * zn);
                // keep these loads ahead of the prefetch in issue order
                __builtin_amdgcn_sched_barrier(0);
            }
            fetch(min(z + 4, z1 + 1), below);
        }
        const float (&cur)[3][MT_LOADS] = curP.u;
        // lower x face of the own cell (and the tile's upper x column)
        float Fxlo[3], Fylo[3];
        {
            const float a0 = U(0, s0, own);
            const float ab[3] = {U(0, s0, own - 1), U(0, s0, own - MT_LX), U(0, sm1, own)};
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                Fxlo[c] = flux2(U(c, s0, own - 2), U(c, s0, own - 1), w0[c], U(c, s0, own + 1),
                                a0 + ab[c], nu2);
                sFx[c][ty][tx] = Fxlo[c];
            }
        }
        if (xtra_x) {
            const int p = xx_pos;
            const float a0 = U(0, s0, p);
            const float ab[3] = {U(0, s0, p - 1), U(0, s0, p - MT_LX), U(0, sm1, p)};
#pragma unroll
            for (int c = 0; c < 3; ++c)
                sFx[c][t - 64][MT_X] = flux2(U(c, s0, p - 2), U(c, s0, p - 1), U(c, s0, p),
                                             U(c, s0, p + 1), a0 + ab[c], nu2);
        }
        // lower y face of the own cell (and the tile's upper y row)
        {
            const float a0 = U(1, s0, own);
            const float ab[3] = {U(1, s0, own - 1), U(1, s0, own - MT_LX), U(1, sm1, own)};
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                Fylo[c] = flux2(U(c, s0, own - 2 * MT_LX), U(c, s0, own - MT_LX), w0[c],
                                U(c, s0, own + MT_LX), a0 + ab[c], nu2);
                sFy[c][ty][tx] = Fylo[c];
            }
        }
        if (xtra_y) {
            const int p = xy_pos;
            const float a0 = U(1, s0, p);
            const float ab[3] = {U(1, s0, p - 1), U(1, s0, p - MT_LX), U(1, sm1, p)};
#pragma unroll
            for (int c = 0; c < 3; ++c)
                sFy[c][MT_Y][t - 128] = flux2(U(c, s0, p - 2 * MT_LX), U(c, s0, p - MT_LX),
                                              U(c, s0, p), U(c, s0, p + MT_LX), a0 + ab[c], nu2);
        }
        // upper z face of the own cell
        {
            const float wb[3] = {U(2, sp1, own - 1), U(2, sp1, own - MT_LX), w0[2]};
#pragma unroll
            for (int c = 0; c < 3; ++c)
                Fzhi[c] = flux2(wm1[c], w0[c], wp1[c], cur[c][0], wp1[2] + wb[c], nu2);
        }
        __syncthreads();
        if (inside) {
            const int coord[3] = {gx, gy, z};
            const int per[3] = {g.per0, g.per1, g.per2};
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                float v;
                if (!ALLPER && !per[c] && coord[c] == 0) {
                    v = (E.bclo[c] == WL_BC_INFLOW) ? E.U[c] : 0.f;
                } else {
                    float R = -(sFx[c][ty][tx + 1] - Fxlo[c]);
                    R -= sFy[c][ty + 1][tx] - Fylo[c];
                    R -= Fzhi[c] - Fzlo[c];
                    v = CORR ? 0.5f * (ubase[c] + w0[c] + hdt * R) : w0[c] + hdt * R;
                }
                stf(c, col, zpl, v);
            }
        }
        // plane z - 1 leaves the window, plane z + 2 enters its slot
#pragma unroll
        for (int c = 0; c < 3; ++c) wm1[c] = cur[c][0];
        if (more) store(sm1, curP);
        __syncthreads();
    };
    using R0 = std::integral_constant<int, 0>;
    using R1 = std::integral_constant<int, 1>;
    using R2 = std::integral_constant<int, 2>;
    for (int z = z0; z < z1;) {
        do_plane(R0{}, z);
        if (++z >= z1) break;
        do_plane(R1{}, z);
        if (++z >= z1) break;
        do_plane(R2{}, z);
        ++z;
    }
}

// The two entry points differ only in their register budget: without the
// projection, at most 128 VGPRs (4 waves per SIMD, two blocks per CU), and
// 80 for the periodic predictor (6 waves, three blocks per CU, no spills),
// which keeps the two-plane lookahead from stretching the schedule; the
// projecting corrector measured faster with the compiler's own choice.
template <bool ALLPER, bool CORR, bool BUF>
__global__ __launch_bounds__(MT_T) __attribute__((amdgpu_waves_per_eu(ALLPER && !CORR ? 6 : 4))) void k_momentum_tiled(
    VelField<float> E, const float* __restrict__ un0, const float* __restrict__ un1,
    const float* __restrict__ un2, float* __restrict__ f0, float* __restrict__ f1,
    float* __restrict__ f2, float nu, const double* __restrict__ dt_dev, TileMap tm) {
    momentum_tile<ALLPER, CORR, false, BUF>(E, un0, un1, un2, f0, f1, f2, nu, dt_dev, tm, nullptr,
                                            0.f);
}

template <bool BUF>
__global__ __launch_bounds__(MT_T) void k_momentum_tiled_proj(
    VelField<float> E, const float* __restrict__ un0, const float* __restrict__ un1,
    const float* __restrict__ un2, float* __restrict__ f0, float* __restrict__ f1,
    float* __restrict__ f2, float nu, const double* __restrict__ dt_dev, TileMap tm,
    const float* __restrict__ pp, float Lc) {
    momentum_tile<true, true, true, BUF>(E, un0, un1, un2, f0, f1, f2, nu, dt_dev, tm, pp, Lc);
}

// Buffer descriptors address 32-bit byte offsets: arrays below 4 GiB.  The
// environment variable WL_GLOBAL_ADDRESSING=1 (read at every launch) selects
// the global-address kernels on any grid, so that the path arrays of 4 GiB
// and more take can be checked on small ones.
static bool buffer_addressing(const Grid& g) {
    const char* e = std::getenv("WL_GLOBAL_ADDRESSING");
    return cells(g) < (size_t(1) << 30) && !(e && e[0] == '1');
}
static bool momentum_buf(const Grid& g) { return buffer_addressing(g); }

// Outflow plane (upper x face): convective update d(uout)/dt = -U_x (uout -
// u_x(n0-1)) in the same stage form, then a uniform shift making its total
// flux equal to the inflow plane's.  Two launches over the plane's cells
// (the plane's and the inflow plane's cells are a column stride apart in
// memory, so each thread takes one and all loads are in flight at once):
// the first writes the unshifted plane and per-workgroup FP64 sums of both
// fluxes, the second forms the totals from those sums in a fixed order (every
// workgroup the same) and adds the shift.
constexpr int kOutflowThreads = 256;

template <typename T, bool CORR>
__global__ __launch_bounds__(kOutflowThreads) void k_outflow_flux(Grid g, const T* __restrict__ ue_x,
                                                                  const T* __restrict__ out_e,
                                                                  const T* __restrict__ out_n,
                                                                  const T* __restrict__ f_x, T Ux,
                                                                  const double* __restrict__ dt_dev,
                                                                  T* __restrict__ fout,
                                                                  double* __restrict__ part) {
    __shared__ double lds[2][kOutflowThreads / 64];
    const int P = g.n1 * g.n2;
    const int q = int(blockIdx.x) * kOutflowThreads + int(threadIdx.x);
    double sin_ = 0.0, sout = 0.0;
    if (q < P) {
        const T dt = T(*dt_dev);
        const int j = q % g.n1, k = q / g.n1;
        const T last = ue_x[cid(g, g.n0 - 1, j, k)];
        const T R = -Ux * (out_e[q] - last);
        const T f = CORR ? T(0.5) * (out_n[q] + out_e[q] + dt * R) : out_e[q] + dt * R;
        fout[q] = f;
        sout = double(f);
        sin_ = double(f_x[cid(g, 0, j, k)]);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        sin_ += __shfl_xor(sin_, off, 64);
        sout += __shfl_xor(sout, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        lds[0][threadIdx.x >> 6] = sin_;
        lds[1][threadIdx.x >> 6] = sout;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, c = 0.0;
        for (int w = 0; w < kOutflowThreads / 64; ++w) {
            a += lds[0][w];
            c += lds[1][w];
        }
        part[2 * blockIdx.x] = a;
        part[2 * blockIdx.x + 1] = c;
    }
}

template <typename T>
__global__ __launch_bounds__(kOutflowThreads) void k_outflow_shift(Grid g,
                                                                   const double* __restrict__ part,
                                                                   int nblk, T* __restrict__ fout) {
    __shared__ double lds[2][kOutflowThreads / 64];
    __shared__ double shift_s;
    double a = 0.0, c = 0.0;
    for (int w = int(threadIdx.x); w < nblk; w += kOutflowThreads) {
        a += part[2 * w];
        c += part[2 * w + 1];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_xor(a, off, 64);
        c += __shfl_xor(c, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        lds[0][threadIdx.x >> 6] = a;
        lds[1][threadIdx.x >> 6] = c;
    }
    __syncthreads();
    const int P = g.n1 * g.n2;
    if (threadIdx.x == 0) {
        double tin = 0.0, tout = 0.0;
        for (int w = 0; w < kOutflowThreads / 64; ++w) {
            tin += lds[0][w];
            tout += lds[1][w];
        }
        shift_s = (tin - tout) / double(P);
    }
    __syncthreads();
    const int q = int(blockIdx.x) * kOutflowThreads + int(threadIdx.x);
    if (q < P) fout[q] += T(shift_s);
}

// First-order BDIM blend on interior faces:
//   u*_c = mu0_c f_c + (1 - mu0_c) V_b,c
//          + sum_d (mu1 n)_cd [(f_c(I+delta_d) - f_c(I-delta_d)) / 2 - dV_b,c/dx_d],
// V_b the body velocity at the face (zero for a body at rest).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_bdim(TileDev TL, VelField<T> F, BdimFields<T> B,
                                                 T* __restrict__ o0, T* __restrict__ o1,
                                                 T* __restrict__ o2, BodyMotionDev mo) {
    const Grid& g = F.g;
    const Span sp = tile_span(TL, g.n0, g.n1, g.n2);
    const int i = sp.i, j = sp.j;
    if (i >= g.n0 || j >= g.n1) return;
    if (B.cls && B.cls[block_linear()] == 0) {
        // away from the body: u* = 1 * f exactly
        T* out[3] = {o0, o1, o2};
        for (int k = sp.z0; k < sp.z1; ++k) {
            const size_t id = cid(g, i, j, k);
            for (int c = 0; c < g.ndim; ++c) out[c][id] = F.u[c][id];
        }
        return;
    }
    T* out[3] = {o0, o1, o2};
    for (int k = sp.z0; k < sp.z1; ++k) {
        const size_t id = cid(g, i, j, k);
        for (int c = 0; c < g.ndim; ++c) out[c][id] = bdim_face<T>(F, B, mo, c, i, j, k);
    }
}

// The same blend on the flagged cells only (B.cflag), one thread per cell,
// into w: the few cells near the body each take one thread, so no thread
// walks a chain of them.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_bdim_cells(VelField<T> F, BdimFields<T> B,
                                                       T* __restrict__ w0, T* __restrict__ w1,
                                                       T* __restrict__ w2, BodyMotionDev mo) {
    const Grid& g = F.g;
    const size_t id = size_t(blockIdx.x) * kBlock + threadIdx.x;
    if (id >= cells(g) || !B.cflag[id]) return;
    const size_t plane = size_t(g.n0) * size_t(g.n1);
    const int k = int(id / plane);
    const size_t r = id - size_t(k) * plane;
    const int j = int(r / size_t(g.n0)), i = int(r - size_t(j) * size_t(g.n0));
    // every component's loads before any store
    T v[3] = {T(0), T(0), T(0)};
    for (int c = 0; c < g.ndim; ++c) v[c] = bdim_face<T, true>(F, B, mo, c, i, j, k);
    w0[id] = v[0];
    w1[id] = v[1];
    if (g.ndim == 3) w2[id] = v[2];
}

// The flagged cells' u* (k_bdim_cells, in w) copied into f, after every
// thread has read f.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_bdim_commit(Grid g,
                                                        const unsigned char* __restrict__ cflag,
                                                        const T* __restrict__ w0,
                                                        const T* __restrict__ w1,
                                                        const T* __restrict__ w2,
                                                        T* __restrict__ f0, T* __restrict__ f1,
                                                        T* __restrict__ f2) {
    const size_t id = size_t(blockIdx.x) * kBlock + threadIdx.x;
    if (id >= cells(g) || !cflag[id]) return;
    f0[id] = w0[id];
    f1[id] = w1[id];
    if (g.ndim == 3) f2[id] = w2[id];
}

// Tile class of each block: 1 if any face of its tile has mu0 != 1 or a
// nonzero mu1 n component.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_tile_class(TileDev TL, Grid g, BdimFields<T> B,
                                                       unsigned char* __restrict__ cls,
                                                       unsigned char* __restrict__ cflag) {
    __shared__ int any;
    if (threadIdx.x == 0) any = 0;
    __syncthreads();
    const Span sp = tile_span(TL, g.n0, g.n1, g.n2);
    const int i = sp.i, j = sp.j;
    bool near = false;
    if (i < g.n0 && j < g.n1)
        for (int k = sp.z0; k < sp.z1 && (cflag || !near); ++k) {
            const size_t id = cid(g, i, j, k);
            bool cell = false;
            for (int c = 0; c < g.ndim; ++c) {
                cell = cell || B.mu0[c][id] != T(1);
                for (int d = 0; d < g.ndim; ++d) cell = cell || B.mu1n[3 * c + d][id] != T(0);
            }
            if (cflag) cflag[id] = cell ? 1 : 0;
            near = near || cell;
        }
    if (near) any = 1;  // benign race: every writer stores 1
    __syncthreads();
    if (threadIdx.x == 0) cls[block_linear()] = any ? 1 : 0;
}

// sigma = div(u*) / (c dt), plus per-block partial sums of sigma over the
// active cells (D != 0; every cell when the coefficients are uniform) for the
// mean removal of the pressure solve.  CHK (periodic, uniform coefficient Lp,
// 3D) also evaluates the pressure solve's first residual check here: with the
// solve's initial iterate p and c = sigma - A p, the per-block sums
// [sigma, sigma^2, c, c^2] (partial[4 * block + q]), from which the mean m and
// ||r||^2 = sum (c - m)^2, ||b - m||^2 follow without another pass.
// Component d on the cell above (i, j, k) in direction d when that cell lies
// past a non-periodic upper face (the other coordinates inside): the ghost
// rule's value there, the outflow plane or zero (vget's branch for it,
// without the rest of the rule).
template <typename T>
__device__ __forceinline__ T ghost_up(const VelField<T>& V, int d, int j, int k) {
    const Grid& g = V.g;
    const int bh = d == 0 ? V.bchi[0] : (d == 1 ? V.bchi[1] : V.bchi[2]);
    if (bh != WL_BC_OUTFLOW) return T(0);
    const int a = min(j + (d == 1), g.n1 - 1), b = min(k + (d == 2), g.n2 - 1);
    return V.uout[a + size_t(g.n1) * b];
}

template <typename T, bool ALLPER, bool UNIF, bool CHK>
__global__ __launch_bounds__(kBlock) void k_divergence(TileDev TL, VelField<T> V, ProjCoeffs<T> C,
                                                       double c, const double* __restrict__ dt_dev,
                                                       T* __restrict__ sigma,
                                                       double* __restrict__ partial,
                                                       const T* __restrict__ p, T Lp) {
    __shared__ double lds[16];
    const Grid& g = V.g;
    const Span sp = tile_span(TL, g.n0, g.n1, g.n2);
    const int i = sp.i, j = sp.j;
    const T scale = T(1.0 / (c * *dt_dev));
    double sum = 0.0, sb2 = 0.0, sc = 0.0, sc2 = 0.0;
    if (i < g.n0 && j < g.n1 && sp.z0 < sp.z1) {
        const unsigned n0 = unsigned(g.n0), plane = n0 * unsigned(g.n1);
        const bool d3 = g.ndim == 3;
        // upper x / y neighbour offsets (fixed along the column); the
        // non-periodic upper boundary goes through the ghost rules
        const bool xin = i + 1 < g.n0 || ALLPER || g.per0;
        const bool yin = j + 1 < g.n1 || ALLPER || g.per1;
        const int dxp = i + 1 < g.n0 ? 1 : -(g.n0 - 1);
        const int dyp = j + 1 < g.n1 ? int(n0) : -int(n0) * (g.n1 - 1);
        const T* __restrict__ ux = V.u[0];
        const T* __restrict__ uy = V.u[1];
        const T* __restrict__ uz = V.u[2];
        unsigned id = unsigned(i) + n0 * unsigned(j) + plane * unsigned(sp.z0);
        T wlo = d3 ? uz[id] : T(0);  // lower z face, carried up the column
        // a class-0 block: every cell active, no coefficient read
        const bool walled = !UNIF && C.cls && C.cls[block_linear()] == 0;
        // CHK: periodic x / y neighbour offsets of p; p at k - 1 and k carried
        const int dxm = i > 0 ? -1 : g.n0 - 1;
        const int dym = j > 0 ? -int(n0) : int(n0) * (g.n1 - 1);
        T pzl = T(0), pI = T(0);
        if (CHK) {
            pI = p[id];
            pzl = p[sp.z0 > 0 ? id - plane : id + plane * unsigned(g.n2 - 1)];
        }
        for (int k = sp.z0; k < sp.z1; ++k, id += plane) {
            const T xu = xin ? ux[id + dxp] : ghost_up<T>(V, 0, j, k);
            const T yu = yin ? uy[id + dyp] : ghost_up<T>(V, 1, j, k);
            T div = (xu - ux[id]) + (yu - uy[id]);
            if (d3) {
                T wup;
                if (k + 1 < g.n2) wup = uz[id + plane];
                else if (ALLPER || g.per2) wup = uz[id - plane * unsigned(g.n2 - 1)];
                else wup = ghost_up<T>(V, 2, j, k);
                div += wup - wlo;
                wlo = wup;
            }
            const T sg = div * scale;
            sigma[id] = sg;
            if (CHK) {
                const T pzu = p[k + 1 < g.n2 ? id + plane : id - plane * unsigned(g.n2 - 1)];
                const T Ax = jacobi_ax_uniform(pI, p[id + dxm], p[id + dxp], p[id + dym],
                                               p[id + dyp], pzl, pzu, Lp, true);
                const double cr = double(sg - Ax);
                sb2 += double(sg) * double(sg);
                sc += cr;
                sc2 += cr * cr;
                pzl = pI;
                pI = pzu;
            }
            bool active = true;
            if (!UNIF && !walled) {
                T D = T(0);
                const int n[3] = {g.n0, g.n1, g.n2};
                const int per[3] = {g.per0, g.per1, g.per2};
                const int q[3] = {i, j, k};
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    if (d >= g.ndim) break;
                    D += C.L[d][id];
                    if (q[d] + 1 < n[d] || per[d]) {
                        int r[3] = {i, j, k};
                        r[d] = q[d] + 1 < n[d] ? q[d] + 1 : 0;
                        D += C.L[d][cid(g, r[0], r[1], r[2])];
                    }
                }
                active = D > T(0);
            }
            if (active) sum += double(sg);
        }
    }
    if (CHK) {
        double t0, t1, t2, t3;
        block_sum2(sum, sb2, lds, t0, t1);
        block_sum2(sc, sc2, lds + 8, t2, t3);
        if (threadIdx.x == 0) {
            double* q = partial + 4 * size_t(block_linear());
            q[0] = t0;
            q[1] = t1;
            q[2] = t2;
            q[3] = t3;
        }
        return;
    }
    const double bs = block_sum(sum, lds);
    if (threadIdx.x == 0) partial[block_linear()] = bs;
}

// The same divergence with the pressure solve's first residual check on a
// periodic grid with a uniform Poisson coefficient Lp (3D, x / y extents
// multiples of 64 / 8): a 64 x 8 column tile walks a z chunk; per plane the
// iterate p is staged in LDS with a one-cell ring (the first 148 threads hold
// a ring cell each) for the x / y neighbours, the z neighbours come from the
// thread's own column.  sigma is computed with the same operations as
// k_divergence; partials as its CHK variant, one slot per workgroup.
constexpr int DC_TX = 64, DC_TY = 8, DC_T = DC_TX * DC_TY;
constexpr int DC_HX = DC_TX + 2, DC_HY = DC_TY + 2, DC_RING = DC_HX * DC_HY - DC_T;

template <typename T, bool BUF>
__global__ __launch_bounds__(DC_T) void k_div_check(TileMap tm, VelField<T> V, double c,
                                                    const double* __restrict__ dt_dev,
                                                    T* __restrict__ sigma,
                                                    double* __restrict__ partial,
                                                    const T* __restrict__ p, T Lp) {
    __shared__ T sp[2][DC_HY * DC_HX];
    __shared__ double red[4][DC_T / 64];
    const Grid& g = V.g;
    unsigned blk = blockIdx.x;
    if (tm.remap) blk = (blk & 7u) * (tm.nblocks >> 3) + (blk >> 3);
    const int tix = int(blk % unsigned(tm.tiles_x));
    blk /= unsigned(tm.tiles_x);
    const int tiy = int(blk % unsigned(tm.tiles_y));
    const int z0 = int(blk / unsigned(tm.tiles_y)) * tm.zc;
    const int z1 = min(z0 + tm.zc, g.n2);
    const int i0 = tix * DC_TX, j0 = tiy * DC_TY;
    const int t = int(threadIdx.x), ax = t % DC_TX, ay = t / DC_TX;
    const unsigned n0 = unsigned(g.n0), plane = n0 * unsigned(g.n1);
    // periodic grid column of ring-box position (hx, hy)
    auto col = [&](int hx, int hy) -> unsigned {
        int i = i0 + hx - 1, j = j0 + hy - 1;
        i = i < 0 ? i + g.n0 : (i >= g.n0 ? i - g.n0 : i);
        j = j < 0 ? j + g.n1 : (j >= g.n1 ? j - g.n1 : j);
        return unsigned(i) + n0 * unsigned(j);
    };
    const unsigned cA = col(ax + 1, ay + 1);
    const int hA = (ay + 1) * DC_HX + ax + 1;
    const bool hasB = t < DC_RING;
    unsigned cB = cA;  // threads without a ring cell load their own again
    int hB = hA;
    if (hasB) {
        int hx, hy;
        ring_cell(t, DC_TX, DC_TY, hx, hy);
        cB = col(hx, hy);
        hB = hy * DC_HX + hx;
    }
    const int i = i0 + ax, j = j0 + ay;
    const int dxp = i + 1 < g.n0 ? 1 : -(g.n0 - 1);
    const int dyp = j + 1 < g.n1 ? int(n0) : -int(n0) * (g.n1 - 1);
    const T* __restrict__ ux = V.u[0];
    const T* __restrict__ uy = V.u[1];
    const T* __restrict__ uz = V.u[2];
    const T scale = T(1.0 / (c * *dt_dev));
    // BUF (FP32, arrays below 4 GiB): loads and stores through buffer
    // descriptors, the plane's byte offset uniform (scalar), the column's in a
    // vector register; the plane offsets are uniform over the block, which
    // readfirstlane tells the compiler
    static_assert(!BUF || sizeof(T) == 4, "buffer addressing is for FP32 arrays");
    const int nbytes = BUF ? int(unsigned(size_t(plane) * unsigned(g.n2) * 4u)) : 0;
    auto rsrc = [&](const T* q) {
        return __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(q), 0, nbytes, 0x00020000);
    };
    const auto dX = rsrc(ux), dY = rsrc(uy), dZ = rsrc(uz), dP = rsrc(p), dS = rsrc(sigma);
    auto uni = [](unsigned v) { return int(__builtin_amdgcn_readfirstlane(int(v))); };
    // value of array a (descriptor d) at column offset cl (may be negative:
    // a wrapped neighbour) of plane w
    auto ld = [&](const T* a, const __amdgpu_buffer_rsrc_t& d, int cl, int w) -> T {
        if constexpr (BUF)
            return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(
                                             d, cl * 4, uni(unsigned(w) * plane * 4u), 0));
        else
            return a[unsigned(int(unsigned(w) * plane) + cl)];
    };
    auto wrap = [&](int q) {
        q %= g.n2;
        return q < 0 ? q + g.n2 : q;
    };
    auto next = [&](int w) { return w + 1 == g.n2 ? 0 : w + 1; };
    // p rings indexed by plane (mod 4): own column and ring cell planes up
    // to k + 2 (loaded two planes ahead); velocity rings: the faces of planes
    // k and k + 1 (loaded one plane ahead); the loop is unrolled 4 times
    T pA[4] = {}, pB[4] = {};
    T xl[4] = {}, xh[4] = {}, yl[4] = {}, yh[4] = {}, zh[4] = {};
    const int iA = int(cA), iB = int(cB);
    int w = wrap(z0 - 1);
    pA[3] = ld(p, dP, iA, w);
    w = next(w);
    int wk = w;  // wrapped plane k
    pA[0] = ld(p, dP, iA, w);
    pB[0] = ld(p, dP, iB, w);
    w = next(w);
    pA[1] = ld(p, dP, iA, w);
    pB[1] = ld(p, dP, iB, w);
    int wp1 = w, wp2 = next(w);  // wrapped planes k + 1, k + 2
    T wlo = ld(uz, dZ, iA, wk);
    // x, y faces of plane k and the upper z face (plane k + 1) of the own cell
    auto ldu = [&](int q, int wq, int wq1) {
        xl[q] = ld(ux, dX, iA, wq);
        xh[q] = ld(ux, dX, iA + dxp, wq);
        yl[q] = ld(uy, dY, iA, wq);
        yh[q] = ld(uy, dY, iA + dyp, wq);
        zh[q] = ld(uz, dZ, iA, wq1);
    };
    ldu(0, wk, wp1);
    double sum = 0.0, sb2 = 0.0, sc = 0.0, sc2 = 0.0;
    int k = z0;
    auto step = [&](auto rc) {
        constexpr int r = decltype(rc)::value;
        constexpr int im1 = (r + 3) % 4, ip1 = (r + 1) % 4, ip2 = (r + 2) % 4;
        T* S = sp[k & 1];
        S[hA] = pA[r];
        // unconditional: a thread without a ring cell stores its own value
        // again (hB = hA, cB = cA); a conditional store would pull the load
        // of pB into its branch and wait for it there
        S[hB] = pB[r];
        __syncthreads();
        // unconditional: no branch around loads keeps the wait counts exact;
        // the chunk's last plane repeats planes it already holds (cache hits)
        // instead of fetching ones it never uses
        const int wl1 = k + 1 < z1 ? wp1 : wk, wl2 = k + 1 < z1 ? wp2 : wp1;
        ldu(ip1, wl1, wl2);
        pA[ip2] = ld(p, dP, iA, wl2);
        pB[ip2] = ld(p, dP, iB, wl2);
        // issue the next planes' loads here, not after this plane's work
        __builtin_amdgcn_sched_barrier(0);
        const T wup = zh[r];
        T div = (xh[r] - xl[r]) + (yh[r] - yl[r]);
        div += wup - wlo;
        wlo = wup;
        const T sg = div * scale;
        if constexpr (BUF)
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, sg), dS, iA * 4,
                                                  uni(unsigned(wk) * plane * 4u), 0);
        else
            sigma[cA + unsigned(wk) * plane] = sg;
        const T Ax = jacobi_ax_uniform(pA[r], S[hA - 1], S[hA + 1], S[hA - DC_HX], S[hA + DC_HX],
                                       pA[im1], pA[ip1], Lp, true);
        const double cr = double(sg - Ax);
        sum += double(sg);
        sb2 += double(sg) * double(sg);
        sc += cr;
        sc2 += cr * cr;
        wk = wp1;
        wp1 = wp2;
        wp2 = next(wp2);
        ++k;
    };
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using I3 = std::integral_constant<int, 3>;
    // whole groups of four planes without exits between them (an exit
    // between two planes would let the compiler sink the next plane's loads
    // behind it, up to their use), then the remainder
    while (k + 4 <= z1) {
        step(I0{});
        step(I1{});
        step(I2{});
        step(I3{});
    }
    if (k < z1) {
        step(I0{});
        if (k < z1) {
            step(I1{});
            if (k < z1) step(I2{});
        }
    }
    // fixed-order workgroup sums: wave butterflies, then waves in order
    double v[4] = {sum, sb2, sc, sc2};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[q] += __shfl_xor(v[q], off, 64);
        if ((t & 63) == 0) red[q][t >> 6] = v[q];
    }
    __syncthreads();
    if (t == 0) {
        double* out = partial + 4 * size_t(blockIdx.x);
        for (int q = 0; q < 4; ++q) {
            double s = 0.0;
            for (int wv = 0; wv < DC_T / 64; ++wv) s += red[q][wv];
            out[q] = s;
        }
    }
}

// Workgroups of k_div_check on g (0 when it does not apply): about 1024
// (32-plane chunks at 256^3; 2048 and 4096 blocks measured 1.4 and 2.4 us
// slower there), chunks of at least 8 planes.
TileMap div_check_map(const Grid& g) {
    TileMap tm{};
    if (g.ndim != 3 || g.n0 % DC_TX != 0 || g.n1 % DC_TY != 0) return tm;
    const size_t cols = size_t(g.n0 / DC_TX) * size_t(g.n1 / DC_TY);
    int zc = int((cols * size_t(g.n2) + 1023) / 1024);
    zc = zc < 8 ? 8 : zc;
    return tile_map(g, DC_TX, DC_TY, zc);
}

// u = u* - c dt L grad(p) for every direction in one pass (the gradient loop
// of Sec. 2 with coeff = c dt L, fused over directions).  Each thread walks
// its column up the z chunk and evaluates every face once: the lower x and y
// faces of its cell and the upper z face, which (with p there) is carried to
// the next plane as its lower z face.  Without CFL the output may alias u*
// (a thread reads u* only on faces it writes later).  With CFL, also the
// per-block maximum of sum_d max(u_d(I+delta_d),0) - min(u_d(I),0) of the
// projected field: the upper x / y faces come from the neighbouring thread
// through LDS, or are recomputed at the edge of the block's tile (the output
// must then not alias u*).
template <typename T, bool ALLPER, bool UNIF, bool CFL>
__global__ __launch_bounds__(kBlock) void k_project(TileDev TL, VelField<T> V, const T* __restrict__ p,
                                                    ProjCoeffs<T> C, double c,
                                                    const double* __restrict__ dt_dev,
                                                    T* o0, T* o1, T* o2,
                                                    double* __restrict__ partial) {
    __shared__ double lds[8];
    __shared__ T sX[CFL ? kBlock : 1], sY[CFL ? kBlock : 1];
    const Grid& g = V.g;
    const Span sp = tile_span(TL, g.n0, g.n1, g.n2);
    const int i = sp.i, j = sp.j;
    const int t = threadIdx.x, bx = 1 << TL.lbx;
    const bool valid = i < g.n0 && j < g.n1;
    const T coef = T(c * *dt_dev);
    const bool d3 = g.ndim == 3;
    const bool per0 = ALLPER || g.per0, per1 = ALLPER || g.per1, per2 = ALLPER || g.per2;
    const unsigned n0 = unsigned(g.n0), plane = n0 * unsigned(g.n1);
    const int dxm = i > 0 ? -1 : g.n0 - 1;                       // lower x neighbour
    const int dym = j > 0 ? -int(n0) : int(n0) * (g.n1 - 1);      // lower y neighbour
    const bool bx0 = !per0 && i == 0, by0 = !per1 && j == 0;      // boundary faces (L = 0)
    const T* sx = V.u[0];  // no restrict: the output may alias u*
    const T* sy = V.u[1];
    const T* sz = V.u[2];
    // a class-0 block reads no coefficient: every face it projects is Lc
    // (the wall faces are handled apart)
    const bool walled = !UNIF && C.cls && C.cls[block_linear()] == 0;
    auto Lat = [&](int d, unsigned id) -> T { return (UNIF || walled) ? C.Lc : C.L[d][id]; };
    // projected face d with lower cell offset dm (its cell holds pI)
    auto face = [&](int d, const T* u, unsigned id, int dm, T pI) -> T {
        return proj_face(u[id], coef * Lat(d, id), pI, p[id + dm]);
    };
    // CFL edge recompute: projected upper face of direction d of cell (i,j,k)
    auto upper = [&](int d, unsigned id, int k, T pI) -> T {
        const int q[3] = {i, j, k};
        const int n[3] = {g.n0, g.n1, g.n2};
        const bool per[3] = {per0, per1, per2};
        const int st[3] = {1, int(n0), int(plane)};
        if (q[d] + 1 < n[d] || per[d]) {
            const int du = q[d] + 1 < n[d] ? st[d] : -st[d] * (n[d] - 1);
            const unsigned idu = id + du;
            return proj_face(V.u[d][idu], coef * Lat(d, idu), p[idu], pI);
        }
        return ghost_up<T>(V, d, j, k);
    };
    double cfl = 0.0;
    unsigned id = unsigned(i) + n0 * unsigned(j) + plane * unsigned(sp.z0);
    T pI = T(0), wlo = T(0);
    if (valid && sp.z0 < sp.z1) {
        pI = p[id];
        if (d3) {
            if (!per2 && sp.z0 == 0) wlo = sz[id];
            else wlo = face(2, sz, id, sp.z0 > 0 ? -int(plane) : int(plane) * (g.n2 - 1), pI);
        }
    }
    for (int k = sp.z0; k < sp.z1; ++k, id += plane) {
        T ux = T(0), uy = T(0), wup = T(0), pU = T(0);
        const bool carry = k + 1 < sp.z1;
        if (valid) {
            ux = bx0 ? sx[id] : face(0, sx, id, dxm, pI);
            uy = by0 ? sy[id] : face(1, sy, id, dym, pI);
            if (d3 && (carry || CFL)) {
                if (k + 1 < g.n2) {
                    pU = p[id + plane];
                    wup = proj_face(sz[id + plane], coef * Lat(2, id + plane), pU, pI);
                } else if (per2) {
                    const unsigned i0 = id - plane * unsigned(g.n2 - 1);
                    wup = proj_face(sz[i0], coef * Lat(2, i0), p[i0], pI);
                } else {
                    wup = ghost_up<T>(V, 2, j, k);
                }
            }
            o0[id] = ux;
            o1[id] = uy;
            if (d3) o2[id] = wlo;
        }
        if (CFL) {
            sX[t] = ux;
            sY[t] = uy;
            __syncthreads();
            if (valid) {
                const T xu = ((t & (bx - 1)) < bx - 1 && i + 1 < g.n0) ? sX[t + 1] : upper(0, id, k, pI);
                const T yu = (t + bx < kBlock && j + 1 < g.n1) ? sY[t + bx] : upper(1, id, k, pI);
                T s = fmax(xu, T(0)) - fmin(ux, T(0));
                s += fmax(yu, T(0)) - fmin(uy, T(0));
                if (d3) s += fmax(wup, T(0)) - fmin(wlo, T(0));
                cfl = fmax(cfl, double(s));
            }
            __syncthreads();
        }
        wlo = wup;
        pI = pU;
        if (valid && carry && !d3) pI = p[id + plane];
    }
    if (CFL) {
        const double m = block_max(cfl, lds);
        if (threadIdx.x == 0) partial[block_linear()] = m;
    }
}

// Per-block CFL maximum of the current field.
template <typename T, bool ALLPER>
__global__ __launch_bounds__(kBlock) void k_cfl(TileDev TL, VelField<T> V, double* __restrict__ partial) {
    __shared__ double lds[8];
    const Grid& g = V.g;
    const Span sp = tile_span(TL, g.n0, g.n1, g.n2);
    const int i = sp.i, j = sp.j;
    double v = 0.0;
    if (i < g.n0 && j < g.n1) {
        for (int k = sp.z0; k < sp.z1; ++k) {
        const size_t id = cid(g, i, j, k);
        T s = T(0);
        for (int d = 0; d < g.ndim; ++d) {
            const T up = vget<T, ALLPER>(V, d, i + (d == 0), j + (d == 1), k + (d == 2));
            s += fmax(up, T(0)) - fmin(V.u[d][id], T(0));
        }
        v = fmax(v, double(s));
        }
    }
    const double m = block_max(v, lds);
    if (threadIdx.x == 0 && threadIdx.y == 0) partial[block_linear()] = m;
}

// dt = cfl / (max over slots + visc); visc = 2 d nu.  One block; with
// post.vals it also posts dt to the host mailbox.
__global__ __launch_bounds__(1024) void k_dt_from_max(const double* __restrict__ partial,
                                                      size_t nslots, double cfl, double visc,
                                                      double* __restrict__ dt_out,
                                                      double* __restrict__ max_out,
                                                      MailboxPost post) {
    __shared__ double lds[16];
    double m[1];
    wg_slot_reduce<1, true>(partial, nslots, m, lds);
    if (threadIdx.x == 0) {
        const double den = m[0] + visc;
        *max_out = m[0];
        *dt_out = den > 0.0 ? cfl / den : 0.0;
        if (post.vals) mailbox_write(post, dt_out);
    }
}

__global__ void k_set_scalar(double* p, double v) {
    if (threadIdx.x == 0) *p = v;
}

// BDIM moments and Poisson coefficients of every face from the sphere SDF
// d = |x - centre| - R (face centre x = I + 1/2 - delta_c / 2; 2D ignores z):
// mu0 = (1 + r + sin(pi r)/pi)/2, mu1 = eps [(1-r^2)/4 - r sin(pi r)/(2 pi)
// - (1 + cos(pi r))/(2 pi^2)] for |r| = |d/eps| < 1 (1/0 and 0 outside),
// (mu1 n)_cd = mu1 n_d, L_c = mu0 except 0 on non-periodic lower boundary faces.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_measure(TileDev TL, Grid g, BodyDev body, int bclo0, int bclo1,
                                                    int bclo2, MeasureOut<T> M) {
    const Span sp = tile_span(TL, g.n0, g.n1, g.n2);
    const int i = sp.i, j = sp.j;
    if (i >= g.n0 || j >= g.n1) return;
    const int bclo[3] = {bclo0, bclo1, bclo2};
    for (int k = sp.z0; k < sp.z1; ++k) {
        const size_t id = cid(g, i, j, k);
        for (int c = 0; c < 3; ++c) {
            double m0, m1, nrm[3];
            measure_face(g, body, c, i, j, k, m0, m1, nrm);
            if (M.mu0[c]) M.mu0[c][id] = T(m0);
            if (M.mu1n[3 * c])
                for (int d = 0; d < 3; ++d) M.mu1n[3 * c + d][id] = T(m1 * nrm[d]);
            const double L = face_coeff(g, bclo, c, i, j, k, m0);
            if (M.L[c]) M.L[c][id] = T(L);
            if (M.L64[c]) M.L64[c][id] = L;
        }
    }
}

// Initial velocity: U_c on every face, boundary faces at their boundary value.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_init_velocity(TileDev TL, Grid g, int b0, int b1, int b2, T U0, T U1,
                                                          T U2, T* __restrict__ u0,
                                                          T* __restrict__ u1, T* __restrict__ u2) {
    const Span sp = tile_span(TL, g.n0, g.n1, g.n2);
    const int i = sp.i, j = sp.j;
    if (i >= g.n0 || j >= g.n1) return;
    for (int k = sp.z0; k < sp.z1; ++k) {
    const size_t id = cid(g, i, j, k);
    const int coord[3] = {i, j, k};
    const int per[3] = {g.per0, g.per1, g.per2};
    const int bclo[3] = {b0, b1, b2};
    const T U[3] = {U0, U1, U2};
    T* u[3] = {u0, u1, u2};
    for (int c = 0; c < 3; ++c) {
        T v = c < g.ndim ? U[c] : T(0);
        if (!per[c] && coord[c] == 0) v = (bclo[c] == WL_BC_INFLOW) ? U[c] : T(0);
        u[c][id] = v;
    }
    }
}

// ------------------------------------------------------------- launchers

template <typename T>
wl_status ns_init_velocity(const Grid& g, const int bclo[3], const double U[3], T* const u[3],
                           hipStream_t s) {
    const Launch ln = launch_for(g.n0, g.n1, g.n2);
    k_init_velocity<T><<<ln.grid, ln.block, 0, s>>>(ln.td, g, bclo[0], bclo[1], bclo[2], T(U[0]), T(U[1]),
                                                    T(U[2]), u[0], u[1], u[2]);
    WL_CHECK_LAUNCH();
    return WL_OK;
}

template <typename T>
wl_status ns_measure(const Grid& g, const BodyDev& body, const int bclo[3], const MeasureOut<T>& M,
                     hipStream_t s) {
    const Launch ln = launch_for(g.n0, g.n1, g.n2);
    k_measure<T><<<ln.grid, ln.block, 0, s>>>(ln.td, g, body, bclo[0], bclo[1], bclo[2], M);
    WL_CHECK_LAUNCH();
    return WL_OK;
}

// z planes per block of the tiled momentum kernel: enough z chunks that
// every CU gets per_cu resident blocks, each chunk 8 to 64 planes (a chunk
// reloads four planes around it); WL_MOM_ZC overrides.
int momentum_zchunk(const Grid& g, int per_cu) {
    static const int env = [] {
        const char* e = std::getenv("WL_MOM_ZC");
        const int v = e ? std::atoi(e) : 0;
        return v > 0 ? v : 0;
    }();
    if (env) return env;
    // CU count of the current device, queried once per device
    static std::atomic<int> cus[64];
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) == hipSuccess && dev >= 0 && dev < 64) ncu = cus[dev].load();
    if (ncu <= 0) {
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            ncu <= 0)
            ncu = 256;
        if (dev >= 0 && dev < 64) cus[dev].store(ncu);
    }
    const long tiles = long((g.n0 + MT_X - 1) / MT_X) * long((g.n1 + MT_Y - 1) / MT_Y);
    const long want = long(per_cu) * ncu;
    const long nch = std::max(1L, (want + tiles - 1) / tiles);
    const int zc = int((g.n2 + nch - 1) / nch);
    return std::min(64, std::max(8, zc));
}

TileMap tile_map(const Grid& g, int tile_x, int tile_y, int zc) {
    TileMap tm;
    tm.tiles_x = (g.n0 + tile_x - 1) / tile_x;
    tm.tiles_y = (g.n1 + tile_y - 1) / tile_y;
    tm.zc = zc < g.n2 ? zc : g.n2;
    tm.nchunks = (g.n2 + tm.zc - 1) / tm.zc;
    tm.nblocks = unsigned(tm.tiles_x) * unsigned(tm.tiles_y) * unsigned(tm.nchunks);
    tm.remap = (tm.nblocks % 8u == 0u) ? 1 : 0;
    return tm;
}

template <typename T>
wl_status ns_momentum(const VelField<T>& E, const T* const un[3], T* const f[3], T nu, bool corr,
                      bool allper, const double* dt_dev, hipStream_t s) {
    const Grid& g = E.g;
    const Launch ln = launch_for(g.n0, g.n1, g.n2);
    ProfScope ps(WL_PROF_MOMENTUM, s, cells(g));
    if constexpr (sizeof(T) == 4) {
        if (g.ndim == 3) {
            // blocks per CU the kernel's registers allow (LDS allows 3): the
            // periodic predictor fits 80 VGPRs (6 waves per SIMD), the others 128
            const TileMap tm = tile_map(g, MT_X, MT_Y, momentum_zchunk(g, allper && !corr ? 3 : 2));
#define WL_MT(AP, CR, BF)                                                                      \
    k_momentum_tiled<AP, CR, BF><<<tm.nblocks, MT_T, 0, s>>>(E, un[0], un[1], un[2], f[0], f[1], \
                                                             f[2], nu, dt_dev, tm)
            const bool bf = momentum_buf(g);
            if (allper) {
                if (corr) {
                    if (bf) WL_MT(true, true, true); else WL_MT(true, true, false);
                } else {
                    if (bf) WL_MT(true, false, true); else WL_MT(true, false, false);
                }
            } else {
                if (corr) WL_MT(false, true, false); else WL_MT(false, false, false);
            }
#undef WL_MT
            WL_CHECK_LAUNCH();
            return WL_OK;
        }
    }
#define WL_MOM(AP, CR)                                                                      \
    k_momentum<T, AP, CR><<<ln.grid, ln.block, 0, s>>>(ln.td, E, un[0], un[1], un[2], f[0], f[1], f[2], \
                                                        nu, dt_dev)
    if (allper) {
        if (corr) WL_MOM(true, true); else WL_MOM(true, false);
    } else {
        if (corr) WL_MOM(false, true); else WL_MOM(false, false);
    }
#undef WL_MOM
    WL_CHECK_LAUNCH();
    return WL_OK;
}

wl_status ns_momentum_proj(const VelField<float>& E, const float* const un[3], float* const f[3],
                           float nu, const double* dt_dev, const float* p, float Lc,
                           hipStream_t s) {
    const Grid& g = E.g;
    if (g.ndim != 3 || !(g.per0 && g.per1 && g.per2)) {
        set_error("fused projection needs a periodic 3D grid");
        return WL_ERR_INVALID_ARG;
    }
    ProfScope ps(WL_PROF_MOMENTUM, s, cells(g));
    const TileMap tm = tile_map(g, MT_X, MT_Y, momentum_zchunk(g, 2));
    if (momentum_buf(g))
        k_momentum_tiled_proj<true><<<tm.nblocks, MT_T, 0, s>>>(E, un[0], un[1], un[2], f[0], f[1],
                                                                f[2], nu, dt_dev, tm, p, Lc);
    else
        k_momentum_tiled_proj<false><<<tm.nblocks, MT_T, 0, s>>>(E, un[0], un[1], un[2], f[0], f[1],
                                                                 f[2], nu, dt_dev, tm, p, Lc);
    WL_CHECK_LAUNCH();
    return WL_OK;
}

template <typename T>
wl_status ns_outflow(const Grid& g, const T* ue_x, const T* out_e, const T* out_n, const T* f_x,
                     T Ux, bool corr, const double* dt_dev, T* fout, double* part,
                     hipStream_t s) {
    const int P = g.n1 * g.n2;
    const int nblk = (P + kOutflowThreads - 1) / kOutflowThreads;
    if (corr)
        k_outflow_flux<T, true><<<nblk, kOutflowThreads, 0, s>>>(g, ue_x, out_e, out_n, f_x, Ux,
                                                                 dt_dev, fout, part);
    else
        k_outflow_flux<T, false><<<nblk, kOutflowThreads, 0, s>>>(g, ue_x, out_e, out_n, f_x, Ux,
                                                                  dt_dev, fout, part);
    WL_CHECK_LAUNCH();
    k_outflow_shift<T><<<nblk, kOutflowThreads, 0, s>>>(g, part, nblk, fout);
    WL_CHECK_LAUNCH();
    return WL_OK;
}

template <typename T>
wl_status ns_bdim(const VelField<T>& F, const BdimFields<T>& B, T* const out[3], hipStream_t s,
                  const BodyMotionDev& motion) {
    const Launch ln = launch_for(F.g.n0, F.g.n1, F.g.n2);
    k_bdim<T><<<ln.grid, ln.block, 0, s>>>(ln.td, F, B, out[0], out[1], out[2], motion);
    WL_CHECK_LAUNCH();
    return WL_OK;
}

template <typename T>
wl_status ns_bdim_in_place(const VelField<T>& F, T* const f[3], const BdimFields<T>& B,
                           T* const w[3], hipStream_t s, const BodyMotionDev& motion) {
    if (!B.cflag) {
        set_error("internal: in-place BDIM needs the per-cell flags");
        return WL_ERR_INVALID_ARG;
    }
    const unsigned nb = unsigned((cells(F.g) + kBlock - 1) / kBlock);
    k_bdim_cells<T><<<nb, kBlock, 0, s>>>(F, B, w[0], w[1], w[2], motion);
    WL_CHECK_LAUNCH();
    k_bdim_commit<T><<<nb, kBlock, 0, s>>>(F.g, B.cflag, w[0], w[1], w[2], f[0], f[1], f[2]);
    WL_CHECK_LAUNCH();
    return WL_OK;
}

template <typename T>
wl_status ns_tile_class(const Grid& g, const BdimFields<T>& B, unsigned char* cls, hipStream_t s,
                        unsigned char* cflag) {
    const Launch ln = launch_for(g.n0, g.n1, g.n2);
    k_tile_class<T><<<ln.grid, ln.block, 0, s>>>(ln.td, g, B, cls, cflag);
    WL_CHECK_LAUNCH();
    return WL_OK;
}

template <typename T>
wl_status ns_divergence(const VelField<T>& V, const ProjCoeffs<T>& C, bool unif, double c,
                        const double* dt_dev, T* sigma, double* partial, bool allper,
                        hipStream_t s, const T* p_check, T Lp, size_t* nslots) {
    const Launch ln = launch_for(V.g.n0, V.g.n1, V.g.n2);
    ProfScope ps(WL_PROF_DIVERGENCE, s, cells(V.g));
    if (nslots) *nslots = ln.nblocks();
    if (p_check) {
        if (!allper || !unif || V.g.ndim != 3) {
            set_error("internal: the fused first residual check needs a periodic uniform 3D grid");
            return WL_ERR_INVALID_ARG;
        }
        const TileMap tm = div_check_map(V.g);
        if (tm.nblocks > 0) {
            if (sizeof(T) == 4 && buffer_addressing(V.g))
                k_div_check<T, sizeof(T) == 4><<<tm.nblocks, DC_T, 0, s>>>(tm, V, c, dt_dev, sigma,
                                                                           partial, p_check, Lp);
            else
                k_div_check<T, false><<<tm.nblocks, DC_T, 0, s>>>(tm, V, c, dt_dev, sigma, partial,
                                                                  p_check, Lp);
            if (nslots) *nslots = tm.nblocks;
        } else {
            k_divergence<T, true, true, true><<<ln.grid, ln.block, 0, s>>>(
                ln.td, V, C, c, dt_dev, sigma, partial, p_check, Lp);
        }
        WL_CHECK_LAUNCH();
        return WL_OK;
    }
#define WL_DIV(AP, UN)                                                                          \
    k_divergence<T, AP, UN, false><<<ln.grid, ln.block, 0, s>>>(ln.td, V, C, c, dt_dev, sigma, \
                                                                partial, nullptr, T(0))
    if (allper) {
        if (unif) WL_DIV(true, true); else WL_DIV(true, false);
    } else {
        if (unif) WL_DIV(false, true); else WL_DIV(false, false);
    }
#undef WL_DIV
    WL_CHECK_LAUNCH();
    return WL_OK;
}

template <typename T>
wl_status ns_project(const VelField<T>& V, const T* p, const ProjCoeffs<T>& C, bool unif, double c,
                     const double* dt_dev, T* const out[3], bool cfl, double* partial, bool allper,
                     hipStream_t s) {
    const Launch ln = launch_for(V.g.n0, V.g.n1, V.g.n2);
    ProfScope ps(WL_PROF_PROJECT, s, cells(V.g));
#define WL_PRJ(AP, UN, CF)                                                                      \
    k_project<T, AP, UN, CF><<<ln.grid, ln.block, 0, s>>>(ln.td, V, p, C, c, dt_dev, out[0], out[1], \
                                                           out[2], partial)
    if (allper) {
        if (unif) {
            if (cfl) WL_PRJ(true, true, true); else WL_PRJ(true, true, false);
        } else {
            if (cfl) WL_PRJ(true, false, true); else WL_PRJ(true, false, false);
        }
    } else {
        if (unif) {
            if (cfl) WL_PRJ(false, true, true); else WL_PRJ(false, true, false);
        } else {
            if (cfl) WL_PRJ(false, false, true); else WL_PRJ(false, false, false);
        }
    }
#undef WL_PRJ
    WL_CHECK_LAUNCH();
    return WL_OK;
}

template <typename T>
wl_status ns_cfl(const VelField<T>& V, bool allper, double* partial, hipStream_t s) {
    const Launch ln = launch_for(V.g.n0, V.g.n1, V.g.n2);
    if (allper)
        k_cfl<T, true><<<ln.grid, ln.block, 0, s>>>(ln.td, V, partial);
    else
        k_cfl<T, false><<<ln.grid, ln.block, 0, s>>>(ln.td, V, partial);
    WL_CHECK_LAUNCH();
    return WL_OK;
}

wl_status ns_dt_from_max(const double* partial, size_t nslots, double cfl, double visc,
                         double* dt_dev, double* max_dev, hipStream_t s, const MailboxPost* post) {
    k_dt_from_max<<<1, 1024, 0, s>>>(partial, nslots, cfl, visc, dt_dev, max_dev,
                                     post ? *post : MailboxPost{});
    WL_CHECK_LAUNCH();
    return WL_OK;
}

wl_status ns_set_scalar(double* p, double v, hipStream_t s) {
    k_set_scalar<<<1, 64, 0, s>>>(p, v);
    WL_CHECK_LAUNCH();
    return WL_OK;
}

#define WL_INST(T)                                                                               \
    template wl_status ns_tile_class<T>(const Grid&, const BdimFields<T>&, unsigned char*,        \
                                        hipStream_t, unsigned char*);                             \
    template wl_status ns_measure<T>(const Grid&, const BodyDev&, const int*,                     \
                                     const MeasureOut<T>&, hipStream_t);                          \
    template wl_status ns_momentum<T>(const VelField<T>&, const T* const*, T* const*, T, bool,   \
                                      bool, const double*, hipStream_t);                          \
    template wl_status ns_outflow<T>(const Grid&, const T*, const T*, const T*, const T*, T, bool, \
                                     const double*, T*, double*, hipStream_t);                    \
    template wl_status ns_bdim<T>(const VelField<T>&, const BdimFields<T>&, T* const*,            \
                                  hipStream_t, const BodyMotionDev&);                             \
    template wl_status ns_bdim_in_place<T>(const VelField<T>&, T* const*, const BdimFields<T>&,   \
                                           T* const*, hipStream_t, const BodyMotionDev&);         \
    template wl_status ns_divergence<T>(const VelField<T>&, const ProjCoeffs<T>&, bool, double,  \
                                        const double*, T*, double*, bool, hipStream_t, const T*,  \
                                        T, size_t*);                                              \
    template wl_status ns_project<T>(const VelField<T>&, const T*, const ProjCoeffs<T>&, bool,    \
                                     double, const double*, T* const*, bool, double*, bool,        \
                                     hipStream_t);                                                \
    template wl_status ns_cfl<T>(const VelField<T>&, bool, double*, hipStream_t);          \
    template wl_status ns_init_velocity<T>(const Grid&, const int*, const double*, T* const*,   \
                                           hipStream_t);
WL_INST(float)
WL_INST(double)
#undef WL_INST

}  // namespace wl
