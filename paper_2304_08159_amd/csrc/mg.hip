// Matrix-free geometric multigrid for the BDIM-modified pressure Poisson
// system (paper Sec. 2: GMG with a solution time linear in the cell count;
// the operator is fixed by the gradient loop u[I,i] -= coeff*(p[I]-p[I-del(i)])).
//
// One thread per cell; every kernel is an HBM sweep with neighbour reads
// served by L1/L2.  Damped Jacobi (w = 2d/(2d+1), two pre- and two
// post-sweeps), residual fused with sum-restriction, cell-centred linear
// prolongation added in place before the post-sweeps, a one-workgroup FP64 CG on
// the coarsest level, and FP64 fixed-order reductions for the norms and the
// active-set mean.  On 3D levels whose x and y extents are multiples of 8
// each pair of sweeps runs as one LDS-tiled kernel that keeps the
// intermediate iterate on chip.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <type_traits>

#include "wl_cg.h"
#include "wl_device.h"
#include "wl_jacobi.h"

namespace wl {

// ------------------------------------------------------------ host shapes
static unsigned pow2ceil(unsigned v) {
    unsigned p = 1;
    while (p < v) p <<= 1;
    return p;
}

// Target block count of a tiled launch (8 per CU on 256 CUs); WL_TILE_BLOCKS
// overrides it for tuning.
static unsigned target_blocks() {
    static const unsigned v = [] {
        const char* e = std::getenv("WL_TILE_BLOCKS");
        const long t = e ? std::atol(e) : 0;
        return t > 0 ? unsigned(t) : 2048u;
    }();
    return v;
}

Launch launch_for(int n0, int n1, int n2) {
    Launch l;
    unsigned bx = pow2ceil(unsigned(n0));
    if (bx > 64) bx = 64;
    int lbx = 0;
    while ((1u << lbx) < bx) ++lbx;
    const unsigned by = kBlock / bx;
    const int tx = int((unsigned(n0) + bx - 1) / bx);
    const int ty = int((unsigned(n1) + by - 1) / by);
    const size_t cols = size_t(tx) * ty;
    size_t zc = (cols * size_t(n2) + target_blocks() - 1) / target_blocks();
    if (zc < 1) zc = 1;
    if (zc > 64) zc = 64;
    if (zc > size_t(n2)) zc = size_t(n2);
    const unsigned chunks = unsigned((size_t(n2) + zc - 1) / zc);
    l.td.lbx = lbx;
    l.td.tx = tx;
    l.td.ty = ty;
    l.td.zc = int(zc);
    l.td.nb = unsigned(cols) * chunks;
    l.td.remap = (l.td.nb % 8u == 0u) ? 1 : 0;
    l.block = dim3(kBlock, 1, 1);
    l.grid = dim3(l.td.nb, 1, 1);
    return l;
}

size_t reduce_slots_for(const Grid& g) { return launch_for(g.n0, g.n1, g.n2).nblocks(); }

int auto_levels(int ndim, const int n[3], int requested) {
    int m[3] = {n[0], n[1], n[2]};
    int count = 1;
    for (;;) {
        if (requested > 0 && count >= requested) break;
        bool even = true, big = true;
        for (int d = 0; d < ndim; ++d) {
            if (m[d] % 2) even = false;
            if (m[d] / 2 < 4) big = false;
        }
        if (!even) break;
        if (requested <= 0 && !big) break;
        for (int d = 0; d < ndim; ++d) m[d] /= 2;
        ++count;
        if (count >= kMaxLevels) break;
    }
    return count;
}

// Process-wide choice of the fused two-sweep kernels (wl_set_fused_sweeps),
// taken by each hierarchy when it is laid out.
static std::atomic<int> g_pairs{1};

// Levels smaller than this use separate sweeps in mode 1 (default 0: every
// eligible level is fused; WL_PAIR_MIN_CELLS overrides it for tuning).
static size_t pair_min_cells() {
    static const size_t v = [] {
        const char* e = std::getenv("WL_PAIR_MIN_CELLS");
        const long t = e ? std::atol(e) : -1;
        return t >= 0 ? size_t(t) : size_t(0);
    }();
    return v;
}

// WL_DIRECT_COARSE=0 keeps the coarsest level's CG where its inverse would
// solve it (read whenever the coefficients change, so that the two can be
// compared within one process).
static bool direct_coarse_enabled() {
    const char* e = std::getenv("WL_DIRECT_COARSE");
    return !(e && std::atoi(e) == 0);
}

// Target workgroup count of a fused launch (WL_PAIR_BLOCKS overrides it).
static unsigned pair_blocks() {
    static const unsigned v = [] {
        const char* e = std::getenv("WL_PAIR_BLOCKS");
        const long t = e ? std::atol(e) : 0;
        return t > 0 ? unsigned(t) : 1024u;
    }();
    return v;
}

static Launch launch_pairs(const Grid& g);
// Workgroups of the fused-pair tiling of a 3D level (0 when it does not fit).
static unsigned pair_class_slots(const Grid& g);

// Fused pairs on non-uniform or non-periodic levels (WL_GEN_PAIRS=0 turns
// them off, for measurement; the iterates are the same either way).
static bool gen_pairs() {
    static const bool v = [] {
        const char* e = std::getenv("WL_GEN_PAIRS");
        return !(e && std::atoi(e) == 0);
    }();
    return v;
}

// Smallest non-uniform level whose pairs run as two launches, one per kind
// of workgroup (WL_GEN_PAIR_MIN_CELLS overrides it); smaller levels run both
// kinds in one launch (k_smooth_pair mode 3), where a second launch would
// cost more than the shared register budget.
static size_t gen_pair_min_cells() {
    static const size_t v = [] {
        const char* e = std::getenv("WL_GEN_PAIR_MIN_CELLS");
        const long t = e ? std::atol(e) : -1;
        return t >= 0 ? size_t(t) : (size_t(1) << 22);
    }();
    return v;
}

// Largest non-uniform level below gen_pair_min_cells() that runs its pairs in
// one launch (WL_PAIR3_MAX_CELLS overrides it); the levels between keep
// separate sweeps.
static size_t pair3_max_cells() {
    static const size_t v = [] {
        const char* e = std::getenv("WL_PAIR3_MAX_CELLS");
        const long t = e ? std::atol(e) : -1;
        return t >= 0 ? size_t(t) : (size_t(1) << 22);
    }();
    return v;
}

// Largest level that the one-workgroup V-cycle tail takes (WL_TAIL_CELLS
// overrides it; 0 turns the tail off): from 16^3 down, the per-level
// launches cost more than one workgroup's pass over the level.
static size_t tail_cells() {
    static const size_t v = [] {
        const char* e = std::getenv("WL_TAIL_CELLS");
        const long t = e ? std::atol(e) : -1;
        return t >= 0 ? size_t(t) : size_t(4096);
    }();
    return v;
}

// Process-wide smoother of the multigrid levels (wl_set_smoother), taken by
// each hierarchy when it is laid out: 0 damped Jacobi, 1 conjugate gradients.
static std::atomic<int> g_smoother{0};

template <typename T>
void carve_hierarchy(Carver& c, Hierarchy<T>& h, int ndim, const int n[3], const int per[3],
                     int nlev, bool alloc_fine_x) {
    h.nlev = nlev;
    h.smoother = g_smoother.load(std::memory_order_relaxed);
    // the fused two-sweep kernels are Jacobi sweeps
    h.pairs = h.smoother == 0 ? g_pairs.load(std::memory_order_relaxed) : 0;
    h.omega = 2.0 * ndim / (2.0 * ndim + 1.0);
    int m[3] = {n[0], n[1], n[2]};
    for (int l = 0; l < nlev; ++l) {
        Level<T>& L = h.lev[l];
        L.g = Grid{m[0], m[1], m[2], per[0], per[1], per[2], ndim};
        const size_t N = cells(L.g);
        for (int d = 0; d < 3; ++d) L.L[d] = c.take<T>(N);
        L.x[0] = (l > 0 || alloc_fine_x) ? c.take<T>(N) : nullptr;
        L.x[1] = c.take<T>(N);
        L.b = c.take<T>(N);
        L.cls = c.take<unsigned char>(reduce_slots_for(L.g));
        L.cls_pairs = c.take<unsigned char>(launch_pairs(L.g).nblocks());
        const unsigned fp = pair_class_slots(L.g);
        L.cls_fp = fp ? c.take<unsigned char>(fp) : nullptr;
        L.fp_list = fp ? c.take<unsigned>(size_t(fp) + 1) : nullptr;
        if (h.smoother == 1 && l < nlev - 1) {
            L.cr = c.take<T>(N);
            L.cp = c.take<T>(N);
            L.cq = c.take<T>(N);
            L.cd = c.take<T>(N);
            L.cgs = c.take<double>(8);
        }
        for (int d = 0; d < ndim; ++d) m[d] /= 2;
    }
    if (h.smoother == 1) {
        const Grid& g0 = h.lev[0].g;
        h.cgpart = c.take<double>(5 * reduce_slots_for(g0));
    }
    const size_t Nc = cells(h.lev[nlev - 1].g);
    if (Nc <= size_t(kDirectMax)) {
        h.cinv = c.take<double>(Nc * Nc);
        h.cinv_ok = c.take<int>(1);
    }
}

template void carve_hierarchy<float>(Carver&, Hierarchy<float>&, int, const int*, const int*, int,
                                     bool);
template void carve_hierarchy<double>(Carver&, Hierarchy<double>&, int, const int*, const int*,
                                      int, bool);

// ---------------------------------------------------------------- kernels

// One damped-Jacobi sweep  x_out = x - w (b - A x) / D  (zero on inactive
// cells, D = 0); with xout null only the norms are formed.  wgt is w, or on a
// uniform level the factor w / D of its single D.  With bshift, b is the raw right-hand side and the sweep uses
// its projection (b - mean) on active cells, 0 elsewhere, mean = *bshift;
// FIRST with bproj also stores that projection.
// NORM: per-block partial sums of r^2 (and, FIRST, of the projected b^2) in
// FP64.
template <typename T, int XM, bool UNIF, bool NORM, bool FIRST>
__global__ __launch_bounds__(kBlock) void k_smooth(TileDev TL, Grid g, XAccess<T, XM> X, Coeffs<T> C,
                                                   const T* __restrict__ b, T wgt,
                                                   T* __restrict__ xout,
                                                   double* __restrict__ partial,
                                                   const double* __restrict__ bshift,
                                                   T* __restrict__ bproj) {
    __shared__ double lds[8];
    const Span sp = tile_span(TL, g.n0, g.n1, g.n2);
    const int i = sp.i, j = sp.j;
    double r2 = 0.0, b2 = 0.0;
    if (i < g.n0 && j < g.n1 && sp.z0 < sp.z1) {
        // The thread walks its (i, j) column up the z chunk: x / y neighbour
        // offsets are fixed along it, the lower z neighbour and coefficient
        // are carried from the previous cell, and every load of a cell is
        // issued before any of them is used.  Non-periodic boundaries point
        // at the cell itself with a zero coefficient.
        const unsigned n0 = unsigned(g.n0), plane = n0 * unsigned(g.n1);
        const bool d3 = g.ndim == 3;
        const int ixm = i > 0 ? i - 1 : (g.per0 ? g.n0 - 1 : i);
        const int ixp = i < g.n0 - 1 ? i + 1 : (g.per0 ? 0 : i);
        const int jym = j > 0 ? j - 1 : (g.per1 ? g.n1 - 1 : j);
        const int jyp = j < g.n1 - 1 ? j + 1 : (g.per1 ? 0 : j);
        const bool hxu = i < g.n0 - 1 || g.per0, hyu = j < g.n1 - 1 || g.per1;
        const int oxm = ixm - i, oxp = ixp - i;
        const int oym = (jym - j) * int(n0), oyp = (jyp - j) * int(n0);
        auto xv = [&](unsigned idx) -> T { return XM == XM_ZERO ? T(0) : X.x[idx]; };
        const bool shift = bshift != nullptr;
        const T mean = shift ? T(*bshift) : T(0);
        // uniform level: one D, the same for every cell
        T Du = T(0);
        Du += C.Lc + C.Lc;
        Du += C.Lc + C.Lc;
        if (d3) Du += C.Lc + C.Lc;
        // a block of class 0 takes its coefficients from the position
        const bool walled = !UNIF && C.cls && C.cls[block_linear()] == 0;
        const int k0 = sp.z0;
        unsigned id = unsigned(i) + n0 * unsigned(j) + plane * unsigned(k0);
        // z neighbours of the first cell
        T xzl = T(0), xI = xv(id), Lzl = T(0);
        if (d3) {
            const int km = k0 > 0 ? k0 - 1 : (g.per2 ? g.n2 - 1 : k0);
            xzl = xv(id + unsigned(km - k0) * plane);
            if (!UNIF) Lzl = walled ? ((k0 == 0 && !g.per2) ? T(0) : C.Lc) : C.L2[id];
        }
        for (int k = k0; k < sp.z1; ++k, id += plane) {
            // upper z neighbour (carried up as the next centre)
            T xzu = T(0), Lzu = T(0);
            bool hzu = false;
            unsigned idu = id;
            int ku = k;
            if (d3) {
                hzu = k < g.n2 - 1 || g.per2;
                ku = k < g.n2 - 1 ? k + 1 : (g.per2 ? 0 : k);
                idu = id + unsigned(ku - k) * plane;
                xzu = xv(idu);
            }
            const T xxl = xv(id + oxm), xxu = xv(id + oxp);
            const T xyl = xv(id + oym), xyu = xv(id + oyp);
            T bv = b[id];
            T Lxl, Lxu, Lyl, Lyu;
            if (UNIF) {
                Lxl = Lxu = Lyl = Lyu = Lzu = C.Lc;
                Lzl = C.Lc;
            } else if (walled) {
                T zl;
                walled_faces<T>(g, i, j, k, C.Lc, Lxl, Lxu, Lyl, Lyu, zl, Lzu);
            } else {
                Lxl = C.L0[id];
                Lxu = hxu ? C.L0[id + oxp] : T(0);
                Lyl = C.L1[id];
                Lyu = hyu ? C.L1[id + oyp] : T(0);
                if (d3) Lzu = hzu ? C.L2[idu] : T(0);
            }
            T Ax, D;
            if (UNIF) {
                Ax = jacobi_ax_uniform(xI, xxl, xxu, xyl, xyu, xzl, xzu, C.Lc, d3);
                D = Du;
            } else {
                jacobi_terms(xI, xxl, xxu, xyl, xyu, xzl, xzu, Lxl, Lxu, Lyl, Lyu, Lzl, Lzu, d3, Ax,
                             D);
            }
            bv = jacobi_rhs(bv, D > T(0), shift, mean);
            if (FIRST && bproj) bproj[id] = bv;
            const T r = bv - Ax;
            if (xout)
                xout[id] = UNIF ? jacobi_new_scaled(xI, r, D > T(0), wgt)
                                : jacobi_new(xI, r, D, wgt);
            if (NORM) {
                r2 += double(r) * double(r);
                if (FIRST) b2 += double(bv) * double(bv);
            }
            xzl = xI;
            xI = xzu;
            Lzl = Lzu;
        }
    }
    if (NORM) {
        double s, sb;
        block_sum2(r2, b2, lds, s, sb);
        if (threadIdx.x == 0) {
            partial[2 * block_linear()] = s;
            partial[2 * block_linear() + 1] = sb;
        }
    }
}

// ------------------------------------------------- fused pair of sweeps
// Two damped-Jacobi sweeps in one pass over a uniform, fully periodic 3D
// level.  A workgroup owns a 64 x 8 column tile and walks a chunk of z planes;
// per plane it computes the first sweep on the tile widened by one cell (its
// input staged in LDS on the tile widened by two), keeps those values in LDS
// for the x / y neighbours and in registers for the z neighbours, and writes
// only the second sweep.  The widened cells are recomputed by the
// neighbouring workgroups with the same operations, so the result is bitwise
// that of two separate sweeps while the intermediate iterate never reaches
// memory (FP32: 12 instead of 24 bytes per cell for the pair).
// Tiles are TX x 8 cells (TX = 64, 32, 16 or 8, the widest dividing the
// level's x extent), one thread per cell.
constexpr int kPairTY = 8;
template <int TX>
struct PairShape {
    static constexpr int T = TX * kPairTY;                  // threads
    static constexpr int HX = TX + 2, HY = kPairTY + 2;     // first-sweep region
    static constexpr int GX = TX + 4, GY = kPairTY + 4;     // input region
    static constexpr int R1 = HX * HY - T;                  // first-sweep ring cells
    static constexpr int R2 = GX * GY - HX * HY;            // input ring cells
    static_assert(R1 <= T && R2 <= T, "one ring cell per thread at most");
};
constexpr int kPairDepth = 1;  // planes of loads in flight per thread

struct PairTile {
    int tx, ty;   // tiles along x and y
    int zc;       // z planes per workgroup
    unsigned nb;  // workgroups
    int remap;    // XCD-contiguous tile order (nb % 8 == 0)
    int split;    // MODE 2: workgroups per chunk (each walks zc / split planes)
};

// MODE 0: a uniform, fully periodic level (wD = w / D).  MODE 1 / 2: a
// non-uniform level with any boundaries, in two launches over the same
// workgroups: MODE 1 runs the workgroups whose widened region is of class 0
// (see k_pair_class; face coefficients from the position), MODE 2 the others
// (coefficients read), so each instance keeps its own register budget:
// MODE 1 runs over all workgroups and leaves the class-1 ones at once, MODE 2
// over the list fpl of the class-1 workgroups (fpl[P.nb] of them), each
// chunk walked by P.split workgroups, a part of the planes each (the parts
// recompute the first sweep of one plane on either side), so that the few
// body chunks do not make a long tail on a handful of CUs.  Coordinates outside a non-periodic direction are
// clamped (the cells there are only ever weighted by a zero face
// coefficient, so any finite value serves), each cell has its own D, and wD
// is the damping w.  The arithmetic per cell is that of k_smooth's
// non-uniform path, so the result is again bitwise that of two separate
// sweeps.
// MODE 3: both kinds of workgroup in one launch over all of them, each
// taking its class's walk over its whole chunk: small levels, where a second
// launch costs more than the shared register budget.
// NM (MODE 1 / 2): the pair also measures the residual of its input, as a
// measuring check would: per-workgroup FP64 partial sums of r^2 (r = b - A x
// on the tile's cells of its own planes, from the first sweep) and, NM = 2,
// of the projected b^2, in slot blockIdx.x (MODE 1) or P.nb + blockIdx.x
// (MODE 2); workgroups with nothing to do store zeros.
template <typename T, int XM, int TX, int MODE, int NM = 0>
__global__ __launch_bounds__(PairShape<TX>::T) void k_smooth_pair(PairTile P, Grid g, XAccess<T, XM> X,
                                                              Coeffs<T> Cf, const T* __restrict__ b,
                                                              T wD, T* __restrict__ xout,
                                                              const double* __restrict__ bshift,
                                                              const unsigned* __restrict__ fpl,
                                                              double* __restrict__ partial) {
    using Sh = PairShape<TX>;
    const T Lc = Cf.Lc;
    constexpr bool GEN = MODE != 0;
    // MODE 2: part `part` of the chunk of listed workgroup blockIdx.x / split
    unsigned wg = blockIdx.x;
    int part = 0;
    const unsigned pslot = MODE == 2 ? P.nb + blockIdx.x : blockIdx.x;
    auto no_partials = [&]() {
        if (NM != 0 && threadIdx.x == 0) {
            partial[2 * pslot] = 0.0;
            partial[2 * pslot + 1] = 0.0;
        }
    };
    if constexpr (MODE == 1) {
        if (Cf.cls[wg] != 0) {  // the MODE 2 launch takes it
            no_partials();
            return;
        }
    } else if constexpr (MODE == 2) {
        const unsigned q = blockIdx.x / unsigned(P.split);
        if (q >= fpl[P.nb]) {  // the grid covers the largest count met
            no_partials();
            return;
        }
        wg = fpl[q];
        part = int(blockIdx.x % unsigned(P.split));
    }
    constexpr int kPairTX = TX, kPairThreads = Sh::T, kPairHX = Sh::HX, kPairHY = Sh::HY;
    constexpr int kPairGX = Sh::GX, kPairRing1 = Sh::R1, kPairRing2 = Sh::R2;
    __shared__ T s0[2][Sh::GY * Sh::GX];  // input plane, tile widened by two
    __shared__ T s1[2][Sh::HY * Sh::HX];  // first-sweep plane, tile widened by one
    unsigned blk = wg;
    if (P.remap) blk = (blk & 7u) * (P.nb >> 3) + (blk >> 3);
    const int tix = int(blk % unsigned(P.tx));
    blk /= unsigned(P.tx);
    const int tiy = int(blk % unsigned(P.ty));
    int z0 = int(blk / unsigned(P.ty)) * P.zc;
    int z1 = min(z0 + P.zc, g.n2);
    if constexpr (MODE == 2) {
        const int zs = (P.zc + P.split - 1) / P.split;
        z0 += part * zs;
        z1 = min(z0 + zs, z1);
        if (z0 >= z1) {
            no_partials();
            return;
        }
    }
    double nr2 = 0.0, nb2 = 0.0;  // NM: this thread's residual / rhs sums
    const int i0 = tix * kPairTX, j0 = tiy * kPairTY;
    const int t = int(threadIdx.x);
    const unsigned n0 = unsigned(g.n0), plane = n0 * unsigned(g.n1);
    const bool shift = bshift != nullptr;
    const T mean = shift ? T(*bshift) : T(0);
    // A cell this thread handles: periodic grid column and position in the
    // input-region LDS plane.
    struct Slot {
        unsigned col;
        int q;
        int ci, cj;  // grid coordinates of the column
    };
    auto slot = [&](int gx, int gy) -> Slot {
        int i = i0 + gx - 2, j = j0 + gy - 2;
        if (!GEN || g.per0)
            i = i < 0 ? i + g.n0 : (i >= g.n0 ? i - g.n0 : i);
        else
            i = min(max(i, 0), g.n0 - 1);
        if (!GEN || g.per1)
            j = j < 0 ? j + g.n1 : (j >= g.n1 ? j - g.n1 : j);
        else
            j = min(max(j, 0), g.n1 - 1);
        return Slot{unsigned(i) + n0 * unsigned(j), gy * kPairGX + gx, i, j};
    };
    // A: the thread's own tile cell; B: a cell of the first-sweep ring (the
    // first kPairRing1 threads); C: a cell of the input ring (the last
    // kPairRing2 threads), needed only as an x / y neighbour.
    const int ax = t % kPairTX, ay = t / kPairTX;
    const Slot A = slot(ax + 2, ay + 2);
    const int hA = (ay + 1) * kPairHX + ax + 1;
    const bool hasB = t < kPairRing1;
    const bool hasC = t >= kPairThreads - kPairRing2;
    Slot B = A, C = A;
    int hB = hA;
    if (hasB) {
        int hx, hy;
        ring_cell(t, kPairTX, kPairTY, hx, hy);
        B = slot(hx + 1, hy + 1);
        hB = hy * kPairHX + hx;
    }
    if (hasC) {
        int gx, gy;
        ring_cell(t - (kPairThreads - kPairRing2), kPairHX, kPairHY, gx, gy);
        C = slot(gx, gy);
    }
    // w: a plane index already wrapped into [0, n2)
    // plane bases are workgroup-uniform, the per-thread offsets fixed
    // FP32: buffer loads with the plane offset in a scalar register and the
    // thread's fixed column offset in a vector register (no per-load address
    // arithmetic; the descriptors bound each array)
    const unsigned bytes = unsigned(cells(g) * sizeof(T));
    auto rsrc = [](const T* p, unsigned nbytes) {
        return __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(p), 0, int(nbytes), 0x00020000);
    };
    const auto dX = rsrc(XM == XM_ZERO ? b : X.x, bytes);
    const auto dB = rsrc(b, bytes);
    auto at = [&](const T* base, const __amdgpu_buffer_rsrc_t& r, unsigned elem,
                  unsigned off) -> T {
        if constexpr (sizeof(T) == 4)
            return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(
                                             r, int(off * 4u), int(elem * 4u), 0));
        else
            return base[size_t(elem) + off];
    };
    auto ld = [&](const Slot& S, int w) -> T {
        return XM == XM_ZERO ? T(0) : at(X.x, dX, unsigned(w) * plane, S.col);
    };
    auto ldb = [&](const Slot& S, int w) -> T { return at(b, dB, unsigned(w) * plane, S.col); };
    auto wrap = [&](int p) {
        p %= g.n2;
        return p < 0 ? p + g.n2 : p;
    };
    auto next = [&](int w) { return w + 1 == g.n2 ? 0 : w + 1; };
    // modes 1 and 2 keep plane numbers unwrapped and map them at each load
    // (wrapped on a periodic z, clamped otherwise); mode 0 wraps as it walks
    auto zmap = [&](int p) { return g.per2 ? wrap(p) : min(max(p, 0), g.n2 - 1); };
    auto zfirst = [&](int p) { return GEN ? p : wrap(p); };
    auto znext = [&](int w) { return GEN ? w + 1 : next(w); };
    auto zld = [&](int w) { return GEN ? zmap(w) : w; };
    // one D for the whole level; right-hand sides are shifted once, when
    // they become current, and serve both sweeps
    T Du = T(0);
    Du += Lc + Lc;
    Du += Lc + Lc;
    Du += Lc + Lc;
    const bool act = Du > T(0);
    auto rhs = [&](T v) { return jacobi_rhs(v, act, shift, mean); };
    // first sweep at input-region position q of plane S0 (bv shifted)
    auto sweep1 = [&](const T* S0, int q, T xI, T xzl, T xzu, T bv) -> T {
        T xxl = T(0), xxu = T(0), xyl = T(0), xyu = T(0);
        if (XM != XM_ZERO) {
            xxl = S0[q - 1];
            xxu = S0[q + 1];
            xyl = S0[q - kPairGX];
            xyu = S0[q + kPairGX];
        }
        const T Ax = jacobi_ax_uniform(xI, xxl, xxu, xyl, xyu, xzl, xzu, Lc, true);
        return jacobi_new_scaled(xI, bv - Ax, act, wD);
    };
    // second sweep at first-sweep position h of plane S1 (bv shifted)
    auto sweep2 = [&](const T* S1, int h, T xI, T xzl, T xzu, T bv) -> T {
        const T Ax = jacobi_ax_uniform(xI, S1[h - 1], S1[h + 1], S1[h - kPairHX], S1[h + kPairHX],
                                       xzl, xzu, Lc, true);
        return jacobi_new_scaled(xI, bv - Ax, act, wD);
    };
    // mt is the mode of the walk: 1 a workgroup of class 0 (coefficients
    // from the position), 2 one that reads them.
    // Face coefficients of the column S at plane k (k inside the grid).
    auto faces = [&](auto mt, const Slot& S, int k, T& Lxl, T& Lxu, T& Lyl, T& Lyu, T& Lzl,
                     T& Lzu) {
        if constexpr (decltype(mt)::value == 1) {
            walled_faces<T>(g, S.ci, S.cj, k, Lc, Lxl, Lxu, Lyl, Lyu, Lzl, Lzu);
            return;
        }
        const size_t id = size_t(S.col) + size_t(k) * size_t(plane);
        const bool hxu = S.ci < g.n0 - 1 || g.per0, hyu = S.cj < g.n1 - 1 || g.per1;
        const bool hzu = k < g.n2 - 1 || g.per2;
        const long long oxp = S.ci < g.n0 - 1 ? 1 : 1 - (long long)g.n0;
        const long long oyp = S.cj < g.n1 - 1 ? (long long)n0 : -(long long)n0 * (g.n1 - 1);
        const long long ozp =
            k < g.n2 - 1 ? (long long)plane : -(long long)plane * (g.n2 - 1);
        Lxl = Cf.L0[id];
        Lxu = hxu ? Cf.L0[(long long)id + oxp] : T(0);
        Lyl = Cf.L1[id];
        Lyu = hyu ? Cf.L1[(long long)id + oyp] : T(0);
        Lzl = Cf.L2[id];
        Lzu = hzu ? Cf.L2[(long long)id + ozp] : T(0);
    };
    // Mode 1: every cell is active and D = (6 - nb) Lc exactly, nb the
    // cell's non-periodic domain-boundary faces, so w / D is one of four
    // values, formed once by the same division.
    T tb[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) tb[q] = wD / (T(6 - q) * Lc);
    auto wd_walled = [&](const Slot& S, int k) -> T {
        const int nb = int(S.ci == 0 && !g.per0) + int(S.ci == g.n0 - 1 && !g.per0) +
                       int(S.cj == 0 && !g.per1) + int(S.cj == g.n1 - 1 && !g.per1) +
                       int(k == 0 && !g.per2) + int(k == g.n2 - 1 && !g.per2);
        return nb == 0 ? tb[0] : (nb == 1 ? tb[1] : (nb == 2 ? tb[2] : tb[3]));
    };
    // x - (w / D) r as jacobi_new forms it
    auto update = [&](auto mt, const Slot& S, int k, T xI, T r, T D) -> T {
        if constexpr (decltype(mt)::value == 1)
            return xI - wd_walled(S, k) * r;
        else
            return jacobi_new(xI, r, D, wD);
    };
    // First sweep of column S at plane k (input-region position S.q of S0);
    // bv comes in raw and leaves shifted.
    // (Mode 2 passes the coefficients it loaded at the start of the step in
    // F; mode 1 forms them here.)
    auto coef = [&](auto mt, const Slot& S, int k, const T (&F)[6], T& Lxl, T& Lxu, T& Lyl,
                    T& Lyu, T& Lzl, T& Lzu) {
        if constexpr (decltype(mt)::value == 2) {
            Lxl = F[0];
            Lxu = F[1];
            Lyl = F[2];
            Lyu = F[3];
            Lzl = F[4];
            Lzu = F[5];
        } else {
            faces(mt, S, k, Lxl, Lxu, Lyl, Lyu, Lzl, Lzu);
        }
    };
    auto sweep1g = [&](auto mt, const T* S0, const Slot& S, int k, T xI, T xzl, T xzu,
                       T& bv, const T (&F)[6], T& rr) -> T {
        T xxl = T(0), xxu = T(0), xyl = T(0), xyu = T(0);
        if (XM != XM_ZERO) {
            xxl = S0[S.q - 1];
            xxu = S0[S.q + 1];
            xyl = S0[S.q - kPairGX];
            xyu = S0[S.q + kPairGX];
        }
        T Lxl, Lxu, Lyl, Lyu, Lzl, Lzu, Ax, D;
        coef(mt, S, k, F, Lxl, Lxu, Lyl, Lyu, Lzl, Lzu);
        jacobi_terms(xI, xxl, xxu, xyl, xyu, xzl, xzu, Lxl, Lxu, Lyl, Lyu, Lzl, Lzu, true, Ax, D);
        bv = jacobi_rhs(bv, decltype(mt)::value == 1 || D > T(0), shift, mean);
        rr = bv - Ax;
        return update(mt, S, k, xI, rr, D);
    };
    // Second sweep of column S at plane k (first-sweep position h of S1; bv
    // already shifted).
    auto sweep2g = [&](auto mt, const T* S1, int h, const Slot& S, int k, T xI, T xzl, T xzu,
                       T bv, const T (&F)[6]) -> T {
        T Lxl, Lxu, Lyl, Lyu, Lzl, Lzu, Ax, D;
        coef(mt, S, k, F, Lxl, Lxu, Lyl, Lyu, Lzl, Lzu);
        jacobi_terms(xI, S1[h - 1], S1[h + 1], S1[h - kPairHX], S1[h + kPairHX], xzl, xzu, Lxl,
                     Lxu, Lyl, Lyu, Lzl, Lzu, true, Ax, D);
        return update(mt, S, k, xI, bv - Ax, D);
    };
    // Step s computes the first sweep on plane s and the second on plane
    // s - 1, for s = z0 - 1 .. z1, and issues the loads of plane s + 1 + Dp.
    // Per-plane values live in register rings indexed by plane (mod R); the
    // loop is unrolled R times so that the indices are compile-time and an
    // in-flight load is never copied before its use.
    //   xA, xB: inputs of slots A, B (planes s - 1 .. s + 1 in use)
    //   rA, rB: right-hand sides (shifted when they become current; A keeps
    //           plane s - 1 for the second sweep)
    //   xC:     input of slot C at plane s
    //   yA:     A's first-sweep values (planes s - 2 .. s)
    // The whole walk, for one mode (0: the uniform kernel); a workgroup runs
    // the instance of its class, so no cell branches on it.
    auto run = [&](auto mt) {
    constexpr int Dp = kPairDepth;
    constexpr int R = Dp + 3;
    static_assert(R % 2 == 0, "the LDS buffers alternate with the ring index");
    T xA[R] = {}, xB[R] = {}, rA[R] = {}, rB[R] = {}, xC[R] = {}, yA[R] = {};
    // mode 2: face coefficients of A at planes s and s - 1 (by step parity)
    // and of B at plane s
    T fA[2][6] = {}, fB[6] = {};
    const int s0p = z0 - 1;  // first step; ring slot of plane p is (p - s0p) mod R
    int wx;                  // wrapped plane of the next loads, s + 1 + Dp
    int wxm;                 // the last plane loaded
    {
        // every thread issues the same loads (B and C default to A), so that
        // waits on earlier loads can count them; planes past z1 + 1 that a
        // short chunk loads here are not used
        int w = zfirst(s0p - 1);
        xA[R - 1] = ld(A, zld(w));
        xB[R - 1] = ld(B, zld(w));
#pragma unroll
        for (int k = 0; k <= Dp; ++k) {
            w = znext(w);  // s0p + k
            xA[k] = ld(A, zld(w));
            xB[k] = ld(B, zld(w));
            rA[k] = ldb(A, zld(w));
            rB[k] = ldb(B, zld(w));
            xC[k] = ld(C, zld(w));
        }
        wxm = w;        // s0p + Dp
        wx = znext(w);  // s0p + 1 + Dp
    }
    int s = s0p;
    // one step; r = (s - s0p) mod R; st: whether plane s - 1 gets its second
    // sweep (not in the first two steps, whose s - 1 lies below the chunk)
    auto step = [&](auto rc, auto st) {
        constexpr int r = decltype(rc)::value;
        constexpr bool store = decltype(st)::value;
        constexpr int im1 = (r + R - 1) % R, i0 = r, ip1 = (r + 1) % R, im2 = (r + R - 2) % R;
        // consecutive steps alternate buffers (R is even)
        T* S0 = s0[r & 1];
        T* S1 = s1[r & 1];
        const T* S1m = s1[(r & 1) ^ 1];
        if constexpr (decltype(mt)::value == 2) {
            // all twelve coefficient loads of the step in flight together
            // (B defaults to A: the loads are unconditional)
            const int kc = zmap(s);
            faces(mt, A, kc, fA[r & 1][0], fA[r & 1][1], fA[r & 1][2], fA[r & 1][3],
                  fA[r & 1][4], fA[r & 1][5]);
            faces(mt, B, kc, fB[0], fB[1], fB[2], fB[3], fB[4], fB[5]);
        }
        // Stores and loads are unconditional: a thread without a ring cell
        // stores its own value again (B and C default to A), and the chunk's
        // last steps load wrapped planes they do not use.  A branch around a
        // load, or around the only use of a loaded value, makes the compiler
        // wait for it there (or for everything in flight).
        if (XM != XM_ZERO) {
            S0[A.q] = xA[i0];
            S0[B.q] = xB[i0];
            S0[C.q] = xC[i0];
        }
        __syncthreads();
        {
            // plane s + 1 + Dp; the chunk's last steps, which never use it
            // (past z1 + 1), repeat the last plane loaded (cache hits)
            constexpr int j = (r + 1 + Dp) % R;
            const int wl = zld(s + Dp <= z1 ? wx : wxm);
            xA[j] = ld(A, wl);
            xB[j] = ld(B, wl);
            rA[j] = ldb(A, wl);
            rB[j] = ldb(B, wl);
            xC[j] = ld(C, wl);
        }
        if constexpr (decltype(mt)::value != 0) {
            const int kc = zmap(s);
            T rrA, rrB;
            const T y =
                sweep1g(mt, S0, A, kc, xA[i0], xA[im1], xA[ip1], rA[i0], fA[r & 1], rrA);
            yA[i0] = y;
            S1[hA] = y;
            if constexpr (NM != 0) {
                // the tile's cells of this workgroup's own planes
                if (s >= z0 && s < z1) {
                    nr2 += double(rrA) * double(rrA);
                    if (NM == 2) nb2 += double(rA[i0]) * double(rA[i0]);
                }
            }
            if (hasB) {
                T bvB = rB[i0];
                S1[hB] = sweep1g(mt, S0, B, kc, xB[i0], xB[im1], xB[ip1], bvB, fB, rrB);
            }
            if (store)
                xout[A.col + unsigned(s - 1) * plane] = sweep2g(
                    mt, S1m, hA, A, s - 1, yA[im1], yA[im2], y, rA[im1], fA[(r & 1) ^ 1]);
        } else {
            rA[i0] = rhs(rA[i0]);
            const T y = sweep1(S0, A.q, xA[i0], xA[im1], xA[ip1], rA[i0]);
            yA[i0] = y;
            S1[hA] = y;
            if (hasB) S1[hB] = sweep1(S0, B.q, xB[i0], xB[im1], xB[ip1], rhs(rB[i0]));
            if (store)
                xout[A.col + unsigned(s - 1) * plane] =
                    sweep2(S1m, hA, yA[im1], yA[im2], y, rA[im1]);
        }
        if (s + Dp <= z1) wxm = wx;
        wx = znext(wx);
        ++s;
    };
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using I3 = std::integral_constant<int, 3>;
    using Skip = std::false_type;
    using Store = std::true_type;
    using I4 = std::integral_constant<int, 4 % R>;
    using I5 = std::integral_constant<int, 5 % R>;
    static_assert(R == 4 || R == 6, "the unrolled steps below cover rings of 4 or 6 planes");
    // steps s = z0 - 1 .. z1 (at least two): the first two store nothing,
    // then whole groups of R without exits between them (an exit between two
    // steps would let the compiler sink the next step's loads behind it),
    // then the remainder
    step(I0{}, Skip{});
    step(I1{}, Skip{});
    if constexpr (R == 4) {
        while (s + 3 <= z1) {
            step(I2{}, Store{});
            step(I3{}, Store{});
            step(I0{}, Store{});
            step(I1{}, Store{});
        }
        if (s <= z1) {
            step(I2{}, Store{});
            if (s <= z1) {
                step(I3{}, Store{});
                if (s <= z1) step(I0{}, Store{});
            }
        }
    } else {
        while (s + 5 <= z1) {
            step(I2{}, Store{});
            step(I3{}, Store{});
            step(I4{}, Store{});
            step(I5{}, Store{});
            step(I0{}, Store{});
            step(I1{}, Store{});
        }
        if (s <= z1) step(I2{}, Store{});
        if (s <= z1) step(I3{}, Store{});
        if (s <= z1) step(I4{}, Store{});
        if (s <= z1) step(I5{}, Store{});
        if (s <= z1) step(I0{}, Store{});
    }
    };
    if constexpr (MODE == 3) {
        if (Cf.cls[wg] == 0)
            run(std::integral_constant<int, 1>{});
        else
            run(std::integral_constant<int, 2>{});
    } else {
        run(std::integral_constant<int, MODE>{});
    }
    if constexpr (NM != 0) {
        // fixed-order workgroup sums
        __shared__ double red[2][Sh::T / 64];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            nr2 += __shfl_xor(nr2, off, 64);
            nb2 += __shfl_xor(nb2, off, 64);
        }
        if ((t & 63) == 0) {
            red[0][t >> 6] = nr2;
            red[1][t >> 6] = nb2;
        }
        __syncthreads();
        if (t == 0) {
            double a = 0.0, c = 0.0;
            for (int w = 0; w < Sh::T / 64; ++w) {
                a += red[0][w];
                c += red[1][w];
            }
            partial[2 * pslot] = a;
            partial[2 * pslot + 1] = c;
        }
    }
}

// x += P xc: the coarse correction interpolated linearly onto the fine
// level (prolong_at: 3/4 parent + 1/4 neighbour per direction, wrapped on
// periodic directions, reflected at domain faces).  In place: a cell reads
// only its own x and coarse values.  The thread walks its (i, j) column up
// the z chunk; the 2^d coarse values a cell reads are shared with its
// neighbours and come from L1 / L2 (the coarse level is 1/2^d the size).
// In 3D each coarse plane's x / y interpolation onto the thread's column
// (prolong_at's per-plane value, the same operations) is formed once and
// kept while the walk needs it: two fine planes share each coarse plane, so
// a fine cell costs two coarse loads instead of eight.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_prolong(TileDev TL, Grid g, Grid gc,
                                                    const T* __restrict__ xc, T* __restrict__ x) {
    const Span sp = tile_span(TL, g.n0, g.n1, g.n2);
    if (sp.i >= g.n0 || sp.j >= g.n1) return;
    const size_t plane = size_t(g.n0) * size_t(g.n1);
    size_t id = size_t(sp.i) + size_t(g.n0) * size_t(sp.j) + plane * size_t(sp.z0);
    if (gc.n2 == g.n2) {  // z not coarsened (2D)
        for (int k = sp.z0; k < sp.z1; ++k, id += plane)
            x[id] += prolong_at<T>(g, gc, xc, sp.i, sp.j, k);
        return;
    }
    int ip, iq, jp, jq;
    prolong_pair(sp.i, gc.n0, g.per0, ip, iq);
    prolong_pair(sp.j, gc.n1, g.per1, jp, jq);
    const size_t cn0 = size_t(gc.n0), cpl = cn0 * size_t(gc.n1);
    auto cplane = [&](int K) -> T {
        const T* r = xc + cpl * size_t(K);
        const T lo = lerp34(r[ip + cn0 * jp], r[iq + cn0 * jp]);
        const T hi = lerp34(r[ip + cn0 * jq], r[iq + cn0 * jq]);
        return lerp34(lo, hi);
    };
    // the last three coarse planes formed (plane numbers are the same for
    // the whole workgroup, so the lookups do not diverge)
    int ka = -1, kb = -1, kc = -1;
    T va = T(0), vb = T(0), vc = T(0);
    auto get = [&](int K) -> T {
        if (K == kc) return vc;
        if (K == kb) return vb;
        if (K == ka) return va;
        const T v = cplane(K);
        ka = kb;
        va = vb;
        kb = kc;
        vb = vc;
        kc = K;
        vc = v;
        return v;
    };
    for (int k = sp.z0; k < sp.z1; ++k, id += plane) {
        int kp, kq;
        prolong_pair(k, gc.n2, g.per2, kp, kq);
        const T near = get(kp);
        const T far = get(kq);
        x[id] += lerp34(near, far);
    }
}

// Coarse right-hand side = sum of the 2^d child residuals r = b - A x.  The
// launch covers the fine grid (even z chunks): a thread adds the residuals of
// its z pair, the x pair is combined across neighbouring lanes and the y
// pair through LDS, and the thread at the even (i, j) corner writes the
// coarse cell.
template <typename T, bool UNIF>
__global__ __launch_bounds__(kBlock) void k_resid_restrict(TileDev TL, Grid g, Grid gc, XAccess<T, XM_PLAIN> X,
                                                           Coeffs<T> C, const T* __restrict__ b,
                                                           const double* __restrict__ bshift,
                                                           T* __restrict__ bc) {
    __shared__ T sy[kBlock];
    const Span sp = tile_span(TL, g.n0, g.n1, g.n2);
    const int i = sp.i, j = sp.j;
    const bool valid = i < g.n0 && j < g.n1;
    const bool d3 = g.ndim == 3;
    const int fz = (g.n2 > gc.n2) ? 2 : 1;
    const int t = threadIdx.x, bx = 1 << TL.lbx;
    const unsigned n0 = unsigned(g.n0), plane = n0 * unsigned(g.n1);
    // column geometry as in k_smooth (non-periodic boundaries: self, L = 0)
    const int ixm = i > 0 ? i - 1 : (g.per0 ? g.n0 - 1 : i);
    const int ixp = i < g.n0 - 1 ? i + 1 : (g.per0 ? 0 : i);
    const int jym = j > 0 ? j - 1 : (g.per1 ? g.n1 - 1 : j);
    const int jyp = j < g.n1 - 1 ? j + 1 : (g.per1 ? 0 : j);
    const bool hxu = i < g.n0 - 1 || g.per0, hyu = j < g.n1 - 1 || g.per1;
    const int oxm = ixm - i, oxp = ixp - i;
    const int oym = (jym - j) * int(n0), oyp = (jyp - j) * int(n0);
    unsigned id = unsigned(i) + n0 * unsigned(j) + plane * unsigned(sp.z0);
    // residual of one cell given its z neighbours and z coefficients
    const bool shift = bshift != nullptr;
    const double mean = shift ? *bshift : 0.0;
    // a block of class 0 takes its coefficients from the position
    const bool walled = !UNIF && C.cls && C.cls[block_linear()] == 0;
    const T Lxl_w = (i == 0 && !g.per0) ? T(0) : C.Lc;
    const T Lxu_w = (i == g.n0 - 1 && !g.per0) ? T(0) : C.Lc;
    const T Lyl_w = (j == 0 && !g.per1) ? T(0) : C.Lc;
    const T Lyu_w = (j == g.n1 - 1 && !g.per1) ? T(0) : C.Lc;
    auto Lz_at = [&](int kk, unsigned c) -> T {     // lower z face of cell kk
        if (UNIF) return C.Lc;
        if (walled) return (kk == 0 && !g.per2) ? T(0) : C.Lc;
        return C.L2[c];
    };
    auto resid = [&](unsigned c, T xI, T xzl, T xzu, T Lzl, T Lzu) -> T {
        const T xxl = X.x[c + oxm], xxu = X.x[c + oxp], xyl = X.x[c + oym], xyu = X.x[c + oyp];
        T bv = b[c];
        T Lxl, Lxu, Lyl, Lyu;
        if (UNIF) {
            Lxl = Lxu = Lyl = Lyu = C.Lc;
        } else if (walled) {
            Lxl = Lxl_w;
            Lxu = Lxu_w;
            Lyl = Lyl_w;
            Lyu = Lyu_w;
        } else {
            Lxl = C.L0[c];
            Lxu = hxu ? C.L0[c + oxp] : T(0);
            Lyl = C.L1[c];
            Lyu = hyu ? C.L1[c + oyp] : T(0);
        }
        if (shift) {
            T D = T(0);
            D += Lxl + Lxu;
            D += Lyl + Lyu;
            if (d3) D += Lzl + Lzu;
            bv = D > T(0) ? T(double(bv) - mean) : T(0);
        }
        return resid_row(bv, xI, xxl, xxu, xyl, xyu, xzl, xzu, Lxl, Lxu, Lyl, Lyu, Lzl, Lzu, d3);
    };
    auto zup = [&](int k, unsigned c, bool& live) -> unsigned {  // index of the upper z neighbour
        live = k < g.n2 - 1 || g.per2;
        return c + unsigned((k < g.n2 - 1 ? k + 1 : (g.per2 ? 0 : k)) - k) * plane;
    };
    T xzl = T(0), xI = T(0), Lzl = T(0);
    if (valid && sp.z0 < sp.z1) {
        xI = X.x[id];
        if (d3) {
            const int k0 = sp.z0, km = k0 > 0 ? k0 - 1 : (g.per2 ? g.n2 - 1 : k0);
            xzl = X.x[id + unsigned(km - k0) * plane];
            Lzl = Lz_at(k0, id);
        }
    }
    for (int k = sp.z0; k < sp.z1; k += fz, id += unsigned(fz) * plane) {
        T r = T(0);
        if (valid) {
            if (d3) {
                // cells k and k + 1 (fz = 2): the upper neighbour of k is the
                // centre of k + 1
                bool l1, l2;
                const unsigned u1 = zup(k, id, l1);
                const T x1 = X.x[u1];
                const T Lz1 = l1 ? Lz_at(k + 1 < g.n2 ? k + 1 : 0, u1) : T(0);
                if (fz == 2) {
                    const unsigned u2 = zup(k + 1, u1, l2);
                    const T x2 = X.x[u2];
                    const T Lz2 = l2 ? Lz_at(k + 2 < g.n2 ? k + 2 : 0, u2) : T(0);
                    r = resid(id, xI, xzl, x1, Lzl, Lz1);
                    r += resid(u1, x1, xI, x2, Lz1, Lz2);
                    xzl = x1;
                    xI = x2;
                    Lzl = Lz2;
                } else {
                    r = resid(id, xI, xzl, x1, Lzl, Lz1);
                    xzl = xI;
                    xI = x1;
                    Lzl = Lz1;
                }
            } else {
                r = resid(id, xI, T(0), T(0), T(0), T(0));
            }
        }
        r += __shfl_xor(r, 1, 64);
        sy[t] = r;
        __syncthreads();
        if (valid && (i & 1) == 0 && (j & 1) == 0)
            bc[cid(gc, i >> 1, j >> 1, k / fz)] = r + sy[t + bx];
        __syncthreads();
    }
}

// Per-block partial sums of v over active cells (v == nullptr counts them).
// Every cell of a class-0 block (C.cls) is active: no coefficient is read.
template <typename T, bool UNIF>
__global__ __launch_bounds__(kBlock) void k_sum_active(TileDev TL, Grid g, Coeffs<T> C, const T* __restrict__ v,
                                                       double* __restrict__ partial) {
    __shared__ double lds[8];
    const Span sp = tile_span(TL, g.n0, g.n1, g.n2);
    const int i = sp.i, j = sp.j;
    const bool walled = !UNIF && C.cls && C.cls[block_linear()] == 0;
    double s = 0.0;
    if (i < g.n0 && j < g.n1) {
        for (int k = sp.z0; k < sp.z1; ++k) {
        bool act = true;
        if (!walled) {
            XAccess<T, XM_ZERO> X{nullptr};
            T xI, Ax, D;
            apply_row<T, XM_ZERO, UNIF>(g, X, C, i, j, k, xI, Ax, D);
            act = D > T(0);
        }
        if (act) s += v ? double(v[cid(g, i, j, k)]) : 1.0;
        }
    }
    s = block_sum(s, lds);
    if (threadIdx.x == 0 && threadIdx.y == 0) partial[block_linear()] = s;
}

// Copies n doubles to pinned host memory, then (after a system-scope fence)
// the sequence number the host is waiting for.  One thread.
template <typename T>
__global__ void k_fill(T* __restrict__ p, size_t n, T v);

__global__ void k_publish(const double* __restrict__ src, MailboxPost P) { mailbox_write(P, src); }

HostMailbox::~HostMailbox() {
    if (vals) (void)hipHostFree(vals);
}

wl_status mailbox_post_args(Reduce& red, int slot, int n, hipStream_t s, MailboxPost* out) {
    HostMailbox& mb = red.mb;
    if (n < 0 || slot < 0 || slot + n > HostMailbox::kSlots) {
        set_error("mailbox post: slot range outside the mailbox");
        return WL_ERR_INVALID_ARG;
    }
    double* counter = red.result + kResultCounter;
    if (!mb.vals) {
        void* p = nullptr;
        WL_CHECK_HIP(hipHostMalloc(&p, 256, hipHostMallocCoherent | hipHostMallocMapped));
        mb.vals = static_cast<double*>(p);
        mb.seqw = reinterpret_cast<unsigned*>(mb.vals + HostMailbox::kSlots);
        *mb.seqw = 0u;
        mb.seq = 0u;
        void* d = nullptr;
        WL_CHECK_HIP(hipHostGetDevicePointer(&d, p, 0));
        mb.vals_dev = static_cast<double*>(d);
        mb.seqw_dev = reinterpret_cast<unsigned*>(mb.vals_dev + HostMailbox::kSlots);
        // the device count starts with the host's (a fill kernel: this may be
        // enqueued while a caller captures)
        k_fill<double><<<1, 64, 0, s>>>(counter, 1, 0.0);
        WL_CHECK_LAUNCH();
    }
    *out = MailboxPost{mb.vals_dev, mb.seqw_dev, counter, slot, n};
    return WL_OK;
}

void host_posted(Reduce& red) { ++red.mb.seq; }

wl_status host_post(Reduce& red, const double* src, int n, int slot, hipStream_t s) {
    MailboxPost P;
    WL_TRY(mailbox_post_args(red, slot, n, s, &P));
    k_publish<<<1, 1, 0, s>>>(src, P);
    WL_CHECK_LAUNCH();
    host_posted(red);
    return WL_OK;
}

wl_status host_wait(Reduce& red, hipStream_t s) { return host_wait_seq(red, red.mb.seq, s); }

wl_status host_wait_seq(Reduce& red, unsigned q, hipStream_t s) {
    HostMailbox& mb = red.mb;
    if (!mb.vals) return WL_OK;
    // arrived: the published count has reached q (wrap-safe)
    auto arrived = [&] { return int(__atomic_load_n(mb.seqw, __ATOMIC_ACQUIRE) - q) >= 0; };
    // Poll for up to 20 ms (a step's solves publish every few hundred
    // microseconds), then let HIP wait and report any kernel failure.
    const auto t0 = std::chrono::steady_clock::now();
    unsigned spins = 0;
    while (!arrived()) {
        if ((++spins & 1023u) == 0u &&
            std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(20)) {
            WL_CHECK_HIP(hipStreamSynchronize(s));
            if (!arrived()) {
                set_error("device result did not arrive in the host mailbox");
                return WL_ERR_HIP;
            }
            break;
        }
    }
    return WL_OK;
}

wl_status host_read(Reduce& red, const double* src, int n, double* out, hipStream_t s) {
    WL_TRY(host_post(red, src, n, 0, s));
    WL_TRY(host_wait(red, s));
    for (int k = 0; k < n; ++k) out[k] = red.mb.vals[k];
    return WL_OK;
}

// out[c] = sum over slots of partial[slot*ncomp + c] in slot order; then
// out[ncomp + c] = out[c] * scale, or with count (ncomp == 1) the mean
// out[1] = out[0] / *count (0 when nothing is active); with post.vals the
// first post.n outputs are posted to the host mailbox.  One block of 1024
// threads.
__global__ __launch_bounds__(1024) void k_reduce(const double* __restrict__ partial, size_t nslots,
                                                 int ncomp, double scale, double* __restrict__ out,
                                                 const double* __restrict__ count,
                                                 MailboxPost post) {
    __shared__ double lds[32];
    double S[2] = {0.0, 0.0};
    if (ncomp == 2) {
        wg_slot_reduce<2, false>(partial, nslots, S, lds);
    } else {
        double S1[1];
        wg_slot_reduce<1, false>(partial, nslots, S1, lds);
        S[0] = S1[0];
    }
    if (threadIdx.x == 0) {
        for (int c = 0; c < ncomp; ++c) {
            out[c] = S[c];
            out[ncomp + c] = count ? (*count > 0.0 ? S[c] / *count : 0.0) : S[c] * scale;
        }
        if (post.vals) mailbox_write(post, out);
    }
}

// Coarsest level: the iteration of coarse_cg_regs (CG on -A over the active
// cells, mean-free right-hand side and result, FP64) with one cell per thread
// (N <= blockDim <= 1024).  Each thread builds its cell's stencil once (the
// diagonal, six face coefficients and six neighbour slots, a missing
// neighbour being the cell itself with the coefficient the generic solver
// uses), so an iteration is six LDS reads of the search direction, two
// fixed-order sums (one barrier each, alternating buffers) and the barrier
// after the direction update.  The sums run over the first nw waves (those
// that can own a cell: every wave of the workgroup executes each barrier, so
// a larger workgroup, as in the V-cycle tail, gets the same sums bitwise).
// sp: kCoarseMax doubles of LDS, red: 2 x 16 of LDS.
template <typename T>
__device__ void coarse_cg_regs(const Grid& g, const T* L0, const T* L1, const T* L2, T Lc,
                                int uniform, const T* b, T* xout, double tol, int maxit, int nw,
                                double* sp, double (*red)[16]) {
    const int N = int(cells(g));
    const int t = int(threadIdx.x);
    const bool own = t < N;
    auto wsum = [&](double v, int buf) -> double {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if ((t & 63) == 0 && (t >> 6) < nw) red[buf][t >> 6] = v;
        __syncthreads();
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += red[buf][w];
        return s;
    };
    double D = 0.0, cf[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int nb[6] = {t, t, t, t, t, t};
    if (own) {
        const int i = t % g.n0, j = (t / g.n0) % g.n1, k = t / (g.n0 * g.n1);
        const int n[3] = {g.n0, g.n1, g.n2}, per[3] = {g.per0, g.per1, g.per2};
        const int co[3] = {i, j, k}, st[3] = {1, g.n0, g.n0 * g.n1};
        const T* Ld[3] = {L0, L1, L2};
        for (int d = 0; d < g.ndim; ++d) {
            const int lo = nb_lo(co[d], n[d], per[d]), up = nb_up(co[d], n[d], per[d]);
            nb[2 * d] = t + (lo - co[d]) * st[d];
            nb[2 * d + 1] = t + (up - co[d]) * st[d];
            const double Ll = uniform ? double(Lc) : double(Ld[d][t]);
            const double Lu = (co[d] < n[d] - 1 || per[d])
                                  ? (uniform ? double(Lc) : double(Ld[d][nb[2 * d + 1]]))
                                  : 0.0;
            cf[2 * d] = Ll;
            cf[2 * d + 1] = Lu;
            D += Ll + Lu;
        }
    }
    const bool act = D > 0.0;
    const double bt = own ? double(b[t]) : 0.0;
    // mean of b over the active cells
    const double sumb = wsum(act ? bt : 0.0, 0);
    const double cnt = wsum(act ? 1.0 : 0.0, 1);
    const double mean = cnt > 0.0 ? sumb / cnt : 0.0;
    // solve M x = B with M = -A, B = -(b - mean) on active cells
    const double B = act ? -(bt - mean) : 0.0;
    double x = 0.0, r = B, p = B;
    if (own) sp[t] = p;
    double rr = wsum(B * B, 0);  // its barrier also publishes sp
    const double rr0 = rr;
    if (rr0 > 0.0) {
        for (int it = 0; it < maxit; ++it) {
            double Mp = 0.0;
            if (act) {
                Mp = D * p;
#pragma unroll
                for (int m = 0; m < 6; ++m) Mp -= cf[m] * sp[nb[m]];
            }
            const double pq = wsum(p * Mp, 1);
            if (!(pq > 0.0)) break;
            const double alpha = rr / pq;
            x += alpha * p;
            r -= alpha * Mp;
            const double rn = wsum(r * r, 0);
            if (rn <= tol * tol * rr0) break;
            const double beta = rn / rr;
            rr = rn;
            p = r + beta * p;
            if (own) sp[t] = p;
            __syncthreads();
        }
    }
    // mean-free result on the active cells (the barrier keeps the last
    // sum's buffer until every wave has read it)
    __syncthreads();
    const double xs = wsum(act ? x : 0.0, 1);
    const double xm = cnt > 0.0 ? xs / cnt : 0.0;
    if (own) xout[t] = act ? T(x - xm) : T(0);
}

// Coarsest level of at most kCgWaveMax cells in one wave: the same CG as
// coarse_cg_regs with lane l owning cells l, l + 64, ... (PER of them), the
// stencils in registers and the search direction in LDS (sp, wave-
// synchronous: one wave writes and reads it).  Every rounding is spelled out
// (contraction off, fused multiply-adds written as such), so the standalone
// kernel and the V-cycle tail, which both call it, agree bit for bit.  Sums:
// per lane over its cells in order, then wave_sum_f64.
constexpr int kCgWaveMax = 256;

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): this wave's LDS traffic done
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Data-parallel move of a double across the lanes of a row (CTRL: a DPP
// control, every lane valid).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, int(u), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, int(u >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double((static_cast<long long>(hi) << 32) |
                                static_cast<long long>(static_cast<unsigned>(lo)));
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
    const long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane(int(u), lane);
    const int hi = __builtin_amdgcn_readlane(int(u >> 32), lane);
    return __longlong_as_double((static_cast<long long>(hi) << 32) |
                                static_cast<long long>(static_cast<unsigned>(lo)));
}

// Sum over the 64 lanes of a full wave, the same value in every lane: lane
// pairs, quads, half rows and rows by data-parallel moves (each add takes
// two equal partial sums in either order, so every lane of a row ends with
// the same bits), then the four row sums in row order.
__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma clang fp contract(off)
    v = v + dpp_f64<0xB1>(v);   // quad_perm [1, 0, 3, 2]
    v = v + dpp_f64<0x4E>(v);   // quad_perm [2, 3, 0, 1]
    v = v + dpp_f64<0x141>(v);  // row_half_mirror
    v = v + dpp_f64<0x140>(v);  // row_mirror
    return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}

template <typename T, int PER>
__device__ void coarse_cg_wave(const Grid& g, const T* L0, const T* L1, const T* L2, T Lc,
                               int uniform, const T* b, T* xout, double tol, int maxit,
                               double* sp) {
#pragma clang fp contract(off)
    const int N = int(cells(g));
    const int lane = int(threadIdx.x) & 63;
    double D[PER], cf[PER][6], x[PER], r[PER], p[PER], Mp[PER], bt[PER];
    int nb[PER][6];
    bool act[PER], own[PER];
#pragma unroll
    for (int m = 0; m < PER; ++m) {
        const int c = lane + 64 * m;
        own[m] = c < N;
        D[m] = 0.0;
        bt[m] = 0.0;
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            cf[m][f] = 0.0;
            nb[m][f] = own[m] ? c : 0;
        }
        if (own[m]) {
            const int i = c % g.n0, j = (c / g.n0) % g.n1, k = c / (g.n0 * g.n1);
            const int n[3] = {g.n0, g.n1, g.n2}, per[3] = {g.per0, g.per1, g.per2};
            const int co[3] = {i, j, k}, st[3] = {1, g.n0, g.n0 * g.n1};
            const T* Ld[3] = {L0, L1, L2};
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                if (d >= g.ndim) break;
                const int lo = nb_lo(co[d], n[d], per[d]), up = nb_up(co[d], n[d], per[d]);
                nb[m][2 * d] = c + (lo - co[d]) * st[d];
                nb[m][2 * d + 1] = c + (up - co[d]) * st[d];
                const double Ll = uniform ? double(Lc) : double(Ld[d][c]);
                const double Lu = (co[d] < n[d] - 1 || per[d])
                                      ? (uniform ? double(Lc) : double(Ld[d][nb[m][2 * d + 1]]))
                                      : 0.0;
                cf[m][2 * d] = Ll;
                cf[m][2 * d + 1] = Lu;
                D[m] = D[m] + (Ll + Lu);
            }
            bt[m] = double(b[c]);
        }
        act[m] = D[m] > 0.0;
    }
    auto wsum = [&](const double (&v)[PER]) -> double {
        double s = v[0];
#pragma unroll
        for (int m = 1; m < PER; ++m) s = s + v[m];
        return wave_sum_f64(s);
    };
    double t0[PER], t1[PER];
#pragma unroll
    for (int m = 0; m < PER; ++m) {
        t0[m] = act[m] ? bt[m] : 0.0;
        t1[m] = act[m] ? 1.0 : 0.0;
    }
    const double sumb = wsum(t0), cnt = wsum(t1);
    const double mean = cnt > 0.0 ? sumb / cnt : 0.0;
    // solve M x = B with M = -A, B = -(b - mean) on active cells
#pragma unroll
    for (int m = 0; m < PER; ++m) {
        const double B = act[m] ? -(bt[m] - mean) : 0.0;
        x[m] = 0.0;
        r[m] = B;
        p[m] = B;
        if (own[m]) sp[lane + 64 * m] = B;
        t0[m] = B * B;
    }
    double rr = wsum(t0);
    const double rr0 = rr;
    wave_lds_sync();
    if (rr0 > 0.0) {
        for (int it = 0; it < maxit; ++it) {
#pragma unroll
            for (int m = 0; m < PER; ++m) {
                double v = 0.0;
                if (act[m]) {
                    v = D[m] * p[m];
#pragma unroll
                    for (int f = 0; f < 6; ++f) v = fma(-cf[m][f], sp[nb[m][f]], v);
                }
                Mp[m] = v;
                t0[m] = p[m] * v;
            }
            const double pq = wsum(t0);
            if (!(pq > 0.0)) break;
            const double alpha = rr / pq;
#pragma unroll
            for (int m = 0; m < PER; ++m) {
                x[m] = fma(alpha, p[m], x[m]);
                r[m] = fma(-alpha, Mp[m], r[m]);
                t0[m] = r[m] * r[m];
            }
            const double rn = wsum(t0);
            if (rn <= tol * tol * rr0) break;
            const double beta = rn / rr;
            rr = rn;
            wave_lds_sync();  // every lane has read sp
#pragma unroll
            for (int m = 0; m < PER; ++m) {
                p[m] = fma(beta, p[m], r[m]);
                if (own[m]) sp[lane + 64 * m] = p[m];
            }
            wave_lds_sync();
        }
    }
    // mean-free result on the active cells
#pragma unroll
    for (int m = 0; m < PER; ++m) t0[m] = act[m] ? x[m] : 0.0;
    const double xm = cnt > 0.0 ? wsum(t0) / cnt : 0.0;
#pragma unroll
    for (int m = 0; m < PER; ++m)
        if (own[m]) xout[lane + 64 * m] = act[m] ? T(x[m] - xm) : T(0);
}

// The one-wave solve for the level's size (PER = cells per lane, at most
// MAXPER).
template <typename T, int MAXPER>
__device__ __forceinline__ void coarse_cg_wave_any(const Grid& g, const T* L0, const T* L1,
                                                   const T* L2, T Lc, int uniform, const T* b,
                                                   T* xout, double tol, int maxit, double* sp) {
    const int N = int(cells(g));
    if (N <= 64)
        coarse_cg_wave<T, 1>(g, L0, L1, L2, Lc, uniform, b, xout, tol, maxit, sp);
    else if (MAXPER < 4 || N <= 128)
        coarse_cg_wave<T, 2>(g, L0, L1, L2, Lc, uniform, b, xout, tol, maxit, sp);
    else
        coarse_cg_wave<T, 4>(g, L0, L1, L2, Lc, uniform, b, xout, tol, maxit, sp);
}

// Coarsest level by its inverse (non-uniform levels of at most kDirectMax
// cells).  On the active cells (D > 0) M = -A is singular with the constant
// as null vector (per connected set of active cells); M + a 1 1^T, a = (mean D) /
// n_act, is positive definite when the active cells are connected, and its
// inverse G maps every mean-free right-hand side B to the mean-free solution
// of M x = B: the minimum-norm solution a pseudo-inverse gives.  Formed once
// per coefficient change by Gauss-Jordan elimination without pivoting (one
// workgroup, the matrix in LDS); a pivot that is not positive (disconnected
// active cells, or a singular level) clears *ok and the CG solves instead.
// Inactive rows and columns of G are zero.
template <typename T>
__global__ __launch_bounds__(1024) void k_coarse_inverse(Grid g, Coeffs<T> C, int uniform,
                                                         double* __restrict__ G,
                                                         int* __restrict__ ok) {
    // the matrix in LDS with row stride kS; thread t owns row t / 16 and
    // columns t % 16 + 16 q (q < 4) of the elimination
    constexpr int kS = kDirectMax, kQ = kDirectMax / 16;
    static_assert(kDirectMax % 16 == 0 && kDirectMax * 16 <= 1024, "one element group per thread");
    __shared__ double A[kS * kS];
    __shared__ double actf[kS];
    __shared__ double red[2 * 16];
    const int N = int(cells(g));
    const int t = int(threadIdx.x), nt = int(blockDim.x);
    const int ri = t >> 4, cj = t & 15;
#pragma unroll
    for (int q = 0; q < kQ; ++q) A[ri * kS + cj + 16 * q] = 0.0;
    __syncthreads();
    double D = 0.0;
    if (t < N) {
        const int i = t % g.n0, j = (t / g.n0) % g.n1, k = t / (g.n0 * g.n1);
        const int n[3] = {g.n0, g.n1, g.n2}, per[3] = {g.per0, g.per1, g.per2};
        const int co[3] = {i, j, k}, st[3] = {1, g.n0, g.n0 * g.n1};
        const T* Ld[3] = {C.L0, C.L1, C.L2};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            if (d >= g.ndim) break;
            const int lo = nb_lo(co[d], n[d], per[d]), up = nb_up(co[d], n[d], per[d]);
            const int nlo = t + (lo - co[d]) * st[d], nup = t + (up - co[d]) * st[d];
            const double Ll = uniform ? double(C.Lc) : double(Ld[d][t]);
            const double Lu =
                (co[d] < n[d] - 1 || per[d]) ? (uniform ? double(C.Lc) : double(Ld[d][nup])) : 0.0;
            D += Ll + Lu;
            A[t * kS + nlo] -= Ll;
            A[t * kS + nup] -= Lu;
        }
        A[t * kS + t] += D;
    }
    const bool act = t < N && D > 0.0;
    // active count and diagonal sum (fixed order over the waves)
    double c0 = act ? 1.0 : 0.0, c1 = act ? D : 0.0;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        c0 += __shfl_xor(c0, off, 64);
        c1 += __shfl_xor(c1, off, 64);
    }
    if ((t & 63) == 0) {
        red[2 * (t >> 6)] = c0;
        red[2 * (t >> 6) + 1] = c1;
    }
    // an inactive cell's row and column are zero (its faces are): its
    // diagonal becomes 1, its flag 0
    if (t < N && !act) A[t * kS + t] = 1.0;
    if (t < kS) actf[t] = act ? 1.0 : 0.0;
    __syncthreads();
    double nact = 0.0, dsum = 0.0;
    for (int w = 0; w < nt / 64; ++w) {
        nact += red[2 * w];
        dsum += red[2 * w + 1];
    }
    const double scale = nact > 0.0 ? dsum / nact : 1.0;
    const double a = nact > 0.0 ? scale / nact : 0.0;
    const bool rowact = ri < N && actf[ri] != 0.0;
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
        const int j = cj + 16 * q;
        if (rowact && j < N && actf[j] != 0.0) A[ri * kS + j] += a;
    }
    __syncthreads();
    bool good = true;
    for (int p = 0; p < N; ++p) {
        const double piv = A[p * kS + p];
        good = piv > 1e-12 * scale;  // the same value in every thread
        if (!good) break;
        const double cv = A[ri * kS + p];
        double rv[kQ];
#pragma unroll
        for (int q = 0; q < kQ; ++q) rv[q] = A[p * kS + cj + 16 * q];
        __syncthreads();
        const double inv = 1.0 / piv;
        if (ri < N) {
#pragma unroll
            for (int q = 0; q < kQ; ++q) {
                const int j = cj + 16 * q;
                if (j >= N) continue;
                const double prow = (j == p) ? inv : rv[q] * inv;  // the scaled pivot row
                double& e = A[ri * kS + j];
                e = (ri == p) ? prow : (j == p) ? -cv * inv : e - cv * prow;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
        const int j = cj + 16 * q;
        if (ri < N && j < N)
            G[ri * N + j] = (good && actf[ri] != 0.0 && actf[j] != 0.0) ? A[ri * kS + j] : 0.0;
    }
    if (t == 0) *ok = good ? 1 : 0;
}

// x = G B on the coarsest level in one wave, B the mean-free right-hand side
// (as coarse_cg_wave forms it), then the mean of x over the active cells
// removed.  Sums as in coarse_cg_wave; sp: LDS for N doubles.
template <typename T, int PER>
__device__ void coarse_direct_wave(const Grid& g, const T* L0, const T* L1, const T* L2, T Lc,
                                   int uniform, const T* b, T* xout, const double* G,
                                   double* sp) {
#pragma clang fp contract(off)
    const int N = int(cells(g));
    const int lane = int(threadIdx.x) & 63;
    double bt[PER], x[PER], t0[PER], t1[PER];
    bool act[PER], own[PER];
#pragma unroll
    for (int m = 0; m < PER; ++m) {
        const int c = lane + 64 * m;
        own[m] = c < N;
        double D = 0.0;
        bt[m] = 0.0;
        if (own[m]) {
            const int i = c % g.n0, j = (c / g.n0) % g.n1, k = c / (g.n0 * g.n1);
            const int n[3] = {g.n0, g.n1, g.n2}, per[3] = {g.per0, g.per1, g.per2};
            const int co[3] = {i, j, k}, st[3] = {1, g.n0, g.n0 * g.n1};
            const T* Ld[3] = {L0, L1, L2};
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                if (d >= g.ndim) break;
                const int up = nb_up(co[d], n[d], per[d]);
                const double Ll = uniform ? double(Lc) : double(Ld[d][c]);
                const double Lu = (co[d] < n[d] - 1 || per[d])
                                      ? (uniform ? double(Lc) : double(Ld[d][c + (up - co[d]) * st[d]]))
                                      : 0.0;
                D = D + (Ll + Lu);
            }
            bt[m] = double(b[c]);
        }
        act[m] = D > 0.0;
        t0[m] = act[m] ? bt[m] : 0.0;
        t1[m] = act[m] ? 1.0 : 0.0;
    }
    auto wsum = [&](const double (&v)[PER]) -> double {
        double s = v[0];
#pragma unroll
        for (int m = 1; m < PER; ++m) s = s + v[m];
        return wave_sum_f64(s);
    };
    const double sumb = wsum(t0), cnt = wsum(t1);
    const double mean = cnt > 0.0 ? sumb / cnt : 0.0;
#pragma unroll
    for (int m = 0; m < PER; ++m)
        if (own[m]) sp[lane + 64 * m] = act[m] ? -(bt[m] - mean) : 0.0;
    wave_lds_sync();
#pragma unroll
    for (int m = 0; m < PER; ++m) x[m] = 0.0;
    // G is symmetric: column c read along the rows keeps the lanes' loads
    // consecutive; 16 / PER rows' loads are issued before they are used
    constexpr int U = 16 / PER;
    int cc[PER];
#pragma unroll
    for (int m = 0; m < PER; ++m) cc[m] = own[m] ? lane + 64 * m : 0;
    int j = 0;
    for (; j + U <= N; j += U) {
        double gv[PER][U];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int m = 0; m < PER; ++m) gv[m][u] = G[size_t(j + u) * N + cc[m]];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const double Bj = sp[j + u];
#pragma unroll
            for (int m = 0; m < PER; ++m) x[m] = fma(gv[m][u], Bj, x[m]);
        }
    }
    for (; j < N; ++j) {
        const double Bj = sp[j];
#pragma unroll
        for (int m = 0; m < PER; ++m) x[m] = fma(G[size_t(j) * N + cc[m]], Bj, x[m]);
    }
#pragma unroll
    for (int m = 0; m < PER; ++m) t0[m] = act[m] ? x[m] : 0.0;
    const double xm = cnt > 0.0 ? wsum(t0) / cnt : 0.0;
#pragma unroll
    for (int m = 0; m < PER; ++m)
        if (own[m]) xout[lane + 64 * m] = act[m] ? T(x[m] - xm) : T(0);
}

// The coarsest solve of a one-wave level: the inverse when it is valid, else
// the CG.
template <typename T, int MAXPER>
__device__ __forceinline__ void coarse_wave_solve(const Grid& g, const T* L0, const T* L1,
                                                  const T* L2, T Lc, int uniform, const T* b,
                                                  T* xout, double tol, int maxit, double* sp,
                                                  const double* G, const int* ok) {
    const int N = int(cells(g));
    if (G && N <= 64 && *ok) {
        coarse_direct_wave<T, 1>(g, L0, L1, L2, Lc, uniform, b, xout, G, sp);
        return;
    }
    coarse_cg_wave_any<T, MAXPER>(g, L0, L1, L2, Lc, uniform, b, xout, tol, maxit, sp);
}

template <typename T>
__global__ __launch_bounds__(64) void k_coarse_cg_wave(Grid g, Coeffs<T> C, int uniform,
                                                       const T* __restrict__ b,
                                                       T* __restrict__ xout, double tol,
                                                       int maxit, const double* G,
                                                       const int* ok) {
    __shared__ double sp[kCgWaveMax];
    coarse_wave_solve<T, 4>(g, C.L0, C.L1, C.L2, C.Lc, uniform, b, xout, tol, maxit, sp, G, ok);
}

template <typename T>
__global__ __launch_bounds__(1024) void k_coarse_cg(Grid g, Coeffs<T> C, int uniform,
                                                    const T* __restrict__ b, T* __restrict__ xout,
                                                    double tol, int maxit) {
    __shared__ double sp[kCoarseMax];
    __shared__ double red[2][16];
    coarse_cg_regs<T>(g, C.L0, C.L1, C.L2, C.Lc, uniform, b, xout, tol, maxit,
                      int(blockDim.x) >> 6, sp, red);
}

// ------------------------------------------------- V-cycle tail, one workgroup
// The coarse end of a V-cycle (Sec. 2's GMG on its smallest levels) in one
// launch: below a few thousand cells every per-level kernel is a handful of
// waves whose launch costs more than its work.  One workgroup of
// kTailThreads runs the levels from the first small one down to the
// coarsest and back up with every iterate and right-hand side in LDS: the
// top level's right-hand side is read once, its corrected iterate written
// once, and the steps in between are separated by barriers.  Per level, as
// the per-level kernels do it: a sweep from zero into x0, a sweep from x0
// into x1, the residual of x1 (kept in x0, free until the post-smoothing)
// summed into the coarse right-hand side, and on the way up the in-place
// prolongation into x1 and two sweeps back into x1; the coarsest level is
// coarse_cg_wave, run by the first wave.  Each cell's arithmetic is that of
// k_smooth, k_resid_restrict (resid_row and the same sum order over the 2^d
// children), k_prolong and k_coarse_cg, so the result is bitwise that of
// the per-level launches.  Face coefficients are read from global memory
// (L1 / L2).
constexpr int kTailLevels = 8;
constexpr int kTailThreads = 1024;
constexpr int kTailPer = 4;                               // cells per thread and level
constexpr int kTailLdsCells = kTailThreads * kTailPer * 4 / 3 + 64;  // all levels, 2D included
constexpr int kTailCgMax = 128;  // coarsest level: two cells per lane

template <typename T>
struct TailLevel {
    Grid g;
    const T* L0;
    const T* L1;
    const T* L2;
    T Lc;
    T wD;                      // w / D of a uniform level
    unsigned long long m0, mc;  // ceil(2^32 / d) for n0 and the column count: exact quotients
    int parts, seg;             // column walks: z segments per column, planes per segment
    int ox0, ox1, ob;           // LDS offsets of x0, x1 and b
};

template <typename T>
struct TailArgs {
    TailLevel<T> lev[kTailLevels];
    const T* b;  // right-hand side of the top tail level
    T* x;        // its corrected iterate
    const double* G;  // the coarsest level's inverse and its flag (null: CG)
    const int* ok;
    int n;       // levels: n - 1 smoothed, the last one solved
    T omega;
    double tol;
};

// Column walks: a level of n0 x n1 columns; with fewer columns than
// threads each column is split into `parts` z segments of `seg` planes and
// thread t takes column t mod cols, segment t / cols; otherwise thread t
// takes the whole columns t, t + kTailThreads, ...  fn(col, i, j, k0, k1)
// walks its cells up z as the tiled kernels do (x / y neighbour offsets
// fixed along the column, the lower z neighbour carried), so a cell costs
// little besides its own arithmetic.  Ends with a barrier.
template <typename T, typename Fn>
__device__ __forceinline__ void tail_columns(const TailLevel<T>& L, Fn&& fn) {
    const int t = int(threadIdx.x);
    const int cols = L.g.n0 * L.g.n1;
    auto run = [&](int col, int k0, int k1) {
        const int j = int((unsigned long long)unsigned(col) * L.m0 >> 32);
        fn(col, col - j * L.g.n0, j, k0, k1);
    };
    if (cols >= kTailThreads) {
        for (int col = t; col < cols; col += kTailThreads) run(col, 0, L.g.n2);
    } else if (t < L.parts * cols) {
        const int part = int((unsigned long long)unsigned(t) * L.mc >> 32);
        const int k0 = part * L.seg;
        run(t - part * cols, k0, min(L.g.n2, k0 + L.seg));
    }
    __syncthreads();
}

// x / y neighbour offsets of column (i, j) as the tiled kernels form them: a
// non-periodic boundary points at the cell itself (its face coefficient is
// zero), a periodic one wraps.
struct TailCol {
    int oxm, oxp, oym, oyp;
    bool hxu, hyu;
};

__device__ __forceinline__ TailCol tail_col(const Grid& g, int i, int j) {
    TailCol q;
    const int ixm = i > 0 ? i - 1 : (g.per0 ? g.n0 - 1 : i);
    const int ixp = i < g.n0 - 1 ? i + 1 : (g.per0 ? 0 : i);
    const int jym = j > 0 ? j - 1 : (g.per1 ? g.n1 - 1 : j);
    const int jyp = j < g.n1 - 1 ? j + 1 : (g.per1 ? 0 : j);
    q.oxm = ixm - i;
    q.oxp = ixp - i;
    q.oym = (jym - j) * g.n0;
    q.oyp = (jyp - j) * g.n0;
    q.hxu = i < g.n0 - 1 || g.per0;
    q.hyu = j < g.n1 - 1 || g.per1;
    return q;
}

// Offset of the upper / lower z neighbour of plane k (self at a
// non-periodic end) and whether the upper face exists.
__device__ __forceinline__ int tail_zup(const Grid& g, int k, int plane, bool& hzu) {
    hzu = k < g.n2 - 1 || g.per2;
    return (k < g.n2 - 1 ? plane : (g.per2 ? -(g.n2 - 1) * plane : 0));
}
__device__ __forceinline__ int tail_zlo(const Grid& g, int k, int plane) {
    return k > 0 ? -plane : (g.per2 ? (g.n2 - 1) * plane : 0);
}

// Damped-Jacobi sweep of the whole level, x -> xout (ZERO: from x = 0), or
// (RESID) the residual b - A x into xout; each cell as k_smooth updates it
// (resid_row as k_resid_restrict forms it).
template <typename T, bool UNIF, bool D3, bool ZERO, bool RESID>
__device__ void tail_sweep(const TailLevel<T>& L, const T* __restrict__ x,
                           const T* __restrict__ b, T omega, T* __restrict__ xout) {
    const Grid& g = L.g;
    const int plane = g.n0 * g.n1;
    tail_columns(L, [&](int col, int i, int j, int k0, int k1) {
        const TailCol q = tail_col(g, i, j);
        auto xv = [&](int idx) -> T { return ZERO ? T(0) : x[idx]; };
        int c = col + k0 * plane;
        T xI = xv(c), xzl = T(0), Lzl = T(0);
        if (D3) {
            xzl = xv(c + tail_zlo(g, k0, plane));
            if (!UNIF) Lzl = L.L2[c];
        }
        for (int k = k0; k < k1; ++k, c += plane) {
            T xzu = T(0), Lzu = T(0);
            bool hzu = false;
            if (D3) {
                const int cu = c + tail_zup(g, k, plane, hzu);
                xzu = xv(cu);
                if (!UNIF) {
                    Lzu = L.L2[cu];
                    if (!hzu) Lzu = T(0);
                }
            }
            const T xxl = xv(c + q.oxm), xxu = xv(c + q.oxp);
            const T xyl = xv(c + q.oym), xyu = xv(c + q.oyp);
            const T bv = b[c];
            T Lxl, Lxu, Lyl, Lyu;
            if (UNIF) {
                Lxl = Lxu = Lyl = Lyu = L.Lc;
            } else {
                Lxl = L.L0[c];
                Lxu = L.L0[c + q.oxp];
                Lyl = L.L1[c];
                Lyu = L.L1[c + q.oyp];
                if (!q.hxu) Lxu = T(0);
                if (!q.hyu) Lyu = T(0);
            }
            if (RESID) {
                const T Lz0 = UNIF ? (D3 ? L.Lc : T(0)) : Lzl, Lz1 = UNIF ? (D3 ? L.Lc : T(0)) : Lzu;
                xout[c] = resid_row(bv, xI, xxl, xxu, xyl, xyu, xzl, xzu, Lxl, Lxu, Lyl, Lyu, Lz0,
                                    Lz1, D3);
            } else if (UNIF) {
                // the sweep of a uniform level: one D, second differences
                const T Ax = jacobi_ax_uniform(xI, xxl, xxu, xyl, xyu, xzl, xzu, L.Lc, D3);
                T D = T(0);
                D += L.Lc + L.Lc;
                D += L.Lc + L.Lc;
                if (D3) D += L.Lc + L.Lc;
                xout[c] = jacobi_new_scaled(xI, bv - Ax, D > T(0), L.wD);
            } else {
                T Ax, D;
                jacobi_terms(xI, xxl, xxu, xyl, xyu, xzl, xzu, Lxl, Lxu, Lyl, Lyu, Lzl, Lzu, D3, Ax,
                             D);
                xout[c] = jacobi_new(xI, bv - Ax, D, omega);
            }
            xzl = xI;
            xI = xzu;
            Lzl = Lzu;
        }
    });
}

// Coarse right-hand side bc from the residual rs of level F: the z pair of
// each child column summed first, then the x pair, then the y pair (the
// order of k_resid_restrict).
template <typename T, bool D3>
__device__ void tail_restrict_sum(const TailLevel<T>& F, const T* __restrict__ rs,
                                  const TailLevel<T>& C, T* __restrict__ bc) {
    const int n0 = F.g.n0, plane = F.g.n0 * F.g.n1, cplane = C.g.n0 * C.g.n1;
    tail_columns(C, [&](int col, int ic, int jc, int k0, int k1) {
        const int f0 = 2 * ic + n0 * (2 * jc);
        for (int kc = k0; kc < k1; ++kc) {
            const int f = f0 + plane * (D3 ? 2 * kc : kc);
            auto zs = [&](int o) -> T { return D3 ? rs[f + o] + rs[f + o + plane] : rs[f + o]; };
            bc[col + kc * cplane] = (zs(0) + zs(1)) + (zs(n0) + zs(n0 + 1));
        }
    });
}

// xout = x + P xc: the coarse correction interpolated onto the level, each
// coarse plane's x / y interpolation formed once per column walk (the
// operations of prolong_at).
template <typename T, bool D3>
__device__ void tail_prolong(const TailLevel<T>& L, const TailLevel<T>& C,
                             const T* __restrict__ xc, const T* __restrict__ x,
                             T* __restrict__ xout) {
    const Grid& g = L.g;
    const int plane = g.n0 * g.n1;
    tail_columns(L, [&](int col, int i, int j, int k0, int k1) {
        int ip, iq, jp, jq;
        prolong_pair(i, C.g.n0, g.per0, ip, iq);
        prolong_pair(j, C.g.n1, g.per1, jp, jq);
        const int cn0 = C.g.n0, cpl = C.g.n0 * C.g.n1;
        auto cplane = [&](int K) -> T {
            const T* r = xc + cpl * K;
            const T lo = lerp34(r[ip + cn0 * jp], r[iq + cn0 * jp]);
            const T hi = lerp34(r[ip + cn0 * jq], r[iq + cn0 * jq]);
            return lerp34(lo, hi);
        };
        int c = col + k0 * plane;
        if (!D3) {
            xout[c] = x[c] + cplane(0);
            return;
        }
        for (int k = k0; k < k1; ++k, c += plane) {
            int kp, kq;
            prolong_pair(k, C.g.n2, g.per2, kp, kq);
            xout[c] = x[c] + lerp34(cplane(kp), cplane(kq));
        }
    });
}

template <typename T, bool UNIF, bool D3>
__global__ __launch_bounds__(kTailThreads) void k_vcycle_tail(TailArgs<T> A) {
    // per level: x0, x1 and b, level after level
    __shared__ T lds[3 * kTailLdsCells];
    __shared__ double sp[kTailCgMax];
    const int n = A.n;
    auto X0 = [&](int l) -> T* { return lds + A.lev[l].ox0; };
    auto X1 = [&](int l) -> T* { return lds + A.lev[l].ox1; };
    auto Bv = [&](int l) -> T* { return lds + A.lev[l].ob; };
    {
        const T* __restrict__ bg = A.b;
        T* __restrict__ b0 = Bv(0);
        const int N = int(cells(A.lev[0].g));
        for (int c = int(threadIdx.x); c < N; c += kTailThreads) b0[c] = bg[c];
        __syncthreads();
    }
    // down: the pre-smoothed iterate stays in x1, x0 takes the residual
    for (int l = 0; l < n - 1; ++l) {
        const TailLevel<T>& L = A.lev[l];
        tail_sweep<T, UNIF, D3, true, false>(L, nullptr, Bv(l), A.omega, X0(l));
        tail_sweep<T, UNIF, D3, false, false>(L, X0(l), Bv(l), A.omega, X1(l));
        tail_sweep<T, UNIF, D3, false, true>(L, X1(l), Bv(l), A.omega, X0(l));
        tail_restrict_sum<T, D3>(L, X0(l), A.lev[l + 1], Bv(l + 1));
    }
    // coarsest: the first wave; each level's corrected iterate then lands in
    // its x0 (the top level's in global memory)
    if (threadIdx.x < 64) {
        const TailLevel<T>& C = A.lev[n - 1];
        coarse_wave_solve<T, 2>(C.g, C.L0, C.L1, C.L2, C.Lc, UNIF ? 1 : 0, Bv(n - 1), X0(n - 1),
                                A.tol, int(cells(C.g)) + 64, sp, A.G, A.ok);
    }
    __syncthreads();
    for (int l = n - 2; l >= 0; --l) {
        const TailLevel<T>& L = A.lev[l];
        tail_prolong<T, D3>(L, A.lev[l + 1], X0(l + 1), X1(l), X0(l));
        tail_sweep<T, UNIF, D3, false, false>(L, X0(l), Bv(l), A.omega, X1(l));
        tail_sweep<T, UNIF, D3, false, false>(L, X1(l), Bv(l), A.omega, l == 0 ? A.x : X0(l));
    }
}

// Per-block class of a level for a tiling (see Coeffs::cls): 0 when every
// face any cell of the block reads equals Lc, or 0 on a non-periodic
// domain-boundary face (exact comparisons: class-0 blocks then compute
// bitwise what reading the arrays gives).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_level_class(TileDev TL, Grid g, Coeffs<T> C,
                                                        unsigned char* __restrict__ cls) {
    __shared__ int any;
    if (threadIdx.x == 0) any = 0;
    __syncthreads();
    const Span sp = tile_span(TL, g.n0, g.n1, g.n2);
    const int i = sp.i, j = sp.j;
    bool odd = false;
    if (i < g.n0 && j < g.n1)
        for (int k = sp.z0; k < sp.z1 && !odd; ++k) {
            const size_t id = cid(g, i, j, k);
            T Lxl, Lxu, Lyl, Lyu, Lzl, Lzu;
            walled_faces<T>(g, i, j, k, C.Lc, Lxl, Lxu, Lyl, Lyu, Lzl, Lzu);
            odd = odd || C.L0[id] != Lxl || C.L1[id] != Lyl;
            if (i < g.n0 - 1 || g.per0) odd = odd || C.L0[cid(g, nb_up(i, g.n0, g.per0), j, k)] != Lxu;
            if (j < g.n1 - 1 || g.per1) odd = odd || C.L1[cid(g, i, nb_up(j, g.n1, g.per1), k)] != Lyu;
            if (g.ndim == 3) {
                odd = odd || C.L2[id] != Lzl;
                if (k < g.n2 - 1 || g.per2)
                    odd = odd || C.L2[cid(g, i, j, nb_up(k, g.n2, g.per2))] != Lzu;
            }
        }
    if (odd) any = 1;  // benign race: every writer stores 1
    __syncthreads();
    if (threadIdx.x == 0) cls[block_linear()] = any ? 1 : 0;
}

// Class of each fused-pair workgroup (k_smooth_pair, MODE 1 / 2): 0 when every
// face of every cell whose first sweep the workgroup computes (its tile
// widened by one cell in x and y, its z chunk by one plane on either side;
// cells outside a non-periodic direction excluded) equals what walled_faces
// gives, else 1.  The workgroup-to-tile map is the pair kernel's.
template <typename T>
__global__ __launch_bounds__(256) void k_pair_class(PairTile P, Grid g, int tx, Coeffs<T> C,
                                                    unsigned char* __restrict__ cls) {
    __shared__ int any;
    if (threadIdx.x == 0) any = 0;
    __syncthreads();
    unsigned blk = blockIdx.x;
    if (P.remap) blk = (blk & 7u) * (P.nb >> 3) + (blk >> 3);
    const int tix = int(blk % unsigned(P.tx));
    blk /= unsigned(P.tx);
    const int tiy = int(blk % unsigned(P.ty));
    const int z0 = int(blk / unsigned(P.ty)) * P.zc;
    const int z1 = min(z0 + P.zc, g.n2);
    const int i0 = tix * tx, j0 = tiy * kPairTY;
    const int wx = tx + 2, wy = kPairTY + 2, wz = z1 - z0 + 2;
    const int count = wx * wy * wz;
    bool odd = false;
    for (int q = int(threadIdx.x); q < count && !odd; q += int(blockDim.x)) {
        int i = i0 - 1 + q % wx;
        int j = j0 - 1 + (q / wx) % wy;
        int k = z0 - 1 + q / (wx * wy);
        if (i < 0 || i >= g.n0) {
            if (!g.per0) continue;
            i = i < 0 ? i + g.n0 : i - g.n0;
        }
        if (j < 0 || j >= g.n1) {
            if (!g.per1) continue;
            j = j < 0 ? j + g.n1 : j - g.n1;
        }
        if (k < 0 || k >= g.n2) {
            if (!g.per2) continue;
            k = k < 0 ? k + g.n2 : k - g.n2;
        }
        const size_t id = cid(g, i, j, k);
        T Lxl, Lxu, Lyl, Lyu, Lzl, Lzu;
        walled_faces<T>(g, i, j, k, C.Lc, Lxl, Lxu, Lyl, Lyu, Lzl, Lzu);
        odd = odd || C.L0[id] != Lxl || C.L1[id] != Lyl || C.L2[id] != Lzl;
        if (i < g.n0 - 1 || g.per0) odd = odd || C.L0[cid(g, nb_up(i, g.n0, g.per0), j, k)] != Lxu;
        if (j < g.n1 - 1 || g.per1) odd = odd || C.L1[cid(g, i, nb_up(j, g.n1, g.per1), k)] != Lyu;
        if (k < g.n2 - 1 || g.per2) odd = odd || C.L2[cid(g, i, j, nb_up(k, g.n2, g.per2))] != Lzu;
    }
    if (odd) any = 1;  // benign race: every writer stores 1
    __syncthreads();
    if (threadIdx.x == 0) cls[blockIdx.x] = any ? 1 : 0;
}

// Ordered list of the class-1 workgroups of a fused-pair tiling: list[k] the
// k-th of them, list[nb] their count.  One workgroup of 1024 threads, each
// scanning a contiguous run of the classes.
__global__ __launch_bounds__(1024) void k_pair_list(const unsigned char* __restrict__ cls,
                                                    unsigned nb, unsigned* __restrict__ list) {
    __shared__ unsigned part[1024];
    const unsigned t = threadIdx.x, per = (nb + 1023u) / 1024u;
    const unsigned a = min(nb, t * per), e = min(nb, a + per);
    unsigned c = 0;
    for (unsigned q = a; q < e; ++q) c += cls[q] != 0 ? 1u : 0u;
    part[t] = c;
    __syncthreads();
    for (unsigned off = 1; off < 1024u; off <<= 1) {  // inclusive scan
        const unsigned v = t >= off ? part[t - off] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    unsigned pos = part[t] - c;
    for (unsigned q = a; q < e; ++q)
        if (cls[q] != 0) list[pos++] = q;
    if (t == 1023u) list[nb] = part[1023];
}

// Coarse coefficient = 1/2 * sum of the fine faces the coarse face covers.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_coarsen(TileDev TL, Grid gf, Grid gc, const T* __restrict__ f0,
                                                    const T* __restrict__ f1,
                                                    const T* __restrict__ f2, T* __restrict__ c0,
                                                    T* __restrict__ c1, T* __restrict__ c2) {
    const Span sp = tile_span(TL, gc.n0, gc.n1, gc.n2);
    const int i = sp.i, j = sp.j;
    if (i >= gc.n0 || j >= gc.n1) return;
    for (int k = sp.z0; k < sp.z1; ++k) {
    const int fz = (gf.n2 > gc.n2) ? 2 : 1;
    const int I = 2 * i, J = 2 * j, K = fz * k;
    T s0 = T(0), s1 = T(0), s2 = T(0);
    for (int dz = 0; dz < fz; ++dz)
        for (int dy = 0; dy < 2; ++dy) s0 += f0[cid(gf, I, J + dy, K + dz)];
    for (int dz = 0; dz < fz; ++dz)
        for (int dx = 0; dx < 2; ++dx) s1 += f1[cid(gf, I + dx, J, K + dz)];
    if (gf.ndim == 3)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) s2 += f2[cid(gf, I + dx, J + dy, K)];
    const size_t id = cid(gc, i, j, k);
    c0[id] = T(0.5) * s0;
    c1[id] = T(0.5) * s1;
    c2[id] = T(0.5) * s2;
    }
}

template <typename T>
__global__ void k_fill(T* __restrict__ p, size_t n, T v) {
    const size_t q = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (q < n) p[q] = v;
}

// x64 += e32 (mixed-precision correction).
__global__ __launch_bounds__(kBlock) void k_axpy64(size_t n, const float* __restrict__ e,
                                                   double* __restrict__ x) {
    const size_t q = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (q < n) x[q] += double(e[q]);
}

// FP64 defect r = (b - mean)|active - A64 x, rounded to FP32 for the inner
// solve; partial sums of r^2 and of the projected b^2.
__global__ __launch_bounds__(kBlock) void k_resid64(TileDev TL, Grid g, XAccess<double, XM_PLAIN> X,
                                                    Coeffs<double> C, const double* __restrict__ b,
                                                    const double* __restrict__ bmean,
                                                    float* __restrict__ r32,
                                                    double* __restrict__ partial) {
    __shared__ double lds[8];
    const Span sp = tile_span(TL, g.n0, g.n1, g.n2);
    const int i = sp.i, j = sp.j;
    double r2 = 0.0, b2 = 0.0;
    // a block of class 0 takes its coefficients from the position (the same
    // values, so the same residual)
    const bool walled = C.cls && C.cls[block_linear()] == 0;
    if (i < g.n0 && j < g.n1 && sp.z0 < sp.z1) {
        // the column walk of k_smooth: x / y neighbour offsets fixed, the
        // lower z neighbour and coefficient carried, every load of a cell
        // issued before any is used (the operations of apply_row, in order)
        const unsigned n0 = unsigned(g.n0), plane = n0 * unsigned(g.n1);
        const bool d3 = g.ndim == 3;
        const int ixm = i > 0 ? i - 1 : (g.per0 ? g.n0 - 1 : i);
        const int ixp = i < g.n0 - 1 ? i + 1 : (g.per0 ? 0 : i);
        const int jym = j > 0 ? j - 1 : (g.per1 ? g.n1 - 1 : j);
        const int jyp = j < g.n1 - 1 ? j + 1 : (g.per1 ? 0 : j);
        const bool hxu = i < g.n0 - 1 || g.per0, hyu = j < g.n1 - 1 || g.per1;
        const int oxm = ixm - i, oxp = ixp - i;
        const int oym = (jym - j) * int(n0), oyp = (jyp - j) * int(n0);
        const double mean = *bmean;
        const double* x = X.x;
        const int k0 = sp.z0;
        unsigned id = unsigned(i) + n0 * unsigned(j) + plane * unsigned(k0);
        double xzl = 0.0, xI = x[id], Lzl = 0.0;
        if (d3) {
            const int km = k0 > 0 ? k0 - 1 : (g.per2 ? g.n2 - 1 : k0);
            xzl = x[id + unsigned(km - k0) * plane];
            Lzl = walled ? ((k0 == 0 && !g.per2) ? 0.0 : C.Lc) : C.L2[id];
        }
        for (int k = k0; k < sp.z1; ++k, id += plane) {
            double xzu = 0.0, Lzu = 0.0;
            bool hzu = false;
            unsigned idu = id;
            if (d3) {
                hzu = k < g.n2 - 1 || g.per2;
                const int ku = k < g.n2 - 1 ? k + 1 : (g.per2 ? 0 : k);
                idu = id + unsigned(ku - k) * plane;
                xzu = x[idu];
            }
            const double xxl = x[id + oxm], xxu = x[id + oxp];
            const double xyl = x[id + oym], xyu = x[id + oyp];
            const double bb = b[id];
            double Lxl, Lxu, Lyl, Lyu;
            if (walled) {
                double zl;
                walled_faces<double>(g, i, j, k, C.Lc, Lxl, Lxu, Lyl, Lyu, zl, Lzu);
            } else {
                Lxl = C.L0[id];
                Lxu = hxu ? C.L0[id + oxp] : 0.0;
                Lyl = C.L1[id];
                Lyu = hyu ? C.L1[id + oyp] : 0.0;
                if (d3) Lzu = hzu ? C.L2[idu] : 0.0;
            }
            double Ax, D;
            jacobi_terms(xI, xxl, xxu, xyl, xyu, xzl, xzu, Lxl, Lxu, Lyl, Lyu, Lzl, Lzu, d3, Ax,
                         D);
            const double bv = (D > 0.0) ? bb - mean : 0.0;
            const double r = bv - Ax;
            r32[id] = float(r);
            r2 += r * r;
            b2 += bv * bv;
            xzl = xI;
            xI = xzu;
            Lzl = Lzu;
        }
    }
    double s, sb;
    block_sum2(r2, b2, lds, s, sb);
    if (threadIdx.x == 0) {
        partial[2 * block_linear()] = s;
        partial[2 * block_linear() + 1] = sb;
    }
}

// Load caller coefficients (ndim consecutive face arrays) into a level,
// forcing zero on non-periodic lower boundary faces and on the z faces in 2D;
// optionally keep an FP64 copy.
template <typename Tin, typename Tout>
__global__ __launch_bounds__(kBlock) void k_load_coeffs(TileDev TL, Grid g, const Tin* __restrict__ src,
                                                        Tout* __restrict__ L0, Tout* __restrict__ L1,
                                                        Tout* __restrict__ L2, double* M0,
                                                        double* M1, double* M2) {
    const Span sp = tile_span(TL, g.n0, g.n1, g.n2);
    const int i = sp.i, j = sp.j;
    if (i >= g.n0 || j >= g.n1) return;
    for (int k = sp.z0; k < sp.z1; ++k) {
    const size_t id = cid(g, i, j, k);
    const size_t N = cells(g);
    const int coord[3] = {i, j, k};
    const int per[3] = {g.per0, g.per1, g.per2};
    Tout* dst[3] = {L0, L1, L2};
    double* d64[3] = {M0, M1, M2};
    for (int d = 0; d < 3; ++d) {
        double v = (d < g.ndim) ? double(src[d * N + id]) : 0.0;
        if (!per[d] && coord[d] == 0) v = 0.0;
        dst[d][id] = Tout(v);
        if (d64[d]) d64[d][id] = v;
    }
    }
}

template <typename Tin, typename Tout>
wl_status mg_load_coeffs(const Grid& g, const Tin* src, Tout* const L[3], double* const L64[3],
                         hipStream_t s) {
    const Launch ln = launch_for(g.n0, g.n1, g.n2);
    k_load_coeffs<Tin, Tout><<<ln.grid, ln.block, 0, s>>>(ln.td, g, src, L[0], L[1], L[2],
                                                          L64 ? L64[0] : nullptr,
                                                          L64 ? L64[1] : nullptr,
                                                          L64 ? L64[2] : nullptr);
    WL_CHECK_LAUNCH();
    return WL_OK;
}
template wl_status mg_load_coeffs<float, float>(const Grid&, const float*, float* const*,
                                                double* const*, hipStream_t);
template wl_status mg_load_coeffs<double, double>(const Grid&, const double*, double* const*,
                                                  double* const*, hipStream_t);
template wl_status mg_load_coeffs<double, float>(const Grid&, const double*, float* const*,
                                                 double* const*, hipStream_t);

template <typename T>
wl_status fill(T* p, size_t n, T v, hipStream_t s) {
    if (n == 0) return WL_OK;
    k_fill<T><<<unsigned((n + 255) / 256), 256, 0, s>>>(p, n, v);
    WL_CHECK_LAUNCH();
    return WL_OK;
}
template wl_status fill<float>(float*, size_t, float, hipStream_t);
template wl_status fill<double>(double*, size_t, double, hipStream_t);

template <typename Tin, typename Tout>
__global__ void k_convert(const Tin* __restrict__ a, Tout* __restrict__ b, size_t n) {
    const size_t q = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (q < n) b[q] = Tout(a[q]);
}

template <typename Tin, typename Tout>
wl_status convert(const Tin* a, Tout* b, size_t n, hipStream_t s) {
    if (n == 0) return WL_OK;
    k_convert<Tin, Tout><<<unsigned((n + 255) / 256), 256, 0, s>>>(a, b, n);
    WL_CHECK_LAUNCH();
    return WL_OK;
}
template wl_status convert<float, double>(const float*, double*, size_t, hipStream_t);
template wl_status convert<double, float>(const double*, float*, size_t, hipStream_t);

// Count of active cells from FP64 coefficients (mixed-precision solver).
wl_status mg_count_active64(const Grid& g, double* const L64[3], Reduce& red, size_t* count,
                            hipStream_t s) {
    const Launch ln = launch_for(g.n0, g.n1, g.n2);
    Coeffs<double> C{L64[0], L64[1], L64[2], 1.0};
    k_sum_active<double, false><<<ln.grid, ln.block, 0, s>>>(ln.td, g, C, nullptr, red.partial);
    WL_CHECK_LAUNCH();
    k_reduce<<<1, 1024, 0, s>>>(red.partial, ln.nblocks(), 1, 1.0, red.result + 6, nullptr,
                                MailboxPost{});
    WL_CHECK_LAUNCH();
    double cnt = 0.0;
    WL_CHECK_HIP(hipMemcpyAsync(&cnt, red.result + 6, sizeof(double), hipMemcpyDeviceToHost, s));
    WL_CHECK_HIP(hipStreamSynchronize(s));
    *count = size_t(cnt);
    return WL_OK;
}

// ----------------------------------------------------------- host driving

template <typename T>
static Coeffs<T> coeffs_of(const Level<T>& L, const unsigned char* cls = nullptr) {
    Coeffs<T> C{L.L[0], L.L[1], L.L[2], L.Lc};
    C.cls = L.uniform ? nullptr : cls;
    return C;
}

// w / D of a uniform level, D summed in the kernels' order.
template <typename T>
static T uniform_wd(const Level<T>& L, T omega) {
    T D = T(0);
    D += L.Lc + L.Lc;
    D += L.Lc + L.Lc;
    if (L.g.ndim == 3) D += L.Lc + L.Lc;
    return D > T(0) ? T(omega / D) : T(0);
}

template <typename T, int XM, bool NORM, bool FIRST>
static wl_status smooth(const Level<T>& L, const T* xin, const T* b, T omega, T* xout,
                        double* partial, const double* bshift, hipStream_t s, int prof = -1,
                        T* bproj = nullptr) {
    const Launch ln = launch_for(L.g.n0, L.g.n1, L.g.n2);
    ProfScope ps(prof, s, cells(L.g));
    XAccess<T, XM> X{xin};
    if (L.uniform)
        k_smooth<T, XM, true, NORM, FIRST><<<ln.grid, ln.block, 0, s>>>(ln.td, 
            L.g, X, coeffs_of(L), b, uniform_wd(L, omega), xout, partial, bshift, bproj);
    else
        k_smooth<T, XM, false, NORM, FIRST><<<ln.grid, ln.block, 0, s>>>(ln.td, 
            L.g, X, coeffs_of(L, L.cls), b, omega, xout, partial, bshift, bproj);
    WL_CHECK_LAUNCH();
    return WL_OK;
}

// Fused pairs run on 3D levels whose x and y extents are multiples of 8:
// uniform, fully periodic levels (one coefficient, w / D per level) and
// non-uniform levels with any boundaries (per-workgroup classes; see
// k_pair_class).  Mode 1: only levels of at least pair_min_cells() cells.
static int pair_tx(int n0) {
    for (int w = 64; w >= 8; w >>= 1)
        if (n0 % w == 0) return w;
    return 0;
}

template <typename T>
static bool pair_ok(const Hierarchy<T>& h, const Level<T>& L) {
    if (!h.pairs || L.g.ndim != 3) return false;
    if (pair_tx(L.g.n0) == 0 || L.g.n1 % kPairTY != 0) return false;
    if (L.uniform) {
        // the uniform kernel wraps every direction
        if (!(L.g.per0 && L.g.per1 && L.g.per2)) return false;
    } else {
        if (!L.cls_fp || !gen_pairs()) return false;
        // mode 1: single-launch pairs up to pair3_max_cells(), two launches
        // from gen_pair_min_cells() on, separate sweeps between
        if (h.pairs != 2 && cells(L.g) > pair3_max_cells() && cells(L.g) < gen_pair_min_cells())
            return false;
    }
    // FP32 pairs address their arrays through buffer descriptors, whose
    // 32-bit byte offsets cover arrays below 4 GiB (2^30 cells)
    if (sizeof(T) == 4 && cells(L.g) >= (size_t(1) << 30)) return false;
    return h.pairs == 2 || cells(L.g) >= pair_min_cells();
}

static PairTile pair_tile(const Grid& g);
static unsigned pair_class_slots(const Grid& g) {
    if (g.ndim != 3 || pair_tx(g.n0) == 0 || g.n1 % kPairTY != 0) return 0;
    return pair_tile(g).nb;
}

static PairTile pair_tile(const Grid& g) {
    PairTile p;
    p.tx = g.n0 / pair_tx(g.n0);
    p.ty = g.n1 / kPairTY;
    const size_t cols = size_t(p.tx) * size_t(p.ty);
    size_t zc = (cols * size_t(g.n2) + pair_blocks() - 1) / pair_blocks();
    // a chunk re-reads two input planes on either side: keep it >= 8 on
    // large levels; small ones favour more, shorter workgroups
    const size_t zmin = cells(g) >= (size_t(1) << 20) ? 8 : 2;
    zc = std::min(std::max(zc, zmin), size_t(g.n2));
    const unsigned chunks = unsigned((size_t(g.n2) + zc - 1) / zc);
    p.zc = int(zc);
    p.nb = unsigned(cols) * chunks;
    p.remap = (p.nb % 8u == 0u) ? 1 : 0;
    // the body chunks of a non-uniform level are walked in parts of about
    // four planes
    p.split = std::max(1, p.zc / 4);
    return p;
}

// xout = S(S(xin)) (XM_ZERO: from zero).  xout must not alias the inputs.
template <typename T, int XM>
static wl_status pair(const Level<T>& L, const T* xin, const T* b, T omega, T* xout,
                      const double* bshift, hipStream_t s, int prof = -1) {
    if (xout == xin || xout == b) {
        set_error("internal: fused sweep pair output aliases an input");
        return WL_ERR_INVALID_ARG;
    }
    const PairTile P = pair_tile(L.g);
    ProfScope ps(prof, s, cells(L.g));
    XAccess<T, XM> X{xin};
    // uniform levels pass w / D, the others w and their classes
    const bool gen = !L.uniform;
    const T wd = gen ? omega : uniform_wd(L, omega);
    const Coeffs<T> C = coeffs_of(L, L.cls_fp);
#define WL_PAIR(TX)                                                                             \
    do {                                                                                        \
        if (gen && cells(L.g) < gen_pair_min_cells()) {                                         \
            k_smooth_pair<T, XM, TX, 3><<<P.nb, PairShape<TX>::T, 0, s>>>(                      \
                P, L.g, X, C, b, wd, xout, bshift, nullptr, nullptr);                           \
        } else if (gen) {                                                                       \
            k_smooth_pair<T, XM, TX, 1><<<P.nb, PairShape<TX>::T, 0, s>>>(                      \
                P, L.g, X, C, b, wd, xout, bshift, nullptr, nullptr);                           \
            if (L.fp_grid)                                                                      \
                k_smooth_pair<T, XM, TX, 2>                                                     \
                    <<<L.fp_grid * unsigned(P.split), PairShape<TX>::T, 0, s>>>(                \
                        P, L.g, X, C, b, wd, xout, bshift, L.fp_list, nullptr);                 \
        } else {                                                                                \
            k_smooth_pair<T, XM, TX, 0><<<P.nb, PairShape<TX>::T, 0, s>>>(                      \
                P, L.g, X, C, b, wd, xout, bshift, nullptr, nullptr);                           \
        }                                                                                       \
    } while (0)
    switch (pair_tx(L.g.n0)) {
        case 64: WL_PAIR(64); break;
        case 32: WL_PAIR(32); break;
        case 16: WL_PAIR(16); break;
        case 8: WL_PAIR(8); break;
        default:
            set_error("internal: no fused-pair tile for this level");
            return WL_ERR_INVALID_ARG;
    }
#undef WL_PAIR
    WL_CHECK_LAUNCH();
    return WL_OK;
}

// Partial-sum slots a measuring pair on a non-uniform level writes (see
// k_smooth_pair's NM).
template <typename T>
static size_t pair_norm_slots(const Level<T>& L) {
    const PairTile P = pair_tile(L.g);
    return size_t(P.nb) + size_t(L.fp_grid) * size_t(P.split);
}

// xout = S(S(xin)) on a non-uniform level, with the residual norm of xin
// (and, FIRST, of the projected b) in partial[0 .. 2 * pair_norm_slots).
template <typename T, bool FIRST>
static wl_status pair_norm(const Level<T>& L, const T* xin, const T* b, T omega, T* xout,
                           const double* bshift, double* partial, hipStream_t s, int prof = -1) {
    if (xout == xin || xout == b || L.uniform) {
        set_error("internal: measuring pair on a uniform level or with aliased buffers");
        return WL_ERR_INVALID_ARG;
    }
    const PairTile P = pair_tile(L.g);
    ProfScope ps(prof, s, cells(L.g));
    XAccess<T, XM_PLAIN> X{xin};
    const Coeffs<T> C = coeffs_of(L, L.cls_fp);
    constexpr int NM = FIRST ? 2 : 1;
#define WL_PAIRN(TX)                                                                            \
    do {                                                                                        \
        k_smooth_pair<T, XM_PLAIN, TX, 1, NM><<<P.nb, PairShape<TX>::T, 0, s>>>(                \
            P, L.g, X, C, b, omega, xout, bshift, nullptr, partial);                            \
        if (L.fp_grid)                                                                          \
            k_smooth_pair<T, XM_PLAIN, TX, 2, NM>                                               \
                <<<L.fp_grid * unsigned(P.split), PairShape<TX>::T, 0, s>>>(                    \
                    P, L.g, X, C, b, omega, xout, bshift, L.fp_list, partial);                  \
    } while (0)
    switch (pair_tx(L.g.n0)) {
        case 64: WL_PAIRN(64); break;
        case 32: WL_PAIRN(32); break;
        case 16: WL_PAIRN(16); break;
        case 8: WL_PAIRN(8); break;
        default:
            set_error("internal: no fused-pair tile for this level");
            return WL_ERR_INVALID_ARG;
    }
#undef WL_PAIRN
    WL_CHECK_LAUNCH();
    return WL_OK;
}

template <typename T>
static wl_status prolong(const Level<T>& L, const Level<T>& C, T* x, hipStream_t s,
                         int prof = -1) {
    const Launch ln = launch_for(L.g.n0, L.g.n1, L.g.n2);
    ProfScope ps(prof, s, cells(L.g));
    k_prolong<T><<<ln.grid, ln.block, 0, s>>>(ln.td, L.g, C.g, C.x[1], x);
    WL_CHECK_LAUNCH();
    return WL_OK;
}

// launch_for over a fine level with its z chunk rounded up to even, so that
// every chunk holds whole z pairs of a restriction.
static Launch launch_pairs(const Grid& g) {
    Launch l = launch_for(g.n0, g.n1, g.n2);
    if (g.n2 > 1 && (l.td.zc & 1)) {
        l.td.zc += 1;
        const unsigned cols = unsigned(l.td.tx) * unsigned(l.td.ty);
        const unsigned chunks = unsigned((g.n2 + l.td.zc - 1) / l.td.zc);
        l.td.nb = cols * chunks;
        l.td.remap = (l.td.nb % 8u == 0u) ? 1 : 0;
        l.grid = dim3(l.td.nb, 1, 1);
    }
    return l;
}

template <typename T>
static wl_status resid_restrict(const Level<T>& L, const T* x, const T* b, const double* bshift,
                                Level<T>& C, hipStream_t s, int prof = -1) {
    const Launch ln = launch_pairs(L.g);
    ProfScope ps(prof, s, cells(L.g));
    XAccess<T, XM_PLAIN> X{x};
    if (L.uniform)
        k_resid_restrict<T, true><<<ln.grid, ln.block, 0, s>>>(ln.td, L.g, C.g, X, coeffs_of(L), b, bshift,
                                                               C.b);
    else
        k_resid_restrict<T, false><<<ln.grid, ln.block, 0, s>>>(ln.td, L.g, C.g, X,
                                                                coeffs_of(L, L.cls_pairs), b,
                                                                bshift, C.b);
    WL_CHECK_LAUNCH();
    return WL_OK;
}

template <typename T>
static wl_status coarse_solve(const Hierarchy<T>& h, const Level<T>& L, T* xout, hipStream_t s) {
    const int N = int(cells(L.g));
    const int maxit = N + 64;
    if (N > kCoarseMax) {
        set_error("internal: coarsest level larger than the one-workgroup solver");
        return WL_ERR_INVALID_ARG;
    }
    if (N <= kCgWaveMax) {
        const bool dir = h.cinv_set && &L == &h.lev[h.nlev - 1];
        k_coarse_cg_wave<T><<<1, 64, 0, s>>>(L.g, coeffs_of(L), L.uniform, L.b, xout, h.coarse_tol,
                                             maxit, dir ? h.cinv : nullptr,
                                             dir ? h.cinv_ok : nullptr);
    } else {
        const unsigned nt = unsigned((N + 63) / 64 * 64);
        k_coarse_cg<T><<<1, nt, 0, s>>>(L.g, coeffs_of(L), L.uniform, L.b, xout, h.coarse_tol,
                                        maxit);
    }
    WL_CHECK_LAUNCH();
    return WL_OK;
}

// First level of the V-cycle tail (k_vcycle_tail), 0 for none: with fused
// kernels on (wl_set_fused_sweeps) and the Jacobi smoother, the first level
// below the fine one of at most tail_cells() cells, provided at least one
// smoothed level lies above the coarsest, the coarsest fits the one-wave
// solve and the levels fit the tail's LDS.
template <typename T>
static int tail_level(const Hierarchy<T>& h) {
    const size_t lim = std::min(tail_cells(), size_t(kTailThreads) * kTailPer);
    if (h.pairs == 0 || h.smoother != 0 || h.nlev < 3 || lim == 0) return 0;
    if (cells(h.lev[h.nlev - 1].g) > size_t(kTailCgMax)) return 0;
    for (int l = 1; l < h.nlev - 1; ++l) {
        if (cells(h.lev[l].g) > lim) continue;
        const int lt = std::max(l, h.nlev - kTailLevels);
        size_t sum = 0;
        for (int q = lt; q < h.nlev; ++q) sum += cells(h.lev[q].g);
        return sum <= size_t(kTailLdsCells) ? lt : 0;
    }
    return 0;
}

template <typename T>
static wl_status vcycle_tail(const Hierarchy<T>& h, int lt, hipStream_t s) {
    TailArgs<T> A{};
    A.n = h.nlev - lt;
    A.omega = T(h.omega);
    A.tol = h.coarse_tol;
    A.b = h.lev[lt].b;
    A.x = h.lev[lt].x[1];
    A.G = h.cinv_set ? h.cinv : nullptr;
    A.ok = h.cinv_set ? h.cinv_ok : nullptr;
    if (A.n < 2 || A.n > kTailLevels) {
        set_error("internal: V-cycle tail of an unsupported depth");
        return WL_ERR_INVALID_ARG;
    }
    const unsigned long long two32 = 1ull << 32;
    int off = 0;
    for (int t = 0; t < A.n; ++t) {
        const Level<T>& L = h.lev[lt + t];
        TailLevel<T>& D = A.lev[t];
        D.g = L.g;
        D.L0 = L.L[0];
        D.L1 = L.L[1];
        D.L2 = L.L[2];
        D.Lc = L.Lc;
        D.wD = uniform_wd(L, T(h.omega));
        const int N = int(cells(L.g)), cols = L.g.n0 * L.g.n1;
        D.m0 = (two32 + unsigned(L.g.n0) - 1) / unsigned(L.g.n0);
        D.mc = (two32 + unsigned(cols) - 1) / unsigned(cols);
        int parts = cols >= kTailThreads ? 1 : std::max(1, std::min(L.g.n2, kTailThreads / cols));
        D.seg = (L.g.n2 + parts - 1) / parts;
        D.parts = (L.g.n2 + D.seg - 1) / D.seg;
        D.ox0 = off;
        D.ox1 = off + N;
        D.ob = off + 2 * N;
        off += 3 * N;
    }
    if (off > 3 * kTailLdsCells) {
        set_error("internal: V-cycle tail levels exceed its LDS");
        return WL_ERR_INVALID_ARG;
    }
    const bool d3 = h.lev[lt].g.ndim == 3;
    if (h.lev[lt].uniform)
        d3 ? k_vcycle_tail<T, true, true><<<1, kTailThreads, 0, s>>>(A)
           : k_vcycle_tail<T, true, false><<<1, kTailThreads, 0, s>>>(A);
    else
        d3 ? k_vcycle_tail<T, false, true><<<1, kTailThreads, 0, s>>>(A)
           : k_vcycle_tail<T, false, false><<<1, kTailThreads, 0, s>>>(A);
    WL_CHECK_LAUNCH();
    return WL_OK;
}

template <typename T>
static wl_status reduce(Reduce& red, size_t nslots, int ncomp, double scale, double* out,
                        hipStream_t s, const MailboxPost& post = MailboxPost{}) {
    k_reduce<<<1, 1024, 0, s>>>(red.partial, nslots, ncomp, scale, out, nullptr, post);
    WL_CHECK_LAUNCH();
    return WL_OK;
}

template <typename T>
wl_status mg_coarsen_all(Hierarchy<T>& h, hipStream_t s) {
    for (int l = 1; l < h.nlev; ++l) {
        Level<T>& F = h.lev[l - 1];
        Level<T>& C = h.lev[l];
        const Launch ln = launch_for(C.g.n0, C.g.n1, C.g.n2);
        k_coarsen<T><<<ln.grid, ln.block, 0, s>>>(ln.td, F.g, C.g, F.L[0], F.L[1], F.L[2], C.L[0],
                                                  C.L[1], C.L[2]);
        WL_CHECK_LAUNCH();
        C.uniform = F.uniform;
        C.Lc = F.Lc * (F.g.ndim == 3 ? T(2) : T(1));
    }
    // block classes of the non-uniform levels for both tilings
    for (int l = 0; l < h.nlev; ++l) {
        Level<T>& L = h.lev[l];
        if (L.uniform || !L.cls) continue;
        const Coeffs<T> C{L.L[0], L.L[1], L.L[2], L.Lc};
        const Launch a = launch_for(L.g.n0, L.g.n1, L.g.n2);
        k_level_class<T><<<a.grid, a.block, 0, s>>>(a.td, L.g, C, L.cls);
        WL_CHECK_LAUNCH();
        const Launch b = launch_pairs(L.g);
        k_level_class<T><<<b.grid, b.block, 0, s>>>(b.td, L.g, C, L.cls_pairs);
        WL_CHECK_LAUNCH();
        if (L.cls_fp) {
            const PairTile P = pair_tile(L.g);
            k_pair_class<T><<<P.nb, 256, 0, s>>>(P, L.g, pair_tx(L.g.n0), C, L.cls_fp);
            WL_CHECK_LAUNCH();
            k_pair_list<<<1, 1024, 0, s>>>(L.cls_fp, P.nb, L.fp_list);
            WL_CHECK_LAUNCH();
        }
    }
    // the coarsest level's inverse on non-uniform levels, where the CG takes
    // many iterations (formed in about a fifth of a V-cycle's time,
    // recovered within a solve); on uniform ones the CG converges in a few
    // and keeps the solve (a cleared flag)
    if (h.cinv) {
        const Level<T>& Cst = h.lev[h.nlev - 1];
        if (h.direct_coarse && !Cst.uniform && direct_coarse_enabled()) {
            k_coarse_inverse<T><<<1, 1024, 0, s>>>(Cst.g, coeffs_of(Cst), Cst.uniform, h.cinv,
                                                   h.cinv_ok);
        } else {
            k_fill<int><<<1, 64, 0, s>>>(h.cinv_ok, 1, 0);
        }
        WL_CHECK_LAUNCH();
        h.cinv_set = true;
    }
    // the class-1 launch's grid covers the largest count met so far; when it
    // grows, captured bodies (whose grids are baked in) are dropped
    unsigned cnt[kMaxLevels] = {};
    bool any = false;
    for (int l = 0; l < h.nlev; ++l) {
        const Level<T>& L = h.lev[l];
        if (L.uniform || !L.cls || !L.cls_fp) continue;
        WL_CHECK_HIP(hipMemcpyAsync(&cnt[l], L.fp_list + pair_tile(L.g).nb, sizeof(unsigned),
                                    hipMemcpyDeviceToHost, s));
        any = true;
    }
    if (any) {
        WL_CHECK_HIP(hipStreamSynchronize(s));
        bool grew = false;
        for (int l = 0; l < h.nlev; ++l) {
            if (cnt[l] > h.lev[l].fp_grid) {
                h.lev[l].fp_grid = cnt[l];
                grew = true;
            }
        }
        if (grew) h.graphs.clear();
    }
    return WL_OK;
}

template <typename T>
wl_status mg_count_active(Hierarchy<T>& h, Reduce& red, hipStream_t s) {
    const Level<T>& F = h.lev[0];
    const Launch ln = launch_for(F.g.n0, F.g.n1, F.g.n2);
    if (F.uniform)
        k_sum_active<T, true><<<ln.grid, ln.block, 0, s>>>(ln.td, F.g, coeffs_of(F), nullptr, red.partial);
    else
        k_sum_active<T, false><<<ln.grid, ln.block, 0, s>>>(ln.td, F.g, coeffs_of(F), nullptr, red.partial);
    WL_CHECK_LAUNCH();
    // result[6] = active count (kept on the device for the mean kernels)
    k_reduce<<<1, 1024, 0, s>>>(red.partial, ln.nblocks(), 1, 1.0, red.result + 6, nullptr,
                                MailboxPost{});
    WL_CHECK_LAUNCH();
    double cnt = 0.0;
    WL_CHECK_HIP(hipMemcpyAsync(&cnt, red.result + 6, sizeof(double), hipMemcpyDeviceToHost, s));
    WL_CHECK_HIP(hipStreamSynchronize(s));
    h.n_active = size_t(cnt);
    return WL_OK;
}

template wl_status mg_coarsen_all<float>(Hierarchy<float>&, hipStream_t);
template wl_status mg_coarsen_all<double>(Hierarchy<double>&, hipStream_t);
template wl_status mg_count_active<float>(Hierarchy<float>&, Reduce&, hipStream_t);
template wl_status mg_count_active<double>(Hierarchy<double>&, Reduce&, hipStream_t);

// How a V-cycle finds the fine level's pre-smoothing: the first sweep
// already done into x[1] (Half), both sweeps still to do from the fine
// iterate (Full) or from zero (Zero).
enum class Pre { Half, Full, Zero, PairDone };

// Pre-smoothing of one level: two sweeps from `home` (or zero), with `other`
// as the second buffer.  Separate sweeps end in home, a fused pair in other;
// *out says where.  b / bs: right-hand side and the mean to remove from it
// (null: none).
template <typename T>
static wl_status pre_smooth(const Hierarchy<T>& h, const Level<T>& L, Pre mode, T* home, T* other,
                            const T* b, const double* bs, hipStream_t s, const T** out,
                            bool fine) {
    const T w = T(h.omega);
    if (mode == Pre::PairDone) {
        // a measuring pair already smoothed home into other
        *out = other;
        return WL_OK;
    }
    if (h.smoother == 1) {
        // conjugate gradients: two iterations from the iterate (or zero), in place
        if (mode == Pre::Half) {
            set_error("internal: half-done pre-smoothing with the CG smoother");
            return WL_ERR_INVALID_ARG;
        }
        WL_TRY(cg_smooth<T>(h, L, home, mode == Pre::Zero, b, bs, 2, s));
        *out = home;
        return WL_OK;
    }
    if (mode != Pre::Half && pair_ok(h, L)) {
        if (mode == Pre::Zero)
            WL_TRY((pair<T, XM_ZERO>(L, nullptr, b, w, other, bs, s,
                                     fine ? WL_PROF_PAIR_FINE : -1)));
        else
            WL_TRY((pair<T, XM_PLAIN>(L, home, b, w, other, bs, s,
                                      fine ? WL_PROF_PAIR_FINE : -1)));
        *out = other;
        return WL_OK;
    }
    if (mode == Pre::Zero)
        WL_TRY((smooth<T, XM_ZERO, false, false>(L, nullptr, b, w, other, nullptr,
                                                 bs, s)));
    else if (mode == Pre::Full)
        WL_TRY((smooth<T, XM_PLAIN, false, false>(L, home, b, w, other, nullptr,
                                                  bs, s)));
    WL_TRY((smooth<T, XM_PLAIN, false, false>(L, other, b, w, home, nullptr, bs, s,
                                              fine ? WL_PROF_SMOOTH_FINE : -1)));
    *out = home;
    return WL_OK;
}

// Post-smoothing of one level: the coarse correction C.x[1] interpolated onto
// the pre-smoothed iterate `pre` (in place), then two sweeps; the result
// lands in home.
template <typename T>
static wl_status post_smooth(const Hierarchy<T>& h, const Level<T>& L, const T* pre, T* home,
                             T* other, const Level<T>& C, const T* b, const double* bs,
                             hipStream_t s, bool fine) {
    const T w = T(h.omega);
    if (h.smoother == 1) {
        WL_TRY(prolong(L, C, home, s, fine ? WL_PROF_PROLONG_FINE : -1));
        return cg_smooth<T>(h, L, home, false, b, bs, 2, s);
    }
    if (pre == other) {
        // only a fused pre-smoothing leaves its result in other
        if (!pair_ok(h, L)) {
            set_error("internal: unfused post-smoothing after a fused pre-smoothing");
            return WL_ERR_INVALID_ARG;
        }
        WL_TRY(prolong(L, C, other, s, fine ? WL_PROF_PROLONG_FINE : -1));
        return pair<T, XM_PLAIN>(L, other, b, w, home, bs, s,
                                 fine ? WL_PROF_PAIR_PROLONG_FINE : -1);
    }
    WL_TRY(prolong(L, C, home, s, fine ? WL_PROF_PROLONG_FINE : -1));
    WL_TRY((smooth<T, XM_PLAIN, false, false>(L, home, b, w, other, nullptr, bs, s,
                                              fine ? WL_PROF_SMOOTH_FINE : -1)));
    return smooth<T, XM_PLAIN, false, false>(L, other, b, w, home, nullptr, bs, s,
                                             fine ? WL_PROF_SMOOTH_FINE : -1);
}

// Remainder of one V-cycle: fine pre-smoothing as `mode` says, restriction,
// the coarse levels, and post-smoothing; leaves the fine iterate in
// lev[0].x[0].  Level l > 0 keeps its result in x[1] (where the next finer
// prolongation reads it) and uses x[0] as the second buffer.
template <typename T>
static wl_status vcycle_rest(Hierarchy<T>& h, Pre mode, const T* fb, const double* fshift,
                             hipStream_t s) {
    // fb / fshift: fine-level right-hand side and the mean to remove from it
    // on the fly (null: fb is already projected)
    Level<T>& F = h.lev[0];
    if (h.nlev == 1) return coarse_solve(h, F, F.x[0], s);
    const T* pre[kMaxLevels];
    // levels 1 .. top - 1 run per-level kernels; from top on, the tail
    // kernel (or, without one, the coarsest solve alone)
    const int lt = tail_level(h);
    const int top = lt > 0 ? lt : h.nlev - 1;
    WL_TRY(pre_smooth(h, F, mode, F.x[0], F.x[1], fb, fshift, s, &pre[0], true));
    WL_TRY(resid_restrict(F, pre[0], fb, fshift, h.lev[1], s, WL_PROF_RESTRICT_FINE));
    for (int l = 1; l < top; ++l) {
        Level<T>& L = h.lev[l];
        WL_TRY(pre_smooth(h, L, Pre::Zero, L.x[1], L.x[0], L.b, nullptr, s, &pre[l], false));
        WL_TRY(resid_restrict(L, pre[l], L.b, nullptr, h.lev[l + 1], s));
    }
    if (lt > 0) {
        WL_TRY(vcycle_tail(h, lt, s));
    } else {
        Level<T>& Cst = h.lev[h.nlev - 1];
        WL_TRY(coarse_solve(h, Cst, Cst.x[1], s));
    }
    for (int l = top - 1; l >= 1; --l) {
        Level<T>& L = h.lev[l];
        WL_TRY(post_smooth(h, L, pre[l], L.x[1], L.x[0], h.lev[l + 1], L.b, nullptr, s, false));
    }
    return post_smooth(h, F, pre[0], F.x[0], F.x[1], h.lev[1], fb, fshift, s, true);
}

// Sums [b, b^2, c, c^2] of a producer-side first check (see BPartials) ->
// result[4] = sum b, result[5] = mean m over the active count *count,
// result[1] = ||b - m||^2 and result[0] = an upper bound of ||c - m||^2:
// sum c^2 - 2 m sum c + n m^2 plus a bound of the FP64 rounding of those
// sums (negligible when m is small, as on periodic grids); posts result[0..1].
__global__ __launch_bounds__(1024) void k_check_reduce(const double* __restrict__ partial,
                                                       size_t nslots,
                                                       const double* __restrict__ count,
                                                       double* __restrict__ out,
                                                       MailboxPost post) {
    __shared__ double lds[64];
    double S[4];
    wg_slot_reduce<4, false>(partial, nslots, S, lds);
    if (threadIdx.x == 0) {
        const double n = *count;
        const double m = n > 0.0 ? S[0] / n : 0.0;
        const double nm2 = n * m * m;
        const double r2 = S[3] - 2.0 * m * S[2] + nm2;
        // relative rounding of sums of up to 2^31 terms, taken generously
        const double err = 1e-6 * (S[3] + 2.0 * fabs(m * S[2]) + nm2);
        out[0] = fmax(r2, 0.0) + err;
        out[1] = fmax(S[1] - m * S[0], 0.0);
        out[4] = S[0];
        out[5] = m;
        if (post.vals) mailbox_write(post, out);
    }
}

template <typename T>
bool mg_producer_check(const Hierarchy<T>& h) {
    return h.nlev > 1 && h.lev[0].uniform && pair_ok(h, h.lev[0]);
}
template bool mg_producer_check<float>(const Hierarchy<float>&);
template bool mg_producer_check<double>(const Hierarchy<double>&);

template <typename T>
static wl_status active_mean(Hierarchy<T>& h, Reduce& red, const T* b, bool have_partials,
                             hipStream_t s) {
    const Level<T>& F = h.lev[0];
    const Launch ln = launch_for(F.g.n0, F.g.n1, F.g.n2);
    if (have_partials) {
        // the producer of b left its per-block active sums in red.partial
    } else if (F.uniform)
        k_sum_active<T, true><<<ln.grid, ln.block, 0, s>>>(ln.td, F.g, coeffs_of(F), b, red.partial);
    else
        k_sum_active<T, false><<<ln.grid, ln.block, 0, s>>>(ln.td, F.g, coeffs_of(F, F.cls), b,
                                                            red.partial);
    WL_CHECK_LAUNCH();
    // result[4] = sum, result[5] = mean over the active count result[6]
    k_reduce<<<1, 1024, 0, s>>>(red.partial, ln.nblocks(), 1, 1.0, red.result + 4,
                                red.result + 6, MailboxPost{});
    WL_CHECK_LAUNCH();
    return WL_OK;
}

template <typename T>
wl_status mg_solve(Hierarchy<T>& h, Reduce& red, T* x, const T* b, double tol, double abs_r2,
                   int max_vcycles, hipStream_t s, SolveResult* res, BPartials bp,
                   const SolveTail* tail) {
    Level<T>& F = h.lev[0];
    F.x[0] = x;
    const T w = T(h.omega);
    const Launch ln = launch_for(F.g.n0, F.g.n1, F.g.n2);
    // With fused fine pairs each V-cycle starts with both pre-sweeps from x
    // and the residual checks only measure; otherwise every check is also
    // the first pre-sweep of the next V-cycle (into F.x[1]).
    const bool fused = h.nlev > 1 && pair_ok(h, F);
    // with CG smoothing, too, the checks only measure and each V-cycle
    // smooths from the iterate
    const bool measure = fused || h.smoother == 1;
    T* const xnext = measure ? nullptr : F.x[1];
    // On a fused non-uniform fine level each check is the next V-cycle's
    // pre-smoothing pair, which measures its input as it goes (into F.x[1];
    // the last one, after convergence, is not used): no separate pass reads
    // x and b for the norm.
    const bool pairnorm = fused && !F.uniform && pair_norm_slots(F) <= red.slots;
    const size_t nslots = pairnorm ? pair_norm_slots(F) : ln.nblocks();
    if (bp == BPartials::Check && !mg_producer_check(h)) {
        set_error("internal: first residual check given for a hierarchy that cannot take it");
        return WL_ERR_INVALID_ARG;
    }
    // the norm reductions post ||r||^2, ||b - mean||^2 to mailbox slots 0, 1
    MailboxPost post;
    WL_TRY(mailbox_post_args(red, 0, 2, s, &post));
    const double* bshift = red.result + 5;
    if (bp == BPartials::Check) {
        // the producer of b evaluated the first check
        k_check_reduce<<<1, 1024, 0, s>>>(red.partial, red.pslots ? red.pslots : ln.nblocks(),
                                          red.result + 6, red.result, post);
        WL_CHECK_LAUNCH();
    } else {
        WL_TRY(active_mean(h, red, b, bp == BPartials::Sums, s));
        // first check: ||r0|| and ||b - mean||.  Every fine-level sweep
        // removes the mean of b on the fly; only a one-level hierarchy (whose
        // coarse solve reads F.b) stores the projected copy.
        if (pairnorm)
            WL_TRY((pair_norm<T, true>(F, x, b, w, F.x[1], bshift, red.partial, s)));
        else
            WL_TRY((smooth<T, XM_PLAIN, true, true>(F, x, b, w, xnext, red.partial,
                                                    bshift, s, -1, h.nlev == 1 ? F.b : nullptr)));
        WL_TRY(reduce<T>(red, nslots, 2, 1.0, red.result, s, post));
    }
    host_posted(red);
    const unsigned q_check = red.mb.seq;
    // speculate that the initial iterate already converges: the tail runs on
    // it while the host waits for the norms (not for the tail's own posts,
    // which the caller reads later)
    if (tail) WL_TRY((*tail)(s));
    WL_TRY(host_wait_seq(red, q_check, s));
    double nr[2] = {host_slot(red, 0), host_slot(red, 1)};
    if (!std::isfinite(nr[0]) || !std::isfinite(nr[1])) {
        set_error("non-finite residual norm in the pressure solve");
        return WL_ERR_NONFINITE;
    }
    const double b2 = nr[1];
    res->bnorm = std::sqrt(b2);
    if (b2 == 0.0) {
        const size_t N = cells(F.g);
        k_fill<T><<<unsigned((N + 255) / 256), 256, 0, s>>>(x, N, T(0));
        WL_CHECK_LAUNCH();
        res->vcycles = 0;
        res->rel = 0.0;
        if (tail) WL_TRY((*tail)(s));
        return WL_OK;
    }
    double r2 = nr[0];
    auto done = [&](double q) { return q <= tol * tol * b2 || q <= abs_r2; };
    int k = 0;
    // one V-cycle and the residual norms it leaves (replayed as a graph)
    auto body = [&](hipStream_t q) -> wl_status {
        if (pairnorm) {
            WL_TRY(vcycle_rest(h, Pre::PairDone, b, bshift, q));
            WL_TRY((pair_norm<T, false>(F, x, b, w, F.x[1], bshift, red.partial, q,
                                        WL_PROF_PAIR_FINE)));
            return reduce<T>(red, nslots, 2, 1.0, red.result, q, post);
        }
        WL_TRY(vcycle_rest(h, measure ? Pre::Full : Pre::Half, b, bshift, q));
        WL_TRY((smooth<T, XM_PLAIN, true, false>(F, x, b, w, xnext, red.partial,
                                                 bshift, q,
                                                 measure ? WL_PROF_NORM_FINE : WL_PROF_SMOOTH_NORM)));
        return reduce<T>(red, ln.nblocks(), 2, 1.0, red.result, q, post);
    };
    while (!done(r2) && k < max_vcycles) {
        WL_TRY(run_cached(h.graphs, x, b, s, body));
        ++k;
        host_posted(red);
        WL_TRY(host_wait(red, s));
        nr[0] = host_slot(red, 0);
        nr[1] = host_slot(red, 1);
        if (!std::isfinite(nr[0])) {
            set_error("non-finite residual norm in the pressure solve");
            return WL_ERR_NONFINITE;
        }
        r2 = nr[0];
    }
    res->vcycles = k;
    res->rel = std::sqrt(r2 / b2);
    res->r2 = r2;
    // the speculative tail saw the initial iterate: run it again
    if (tail && k > 0) WL_TRY((*tail)(s));
    if (!done(r2)) {
        set_error("pressure solve reached max_vcycles before the tolerance");
        return WL_ERR_NOT_CONVERGED;
    }
    return WL_OK;
}

template wl_status mg_solve<float>(Hierarchy<float>&, Reduce&, float*, const float*, double,
                                   double, int, hipStream_t, SolveResult*, BPartials,
                                   const SolveTail*);
template wl_status mg_solve<double>(Hierarchy<double>&, Reduce&, double*, const double*, double,
                                    double, int, hipStream_t, SolveResult*, BPartials,
                                    const SolveTail*);

wl_status mg_mixed_classes(const Grid& g, const Mixed64& m, hipStream_t s) {
    if (!m.cls) return WL_OK;
    const Launch ln = launch_for(g.n0, g.n1, g.n2);
    const Coeffs<double> C{m.L[0], m.L[1], m.L[2], 1.0};
    k_level_class<double><<<ln.grid, ln.block, 0, s>>>(ln.td, g, C, m.cls);
    WL_CHECK_LAUNCH();
    return WL_OK;
}

wl_status mg_solve_mixed(Hierarchy<float>& h32, const Mixed64& m, Reduce& red, double* x,
                         const double* b, double tol, double abs_r2, int max_vcycles,
                         hipStream_t s, SolveResult* res) {
    Level<float>& F = h32.lev[0];
    const Grid g = F.g;
    const Launch ln = launch_for(g.n0, g.n1, g.n2);
    const size_t N = cells(g);
    Coeffs<double> C64{m.L[0], m.L[1], m.L[2], 1.0};
    C64.cls = m.cls;
    // active mean of b in FP64 (result[5])
    k_sum_active<double, false><<<ln.grid, ln.block, 0, s>>>(ln.td, g, C64, b, red.partial);
    WL_CHECK_LAUNCH();
    k_reduce<<<1, 1024, 0, s>>>(red.partial, ln.nblocks(), 1, 1.0, red.result + 4,
                                red.result + 6, MailboxPost{});
    WL_CHECK_LAUNCH();
    int inner_total = 0;
    double b2 = -1.0, r2 = 0.0;
    auto done = [&](double q) { return q <= tol * tol * b2 || q <= abs_r2; };
    // FP64 residual (projected into the FP32 fine RHS) and its norms, posted
    // to mailbox slots 0, 1 (each execution is matched by one host_posted)
    MailboxPost post;
    WL_TRY(mailbox_post_args(red, 0, 2, s, &post));
    auto resid = [&](hipStream_t q) -> wl_status {
        XAccess<double, XM_PLAIN> X{x};
        k_resid64<<<ln.grid, ln.block, 0, q>>>(ln.td, g, X, C64, b, red.result + 5, F.b, red.partial);
        WL_CHECK_LAUNCH();
        return reduce<double>(red, ln.nblocks(), 2, 1.0, red.result, q, post);
    };
    // `count` inner FP32 V-cycles on A e = r from e = 0, x += e in FP64, and
    // the next residual
    auto outer = [&](hipStream_t q, int count) -> wl_status {
        for (int v = 0; v < count; ++v)
            WL_TRY(vcycle_rest(h32, v == 0 ? Pre::Zero : Pre::Full, static_cast<const float*>(F.b),
                               nullptr, q));
        k_axpy64<<<unsigned((N + kBlock - 1) / kBlock), kBlock, 0, q>>>(N, F.x[0], x);
        WL_CHECK_LAUNCH();
        return resid(q);
    };
    WL_TRY(resid(s));
    for (;;) {
        // one resid has run since the last wait
        host_posted(red);
        WL_TRY(host_wait(red, s));
        const double nr[2] = {host_slot(red, 0), host_slot(red, 1)};
        if (!std::isfinite(nr[0]) || !std::isfinite(nr[1])) {
            set_error("non-finite residual norm in the mixed-precision solve");
            return WL_ERR_NONFINITE;
        }
        if (b2 < 0.0) {
            b2 = nr[1];
            res->bnorm = std::sqrt(b2);
            if (b2 == 0.0) {
                k_fill<double><<<unsigned((N + 255) / 256), 256, 0, s>>>(x, N, 0.0);
                WL_CHECK_LAUNCH();
                res->vcycles = 0;
                res->rel = 0.0;
                return WL_OK;
            }
        }
        r2 = nr[0];
        if (done(r2) || inner_total >= max_vcycles) break;
        const int count = std::min(m.inner, max_vcycles - inner_total);
        if (count == m.inner)
            WL_TRY(run_cached(h32.graphs, x, b, s, [&](hipStream_t q) { return outer(q, count); }));
        else
            WL_TRY(outer(s, count));
        inner_total += count;
    }
    res->vcycles = inner_total;
    res->rel = std::sqrt(r2 / b2);
    res->r2 = r2;
    if (!done(r2)) {
        set_error("mixed-precision solve reached max_vcycles before the tolerance");
        return WL_ERR_NOT_CONVERGED;
    }
    return WL_OK;
}

}  // namespace wl

extern "C" wl_status wl_set_smoother(int kind) {
    wl::clear_error();
    if (kind != WL_SMOOTH_JACOBI && kind != WL_SMOOTH_CG) {
        wl::set_error("wl_set_smoother: kind must be WL_SMOOTH_JACOBI or WL_SMOOTH_CG");
        return WL_ERR_INVALID_ARG;
    }
    wl::g_smoother.store(kind, std::memory_order_relaxed);
    return WL_OK;
}

extern "C" wl_status wl_set_fused_sweeps(int mode) {
    wl::clear_error();
    if (mode < 0 || mode > 2) {
        wl::set_error("wl_set_fused_sweeps: mode must be 0, 1 or 2");
        return WL_ERR_INVALID_ARG;
    }
    wl::g_pairs.store(mode, std::memory_order_relaxed);
    return WL_OK;
}
