// Device-side helpers shared by the HIP translation units: cell indexing,
// the coefficient-weighted 2d-point stencil and deterministic block sums.
#pragma once

#include "wl_internal.h"

namespace wl {

struct Span {
    int i, j;    // cell column of this thread
    int z0, z1;  // z planes [z0, z1) it walks
};

__device__ __forceinline__ Span tile_span(const TileDev& T, int n0, int n1, int n2) {
    unsigned b = blockIdx.x;
    if (T.remap) b = (b & 7u) * (T.nb >> 3) + (b >> 3);
    const unsigned tix = b % unsigned(T.tx);
    b /= unsigned(T.tx);
    const unsigned tiy = b % unsigned(T.ty);
    const unsigned ch = b / unsigned(T.ty);
    const int bx = 1 << T.lbx;
    Span s;
    s.i = int(tix) * bx + int(threadIdx.x & unsigned(bx - 1));
    s.j = int(tiy) * (kBlock >> T.lbx) + int(threadIdx.x >> T.lbx);
    s.z0 = int(ch) * T.zc;
    s.z1 = min(s.z0 + T.zc, n2);
    return s;
}

__device__ __forceinline__ size_t cid(const Grid& g, int i, int j, int k) {
    return size_t(i) + size_t(g.n0) * (size_t(j) + size_t(g.n1) * size_t(k));
}

// Lower / upper neighbour coordinate along one direction (clamped when the
// direction is not periodic; the face coefficient is zero there).
__device__ __forceinline__ int nb_lo(int c, int n, int per) {
    return c > 0 ? c - 1 : (per ? n - 1 : c);
}
__device__ __forceinline__ int nb_up(int c, int n, int per) {
    return c < n - 1 ? c + 1 : (per ? 0 : c);
}

// How a smoother reads the iterate: the stored x, or zero (first sweep on a
// coarse level).
enum { XM_PLAIN = 0, XM_ZERO = 1 };

template <typename T, int XM>
struct XAccess {
    const T* __restrict__ x;
    __device__ __forceinline__ T operator()(const Grid& g, int i, int j, int k) const {
        if (XM == XM_ZERO) return T(0);
        return x[cid(g, i, j, k)];
    }
};

// Cell-centred linear interpolation weights along one direction: fine cell
// c sits a quarter of a coarse cell from the centre of its parent c >> 1,
// towards the parent's lower neighbour when c is even and its upper one when
// c is odd; it takes 3/4 of the parent and 1/4 of that neighbour.  Across a
// periodic direction the neighbour wraps; across a non-periodic domain face
// it is the parent itself (the even reflection of a zero normal gradient).
__device__ __forceinline__ void prolong_pair(int c, int nc, int per, int& p, int& q) {
    p = c >> 1;
    q = (c & 1) ? p + 1 : p - 1;
    if (q < 0) q = per ? nc - 1 : p;
    if (q >= nc) q = per ? 0 : p;
}

template <typename T>
__device__ __forceinline__ T lerp34(T nearv, T farv) {
    return fma(T(0.75), nearv, T(0.25) * farv);
}

// (P xc)(i, j, k): the coarse correction interpolated onto fine cell
// (i, j, k), direction by direction (x, then y, then z; z only when it was
// coarsened, i.e. in 3D).
template <typename T>
__device__ __forceinline__ T prolong_at(const Grid& g, const Grid& gc, const T* __restrict__ xc,
                                        int i, int j, int k) {
    int ip, iq, jp, jq;
    prolong_pair(i, gc.n0, g.per0, ip, iq);
    prolong_pair(j, gc.n1, g.per1, jp, jq);
    const size_t n0 = size_t(gc.n0), pl = n0 * size_t(gc.n1);
    auto plane = [&](size_t base) -> T {
        const T* r = xc + base;
        const T lo = lerp34(r[ip + n0 * jp], r[iq + n0 * jp]);
        const T hi = lerp34(r[ip + n0 * jq], r[iq + n0 * jq]);
        return lerp34(lo, hi);
    };
    if (gc.n2 == g.n2) return plane(pl * size_t(k));
    int kp, kq;
    prolong_pair(k, gc.n2, g.per2, kp, kq);
    return lerp34(plane(pl * size_t(kp)), plane(pl * size_t(kq)));
}

template <typename T>
struct Coeffs {
    const T* __restrict__ L0;
    const T* __restrict__ L1;
    const T* __restrict__ L2;
    T Lc;  // the constant coefficient when the level is uniform
    // Optional per-block classes of the launching kernel's tiling: 0 where
    // every face of every cell of the block equals Lc except non-periodic
    // domain-boundary faces (0), so the coefficients follow from the position
    // and need not be read; null: always read them.
    const unsigned char* __restrict__ cls = nullptr;
};

// Face coefficients of cell (i, j, k) on a block of class 0 (see Coeffs::cls):
// Lc, or 0 on a non-periodic domain-boundary face.  Exactly the stored values.
template <typename T>
__device__ __forceinline__ void walled_faces(const Grid& g, int i, int j, int k, T Lc, T& Lxl,
                                             T& Lxu, T& Lyl, T& Lyu, T& Lzl, T& Lzu) {
    Lxl = (i == 0 && !g.per0) ? T(0) : Lc;
    Lxu = (i == g.n0 - 1 && !g.per0) ? T(0) : Lc;
    Lyl = (j == 0 && !g.per1) ? T(0) : Lc;
    Lyu = (j == g.n1 - 1 && !g.per1) ? T(0) : Lc;
    Lzl = (g.ndim == 3 && !(k == 0 && !g.per2)) ? Lc : T(0);
    Lzu = (g.ndim == 3 && !(k == g.n2 - 1 && !g.per2)) ? Lc : T(0);
}

// (A x)(I) and the diagonal magnitude D(I) = sum of the 2d face coefficients,
// for A x = sum_d L_d(I+delta_d)(x(I+delta_d)-x(I)) - L_d(I)(x(I)-x(I-delta_d)).
template <typename T, int XM, bool UNIF>
__device__ __forceinline__ void apply_row(const Grid& g, const XAccess<T, XM>& X, const Coeffs<T>& C,
                                          int i, int j, int k, T& xI, T& Ax, T& D) {
    xI = X(g, i, j, k);
    Ax = T(0);
    D = T(0);
    const size_t id = cid(g, i, j, k);
    // direction 0
    {
        T Llo, Lup;
        if (UNIF) {
            Llo = C.Lc;
            Lup = C.Lc;
        } else {
            Llo = C.L0[id];
            Lup = (i < g.n0 - 1) ? C.L0[id + 1] : (g.per0 ? C.L0[id - (g.n0 - 1)] : T(0));
        }
        const T xl = X(g, nb_lo(i, g.n0, g.per0), j, k);
        const T xu = X(g, nb_up(i, g.n0, g.per0), j, k);
        Ax += Lup * (xu - xI) - Llo * (xI - xl);
        D += Llo + Lup;
    }
    // direction 1
    {
        T Llo, Lup;
        if (UNIF) {
            Llo = C.Lc;
            Lup = C.Lc;
        } else {
            Llo = C.L1[id];
            Lup = (j < g.n1 - 1) ? C.L1[id + g.n0]
                                 : (g.per1 ? C.L1[id - size_t(g.n1 - 1) * g.n0] : T(0));
        }
        const T xl = X(g, i, nb_lo(j, g.n1, g.per1), k);
        const T xu = X(g, i, nb_up(j, g.n1, g.per1), k);
        Ax += Lup * (xu - xI) - Llo * (xI - xl);
        D += Llo + Lup;
    }
    // direction 2 (absent in 2D, where the z faces carry zero coefficients)
    if (g.ndim == 3) {
        const size_t plane = size_t(g.n0) * g.n1;
        T Llo, Lup;
        if (UNIF) {
            Llo = C.Lc;
            Lup = C.Lc;
        } else {
            Llo = C.L2[id];
            Lup = (k < g.n2 - 1) ? C.L2[id + plane]
                                 : (g.per2 ? C.L2[id - size_t(g.n2 - 1) * plane] : T(0));
        }
        const T xl = X(g, i, j, nb_lo(k, g.n2, g.per2));
        const T xu = X(g, i, j, nb_up(k, g.n2, g.per2));
        Ax += Lup * (xu - xI) - Llo * (xI - xl);
        D += Llo + Lup;
    }
}

// Deterministic sum of one double per thread over a 256-thread block: wave
// butterflies, then the 4 wave totals in index order.  Returns the total in
// thread 0 (other threads get an unspecified value).
__device__ __forceinline__ double block_sum(double v, double* lds /* >= 4 */) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int t = threadIdx.x + blockDim.x * threadIdx.y;
    if ((t & 63) == 0) lds[t >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (t == 0) {
        const int nw = (blockDim.x * blockDim.y + 63) >> 6;
        for (int w = 0; w < nw; ++w) s += lds[w];
    }
    return s;
}

// Two deterministic block sums in one pass (lds >= 8 doubles); totals in
// thread 0.
__device__ __forceinline__ void block_sum2(double a, double b, double* lds, double& sa,
                                           double& sb) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_xor(a, off, 64);
        b += __shfl_xor(b, off, 64);
    }
    const int t = threadIdx.x;
    if ((t & 63) == 0) {
        lds[t >> 6] = a;
        lds[4 + (t >> 6)] = b;
    }
    __syncthreads();
    sa = sb = 0.0;
    if (t == 0)
        for (int w = 0; w < (kBlock >> 6); ++w) {
            sa += lds[w];
            sb += lds[4 + w];
        }
}

__device__ __forceinline__ double block_max(double v, double* lds) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    const int t = threadIdx.x + blockDim.x * threadIdx.y;
    if ((t & 63) == 0) lds[t >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (t == 0) {
        const int nw = (blockDim.x * blockDim.y + 63) >> 6;
        s = lds[0];
        for (int w = 1; w < nw; ++w) s = fmax(s, lds[w]);
    }
    return s;
}

__device__ __forceinline__ unsigned block_linear() { return blockIdx.x; }

// One workgroup: fixed-order sums (MAX: maxima, of values >= 0) of K values
// per slot over nslots slots (partial[K * q + k]): thread t takes slots t,
// t + blockDim.x, ..., then wave butterflies, then the waves in index order.
// Results in out[] of thread 0.  lds: >= 16 * K doubles.
template <int K, bool MAX>
__device__ inline void wg_slot_reduce(const double* __restrict__ partial, size_t nslots,
                                      double (&out)[K], double* lds) {
    double v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = 0.0;
    for (size_t q = threadIdx.x; q < nslots; q += blockDim.x)
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const double p = partial[K * q + k];
            v[k] = MAX ? fmax(v[k], p) : v[k] + p;
        }
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const double o = __shfl_xor(v[k], off, 64);
            v[k] = MAX ? fmax(v[k], o) : v[k] + o;
        }
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) lds[(threadIdx.x >> 6) * K + k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = int(blockDim.x + 63) >> 6;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double s = 0.0;
            for (int w = 0; w < nw; ++w) s = MAX ? fmax(s, lds[w * K + k]) : s + lds[w * K + k];
            out[k] = s;
        }
    }
}

// One thread: a mailbox post, the values, then (after a system-scope fence)
// the next sequence number, counted in device memory.
__device__ inline void mailbox_write(const MailboxPost& P, const double* src) {
    for (int k = 0; k < P.n; ++k) P.vals[P.slot + k] = src[k];
    const double q = *P.counter + 1.0;
    *P.counter = q;
    __threadfence_system();
    __hip_atomic_store(P.seqw, unsigned(q), __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Cell r of the one-cell ring around a w x h rectangle, in coordinates of the
// ring's (w + 2) x (h + 2) box: bottom row, top row, left and right columns.
__device__ __forceinline__ void ring_cell(int r, int w, int h, int& x, int& y) {
    const int W = w + 2;
    if (r < W) {
        x = r;
        y = 0;
    } else if (r < 2 * W) {
        x = r - W;
        y = h + 1;
    } else if (r < 2 * W + h) {
        x = 0;
        y = r - 2 * W + 1;
    } else {
        x = W - 1;
        y = r - 2 * W - h + 1;
    }
}

}  // namespace wl
