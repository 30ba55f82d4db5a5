// Batched Navier-Stokes runs for serving many small simulations: one
// persistent kernel whose workgroups take requests from a device work queue
// (an atomic head over the request table) until it is empty.  A request is a
// whole run of `steps` CFL-adaptive Heun steps (Sec. 3's simstep!) taken by
// the one workgroup that took it: every phase of the step (CFL!, convdiff!,
// BC!, BDIM!, project!) is a loop of the workgroup over the cells followed by
// a barrier, with FP32 fields and each pressure solve in FP32 V-cycles with
// an FP64 defect correction (Sec. 2's GMG; the mixed precision of WL_MIXED).
// Every reduction is a fixed-order workgroup sum, so a request's result does
// not depend on which workgroup ran it or on the rest of the batch.  The
// per-face arithmetic (limited flux, ghost rules, BDIM blend, measure) is the
// device code the tiled kernels use.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "wl_internal.h"
#include "wl_ns.h"
#include "wl_nsdev.h"
#include "wl_vel.h"
#include "wl_wg.h"
#include "wl_wgsolve.h"

namespace wl {
namespace {

constexpr int kNsThreads = 512;
constexpr size_t kNsMaxCells = 262144;  // per request (e.g. 512^2, 64^3)

struct NsReq {
    Grid g;
    int bclo[3], bchi[3];
    float U[3];
    float nu;
    double cfl;
    BodyDev body;
    double tol;
    int max_vcycles, steps, nlev;
    float omega;
    int outflow;
    float* u[3];          // state (caller, in/out)
    float* uout;          // state outflow plane (caller) or null
    float* u1[3];         // predictor result
    float* f[3];          // stage field before BDIM
    float* gg[3];         // stage field after BDIM
    float* out1;          // predictor's outflow plane
    float* fo;            // stage plane
    float* mu0[3];
    float* mu1n[9];
    float* p32;
    double* sigma;        // projection right-hand side (FP64)
    WgLevel<double> F;    // x[0] = caller pressure (FP64), b = projected sigma, L = FP64 coefficients
    WgLevel<float> lev[kMaxLevels];
};

struct NsRes {
    int status, vcycles;
    double t, dt;
};

__device__ inline double wg_max(double v, double* red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < int(blockDim.x + 63) / 64; ++w) s = fmax(s, red[w]);
    __syncthreads();
    return s;
}

__device__ inline VelField<float> field(const NsReq& q, float* const u[3], const float* plane) {
    VelField<float> V;
    for (int c = 0; c < 3; ++c) {
        V.u[c] = u[c];
        V.bclo[c] = q.bclo[c];
        V.bchi[c] = q.bchi[c];
        V.U[c] = q.U[c];
    }
    V.uout = plane;
    V.g = q.g;
    return V;
}

// dt = cfl / (max_I sum_c [max(u_c(I + delta_c), 0) - min(u_c(I), 0)] + 2 d nu)
__device__ double wg_cfl(const NsReq& q, const VelField<float>& V, double* red) {
    const Grid& g = q.g;
    const int N = int(cells(g));
    double m = 0.0;
    for (int c = threadIdx.x; c < N; c += blockDim.x) {
        int i, j, k;
        wg_coords(g, c, i, j, k);
        float s = 0.0f;
        for (int d = 0; d < g.ndim; ++d) {
            const float up = vget<float, false>(V, d, i + (d == 0), j + (d == 1), k + (d == 2));
            s += fmaxf(up, 0.0f) - fminf(V.u[d][c], 0.0f);
        }
        m = fmax(m, double(s));
    }
    m = wg_max(m, red);
    const double den = m + 2.0 * g.ndim * double(q.nu);
    return den > 0.0 ? q.cfl / den : 0.0;
}

// Stage field: f = u_e + dt R(u_e) (predictor) or (u_n + u_e + dt R(u_e)) / 2,
// R_c = -sum_d [F_cd(I + delta_d) - F_cd(I)]; boundary faces at their value.
__device__ void wg_momentum(const NsReq& q, const VelField<float>& E, float* const un[3],
                            float* const fo[3], float dt, bool corr) {
    const Grid& g = q.g;
    const int N = int(cells(g));
    const int per[3] = {g.per0, g.per1, g.per2};
    for (int cc = threadIdx.x; cc < N; cc += blockDim.x) {
        int i, j, k;
        wg_coords(g, cc, i, j, k);
        const int coord[3] = {i, j, k};
        for (int c = 0; c < g.ndim; ++c) {
            if (!per[c] && coord[c] == 0) {
                fo[c][cc] = (E.bclo[c] == WL_BC_INFLOW) ? E.U[c] : 0.0f;
                continue;
            }
            float R = 0.0f;
            for (int d = 0; d < g.ndim; ++d) {
                const float Flo = face_flux<float, false>(E, c, d, i, j, k, q.nu);
                const float Fhi =
                    face_flux<float, false>(E, c, d, i + (d == 0), j + (d == 1), k + (d == 2), q.nu);
                R -= Fhi - Flo;
            }
            const float ue = E.u[c][cc];
            fo[c][cc] = corr ? 0.5f * (un[c][cc] + ue + dt * R) : ue + dt * R;
        }
    }
    __syncthreads();
}

// Outflow plane: d(uout)/dt = -U_x (uout - u_x(n0-1)) in the stage form, then
// a uniform shift making its flux equal to the inflow plane's.
__device__ void wg_outflow(const NsReq& q, const float* ue_x, const float* out_e, const float* out_n,
                           const float* f_x, float dt, bool corr, float* fout, double* red) {
    const Grid& g = q.g;
    const int P = g.n1 * g.n2;
    const float Ux = q.U[0];
    double sin_ = 0.0, sout = 0.0;
    for (int p = threadIdx.x; p < P; p += blockDim.x) {
        const int j = p % g.n1, k = p / g.n1;
        const float last = ue_x[cid(g, g.n0 - 1, j, k)];
        const float R = -Ux * (out_e[p] - last);
        const float f = corr ? 0.5f * (out_n[p] + out_e[p] + dt * R) : out_e[p] + dt * R;
        fout[p] = f;
        sout += double(f);
        sin_ += double(f_x[cid(g, 0, j, k)]);
    }
    const double tin = wg_sum(sin_, red);
    const double tout = wg_sum(sout, red);
    const float shift = float((tin - tout) / double(P));
    for (int p = threadIdx.x; p < P; p += blockDim.x) fout[p] += shift;
    __syncthreads();
}

// One projected stage from the stage field in q.f / q.fo: BDIM, divergence,
// the mixed-precision pressure solve (warm-started, relative tolerance) and
// the pressure-gradient update into out (coef = c dt).  Returns the solve's
// status; adds its V-cycles to *vc.
__device__ int wg_project_stage(const NsReq& q, double coef, float* const out[3], int* vc,
                                CoarseLds& S) {
    const Grid& g = q.g;
    const int N = int(cells(g));
    const int per[3] = {g.per0, g.per1, g.per2};
    float* const* us = q.f;
    if (q.body.kind != 0) {
        BdimFields<float> B;
        for (int c = 0; c < 3; ++c) B.mu0[c] = q.mu0[c];
        for (int c = 0; c < 9; ++c) B.mu1n[c] = q.mu1n[c];
        B.cls = nullptr;
        const VelField<float> Fv = field(q, q.f, q.fo);
        const BodyMotionDev rest{};
        for (int cc = threadIdx.x; cc < N; cc += blockDim.x) {
            int i, j, k;
            wg_coords(g, cc, i, j, k);
            for (int c = 0; c < g.ndim; ++c) q.gg[c][cc] = bdim_face<float>(Fv, B, rest, c, i, j, k);
        }
        __syncthreads();
        us = q.gg;
    }
    const VelField<float> V = field(q, us, q.fo);
    const float scale = float(1.0 / coef);
    for (int cc = threadIdx.x; cc < N; cc += blockDim.x) {
        int i, j, k;
        wg_coords(g, cc, i, j, k);
        float div = 0.0f;
        for (int d = 0; d < g.ndim; ++d)
            div += vget<float, false>(V, d, i + (d == 0), j + (d == 1), k + (d == 2)) - V.u[d][cc];
        q.sigma[cc] = double(div * scale);
    }
    __syncthreads();
    const double b2 = wg_project_rhs(q.F, q.sigma, S.red);
    int status = WL_OK;
    if (b2 > 0.0) {
        int k = 0;
        double r2 = 0.0;
        status = wg_solve_mixed(q.F, q.lev, q.nlev, q.omega, q.tol * q.tol * b2, 0.0,
                                q.max_vcycles, S, &k, &r2);
        *vc += k;
    } else {
        for (int cc = threadIdx.x; cc < N; cc += blockDim.x) q.F.x[0][cc] = 0.0;
        __syncthreads();
    }
    for (int cc = threadIdx.x; cc < N; cc += blockDim.x) q.p32[cc] = float(q.F.x[0][cc]);
    __syncthreads();
    const float* L[3] = {q.lev[0].L[0], q.lev[0].L[1], q.lev[0].L[2]};
    for (int cc = threadIdx.x; cc < N; cc += blockDim.x) {
        int i, j, k;
        wg_coords(g, cc, i, j, k);
        const int coord[3] = {i, j, k};
        const int n[3] = {g.n0, g.n1, g.n2};
        for (int c = 0; c < g.ndim; ++c) {
            int lo[3] = {i, j, k};
            lo[c] = coord[c] > 0 ? coord[c] - 1 : (per[c] ? n[c] - 1 : coord[c]);
            const float cl = float(coef) * L[c][cc];
            out[c][cc] = proj_face(us[c][cc], cl, q.p32[cc], q.p32[cid(g, lo[0], lo[1], lo[2])]);
        }
    }
    __syncthreads();
    return status;
}

__device__ void run_one(const NsReq& q, NsRes& res, CoarseLds& S) {
    const Grid& g = q.g;
    const int N = int(cells(g));
    // geometry of the body (at rest): moments, FP64 coefficients, FP32 levels
    for (int cc = threadIdx.x; cc < N; cc += blockDim.x) {
        int i, j, k;
        wg_coords(g, cc, i, j, k);
        for (int c = 0; c < g.ndim; ++c) {
            double m0, m1, nrm[3];
            measure_face(g, q.body, c, i, j, k, m0, m1, nrm);
            q.mu0[c][cc] = float(m0);
            for (int d = 0; d < g.ndim; ++d) q.mu1n[3 * c + d][cc] = float(m1 * nrm[d]);
            q.F.L[c][cc] = face_coeff(g, q.bclo, c, i, j, k, m0);
        }
    }
    __syncthreads();
    wg_coeffs32(q.F, q.lev, q.nlev);
    double t = 0.0, dt = 0.0;
    int vc = 0, status = WL_OK;
    for (int step = 0; step < q.steps; ++step) {
        dt = wg_cfl(q, field(q, q.u, q.uout), S.red);
        if (!(dt > 0.0) || !isfinite(dt)) {
            status = WL_ERR_INVALID_ARG;
            break;
        }
        const float dtf = float(dt);
        // predictor (c = 1)
        wg_momentum(q, field(q, q.u, q.uout), q.u, q.f, dtf, false);
        if (q.outflow) wg_outflow(q, q.u[0], q.uout, q.uout, q.f[0], dtf, false, q.fo, S.red);
        int st = wg_project_stage(q, dt, q.u1, &vc, S);
        if (st != WL_OK && status == WL_OK) status = st;
        if (q.outflow) {
            for (int p = threadIdx.x; p < g.n1 * g.n2; p += blockDim.x) q.out1[p] = q.fo[p];
            __syncthreads();
        }
        // corrector (c = 1/2)
        wg_momentum(q, field(q, q.u1, q.out1), q.u, q.f, dtf, true);
        if (q.outflow) wg_outflow(q, q.u1[0], q.out1, q.uout, q.f[0], dtf, true, q.fo, S.red);
        st = wg_project_stage(q, 0.5 * dt, q.u, &vc, S);
        if (st != WL_OK && status == WL_OK) status = st;
        if (q.outflow) {
            for (int p = threadIdx.x; p < g.n1 * g.n2; p += blockDim.x) q.uout[p] = q.fo[p];
            __syncthreads();
        }
        t += dt;
    }
    if (threadIdx.x == 0) res = NsRes{status, vc, t, dt};
    __syncthreads();
}

__global__ __launch_bounds__(kNsThreads) void k_ns_batch(const NsReq* __restrict__ reqs, int count,
                                                         unsigned* head, NsRes* __restrict__ res) {
    __shared__ CoarseLds S;
    __shared__ int take;
    for (;;) {
        if (threadIdx.x == 0) take = int(atomicAdd(head, 1u));
        __syncthreads();
        const int r = take;
        __syncthreads();
        if (r >= count) return;
        run_one(reqs[r], res[r], S);
    }
}

wl_status bad(int r, const std::string& msg) {
    set_error("NS request " + std::to_string(r) + ": " + msg);
    return WL_ERR_INVALID_ARG;
}

// Checks one request and fills its descriptor, carving its arrays.
wl_status plan_one(const wl_ns_request& in, int r, Carver& c, NsReq& q) {
    const int ndim = in.ndim;
    if (ndim != 2 && ndim != 3) return bad(r, "ndim must be 2 or 3");
    if (ndim == 2 && in.n[2] != 1) return bad(r, "2D problems need n[2] == 1");
    int blo[3] = {in.bc_lo[0], in.bc_lo[1], in.bc_lo[2]};
    int bhi[3] = {in.bc_hi[0], in.bc_hi[1], in.bc_hi[2]};
    if (ndim == 2) blo[2] = bhi[2] = WL_BC_WALL;
    for (int d = 0; d < ndim; ++d) {
        if (in.n[d] < 4) return bad(r, "every direction needs at least 4 cells");
        if (blo[d] < 0 || blo[d] > 3 || bhi[d] < 0 || bhi[d] > 3) return bad(r, "unknown boundary code");
        if ((blo[d] == WL_BC_PERIODIC) != (bhi[d] == WL_BC_PERIODIC))
            return bad(r, "periodic boundaries must be set on both faces of a direction");
        if (blo[d] == WL_BC_OUTFLOW || bhi[d] == WL_BC_INFLOW ||
            (d > 0 && (blo[d] == WL_BC_INFLOW || bhi[d] == WL_BC_OUTFLOW)))
            return bad(r, "INFLOW only on the lower and OUTFLOW only on the upper x face");
    }
    const size_t N = size_t(in.n[0]) * in.n[1] * in.n[2];
    if (N > kNsMaxCells) return bad(r, "more than 262144 cells (use a simulation handle)");
    if (in.body.kind < 0 || in.body.kind > 2) return bad(r, "body.kind must be 0, 1 or 2");
    for (int d = 0; d < 3; ++d)
        if (in.body.velocity[d] != 0.0 || in.body.amplitude[d] != 0.0 || in.body.spin[d] != 0.0)
            return bad(r, "batched runs take bodies at rest");
    if (in.body.kind != 0 && !(in.body.radius > 0.0)) return bad(r, "body radius must be > 0");
    if (in.body.kind == 2 && (ndim != 3 || !(in.body.radius2 > 0.0)))
        return bad(r, "a torus needs ndim = 3 and radius2 > 0");
    if (!(in.tol >= 0.0) || in.max_vcycles < 0 || in.steps < 0 || !(in.nu >= 0.0))
        return bad(r, "tol, nu, max_vcycles and steps must be >= 0");
    const bool outflow = bhi[0] == WL_BC_OUTFLOW;
    if (!in.u || !in.p || (outflow && !in.uout)) return bad(r, "u / p (/ uout) is NULL");
    const int nlev = auto_levels(ndim, in.n, 0);
    int m[3] = {in.n[0], in.n[1], in.n[2]};
    for (int l = 1; l < nlev; ++l)
        for (int d = 0; d < ndim; ++d) m[d] /= 2;
    if (size_t(m[0]) * m[1] * m[2] > size_t(kCoarseMax))
        return bad(r, "coarsest multigrid level exceeds 1024 cells");
    q = NsReq{};
    q.g = Grid{in.n[0], in.n[1], in.n[2], blo[0] == WL_BC_PERIODIC, blo[1] == WL_BC_PERIODIC,
               ndim == 3 && blo[2] == WL_BC_PERIODIC, ndim};
    for (int d = 0; d < 3; ++d) {
        q.bclo[d] = blo[d];
        q.bchi[d] = bhi[d];
        q.U[d] = float(in.U[d]);
    }
    q.nu = float(in.nu);
    q.cfl = in.cfl > 0.0 ? in.cfl : 0.5;
    q.body = BodyDev{in.body.kind, {in.body.centre[0], in.body.centre[1], in.body.centre[2]},
                     in.body.radius, in.body.eps > 0.0 ? in.body.eps : 1.0, in.body.radius2};
    q.tol = in.tol;
    q.max_vcycles = in.max_vcycles > 0 ? in.max_vcycles : 100;
    q.steps = in.steps;
    q.nlev = nlev;
    q.omega = float(2.0 * ndim / (2.0 * ndim + 1.0));
    q.outflow = outflow ? 1 : 0;
    const size_t P = size_t(in.n[1]) * in.n[2];
    float* u = static_cast<float*>(const_cast<void*>(in.u));
    for (int d = 0; d < 3; ++d) q.u[d] = d < ndim ? u + d * N : nullptr;
    q.uout = outflow ? static_cast<float*>(in.uout) : nullptr;
    for (int d = 0; d < 3; ++d) {
        q.u1[d] = d < ndim ? c.take<float>(N) : nullptr;
        q.f[d] = d < ndim ? c.take<float>(N) : nullptr;
        q.gg[d] = d < ndim ? c.take<float>(N) : nullptr;
        q.mu0[d] = d < ndim ? c.take<float>(N) : nullptr;
    }
    for (int e = 0; e < 9; ++e) q.mu1n[e] = (e / 3 < ndim && e % 3 < ndim) ? c.take<float>(N) : nullptr;
    q.out1 = outflow ? c.take<float>(P) : nullptr;
    q.fo = outflow ? c.take<float>(P) : nullptr;
    q.p32 = c.take<float>(N);
    q.sigma = c.take<double>(N);
    q.F.g = q.g;
    q.F.x[0] = static_cast<double*>(in.p);
    q.F.x[1] = nullptr;
    q.F.b = c.take<double>(N);
    for (int d = 0; d < 3; ++d) q.F.L[d] = d < ndim ? c.take<double>(N) : nullptr;
    q.F.Lc = 1.0;
    q.F.uniform = 0;
    int n[3] = {in.n[0], in.n[1], in.n[2]};
    for (int l = 0; l < nlev; ++l) {
        WgLevel<float>& L = q.lev[l];
        L.g = Grid{n[0], n[1], n[2], q.g.per0, q.g.per1, q.g.per2, ndim};
        L.Lc = 1.0f;
        L.uniform = 0;
        const size_t Nl = size_t(n[0]) * n[1] * n[2];
        L.x[0] = c.take<float>(Nl);
        L.x[1] = c.take<float>(Nl);
        L.b = c.take<float>(Nl);
        for (int d = 0; d < 3; ++d) L.L[d] = d < ndim ? c.take<float>(Nl) : nullptr;
        for (int d = 0; d < ndim; ++d) n[d] /= 2;
    }
    return WL_OK;
}

struct NsLayout {
    NsReq* dev_reqs = nullptr;
    NsRes* dev_res = nullptr;
    unsigned* dev_head = nullptr;
};

wl_status plan(const wl_ns_request* reqs, int count, Carver& c, NsLayout& lay, NsReq* table) {
    if (count < 0) return set_error("count must be >= 0"), WL_ERR_INVALID_ARG;
    if (count > 0 && !reqs) return set_error("reqs is NULL"), WL_ERR_INVALID_ARG;
    lay.dev_reqs = c.take<NsReq>(size_t(count > 0 ? count : 1));
    lay.dev_res = c.take<NsRes>(size_t(count > 0 ? count : 1));
    lay.dev_head = c.take<unsigned>(1);
    for (int r = 0; r < count; ++r) {
        NsReq q;
        WL_TRY(plan_one(reqs[r], r, c, q));
        if (table) table[r] = q;
    }
    return WL_OK;
}

int ns_compute_units() {
    static const int n = [] {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) != hipSuccess) return 256;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return 256;
        return v > 0 ? v : 256;
    }();
    return n;
}

}  // namespace
}  // namespace wl

using namespace wl;

extern "C" {

wl_status wl_ns_batch_footprint(const wl_ns_request* reqs, int count, size_t* bytes) {
    clear_error();
    if (!bytes) return set_error("bytes is NULL"), WL_ERR_INVALID_ARG;
    if (count < 0) return set_error("count must be >= 0"), WL_ERR_INVALID_ARG;
    if (count > 0 && !reqs) return set_error("reqs is NULL"), WL_ERR_INVALID_ARG;
    Carver c;
    c.take<NsReq>(size_t(count > 0 ? count : 1));
    c.take<NsRes>(size_t(count > 0 ? count : 1));
    c.take<unsigned>(1);
    for (int r = 0; r < count; ++r) {
        // the caller's arrays need not exist yet for a footprint query
        wl_ns_request probe = reqs[r];
        probe.u = probe.p = probe.uout = reinterpret_cast<void*>(uintptr_t(256));
        NsReq q;
        WL_TRY(plan_one(probe, r, c, q));
    }
    *bytes = c.off;
    return WL_OK;
}

wl_status wl_ns_batch_run(const wl_ns_request* reqs, int count, void* workspace, size_t ws_bytes,
                          void* hip_stream, wl_ns_result* results) {
    clear_error();
    if (count == 0) return WL_OK;
    if (count < 0) return set_error("count must be >= 0"), WL_ERR_INVALID_ARG;
    if (!workspace || !results) return set_error("workspace / results is NULL"), WL_ERR_INVALID_ARG;
    if (reinterpret_cast<uintptr_t>(workspace) % 256)
        return set_error("workspace must be 256-byte aligned"), WL_ERR_INVALID_ARG;
    Carver need;
    NsLayout dry;
    WL_TRY(plan(reqs, count, need, dry, nullptr));
    if (ws_bytes < need.off) {
        set_error("workspace smaller than wl_ns_batch_footprint");
        return WL_ERR_OUT_OF_MEMORY;
    }
    std::vector<NsReq> table(static_cast<size_t>(count));
    Carver c;
    c.base = static_cast<char*>(workspace);
    NsLayout lay;
    WL_TRY(plan(reqs, count, c, lay, table.data()));
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    const unsigned zero = 0u;
    WL_CHECK_HIP(hipMemcpyAsync(lay.dev_reqs, table.data(), sizeof(NsReq) * size_t(count),
                                hipMemcpyHostToDevice, s));
    WL_CHECK_HIP(hipMemcpyAsync(lay.dev_head, &zero, sizeof(zero), hipMemcpyHostToDevice, s));
    const int grid = std::min(count, ns_compute_units());
    k_ns_batch<<<grid, kNsThreads, 0, s>>>(lay.dev_reqs, count, lay.dev_head, lay.dev_res);
    WL_CHECK_HIP(hipGetLastError());
    std::vector<NsRes> res(static_cast<size_t>(count));
    WL_CHECK_HIP(hipMemcpyAsync(res.data(), lay.dev_res, sizeof(NsRes) * size_t(count),
                                hipMemcpyDeviceToHost, s));
    WL_CHECK_HIP(hipStreamSynchronize(s));
    wl_status worst = WL_OK;
    for (int r = 0; r < count; ++r) {
        results[r].status = res[r].status;
        results[r].vcycles = res[r].vcycles;
        results[r].t = res[r].t;
        results[r].dt = res[r].dt;
        if (res[r].status != WL_OK && worst == WL_OK) worst = wl_status(res[r].status);
    }
    if (worst == WL_ERR_NOT_CONVERGED) set_error("some pressure solves reached max_vcycles");
    if (worst == WL_ERR_NONFINITE) set_error("non-finite residual in a batched run");
    if (worst == WL_ERR_INVALID_ARG) set_error("a batched run met a non-positive time step");
    return worst;
}

}  // extern "C"
