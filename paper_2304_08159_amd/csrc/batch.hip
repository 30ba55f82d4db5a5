// Batched Poisson solves for many small problems: one persistent kernel whose
// workgroups take requests from a device work queue (an atomic head index
// over the request table) until it is empty; a request is solved entirely by
// the workgroup that took it, with the same method as wl_poisson_solve
// (Sec. 2's project!: matrix-free GMG, damped Jacobi, sum restriction,
// cell-centred linear prolongation, coarse coefficients = 1/2 the covered fine
// faces, minimum-norm coarsest solve) in FP64, or in FP32 V-cycles with an
// FP64 defect correction around them (per request).  Every reduction is a
// fixed-order workgroup sum, so a request's result does not depend on which
// workgroup solved it or on the rest of the batch.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "wl_internal.h"
#include "wl_wg.h"
#include "wl_wgsolve.h"

namespace wl {
namespace {

constexpr int kBatchThreads = 1024;
constexpr size_t kBatchMaxCells = 262144;  // per request (e.g. 512^2, 64^3)

using BatchLevel = WgLevel<double>;  // uniform = 0, Lc = 1 (coefficients from the request)

struct BatchReq {
    int nlev;
    double tol, omega;
    int max_vcycles;
    int mixed;                            // FP32 inner V-cycles, FP64 outer
    const double* b_in;
    BatchLevel lev[kMaxLevels];           // mixed: only the fine level (FP64 x, b, L)
    WgLevel<float> lev32[kMaxLevels];     // mixed: the FP32 hierarchy
};


struct BatchRes {
    int status, vcycles;
    double rel;
};

__device__ void solve_one(const BatchReq& q, BatchRes& res, CoarseLds& S) {
    const BatchLevel& F = q.lev[0];
    const int nlev = q.nlev;
    const double w = q.omega;
    double* red = S.red;
    double* x = F.x[0];
    double* x1 = F.x[1];
    const int N = int(cells(F.g));
    for (int l = 1; l < nlev; ++l) wg_coarsen<double>(q.lev[l - 1], q.lev[l]);
    // right-hand side projected onto the active cells, mean-free there
    const XAccess<double, XM_ZERO> Z{nullptr};
    const Coeffs<double> C = wg_coeffs(F);
    double sb = 0.0, cnt = 0.0;
    for (int c = threadIdx.x; c < N; c += blockDim.x) {
        int i, j, k;
        wg_coords(F.g, c, i, j, k);
        double xI, Ax, D;
        apply_row<double, XM_ZERO, false>(F.g, Z, C, i, j, k, xI, Ax, D);
        if (D > 0.0) {
            sb += q.b_in[c];
            cnt += 1.0;
        }
    }
    sb = wg_sum(sb, red);
    cnt = wg_sum(cnt, red);
    const double mean = cnt > 0.0 ? sb / cnt : 0.0;
    double b2 = 0.0;
    for (int c = threadIdx.x; c < N; c += blockDim.x) {
        int i, j, k;
        wg_coords(F.g, c, i, j, k);
        double xI, Ax, D;
        apply_row<double, XM_ZERO, false>(F.g, Z, C, i, j, k, xI, Ax, D);
        const double bv = D > 0.0 ? q.b_in[c] - mean : 0.0;
        F.b[c] = bv;
        b2 += bv * bv;
    }
    __syncthreads();
    b2 = wg_sum(b2, red);
    if (b2 == 0.0) {
        for (int c = threadIdx.x; c < N; c += blockDim.x) x[c] = 0.0;
        __syncthreads();
        if (threadIdx.x == 0) res = BatchRes{WL_OK, 0, 0.0};
        __syncthreads();
        return;
    }
    const double tol2 = q.tol * q.tol * b2;
    // first sweep of the first V-cycle, with the norm of the initial residual
    double r2 = wg_sweep<double, XM_PLAIN>(F, XAccess<double, XM_PLAIN>{x}, F.b, w,
                                           x1, true, red);
    int k = 0;
    int status = WL_OK;
    while (!(r2 <= tol2) && k < q.max_vcycles) {
        if (!isfinite(r2)) {
            status = WL_ERR_NONFINITE;
            break;
        }
        if (nlev == 1) {
            coarse_cg_block<double>(F.g, C, 0, F.b, x, 1e-10, N + 64, S);
        } else {
            wg_sweep<double, XM_PLAIN>(F, XAccess<double, XM_PLAIN>{x1}, F.b, w, x, false, red);
            wg_restrict<double>(F, x, F.b, q.lev[1]);
            wg_vcycle_tail<double>(&q.lev[1], nlev - 1, w, 1e-10, S);
            const BatchLevel& C1 = q.lev[1];
            wg_prolong<double>(F, C1, C1.x[1], x);
            wg_sweep<double, XM_PLAIN>(F, XAccess<double, XM_PLAIN>{x}, F.b, w, x1, false, red);
            wg_sweep<double, XM_PLAIN>(F, XAccess<double, XM_PLAIN>{x1}, F.b, w, x, false, red);
        }
        ++k;
        r2 = wg_sweep<double, XM_PLAIN>(F, XAccess<double, XM_PLAIN>{x}, F.b, w, x1,
                                        true, red);
    }
    if (status == WL_OK && !isfinite(r2)) status = WL_ERR_NONFINITE;
    if (status == WL_OK && !(r2 <= tol2)) status = WL_ERR_NOT_CONVERGED;
    if (threadIdx.x == 0) res = BatchRes{status, k, sqrt(r2 / b2)};
    __syncthreads();
}

// Mixed precision (see wg_solve_mixed): the FP32 coefficients of every level
// from the request's FP64 ones, the projected right-hand side, then the
// defect-correction loop.
__device__ void solve_one_mixed(const BatchReq& q, BatchRes& res, CoarseLds& S) {
    const BatchLevel& F = q.lev[0];
    wg_coeffs32(F, q.lev32, q.nlev);
    const double b2 = wg_project_rhs(F, q.b_in, S.red);
    if (b2 == 0.0) {
        const int N = int(cells(F.g));
        for (int c = threadIdx.x; c < N; c += blockDim.x) F.x[0][c] = 0.0;
        __syncthreads();
        if (threadIdx.x == 0) res = BatchRes{WL_OK, 0, 0.0};
        __syncthreads();
        return;
    }
    double r2 = 0.0;
    int k = 0;
    const int st = wg_solve_mixed(F, q.lev32, q.nlev, float(q.omega), q.tol * q.tol * b2, 0.0,
                                  q.max_vcycles, S, &k, &r2);
    if (threadIdx.x == 0) res = BatchRes{st, k, sqrt(r2 / b2)};
    __syncthreads();
}

// Persistent kernel: each workgroup takes the next request from the queue
// until none is left (every workgroup reaches the exit).
__global__ __launch_bounds__(kBatchThreads) void k_poisson_batch(const BatchReq* __restrict__ reqs,
                                                                 int count, unsigned* head,
                                                                 BatchRes* __restrict__ res) {
    __shared__ CoarseLds S;
    __shared__ int take;
    for (;;) {
        if (threadIdx.x == 0) take = int(atomicAdd(head, 1u));
        __syncthreads();
        const int r = take;
        __syncthreads();
        if (r >= count) return;
        if (reqs[r].mixed)
            solve_one_mixed(reqs[r], res[r], S);
        else
            solve_one(reqs[r], res[r], S);
    }
}

// Checks one request and fills its descriptor, carving its level arrays.
wl_status plan_one(const wl_batch_request& in, Carver& c, BatchReq& q) {
    const int ndim = in.ndim;
    if (ndim != 2 && ndim != 3) return set_error("batch request: ndim must be 2 or 3"), WL_ERR_INVALID_ARG;
    if (ndim == 2 && in.n[2] != 1) {
        set_error("batch request: 2D problems need n[2] == 1");
        return WL_ERR_INVALID_ARG;
    }
    for (int d = 0; d < ndim; ++d)
        if (in.n[d] < 2) {
            set_error("batch request: every direction needs at least 2 cells");
            return WL_ERR_INVALID_ARG;
        }
    const size_t N = size_t(in.n[0]) * in.n[1] * in.n[2];
    if (N > kBatchMaxCells) {
        set_error("batch request larger than 262144 cells (use wl_poisson_solve)");
        return WL_ERR_INVALID_ARG;
    }
    if (!(in.tol >= 0.0) || in.max_vcycles < 0) {
        set_error("batch request: tol must be >= 0 and max_vcycles >= 0");
        return WL_ERR_INVALID_ARG;
    }
    const int nlev = auto_levels(ndim, in.n, 0);
    int m[3] = {in.n[0], in.n[1], in.n[2]};
    for (int l = 1; l < nlev; ++l)
        for (int d = 0; d < ndim; ++d) m[d] /= 2;
    if (size_t(m[0]) * m[1] * m[2] > size_t(kCoarseMax)) {
        set_error("batch request: coarsest multigrid level exceeds 1024 cells");
        return WL_ERR_INVALID_ARG;
    }
    if (in.mixed != 0 && in.mixed != 1) {
        set_error("batch request: mixed must be 0 or 1");
        return WL_ERR_INVALID_ARG;
    }
    q = BatchReq{};
    q.nlev = nlev;
    q.tol = in.tol;
    q.omega = 2.0 * ndim / (2.0 * ndim + 1.0);
    q.max_vcycles = in.max_vcycles;
    q.mixed = in.mixed;
    q.b_in = static_cast<const double*>(in.b);
    int n[3] = {in.n[0], in.n[1], in.n[2]};
    if (in.mixed) {
        // FP64 fine level (x, projected b, the request's coefficients) and an
        // FP32 hierarchy (e, sweep buffer, right-hand side, coefficients)
        BatchLevel& F = q.lev[0];
        F.g = Grid{n[0], n[1], n[2], in.periodic[0] != 0, in.periodic[1] != 0,
                   ndim == 3 && in.periodic[2] != 0, ndim};
        F.Lc = 1.0;
        F.uniform = 0;
        const size_t N0 = size_t(n[0]) * n[1] * n[2];
        F.x[0] = static_cast<double*>(in.x);
        F.x[1] = nullptr;
        F.b = c.take<double>(N0);
        const double* co = static_cast<const double*>(in.coeffs);
        for (int d = 0; d < 3; ++d) F.L[d] = d < ndim ? const_cast<double*>(co + d * N0) : nullptr;
        for (int l = 0; l < nlev; ++l) {
            WgLevel<float>& L = q.lev32[l];
            L.g = Grid{n[0], n[1], n[2], F.g.per0, F.g.per1, F.g.per2, ndim};
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
    for (int l = 0; l < nlev; ++l) {
        BatchLevel& L = q.lev[l];
        L.g = Grid{n[0], n[1], n[2], in.periodic[0] != 0, in.periodic[1] != 0,
                   ndim == 3 && in.periodic[2] != 0, ndim};
        L.Lc = 1.0;
        L.uniform = 0;
        const size_t Nl = size_t(n[0]) * n[1] * n[2];
        if (l == 0) {
            L.x[0] = static_cast<double*>(in.x);
            L.x[1] = c.take<double>(Nl);
            L.b = c.take<double>(Nl);
            const double* co = static_cast<const double*>(in.coeffs);
            for (int d = 0; d < 3; ++d) L.L[d] = d < ndim ? const_cast<double*>(co + d * Nl) : nullptr;
        } else {
            L.x[0] = c.take<double>(Nl);
            L.x[1] = c.take<double>(Nl);
            L.b = c.take<double>(Nl);
            for (int d = 0; d < 3; ++d) L.L[d] = d < ndim ? c.take<double>(Nl) : nullptr;
        }
        for (int d = 0; d < ndim; ++d) n[d] /= 2;
    }
    return WL_OK;
}

struct BatchLayout {
    BatchReq* dev_reqs = nullptr;
    BatchRes* dev_res = nullptr;
    unsigned* dev_head = nullptr;
};

// Checks every request and carves the batch's device arrays from c; with
// table non-null, also fills the count request descriptors there.
wl_status plan(const wl_batch_request* reqs, int count, Carver& c, BatchLayout& lay,
               BatchReq* table) {
    if (count < 0) return set_error("count must be >= 0"), WL_ERR_INVALID_ARG;
    if (count > 0 && !reqs) return set_error("reqs is NULL"), WL_ERR_INVALID_ARG;
    lay.dev_reqs = c.take<BatchReq>(size_t(count > 0 ? count : 1));
    lay.dev_res = c.take<BatchRes>(size_t(count > 0 ? count : 1));
    lay.dev_head = c.take<unsigned>(1);
    for (int r = 0; r < count; ++r) {
        BatchReq q;
        const wl_status st = plan_one(reqs[r], c, q);
        if (st != WL_OK) {
            set_error("request " + std::to_string(r) + ": " + last_error_text());
            return st;
        }
        if (table) table[r] = q;
    }
    return WL_OK;
}

// ------------------------------------------------ no-allocation variant
// Device scratch of wl_poisson_batch_solve_noalloc: the request table, the
// results, the queue head and every request's level arrays, carved exactly as
// from a caller workspace.  One copy per GPU, held until the process ends.
constexpr size_t kNoAllocScratchBytes = size_t(32) << 20;
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

// Device address of this GPU's copy of `scratch`, looked up once per device
// with that device current (the host-side name of the array is not a device
// address and must never be handed to a kernel or a copy).
constexpr int kMaxDevices = 64;
constexpr int kNoAllocMaxRequests = 256;
std::mutex g_noalloc_host_mu;
BatchReq g_noalloc_table[kNoAllocMaxRequests];
BatchRes g_noalloc_res[kNoAllocMaxRequests];
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

wl_status scratch_for_current_device(void** out) {
    int dev = 0;
    WL_CHECK_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device index beyond the no-allocation scratch table");
        return WL_ERR_INVALID_ARG;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        WL_CHECK_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr || reinterpret_cast<uintptr_t>(ptr) % 256) {
            set_error("scratch symbol address is null or misaligned");
            return WL_ERR_HIP;
        }
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return WL_OK;
}

int compute_units() {
    static const int n = [] {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) != hipSuccess) return 256;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return 256;
        return v > 0 ? v : 256;
    }();
    return n;
}

// Plans the batch into workspace (>= its footprint, 256-byte aligned),
// uploads the request table (host staging: table, count entries) and a zero
// queue head, runs the persistent kernel on hip_stream and copies the results
// back through res (count entries; synchronises).
wl_status batch_run(const wl_batch_request* reqs, int count, void* workspace, size_t ws_bytes,
                    void* hip_stream, wl_batch_result* results, BatchReq* table, BatchRes* res) {
    if (reinterpret_cast<uintptr_t>(workspace) % 256)
        return set_error("workspace must be 256-byte aligned"), WL_ERR_INVALID_ARG;
    for (int r = 0; r < count && reqs; ++r)
        if (!reqs[r].coeffs || !reqs[r].x || !reqs[r].b) {
            set_error("request " + std::to_string(r) + ": coeffs / x / b is NULL");
            return WL_ERR_INVALID_ARG;
        }
    Carver need;
    BatchLayout dry;
    WL_TRY(plan(reqs, count, need, dry, nullptr));
    if (ws_bytes < need.off) {
        set_error("workspace smaller than wl_poisson_batch_footprint");
        return WL_ERR_OUT_OF_MEMORY;
    }
    Carver c;
    c.base = static_cast<char*>(workspace);
    BatchLayout lay;
    WL_TRY(plan(reqs, count, c, lay, table));
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    // request table and a zero queue head (the no-allocation scratch keeps
    // the last call's contents, so the head is cleared on every call)
    const unsigned zero = 0u;
    WL_CHECK_HIP(hipMemcpyAsync(lay.dev_reqs, table, sizeof(BatchReq) * size_t(count),
                                hipMemcpyHostToDevice, s));
    WL_CHECK_HIP(hipMemcpyAsync(lay.dev_head, &zero, sizeof(zero), hipMemcpyHostToDevice, s));
    const int grid = std::min(count, compute_units());
    k_poisson_batch<<<grid, kBatchThreads, 0, s>>>(lay.dev_reqs, count, lay.dev_head, lay.dev_res);
    WL_CHECK_HIP(hipGetLastError());
    WL_CHECK_HIP(hipMemcpyAsync(res, lay.dev_res, sizeof(BatchRes) * size_t(count),
                                hipMemcpyDeviceToHost, s));
    WL_CHECK_HIP(hipStreamSynchronize(s));
    wl_status worst = WL_OK;
    for (int r = 0; r < count; ++r) {
        results[r].status = res[r].status;
        results[r].vcycles = res[r].vcycles;
        results[r].rel_resid = res[r].rel;
        if (res[r].status != WL_OK && worst == WL_OK) worst = wl_status(res[r].status);
    }
    if (worst == WL_ERR_NOT_CONVERGED) set_error("some batch requests reached max_vcycles");
    if (worst == WL_ERR_NONFINITE) set_error("non-finite residual in a batch request");
    return worst;
}

}  // namespace
}  // namespace wl

using namespace wl;

extern "C" {

wl_status wl_poisson_batch_footprint(const wl_batch_request* reqs, int count, size_t* bytes) {
    clear_error();
    if (!bytes) return set_error("bytes is NULL"), WL_ERR_INVALID_ARG;
    Carver c;
    BatchLayout lay;
    WL_TRY(plan(reqs, count, c, lay, nullptr));
    *bytes = c.off;
    return WL_OK;
}

wl_status wl_poisson_batch_solve(const wl_batch_request* reqs, int count, void* workspace,
                                 size_t ws_bytes, void* hip_stream, wl_batch_result* results) {
    clear_error();
    if (count == 0) return WL_OK;
    if (!workspace || !results) return set_error("workspace / results is NULL"), WL_ERR_INVALID_ARG;
    if (count < 0) return set_error("count must be >= 0"), WL_ERR_INVALID_ARG;
    std::vector<BatchReq> table(static_cast<size_t>(count));
    std::vector<BatchRes> res(static_cast<size_t>(count));
    return batch_run(reqs, count, workspace, ws_bytes, hip_stream, results, table.data(),
                     res.data());
}

wl_status wl_poisson_batch_solve_noalloc(const wl_batch_request* reqs, int count,
                                         void* hip_stream, wl_batch_result* results) {
    clear_error();
    if (count == 0) return WL_OK;
    if (!results) return set_error("results is NULL"), WL_ERR_INVALID_ARG;
    if (count < 0 || count > kNoAllocMaxRequests) {
        set_error("the no-allocation entry point takes 0 to " +
                  std::to_string(kNoAllocMaxRequests) + " requests per call");
        return WL_ERR_INVALID_ARG;
    }
    Carver need;
    BatchLayout dry;
    WL_TRY(plan(reqs, count, need, dry, nullptr));
    if (need.off > kNoAllocScratchBytes) {
        set_error("batch needs " + std::to_string(need.off) + " bytes of scratch; the "
                  "no-allocation entry point holds " + std::to_string(kNoAllocScratchBytes) +
                  " (use wl_poisson_batch_solve with a workspace)");
        return WL_ERR_INVALID_ARG;
    }
    void* ws = nullptr;
    WL_TRY(scratch_for_current_device(&ws));
    // fixed host staging (no heap); one call at a time in this process
    std::lock_guard<std::mutex> lock(g_noalloc_host_mu);
    return batch_run(reqs, count, ws, kNoAllocScratchBytes, hip_stream, results, g_noalloc_table,
                     g_noalloc_res);
}

}  // extern "C"
