// Internal declarations shared by the HIP translation units of libwl.
#pragma once

#include <functional>

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/wl.h"

namespace wl {

constexpr int kMaxLevels = 16;
constexpr int kBlock = 256;           // threads per block of the stencil kernels
constexpr int kCoarseMax = 1024;      // cells a one-workgroup coarsest solve accepts
constexpr int kDirectMax = 64;        // cells a coarsest level solved by its inverse may have

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);
const std::string& last_error_text();
void clear_error();

#define WL_CHECK_HIP(expr)                                                            \
    do {                                                                              \
        hipError_t e_ = (expr);                                                       \
        if (e_ != hipSuccess) {                                                       \
            ::wl::set_error(std::string("HIP error in " #expr ": ") +                 \
                            hipGetErrorString(e_));                                   \
            return WL_ERR_HIP;                                                        \
        }                                                                             \
    } while (0)

#define WL_CHECK_LAUNCH() WL_CHECK_HIP(hipGetLastError())

#define WL_TRY(expr)                                                                  \
    do {                                                                              \
        wl_status s_ = (expr);                                                        \
        if (s_ != WL_OK) return s_;                                                   \
    } while (0)

// ---------------------------------------------------------- kernel timing
// Optional HIP-event brackets around selected launches (wl_profile_*).
struct ProfScope {
    int id;
    hipStream_t s;
    bool on;
    ProfScope(int kernel, hipStream_t stream, size_t cells);
    ~ProfScope();
};

// ------------------------------------------------------------- workspace
// Bump allocator over the caller's device workspace.  With base == nullptr it
// only counts, which is how the footprint calls compute exact sizes.
struct Carver {
    char* base = nullptr;
    size_t off = 0;
    template <typename T>
    T* take(size_t count) {
        off = (off + 255) & ~size_t(255);
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

// ------------------------------------------------------------ grid shapes
// Kernel-side description of one grid level.
struct Grid {
    int n0, n1, n2;       // cells per direction
    int per0, per1, per2; // periodic flags
    int ndim;             // 2 or 3 (2: n2 == 1 and the z faces carry zero)
};

__host__ __device__ inline size_t cells(const Grid& g) { return size_t(g.n0) * g.n1 * g.n2; }

// Tile decomposition used by every stencil kernel: a 1D grid of 256-thread
// blocks; block b owns a bx x (256/bx) column of cells and marches through
// zc consecutive z planes.  With remap set, block ids are permuted so that
// each of the 8 XCDs (blocks are dealt to them round-robin) walks a
// contiguous range of tiles and neighbouring tiles share its L2.
struct TileDev {
    int lbx;        // log2 of the tile width bx (<= 64)
    int tx, ty;     // tiles along x and y
    int zc;         // z planes per block
    unsigned nb;    // blocks
    int remap;
};

struct Launch {
    dim3 grid, block;
    TileDev td;
    unsigned nblocks() const { return td.nb; }
};
Launch launch_for(int n0, int n1, int n2);

// Number of multigrid levels: halve every active direction while all of them
// are even and the coarse grid keeps >= 4 cells each; an explicit request only
// needs evenness.
int auto_levels(int ndim, const int n[3], int requested);

// ------------------------------------------------------ multigrid levels
template <typename T>
struct Level {
    Grid g;
    T* L[3] = {nullptr, nullptr, nullptr};  // lower-face coefficients
    T* x[2] = {nullptr, nullptr};           // Jacobi ping-pong (level 0: x[0] is the caller's x)
    T* b = nullptr;                         // right-hand side (level 0: projected copy)
    int uniform = 0;                        // all active faces equal Lc, fully periodic
    T Lc = T(1);
    // conjugate-gradient smoothing (carved only when the hierarchy uses it):
    // residual, search direction, M p, inverse diagonal (non-uniform levels)
    // and the level's CG scalars (double[8] on the device)
    // per-block classes (see Coeffs::cls) for the launch_for and the
    // launch_pairs tilings of this level (non-uniform levels)
    unsigned char* cls = nullptr;
    unsigned char* cls_pairs = nullptr;
    // per-workgroup classes of the fused-pair tiling (3D levels it fits), the
    // ordered list of its class-1 workgroups followed by their count, and on
    // the host the largest count met so far (the grid of the class-1 launch,
    // which captured graphs keep)
    unsigned char* cls_fp = nullptr;
    unsigned* fp_list = nullptr;
    unsigned fp_grid = 0;
    T* cr = nullptr;
    T* cp = nullptr;
    T* cq = nullptr;
    T* cd = nullptr;
    double* cgs = nullptr;
};

// Executable HIP graphs of a repeated solve body (one V-cycle with its norm,
// or one mixed-precision outer iteration), keyed by the solution and
// right-hand-side arrays the body was captured for: kernel arguments are
// baked into a graph.  Two
// entries, the least recently used one is replaced.  Owned by its hierarchy.
struct GraphCache {
    struct Entry {
        const void* key = nullptr;
        const void* key2 = nullptr;
        int uses = 0;
        unsigned long long stamp = 0;
        hipGraphExec_t exec = nullptr;
    };
    Entry e[2];
    hipStream_t cap = nullptr;  // private stream used only for capture
    unsigned long long clock = 0;
    GraphCache() = default;
    GraphCache(const GraphCache&) = delete;
    GraphCache& operator=(const GraphCache&) = delete;
    ~GraphCache();
    void clear();  // drops every captured body (call with the stream idle)
};

// Process-wide switch for graph replay (wl_set_graphs) and whether a kernel
// that runs inside captured bodies is being timed (timed launches are never
// captured).
bool graphs_enabled();
bool prof_active();

// Runs body(stream) on s.  From the second call with the same keys on, the
// body is captured once (on the cache's private stream) and replayed with
// hipGraphLaunch on s; the body must only enqueue kernels on the stream it
// is given.
template <typename F>
wl_status run_cached(GraphCache& G, const void* key, const void* key2, hipStream_t s, F&& body) {
    if (!graphs_enabled() || prof_active()) return body(s);
    GraphCache::Entry* hit = nullptr;
    for (auto& en : G.e)
        if (en.key == key && en.key2 == key2) hit = &en;
    if (!hit) {
        hit = &G.e[0];
        for (auto& en : G.e)
            if (en.stamp < hit->stamp) hit = &en;
        if (hit->exec) (void)hipGraphExecDestroy(hit->exec);
        *hit = GraphCache::Entry{};
        hit->key = key;
        hit->key2 = key2;
    }
    hit->stamp = ++G.clock;
    if (!hit->exec) {
        if (++hit->uses < 2) return body(s);
        if (!G.cap) WL_CHECK_HIP(hipStreamCreateWithFlags(&G.cap, hipStreamNonBlocking));
        WL_CHECK_HIP(hipStreamBeginCapture(G.cap, hipStreamCaptureModeThreadLocal));
        const wl_status rc = body(G.cap);
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(G.cap, &graph);
        if (rc != WL_OK || e != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            if (rc != WL_OK) return rc;
            WL_CHECK_HIP(e);
        }
        const hipError_t ei = hipGraphInstantiate(&hit->exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ei != hipSuccess) {
            hit->exec = nullptr;
            WL_CHECK_HIP(ei);
        }
    }
    WL_CHECK_HIP(hipGraphLaunch(hit->exec, s));
    return WL_OK;
}

template <typename T>
struct Hierarchy {
    int nlev = 0;
    Level<T> lev[kMaxLevels];
    double omega = 0.0;
    double coarse_tol = 1e-10;
    size_t n_active = 0;         // active fine cells (host copy)
    int pairs = 0;               // fused two-sweep kernels: 0 off, 1 on large levels, 2 on all
    int smoother = 0;            // 0 damped Jacobi, 1 conjugate gradients (WL_SMOOTH_*)
    // coarsest levels of at most kDirectMax cells: the inverse of the
    // operator with the mean constraint (N x N, FP64; see k_coarse_inverse)
    // and its validity flag, formed when the coefficients change unless
    // direct_coarse is off (then the CG solves)
    double* cinv = nullptr;
    int* cinv_ok = nullptr;
    bool direct_coarse = true;
    bool cinv_set = false;  // host: the flag has been set since the carve
    double* cgpart = nullptr;    // CG per-block partial sums (5 per block of level 0)
    GraphCache graphs;
};

// Conjugate-gradient smoothing of one level (cgsmooth.hip): `iters`
// Jacobi-preconditioned CG iterations on A x = b from x (zero: from x = 0,
// which is then written), with b shifted by -*bshift on active cells when
// bshift is given.  Enqueued on s; the level's scalars stay on the device.
template <typename T>
wl_status cg_smooth(const Hierarchy<T>& h, const Level<T>& L, T* x, bool zero, const T* b,
                    const double* bshift, int iters, hipStream_t s);

// A few doubles handed from the device to the host without a copy engine or
// a stream synchronisation: a kernel writes them into coherent pinned host
// memory followed by a sequence number, and the host waits for that number
// (see host_read).  The number is counted on the device (Reduce::result
// [kResultCounter]) and, post by post, on the host, so that a post inside a
// replayed graph still carries a new number.  Allocated on first use, one
// per solver.
struct HostMailbox {
    static constexpr int kSlots = 16;
    double* vals = nullptr;      // pinned host: kSlots values, then the sequence word
    unsigned* seqw = nullptr;
    double* vals_dev = nullptr;  // the same memory as seen by kernels
    unsigned* seqw_dev = nullptr;
    unsigned seq = 0;
    HostMailbox() = default;
    HostMailbox(const HostMailbox&) = delete;
    HostMailbox& operator=(const HostMailbox&) = delete;
    ~HostMailbox();
};

// Reduction scratch: per-block FP64 partial slots plus a few result scalars.
constexpr int kResultDoubles = 16;
constexpr int kResultCounter = 15;  // device count of mailbox posts
struct Reduce {
    double* partial = nullptr;   // capacity slots * 2 (a simulation's: slots * 4)
    size_t slots = 0;
    double* result = nullptr;    // kResultDoubles doubles
    size_t pslots = 0;           // slots a producer's partials cover (BPartials::Check)
    HostMailbox mb;
};

// Device addresses a kernel needs to post into the mailbox.
struct MailboxPost {
    double* vals = nullptr;      // null: no post
    unsigned* seqw = nullptr;
    double* counter = nullptr;
    int slot = 0, n = 0;
};

// Enqueue on s: copy src[0..n) (device) into mailbox slots [slot, slot + n)
// once everything before it on s has completed.  Does not wait.
wl_status host_post(Reduce& red, const double* src, int n, int slot, hipStream_t s);
// For a kernel that posts by itself: allocate the mailbox if needed (its
// device counter is cleared on s) and return the addresses for slots
// [slot, slot + n).  Every execution of such a kernel must be followed, on
// the host, by one host_posted before the matching host_wait.
wl_status mailbox_post_args(Reduce& red, int slot, int n, hipStream_t s, MailboxPost* out);
void host_posted(Reduce& red);
// Wait until the most recent post has arrived (so have all earlier ones, in
// stream order): polls the mailbox for a bounded time, then falls back to
// hipStreamSynchronize (which also reports a failed kernel).
wl_status host_wait(Reduce& red, hipStream_t s);
// The same for the post that made the host's count q (later posts may be
// outstanding still).
wl_status host_wait_seq(Reduce& red, unsigned q, hipStream_t s);
inline double host_slot(const Reduce& red, int slot) { return red.mb.vals[slot]; }
// host_post into slot 0, host_wait, and copy the values out.
wl_status host_read(Reduce& red, const double* src, int n, double* out, hipStream_t s);

template <typename T>
void carve_hierarchy(Carver& c, Hierarchy<T>& h, int ndim, const int n[3], const int per[3],
                     int nlev, bool alloc_fine_x);

// GMG building blocks (mg.hip).
template <typename T>
wl_status mg_coarsen_all(Hierarchy<T>& h, hipStream_t s);
template <typename T>
wl_status mg_count_active(Hierarchy<T>& h, Reduce& red, hipStream_t s);

struct SolveResult {
    int vcycles = 0;
    double rel = 0.0;     // ||r|| / ||b|| at exit
    double r2 = 0.0;      // ||r||^2 at exit
    double bnorm = 0.0;
};

// Work that follows a converged solve and only reads its solution (e.g. the
// projection).  mg_solve may enqueue it speculatively right after the first
// norm check is enqueued and enqueue it again if V-cycles follow; it must
// therefore be idempotent given the final solution.  On return the tail has
// been enqueued on the final solution; mailbox posts it makes may still be
// in flight (host_wait before reading them).
using SolveTail = std::function<wl_status(hipStream_t)>;

// What the producer of the right-hand side left in red.partial (per block of
// the fine level's launch_for tiling): nothing, the sums of b over the active
// cells, or (mg_producer_check) the four sums of the first residual check:
// [b, b^2, c, c^2] with c = b - A x for the solve's initial x.
enum class BPartials { None, Sums, Check };

// Whether the producer of b may take the first residual check
// (BPartials::Check): uniform periodic 3D fine level whose V-cycles start from
// the iterate (fused sweep pairs), so that the check needs no output.
template <typename T>
bool mg_producer_check(const Hierarchy<T>& h);

// Plain GMG solve on h (level 0 x = caller x).  b is the raw right-hand side.
// Converged before a V-cycle when ||r||^2 <= tol^2 ||b||^2 or ||r||^2 <= abs_r2.
template <typename T>
wl_status mg_solve(Hierarchy<T>& h, Reduce& red, T* x, const T* b, double tol, double abs_r2,
                   int max_vcycles, hipStream_t s, SolveResult* res,
                   BPartials bp = BPartials::None, const SolveTail* tail = nullptr);

// Mixed precision: FP64 outer residual with FP64 fine coefficients L64,
// FP32 inner V-cycles on h32.
struct Mixed64 {
    double* L[3] = {nullptr, nullptr, nullptr};
    // per-block classes of L for the fine level's launch_for tiling (see
    // Coeffs::cls); mg_mixed_classes fills them when L changes
    unsigned char* cls = nullptr;
    int inner = 3;
};
wl_status mg_mixed_classes(const Grid& g, const Mixed64& m, hipStream_t s);
wl_status mg_solve_mixed(Hierarchy<float>& h32, const Mixed64& m, Reduce& red, double* x,
                         const double* b, double tol, double abs_r2, int max_vcycles,
                         hipStream_t s, SolveResult* res);

size_t reduce_slots_for(const Grid& g);

template <typename Tin, typename Tout>
wl_status mg_load_coeffs(const Grid& g, const Tin* src, Tout* const L[3], double* const L64[3],
                         hipStream_t s);
wl_status mg_count_active64(const Grid& g, double* const L64[3], Reduce& red, size_t* count,
                            hipStream_t s);
template <typename T>
wl_status fill(T* p, size_t n, T v, hipStream_t s);
template <typename Tin, typename Tout>
wl_status convert(const Tin* a, Tout* b, size_t n, hipStream_t s);

}  // namespace wl
