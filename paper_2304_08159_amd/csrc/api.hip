// C ABI of libwl: argument checking, workspace carving and the orchestration
// of one Navier-Stokes step (paper Sec. 2-3: simstep! = convdiff!, BDIM!,
// BC!, project!, CFL!) and of the standalone GMG pressure solve.
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "wl_adj.h"
#include "wl_internal.h"
#include "wl_ns.h"

namespace wl {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }
void clear_error() { g_err.clear(); }
const std::string& last_error_text() { return g_err; }

static wl_status invalid(const std::string& msg) {
    set_error(msg);
    return WL_ERR_INVALID_ARG;
}

// ------------------------------------------------------------ simulation

struct SimConfig {
    wl_sim_desc d;
    Grid g;
    int nlev;
    bool allper, unif, outflow, body;
    bool moving;  // the body follows a rigid motion (re-measured every step)
    size_t N, P;  // cells, outflow-plane points
};

static bool body_moves(const wl_body& b) {
    if (b.kind == 0) return false;
    for (int i = 0; i < 3; ++i)
        if (b.velocity[i] != 0.0 || b.amplitude[i] != 0.0 || b.spin[i] != 0.0) return true;
    return false;
}

// The body placed where its motion has taken it at time t (the measure
// kernels see a body at rest there), and its rigid motion at t.
static BodyDev body_at(const wl_body& b, double t) {
    BodyDev d{b.kind, {b.centre[0], b.centre[1], b.centre[2]}, b.radius, b.eps, b.radius2};
    for (int i = 0; i < 3; ++i)
        d.centre[i] += b.velocity[i] * t + b.amplitude[i] * std::sin(b.omega * t);
    return d;
}

static BodyMotionDev motion_at(const wl_body& b, double t) {
    BodyMotionDev m{};
    if (!body_moves(b)) return m;
    m.on = 1;
    const BodyDev at = body_at(b, t);
    for (int i = 0; i < 3; ++i) {
        m.X[i] = at.centre[i];
        m.xdot[i] = b.velocity[i] + b.amplitude[i] * b.omega * std::cos(b.omega * t);
        m.w[i] = b.spin[i];
    }
    return m;
}

static wl_status check_desc(const wl_sim_desc* desc, SimConfig* cfg) {
    if (!desc) return invalid("desc is NULL");
    wl_sim_desc d = *desc;
    if (d.ndim != 2 && d.ndim != 3) return invalid("ndim must be 2 or 3");
    if (d.ndim == 2) {
        if (d.n[2] != 1) return invalid("2D problems need n[2] == 1");
        d.bc_lo[2] = d.bc_hi[2] = WL_BC_WALL;
    }
    for (int i = 0; i < d.ndim; ++i) {
        if (d.n[i] < 4) return invalid("every direction needs at least 4 cells");
        const int lo = d.bc_lo[i], hi = d.bc_hi[i];
        if (lo < 0 || lo > 3 || hi < 0 || hi > 3) return invalid("unknown boundary code");
        if ((lo == WL_BC_PERIODIC) != (hi == WL_BC_PERIODIC))
            return invalid("periodic boundaries must be set on both faces of a direction");
        if (lo == WL_BC_OUTFLOW) return invalid("OUTFLOW is only valid on the upper x face");
        if (hi == WL_BC_INFLOW) return invalid("INFLOW is only valid on the lower x face");
        if (i > 0 && (lo == WL_BC_INFLOW || hi == WL_BC_OUTFLOW))
            return invalid("INFLOW/OUTFLOW are only valid on the x faces");
    }
    if (d.prec < 0 || d.prec > 2) return invalid("prec must be WL_FP32, WL_FP64 or WL_MIXED");
    if (!(d.nu >= 0.0)) return invalid("nu must be >= 0");
    if (d.cfl <= 0.0) d.cfl = 0.5;
    if (d.max_vcycles <= 0) d.max_vcycles = 100;
    if (d.inner_vcycles <= 0) d.inner_vcycles = 3;
    if (!(d.tol >= 0.0)) return invalid("tol must be >= 0");
    if (d.stop_rule != WL_STOP_DIVERGENCE && d.stop_rule != WL_STOP_RELATIVE)
        return invalid("stop_rule must be WL_STOP_DIVERGENCE or WL_STOP_RELATIVE");
    if (d.body.kind < 0 || d.body.kind > 2) return invalid("body.kind must be 0, 1 or 2");
    if (d.body.kind != 0 && !(d.body.radius > 0.0)) return invalid("body radius must be > 0");
    if (d.body.kind == 2 && (d.ndim != 3 || !(d.body.radius2 > 0.0)))
        return invalid("a torus needs ndim = 3 and radius2 > 0");
    if (d.body.kind == 2 && d.tape_steps > 0)
        return invalid("the adjoint step supports sphere bodies only");
    if (!(d.body.eps > 0.0)) d.body.eps = 1.0;
    for (int i = 0; i < 3; ++i)
        if (!std::isfinite(d.body.velocity[i]) || !std::isfinite(d.body.amplitude[i]) ||
            !std::isfinite(d.body.spin[i]) || !std::isfinite(d.body.omega))
            return invalid("body motion parameters must be finite");
    if (body_moves(d.body)) {
        if (d.body.kind != 1 && (d.body.spin[0] != 0.0 || d.body.spin[1] != 0.0 ||
                                 d.body.spin[2] != 0.0))
            return invalid("a spinning body must be a sphere or circle (kind 1)");
        if (d.ndim == 2 && (d.body.velocity[2] != 0.0 || d.body.amplitude[2] != 0.0 ||
                            d.body.spin[0] != 0.0 || d.body.spin[1] != 0.0))
            return invalid("a 2D body moves in the x-y plane and spins about z only");
        if (d.tape_steps > 0) return invalid("the adjoint step supports bodies at rest only");
    }
    if (d.mg_levels < 0 || d.mg_levels > kMaxLevels) return invalid("mg_levels out of range");
    if (d.tape_steps < 0 || d.tape_steps > 100000) return invalid("tape_steps out of range");
    SimConfig c;
    c.d = d;
    c.g = Grid{d.n[0], d.n[1], d.n[2], d.bc_lo[0] == WL_BC_PERIODIC, d.bc_lo[1] == WL_BC_PERIODIC,
               d.ndim == 3 && d.bc_lo[2] == WL_BC_PERIODIC, d.ndim};
    c.nlev = auto_levels(d.ndim, d.n, d.mg_levels);
    if (d.mg_levels > 0 && c.nlev != d.mg_levels)
        return invalid("the requested number of multigrid levels needs more even halvings");
    {
        int m[3] = {d.n[0], d.n[1], d.n[2]};
        for (int l = 1; l < c.nlev; ++l)
            for (int i = 0; i < d.ndim; ++i) m[i] /= 2;
        if (size_t(m[0]) * m[1] * m[2] > size_t(kCoarseMax))
            return invalid("coarsest multigrid level exceeds 1024 cells (request more levels)");
    }
    c.allper = c.g.per0 && c.g.per1 && (d.ndim == 2 || c.g.per2);
    c.body = d.body.kind != 0;
    c.moving = body_moves(d.body);
    c.unif = c.allper && !c.body;
    c.outflow = d.bc_hi[0] == WL_BC_OUTFLOW;
    c.N = cells(c.g);
    c.P = size_t(d.n[1]) * d.n[2];
    *cfg = c;
    return WL_OK;
}

// One recorded step: everything the reverse pass needs.
template <typename T>
struct TapeSlot {
    T* un[3];
    T* outn;   // state at the step start (evaluation field of the predictor)
    T* u1[3];
    T* out1;   // predictor result (evaluation field of the corrector)
    T* f1[3];
    T* fo1;    // predictor stage field before BDIM
    T* f2[3];
    T* fo2;    // corrector stage field before BDIM
    T* p1;
    T* p2;     // stage pressures
    double dt;
};

// Adjoint workspace (carved with the simulation when tape_steps > 0).
template <typename T>
struct AdjointWS {
    int cap = 0, count = 0;
    bool recording = false;
    TapeSlot<T>* tape = nullptr;  // host array of cap slots
    PadGrid pg;
    T* pad[3];
    T* ub[3];
    T* uob;     // adjoint of the state after the step (working copy)
    T* u1b[3];
    T* u1ob;    // adjoint of the predictor result
    T* unb[3];
    T* unob;    // adjoint of the state before the step
    T* gb[3];   // adjoint of the post-BDIM stage field
    T* fb[3];
    T* fob;     // adjoint of the stage field and its outflow plane
    T* Rb[3];   // adjoint of the convection-diffusion tendency
    T* rhs;
    T* sbar;
    T* pbar;    // cells
    T* Lb[3];
    T* mu0b[3];
    T* mu1nb[9];
    double* rhs64 = nullptr;
    double* x64 = nullptr;
    double* part4;  // 4 * slots
    double* res;    // 16
    T* dummy;       // P (plane-sized scratch)
};

template <typename T>
struct SimImpl {
    SimConfig cfg;
    T* vel[3][3];         // three buffer sets of the velocity components
    T* plane[3] = {nullptr, nullptr, nullptr};  // outflow planes
    int S = 0;            // buffer set holding the state
    int PS = 0;           // plane holding the state's outflow plane
    T* p = nullptr;
    T* sigma = nullptr;
    T* mu0[3];
    T* mu1n[9];
    unsigned char* tile_cls = nullptr;  // BDIM tile classes (one per block of the cell tiling)
    unsigned char* cell_flag = nullptr;  // BDIM per-cell flags (bodies only)
    Hierarchy<T> h;
    Reduce red;
    double* scal = nullptr;  // [0] dt, [1] dt_next, [2] cfl max
    int dt_cur = 0;          // which scalar holds the current dt
    // mixed precision (T == float only)
    Hierarchy<float>* h32 = nullptr;
    Mixed64 mix;
    double* p64 = nullptr;
    double* sigma64 = nullptr;
    double t = 0.0;
    bool cfl_valid = false;
    double dt_host = 0.0;    // the next step's dt when the host already knows it
                             // (a restored state), else 0: read from the post
    AdjointWS<T>* adj = nullptr;  // host bookkeeping of the adjoint workspace
    ~SimImpl() {
        if (adj) {
            delete[] adj->tape;
            delete adj;
        }
    }
};

template <typename T>
static void carve_sim(Carver& c, SimImpl<T>& s, const SimConfig& cfg) {
    s.cfg = cfg;
    const size_t N = cfg.N;
    for (int b = 0; b < 3; ++b)
        for (int i = 0; i < 3; ++i) s.vel[b][i] = c.take<T>(N);
    if (cfg.outflow)
        for (int b = 0; b < 3; ++b) s.plane[b] = c.take<T>(cfg.P);
    s.p = c.take<T>(N);
    s.sigma = c.take<T>(N);
    for (int i = 0; i < 3; ++i) s.mu0[i] = c.take<T>(N);
    for (int i = 0; i < 9; ++i) s.mu1n[i] = c.take<T>(N);
    s.tile_cls = c.take<unsigned char>(reduce_slots_for(cfg.g));
    s.cell_flag = cfg.body ? c.take<unsigned char>(N) : nullptr;
    const int per[3] = {cfg.g.per0, cfg.g.per1, cfg.g.per2};
    carve_hierarchy<T>(c, s.h, cfg.d.ndim, cfg.d.n, per, cfg.nlev, cfg.d.prec == WL_MIXED);
    // a body that moves re-measures every step: the coarsest inverse would be
    // formed again each time, so its solve stays the CG
    s.h.direct_coarse = !cfg.moving;
    s.red.slots = reduce_slots_for(cfg.g);
    s.red.partial = c.take<double>(4 * std::max(s.red.slots, size_t(div_check_map(cfg.g).nblocks)));
    s.red.result = c.take<double>(kResultDoubles);
    s.scal = c.take<double>(4);
    if (cfg.d.prec == WL_MIXED) {
        for (int i = 0; i < 3; ++i) s.mix.L[i] = c.take<double>(N);
        s.mix.cls = c.take<unsigned char>(reduce_slots_for(cfg.g));
        s.mix.inner = cfg.d.inner_vcycles;
        s.p64 = c.take<double>(N);
        s.sigma64 = c.take<double>(N);
    }
    if (cfg.d.tape_steps > 0) {
        if (!s.adj) s.adj = new AdjointWS<T>;
        AdjointWS<T>& A = *s.adj;
        A.cap = cfg.d.tape_steps;
        delete[] A.tape;
        A.tape = new TapeSlot<T>[A.cap];
        const size_t P = cfg.outflow ? cfg.P : 1;
        for (int q = 0; q < A.cap; ++q) {
            TapeSlot<T>& t = A.tape[q];
            for (int i = 0; i < 3; ++i) {
                t.un[i] = c.take<T>(N);
                t.u1[i] = c.take<T>(N);
                t.f1[i] = c.take<T>(N);
                t.f2[i] = c.take<T>(N);
            }
            t.outn = c.take<T>(P);
            t.out1 = c.take<T>(P);
            t.fo1 = c.take<T>(P);
            t.fo2 = c.take<T>(P);
            t.p1 = c.take<T>(N);
            t.p2 = c.take<T>(N);
            t.dt = 0.0;
        }
        A.pg = pad_grid(cfg.g);
        const size_t NP = pad_cells(A.pg);
        for (int i = 0; i < 3; ++i) {
            A.pad[i] = c.take<T>(NP);
            A.ub[i] = c.take<T>(N);
            A.u1b[i] = c.take<T>(N);
            A.unb[i] = c.take<T>(N);
            A.gb[i] = c.take<T>(N);
            A.fb[i] = c.take<T>(N);
            A.Rb[i] = c.take<T>(N);
            A.Lb[i] = c.take<T>(N);
            A.mu0b[i] = c.take<T>(N);
        }
        for (int i = 0; i < 9; ++i) A.mu1nb[i] = c.take<T>(N);
        A.uob = c.take<T>(P);
        A.u1ob = c.take<T>(P);
        A.unob = c.take<T>(P);
        A.fob = c.take<T>(P);
        A.dummy = c.take<T>(P);
        A.rhs = c.take<T>(N);
        A.sbar = c.take<T>(N);
        A.pbar = c.take<T>(N);
        if (cfg.d.prec == WL_MIXED) {
            A.rhs64 = c.take<double>(N);
            A.x64 = c.take<double>(N);
        }
        A.part4 = c.take<double>(4 * s.red.slots);
        A.res = c.take<double>(16);
    }
}

template <typename T>
static VelField<T> field_of(const SimImpl<T>& s, int set, const T* plane) {
    VelField<T> V;
    for (int i = 0; i < 3; ++i) V.u[i] = s.vel[set][i];
    V.uout = plane;
    V.g = s.cfg.g;
    for (int i = 0; i < 3; ++i) {
        V.bclo[i] = s.cfg.d.bc_lo[i];
        V.bchi[i] = s.cfg.d.bc_hi[i];
        V.U[i] = T(s.cfg.d.U[i]);
    }
    return V;
}

}  // namespace wl

struct wl_sim {
    int prec;
    hipStream_t stream;
    void* impl;  // wl::SimImpl<float> or wl::SimImpl<double>
};

struct wl_poisson {
    int prec;
    hipStream_t stream;
    void* impl;
};

namespace wl {

template <typename T>
static BdimFields<T> bdim_fields(const SimImpl<T>& s) {
    BdimFields<T> b;
    for (int i = 0; i < 3; ++i) b.mu0[i] = s.mu0[i];
    for (int i = 0; i < 9; ++i) b.mu1n[i] = s.mu1n[i];
    b.cls = s.tile_cls;
    b.cflag = s.cell_flag;
    return b;
}

// Geometry of the body where it is at time t: BDIM moments, fine Poisson
// coefficients (and their FP64 copy), tile classes, coarse coefficients and
// the active-cell count (synchronises).
template <typename T>
static wl_status sim_measure(SimImpl<T>& s, double t, hipStream_t st) {
    const SimConfig& c = s.cfg;
    const BodyDev body = body_at(c.d.body, t);
    MeasureOut<T> M;
    for (int i = 0; i < 3; ++i) {
        M.mu0[i] = s.mu0[i];
        M.L[i] = s.h.lev[0].L[i];
        M.L64[i] = s.mix.L[i];
    }
    for (int i = 0; i < 9; ++i) M.mu1n[i] = s.mu1n[i];
    WL_TRY(ns_measure<T>(c.g, body, c.d.bc_lo, M, st));
    if (c.body) WL_TRY(ns_tile_class<T>(c.g, bdim_fields(s), s.tile_cls, st, s.cell_flag));
    s.h.lev[0].uniform = c.unif ? 1 : 0;
    s.h.lev[0].Lc = T(1);
    WL_TRY(mg_coarsen_all<T>(s.h, st));
    if (c.d.prec == WL_MIXED) WL_TRY(mg_mixed_classes(c.g, s.mix, st));
    return mg_count_active<T>(s.h, s.red, st);
}

template <typename T>
static wl_status sim_init(SimImpl<T>& s, hipStream_t st) {
    const SimConfig& c = s.cfg;
    const size_t N = c.N;
    WL_TRY(sim_measure(s, 0.0, st));
    if (c.d.prec == WL_MIXED) {
        s.h.coarse_tol = 1e-6;
    } else {
        s.h.coarse_tol = sizeof(T) == 8 ? 1e-10 : 1e-6;
    }
    // initial state: u = U on every face, boundary faces at their values, p = 0
    {
        T* u0[3] = {s.vel[0][0], s.vel[0][1], s.vel[0][2]};
        WL_TRY(ns_init_velocity<T>(c.g, c.d.bc_lo, c.d.U, u0, st));
    }
    if (c.outflow)
        for (int b = 0; b < 3; ++b) WL_TRY(fill<T>(s.plane[b], c.P, T(c.d.U[0]), st));
    WL_TRY(fill<T>(s.p, N, T(0), st));
    if (s.p64) WL_TRY(fill<double>(s.p64, N, 0.0, st));
    s.S = 0;
    s.PS = 0;
    s.t = 0.0;
    s.cfl_valid = false;
    WL_CHECK_HIP(hipStreamSynchronize(st));
    return WL_OK;
}

// Pressure solve of one stage.  WL_STOP_DIVERGENCE: it stops once the
// divergence it leaves in the projected velocity, c dt (sigma - A p), has RMS
// over the active cells <= tol, i.e. ||r||^2 <= (tol sqrt(n_active) / (c dt))^2;
// WL_STOP_RELATIVE: once ||r|| <= tol ||sigma||.  `tail` (may be null) is
// work that reads the final pressure, done before returning (see SolveTail).
// The divergence kernel also takes the pressure solve's first residual
// check (plain periodic FP32/FP64 solves on hierarchies that allow it).
template <typename T>
static bool producer_check(const SimImpl<T>& s) {
    return s.cfg.d.prec != WL_MIXED && s.cfg.unif && s.cfg.d.ndim == 3 && mg_producer_check(s.h);
}

template <typename T>
static wl_status pressure_solve(SimImpl<T>& s, double cfac, double dt, hipStream_t st,
                                SolveResult* r, const SolveTail* tail = nullptr) {
    const SimConfig& c = s.cfg;
    const bool rel = c.d.stop_rule == WL_STOP_RELATIVE;
    const double a = c.d.tol * std::sqrt(double(s.h.n_active)) / (cfac * dt);
    const double abs_r2 = rel ? 0.0 : a * a;
    const double rtol = rel ? c.d.tol : 0.0;
    if (c.d.prec == WL_MIXED) {
        if constexpr (sizeof(T) == 4) {
            WL_TRY((convert<float, double>(s.sigma, s.sigma64, c.N, st)));
            wl_status rc = mg_solve_mixed(s.h, s.mix, s.red, s.p64, s.sigma64, rtol, abs_r2,
                                          c.d.max_vcycles, st, r);
            if (rc != WL_OK && rc != WL_ERR_NOT_CONVERGED) return rc;
            WL_TRY((convert<double, float>(s.p64, s.p, c.N, st)));
            if (tail) WL_TRY((*tail)(st));
            return rc;
        }
        return invalid("mixed precision needs FP32 fields");
    }
    return mg_solve<T>(s.h, s.red, s.p, s.sigma, rtol, abs_r2, c.d.max_vcycles, st, r,
                       producer_check(s) ? BPartials::Check : BPartials::Sums, tail);
}

template <typename T>
static wl_status sim_step(SimImpl<T>& s, double dt_in, wl_step_stats* stats, hipStream_t st) {
    const SimConfig& c = s.cfg;
    const bool ap = c.allper;
    double* dt_dev = s.scal + s.dt_cur;
    double dt = 0.0;
    bool dt_pending = false;
    if (dt_in > 0.0) {
        WL_TRY(ns_set_scalar(dt_dev, dt_in, st));
        dt = dt_in;
    } else if (s.cfl_valid && s.dt_host > 0.0) {
        // restored state: dt_dev already holds the saved dt
        dt = s.dt_host;
    } else if (s.cfl_valid) {
        // the last projection formed dt on the device (dt_dev) and posted it
        // to mailbox slot 8; the host needs it only for the first
        // convergence test, so the step's first kernels are enqueued before
        // it is read
        dt_pending = true;
    } else {
        WL_TRY(ns_cfl<T>(field_of(s, s.S, s.plane[s.PS]), ap, s.red.partial, st));
        WL_TRY(ns_dt_from_max(s.red.partial, s.red.slots, c.d.cfl, 2.0 * c.d.ndim * c.d.nu, dt_dev,
                              s.scal + 2, st));
        WL_TRY(host_read(s.red, dt_dev, 1, &dt, st));
    }
    auto resolve_dt = [&]() -> wl_status {
        if (dt_pending) {
            // the latest post: no solve has posted since that projection
            WL_TRY(host_wait(s.red, st));
            dt = host_slot(s.red, 8);
            dt_pending = false;
        }
        if (!(dt > 0.0) || !std::isfinite(dt)) {
            set_error("time step is not positive (zero velocity and zero viscosity?)");
            return WL_ERR_INVALID_ARG;
        }
        return WL_OK;
    };
    const int S = s.S;
    const int A = (S + 1) % 3, B = (S + 2) % 3;
    const int PS = s.PS, P1 = (PS + 1) % 3, P2 = (PS + 2) % 3;
    BodyMotionDev motion{};
    if (c.moving) {
        // both stages advance to t + dt: the body is measured there
        WL_TRY(resolve_dt());
        WL_TRY(sim_measure(s, s.t + dt, st));
        motion = motion_at(c.d.body, s.t + dt);
    }
    TapeSlot<T>* tp = nullptr;
    if (s.adj && s.adj->recording && s.adj->count < s.adj->cap) {
        WL_TRY(resolve_dt());
        tp = &s.adj->tape[s.adj->count];
        tp->dt = dt;
    }
    auto rec = [&](T* dst, const T* src, size_t n) -> wl_status {
        if (!dst || !src || n == 0) return WL_OK;
        WL_CHECK_HIP(hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyDeviceToDevice, st));
        return WL_OK;
    };
    auto rec3 = [&](T* const* dst, T* const* src) -> wl_status {
        for (int i = 0; i < 3; ++i) WL_TRY(rec(dst[i], src[i], c.N));
        return WL_OK;
    };
    if (tp) {
        WL_TRY(rec3(tp->un, s.vel[S]));
        if (c.outflow) WL_TRY(rec(tp->outn, s.plane[PS], c.P));
    }
    const T* un[3] = {s.vel[S][0], s.vel[S][1], s.vel[S][2]};
    wl_status worst = WL_OK;
    SolveResult r1, r2;
    const ProjCoeffs<T> pc{{s.h.lev[0].L[0], s.h.lev[0].L[1], s.h.lev[0].L[2]}, T(1),
                           s.h.lev[0].uniform ? nullptr : s.h.lev[0].cls};
    // ---- predictor (c = 1)
    {
        T* f[3] = {s.vel[A][0], s.vel[A][1], s.vel[A][2]};
        WL_TRY(ns_momentum<T>(field_of(s, S, s.plane[PS]), un, f, T(c.d.nu), false, ap, dt_dev, st));
        if (c.outflow)
            WL_TRY(ns_outflow<T>(c.g, s.vel[S][0], s.plane[PS], s.plane[PS], s.vel[A][0],
                                 T(c.d.U[0]), false, dt_dev, s.plane[P1], s.red.partial, st));
        if (tp) {
            WL_TRY(rec3(tp->f1, s.vel[A]));
            if (c.outflow) WL_TRY(rec(tp->fo1, s.plane[P1], c.P));
        }
        // BDIM in place: u* stays in A (set B is its scratch on the body's tiles)
        const int us = A;
        if (c.body) {
            T* w[3] = {s.vel[B][0], s.vel[B][1], s.vel[B][2]};
            WL_TRY(ns_bdim_in_place<T>(field_of(s, A, s.plane[P1]), f, bdim_fields(s), w, st,
                                       motion));
        }
        const VelField<T> V = field_of(s, us, s.plane[P1]);
        WL_TRY(ns_divergence<T>(V, pc, c.unif, 1.0, dt_dev, s.sigma, s.red.partial, ap, st,
                                producer_check(s) ? s.p : nullptr, s.h.lev[0].Lc,
                                &s.red.pslots));
        WL_TRY(resolve_dt());
        wl_status rc = pressure_solve(s, 1.0, dt, st, &r1);
        if (rc == WL_ERR_NOT_CONVERGED) worst = rc;
        else if (rc != WL_OK) return rc;
        if (tp) WL_TRY(rec(tp->p1, s.p, c.N));
        T* o[3] = {s.vel[us][0], s.vel[us][1], s.vel[us][2]};
        // Periodic FP32 3D grids with uniform coefficients skip storing the
        // predictor's projection: the corrector's convection-diffusion
        // kernel applies it as it loads u* (bitwise the same result).  The
        // adjoint tape needs u1 itself, so recording steps store it.
        const bool fuse = sizeof(T) == 4 && c.d.ndim == 3 && c.unif && !tp;
        if (!fuse) WL_TRY(ns_project<T>(V, s.p, pc, c.unif, 1.0, dt_dev, o, false, nullptr, ap, st));
        // stage result now in set `us` (u1, or u* when fused); the remaining set is free
        const int u1 = us;
        const int fr = (u1 == A) ? B : A;
        if (tp) {
            WL_TRY(rec3(tp->u1, s.vel[u1]));
            if (c.outflow) WL_TRY(rec(tp->out1, s.plane[P1], c.P));
        }
        // ---- corrector (c = 1/2)
        T* f2[3] = {s.vel[fr][0], s.vel[fr][1], s.vel[fr][2]};
        if constexpr (sizeof(T) == 4) {
            if (fuse)
                WL_TRY(ns_momentum_proj(field_of(s, u1, s.plane[P1]), un, f2, float(c.d.nu), dt_dev,
                                        s.p, float(pc.Lc), st));
            else
                WL_TRY(ns_momentum<T>(field_of(s, u1, s.plane[P1]), un, f2, T(c.d.nu), true, ap,
                                      dt_dev, st));
        } else {
            WL_TRY(ns_momentum<T>(field_of(s, u1, s.plane[P1]), un, f2, T(c.d.nu), true, ap, dt_dev,
                                  st));
        }
        if (c.outflow)
            WL_TRY(ns_outflow<T>(c.g, s.vel[u1][0], s.plane[P1], s.plane[PS], s.vel[fr][0],
                                 T(c.d.U[0]), true, dt_dev, s.plane[P2], s.red.partial, st));
        if (tp) {
            WL_TRY(rec3(tp->f2, s.vel[fr]));
            if (c.outflow) WL_TRY(rec(tp->fo2, s.plane[P2], c.P));
        }
        // u* stays in fr; u^n (set S) is no longer read and serves as scratch
        const int us2 = fr;
        if (c.body) {
            T* w2[3] = {s.vel[S][0], s.vel[S][1], s.vel[S][2]};
            WL_TRY(ns_bdim_in_place<T>(field_of(s, fr, s.plane[P2]), f2, bdim_fields(s), w2, st,
                                       motion));
        }
        const VelField<T> V2 = field_of(s, us2, s.plane[P2]);
        WL_TRY(ns_divergence<T>(V2, pc, c.unif, 0.5, dt_dev, s.sigma, s.red.partial, ap, st,
                                producer_check(s) ? s.p : nullptr, s.h.lev[0].Lc,
                                &s.red.pslots));
        // projection, CFL maximum and next dt read only the final pressure
        // and write buffers nothing else reads: the solve may run them
        // speculatively before its first convergence check returns
        const int dest = (us2 == S) ? u1 : S;
        T* o3[3] = {s.vel[dest][0], s.vel[dest][1], s.vel[dest][2]};
        double* dt_next = s.scal + (1 - s.dt_cur);
        MailboxPost dt_post;
        WL_TRY(mailbox_post_args(s.red, 8, 1, st, &dt_post));
        const SolveTail tail = [&](hipStream_t q) -> wl_status {
            WL_TRY(ns_project<T>(V2, s.p, pc, c.unif, 0.5, dt_dev, o3, true, s.red.partial, ap, q));
            WL_TRY(ns_dt_from_max(s.red.partial, s.red.slots, c.d.cfl, 2.0 * c.d.ndim * c.d.nu,
                                  dt_next, s.scal + 2, q, &dt_post));
            host_posted(s.red);
            return WL_OK;
        };
        rc = pressure_solve(s, 0.5, dt, st, &r2, &tail);
        if (rc == WL_ERR_NOT_CONVERGED) worst = rc;
        else if (rc != WL_OK) return rc;
        if (tp) WL_TRY(rec(tp->p2, s.p, c.N));
        s.S = dest;
        s.PS = P2;
    }
    s.dt_cur = 1 - s.dt_cur;
    s.cfl_valid = true;
    s.dt_host = 0.0;
    s.t += dt;
    if (tp) s.adj->count += 1;
    if (stats) {
        stats->dt = dt;
        stats->t = s.t;
        stats->vcycles[0] = r1.vcycles;
        stats->vcycles[1] = r2.vcycles;
        const double na = double(s.h.n_active > 0 ? s.h.n_active : 1);
        stats->resid[0] = 1.0 * dt * std::sqrt(r1.r2 / na);
        stats->resid[1] = 0.5 * dt * std::sqrt(r2.r2 / na);
        stats->rel_resid[0] = r1.rel;
        stats->rel_resid[1] = r2.rel;
    }
    return worst;
}

// Adjoint Poisson solve  A sbar = rhs  (treated as exact: same hierarchy,
// tight relative tolerance).
template <typename T>
static wl_status adj_solve(SimImpl<T>& s, hipStream_t st) {
    AdjointWS<T>& A = *s.adj;
    const SimConfig& c = s.cfg;
    SolveResult r;
    wl_status rc;
    if (c.d.prec == WL_MIXED) {
        if constexpr (sizeof(T) == 4) {
            WL_TRY((convert<float, double>(A.rhs, A.rhs64, c.N, st)));
            WL_TRY(fill<double>(A.x64, c.N, 0.0, st));
            rc = mg_solve_mixed(s.h, s.mix, s.red, A.x64, A.rhs64, 1e-10, 0.0, 400, st, &r);
            if (rc != WL_OK && rc != WL_ERR_NOT_CONVERGED) return rc;
            WL_TRY((convert<double, float>(A.x64, A.sbar, c.N, st)));
            return WL_OK;
        }
        return invalid("mixed precision needs FP32 fields");
    }
    WL_TRY(fill<T>(A.sbar, c.N, T(0), st));
    rc = mg_solve<T>(s.h, s.red, A.sbar, A.rhs, sizeof(T) == 8 ? 1e-11 : 1e-6, 0.0,
                     sizeof(T) == 8 ? 400 : 60, st, &r, BPartials::None);
    if (rc != WL_OK && rc != WL_ERR_NOT_CONVERGED) return rc;
    return WL_OK;
}

// Adjoint of one projected stage: u = g - coef L G p, p = A^+ div(g)/coef
// (coef = c dt), outflow plane = the exit-flux-balanced stage plane.  In: the
// adjoint of the stage result (faces ubar, plane uoutb) and of its pressure
// (pbar, may be null).  Out: A.fb / A.fob = adjoint of the stage field before
// BDIM; geometry adjoints accumulate into A.Lb, A.mu0b, A.mu1nb.
template <typename T>
static wl_status adj_stage_projection(SimImpl<T>& s, T* const ubar[3], const T* uoutb, const T* pbar,
                                      const T* p, T* const f[3], const T* fo, double coef,
                                      hipStream_t st) {
    AdjointWS<T>& A = *s.adj;
    const SimConfig& c = s.cfg;
    const Grid& g = c.g;
    T* L[3] = {s.h.lev[0].L[0], s.h.lev[0].L[1], s.h.lev[0].L[2]};
    WL_TRY(adj_proj_rhs<T>(g, pbar, ubar, L, T(1), c.unif, coef, A.rhs, st));
    WL_TRY(adj_solve(s, st));
    WL_TRY(adj_proj_update<T>(g, ubar, A.sbar, p, L, T(1), c.unif, coef, A.gb, A.Lb, st));
    // The stage plane is balanced (exit flux) before BDIM and the divergence
    // read it, so both of their plane adjoints go through the balance's
    // transpose: collect BDIM's share first, then add the divergence's and
    // remove the mean.
    if (c.outflow) WL_TRY(fill<T>(A.fob, c.P, T(0), st));
    if (c.body) {
        const PadField<T> pf{{A.pad[0], A.pad[1], A.pad[2]}, A.pg};
        T* m0[3] = {s.mu0[0], s.mu0[1], s.mu0[2]};
        WL_TRY(adj_bdim<T>(g, A.gb, m0, s.mu1n, pf, st));
        WL_TRY(adj_faces_axpy<T>(g, A.gb, 0.0, A.fb, false, st));   // fb = 0
        WL_TRY(adj_fold<T>(field_of(s, 0, static_cast<const T*>(nullptr)), pf, A.fb,
                           c.outflow ? A.fob : nullptr, st));
        VelField<T> F = field_of(s, 0, fo);
        for (int i = 0; i < 3; ++i) F.u[i] = f[i];
        WL_TRY(adj_bdim_param<T>(F, A.gb, A.mu0b, A.mu1nb, st));
    } else {
        WL_TRY(adj_faces_axpy<T>(g, A.gb, 1.0, A.fb, false, st));
    }
    if (c.outflow) WL_TRY(adj_plane_proj<T>(g, uoutb, A.sbar, coef, A.fob, st));
    return WL_OK;
}

// Adjoint of R'(e)^T applied to Rbar, added into ebar (faces) and eoutb.
template <typename T>
static wl_status adj_tendency(SimImpl<T>& s, T* const e[3], const T* eout, T* const ebar[3],
                              T* eoutb, hipStream_t st) {
    AdjointWS<T>& A = *s.adj;
    const SimConfig& c = s.cfg;
    VelField<T> E = field_of(s, 0, eout);
    for (int i = 0; i < 3; ++i) E.u[i] = e[i];
    const PadField<T> pf{{A.pad[0], A.pad[1], A.pad[2]}, A.pg};
    WL_TRY(adj_flux<T>(E, A.Rb, T(c.d.nu), pf, c.allper, st));
    WL_TRY(adj_fold<T>(E, pf, ebar, c.outflow ? eoutb : nullptr, st));
    return WL_OK;
}

template <typename T>
static wl_status read_doubles(const double* dev, double* host, int n, hipStream_t st) {
    WL_CHECK_HIP(hipMemcpyAsync(host, dev, n * sizeof(double), hipMemcpyDeviceToHost, st));
    WL_CHECK_HIP(hipStreamSynchronize(st));
    return WL_OK;
}

// F_x = -sum_active (p - mean p) n_x K(d) of the current pressure.
template <typename T>
static wl_status sim_drag(SimImpl<T>& s, double* F, hipStream_t st) {
    const SimConfig& c = s.cfg;
    if (!c.body) {
        *F = 0.0;
        return WL_OK;
    }
    if (c.d.body.kind != 1) return invalid("drag supports sphere bodies only");
    const BodyDev body = body_at(c.d.body, s.t);
    T* L[3] = {s.h.lev[0].L[0], s.h.lev[0].L[1], s.h.lev[0].L[2]};
    WL_TRY(drag_sums<T>(c.g, body, s.p, L, s.red.partial, st));
    WL_TRY(reduce_cols(s.red.partial, s.red.slots, 4, s.red.result + 8, st));
    double sums[4];
    WL_TRY(read_doubles<T>(s.red.result + 8, sums, 4, st));
    const double cnt = sums[3] > 0.0 ? sums[3] : 1.0;
    *F = -(sums[2] - sums[1] * sums[0] / cnt);
    return WL_OK;
}

template <typename T>
static wl_status sim_step_adjoint(SimImpl<T>& s, const void* ubar_in, const void* pbar_in,
                                  double drag_weight, void* ubar_out, double* gp, hipStream_t st) {
    if (!s.adj || s.adj->count <= 0) {
        set_error("the adjoint tape is empty (record steps with wl_tape_record first)");
        return WL_ERR_STATE;
    }
    AdjointWS<T>& A = *s.adj;
    const SimConfig& c = s.cfg;
    const Grid& g = c.g;
    const size_t N = c.N;
    TapeSlot<T>& tp = A.tape[--A.count];
    const double dt = tp.dt;
    const BodyDev body{c.d.body.kind,
                       {c.d.body.centre[0], c.d.body.centre[1], c.d.body.centre[2]},
                       c.d.body.radius,
                       c.d.body.eps,
                       c.d.body.radius2};
    T* L[3] = {s.h.lev[0].L[0], s.h.lev[0].L[1], s.h.lev[0].L[2]};
    const T* in = static_cast<const T*>(ubar_in);
    for (int i = 0; i < c.d.ndim; ++i)
        WL_CHECK_HIP(hipMemcpyAsync(A.ub[i], in + i * N, N * sizeof(T), hipMemcpyDeviceToDevice, st));
    if (c.outflow)
        WL_CHECK_HIP(hipMemcpyAsync(A.uob, in + c.d.ndim * N, c.P * sizeof(T),
                                    hipMemcpyDeviceToDevice, st));
    WL_TRY(adj_faces_axpy<T>(g, A.ub, 1.0, A.ub, false, st));  // constants on boundary faces
    double gsum[4] = {0.0, 0.0, 0.0, 0.0};
    // ---- drag of the step (corrector pressure p2): pbar and its direct theta term
    const T* pbar = nullptr;
    if (c.body && drag_weight != 0.0) {
        WL_TRY(drag_sums<T>(g, body, tp.p2, L, A.part4, st));
        WL_TRY(reduce_cols(A.part4, s.red.slots, 4, A.res, st));
        double sums[4];
        WL_TRY(read_doubles<T>(A.res, sums, 4, st));
        const double cnt = sums[3] > 0.0 ? sums[3] : 1.0;
        WL_TRY(ns_set_scalar(A.res + 8, sums[0] / cnt, st));
        WL_TRY(ns_set_scalar(A.res + 9, sums[1] / cnt, st));
        WL_TRY(drag_adj<T>(g, body, tp.p2, L, drag_weight, A.res + 8, A.pbar, A.part4, st));
        WL_TRY(reduce_cols(A.part4, s.red.slots, 4, A.res, st));
        double dg[4];
        WL_TRY(read_doubles<T>(A.res, dg, 4, st));
        for (int q = 0; q < 4; ++q) gsum[q] += dg[q];
        pbar = A.pbar;
    }
    // ---- the caller's adjoint of the step's pressure adds to the drag's
    if (pbar_in) {
        if (pbar)
            WL_TRY(adj_cells_add<T>(N, static_cast<const T*>(pbar_in), A.pbar, st));
        else
            WL_CHECK_HIP(hipMemcpyAsync(A.pbar, pbar_in, N * sizeof(T), hipMemcpyDeviceToDevice, st));
        pbar = A.pbar;
    }
    // ---- corrector projection (c = 1/2) and BDIM: fb, fob
    WL_TRY(adj_stage_projection<T>(s, A.ub, A.uob, pbar, tp.p2, tp.f2, tp.fo2, 0.5 * dt, st));
    // ---- corrector stage f2 = (u^n + u1)/2 + dt/2 R(u1)
    WL_TRY(adj_faces_axpy<T>(g, A.fb, 0.5, A.unb, false, st));
    WL_TRY(adj_faces_axpy<T>(g, A.fb, 0.5, A.u1b, false, st));
    WL_TRY(adj_faces_axpy<T>(g, A.fb, 0.5 * dt, A.Rb, false, st));
    if (c.outflow) {
        WL_TRY(fill<T>(A.unob, c.P, T(0), st));
        WL_TRY(fill<T>(A.u1ob, c.P, T(0), st));
        WL_TRY(adj_plane_stage<T>(g, A.fob, 0.5, 0.5 * dt, T(c.d.U[0]), A.unob, A.u1ob, A.u1b[0], st));
        WL_TRY(adj_plane_stage<T>(g, A.fob, 0.5, 0.0, T(c.d.U[0]), A.u1ob, A.dummy, A.u1b[0], st));
    }
    WL_TRY(adj_tendency<T>(s, tp.u1, tp.out1, A.u1b, A.u1ob, st));
    // ---- predictor projection (c = 1) and BDIM
    WL_TRY(adj_stage_projection<T>(s, A.u1b, A.u1ob, nullptr, tp.p1, tp.f1, tp.fo1, dt, st));
    // ---- predictor stage f1 = u^n + dt R(u^n)
    WL_TRY(adj_faces_axpy<T>(g, A.fb, 1.0, A.unb, true, st));
    WL_TRY(adj_faces_axpy<T>(g, A.fb, dt, A.Rb, false, st));
    if (c.outflow)
        WL_TRY(adj_plane_stage<T>(g, A.fob, 1.0, dt, T(c.d.U[0]), A.unob, A.unob, A.unb[0], st));
    WL_TRY(adj_tendency<T>(s, tp.un, tp.outn, A.unb, A.unob, st));
    // ---- geometry adjoints -> parameters
    if (c.body) {
        WL_TRY(adj_params<T>(g, body, A.Lb, A.mu0b, A.mu1nb, A.part4, st));
        WL_TRY(reduce_cols(A.part4, s.red.slots, 4, A.res, st));
        double dg[4];
        WL_TRY(read_doubles<T>(A.res, dg, 4, st));
        for (int q = 0; q < 4; ++q) gsum[q] += dg[q];
    }
    // ---- output
    T* out = static_cast<T*>(ubar_out);
    for (int i = 0; i < c.d.ndim; ++i)
        WL_CHECK_HIP(hipMemcpyAsync(out + i * N, A.unb[i], N * sizeof(T), hipMemcpyDeviceToDevice, st));
    if (c.outflow)
        WL_CHECK_HIP(hipMemcpyAsync(out + c.d.ndim * N, A.unob, c.P * sizeof(T),
                                    hipMemcpyDeviceToDevice, st));
    WL_CHECK_HIP(hipStreamSynchronize(st));
    if (gp)
        for (int q = 0; q < 4; ++q) gp[q] += gsum[q];
    return WL_OK;
}

template <typename T>
static wl_status sim_field_ptr(SimImpl<T>& s, int field, T** ptr, size_t* count, bool writable) {
    const SimConfig& c = s.cfg;
    *count = c.N;
    if (field >= WL_FIELD_U0 && field <= WL_FIELD_U2) {
        if (field - WL_FIELD_U0 >= c.d.ndim) return invalid("velocity component beyond ndim");
        *ptr = s.vel[s.S][field - WL_FIELD_U0];
        return WL_OK;
    }
    if (field == WL_FIELD_P) {
        *ptr = s.p;
        return WL_OK;
    }
    if (field == WL_FIELD_UOUT) {
        if (!c.outflow) return invalid("no outflow plane in this simulation");
        *ptr = s.plane[s.PS];
        *count = c.P;
        return WL_OK;
    }
    if (writable) return invalid("field is read-only");
    if (field >= WL_FIELD_L0 && field <= WL_FIELD_L2) {
        *ptr = s.h.lev[0].L[field - WL_FIELD_L0];
        return WL_OK;
    }
    if (field >= WL_FIELD_MU0_0 && field <= WL_FIELD_MU0_2) {
        *ptr = s.mu0[field - WL_FIELD_MU0_0];
        return WL_OK;
    }
    if (field >= WL_FIELD_MU1N && field < WL_FIELD_MU1N + 9) {
        *ptr = s.mu1n[field - WL_FIELD_MU1N];
        return WL_OK;
    }
    if (field == WL_FIELD_SIGMA) {
        *ptr = s.sigma;
        return WL_OK;
    }
    return invalid("unknown field id");
}

static size_t sim_bytes(const SimConfig& cfg) {
    Carver c;
    if (cfg.d.prec == WL_FP64) {
        SimImpl<double> s;
        carve_sim<double>(c, s, cfg);
    } else {
        SimImpl<float> s;
        carve_sim<float>(c, s, cfg);
    }
    return c.off;
}

// ------------------------------------------------------------ Poisson
template <typename T>
struct PoissonImpl {
    Grid g;
    int nlev;
    Hierarchy<T> h;
    Reduce red;
    bool have = false;
};

struct PoissonMixedImpl {
    Grid g;
    int nlev;
    Hierarchy<float> h;
    Mixed64 mix;
    Reduce red;
    bool have = false;
};

static wl_status check_poisson(int ndim, const int n[3], const int periodic[3], int prec, int levels,
                               Grid* g, int* nlev) {
    if (ndim != 2 && ndim != 3) return invalid("ndim must be 2 or 3");
    if (!n || !periodic) return invalid("n / periodic is NULL");
    if (ndim == 2 && n[2] != 1) return invalid("2D problems need n[2] == 1");
    for (int i = 0; i < ndim; ++i)
        if (n[i] < 2) return invalid("every direction needs at least 2 cells");
    if (prec < 0 || prec > 2) return invalid("prec must be WL_FP32, WL_FP64 or WL_MIXED");
    if (levels < 0 || levels > kMaxLevels) return invalid("levels out of range");
    *g = Grid{n[0], n[1], n[2], periodic[0] != 0, periodic[1] != 0, ndim == 3 && periodic[2] != 0,
              ndim};
    *nlev = auto_levels(ndim, n, levels);
    if (levels > 0 && *nlev != levels)
        return invalid("the requested number of multigrid levels needs more even halvings");
    int m[3] = {n[0], n[1], n[2]};
    for (int l = 1; l < *nlev; ++l)
        for (int i = 0; i < ndim; ++i) m[i] /= 2;
    if (size_t(m[0]) * m[1] * m[2] > size_t(kCoarseMax))
        return invalid("coarsest multigrid level exceeds 1024 cells (request more levels)");
    return WL_OK;
}

template <typename H>
static void carve_poisson_common(Carver& c, H& P, const Grid& g, int nlev, bool fine_x) {
    const int n[3] = {g.n0, g.n1, g.n2};
    const int per[3] = {g.per0, g.per1, g.per2};
    carve_hierarchy(c, P.h, g.ndim, n, per, nlev, fine_x);
    P.red.slots = reduce_slots_for(g);
    P.red.partial = c.take<double>(2 * P.red.slots);
    P.red.result = c.take<double>(kResultDoubles);
}

template <typename T>
static wl_status copy_field(wl_sim* sim, int field, const void* src, void* dst) {
    SimImpl<T>& s = *static_cast<SimImpl<T>*>(sim->impl);
    T* ptr = nullptr;
    size_t count = 0;
    WL_TRY(sim_field_ptr<T>(s, field, &ptr, &count, src != nullptr));
    if (src) {
        WL_CHECK_HIP(hipMemcpyAsync(ptr, src, count * sizeof(T), hipMemcpyDeviceToDevice, sim->stream));
        if (field != WL_FIELD_P) {
            s.cfl_valid = false;
            s.dt_host = 0.0;
        }
        if (field == WL_FIELD_P && s.p64)
            WL_TRY((convert<float, double>(reinterpret_cast<float*>(s.p), s.p64, count, sim->stream)));
    } else {
        WL_CHECK_HIP(hipMemcpyAsync(dst, ptr, count * sizeof(T), hipMemcpyDeviceToDevice, sim->stream));
    }
    WL_CHECK_HIP(hipStreamSynchronize(sim->stream));
    return WL_OK;
}

template <typename T>
static wl_status poisson_solve_plain(wl_poisson* ps, const void* coeffs, void* x, const void* b,
                                     double tol, int maxv, int* vc, double* rel) {
    PoissonImpl<T>& P = *static_cast<PoissonImpl<T>*>(ps->impl);
    hipStream_t st = ps->stream;
    if (coeffs) {
        WL_TRY((mg_load_coeffs<T, T>(P.g, static_cast<const T*>(coeffs), P.h.lev[0].L, nullptr, st)));
        P.h.lev[0].uniform = 0;
        WL_TRY(mg_coarsen_all<T>(P.h, st));
        WL_TRY(mg_count_active<T>(P.h, P.red, st));
        P.have = true;
    }
    if (!P.have) return invalid("no coefficients given yet");
    SolveResult r;
    wl_status rc = mg_solve<T>(P.h, P.red, static_cast<T*>(x), static_cast<const T*>(b), tol, 0.0,
                               maxv, st, &r);
    if (vc) *vc = r.vcycles;
    if (rel) *rel = r.rel;
    return rc;
}

static wl_status poisson_solve_mixed(wl_poisson* ps, const void* coeffs, void* x, const void* b,
                                     double tol, int maxv, int* vc, double* rel) {
    PoissonMixedImpl& P = *static_cast<PoissonMixedImpl*>(ps->impl);
    hipStream_t st = ps->stream;
    if (coeffs) {
        WL_TRY((mg_load_coeffs<double, float>(P.g, static_cast<const double*>(coeffs), P.h.lev[0].L,
                                              P.mix.L, st)));
        P.h.lev[0].uniform = 0;
        WL_TRY(mg_coarsen_all<float>(P.h, st));
        WL_TRY(mg_mixed_classes(P.g, P.mix, st));
        WL_TRY(mg_count_active64(P.g, P.mix.L, P.red, &P.h.n_active, st));
        P.have = true;
    }
    if (!P.have) return invalid("no coefficients given yet");
    SolveResult r;
    wl_status rc = mg_solve_mixed(P.h, P.mix, P.red, static_cast<double*>(x),
                                  static_cast<const double*>(b), tol, 0.0, maxv, st, &r);
    if (vc) *vc = r.vcycles;
    if (rel) *rel = r.rel;
    return rc;
}

// Clear the geometry-adjoint accumulators (the workspace starts uninitialised).
template <typename T>
static wl_status adj_clear(SimImpl<T>& s, hipStream_t st) {
    AdjointWS<T>& A = *s.adj;
    const size_t N = s.cfg.N;
    for (int i = 0; i < 3; ++i) {
        WL_TRY(fill<T>(A.Lb[i], N, T(0), st));
        WL_TRY(fill<T>(A.mu0b[i], N, T(0), st));
    }
    for (int i = 0; i < 9; ++i) WL_TRY(fill<T>(A.mu1nb[i], N, T(0), st));
    WL_CHECK_HIP(hipStreamSynchronize(st));
    return WL_OK;
}

template <typename T>
static wl_status tape_record(SimImpl<T>& s, int on, hipStream_t st) {
    if (!s.adj) {
        set_error("this simulation was created with tape_steps = 0");
        return WL_ERR_STATE;
    }
    s.adj->recording = on != 0;
    if (on) {
        s.adj->count = 0;
        WL_TRY(adj_clear(s, st));
    }
    return WL_OK;
}

// ------------------------------------------------------- checkpoint state
// Snapshot layout (see wl_state_size in wl.h): a 64-byte header of doubles
// (tag, t, next dt, ndim, n0, n1, n2, precision), then velocity components,
// outflow plane, pressure and (MIXED) the FP64 pressure, each at the next
// 256-byte boundary.
constexpr double kStateTag = 1.0;

struct StateLayout {
    size_t vel[3] = {0, 0, 0};
    size_t plane = 0, p = 0, p64 = 0, bytes = 0;
};

template <typename T>
static StateLayout state_layout(const SimImpl<T>& s) {
    const SimConfig& c = s.cfg;
    StateLayout Lo;
    size_t off = 256;
    auto take = [&](size_t nbytes) {
        const size_t at = off;
        off = (off + nbytes + 255) & ~size_t(255);
        return at;
    };
    for (int i = 0; i < c.d.ndim; ++i) Lo.vel[i] = take(c.N * sizeof(T));
    if (c.outflow) Lo.plane = take(c.P * sizeof(T));
    Lo.p = take(c.N * sizeof(T));
    if (s.p64) Lo.p64 = take(c.N * sizeof(double));
    Lo.bytes = off;
    return Lo;
}

template <typename T>
static void state_header(const SimImpl<T>& s, double h[8]) {
    const SimConfig& c = s.cfg;
    h[0] = kStateTag;
    h[1] = s.t;
    h[2] = 0.0;
    h[3] = c.d.ndim;
    h[4] = c.d.n[0];
    h[5] = c.d.n[1];
    h[6] = c.d.n[2];
    h[7] = c.d.prec;
}

template <typename T>
static wl_status sim_get_state(SimImpl<T>& s, void* dst, hipStream_t st) {
    const SimConfig& c = s.cfg;
    const StateLayout Lo = state_layout(s);
    char* d = static_cast<char*>(dst);
    double h[8];
    state_header(s, h);
    WL_CHECK_HIP(hipMemcpyAsync(d, h, sizeof(h), hipMemcpyHostToDevice, st));
    // the next dt lives on the device (the last projection formed it)
    if (s.cfl_valid)
        WL_CHECK_HIP(hipMemcpyAsync(d + 2 * sizeof(double), s.scal + s.dt_cur, sizeof(double),
                                    hipMemcpyDeviceToDevice, st));
    for (int i = 0; i < c.d.ndim; ++i)
        WL_CHECK_HIP(hipMemcpyAsync(d + Lo.vel[i], s.vel[s.S][i], c.N * sizeof(T),
                                    hipMemcpyDeviceToDevice, st));
    if (c.outflow)
        WL_CHECK_HIP(hipMemcpyAsync(d + Lo.plane, s.plane[s.PS], c.P * sizeof(T),
                                    hipMemcpyDeviceToDevice, st));
    WL_CHECK_HIP(hipMemcpyAsync(d + Lo.p, s.p, c.N * sizeof(T), hipMemcpyDeviceToDevice, st));
    if (s.p64)
        WL_CHECK_HIP(hipMemcpyAsync(d + Lo.p64, s.p64, c.N * sizeof(double),
                                    hipMemcpyDeviceToDevice, st));
    WL_CHECK_HIP(hipStreamSynchronize(st));  // h must outlive its copy
    return WL_OK;
}

template <typename T>
static wl_status sim_set_state(SimImpl<T>& s, const void* src, hipStream_t st) {
    const SimConfig& c = s.cfg;
    const StateLayout Lo = state_layout(s);
    const char* d = static_cast<const char*>(src);
    double h[8], want[8];
    WL_CHECK_HIP(hipMemcpyAsync(h, d, sizeof(h), hipMemcpyDeviceToHost, st));
    WL_CHECK_HIP(hipStreamSynchronize(st));
    state_header(s, want);
    if (h[0] != want[0]) return invalid("state buffer has no snapshot header");
    for (int q = 3; q < 8; ++q)
        if (h[q] != want[q]) return invalid("snapshot belongs to another grid or precision");
    if (!std::isfinite(h[1]) || !(h[2] >= 0.0) || !std::isfinite(h[2]))
        return invalid("snapshot time / dt is not finite");
    for (int i = 0; i < c.d.ndim; ++i)
        WL_CHECK_HIP(hipMemcpyAsync(s.vel[s.S][i], d + Lo.vel[i], c.N * sizeof(T),
                                    hipMemcpyDeviceToDevice, st));
    if (c.outflow)
        WL_CHECK_HIP(hipMemcpyAsync(s.plane[s.PS], d + Lo.plane, c.P * sizeof(T),
                                    hipMemcpyDeviceToDevice, st));
    WL_CHECK_HIP(hipMemcpyAsync(s.p, d + Lo.p, c.N * sizeof(T), hipMemcpyDeviceToDevice, st));
    if (s.p64)
        WL_CHECK_HIP(hipMemcpyAsync(s.p64, d + Lo.p64, c.N * sizeof(double),
                                    hipMemcpyDeviceToDevice, st));
    s.t = h[1];
    if (h[2] > 0.0) {
        WL_CHECK_HIP(hipMemcpyAsync(s.scal + s.dt_cur, d + 2 * sizeof(double), sizeof(double),
                                    hipMemcpyDeviceToDevice, st));
        s.cfl_valid = true;
        s.dt_host = h[2];
    } else {
        s.cfl_valid = false;
        s.dt_host = 0.0;
    }
    WL_CHECK_HIP(hipStreamSynchronize(st));
    return WL_OK;
}

}  // namespace wl

using namespace wl;

extern "C" {

const char* wl_last_error(void) { return g_err.c_str(); }
const char* wl_version(void) { return "wl 0.1 (gfx950)"; }

wl_status wl_sim_footprint(const wl_sim_desc* desc, size_t* bytes) {
    clear_error();
    if (!bytes) return invalid("bytes is NULL");
    SimConfig cfg;
    WL_TRY(check_desc(desc, &cfg));
    *bytes = sim_bytes(cfg);
    return WL_OK;
}

wl_status wl_sim_create(const wl_sim_desc* desc, void* workspace, size_t ws_bytes, void* hip_stream,
                        wl_sim** out) {
    clear_error();
    if (!out) return invalid("out is NULL");
    *out = nullptr;
    SimConfig cfg;
    WL_TRY(check_desc(desc, &cfg));
    const size_t need = sim_bytes(cfg);
    if (!workspace) return invalid("workspace is NULL");
    if (reinterpret_cast<uintptr_t>(workspace) % 256) return invalid("workspace must be 256-byte aligned");
    if (ws_bytes < need) {
        set_error("workspace smaller than wl_sim_footprint");
        return WL_ERR_OUT_OF_MEMORY;
    }
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    wl_sim* sim = new (std::nothrow) wl_sim;
    if (!sim) return invalid("host allocation failed");
    sim->prec = cfg.d.prec;
    sim->stream = st;
    Carver c;
    c.base = static_cast<char*>(workspace);
    wl_status rc;
    if (cfg.d.prec == WL_FP64) {
        auto* s = new (std::nothrow) SimImpl<double>;
        carve_sim<double>(c, *s, cfg);
        sim->impl = s;
        rc = sim_init<double>(*s, st);
    } else {
        auto* s = new (std::nothrow) SimImpl<float>;
        carve_sim<float>(c, *s, cfg);
        sim->impl = s;
        rc = sim_init<float>(*s, st);
    }
    if (rc != WL_OK) {
        wl_sim_destroy(sim);
        return rc;
    }
    *out = sim;
    return WL_OK;
}

wl_status wl_sim_destroy(wl_sim* sim) {
    clear_error();
    if (!sim) return WL_OK;
    if (sim->prec == WL_FP64)
        delete static_cast<SimImpl<double>*>(sim->impl);
    else
        delete static_cast<SimImpl<float>*>(sim->impl);
    delete sim;
    return WL_OK;
}

wl_status wl_set_field(wl_sim* sim, int field, const void* src) {
    clear_error();
    if (!sim || !src) return invalid("sim / src is NULL");
    return sim->prec == WL_FP64 ? copy_field<double>(sim, field, src, nullptr)
                                : copy_field<float>(sim, field, src, nullptr);
}

wl_status wl_get_field(const wl_sim* sim, int field, void* dst) {
    clear_error();
    if (!sim || !dst) return invalid("sim / dst is NULL");
    wl_sim* s = const_cast<wl_sim*>(sim);
    return sim->prec == WL_FP64 ? copy_field<double>(s, field, nullptr, dst)
                                : copy_field<float>(s, field, nullptr, dst);
}

wl_status wl_set_time(wl_sim* sim, double t) {
    clear_error();
    if (!sim) return invalid("sim is NULL");
    if (sim->prec == WL_FP64)
        static_cast<SimImpl<double>*>(sim->impl)->t = t;
    else
        static_cast<SimImpl<float>*>(sim->impl)->t = t;
    return WL_OK;
}

wl_status wl_state_size(const wl_sim* sim, size_t* bytes) {
    clear_error();
    if (!sim || !bytes) return invalid("sim / bytes is NULL");
    if (sim->prec == WL_FP64)
        *bytes = state_layout(*static_cast<const SimImpl<double>*>(sim->impl)).bytes;
    else
        *bytes = state_layout(*static_cast<const SimImpl<float>*>(sim->impl)).bytes;
    return WL_OK;
}

wl_status wl_get_state(const wl_sim* sim, void* dst) {
    clear_error();
    if (!sim || !dst) return invalid("sim / dst is NULL");
    if (reinterpret_cast<uintptr_t>(dst) % 256) return invalid("dst must be 256-byte aligned");
    if (sim->prec == WL_FP64)
        return sim_get_state<double>(*static_cast<SimImpl<double>*>(sim->impl), dst, sim->stream);
    return sim_get_state<float>(*static_cast<SimImpl<float>*>(sim->impl), dst, sim->stream);
}

wl_status wl_set_state(wl_sim* sim, const void* src) {
    clear_error();
    if (!sim || !src) return invalid("sim / src is NULL");
    if (reinterpret_cast<uintptr_t>(src) % 256) return invalid("src must be 256-byte aligned");
    if (sim->prec == WL_FP64)
        return sim_set_state<double>(*static_cast<SimImpl<double>*>(sim->impl), src, sim->stream);
    return sim_set_state<float>(*static_cast<SimImpl<float>*>(sim->impl), src, sim->stream);
}

wl_status wl_step(wl_sim* sim, double dt, wl_step_stats* stats) {
    clear_error();
    if (!sim) return invalid("sim is NULL");
    if (sim->prec == WL_FP64)
        return sim_step<double>(*static_cast<SimImpl<double>*>(sim->impl), dt, stats, sim->stream);
    return sim_step<float>(*static_cast<SimImpl<float>*>(sim->impl), dt, stats, sim->stream);
}

wl_status wl_run(wl_sim* sim, int nsteps, double t_end, wl_step_stats* stats, int* taken) {
    clear_error();
    if (taken) *taken = 0;
    if (!sim) return invalid("sim is NULL");
    if (nsteps < 0) return invalid("nsteps must be >= 0");
    for (int k = 0; k < nsteps; ++k) {
        wl_step_stats st{};
        const wl_status rc = wl_step(sim, 0.0, &st);
        if (rc != WL_OK && rc != WL_ERR_NOT_CONVERGED) return rc;
        if (stats) stats[k] = st;
        if (taken) *taken = k + 1;
        if (rc != WL_OK) return rc;
        if (t_end > 0.0 && st.t >= t_end) break;
    }
    return WL_OK;
}

wl_status wl_drag(wl_sim* sim, double* Fx) {
    clear_error();
    if (!sim || !Fx) return invalid("sim / Fx is NULL");
    if (sim->prec == WL_FP64)
        return sim_drag<double>(*static_cast<SimImpl<double>*>(sim->impl), Fx, sim->stream);
    return sim_drag<float>(*static_cast<SimImpl<float>*>(sim->impl), Fx, sim->stream);
}

wl_status wl_tape_record(wl_sim* sim, int on) {
    clear_error();
    if (!sim) return invalid("sim is NULL");
    if (sim->prec == WL_FP64)
        return tape_record<double>(*static_cast<SimImpl<double>*>(sim->impl), on, sim->stream);
    return tape_record<float>(*static_cast<SimImpl<float>*>(sim->impl), on, sim->stream);
}

wl_status wl_step_adjoint(wl_sim* sim, const void* ubar_in, const void* pbar_in,
                          double drag_weight, void* ubar_out, double* g_params) {
    clear_error();
    if (!sim || !ubar_in || !ubar_out) return invalid("sim / ubar_in / ubar_out is NULL");
    if (sim->prec == WL_FP64)
        return sim_step_adjoint<double>(*static_cast<SimImpl<double>*>(sim->impl), ubar_in,
                                        pbar_in, drag_weight, ubar_out, g_params, sim->stream);
    return sim_step_adjoint<float>(*static_cast<SimImpl<float>*>(sim->impl), ubar_in, pbar_in,
                                   drag_weight, ubar_out, g_params, sim->stream);
}

wl_status wl_poisson_footprint(int ndim, const int n[3], const int periodic[3], int prec, int levels,
                               size_t* bytes) {
    clear_error();
    if (!bytes) return invalid("bytes is NULL");
    Grid g;
    int nlev;
    WL_TRY(check_poisson(ndim, n, periodic, prec, levels, &g, &nlev));
    Carver c;
    if (prec == WL_FP32) {
        PoissonImpl<float> P;
        carve_poisson_common(c, P, g, nlev, false);
    } else if (prec == WL_FP64) {
        PoissonImpl<double> P;
        carve_poisson_common(c, P, g, nlev, false);
    } else {
        PoissonMixedImpl P;
        carve_poisson_common(c, P, g, nlev, true);
        for (int i = 0; i < 3; ++i) P.mix.L[i] = c.take<double>(cells(g));
        P.mix.cls = c.take<unsigned char>(reduce_slots_for(g));
    }
    *bytes = c.off;
    return WL_OK;
}

wl_status wl_poisson_create(int ndim, const int n[3], const int periodic[3], int prec, int levels,
                            void* workspace, size_t ws_bytes, void* hip_stream, wl_poisson** out) {
    clear_error();
    if (!out) return invalid("out is NULL");
    *out = nullptr;
    size_t need = 0;
    WL_TRY(wl_poisson_footprint(ndim, n, periodic, prec, levels, &need));
    if (!workspace) return invalid("workspace is NULL");
    if (reinterpret_cast<uintptr_t>(workspace) % 256) return invalid("workspace must be 256-byte aligned");
    if (ws_bytes < need) {
        set_error("workspace smaller than wl_poisson_footprint");
        return WL_ERR_OUT_OF_MEMORY;
    }
    Grid g;
    int nlev;
    WL_TRY(check_poisson(ndim, n, periodic, prec, levels, &g, &nlev));
    wl_poisson* ps = new (std::nothrow) wl_poisson;
    if (!ps) return invalid("host allocation failed");
    ps->prec = prec;
    ps->stream = reinterpret_cast<hipStream_t>(hip_stream);
    Carver c;
    c.base = static_cast<char*>(workspace);
    if (prec == WL_FP32) {
        auto* P = new PoissonImpl<float>;
        P->g = g;
        P->nlev = nlev;
        carve_poisson_common(c, *P, g, nlev, false);
        P->h.coarse_tol = 1e-6;
        ps->impl = P;
    } else if (prec == WL_FP64) {
        auto* P = new PoissonImpl<double>;
        P->g = g;
        P->nlev = nlev;
        carve_poisson_common(c, *P, g, nlev, false);
        P->h.coarse_tol = 1e-10;
        ps->impl = P;
    } else {
        auto* P = new PoissonMixedImpl;
        P->g = g;
        P->nlev = nlev;
        carve_poisson_common(c, *P, g, nlev, true);
        for (int i = 0; i < 3; ++i) P->mix.L[i] = c.take<double>(cells(g));
        P->mix.cls = c.take<unsigned char>(reduce_slots_for(g));
        P->h.coarse_tol = 1e-6;
        ps->impl = P;
    }
    *out = ps;
    return WL_OK;
}

wl_status wl_poisson_solve(wl_poisson* ps, const void* coeffs, void* x, const void* b, double tol,
                           int max_vcycles, int* vcycles_out, double* rel_resid_out) {
    clear_error();
    if (!ps || !x || !b) return invalid("ps / x / b is NULL");
    if (!(tol >= 0.0)) return invalid("tol must be >= 0");
    if (max_vcycles <= 0) max_vcycles = 100;
    if (ps->prec == WL_FP32)
        return poisson_solve_plain<float>(ps, coeffs, x, b, tol, max_vcycles, vcycles_out,
                                          rel_resid_out);
    if (ps->prec == WL_FP64)
        return poisson_solve_plain<double>(ps, coeffs, x, b, tol, max_vcycles, vcycles_out,
                                           rel_resid_out);
    return poisson_solve_mixed(ps, coeffs, x, b, tol, max_vcycles, vcycles_out, rel_resid_out);
}

wl_status wl_body_coeffs(const wl_body* body, int ndim, const int n[3], const int periodic[3],
                         int prec, void* L_out, void* hip_stream) {
    clear_error();
    if (!body || !n || !periodic || !L_out) return invalid("NULL argument");
    if (ndim != 2 && ndim != 3) return invalid("ndim must be 2 or 3");
    if (ndim == 2 && n[2] != 1) return invalid("2D problems need n[2] == 1");
    for (int i = 0; i < ndim; ++i)
        if (n[i] < 1) return invalid("grid dimensions must be positive");
    if (prec < 0 || prec > 2) return invalid("prec must be WL_FP32, WL_FP64 or WL_MIXED");
    if (body->kind < 0 || body->kind > 2) return invalid("body.kind must be 0, 1 or 2");
    if (body->kind != 0 && !(body->radius > 0.0)) return invalid("body radius must be > 0");
    if (body->kind == 2 && (ndim != 3 || !(body->radius2 > 0.0)))
        return invalid("a torus needs ndim = 3 and radius2 > 0");
    const Grid g{n[0], n[1], n[2], periodic[0] != 0, periodic[1] != 0,
                 ndim == 3 && periodic[2] != 0, ndim};
    const int bclo[3] = {g.per0 ? WL_BC_PERIODIC : WL_BC_WALL, g.per1 ? WL_BC_PERIODIC : WL_BC_WALL,
                         g.per2 ? WL_BC_PERIODIC : WL_BC_WALL};
    BodyDev bd{body->kind,
               {body->centre[0], body->centre[1], body->centre[2]},
               body->radius,
               body->eps > 0.0 ? body->eps : 1.0,
               body->radius2};
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    const size_t N = cells(g);
    if (prec == WL_FP32) {
        float* L = static_cast<float*>(L_out);
        MeasureOut<float> M{{nullptr, nullptr, nullptr},
                            {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                             nullptr},
                            {L, L + N, ndim == 3 ? L + 2 * N : nullptr},
                            {nullptr, nullptr, nullptr}};
        WL_TRY(ns_measure<float>(g, bd, bclo, M, st));
    } else {
        double* L = static_cast<double*>(L_out);
        MeasureOut<double> M{{nullptr, nullptr, nullptr},
                             {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                              nullptr, nullptr},
                             {L, L + N, ndim == 3 ? L + 2 * N : nullptr},
                             {nullptr, nullptr, nullptr}};
        WL_TRY(ns_measure<double>(g, bd, bclo, M, st));
    }
    WL_CHECK_HIP(hipStreamSynchronize(st));
    return WL_OK;
}

wl_status wl_poisson_destroy(wl_poisson* ps) {
    clear_error();
    if (!ps) return WL_OK;
    if (ps->prec == WL_FP32)
        delete static_cast<PoissonImpl<float>*>(ps->impl);
    else if (ps->prec == WL_FP64)
        delete static_cast<PoissonImpl<double>*>(ps->impl);
    else
        delete static_cast<PoissonMixedImpl*>(ps->impl);
    delete ps;
    return WL_OK;
}

}  // extern "C"
