"""Benchmark: 3D Taylor-Green vortex time steps on one MI355X.

Workload (the metric configuration): triply periodic TGV, N^3 = 256^3 cells,
FP32 fields and FP32 GMG pressure solves, Re = 1600, no body, CFL-adaptive
Heun steps.  The in-step solves stop once the divergence they leave in the
projected velocity has an RMS of at most 1e-5 (the configuration's FP32 GMG
tolerance read as a divergence bound: an FP32 pressure's rounding alone
floors the relative residual near 6e-5 at 256^3); the relative residuals the
solves actually reach are reported beside it.  A step is one full pass of the
hot path: CFL time step, two stages of convection-diffusion + divergence +
GMG solve + projection.  Inputs are resident in HBM before the timed region.

Prints one JSON line: cell-steps/s, the roofline of the dominant kernel
(algorithmic bytes / HIP-event-timed launch duration vs 8 TB/s), the
whole-step algorithmic-byte fraction, a leg with a fixed number of V-cycles
per solve (the GMG loaded: per-V-cycle time and bytes), the standalone
Poisson solve (mixed vs FP64, with its roofline by the byte model below) and
the FP64 oracle timed on the host as a CPU baseline.
"""

import argparse
import ast
import ctypes
import json
import math
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# Algorithmic bytes per fine cell of each timed kernel class (FP32, 3D,
# uniform coefficients: the TGV has no body and is periodic, so the Poisson
# coefficients are never read).  Reads + writes of the fields each kernel
# must touch once.
BYTES_PER_CELL = {
    "smooth_fine": 12.0,     # read x, b; write x'
    "smooth_norm": 12.0,     # same sweep + per-block partial sums
    "prolong_fine": 8.5,     # x += P x_coarse in place: read x, x_coarse (1/8); write x
    "restrict_fine": 8.5,    # read x, b; write b_coarse (1/8)
    "momentum": 32.0,        # predictor 24 (read u, write f); corrector 40 (read u*, p, u^n,
                             # write f: it applies the predictor's projection as it loads)
    "divergence": 20.0,      # read u* (3 comps) and p (the solve's first residual check,
                             # fused in on this grid); write sigma
    "project": 28.0,         # read u* (3), p; write u (3)
    "norm_fine": 8.0,        # residual norm only: read x, b
    "pair_fine": 12.0,       # two sweeps in one pass: read x, b; write x''
    "pair_prolong_fine": 12.0,  # post-smoothing pair after the prolongation: read x, b; write x''
}


# Per V-cycle with fused sweep pairs on every level (FP32, uniform, 3D), per
# fine cell: pre pair 12, restriction 8.5, prolongation 8.5, post pair 12,
# the measuring residual check 8; each coarser level costs 37 B per own cell
# (zero-start pair 8, restriction 8.5, prolongation 8.5, post pair 12), i.e.
# 37 (1/8 + 1/64 + ...) = 37/7 per fine cell.
VCYCLE_FUSED = 12 + 8.5 + 8.5 + 12 + 8 + 37.0 / 7
# Separate sweeps: the check doubles as the first pre-sweep (12), second
# pre-sweep 12, restriction 8.5, prolongation 8.5, two post sweeps 24, and
# 61 B per cell of each coarser level (four sweeps, restriction, prolongation).
VCYCLE_SEPARATE = 12 + 12 + 8.5 + 8.5 + 24 + 61.0 / 7


def step_bytes_per_cell(vcycles_total, fused):
    """Algorithmic bytes of one step per fine cell (FP32, uniform L, 3D).

    momentum 24 + 40 (the corrector applies the predictor's projection as it
    loads u*), divergence 2 x 16, the corrector's projection 28, per solve the
    first residual check (fused pairs: taken inside the divergence, which then
    also reads p, 4; separate sweeps: a check-and-sweep pass, 12), and per
    V-cycle VCYCLE_FUSED or VCYCLE_SEPARATE.
    """
    first = 4.0 if fused else 12.0
    per_vcycle = VCYCLE_FUSED if fused else VCYCLE_SEPARATE
    return 64.0 + 32.0 + 28.0 + 2 * first + per_vcycle * vcycles_total


# Standalone Poisson solve with BDIM coefficients (the C3 workload), per fine
# cell, by the byte model that prices x and b only (the coefficients counted
# as read on the body's tiles alone): plain FP64, the active mean of b (8) and
# the first check (x, b: 16), then 146 B per V-cycle; mixed precision, the
# FP64 mean (8) and first residual (read x, b, write the FP32 defect: 20),
# then per outer iteration the FP64 update (read e, x, write x: 20) and
# residual (20), plus 65 B per inner FP32 V-cycle.
def poisson_bytes_per_cell(prec, vcycles, inner=3):
    if prec == "fp64":
        return 24.0 + 146.0 * vcycles
    outer = -(-vcycles // inner)
    return 28.0 + 40.0 * outer + 65.0 * vcycles


# HBM traffic of the dominant kernel per launch from rocprofv3 counters
# (FETCH_SIZE and WRITE_SIZE runs, each scaled by what the same counter reads
# for a plain device copy of known size), stored with a hash of the kernel
# sources it was measured on; reported only while those sources are unchanged.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "momentum_tgv256_hbm_traffic.md")
KERNEL_SOURCES = ["paper_2304_08159_amd/csrc/ns.hip", "paper_2304_08159_amd/csrc/wl_vel.h",
                  "paper_2304_08159_amd/csrc/wl_device.h", "paper_2304_08159_amd/csrc/wl_ns.h",
                  "paper_2304_08159_amd/csrc/wl_internal.h"]


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel):
    try:
        text = open(TRAFFIC_FILE).read()
        blob = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    except (OSError, IndexError, ValueError):
        return None
    if blob.get("kernel") != kernel or blob.get("sources_sha256") != kernel_sources_sha256():
        return None
    return blob.get("traffic_bytes_per_launch")


def cpu_baseline(N, vcycles):
    """Time the FP64 oracle for one Heun step of the TGV at N^3 on one core."""
    code = (
        "import sys, time; sys.path.insert(0, %r)\n"
        "import workloads as W\n"
        "from oracle import step as S\n"
        "N = %d\n"
        "u, v, w, nu = W.tgv3d(N)\n"
        "sim = S.Sim((N, N, N), [0]*3, [0]*3, (0, 0, 0), nu, tol=1e-5)\n"
        "sim.u = [u, v, w]\n"
        "dt = sim.dt_cfl()\n"
        "t = time.perf_counter()\n"
        "sim.step(dt=dt, force_vcycles=%r)\n"
        "print(time.perf_counter() - t)\n"
    ) % (ROOT, N, tuple(vcycles))
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env,
                       timeout=600)
    if r.returncode != 0:
        raise RuntimeError(r.stderr)
    secs = float(r.stdout.strip().splitlines()[-1])
    return dict(value=N ** 3 / secs, unit="cell-steps/s", cores=1, kind="oracle",
                cpu_model=host_cpu_model(),
                sample=f"one Heun step of the 3D TGV at {N}^3 (FP64 NumPy oracle, one thread, "
                       f"V-cycles per solve {tuple(vcycles)} = the GPU's mean rounded), "
                       f"{secs:.1f} s")


def host_cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_routines(N, vcycles):
    """The oracle's Heun step at N^3 split into the routines the paper's Table 2
    times (convdiff!, BDIM!, BC!, project!, CFL!): its functions are wrapped in
    timers inside a child process and the step itself runs unchanged."""
    code = (
        "import sys, time; sys.path.insert(0, %r)\n"
        "import workloads as W\n"
        "from oracle import step as S\n"
        "T = dict(convdiff=0.0, BDIM=0.0, BC=0.0, project=0.0, CFL=0.0)\n"
        "def timer(key, f):\n"
        "    def g(*a, **k):\n"
        "        t = time.perf_counter(); r = f(*a, **k); T[key] += time.perf_counter() - t\n"
        "        return r\n"
        "    return g\n"
        "M = S.momentum\n"
        "M.rhs = timer('convdiff', M.rhs); M.bdim = timer('BDIM', M.bdim)\n"
        "M.exit_flux_correct = timer('BC', M.exit_flux_correct)\n"
        "S.Sim._set_boundary = timer('BC', S.Sim._set_boundary)\n"
        "M.cfl_dt = timer('CFL', M.cfl_dt)\n"
        "S.divergence = timer('project', S.divergence)\n"
        "S.poisson.solve = timer('project', S.poisson.solve)\n"
        "S.grad_update = timer('project', S.grad_update)\n"
        "N = %d\n"
        "u, v, w, nu = W.tgv3d(N)\n"
        "sim = S.Sim((N, N, N), [0]*3, [0]*3, (0, 0, 0), nu, tol=1e-5)\n"
        "sim.u = [u, v, w]\n"
        "for k in T: T[k] = 0.0\n"
        "t = time.perf_counter()\n"
        "sim.step(force_vcycles=%r)\n"
        "T['step'] = time.perf_counter() - t\n"
        "print(repr(T))\n"
    ) % (ROOT, N, tuple(vcycles))
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env,
                       timeout=600)
    if r.returncode != 0:
        raise RuntimeError(r.stderr)
    T = ast.literal_eval(r.stdout.strip().splitlines()[-1])
    return {k: 1e3 * v for k, v in T.items()}


def poisson_compare(torch, wl, W, n, radius=32.0, tol=1e-8, reps=3):
    """Mixed-precision vs plain FP64 GMG on the sphere-in-a-box Poisson problem
    (BDIM coefficients of a sphere of radius 32 cells, N(0,1) RHS, tol 1e-8)."""
    import numpy as np
    from paper_2304_08159_amd import _lib
    cfg = W.poisson_sphere_config(n, radius)
    # BDIM coefficients come from the library's own geometry kernel (a 3D
    # simulation handle with the same body and Neumann walls)
    sim = wl.Sim(n, cfg["bc_lo"], cfg["bc_hi"], (0.0, 0.0, 0.0), 0.0, body=cfg["body"],
                 prec=wl.WL_FP64, levels=0, tol=tol)
    L = torch.stack([sim.get(wl.FIELD_L0 + i) for i in range(3)]).contiguous()
    sim.close()
    del sim
    b = torch.from_numpy(np.ascontiguousarray(W.random_rhs(n, 2304).transpose(2, 1, 0))).cuda()
    out = {}
    for name, prec in (("fp64", wl.WL_FP64), ("mixed", wl.WL_MIXED)):
        ps = wl.Poisson(n, (False, False, False), prec=prec)
        x = torch.zeros_like(b)
        ps.solve(L, x, b, tol=tol, max_vcycles=400)      # warm-up (also loads coefficients)
        times = []
        for _ in range(reps):
            x.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            k, rel = ps.solve(None, x, b, tol=tol, max_vcycles=400)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        ms = 1e3 * min(times)
        nbytes = poisson_bytes_per_cell(name, k) * n[0] * n[1] * n[2]
        out[name] = {"ms": ms, "vcycles": k, "rel_resid": rel,
                     "footprint_MB": ps.footprint / 1e6,
                     "roofline": {"bound": "hbm", "alg_bytes": nbytes,
                                  "achieved": nbytes / (ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                                  "unit": "GB/s",
                                  "frac": nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}}
        ps.close()
    out["speedup_mixed_over_fp64"] = out["fp64"]["ms"] / out["mixed"]["ms"]
    out["byte_model"] = ("x and b only (coefficients on the body's tiles alone): FP64 "
                         "24 + 146 B/cell per V-cycle; mixed 28 + 40 B/cell per outer iteration "
                         "+ 65 B/cell per inner FP32 V-cycle")
    out["workload"] = (f"Poisson {n[0]}x{n[1]}x{n[2]} Neumann box, sphere r={radius} BDIM "
                       f"coefficients, N(0,1) RHS seed 2304, to relative residual {tol}")
    return out


def batch_compare(torch, wl, count=256, n=(128, 128), tol=1e-8):
    """Many small Poisson problems (circle coefficients, N(0,1) right-hand
    sides, FP64 to tol): one persistent work-queue launch vs the per-problem
    solver one after another."""
    d = len(n)
    body = dict(centre=tuple(m / 2.0 for m in n), radius=min(n) / 4.0)
    L = wl.body_coeffs(n, (False,) * d, body, prec=wl.WL_FP64)
    shape = tuple(reversed(list(n) + [1] * (3 - d)))
    g = torch.Generator(device="cuda")
    g.manual_seed(2304)
    bs = [torch.randn(shape, generator=g, dtype=torch.float64, device="cuda") for _ in range(count)]

    def reqs():
        return [dict(n=n, periodic=(False,) * d, coeffs=L, x=torch.zeros_like(b), b=b, tol=tol,
                     max_vcycles=400) for b in bs]
    wl.poisson_batch_solve(reqs())              # warm-up at full size (workspace allocation)
    rq = reqs()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = wl.poisson_batch_solve(rq)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    ps = wl.Poisson(n, (False,) * d, prec=wl.WL_FP64)
    x = torch.zeros_like(bs[0])
    ps.solve(L, x, bs[0], tol=tol, max_vcycles=400)   # warm-up, loads the coefficients
    nseq = min(count, 64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for b in bs[:nseq]:
        x.zero_()
        ps.solve(None, x, b, tol=tol, max_vcycles=400)
    torch.cuda.synchronize()
    t_seq = (time.perf_counter() - t0) * count / nseq
    ps.close()
    return dict(workload=f"{count} Poisson problems {n[0]}x{n[1]}, circle r={min(n) / 4:.0f}, "
                         f"FP64 to {tol}",
                batched_problems_per_s=count / t_batch, sequential_problems_per_s=count / t_seq,
                speedup=t_seq / t_batch, vcycles_mean=sum(o[1] for o in out) / count)


def vcycle_leg(torch, wl, _lib, lib, W, N, steps=20):
    """The 256^3 TGV step with the GMG loaded: every solve runs a fixed number
    of V-cycles (tolerance 0, max_vcycles = K) for K = 1 and K = 3; the
    per-V-cycle time is the difference over the 4 extra V-cycles per step, and
    the fine-level multigrid kernels of the K = 3 leg are event-timed."""
    import numpy as np
    u, v, w, nu = W.tgv3d(N)
    fields = [torch.from_numpy(np.ascontiguousarray(a.transpose(2, 1, 0))).float().cuda()
              for a in (u, v, w)]
    del u, v, w
    res = {}
    kern = {}
    for K in (1, 3):
        sim = wl.Sim((N, N, N), [0] * 3, [0] * 3, (0.0, 0.0, 0.0), nu, prec=wl.WL_FP32, tol=0.0,
                     max_vcycles=K)
        for i, f in enumerate(fields):
            sim.set(wl.FIELD_U0 + i, f)
        for _ in range(3):
            sim.step(allow_not_converged=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = [sim.step(allow_not_converged=True) for _ in range(steps)]
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        res[K] = dict(ms_per_step=1e3 * el / steps,
                      vcycles_per_solve=[st[-1]["vcycles"][0], st[-1]["vcycles"][1]],
                      rel_resid_mean=[float(np.mean([x["rel_resid"][i] for x in st]))
                                      for i in range(2)])
        if K == 3:
            names = ("pair_fine", "restrict_fine", "prolong_fine", "pair_prolong_fine",
                     "norm_fine")
            mask = sum(1 << _lib.PROF[nm] for nm in names)
            lib.wl_profile_enable(mask)
            lib.wl_profile_reset()
            for _ in range(5):
                sim.step(allow_not_converged=True)
            torch.cuda.synchronize()
            lib.wl_profile_enable(0)
            for nm in names:
                ms, cnt, cellsn = ctypes.c_double(), ctypes.c_longlong(), ctypes.c_longlong()
                lib.wl_profile_read(_lib.PROF[nm], ctypes.byref(ms), ctypes.byref(cnt),
                                    ctypes.byref(cellsn))
                if cnt.value:
                    avg = 1e3 * ms.value / cnt.value
                    b = BYTES_PER_CELL[nm] * cellsn.value
                    kern[nm] = dict(launches=cnt.value, avg_us=avg, gbs=b / (avg * 1e-6) / 1e9)
        sim.close()
        del sim
    per_v_ms = (res[3]["ms_per_step"] - res[1]["ms_per_step"]) / 4.0
    vbytes = VCYCLE_FUSED * N ** 3
    fine_us = sum(kern[k]["avg_us"] for k in ("pair_fine", "restrict_fine", "prolong_fine",
                                              "pair_prolong_fine", "norm_fine") if k in kern)
    fine_bytes = (12 + 8.5 + 8.5 + 12 + 8) * N ** 3
    return dict(workload=f"256^3 TGV steps with every solve fixed at K V-cycles (K = 1, 3)",
                legs={str(k): v for k, v in res.items()}, ms_per_vcycle=per_v_ms,
                vcycle_bytes_per_cell=VCYCLE_FUSED,
                vcycle_roofline={"bound": "hbm", "achieved": vbytes / (per_v_ms * 1e-3) / 1e9,
                                 "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                 "frac": vbytes / (per_v_ms * 1e-3) / 1e9 / HBM_PEAK_GBS},
                fine_level_kernels=kern,
                fine_level_roofline={"bytes_per_cell": 49.0, "kernel_us": fine_us,
                                     "achieved": fine_bytes / (fine_us * 1e-6) / 1e9 if fine_us
                                     else None})


def donut_bench(wl, W, p=7, steps=50, warmup=5):
    """Flow past a torus at N = (2^(p+1), 2^p, 2^p), Re = 1000 (FP32 fields and
    V-cycles, pressure solves to an RMS divergence of 1e-5): the paper's
    pressure-dominated workload.  Wall time per step after warm-up."""
    import torch
    cfg = W.donut_config(p)
    sim = wl.Sim(cfg["n"], cfg["bc_lo"], cfg["bc_hi"], cfg["U"], cfg["nu"], body=cfg["body"],
                 prec=wl.WL_FP32, tol=cfg["tol"], max_vcycles=100, cfl=cfg["cfl"])
    sim.run(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = sim.run(steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    sim.close()
    cells = cfg["n"][0] * cfg["n"][1] * cfg["n"][2]
    return dict(workload=f"torus in a {cfg['n'][0]}x{cfg['n'][1]}x{cfg['n'][2]} channel, "
                         f"R={cfg['body']['radius']:g}, tube {cfg['body']['radius2']:g}, Re=1000, "
                         f"FP32, solves to 1e-5", steps=len(st),
                ms_per_step=1e3 * el / len(st), cell_steps_per_s=cells * len(st) / el,
                vcycles_per_solve_mean=[sum(x["vcycles"][i] for x in st) / len(st)
                                        for i in range(2)])


def serving_bench(count=512, seed=2304, budget=16e9, slots=8):
    """Served mix: sizes uniform over 2D {64^2,128^2,256^2} and 3D {64^3,96^3,128^3},
    half Poisson solves, half 20-step NS runs with a body, all to a relative
    residual of 1e-8 with FP32 V-cycles and FP64 refinement; HBM budget 16 GB.
    Poisson requests of at most 16384 cells and NS requests of at most 4096
    cells are batched by kind into persistent work-queue kernels, larger ones
    run alone (the limits follow the latency of one request in one workgroup
    against the whole GPU).  Saturated throughput first (all requests at t = 0), then
    Poisson arrivals at 0.5 and 0.8 of it."""
    from paper_2304_08159_amd.serving import GpuExecutor, Server, make_requests, summarize
    ex = GpuExecutor()
    Server(ex, budget, slots=slots).run(make_requests(count=16, seed=seed + 1))   # warm-up

    def batch_stats(srv, reqs):
        done = [r for r in reqs if r.status == "done"]
        nb = sum(1 for r in done if r.result[1].get("batched"))
        return dict(units=len(srv.batches),
                    mean_size=(sum(srv.batches) / len(srv.batches)) if srv.batches else 0.0,
                    batched_fraction=nb / max(len(done), 1))
    srv = Server(ex, budget, slots=slots)
    done = srv.run(make_requests(count=count, seed=seed))
    sat = summarize(done)
    sat["batched"] = batch_stats(srv, done)
    mu = sat["throughput_rps"]
    res = {"saturated": sat}
    for frac in (0.5, 0.8):
        srv = Server(ex, budget, slots=slots)
        done = srv.run(make_requests(count=count, seed=seed, rate=frac * mu))
        r = summarize(done)
        r["arrival_rate_rps"] = frac * mu
        r["peak_bytes"] = srv.peak_bytes
        r["batched"] = batch_stats(srv, done)
        res[f"rate_{frac}"] = r
    res["config"] = dict(requests=count, budget_bytes=budget, slots=slots, seed=seed,
                         batch_cells=ex.batch_cells, ns_batch_cells=ex.ns_batch_cells,
                         tol=1e-8)
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--N", type=int, default=256)
    ap.add_argument("--cpu-N", type=int, default=256)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-poisson", action="store_true",
                    help="skip the mixed-vs-FP64 Poisson comparison")
    ap.add_argument("--no-serving", action="store_true", help="skip the served request mix")
    ap.add_argument("--donut", action="store_true",
                    help="also time flow past a torus at 256x128x128 (Re 1000)")
    ap.add_argument("--only-poisson", action="store_true",
                    help="run only the standalone mixed-vs-FP64 Poisson comparison (profiling)")
    ap.add_argument("--only-serving", action="store_true",
                    help="run only the batched-Poisson and served-mix legs")
    ap.add_argument("--no-vcycle-leg", action="store_true",
                    help="skip the leg with a fixed number of V-cycles per solve")
    ap.add_argument("--routines", action="store_true",
                    help="also split the oracle's step into convdiff/BDIM/BC/project/CFL (ms)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the library and this benchmark run on one GPU only; --gpus "
                                   "must be 1 (multi-GPU sharding is designed, not implemented)"}))
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2304_08159_amd as wl
    from paper_2304_08159_amd import _lib
    import workloads as W

    torch.cuda.set_device(0)
    N = args.N
    if args.only_poisson:
        print(json.dumps({"poisson_mixed_vs_fp64": poisson_compare(torch, wl, W, (N, N, N))}))
        return
    if args.only_serving:
        print(json.dumps({"poisson_batch": batch_compare(torch, wl),
                          "serving": serving_bench()}))
        return
    u, v, w, nu = W.tgv3d(N)
    sim = wl.Sim((N, N, N), [0] * 3, [0] * 3, (0.0, 0.0, 0.0), nu, prec=wl.WL_FP32, tol=1e-5,
                 max_vcycles=100)
    for i, a in enumerate((u, v, w)):
        t = torch.from_numpy(np.ascontiguousarray(a.transpose(2, 1, 0))).float().cuda()
        sim.set(wl.FIELD_U0 + i, t)
    del u, v, w
    if args.warmup:
        sim.run(args.warmup)
    lib = _lib.load()

    def ctypes_mask(on):
        return (1 << len(_lib.PROF)) - 1 if on else 0

    def timed(nsteps, profile):
        lib.wl_profile_enable(ctypes_mask(profile))
        lib.wl_profile_reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        vc = [st["vcycles"] for st in sim.run(nsteps)]
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        lib.wl_profile_enable(0)
        return el, vc

    def read_prof():
        kern = {}
        for name, kid in _lib.PROF.items():
            ms, n, cellsn = ctypes.c_double(), ctypes.c_longlong(), ctypes.c_longlong()
            lib.wl_profile_read(kid, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(cellsn))
            if n.value:
                avg_us = 1e3 * ms.value / n.value
                bytes_launch = BYTES_PER_CELL[name] * cellsn.value
                kern[name] = dict(launches=n.value, total_ms=ms.value, avg_us=avg_us,
                                  bytes_per_launch=bytes_launch,
                                  gbs=bytes_launch / (avg_us * 1e-6) / 1e9)
        return kern

    # short run with HIP-event brackets on every kernel class: the per-kernel
    # table and the dominant kernel (multigrid kernels are then launched
    # individually instead of from their captured graphs)
    prof_steps = min(args.steps, 40)
    elapsed_p, _ = timed(prof_steps, True)
    kern = read_prof()
    dom = max(kern, key=lambda k: kern[k]["total_ms"])
    # timed region: only the dominant kernel is bracketed, on the stream it is
    # launched on; its average launch time gives the roofline
    lib.wl_profile_enable(1 << _lib.PROF[dom])
    lib.wl_profile_reset()
    # the K steps run as one library call (the time loop of the method)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = sim.run(args.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    lib.wl_profile_enable(0)
    if len(stats) != args.steps:
        raise RuntimeError(f"the run stopped after {len(stats)} of {args.steps} steps")
    vcs = [st["vcycles"] for st in stats]
    rel_reached = [float(np.mean([st["rel_resid"][i] for st in stats])) for i in range(2)]
    dom_live = read_prof()[dom]
    ms_step = 1e3 * elapsed / args.steps
    cells = N ** 3
    value = cells * args.steps / elapsed
    vc_mean = [float(np.mean([a[i] for a in vcs])) for i in range(2)]
    step_b = step_bytes_per_cell(sum(vc_mean), "pair_fine" in kern) * cells
    step_gbs = step_b / (ms_step * 1e-3) / 1e9
    out = {
        "metric": f"cell-steps/s (3D TGV {N}^3 FP32)",
        "value": value,
        "unit": "cell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"3D Taylor-Green vortex, triply periodic {N}^3, FP32, Re=1600, "
                               f"no body, CFL 0.5 Heun steps, FP32 GMG solves stopped at an RMS "
                               f"divergence of 1e-5",
                   "N": N, "Re": 1600, "tol": 1e-5, "stop_rule": "rms_divergence",
                   "vcycles_per_solve_mean": vc_mean,
                   "rel_resid_reached_mean": rel_reached},
        "roofline": {
            "bound": "hbm",
            "kernel": dom,
            "achieved": dom_live["gbs"],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": dom_live["gbs"] / HBM_PEAK_GBS,
            "traffic": measured_traffic(dom),
            "bytes_per_cell": BYTES_PER_CELL[dom],
            "alg_bytes_per_launch": dom_live["bytes_per_launch"],
            "avg_launch_us": dom_live["avg_us"],
            "launches": dom_live["launches"],
        },
        "step_roofline": {"alg_bytes_per_step": step_b, "achieved_GBs": step_gbs,
                          "frac": step_gbs / HBM_PEAK_GBS},
        "kernels": kern,
        "kernels_note": f"all kernel classes event-timed over {prof_steps} separate steps "
                        f"(multigrid kernels launched individually there)",
        "profiled_ms_per_step": 1e3 * elapsed_p / prof_steps,
    }
    # plain device copy of 512 MiB (read + write) as the practical HBM ceiling
    src = torch.empty(128 << 20, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(20):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * src.numel() * 4 * 20 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    out["copy_GBs"] = copy_gbs
    out["roofline"]["frac_of_copy"] = kern[dom]["gbs"] / copy_gbs
    out["step_roofline"]["frac_of_copy"] = step_gbs / copy_gbs
    del src, dst
    sim.close()
    del sim
    torch.cuda.empty_cache()
    if not args.no_vcycle_leg:
        out["vcycle_leg"] = vcycle_leg(torch, wl, _lib, lib, W, N)
        torch.cuda.empty_cache()
    if not args.no_poisson:
        out["poisson_mixed_vs_fp64"] = poisson_compare(torch, wl, W, (N, N, N))
    if args.donut:
        out["donut"] = donut_bench(wl, W)
    if not args.no_serving:
        out["poisson_batch"] = batch_compare(torch, wl)
        out["serving"] = serving_bench()
    if not args.no_cpu_baseline:
        vcr = [int(round(x)) for x in vc_mean]
        try:
            out["cpu_baseline"] = cpu_baseline(args.cpu_N, vcr)
            if args.routines:
                out["cpu_baseline"]["routines_ms"] = cpu_routines(args.cpu_N, vcr)
        except Exception as e:  # report, do not hide
            out["cpu_baseline"] = {"error": str(e)[:200]}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
