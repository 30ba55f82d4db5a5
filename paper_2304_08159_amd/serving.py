"""Continuous-batching server for Poisson solves and short Navier-Stokes runs.

Requests of uneven grid sizes arrive over time.  The dispatcher admits a
waiting request as soon as an execution slot is free and the device memory it
needs (the library's exact workspace footprint plus its own fields) fits the
HBM budget; admitted requests run concurrently, each on its own HIP stream from
a worker thread, so their kernels overlap on the GPU while later arrivals keep
being admitted as earlier ones finish.  Every reduction in the library is a
fixed-order FP64 sum, so a request's result does not depend on what runs
beside it (checked bitwise by the tests through result fingerprints).

Small requests are batched: when one of them is admitted, the dispatcher
gathers further waiting small requests of the same kind (FIFO, up to
`batch_max`, within the free budget) into the same unit, which the executor
runs with one persistent work-queue kernel whose workgroups take requests
from a device queue, one request per workgroup at a time: Poisson solves
(`wl_poisson_batch_solve`, FP32 V-cycles with FP64 defect correction) or
whole Navier-Stokes runs (`wl_ns_batch_run`, FP32 fields, mixed-precision
solves).  A unit occupies one slot.

The scheduler is host logic only and talks to an `Executor`; `GpuExecutor`
drives libwl, tests can drive a fake one on the CPU.
"""

import collections
import dataclasses
import math
import threading
import time


@dataclasses.dataclass
class Request:
    id: int
    kind: str                      # "poisson" or "ns"
    n: tuple                       # grid cells (2D or 3D)
    arrival: float = 0.0           # seconds after the start of the run
    radius: float = 8.0            # sphere / circle radius in cells
    steps: int = 20                # NS time steps
    seed: int = 0                  # RHS seed (Poisson)
    tol: float = 1e-8
    # filled in by the server
    footprint: int = 0
    admitted: float = math.nan
    done: float = math.nan
    status: str = "waiting"
    result: object = None
    error: str = ""

    @property
    def latency(self):
        return self.done - self.arrival


class Executor:
    """What the server needs from a backend."""

    def footprint(self, req):      # bytes of device memory the request holds
        raise NotImplementedError

    def run(self, req):            # runs in a worker thread; returns the result
        raise NotImplementedError

    def batchable(self, req):      # may the request share a batched launch?
        return False

    def batch_key(self, req):      # requests with the same key may share a unit
        return "batch" if self.batchable(req) else None

    def run_batch(self, reqs):     # results (or Exception instances), one per request
        raise NotImplementedError


class Server:
    """Admission by memory footprint, FIFO with bounded overtaking, `slots`
    concurrent requests.  A request that does not fit may be overtaken by
    later ones that do, but after `max_overtakes` overtakes it blocks the queue
    until it fits (no starvation).  Requests larger than the whole budget are
    rejected."""

    def __init__(self, executor, budget_bytes, slots=8, max_overtakes=16,
                 clock=time.perf_counter, batch_max=64):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.slots = int(slots)
        self.max_overtakes = int(max_overtakes)
        self.clock = clock
        self.batch_max = int(batch_max)
        self.peak_bytes = 0
        self.peak_active = 0
        self.batches = []          # sizes of the batched units that ran

    def run(self, requests):
        reqs = sorted(requests, key=lambda r: (r.arrival, r.id))
        for r in reqs:
            r.footprint = int(self.ex.footprint(r))
        cv = threading.Condition()
        waiting = collections.deque()
        ready = collections.deque()
        state = dict(free=self.budget, active=0, finished=0, stop=False)
        overtaken = collections.Counter()
        t0 = self.clock()

        def worker():
            while True:
                with cv:
                    while not ready and not state["stop"]:
                        cv.wait()
                    if state["stop"] and not ready:
                        return
                    unit = ready.popleft()
                if len(unit) == 1 and not self.ex.batchable(unit[0]):
                    r = unit[0]
                    try:
                        r.result = self.ex.run(r)
                        r.status = "done"
                    except Exception as e:  # the failure is recorded with the request
                        r.status = "failed"
                        r.error = f"{type(e).__name__}: {e}"
                else:
                    try:
                        outs = self.ex.run_batch(unit)
                    except Exception as e:
                        outs = [e] * len(unit)
                    for r, o in zip(unit, outs):
                        if isinstance(o, Exception):
                            r.status = "failed"
                            r.error = f"{type(o).__name__}: {o}"
                        else:
                            r.result = o
                            r.status = "done"
                with cv:
                    now_done = self.clock() - t0
                    for r in unit:
                        r.done = now_done
                        state["free"] += r.footprint
                    state["active"] -= 1
                    state["finished"] += len(unit)
                    cv.notify_all()

        threads = [threading.Thread(target=worker, daemon=True) for _ in range(self.slots)]
        for th in threads:
            th.start()
        i = 0
        total = len(reqs)
        with cv:
            while state["finished"] < total:
                now = self.clock() - t0
                while i < total and reqs[i].arrival <= now:
                    r = reqs[i]
                    i += 1
                    if r.footprint > self.budget:
                        r.status = "rejected"
                        r.error = "footprint exceeds the HBM budget"
                        r.done = r.admitted = now
                        state["finished"] += 1
                    else:
                        waiting.append(r)
                # admission
                blocked = False
                for r in list(waiting):
                    if state["active"] >= self.slots:
                        break
                    if r not in waiting:       # already taken into a batched unit
                        continue
                    if r.footprint <= state["free"] and not blocked:
                        waiting.remove(r)
                        state["free"] -= r.footprint
                        state["active"] += 1
                        unit = [r]
                        key = self.ex.batch_key(r)
                        if key is not None:
                            for q in list(waiting):
                                if len(unit) >= self.batch_max:
                                    break
                                if self.ex.batch_key(q) == key and q.footprint <= state["free"]:
                                    waiting.remove(q)
                                    state["free"] -= q.footprint
                                    unit.append(q)
                            if len(unit) > 1:
                                self.batches.append(len(unit))
                        for u in unit:
                            u.admitted = now
                            u.status = "running"
                        ready.append(unit)
                        for q in waiting:
                            if q.arrival <= r.arrival and q.footprint > r.footprint:
                                overtaken[q.id] += 1
                        cv.notify_all()
                    elif overtaken[r.id] >= self.max_overtakes:
                        blocked = True
                self.peak_active = max(self.peak_active, state["active"])
                self.peak_bytes = max(self.peak_bytes, self.budget - state["free"])
                if state["finished"] >= total:
                    break
                timeout = None
                if i < total:
                    timeout = max(0.0, reqs[i].arrival - (self.clock() - t0))
                cv.wait(timeout=timeout if timeout is None else min(timeout, 0.05))
            state["stop"] = True
            cv.notify_all()
        for th in threads:
            th.join()
        return reqs


def summarize(reqs):
    done = [r for r in reqs if r.status == "done"]
    lat = sorted(r.latency for r in done)

    def pct(q):
        if not lat:
            return math.nan
        k = min(len(lat) - 1, max(0, int(math.ceil(q * len(lat))) - 1))
        return lat[k]
    span = max((r.done for r in done), default=0.0) - min((r.arrival for r in reqs), default=0.0)
    return dict(requests=len(reqs), done=len(done),
                failed=sum(r.status == "failed" for r in reqs),
                rejected=sum(r.status == "rejected" for r in reqs),
                p50_ms=1e3 * pct(0.50), p99_ms=1e3 * pct(0.99),
                mean_ms=1e3 * (sum(lat) / len(lat) if lat else math.nan),
                throughput_rps=len(done) / span if span > 0 else math.nan,
                makespan_s=span)


def make_requests(count=512, seed=2304, rate=None, sizes=None, ns_fraction=0.5, steps=20):
    """Synthetic request mix: sizes drawn uniformly from `sizes`, Poisson solve
    or NS run with equal probability, exponential inter-arrival gaps of mean
    1/rate (all at t = 0 when rate is None)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    sizes = sizes or [(64, 64), (128, 128), (256, 256), (64, 64, 64), (96, 96, 96),
                      (128, 128, 128)]
    t = 0.0
    out = []
    for k in range(count):
        n = tuple(sizes[int(rng.integers(len(sizes)))])
        kind = "ns" if rng.random() < ns_fraction else "poisson"
        if kind == "poisson":
            m = min(n)
            radius = float(rng.uniform(m / 8, m / 4))
        else:
            radius = float(rng.uniform(n[1] / 16, n[1] / 8))
        if rate:
            t += float(rng.exponential(1.0 / rate))
        out.append(Request(id=k, kind=kind, n=n, arrival=t, radius=radius, steps=steps,
                           seed=seed + k))
    return out


class GpuExecutor(Executor):
    """Runs requests through libwl: a Poisson solve (Neumann box, centred
    sphere / circle coefficients, N(0,1) right-hand side drawn on the device,
    FP32 V-cycles with FP64 defect correction) or `steps` Navier-Stokes steps
    of a body in a uniform inflow (Re 250 in 2D, 100 in 3D, mixed-precision
    pressure solves to the request's relative residual, 1e-8 by default).  Results are (fingerprint, stats) pairs; the fingerprint
    is an exact integer hash of the output bits."""

    # Batching limits from measured latencies of one request (MI355X): a
    # Poisson solve takes 1.8-2.1 ms on the whole GPU at every size of the
    # mix and 1.4 / 2.6 / 7.7 / 46 ms as one workgroup of the persistent
    # kernel at 64^2 / 128^2 / 256^2 / 64^3; a 20-step NS run 35 / 41 / 48 ms
    # alone and 49 / 140 / 538 ms in one workgroup at 64^2 / 128^2 / 256^2.
    # Kinds are batched only where one workgroup stays within about 1.5x of
    # the whole-GPU latency.
    def __init__(self, device="cuda", keep_fields=False, batch_cells=16384,
                 ns_batch_cells=4096):
        import torch

        import paper_2304_08159_amd as wl
        self.torch, self.wl = torch, wl
        self.device = device
        self.keep = keep_fields
        self.batch_cells = int(batch_cells)   # Poisson requests up to this size are batched
        self.ns_batch_cells = int(ns_batch_cells)   # NS requests up to this size are batched
        self._tls = threading.local()

    def _stream(self):
        s = getattr(self._tls, "stream", None)
        if s is None:
            s = self.torch.cuda.Stream(device=self.device)
            self._tls.stream = s
        return s

    def _ns_args(self, r):
        d = len(r.n)
        ndim = d
        U = (1.0,) + (0.0,) * (d - 1)
        centre = (r.n[0] / 4.0,) + tuple(m / 2.0 for m in r.n[1:])
        Re = 250.0 if ndim == 2 else 100.0
        nu = 1.0 * 2 * r.radius / Re
        bc_lo = [1] + [3] * (d - 1)
        bc_hi = [2] + [3] * (d - 1)
        return dict(n=r.n, bc_lo=bc_lo, bc_hi=bc_hi, U=U, nu=nu,
                    body=dict(centre=centre, radius=r.radius))

    def batchable(self, r):
        limit = self.batch_cells if r.kind == "poisson" else self.ns_batch_cells
        return math.prod(r.n) <= limit

    def batch_key(self, r):
        return r.kind if self.batchable(r) else None

    def footprint(self, r):
        import ctypes
        from . import _lib
        lib = _lib.load()
        ndim = len(r.n)
        cells = 1
        for m in r.n:
            cells *= m
        nn = (ctypes.c_int * 3)(*(list(r.n) + [1] * (3 - ndim)))
        sz = ctypes.c_size_t()
        if self.batchable(r) and r.kind == "ns":
            a = self._ns_args(r)
            q = _lib.NsRequest()
            q.ndim = ndim
            for i in range(3):
                q.n[i] = nn[i]
                q.bc_lo[i] = (a["bc_lo"] + [3] * 3)[i]
                q.bc_hi[i] = (a["bc_hi"] + [3] * 3)[i]
            q.nu, q.tol, q.steps = a["nu"], r.tol, r.steps
            _lib.fill_body(q.body, a["body"], ndim)
            _lib.check(lib.wl_ns_batch_footprint(ctypes.byref(q), 1, ctypes.byref(sz)))
            return sz.value + cells * (4 * ndim + 8) + 4 * nn[1] * nn[2] + 512
        if self.batchable(r):
            q = _lib.BatchRequest()
            q.ndim = ndim
            for i in range(3):
                q.n[i] = nn[i]
            q.tol, q.max_vcycles, q.mixed = r.tol, 400, 1
            _lib.check(lib.wl_poisson_batch_footprint(ctypes.byref(q), 1, ctypes.byref(sz)))
            return sz.value + 8 * cells * (2 + ndim) + 256
        if r.kind == "poisson":
            per = (ctypes.c_int * 3)(0, 0, 0)
            _lib.check(lib.wl_poisson_footprint(ndim, nn, per, _lib.WL_MIXED, 0, ctypes.byref(sz)))
            return sz.value + 8 * cells * (2 + ndim) + 256
        a = self._ns_args(r)
        d = _lib.SimDesc()
        d.ndim = ndim
        for i in range(3):
            d.n[i] = nn[i]
            d.bc_lo[i] = (a["bc_lo"] + [3] * 3)[i]
            d.bc_hi[i] = (a["bc_hi"] + [3] * 3)[i]
        d.nu, d.prec, d.tol = a["nu"], _lib.WL_MIXED, r.tol
        d.stop_rule = _lib.STOP_RELATIVE
        d.body.kind = 1
        d.body.radius = r.radius
        _lib.check(lib.wl_sim_footprint(ctypes.byref(d), ctypes.byref(sz)))
        return sz.value + 4 * cells * (ndim + 1) + 256

    def _fingerprint(self, t):
        torch = self.torch
        bits = t.contiguous().view(-1).view(torch.int32) if t.dtype == torch.float32 else \
            t.contiguous().view(-1).view(torch.int64)
        w = (torch.arange(bits.numel(), device=bits.device, dtype=torch.int64) % 1000003) + 1
        return int((bits.to(torch.int64) * w).sum().item())

    def _ns_state(self, r):
        """Initial state of an NS request: U on every face (boundary faces at
        their value), the outflow plane at U, p = 0."""
        torch = self.torch
        ndim = len(r.n)
        shape = tuple(reversed(list(r.n) + [1] * (3 - ndim)))
        u = torch.zeros((ndim,) + shape, dtype=torch.float32, device=self.device)
        u[0].fill_(1.0)
        u[0][..., 0] = 1.0          # inflow face
        for i in range(1, ndim):    # walls: zero normal velocity (already zero)
            pass
        uout = torch.ones(shape[:2], dtype=torch.float32, device=self.device)
        p = torch.zeros(shape, dtype=torch.float64, device=self.device)
        return u, uout, p

    def run_ns_batch(self, rs):
        """Small NS requests through one persistent kernel (a whole run per
        workgroup).  With keep_fields the last step runs as a launch of its
        own, so that the state before it is kept for replays (same bits)."""
        torch, wl = self.torch, self.wl
        stream = self._stream()
        with torch.cuda.stream(stream):
            reqs, states = [], []
            for r in rs:
                a = self._ns_args(r)
                u, uout, p = self._ns_state(r)
                reqs.append(dict(n=a["n"], bc_lo=a["bc_lo"], bc_hi=a["bc_hi"], U=a["U"],
                                 nu=a["nu"], body=a["body"], tol=r.tol, max_vcycles=400,
                                 steps=r.steps, u=u, uout=uout, p=p))
                states.append((u, uout, p))
            before = None
            if self.keep:
                first = [dict(q, steps=max(q["steps"] - 1, 0)) for q in reqs]
                res0 = wl.ns_batch_run(first, allow_not_converged=True)
                before = [(u.clone(), o.clone(), p.clone(), t) for (u, o, p), (_, _, t, _)
                          in zip(states, res0)]
                res = wl.ns_batch_run([dict(q, steps=1) for q in reqs], allow_not_converged=True)
                res = [(s1, v0 + v1, t0 + t1, d1) for (s1, v1, t1, d1), (_, v0, t0, _)
                       in zip(res, res0)]
            else:
                res = wl.ns_batch_run(reqs, allow_not_converged=True)
            outs = []
            for k, ((st, vc, t, dt), (u, uout, p)) in enumerate(zip(res, states)):
                if st != 0:
                    outs.append(RuntimeError(f"batched NS run status {st}"))
                    continue
                fp = self._fingerprint(u) * 1000003 + self._fingerprint(p)
                outs.append((fp, dict(vcycles=vc, t=t, dt=dt, batched=True),
                             (u, uout, p, before[k] if before else None) if self.keep else None))
            stream.synchronize()
        return outs

    def run_batch(self, rs):
        """Small Poisson requests (Neumann box, centred sphere / circle, N(0,1)
        right-hand side; FP32 V-cycles with FP64 defect correction) through one
        persistent work-queue kernel; small NS requests through the batched
        NS kernel."""
        if rs and rs[0].kind == "ns":
            return self.run_ns_batch(rs)
        torch, wl = self.torch, self.wl
        stream = self._stream()
        with torch.cuda.stream(stream):
            reqs, keep = [], []
            for r in rs:
                ndim = len(r.n)
                body = dict(centre=tuple(m / 2.0 for m in r.n), radius=r.radius)
                L = wl.body_coeffs(r.n, (False,) * ndim, body, prec=wl.WL_FP64)
                shape = tuple(reversed(list(r.n) + [1] * (3 - ndim)))
                g = torch.Generator(device=self.device)
                g.manual_seed(int(r.seed))
                b = torch.randn(shape, generator=g, dtype=torch.float64, device=self.device)
                x = torch.zeros_like(b)
                reqs.append(dict(n=r.n, periodic=(False,) * ndim, coeffs=L, x=x, b=b, tol=r.tol,
                                 max_vcycles=400, mixed=True))
                keep.append((x, b, L))
            res = wl.poisson_batch_solve(reqs, allow_not_converged=True)
            outs = []
            for (st, k, rel), (x, b, L) in zip(res, keep):
                if st != 0:
                    outs.append(RuntimeError(f"batched Poisson solve status {st} after {k} V-cycles"))
                    continue
                outs.append((self._fingerprint(x), dict(vcycles=k, rel_resid=rel, batched=True),
                             (x, b, L) if self.keep else None))
            stream.synchronize()
        return outs

    def run(self, r):
        if self.batchable(r):
            out = self.run_batch([r])[0]
            if isinstance(out, Exception):
                raise out
            return out
        torch, wl = self.torch, self.wl
        stream = self._stream()
        with torch.cuda.stream(stream):
            ndim = len(r.n)
            if r.kind == "poisson":
                body = dict(centre=tuple(m / 2.0 for m in r.n), radius=r.radius)
                L = wl.body_coeffs(r.n, (False,) * ndim, body, prec=wl.WL_MIXED)
                shape = tuple(reversed(list(r.n) + [1] * (3 - ndim)))
                g = torch.Generator(device=self.device)
                g.manual_seed(int(r.seed))
                b = torch.randn(shape, generator=g, dtype=torch.float64, device=self.device)
                x = torch.zeros_like(b)
                ps = wl.Poisson(r.n, (False,) * ndim, prec=wl.WL_MIXED)
                k, rel = ps.solve(L, x, b, tol=r.tol, max_vcycles=400)
                ps.close()
                fp = self._fingerprint(x)
                stats = dict(vcycles=k, rel_resid=rel)
                out = (fp, stats, (x, b, L) if self.keep else None)
            else:
                a = self._ns_args(r)
                sim = wl.Sim(a["n"], a["bc_lo"], a["bc_hi"], a["U"], a["nu"], body=a["body"],
                             prec=wl.WL_MIXED, tol=r.tol, stop_rule=wl.STOP_RELATIVE,
                             max_vcycles=400)
                vc = 0
                for _ in range(r.steps):
                    st = sim.step()
                    vc += st["vcycles"][0] + st["vcycles"][1]
                u = sim.velocity()
                p = sim.pressure()
                fp = self._fingerprint(torch.stack(u + [p]))
                out = (fp, dict(vcycles=vc, t=st["t"]), (u, p) if self.keep else None)
                sim.close()
            stream.synchronize()
        return out
