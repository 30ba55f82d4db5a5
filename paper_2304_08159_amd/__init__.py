"""MI355X (gfx950) hot path of a WaterLily-style incompressible NS solver.

Python face of libwl (include/wl.h): torch supplies device memory (the
workspace and field tensors) and the HIP stream; every step of the method
runs in the HIP kernels of libwl.so.  Field tensors use the library layout,
shape (n2, n1, n0) contiguous (x fastest), dtype float32 for WL_FP32 /
WL_MIXED simulations and float64 for WL_FP64.

Paper: Weymouth & Font, arXiv 2304.08159 (Sec. 2: method; Sec. 3: simstep!
and its routines).
"""

import ctypes

from . import _lib
from ._lib import (FIELD_L0, FIELD_MU0_0, FIELD_MU1N, FIELD_P, FIELD_SIGMA, FIELD_U0,  # noqa: F401
                   FIELD_UOUT, INFLOW, OUTFLOW, PERIODIC, STOP_DIVERGENCE, STOP_RELATIVE, WALL,
                   WL_FP32, WL_FP64, WL_MIXED, WlError, check, load)

__all__ = ["Sim", "Poisson", "body_coeffs", "set_graphs", "set_fused_sweeps", "set_smoother",
           "poisson_batch_solve", "ns_batch_run", "ns_batch_footprint", "load", "WlError", "WL_FP32", "WL_FP64", "WL_MIXED",
           "PERIODIC", "INFLOW", "OUTFLOW", "WALL", "STOP_DIVERGENCE", "STOP_RELATIVE"]


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("libwl needs a ROCm GPU (torch.cuda.is_available() is False)")
    return torch


def _stream(torch):
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _workspace(torch, nbytes, device):
    # 256-byte aligned byte buffer owned by torch
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-ws.data_ptr()) % 256
    return ws, ctypes.c_void_p(ws.data_ptr() + off), nbytes


class Sim:
    """One Navier-Stokes configuration resident on the GPU (wl_sim)."""

    def __init__(self, n, bc_lo, bc_hi, U, nu, body=None, prec=WL_FP32, levels=0, tol=1e-5,
                 max_vcycles=100, inner_vcycles=3, cfl=0.5, eps=1.0, tape_steps=0,
                 stop_rule=STOP_DIVERGENCE, device="cuda"):
        torch = _torch()
        lib = load()
        n = tuple(int(m) for m in n)
        ndim = len(n)
        d = _lib.SimDesc()
        d.ndim = ndim
        nn = list(n) + [1] * (3 - ndim)
        bl = list(bc_lo) + [WALL] * (3 - ndim)
        bh = list(bc_hi) + [WALL] * (3 - ndim)
        Uv = list(U) + [0.0] * (3 - ndim)
        for i in range(3):
            d.n[i], d.bc_lo[i], d.bc_hi[i], d.U[i] = nn[i], bl[i], bh[i], float(Uv[i])
        d.nu = float(nu)
        if body is not None:
            _lib.fill_body(d.body, body, ndim, eps)
        d.prec, d.mg_levels, d.tol = int(prec), int(levels), float(tol)
        d.max_vcycles, d.inner_vcycles, d.cfl = int(max_vcycles), int(inner_vcycles), float(cfl)
        d.tape_steps = int(tape_steps)
        d.stop_rule = int(stop_rule)
        nbytes = ctypes.c_size_t()
        check(lib.wl_sim_footprint(ctypes.byref(d), ctypes.byref(nbytes)))
        self.footprint = nbytes.value
        self._ws, wptr, wlen = _workspace(torch, nbytes.value, device)
        h = ctypes.c_void_p()
        check(lib.wl_sim_create(ctypes.byref(d), wptr, wlen, _stream(torch), ctypes.byref(h)))
        self._h = h
        self._lib = lib
        self.desc = d
        self.n = n
        self.ndim = ndim
        self.shape = (nn[2], nn[1], nn[0])
        self.dtype = torch.float64 if prec == WL_FP64 else torch.float32
        self.device = device

    def close(self):
        if getattr(self, "_h", None):
            self._lib.wl_sim_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _field_shape(self, field):
        if field == FIELD_UOUT:
            return (self.shape[0], self.shape[1])
        return self.shape

    def get(self, field):
        torch = _torch()
        t = torch.empty(self._field_shape(field), dtype=self.dtype, device=self.device)
        check(self._lib.wl_get_field(self._h, int(field), _ptr(t)))
        return t

    def set(self, field, value):
        torch = _torch()
        t = value.to(device=self.device, dtype=self.dtype).contiguous()
        if tuple(t.shape) != self._field_shape(field):
            raise ValueError(f"field shape {tuple(t.shape)} != {self._field_shape(field)}")
        check(self._lib.wl_set_field(self._h, int(field), _ptr(t)))
        torch.cuda.current_stream().synchronize()

    def velocity(self):
        return [self.get(FIELD_U0 + i) for i in range(self.ndim)]

    def pressure(self):
        return self.get(FIELD_P)

    def set_time(self, t):
        check(self._lib.wl_set_time(self._h, float(t)))

    @property
    def has_outflow(self):
        return self.desc.bc_hi[0] == OUTFLOW

    def state_size(self):
        cells = self.shape[0] * self.shape[1] * self.shape[2]
        return self.ndim * cells + (self.shape[0] * self.shape[1] if self.has_outflow else 0)

    def get_flow(self):
        """Velocity components and outflow plane as one flat tensor (the
        layout of the adjoint state that step_adjoint takes and returns)."""
        torch = _torch()
        parts = [t.reshape(-1) for t in self.velocity()]
        if self.has_outflow:
            parts.append(self.get(FIELD_UOUT).reshape(-1))
        return torch.cat(parts)

    def set_flow(self, vec, p=None):
        cells = self.shape[0] * self.shape[1] * self.shape[2]
        for i in range(self.ndim):
            self.set(FIELD_U0 + i, vec[i * cells:(i + 1) * cells].reshape(self.shape))
        if self.has_outflow:
            self.set(FIELD_UOUT, vec[self.ndim * cells:].reshape(self.shape[0], self.shape[1]))
        if p is not None:
            self.set(FIELD_P, p)

    def get_state(self):
        """Snapshot of everything later steps read (wl_get_state): velocity,
        outflow plane, pressure (and its FP64 iterate), time and the next dt,
        in a device byte tensor (a view into a 256-byte aligned buffer)."""
        torch = _torch()
        nb = ctypes.c_size_t()
        check(self._lib.wl_state_size(self._h, ctypes.byref(nb)))
        buf, ptr, _ = _workspace(torch, nb.value, self.device)
        check(self._lib.wl_get_state(self._h, ptr))
        off = ptr.value - buf.data_ptr()
        return buf[off:off + nb.value]

    def set_state(self, snap):
        """Restore a snapshot taken by get_state (wl_set_state)."""
        torch = _torch()
        nb = ctypes.c_size_t()
        check(self._lib.wl_state_size(self._h, ctypes.byref(nb)))
        if snap.dtype != torch.uint8 or snap.numel() != nb.value or not snap.is_cuda:
            raise ValueError("not a snapshot of this simulation")
        if snap.data_ptr() % 256:
            buf, ptr, _ = _workspace(torch, nb.value, self.device)
            off = ptr.value - buf.data_ptr()
            buf[off:off + nb.value].copy_(snap)
            snap = buf[off:off + nb.value]
        check(self._lib.wl_set_state(self._h, _ptr(snap)))

    def drag(self):
        F = ctypes.c_double()
        check(self._lib.wl_drag(self._h, ctypes.byref(F)))
        return F.value

    def tape(self, on=True):
        check(self._lib.wl_tape_record(self._h, int(bool(on))))

    def step_adjoint(self, ubar, drag_weight=0.0, pbar=None):
        """Reverse the last recorded step: returns (adjoint of the state before
        it, dJ/d(radius, cx, cy, cz) contributed by this step).  ubar: adjoint
        of the state after it (get_flow layout); pbar: adjoint of the pressure
        after it (None = zero)."""
        torch = _torch()
        ubar = ubar.to(device=self.device, dtype=self.dtype).contiguous()
        if ubar.numel() != self.state_size():
            raise ValueError("adjoint state has the wrong size")
        pptr = ctypes.c_void_p()
        if pbar is not None:
            pbar = pbar.to(device=self.device, dtype=self.dtype).contiguous()
            if tuple(pbar.shape) != self.shape:
                raise ValueError("pressure adjoint has the wrong shape")
            pptr = _ptr(pbar)
        out = torch.empty_like(ubar)
        g = (ctypes.c_double * 4)(0.0, 0.0, 0.0, 0.0)
        check(self._lib.wl_step_adjoint(self._h, _ptr(ubar), pptr, float(drag_weight), _ptr(out),
                                        g))
        return out, [g[0], g[1], g[2], g[3]]

    @staticmethod
    def _stats(st):
        return dict(dt=st.dt, t=st.t, vcycles=(st.vcycles[0], st.vcycles[1]),
                    resid=(st.resid[0], st.resid[1]),
                    rel_resid=(st.rel_resid[0], st.rel_resid[1]))

    def step(self, dt=0.0, allow_not_converged=False):
        st = _lib.StepStats()
        check(self._lib.wl_step(self._h, float(dt), ctypes.byref(st)),
              allow=(-3,) if allow_not_converged else ())
        return self._stats(st)

    def run(self, nsteps, t_end=0.0, allow_not_converged=False):
        """Up to nsteps CFL-adaptive steps in one library call, stopping once
        the time reaches t_end (> 0); returns the per-step stats."""
        sts = (_lib.StepStats * max(int(nsteps), 1))()
        taken = ctypes.c_int(0)
        check(self._lib.wl_run(self._h, int(nsteps), float(t_end), sts, ctypes.byref(taken)),
              allow=(-3,) if allow_not_converged else ())
        return [self._stats(sts[k]) for k in range(taken.value)]


def poisson_batch_solve(requests, allow_not_converged=False):
    """Solve many small Poisson problems with one persistent kernel.

    requests: list of dicts with n (2 or 3 ints), periodic, coeffs (float64
    tensor (ndim, n2, n1, n0)), x (float64, guess in / solution out), b
    (float64), tol (relative, default 1e-8), max_vcycles (default 200),
    mixed (FP32 V-cycles with FP64 defect correction; default FP64).
    Returns a list of (status, vcycles, rel_resid)."""
    torch = _torch()
    lib = load()
    count = len(requests)
    if count == 0:
        return []
    arr = (_lib.BatchRequest * count)()
    dev = None
    for q, r in enumerate(requests):
        n = [int(m) for m in r["n"]]
        ndim = len(n)
        per = [int(bool(p)) for p in r.get("periodic", (False,) * ndim)]
        for t in ("coeffs", "x", "b"):
            ten = r[t]
            if ten.dtype != torch.float64 or not ten.is_cuda or not ten.is_contiguous():
                raise ValueError(f"request {q}: {t} must be a contiguous float64 CUDA tensor")
            dev = ten.device
        a = arr[q]
        a.ndim = ndim
        for i in range(3):
            a.n[i] = (n + [1] * (3 - ndim))[i]
            a.periodic[i] = (per + [0] * (3 - ndim))[i]
        a.coeffs = r["coeffs"].data_ptr()
        a.x = r["x"].data_ptr()
        a.b = r["b"].data_ptr()
        a.tol = float(r.get("tol", 1e-8))
        a.max_vcycles = int(r.get("max_vcycles", 200))
        a.mixed = int(bool(r.get("mixed", False)))
    nbytes = ctypes.c_size_t()
    check(lib.wl_poisson_batch_footprint(arr, count, ctypes.byref(nbytes)))
    ws, ptr, nb = _workspace(torch, nbytes.value, dev)
    res = (_lib.BatchResult * count)()
    allow = (-3,) if allow_not_converged else ()
    check(lib.wl_poisson_batch_solve(arr, count, ptr, nb, _stream(torch), res), allow=allow)
    del ws
    return [(res[q].status, res[q].vcycles, res[q].rel_resid) for q in range(count)]


def _ns_request(r, q):
    """Fill an NsRequest from a dict (see ns_batch_run)."""
    torch = _torch()
    n = [int(m) for m in r["n"]]
    ndim = len(n)
    q.ndim = ndim
    bl = list(r["bc_lo"]) + [WALL] * (3 - ndim)
    bh = list(r["bc_hi"]) + [WALL] * (3 - ndim)
    Uv = list(r.get("U", (0.0,) * ndim)) + [0.0] * (3 - ndim)
    for i in range(3):
        q.n[i] = (n + [1] * (3 - ndim))[i]
        q.bc_lo[i], q.bc_hi[i], q.U[i] = int(bl[i]), int(bh[i]), float(Uv[i])
    q.nu = float(r["nu"])
    if r.get("body") is not None:
        _lib.fill_body(q.body, r["body"], ndim)
    q.tol = float(r.get("tol", 1e-8))
    q.max_vcycles = int(r.get("max_vcycles", 100))
    q.steps = int(r["steps"])
    q.cfl = float(r.get("cfl", 0.5))
    for t, dt in (("u", torch.float32), ("p", torch.float64)):
        ten = r[t]
        if ten.dtype != dt or not ten.is_cuda or not ten.is_contiguous():
            raise ValueError(f"{t} must be a contiguous {dt} CUDA tensor")
    q.u = r["u"].data_ptr()
    q.p = r["p"].data_ptr()
    q.uout = r["uout"].data_ptr() if r.get("uout") is not None else None


def ns_batch_footprint(requests):
    lib = load()
    arr = (_lib.NsRequest * max(len(requests), 1))()
    for q, r in enumerate(requests):
        _ns_request(r, arr[q])
    nb = ctypes.c_size_t()
    check(lib.wl_ns_batch_footprint(arr, len(requests), ctypes.byref(nb)))
    return nb.value


def ns_batch_run(requests, allow_not_converged=False):
    """Run many small simulations with one persistent kernel (FP32 fields,
    mixed-precision solves to a relative residual).

    requests: list of dicts with n, bc_lo, bc_hi, U, nu, body (at rest; may be
    None), tol (default 1e-8), max_vcycles, steps, cfl, and the state tensors
    u (float32, (ndim, n2, n1, n0), in/out), uout (float32 (n2, n1) for an
    OUTFLOW run, in/out) and p (float64 (n2, n1, n0), in/out).  Returns a list
    of (status, vcycles, t, last dt)."""
    torch = _torch()
    lib = load()
    count = len(requests)
    if count == 0:
        return []
    arr = (_lib.NsRequest * count)()
    for q, r in enumerate(requests):
        _ns_request(r, arr[q])
    nb = ctypes.c_size_t()
    check(lib.wl_ns_batch_footprint(arr, count, ctypes.byref(nb)))
    ws, ptr, n = _workspace(torch, nb.value, requests[0]["u"].device)
    res = (_lib.NsResult * count)()
    allow = (-3,) if allow_not_converged else ()
    check(lib.wl_ns_batch_run(arr, count, ptr, n, _stream(torch), res), allow=allow)
    del ws
    return [(res[q].status, res[q].vcycles, res[q].t, res[q].dt) for q in range(count)]


def set_graphs(enable=True):
    """Replay repeated solve bodies as captured HIP graphs (default) or launch
    every kernel individually; results are bitwise the same."""
    check(load().wl_set_graphs(1 if enable else 0))


def set_fused_sweeps(mode=1):
    """Fused pre/post-smoothing sweep pairs on uniform periodic 3D levels:
    0 off, 1 (default) or 2 on every eligible level.  Taken by solvers and
    simulations created afterwards; iterates are bitwise the same in every
    mode."""
    check(load().wl_set_fused_sweeps(int(mode)))


def set_smoother(kind="jacobi"):
    """Smoother of the multigrid levels for solvers and simulations created
    afterwards: "jacobi" (damped Jacobi, default) or "cg" (the paper's
    conjugate-gradient smoothing)."""
    kinds = {"jacobi": _lib.SMOOTH_JACOBI, "cg": _lib.SMOOTH_CG}
    if kind not in kinds:
        raise ValueError("smoother must be 'jacobi' or 'cg'")
    check(load().wl_set_smoother(kinds[kind]))


def body_coeffs(n, periodic, body=None, prec=WL_FP32, device="cuda"):
    """BDIM Poisson coefficients of a sphere/circle or torus body: tensor (ndim, n2, n1, n0)."""
    torch = _torch()
    lib = load()
    n = tuple(int(m) for m in n)
    ndim = len(n)
    nn = (ctypes.c_int * 3)(*(list(n) + [1] * (3 - ndim)))
    per = (ctypes.c_int * 3)(*([int(bool(p)) for p in periodic] + [0] * (3 - ndim)))
    b = _lib.Body()
    if body is not None:
        _lib.fill_body(b, body, ndim)
    dtype = torch.float32 if prec == WL_FP32 else torch.float64
    L = torch.empty((ndim, nn[2], nn[1], nn[0]), dtype=dtype, device=device)
    check(lib.wl_body_coeffs(ctypes.byref(b), ndim, nn, per, int(prec), _ptr(L), _stream(torch)))
    return L


class Poisson:
    """Standalone GMG pressure solver (wl_poisson)."""

    def __init__(self, n, periodic, prec=WL_FP32, levels=0, device="cuda"):
        torch = _torch()
        lib = load()
        n = tuple(int(m) for m in n)
        ndim = len(n)
        nn = (ctypes.c_int * 3)(*(list(n) + [1] * (3 - ndim)))
        per = (ctypes.c_int * 3)(*([int(bool(p)) for p in periodic] + [0] * (3 - ndim)))
        nbytes = ctypes.c_size_t()
        check(lib.wl_poisson_footprint(ndim, nn, per, int(prec), int(levels), ctypes.byref(nbytes)))
        self.footprint = nbytes.value
        self._ws, wptr, wlen = _workspace(torch, nbytes.value, device)
        h = ctypes.c_void_p()
        check(lib.wl_poisson_create(ndim, nn, per, int(prec), int(levels), wptr, wlen,
                                    _stream(torch), ctypes.byref(h)))
        self._h = h
        self._lib = lib
        self.ndim = ndim
        self.shape = (nn[2], nn[1], nn[0])
        self.prec = prec
        self.dtype = torch.float32 if prec == WL_FP32 else torch.float64

    def close(self):
        if getattr(self, "_h", None):
            self._lib.wl_poisson_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, coeffs, x, b, tol=1e-8, max_vcycles=100, allow_not_converged=False):
        """coeffs: tensor (ndim, n2, n1, n0) or None (reuse); x: initial guess,
        overwritten with the solution; b: right-hand side.  Returns
        (vcycles, relative residual)."""
        for t in (x, b) + ((coeffs,) if coeffs is not None else ()):
            if t.dtype != self.dtype or not t.is_contiguous() or not t.is_cuda:
                raise ValueError(f"tensors must be contiguous {self.dtype} on the GPU")
        if tuple(x.shape) != self.shape or tuple(b.shape) != self.shape:
            raise ValueError("x / b shape mismatch")
        if coeffs is not None and tuple(coeffs.shape) != (self.ndim,) + self.shape:
            raise ValueError("coeffs shape mismatch")
        vc = ctypes.c_int()
        rel = ctypes.c_double()
        cptr = _ptr(coeffs) if coeffs is not None else ctypes.c_void_p()
        check(self._lib.wl_poisson_solve(self._h, cptr, _ptr(x), _ptr(b), float(tol),
                                         int(max_vcycles), ctypes.byref(vc), ctypes.byref(rel)),
              allow=(-3,) if allow_not_converged else ())
        return vc.value, rel.value
