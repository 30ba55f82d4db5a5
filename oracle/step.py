"""Projection and the Heun time step: the simstep! analogue (oracle; test-only).

Paper, Sec. 2: the pressure gradient is applied to the velocity by
    u[I,i] -= coeff[I,i] * (p[I] - p[I - del(i)])   for every direction i,
and the pressure comes from the BDIM-modified Poisson system solved by GMG.
Sec. 3 times simstep!, made of convdiff!, BDIM!, BC!, project! and CFL!.

READINGS (the paper gives neither the stage order nor the scaling):
  * projection with factor c:  sigma = div(u*) / (c dt),  A p = sigma,
    u = u* - c dt L grad(p), i.e. coeff = c dt L and p is the physical
    pressure, so warm starts across stages share one scale;
  * Heun / SSP-RK2 with a projection per stage:
      u1      = P_1   B[ u^n + dt R(u^n) ]
      u^{n+1} = P_1/2 B[ (u^n + u1 + dt R(u1)) / 2 ]
    with B = boundary rules after the BDIM blend, P_c the projection;
  * dt from the CFL rule on u^n, held for both stages; p warm-started from the
    previous solve (zero at t = 0);
  * each stage's pressure solve stops (stop_rule "divergence", the default)
    once the divergence it leaves in the projected velocity,
    c dt (sigma - A p), has RMS over the active cells <= tol (velocity per
    cell, grid units).  For FP32 fields a relative residual cannot serve:
    the FP32 rounding of a smooth pressure alone floors ||b - A p|| / ||b||
    at ~1.4e-5 (128^3) and ~6e-5 (256^3) for the Taylor-Green pressure, while
    the divergence it leaves stays at the velocity's own rounding level.
    stop_rule "relative" stops once ||b - A p|| <= tol ||b|| (the residual
    the 2D configuration states, 1e-8, for FP64 fields).

Pins: divergence identity div(u) = c dt (sigma - A p) for any p, max |div u|
<= 1e-10 after a tight solve, idempotence of the projection, discretely
divergence-free 3D Taylor-Green initial field, 2D Taylor-Green decay against
its closed form, mirror symmetry of the cylinder flow.
"""

import numpy as np

from . import geometry, momentum, poisson
from .grid import OUTFLOW, PERIODIC, auto_levels, shift


def divergence(u, uout, bc_lo, bc_hi, U):
    d = len(u)
    n = u[0].shape
    Pd = momentum.pad_velocity(u, uout, bc_lo, bc_hi, U)
    div = np.zeros(n)
    for i in range(d):
        di = [1 if a == i else 0 for a in range(d)]
        div += momentum._view(Pd[i], n, di) - u[i]
    return div


def grad_update(u, p, L, per, coef):
    """u_i(I) -= coef * L_i(I) * (p(I) - p(I - delta_i)) for every i."""
    return [u[i] - coef * L[i] * (p - shift(p, i, -1, per[i])) for i in range(len(u))]


def drag(sim):
    """Pressure drag of the body from the current pressure.

    READING (the paper defines no force): the kernel-smoothed surface integral
    of the pressure, F_x = -sum over active cells of (p - mean p) n_x K(d) at
    cell centres, with K the BDIM kernel and n the SDF gradient; the active
    mean makes it independent of the pressure's free constant.
    """
    if sim.body is None:
        return 0.0
    X = geometry.cell_centres(sim.n)
    body = geometry.body_at(sim.body, sim.t)
    dist, normal = geometry.sphere_sdf(X, body["centre"], body["radius"])
    w = normal[0] * geometry.kernel(dist)
    act = sim.h.active[0]
    p = sim.p[act]
    return float(-np.sum((p - p.mean()) * w[act]))


class Sim:
    """FP64 reference of one NS configuration (uniform grid, optional body,
    at rest or in rigid motion)."""

    def __init__(self, n, bc_lo, bc_hi, U, nu, body=None, cfl=0.5, tol=1e-8,
                 max_vcycles=100, levels=0, eps=1.0, stop_rule="divergence",
                 smoother="jacobi"):
        if stop_rule not in ("divergence", "relative"):
            raise ValueError("stop_rule must be 'divergence' or 'relative'")
        self.stop_rule = stop_rule
        self.n = tuple(n)
        self.d = len(n)
        self.bc_lo, self.bc_hi = list(bc_lo), list(bc_hi)
        self.U = [float(x) for x in U]
        self.nu, self.cfl, self.tol, self.max_vcycles = nu, cfl, tol, max_vcycles
        self.body = body
        self.per = [b == PERIODIC for b in bc_lo]
        self.eps, self.nlev, self.smoother = eps, auto_levels(self.n, levels), smoother
        self.moving = geometry.is_moving(body)
        self.Vb = self.G = None
        self._measure(0.0)
        self.u = [np.full(self.n, self.U[i]) for i in range(self.d)]
        self._set_boundary(self.u)
        self.uout = np.full(self.n[1:], self.U[0]) if bc_hi[0] == OUTFLOW else None
        self.p = np.zeros(self.n)
        self.t = 0.0

    def _measure(self, t):
        """BDIM moments, coefficients and hierarchy of the body where it is at
        time t (moving bodies are re-measured every step, at the time the
        step's stages advance to), and its velocity at the faces."""
        self.mu0, self.mu1n, self.L = geometry.measure(self.n, self.bc_lo, self.body, self.eps, t)
        self.h = poisson.Hierarchy(self.L, self.nlev, self.per, self.smoother)
        if self.moving:
            self.Vb = [geometry.body_velocity(geometry.face_centres(self.n, i), self.body, t)[i]
                       for i in range(self.d)]
            self.G = geometry.body_velocity_gradient(self.body, self.d)

    def _set_boundary(self, u):
        for i in range(self.d):
            m = momentum.boundary_face_mask(self.n, self.bc_lo, i)
            u[i][m] = momentum.boundary_value(self.bc_lo, self.U, i)
        return u

    def dt_cfl(self):
        return momentum.cfl_dt(self.u, self.uout, self.bc_lo, self.bc_hi, self.U,
                               self.nu, self.cfl)

    def stage(self, c, dt, u_n, out_n, u_e, out_e, force_vcycles=None):
        """One projected stage; returns (u, uout, p, vcycles, resid_history)."""
        R, Rout = momentum.rhs(u_e, out_e, self.bc_lo, self.bc_hi, self.U, self.nu)
        if c == 1.0:
            f = [u_n[i] + dt * R[i] for i in range(self.d)]
            fout = None if Rout is None else out_n + dt * Rout
        else:
            f = [0.5 * (u_n[i] + u_e[i] + dt * R[i]) for i in range(self.d)]
            fout = None if Rout is None else 0.5 * (out_n + out_e + dt * Rout)
        if self.body is not None:
            f = momentum.bdim(f, self.mu0, self.mu1n, self.bc_lo, self.bc_hi, self.U, fout,
                              self.Vb, self.G)
        f = self._set_boundary(f)
        fout = momentum.exit_flux_correct(f, fout, self.bc_lo, self.bc_hi)
        sigma = divergence(f, fout, self.bc_lo, self.bc_hi, self.U) / (c * dt)
        if self.stop_rule == "relative":
            rtol, atol = self.tol, 0.0
        else:
            n_active = int(self.h.active[0].sum())
            rtol, atol = 0.0, self.tol * np.sqrt(n_active) / (c * dt)
        p, k, hist, _ = poisson.solve(self.h, sigma, x0=self.p, tol=rtol, atol=atol,
                                      max_vcycles=self.max_vcycles,
                                      force_vcycles=force_vcycles)
        u = grad_update(f, p, self.L, self.per, c * dt)
        return u, fout, p, k, hist

    def step(self, dt=None, force_vcycles=(None, None)):
        if dt is None or dt <= 0.0:
            dt = self.dt_cfl()
        if self.moving:
            # both stages advance to t + dt: the body is placed there
            self._measure(self.t + dt)
        u1, o1, p1, k1, h1 = self.stage(1.0, dt, self.u, self.uout, self.u, self.uout,
                                        force_vcycles[0])
        self.p = p1
        u2, o2, p2, k2, h2 = self.stage(0.5, dt, self.u, self.uout, u1, o1,
                                        force_vcycles[1])
        self.u, self.uout, self.p = u2, o2, p2
        self.t += dt
        return dict(dt=dt, vcycles=(k1, k2), resid=(h1, h2))
