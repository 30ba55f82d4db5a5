"""Time-averaged pressure drag of a rollout and its gradient with respect to
the body (radius and centre) through the hand-written adjoint of the step.

J = sum_n dt_n F_x^n / sum_n dt_n with F_x^n the drag after step n.  The
forward run keeps checkpoints (wl_get_state snapshots: velocity, outflow
plane, pressure, time) every
`checkpoint` steps and the dt sequence; the reverse pass restores each
segment's checkpoint, re-runs it with the tape recording (same dt sequence),
and reverses its steps with wl_step_adjoint.  dt is frozen (the gradient of
the CFL rule is not taken), matching finite differences that replay the same
dt sequence.
"""

import torch

import paper_2304_08159_amd as wl


class Rollout:
    """A body-in-a-stream configuration whose drag can be differentiated."""

    def __init__(self, n, bc_lo, bc_hi, U, nu, centre, radius, prec=wl.WL_MIXED, tol=1e-8,
                 checkpoint=10, levels=0, max_vcycles=200, init=None):
        self.kw = dict(n=n, bc_lo=bc_lo, bc_hi=bc_hi, U=U, nu=nu, prec=prec, tol=tol,
                       levels=levels, max_vcycles=max_vcycles)
        self.base_centre = tuple(float(c) for c in centre)
        self.base_radius = float(radius)
        self.checkpoint = int(checkpoint)
        # initial flow (Sim.get_flow layout; None: the uniform stream U)
        self.init = init

    def make(self, params, tape_steps=0):
        r, cx, cy, cz = [float(v) for v in params]
        centre = (cx, cy, cz)[:len(self.kw["n"])]
        sim = wl.Sim(self.kw["n"], self.kw["bc_lo"], self.kw["bc_hi"], self.kw["U"], self.kw["nu"],
                     body=dict(centre=centre, radius=r), prec=self.kw["prec"],
                     tol=self.kw["tol"], levels=self.kw["levels"],
                     max_vcycles=self.kw["max_vcycles"], tape_steps=tape_steps)
        if self.init is not None:
            sim.set_flow(self.init)
        return sim

    def forward(self, params, nsteps, dts=None, keep=True):
        """Returns (J, dts, checkpoints, sim)."""
        sim = self.make(params, tape_steps=self.checkpoint if keep else 0)
        cps = {}
        used = []
        num = 0.0
        for k in range(nsteps):
            if keep and k % self.checkpoint == 0:
                cps[k] = sim.get_state()
            st = sim.step(dts[k] if dts is not None else 0.0, allow_not_converged=True)
            used.append(st["dt"])
            num += st["dt"] * sim.drag()
        J = num / sum(used)
        return J, used, cps, sim

    def gradient(self, params, nsteps):
        """J and dJ/d(radius, cx, cy, cz) by the checkpointed adjoint."""
        J, dts, cps, sim = self.forward(params, nsteps)
        g = self.reverse(sim, cps, dts)
        sim.close()
        return J, g, dts

    def reverse(self, sim, cps, dts):
        """dJ/d(radius, cx, cy, cz) from a forward run's checkpoints and dt
        sequence: segments are re-run with the tape on and reversed step by
        step, last segment first."""
        nsteps = len(dts)
        T = sum(dts)
        ubar = torch.zeros(sim.state_size(), dtype=sim.dtype, device=sim.device)
        g = [0.0, 0.0, 0.0, 0.0]
        starts = sorted(cps)
        for s0 in reversed(starts):
            s1 = min(s0 + self.checkpoint, nsteps)
            sim.set_state(cps[s0])
            sim.tape(True)
            for k in range(s0, s1):
                sim.step(dts[k], allow_not_converged=True)
            sim.tape(False)
            for k in reversed(range(s0, s1)):
                ubar, gk = sim.step_adjoint(ubar, drag_weight=dts[k] / T)
                g = [a + b for a, b in zip(g, gk)]
        return g

    def fd_gradient(self, params, nsteps, dts, h=1e-3, which=(0, 1, 2, 3)):
        g = [0.0, 0.0, 0.0, 0.0]
        for q in which:
            pp = list(params)
            pm = list(params)
            pp[q] += h
            pm[q] -= h
            Jp = self.forward(pp, nsteps, dts=dts, keep=False)[0]
            Jm = self.forward(pm, nsteps, dts=dts, keep=False)[0]
            g[q] = (Jp - Jm) / (2 * h)
        return g


class DragRolloutFn(torch.autograd.Function):
    """torch.autograd.Function: params (4,) tensor (radius, centre) -> J.

    forward runs the rollout and keeps its checkpoints, dt sequence and the
    simulation; backward runs the checkpointed reverse pass and frees them."""

    @staticmethod
    def forward(ctx, params, rollout, nsteps):
        J, dts, cps, sim = rollout.forward(params.detach().cpu().tolist(), nsteps)
        ctx.rollout, ctx.sim, ctx.cps, ctx.dts = rollout, sim, cps, dts
        return torch.tensor(J, dtype=params.dtype, device=params.device)

    @staticmethod
    def backward(ctx, gJ):
        g = ctx.rollout.reverse(ctx.sim, ctx.cps, ctx.dts)
        ctx.sim.close()
        ctx.sim = ctx.cps = None
        return gJ * torch.tensor(g, dtype=gJ.dtype, device=gJ.device), None, None
