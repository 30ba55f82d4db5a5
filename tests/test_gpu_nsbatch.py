"""Batched small Navier-Stokes runs (one persistent kernel, one workgroup per
request): per-step replay against the FP64 oracle, results independent of
the batch, and argument checks."""

import math

import numpy as np
import pytest

import workloads as W
from oracle import momentum as M
from oracle import poisson as P
from oracle import step as S
from tests.gpu_util import mean_free, plane_to_oracle, rel_l2, to_device, to_oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CASES = {
    "cylinder-2d": dict(n=(64, 32), bc_lo=[1, 3], bc_hi=[2, 3], U=(1.0, 0.0), nu=0.04,
                        body=dict(centre=(16.0, 16.3), radius=4.0)),
    "sphere-3d": dict(n=(48, 24, 24), bc_lo=[1, 3, 3], bc_hi=[2, 3, 3], U=(1.0, 0.0, 0.0),
                      nu=0.06, body=dict(centre=(12.0, 12.2, 11.9), radius=3.5)),
    "tgv-2d-periodic": dict(n=(48, 48), bc_lo=[0, 0], bc_hi=[0, 0], U=(0.0, 0.0), nu=0.01,
                            body=None),
}


def _state(cfg):
    """Initial state: U on every face (boundary faces at their value), p = 0;
    the periodic case starts from the 2D Taylor-Green vortex."""
    n, d = cfg["n"], len(cfg["n"])
    shape = tuple(reversed(list(n) + [1] * (3 - d)))
    if cfg["body"] is None:
        u, v, _, _ = W.tgv2d(n[0], 0.01)
        comps = [u, v]
    else:
        comps = [np.full(n, cfg["U"][i]) for i in range(d)]
        for i in range(d):
            if cfg["bc_lo"][i] != 0:
                idx = [slice(None)] * d
                idx[i] = 0
                comps[i][tuple(idx)] = cfg["U"][i] if cfg["bc_lo"][i] == 1 else 0.0
    u = torch.stack([to_device(a, d, torch, torch.float32) for a in comps]).contiguous()
    p = torch.zeros(shape, dtype=torch.float64, device="cuda")
    uout = None
    if cfg["bc_hi"][0] == 2:
        pl = (shape[0], shape[1])
        uout = torch.full(pl, cfg["U"][0], dtype=torch.float32, device="cuda")
    return u, uout, p


def _req(cfg, u, uout, p, steps, tol=1e-9):
    return dict(n=cfg["n"], bc_lo=cfg["bc_lo"], bc_hi=cfg["bc_hi"], U=cfg["U"], nu=cfg["nu"],
                body=cfg["body"], tol=tol, max_vcycles=200, steps=steps, u=u, uout=uout, p=p)


@pytest.mark.parametrize("name", list(CASES))
def test_batched_steps_replay_against_the_oracle(name):
    """Each step run through the batched kernel from the state it left, then
    the same step by the oracle from that state: the GPU's dt against the
    oracle's CFL rule, velocity and outflow plane to 1e-5 relative L2 (and
    element-wise max), pressure to 1e-5 in the Poisson operator's energy norm."""
    import paper_2304_08159_amd as wl
    cfg = CASES[name]
    n, d = cfg["n"], len(cfg["n"])
    u, uout, p = _state(cfg)
    osim = S.Sim(n, cfg["bc_lo"], cfg["bc_hi"], cfg["U"], cfg["nu"], body=cfg["body"],
                 tol=1e-12, stop_rule="relative", max_vcycles=300)
    for step in range(4):
        un = [to_oracle(u[i], d) for i in range(d)]
        uo = plane_to_oracle(uout, d) if uout is not None else None
        pn = to_oracle(p, d)
        st, vc, t, dt = wl.ns_batch_run([_req(cfg, u, uout, p, 1)])[0]
        assert st == 0
        dt_o = M.cfl_dt(un, uo, cfg["bc_lo"], cfg["bc_hi"], cfg["U"], cfg["nu"], 0.5)
        osim.u, osim.uout, osim.p = un, uo, pn
        osim.step(dt=dt)
        ug = [to_oracle(u[i], d) for i in range(d)]
        eu = math.sqrt(sum(np.sum((a - b) ** 2) for a, b in zip(ug, osim.u)) /
                       sum(np.sum(b ** 2) for b in osim.u))
        mu = max(float(np.abs(a - b).max()) for a, b in zip(ug, osim.u)) / \
            max(float(np.abs(b).max()) for b in osim.u)
        act = osim.h.active[0]
        pg, po = mean_free(to_oracle(p, d), act), mean_free(osim.p, act)
        ep = rel_l2(pg, po, act)
        # pressure in the operator's energy norm: the cells a body covers are
        # coupled through faces of mu0 ~ 1e-3 and converge slowly in plain L2
        per = [b == 0 for b in cfg["bc_lo"]]
        e = pg - po
        ea = math.sqrt(abs(np.sum(e * P.apply_A(osim.L, e, per))) /
                       abs(np.sum(po * P.apply_A(osim.L, po, per))))
        eo = rel_l2(plane_to_oracle(uout, d), osim.uout) if uout is not None else 0.0
        print(f"{name} step {step}: dt={dt:.5f} (oracle {dt_o:.5f}) vc={vc} err_u={eu:.2e} "
              f"(max {mu:.2e}) err_p={ep:.2e} (energy {ea:.2e}) err_uout={eo:.2e}", flush=True)
        assert abs(dt - dt_o) <= 1e-6 * dt_o
        assert eu <= 1e-5 and mu <= 1e-5 and eo <= 1e-5 and ea <= 1e-5


def test_batched_runs_do_not_depend_on_the_batch():
    """The same request alone and in a batch with other sizes: bitwise the
    same state after 5 steps."""
    import paper_2304_08159_amd as wl
    outs = []
    for companions in ([], ["sphere-3d", "tgv-2d-periodic", "cylinder-2d"]):
        reqs, states = [], []
        for name in ["cylinder-2d"] + companions:
            u, uout, p = _state(CASES[name])
            reqs.append(_req(CASES[name], u, uout, p, 5))
            states.append((u, uout, p))
        res = wl.ns_batch_run(reqs)
        assert all(r[0] == 0 for r in res)
        outs.append((res[0], states[0]))
    (ra, (ua, oa, pa)), (rb, (ub, ob, pb)) = outs
    assert ra == rb
    assert torch.equal(ua, ub) and torch.equal(oa, ob) and torch.equal(pa, pb)


def test_batched_run_arguments_are_checked():
    import paper_2304_08159_amd as wl
    cfg = CASES["cylinder-2d"]
    u, uout, p = _state(cfg)
    moving = dict(cfg["body"], velocity=(0.1, 0.0))
    with pytest.raises(wl.WlError):
        wl.ns_batch_run([dict(_req(cfg, u, uout, p, 1), body=moving)])
    with pytest.raises(wl.WlError):
        wl.ns_batch_run([dict(_req(cfg, u, uout, p, 1), n=(640, 512))])
