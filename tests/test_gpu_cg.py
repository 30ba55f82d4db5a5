"""Conjugate-gradient smoothing on the GMG levels (Sec. 2's smoother) on the
GPU: the solve against the oracle's V-cycles with the same smoother, a
Navier-Stokes step with it, and V-cycle counts against damped Jacobi at equal
residual."""

import math
import time

import numpy as np
import pytest

import workloads as W
from oracle import geometry as G
from oracle import poisson as P
from oracle import step as S
from oracle.grid import PERIODIC, WALL, auto_levels
from tests.gpu_util import mean_free, plane_to_oracle, rel_l2, to_device, to_oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture
def cg():
    import paper_2304_08159_amd as wl
    wl.set_smoother("cg")
    try:
        yield wl
    finally:
        wl.set_smoother("jacobi")


CASES = [
    ((32, 32, 32), (False, False, False), dict(centre=(15.6, 16.2, 16.7), radius=6.5), 0),
    ((24, 20, 12), (True, False, True), dict(centre=(11.0, 10.0, 6.0), radius=4.0), 0),
    ((64, 48), (False, True), dict(centre=(30.0, 24.5), radius=9.0), 0),
    ((48, 32, 32), (True, True, True), None, 0),
]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("n,per,body,levels", CASES)
def test_cg_smoothed_gmg_matches_oracle_replay(cg, n, per, body, levels, prec):
    wl = cg
    d = len(n)
    dtype = torch.float64 if prec == "fp64" else torch.float32
    L = G.measure(n, [PERIODIC if p else WALL for p in per], body)[2]
    b = W.random_rhs(n, 17)
    ps = wl.Poisson(n, per, prec=wl.WL_FP64 if prec == "fp64" else wl.WL_FP32, levels=levels)
    x = torch.zeros(ps.shape, dtype=dtype, device="cuda")
    tol = 1e-9 if prec == "fp64" else 1e-5
    coeffs = torch.stack([to_device(L[i], d, torch, dtype) for i in range(d)]).contiguous()
    k, rel = ps.solve(coeffs, x, to_device(b, d, torch, dtype), tol=tol)
    h = P.Hierarchy(L, auto_levels(n, levels), list(per), smoother="cg")
    xo, ko, hist, _ = P.solve(h, b, tol=tol, force_vcycles=k)
    act = h.active[0]
    err = rel_l2(mean_free(to_oracle(x, d), act), mean_free(xo, act), act)
    print(f"cg {n} {per} {prec}: vcycles={k} rel={rel:.3e} oracle_rel={hist[-1]:.3e} err={err:.3e}")
    assert rel <= tol and k >= 1
    assert abs(np.log10(rel) - np.log10(max(hist[-1], 1e-300))) < 0.5
    assert err <= (1e-9 if prec == "fp64" else 1e-5)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_cg_smoothed_step_matches_oracle(cg, prec):
    """A 3D sphere in a channel with CG-smoothed solves: three steps replayed by
    the oracle with the same smoother and V-cycle counts.  CG's step lengths are
    formed from the iterate itself, so rounding enters the (unconverged) pressure
    nonlinearly, unlike the fixed linear map of damped Jacobi: FP64 fields
    agree to 1e-10 in velocity and 1e-7 in pressure (observed 4e-11 / 1e-8),
    FP32 fields to 1e-6 and 1e-4 (observed 2e-7 / 4e-5)."""
    wl = cg
    cfg = dict(n=(64, 32, 32), bc_lo=[1, 3, 3], bc_hi=[2, 3, 3], U=(1.0, 0.0, 0.0), nu=0.08,
               body=dict(centre=(16.0, 16.0, 16.0), radius=4.0))
    fp64 = prec == "fp64"
    tol = 1e-9 if fp64 else 1e-5
    sim = wl.Sim(cfg["n"], cfg["bc_lo"], cfg["bc_hi"], cfg["U"], cfg["nu"], body=cfg["body"],
                 prec=wl.WL_FP64 if fp64 else wl.WL_FP32, tol=tol)
    osim = S.Sim(cfg["n"], cfg["bc_lo"], cfg["bc_hi"], cfg["U"], cfg["nu"], body=cfg["body"],
                 tol=tol, smoother="cg")
    for step in range(3):
        un = [to_oracle(t, 3) for t in sim.velocity()]
        pn = to_oracle(sim.pressure(), 3)
        uo = plane_to_oracle(sim.get(wl.FIELD_UOUT), 3)
        st = sim.step()
        osim.u, osim.p, osim.uout = un, pn, uo
        osim.step(dt=st["dt"], force_vcycles=st["vcycles"])
        ug = [to_oracle(t, 3) for t in sim.velocity()]
        eu = math.sqrt(sum(np.sum((a - b) ** 2) for a, b in zip(ug, osim.u)) /
                       sum(np.sum(b ** 2) for b in osim.u))
        act = osim.h.active[0]
        ep = rel_l2(mean_free(to_oracle(sim.pressure(), 3), act), mean_free(osim.p, act), act)
        print(f"cg {prec} step {step}: vc={st['vcycles']} err_u={eu:.2e} err_p={ep:.2e}")
        if fp64:
            assert eu <= 1e-10 and ep <= 1e-7
        else:
            assert eu <= 1e-6 and ep <= 1e-4


def test_cg_against_jacobi_at_equal_residual(cg):
    """FP64 solves of the sphere-in-a-box problem (radius N/8, N(0,1) right-hand
    side) to 1e-8 with each smoother at 64^3, 128^3 and 256^3: V-cycles and
    time.  CG smoothing must need fewer V-cycles than Jacobi at every size and
    its count may not grow by more than 2 from 64^3 to 256^3 (linear-time GMG,
    Sec. 2)."""
    wl = cg
    out = {}
    for N in (64, 128, 256):
        n = (N, N, N)
        body = dict(centre=(N / 2.0,) * 3, radius=N / 8.0)
        L = wl.body_coeffs(n, (False,) * 3, body, prec=wl.WL_FP64)
        g = torch.Generator(device="cuda")
        g.manual_seed(2304)
        b = torch.randn((N, N, N), generator=g, dtype=torch.float64, device="cuda")
        for kind in ("jacobi", "cg"):
            wl.set_smoother(kind)
            ps = wl.Poisson(n, (False,) * 3, prec=wl.WL_FP64)
            x = torch.zeros_like(b)
            ps.solve(L, x, b, tol=1e-8, max_vcycles=100)          # warm-up, loads L
            x.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            k, rel = ps.solve(None, x, b, tol=1e-8, max_vcycles=100)
            torch.cuda.synchronize()
            out[(N, kind)] = (k, rel, 1e3 * (time.perf_counter() - t0))
            ps.close()
            print(f"{N}^3 {kind}: {k} V-cycles, rel {rel:.2e}, {out[(N, kind)][2]:.2f} ms",
                  flush=True)
        del L, b
    for N in (64, 128, 256):
        assert out[(N, "cg")][0] < out[(N, "jacobi")][0]
    assert out[(256, "cg")][0] - out[(64, "cg")][0] <= 2
