"""GPU parity of the Navier-Stokes step against the FP64 oracle (replay mode).

Replay: the oracle starts from the GPU state u^n, p^n (widened to FP64),
takes the GPU's dt and V-cycle counts, and advances one step; the GPU's
u^{n+1}, p^{n+1} must match to 1e-5 relative L2 (pressure compared mean-free
over active cells).
"""

import math

import numpy as np
import pytest

import workloads as W
from oracle import geometry as G
from oracle import momentum as M
from oracle import step as S
from tests.gpu_util import mean_free, plane_to_oracle, rel_l2, to_device, to_oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _make(cfg, prec, tol):
    import paper_2304_08159_amd as wl
    sim = wl.Sim(cfg["n"], cfg["bc_lo"], cfg["bc_hi"], cfg["U"], cfg["nu"], body=cfg.get("body"),
                 prec=prec, levels=cfg.get("levels", 0), tol=tol, cfl=cfg.get("cfl", 0.5))
    osim = S.Sim(cfg["n"], cfg["bc_lo"], cfg["bc_hi"], cfg["U"], cfg["nu"], body=cfg.get("body"),
                 levels=cfg.get("levels", 0), tol=tol, cfl=cfg.get("cfl", 0.5))
    return sim, osim


def _max_rel(a, b):
    """max |a - b| over max |b| (element-wise bound, any field list)."""
    num = max(float(np.abs(x - y).max()) for x, y in zip(a, b))
    den = max(float(np.abs(y).max()) for y in b)
    return num / (den if den > 0 else 1.0)


def _replay(sim, osim, nsteps, tol_u, tol_p, label, tol_dt=1e-6, tol_pmax=None):
    """Replay nsteps GPU steps through the oracle and compare, per step:
    velocity and outflow plane in relative L2 and element-wise (max |difference|
    <= tol_u x max |field|), the mean-free pressure in relative L2 (tol_p) and
    element-wise (tol_pmax, default 10 tol_p: cells the body nearly closes hold a
    weakly determined pressure), and the GPU's CFL time step against the
    oracle's cfl_dt of the same state (tol_dt relative: the GPU sums each
    cell's outflow in the field precision)."""
    if tol_pmax is None:
        tol_pmax = 10 * tol_p
    d = sim.ndim
    worst_u = worst_p = 0.0
    outflow = osim.bc_hi[0] == 2
    for step in range(nsteps):
        un = [to_oracle(t, d) for t in sim.velocity()]
        pn = to_oracle(sim.pressure(), d)
        uo = plane_to_oracle(sim.get(4), d) if outflow else None
        st = sim.step()
        dt_o = M.cfl_dt(un, uo, osim.bc_lo, osim.bc_hi, osim.U, osim.nu, osim.cfl)
        edt = abs(st["dt"] - dt_o) / dt_o
        osim.u, osim.p, osim.uout = un, pn, uo
        osim.step(dt=st["dt"], force_vcycles=st["vcycles"])
        act = osim.h.active[0]
        ug = [to_oracle(t, d) for t in sim.velocity()]
        eu = math.sqrt(sum(np.sum((a - b) ** 2) for a, b in zip(ug, osim.u)) /
                       sum(np.sum(b ** 2) for b in osim.u))
        mu = _max_rel(ug, osim.u)
        pg, po = mean_free(to_oracle(sim.pressure(), d), act), mean_free(osim.p, act)
        ep = rel_l2(pg, po, act)
        mp = _max_rel([pg], [po])
        eo = mo = 0.0
        if outflow:
            og = plane_to_oracle(sim.get(4), d)
            eo = rel_l2(og, osim.uout)
            mo = _max_rel([og], [osim.uout])
        worst_u = max(worst_u, eu, mu, eo, mo)
        worst_p = max(worst_p, ep, mp * tol_p / tol_pmax)
        print(f"{label} step {step}: dt={st['dt']:.6f} (oracle cfl_dt rel diff {edt:.1e}) "
              f"vc={st['vcycles']} div={st['resid'][0]:.2e},{st['resid'][1]:.2e} "
              f"err_u={eu:.2e} (max {mu:.2e}) err_p={ep:.2e} (max {mp:.2e})"
              + (f" err_uout={eo:.2e} (max {mo:.2e})" if outflow else ""), flush=True)
        assert edt <= tol_dt
    assert worst_u <= tol_u and worst_p <= tol_p
    return worst_u, worst_p


def test_geometry_measure_matches_oracle():
    import paper_2304_08159_amd as wl
    for n, bc_lo, bc_hi, body, prec in [
        ((48, 32), [1, 3], [2, 3], dict(centre=(16.3, 15.8), radius=6.0), wl.WL_FP64),
        ((40, 24, 24), [1, 3, 0], [2, 3, 0], dict(centre=(12.0, 12.2, 11.7), radius=5.0),
         wl.WL_FP32),
    ]:
        d = len(n)
        sim = wl.Sim(n, bc_lo, bc_hi, (1.0,) + (0.0,) * (d - 1), 0.01, body=body, prec=prec)
        mu0, mu1n, L = G.measure(n, bc_lo, body)
        tol = 1e-14 if prec == wl.WL_FP64 else 2e-7
        for i in range(d):
            np.testing.assert_allclose(to_oracle(sim.get(wl.FIELD_L0 + i), d), L[i], atol=tol)
            np.testing.assert_allclose(to_oracle(sim.get(wl.FIELD_MU0_0 + i), d), mu0[i], atol=tol)
            for j in range(d):
                np.testing.assert_allclose(to_oracle(sim.get(wl.FIELD_MU1N + 3 * i + j), d),
                                           mu1n[i][j], atol=tol)


def test_cfl_time_step_closed_form():
    import paper_2304_08159_amd as wl
    n = (32, 16, 16)
    sim = wl.Sim(n, [0, 0, 0], [0, 0, 0], (1.5, 0.0, 0.0), 0.02, prec=wl.WL_FP64, tol=1e-8)
    st = sim.step()
    assert st["dt"] == pytest.approx(0.5 / (1.5 + 6 * 0.02), rel=1e-15)
    assert st["vcycles"] == (0, 0)   # uniform flow: zero divergence, nothing to solve


def test_tgv3d_fp32_replay_parity():
    import paper_2304_08159_amd as wl
    N = 32
    u, v, w, nu = W.tgv3d(N)
    cfg = dict(n=(N, N, N), bc_lo=[0] * 3, bc_hi=[0] * 3, U=(0.0, 0.0, 0.0), nu=nu)
    sim, osim = _make(cfg, wl.WL_FP32, 1e-5)
    for i, a in enumerate((u, v, w)):
        sim.set(wl.FIELD_U0 + i, to_device(a, 3, torch, torch.float32))
    _replay(sim, osim, 4, 1e-5, 1e-5, "tgv32")


def test_tgv256_fp32_full_size_replay_parity():
    """The benchmark's workload at its full size and in the launch
    configuration it times (256^3 FP32 TGV, Re = 1600, tol 1e-5: momentum
    z chunks of 64 planes over several chunks, fused sweep pairs on every
    level, the first residual check inside the divergence, the predictor's
    projection inside the corrector's convection-diffusion): after one warm-up
    step (so that p^n is a real warm start), one step replayed by the oracle
    over the whole field."""
    import paper_2304_08159_amd as wl
    N = 256
    u, v, w, nu = W.tgv3d(N, Re=1600.0)
    cfg = dict(n=(N, N, N), bc_lo=[0] * 3, bc_hi=[0] * 3, U=(0.0, 0.0, 0.0), nu=nu)
    sim, osim = _make(cfg, wl.WL_FP32, 1e-5)
    for i, a in enumerate((u, v, w)):
        sim.set(wl.FIELD_U0 + i, to_device(a, 3, torch, torch.float32))
    del u, v, w
    print("tgv256 warm-up step:", sim.step(), flush=True)
    _replay(sim, osim, 1, 1e-5, 1e-5, "tgv256")
    sim.close()


@pytest.mark.parametrize("n", [(72, 20, 44), (72, 32, 48)])
def test_periodic_ragged_tiles_and_chunks_fp32_replay_parity(n):
    """Periodic FP32 3D grids whose x / y extents leave ragged momentum tiles
    (72 = 64 + 8, 20 = 2 x 8 + 4) and, for n2 = 44, a short last z chunk
    (5 x 8 + 4 planes): the tile and chunk edge paths of the
    convection-diffusion kernels (the predictor's clamped two-plane
    prefetch, the corrector's fused projection); (72, 32, 48) also runs
    fused sweep pairs with 8-wide tiles on its fine level."""
    import paper_2304_08159_amd as wl
    u, v, w = W.periodic_modes3d(n, seed=7)
    cfg = dict(n=n, bc_lo=[0] * 3, bc_hi=[0] * 3, U=(0.0, 0.0, 0.0), nu=0.02)
    sim, osim = _make(cfg, wl.WL_FP32, 1e-5)
    for i, a in enumerate((u, v, w)):
        sim.set(wl.FIELD_U0 + i, to_device(a, 3, torch, torch.float32))
    _replay(sim, osim, 3, 1e-5, 1e-5, f"ragged{n}")
    sim.close()


def test_tgv2d_fp64_free_running_matches_oracle():
    import paper_2304_08159_amd as wl
    N = 48
    u, v, p, nug = W.tgv2d(N, 0.01)
    cfg = dict(n=(N, N), bc_lo=[0, 0], bc_hi=[0, 0], U=(0.0, 0.0), nu=nug)
    sim, osim = _make(cfg, wl.WL_FP64, 1e-10)
    sim.set(wl.FIELD_U0, to_device(u, 2, torch, torch.float64))
    sim.set(wl.FIELD_U0 + 1, to_device(v, 2, torch, torch.float64))
    osim.u = [u.copy(), v.copy()]
    for _ in range(5):
        st = sim.step()
        ost = osim.step()
        assert st["dt"] == pytest.approx(ost["dt"], rel=1e-12)
    ug = [to_oracle(t, 2) for t in sim.velocity()]
    err = math.sqrt(sum(np.sum((a - b) ** 2) for a, b in zip(ug, osim.u)) /
                    sum(np.sum(b ** 2) for b in osim.u))
    print(f"tgv2d fp64 free-running 5 steps: err_u={err:.3e}")
    assert err <= 1e-9


def test_cylinder_fp64_replay_parity():
    import paper_2304_08159_amd as wl
    cfg = W.cylinder_config()
    sim, osim = _make(cfg, wl.WL_FP64, cfg["tol"])
    _replay(sim, osim, 6, 1e-9, 1e-7, "cylinder")
    # mirror symmetry and the inflow / wall boundary values on the GPU
    u, v = [to_oracle(t, 2) for t in sim.velocity()]
    assert np.abs(u - u[:, ::-1]).max() < 1e-10
    assert np.all(u[0] == 1.0) and np.all(v[:, 0] == 0.0)
    uo = plane_to_oracle(sim.get(4), 2)
    assert uo.sum() == pytest.approx(64.0, rel=1e-12)


@pytest.mark.parametrize("case", ["circle-2d-fp64", "sphere-3d-fp32"])
def test_outflow_perturbed_replay_parity(case):
    """Inflow / convective outflow channels started from a disturbed state
    (smooth seeded modes on the velocity and on the outlet plane), so that the
    outflow rule moves a non-uniform plane and the exit-flux balance shifts
    it: velocity, pressure and the outflow plane against the oracle."""
    import paper_2304_08159_amd as wl
    if case == "circle-2d-fp64":
        cfg = dict(n=(96, 48), bc_lo=[1, 3], bc_hi=[2, 3], U=(1.0, 0.0), nu=0.05,
                   body=dict(centre=(24.0, 24.3), radius=5.0), tol=1e-10)
        prec, tdev, tol = wl.WL_FP64, torch.float64, 1e-9
    else:
        cfg = dict(n=(64, 32, 32), bc_lo=[1, 3, 3], bc_hi=[2, 3, 3], U=(1.0, 0.0, 0.0),
                   nu=0.08, body=dict(centre=(16.0, 16.2, 15.8), radius=4.0), tol=1e-5)
        prec, tdev, tol = wl.WL_FP32, torch.float32, 1e-5
    n = cfg["n"]
    d = len(n)
    sim, osim = _make(cfg, prec, cfg["tol"])
    n3 = tuple(n) + (1,) * (3 - d)
    modes = W.periodic_modes3d(n3, seed=11)
    for i in range(d):
        a = cfg["U"][i] + 0.3 * (modes[i][:, :, 0] if d == 2 else modes[i])
        # boundary faces keep their boundary values (inflow U, wall 0)
        if i == 0:
            a[0] = cfg["U"][0]
        else:
            a[(slice(None),) * i + (0,)] = 0.0
        sim.set(wl.FIELD_U0 + i, to_device(a, d, torch, tdev))
    yz = modes[0][-1]                                     # a smooth (n1, n2) pattern
    plane = cfg["U"][0] + 0.3 * (yz[:, 0] if d == 2 else yz)
    sim.set(wl.FIELD_UOUT, torch.from_numpy(np.ascontiguousarray(
        plane[None, :] if d == 2 else plane.T)).to(device="cuda", dtype=tdev))
    _replay(sim, osim, 3, tol, tol * (100 if d == 2 else 1), case)


def test_sphere_fp32_replay_parity():
    import paper_2304_08159_amd as wl
    cfg = dict(n=(64, 32, 32), bc_lo=[1, 3, 3], bc_hi=[2, 3, 3], U=(1.0, 0.0, 0.0),
               nu=0.08, body=dict(centre=(16.0, 16.0, 16.0), radius=4.0), tol=1e-5)
    sim, osim = _make(cfg, wl.WL_FP32, cfg["tol"])
    _replay(sim, osim, 3, 1e-5, 1e-5, "sphere")


def test_sphere_mixed_precision_step_matches_tight_oracle():
    """WL_MIXED: FP32 fields, FP32 V-cycles with FP64 defect correction.  With
    both solves tight, one step from the same state agrees with the oracle."""
    import paper_2304_08159_amd as wl
    cfg = dict(n=(48, 24, 24), bc_lo=[1, 3, 3], bc_hi=[2, 3, 3], U=(1.0, 0.0, 0.0),
               nu=0.06, body=dict(centre=(12.0, 12.0, 12.2), radius=4.0))
    sim = wl.Sim(cfg["n"], cfg["bc_lo"], cfg["bc_hi"], cfg["U"], cfg["nu"], body=cfg["body"],
                 prec=wl.WL_MIXED, tol=1e-9, max_vcycles=300)
    osim = S.Sim(cfg["n"], cfg["bc_lo"], cfg["bc_hi"], cfg["U"], cfg["nu"], body=cfg["body"],
                 tol=1e-13, max_vcycles=300)
    for step in range(3):
        un = [to_oracle(t, 3) for t in sim.velocity()]
        pn = to_oracle(sim.pressure(), 3)
        uo = plane_to_oracle(sim.get(4), 3)
        st = sim.step()
        osim.u, osim.p, osim.uout = un, pn, uo
        osim.step(dt=st["dt"])
        ug = [to_oracle(t, 3) for t in sim.velocity()]
        eu = math.sqrt(sum(np.sum((a - b) ** 2) for a, b in zip(ug, osim.u)) /
                       sum(np.sum(b ** 2) for b in osim.u))
        act = osim.h.active[0]
        ep = rel_l2(mean_free(to_oracle(sim.pressure(), 3), act), mean_free(osim.p, act), act)
        print(f"mixed step {step}: vc={st['vcycles']} div={st['resid']} err_u={eu:.2e} err_p={ep:.2e}")
        assert eu <= 1e-5 and ep <= 1e-5


def test_body_coeffs_matches_oracle():
    import paper_2304_08159_amd as wl
    for n, per, prec in [((40, 30), (False, True), wl.WL_FP32),
                         ((20, 16, 12), (True, False, False), wl.WL_FP64)]:
        body = dict(centre=tuple(m / 2.0 + 0.3 for m in n), radius=4.5)
        L = wl.body_coeffs(n, per, body, prec=prec)
        d = len(n)
        Lo = G.measure(n, [0 if p else 3 for p in per], body)[2]
        tol = 2e-7 if prec == wl.WL_FP32 else 1e-15
        for i in range(d):
            np.testing.assert_allclose(to_oracle(L[i], d), Lo[i], atol=tol)


def test_fused_predictor_projection_is_bitwise_identical():
    """Periodic FP32 3D steps apply the predictor's projection inside the
    corrector's convection-diffusion kernel unless an adjoint tape is being
    recorded; both ways must give the same bits."""
    import paper_2304_08159_amd as wl
    N = 40
    u, v, w, nu = W.tgv3d(N, Re=1600.0)
    runs = []
    for record in (False, True):
        sim = wl.Sim((N, N, N), [0] * 3, [0] * 3, (0.0, 0.0, 0.0), nu, prec=wl.WL_FP32,
                     tol=1e-6, tape_steps=6)
        for i, a in enumerate((u, v, w)):
            sim.set(wl.FIELD_U0 + i,
                    torch.from_numpy(np.ascontiguousarray(a.transpose(2, 1, 0))).float().cuda())
        sim.tape(record)
        stats = [sim.step() for _ in range(5)]
        runs.append((stats, sim.get_flow().clone(), sim.pressure().clone()))
        sim.close()
    (sa, xa, pa), (sb, xb, pb) = runs
    assert sa == sb
    assert torch.equal(xa, xb) and torch.equal(pa, pb)


def test_global_address_kernels_match_buffer_addressed_ones(monkeypatch):
    """Periodic FP32 convection-diffusion and divergence kernels address
    arrays below 4 GiB through buffer descriptors and larger ones through
    global addresses; both ways give the same bits (WL_GLOBAL_ADDRESSING=1
    forces the global path on a small grid)."""
    import paper_2304_08159_amd as wl
    N = 64
    u, v, w, nu = W.tgv3d(N, Re=1600.0)
    runs = []
    for mode in ("0", "1"):
        monkeypatch.setenv("WL_GLOBAL_ADDRESSING", mode)
        sim = wl.Sim((N, N, N), [0] * 3, [0] * 3, (0.0, 0.0, 0.0), nu, prec=wl.WL_FP32, tol=1e-5)
        for i, a in enumerate((u, v, w)):
            sim.set(wl.FIELD_U0 + i, to_device(a, 3, torch, torch.float32))
        stats = [sim.step() for _ in range(3)]
        runs.append((stats, sim.get_flow().clone(), sim.pressure().clone()))
        sim.close()
    (sa, xa, pa), (sb, xb, pb) = runs
    assert sa == sb
    assert torch.equal(xa, xb) and torch.equal(pa, pb)


def test_run_equals_repeated_steps_and_stops_at_t_end():
    """wl_run (many steps in one call) gives bitwise the state of the same
    number of wl_step calls, and stops once the time reaches t_end."""
    import paper_2304_08159_amd as wl
    N = 32
    u, v, w, nu = W.tgv3d(N, Re=1600.0)
    outs = []
    for mode in ("step", "run"):
        sim = wl.Sim((N, N, N), [0] * 3, [0] * 3, (0.0, 0.0, 0.0), nu, prec=wl.WL_FP32,
                     tol=1e-6)
        for i, a in enumerate((u, v, w)):
            sim.set(wl.FIELD_U0 + i,
                    torch.from_numpy(np.ascontiguousarray(a.transpose(2, 1, 0))).float().cuda())
        stats = [sim.step() for _ in range(5)] if mode == "step" else sim.run(5)
        outs.append((stats, sim.get_flow().clone(), sim.pressure().clone()))
        if mode == "run":
            t_end = stats[-1]["t"] + 1.5 * stats[-1]["dt"]
            more = sim.run(50, t_end=t_end)
            assert 1 <= len(more) <= 3 and more[-1]["t"] >= t_end
            assert all(m["t"] < t_end for m in more[:-1])
            assert sim.run(0) == []
        sim.close()
    (sa, xa, pa), (sb, xb, pb) = outs
    assert sa == sb
    assert torch.equal(xa, xb) and torch.equal(pa, pb)


def test_torus_measure_and_coefficients_match_oracle():
    import paper_2304_08159_amd as wl
    cfg = W.donut_config(4)
    n, body = cfg["n"], cfg["body"]
    for prec, tol in ((wl.WL_FP32, 2e-7), (wl.WL_FP64, 1e-14)):
        sim = wl.Sim(n, cfg["bc_lo"], cfg["bc_hi"], cfg["U"], cfg["nu"], body=body, prec=prec)
        mu0, mu1n, L = G.measure(n, cfg["bc_lo"], body)
        for i in range(3):
            np.testing.assert_allclose(to_oracle(sim.get(wl.FIELD_L0 + i), 3), L[i], atol=tol)
            np.testing.assert_allclose(to_oracle(sim.get(wl.FIELD_MU0_0 + i), 3), mu0[i], atol=tol)
            for j in range(3):
                np.testing.assert_allclose(to_oracle(sim.get(wl.FIELD_MU1N + 3 * i + j), 3),
                                           mu1n[i][j], atol=tol)
        sim.close()
    Lc = wl.body_coeffs(n, (False,) * 3, body, prec=wl.WL_FP64)
    Lo = G.measure(n, [3] * 3, body)[2]
    for i in range(3):
        np.testing.assert_allclose(to_oracle(Lc[i], 3), Lo[i], atol=1e-15)


def test_donut_fp32_replay_parity():
    """Velocity to 1e-5 relative L2; the pressure in the energy norm of the
    Poisson operator, sqrt(-e.A e / -p.A p): cells the thin tube nearly closes
    (mu0 of a few 1e-3) are coupled by tiny L, so their pressure is weakly
    determined and FP32 rounding moves it without changing the velocity."""
    import paper_2304_08159_amd as wl
    from oracle import poisson as P
    cfg = W.donut_config(5)          # 64 x 32 x 32, R = 8, tube radius 2
    sim, osim = _make(cfg, wl.WL_FP32, cfg["tol"])
    per = [False] * 3
    for step in range(3):
        un = [to_oracle(t, 3) for t in sim.velocity()]
        pn = to_oracle(sim.pressure(), 3)
        uo = plane_to_oracle(sim.get(4), 3)
        st = sim.step()
        osim.u, osim.p, osim.uout = un, pn, uo
        osim.step(dt=st["dt"], force_vcycles=st["vcycles"])
        ug = [to_oracle(t, 3) for t in sim.velocity()]
        eu = math.sqrt(sum(np.sum((a - b) ** 2) for a, b in zip(ug, osim.u)) /
                       sum(np.sum(b ** 2) for b in osim.u))
        e = to_oracle(sim.pressure(), 3) - osim.p
        ea = math.sqrt(np.sum(e * P.apply_A(osim.L, e, per)) /
                       np.sum(osim.p * P.apply_A(osim.L, osim.p, per)))
        print(f"donut step {step}: dt={st['dt']:.6f} vc={st['vcycles']} err_u={eu:.2e} "
              f"err_p(A-norm)={ea:.2e}")
        assert eu <= 1e-5 and ea <= 1e-5


def test_torus_rejected_where_unsupported():
    import paper_2304_08159_amd as wl
    cfg = W.donut_config(4)
    with pytest.raises(wl.WlError):
        wl.Sim((32, 16), [1, 3], [2, 3], (1.0, 0.0), 0.01, body=cfg["body"])
    sim = wl.Sim(cfg["n"], cfg["bc_lo"], cfg["bc_hi"], cfg["U"], cfg["nu"], body=cfg["body"])
    with pytest.raises(wl.WlError):
        sim.drag()


def test_cylinder_fp64_free_running_100_steps_matches_oracle():
    """The 2D configuration as stated (128 x 64, circle D = 16, Re = 250, FP64,
    4 levels, 100 CFL-adaptive steps, every solve to relative residual 1e-8):
    the GPU and the oracle each run all 100 steps on their own (own dt, own
    V-cycle counts) from the same start; the error of the final state against
    the oracle is stated and bounded."""
    import paper_2304_08159_amd as wl
    cfg = W.cylinder_config()
    sim = wl.Sim(cfg["n"], cfg["bc_lo"], cfg["bc_hi"], cfg["U"], cfg["nu"], body=cfg["body"],
                 prec=wl.WL_FP64, levels=cfg["levels"], tol=cfg["tol"], cfl=cfg["cfl"],
                 stop_rule=wl.STOP_RELATIVE)
    osim = S.Sim(cfg["n"], cfg["bc_lo"], cfg["bc_hi"], cfg["U"], cfg["nu"], body=cfg["body"],
                 levels=cfg["levels"], tol=cfg["tol"], cfl=cfg["cfl"], stop_rule="relative")
    worst_dt = 0.0
    for k in range(cfg["steps"]):
        st = sim.step()
        ost = osim.step()
        worst_dt = max(worst_dt, abs(st["dt"] - ost["dt"]) / ost["dt"])
        assert max(st["rel_resid"]) <= cfg["tol"]
        if k % 20 == 19:
            print(f"cylinder free-running step {k + 1}: t={st['t']:.4f} vc={st['vcycles']}",
                  flush=True)
    act = osim.h.active[0]
    ug = [to_oracle(t, 2) for t in sim.velocity()]
    eu = math.sqrt(sum(np.sum((a - b) ** 2) for a, b in zip(ug, osim.u)) /
                   sum(np.sum(b ** 2) for b in osim.u))
    mu = _max_rel(ug, osim.u)
    pg, po = mean_free(to_oracle(sim.pressure(), 2), act), mean_free(osim.p, act)
    ep, mp = rel_l2(pg, po, act), _max_rel([pg], [po])
    eo = rel_l2(plane_to_oracle(sim.get(4), 2), osim.uout)
    print(f"C1 free-running 100 steps (t = {osim.t:.4f}): dt rel diff max {worst_dt:.1e}, "
          f"velocity {eu:.2e} (max {mu:.2e}), pressure {ep:.2e} (max {mp:.2e}), "
          f"outflow plane {eo:.2e}")
    assert worst_dt <= 1e-6
    assert eu <= 1e-6 and mu <= 1e-6 and eo <= 1e-6 and ep <= 1e-5
