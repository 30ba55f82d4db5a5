"""Pins of the projection and the full Heun step (closed forms, invariants)."""

import math

import numpy as np
import pytest

import workloads as W
from oracle import poisson as P
from oracle import step as S
from oracle.grid import PERIODIC, auto_levels


def test_divergence_identity_for_any_pressure():
    n = (10, 8, 6)
    per = [PERIODIC] * 3
    rng = np.random.default_rng(0)
    L = [rng.uniform(0.2, 1.0, n) for _ in range(3)]
    us = [rng.standard_normal(n) for _ in range(3)]
    c, dt = 0.5, 0.37
    sigma = S.divergence(us, None, per, per, (0, 0, 0)) / (c * dt)
    p = rng.standard_normal(n)
    u = S.grad_update(us, p, L, [True] * 3, c * dt)
    div = S.divergence(u, None, per, per, (0, 0, 0))
    np.testing.assert_allclose(div, c * dt * (sigma - P.apply_A(L, p, [True] * 3)), atol=1e-13)


def test_tight_projection_is_divergence_free_and_idempotent():
    n = (16, 16, 16)
    per = [PERIODIC] * 3
    rng = np.random.default_rng(1)
    us = [rng.standard_normal(n) for _ in range(3)]
    L = [np.ones(n)] * 3
    h = P.Hierarchy(L, auto_levels(n), [True] * 3)
    dt = 0.4
    sigma = S.divergence(us, None, per, per, (0, 0, 0)) / dt
    p, k, hist, ok = P.solve(h, sigma, tol=1e-14, max_vcycles=200)
    u = S.grad_update(us, p, L, [True] * 3, dt)
    assert np.abs(S.divergence(u, None, per, per, (0, 0, 0))).max() <= 1e-10
    sigma2 = S.divergence(u, None, per, per, (0, 0, 0)) / dt
    p2, *_ = P.solve(h, sigma2, tol=1e-14, max_vcycles=200)
    u2 = S.grad_update(u, p2, L, [True] * 3, dt)
    for a, b in zip(u, u2):
        assert np.abs(a - b).max() <= 1e-12
    # a gradient field L grad(phi) is annihilated by the projection
    phi = rng.standard_normal(n)
    g = [np.zeros(n)] * 3
    g = S.grad_update(g, -phi, L, [True] * 3, 1.0)
    sig = S.divergence(g, None, per, per, (0, 0, 0)) / dt
    pg, *_ = P.solve(h, sig, tol=1e-14, max_vcycles=200)
    ug = S.grad_update(g, pg, L, [True] * 3, dt)
    assert max(np.abs(a).max() for a in ug) <= 1e-11


def test_tgv3d_initial_field_is_discretely_solenoidal_with_closed_form_energy():
    u, v, w, nu = W.tgv3d(32)
    per = [PERIODIC] * 3
    div = S.divergence([u, v, w], None, per, per, (0, 0, 0))
    assert np.abs(div).max() < 1e-14
    ke = 0.5 * (np.mean(u * u) + np.mean(v * v) + np.mean(w * w))
    assert ke == pytest.approx(1.0 / 8.0, rel=1e-13)
    assert nu == pytest.approx((32 / (2 * math.pi)) / 1600.0)


def _tgv2d_run(N, nu_phys, T_phys, dt_fixed=None):
    u, v, p, nug = W.tgv2d(N, nu_phys)
    sim = S.Sim((N, N), [PERIODIC] * 2, [PERIODIC] * 2, (0, 0), nug, tol=1e-11)
    sim.u = [u.copy(), v.copy()]
    Tg = T_phys * N / (2 * math.pi)
    while sim.t < Tg - 1e-12:
        dt = dt_fixed if dt_fixed else sim.dt_cfl()
        sim.step(min(dt, Tg - sim.t))
    return sim


def test_tgv2d_decay_matches_closed_form():
    nu_phys, T = 0.01, 1.0
    errs = {}
    for N in (32, 64):
        sim = _tgv2d_run(N, nu_phys, T)
        ue, ve, pe, _ = W.tgv2d(N, nu_phys, T)
        errs[N] = math.sqrt((np.sum((sim.u[0] - ue) ** 2) + np.sum((sim.u[1] - ve) ** 2))
                            / (np.sum(ue ** 2) + np.sum(ve ** 2)))
        if N == 64:
            ke = 0.5 * np.mean(sim.u[0] ** 2 + sim.u[1] ** 2)
            ke_exact = 0.25 * math.exp(-4 * nu_phys * T)
            assert ke == pytest.approx(ke_exact, rel=1e-3)
            # pressure: compare mean-free fields at cell centres
            pn = sim.p - sim.p.mean()
            assert np.linalg.norm(pn - (pe - pe.mean())) / np.linalg.norm(pe) < 2e-2
    order = math.log2(errs[32] / errs[64])
    assert order >= 1.5
    assert errs[64] < 1e-3


def test_heun_is_second_order_in_time():
    N, nu_phys, T = 32, 0.05, 0.5
    Tg = T * N / (2 * math.pi)
    ref = _tgv2d_run(N, nu_phys, T, dt_fixed=Tg / 64)
    errs = []
    for m in (8, 16):
        sim = _tgv2d_run(N, nu_phys, T, dt_fixed=Tg / m)
        errs.append(math.sqrt(sum(np.sum((a - b) ** 2) for a, b in zip(sim.u, ref.u))))
    assert math.log2(errs[0] / errs[1]) >= 1.7


def test_cylinder_flow_keeps_mirror_symmetry_and_zero_velocity_inside():
    c = W.cylinder_config()
    sim = S.Sim(c["n"], c["bc_lo"], c["bc_hi"], c["U"], c["nu"], body=c["body"],
                levels=c["levels"], tol=c["tol"])
    for _ in range(10):
        st = sim.step()
    u, v = sim.u
    assert np.abs(u - u[:, ::-1]).max() < 1e-12
    assert np.abs(v[:, 1:] + v[:, :0:-1]).max() < 1e-12
    X = np.meshgrid(np.arange(128.0), np.arange(64) + 0.5, indexing="ij")
    inside = np.hypot(X[0] - 32.0, X[1] - 32.0) < 8.0 - 1.0
    assert np.all(u[inside] == 0.0)
    # inflow face and walls hold their boundary values; outflow carries the inflow flux
    assert np.all(u[0] == 1.0) and np.all(v[:, 0] == 0.0)
    assert sim.uout.sum() == pytest.approx(64.0, rel=1e-13)
    assert 0.05 < st["dt"] < 0.5


@pytest.mark.parametrize("n,centre,radius,exact", [
    ((40, 40, 40), (20.3, 19.8, 20.1), 7.0, 4.0 / 3.0 * math.pi * 7.0 ** 3),
    ((64, 64), (31.7, 32.2), 10.0, math.pi * 10.0 ** 2),
])
def test_drag_of_a_linear_pressure_is_minus_gradient_times_volume(n, centre, radius, exact):
    """For p = a x the surface integral -oint p n_x dS equals -a V (divergence
    theorem), whatever the pressure's free constant; the kernel-smoothed sum
    reproduces it to second order in the band width over the radius.  A
    pressure even in x about the centre, or independent of x, has zero drag."""
    from oracle.grid import WALL
    d = len(n)
    sim = S.Sim(n, [WALL] * d, [WALL] * d, (0.0,) * d, 0.01,
                body=dict(centre=centre, radius=radius))
    X = np.meshgrid(*[np.arange(m) + 0.5 for m in n], indexing="ij")
    a = 0.37
    sim.p = a * X[0] + 5.0
    F = S.drag(sim)
    # quadrature error O((eps / R)^2): 0.9 % at R = 7 (3D), 0.24 % at R = 10 (2D)
    assert abs(F - (-a * exact)) <= 0.02 * a * exact
    from oracle import geometry as G
    dist, normal = G.sphere_sdf(X, centre, radius)
    for p in ((X[0] - centre[0]) ** 2, X[1] - 3.0):
        sim.p = p
        bound = np.sum(np.abs(p) * np.abs(normal[0]) * G.kernel(dist))
        assert abs(S.drag(sim)) <= 0.01 * bound


def test_relative_stopping_rule_stops_at_the_first_cycle_below_tol():
    """stop_rule "relative": each stage's solve ends at the first V-cycle whose
    relative residual is <= tol, and not before."""
    cfg = W.cylinder_config()
    sim = S.Sim((32, 16), cfg["bc_lo"], cfg["bc_hi"], cfg["U"], 0.02,
                body=dict(centre=(8.0, 8.0), radius=3.0), tol=1e-9, stop_rule="relative")
    for _ in range(2):
        st = sim.step()
    for hist in st["resid"]:
        assert hist[-1] <= 1e-9
        assert all(r > 1e-9 for r in hist[:-1])
    with pytest.raises(ValueError):
        S.Sim((32, 16), cfg["bc_lo"], cfg["bc_hi"], cfg["U"], 0.02, stop_rule="rms")
