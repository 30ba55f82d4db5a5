"""Pins of the moving-body reading (rigid motion from the coordinate map,
Sec. 2): the body velocity and its gradient, the BDIM blend with a body
velocity, the re-measure time, and flows whose exact answer is known."""

import math

import numpy as np
import pytest

from oracle import geometry as G
from oracle import momentum as M
from oracle import step as S
from oracle.grid import PERIODIC


def test_centre_velocity_is_the_time_derivative_of_the_path():
    body = dict(centre=(10.0, 8.0, 6.0), radius=2.0, velocity=(0.3, -0.1, 0.05),
                amplitude=(0.0, 1.5, -0.7), omega=0.4)
    for t in (0.0, 0.7, 3.1):
        X, Xdot, _ = G.body_motion(body, t)
        h = 1e-5
        fd = (G.body_motion(body, t + h)[0] - G.body_motion(body, t - h)[0]) / (2 * h)
        np.testing.assert_allclose(Xdot, fd, rtol=0, atol=1e-9)
    np.testing.assert_allclose(G.body_motion(body, 0.0)[0], body["centre"], atol=0)


def test_body_velocity_is_rigid_and_its_gradient_matches():
    """V_b = dX/dt + Omega x r: every pair of points keeps its distance
    ((V_b(x) - V_b(y)) . (x - y) = 0), V_b at the centre is dX/dt, and the
    stated gradient equals central differences of V_b."""
    body = dict(centre=(10.0, 8.0, 6.0), radius=2.0, velocity=(0.2, 0.0, 0.1),
                spin=(0.3, -0.5, 0.8))
    t = 1.3
    rng = np.random.default_rng(1)
    P = [rng.uniform(0, 20, 50) for _ in range(3)]
    Q = [rng.uniform(0, 20, 50) for _ in range(3)]
    vp, vq = G.body_velocity(P, body, t), G.body_velocity(Q, body, t)
    dot = sum((vp[i] - vq[i]) * (P[i] - Q[i]) for i in range(3))
    assert np.abs(dot).max() <= 1e-12
    Xc, Xdot, _ = G.body_motion(body, t)
    vc = G.body_velocity([np.array([Xc[i]]) for i in range(3)], body, t)
    np.testing.assert_allclose([v[0] for v in vc], Xdot, atol=1e-15)
    Gm = G.body_velocity_gradient(body, 3)
    h = 1e-4
    for j in range(3):
        Pp = [P[i] + (h if i == j else 0.0) for i in range(3)]
        Pm = [P[i] - (h if i == j else 0.0) for i in range(3)]
        vpp, vmm = G.body_velocity(Pp, body, t), G.body_velocity(Pm, body, t)
        for i in range(3):
            np.testing.assert_allclose((vpp[i] - vmm[i]) / (2 * h), Gm[i, j], atol=1e-9)
    # 2D: spin about z only
    b2 = dict(centre=(5.0, 5.0), radius=1.0, spin=0.6)
    np.testing.assert_allclose(G.body_velocity_gradient(b2, 2), [[0.0, -0.6], [0.6, 0.0]])
    v = G.body_velocity([np.array([6.0]), np.array([5.0])], b2, 0.0)
    assert v[0][0] == 0.0 and v[1][0] == pytest.approx(0.6)      # counter-clockwise


@pytest.mark.parametrize("d", [2, 3])
def test_bdim_returns_the_body_velocity_for_a_rigid_motion_field(d):
    """A stage field that already moves rigidly with the body passes the blend
    unchanged: mu0 V_b + (1 - mu0) V_b + mu1 d/dn (V_b - V_b) = V_b, in the
    body, its band and the fluid.  A missing (1 - mu0) V_b term or a wrong
    sign of the gradient correction changes it."""
    n = (24, 20) if d == 2 else (20, 18, 16)
    body = dict(centre=tuple(m / 2.0 + 0.3 for m in n), radius=4.5,
                velocity=(0.2, -0.1, 0.05)[:d], spin=0.7 if d == 2 else (0.2, -0.4, 0.6))
    t = 0.9
    bc = [PERIODIC] * d
    mu0, mu1n, _ = G.measure(n, bc, body, 1.0, t)
    Vb = [G.body_velocity(G.face_centres(n, i), body, t)[i] for i in range(d)]
    Gm = G.body_velocity_gradient(body, d)
    out = M.bdim([v.copy() for v in Vb], mu0, mu1n, bc, bc, [0.0] * d, None, Vb, Gm)
    # the field is linear only away from the periodic seam; the body sits mid-box
    sl = tuple(slice(3, m - 3) for m in n)
    for i in range(d):
        np.testing.assert_allclose(out[i][sl], Vb[i][sl], atol=1e-12)
    assert np.any(mu0[0] < 0.5) and np.any(mu1n[0][0] != 0.0)


def test_fluid_translating_with_the_body_stays_undisturbed():
    """A periodic box whose fluid moves with a translating sphere: the step
    keeps u = V exactly (up to rounding) and the pressure flat."""
    n = (24, 16, 16)
    V = (0.4, 0.1, -0.05)
    body = dict(centre=(8.0, 8.2, 7.9), radius=3.0, velocity=V)
    sim = S.Sim(n, [PERIODIC] * 3, [PERIODIC] * 3, (0.0, 0.0, 0.0), 0.05, body=body, tol=1e-12)
    sim.u = [np.full(n, V[i]) for i in range(3)]
    for _ in range(4):
        sim.step()
    for i in range(3):
        assert np.abs(sim.u[i] - V[i]).max() <= 1e-11
    act = sim.h.active[0]
    assert np.ptp(sim.p[act]) <= 1e-9


def test_moving_body_is_measured_where_the_step_takes_it():
    """The step re-measures the body at t + dt (both stages advance to it)."""
    n = (32, 16)
    body = dict(centre=(10.0, 8.0), radius=3.0, amplitude=(0.0, 2.0), omega=0.5)
    sim = S.Sim(n, [1, 3], [2, 3], (1.0, 0.0), 0.05, body=body, tol=1e-10)
    st = sim.step()
    t1 = st["dt"]
    Xc, _, _ = G.body_motion(body, t1)
    ref = G.measure(n, [1, 3], dict(centre=tuple(Xc[:2]), radius=3.0))
    for i in range(2):
        np.testing.assert_array_equal(sim.mu0[i], ref[0][i])
        np.testing.assert_array_equal(sim.L[i], ref[2][i])
    assert not np.array_equal(sim.mu0[1], G.measure(n, [1, 3], body)[0][1])


def test_spinning_cylinder_drives_a_co_rotating_flow():
    """A circle spinning counter-clockwise in fluid at rest: after a few steps
    the fluid just outside it circulates counter-clockwise (positive
    circulation on a loop around the body) and the body's own faces carry its
    rigid rotation."""
    n = (32, 32)
    Om = 0.2
    body = dict(centre=(16.0, 16.0), radius=5.0, spin=Om)
    sim = S.Sim(n, [PERIODIC] * 2, [PERIODIC] * 2, (0.0, 0.0), 0.05, body=body, tol=1e-12)
    sim.u = [np.zeros(n), np.zeros(n)]
    for _ in range(5):
        sim.step(dt=0.5)
    u, v = sim.u
    # circulation on the square loop x, y in [9, 23] (outside the body)
    lo, hi = 9, 23
    circ = (np.sum(u[lo:hi, lo]) + np.sum(v[hi, lo:hi]) - np.sum(u[lo:hi, hi]) -
            np.sum(v[lo, lo:hi]))
    assert circ > 0.0
    # deep inside the body the velocity is the rigid rotation: the v face of
    # cell (17, 15) sits at x = 17.5, so v = Om (17.5 - 16)
    assert v[17, 15] == pytest.approx(Om * (17.5 - 16.0), abs=1e-9)
