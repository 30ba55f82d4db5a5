"""Pins of the oracle's outflow rule, exit-flux balance and CFL maximum (no GPU).

Each pin comes from something other than the oracle's own formula: the
advection equation the convective outflow discretises, translation
invariance of a field that does not vary along x, global mass conservation
(telescoping of the discrete divergence, solvability of the Neumann
pressure system), and per-cell outflow totals worked out by hand.
"""

import numpy as np
import pytest

from oracle import momentum as M
from oracle import step as S
from oracle.grid import INFLOW, OUTFLOW, PERIODIC, WALL


def _channel(n, ux, uy, uout, U0, bc_y=PERIODIC):
    bc_lo = [INFLOW, bc_y]
    bc_hi = [OUTFLOW, bc_y]
    return [ux, uy], uout, bc_lo, bc_hi, (U0, 0.0)


@pytest.mark.parametrize("U0,b", [(1.0, 0.3), (0.6, -0.45), (1.7, 0.05)])
def test_outflow_plane_advects_a_linear_ramp_at_the_exact_rate(U0, b):
    """The convective outflow discretises du/dt + U du/dx = 0 at the exit
    face.  For a profile linear in x, u = a + b x, the exact rate is -U b,
    and a one-sided difference of a linear function is exact: the outflow
    plane's tendency must equal -U b.  A flipped sign gives +U b, a missing
    rule 0."""
    n = (10, 6)
    a = 0.8
    ux = a + b * np.arange(n[0], dtype=float)[:, None] * np.ones(n)
    uy = np.zeros(n)
    uout = np.full(n[1], a + b * n[0])
    u, uo, lo, hi, U = _channel(n, ux, uy, uout, U0)
    _, Rout = M.rhs(u, uo, lo, hi, U, 0.01)
    np.testing.assert_allclose(Rout, -U0 * b, rtol=1e-13, atol=1e-15)


def test_outflow_plane_at_unit_courant_number_takes_the_upstream_value():
    """First-order upwinding at Courant number U dt = 1 is an exact
    translation by one cell: after one explicit update the outflow face
    carries the value the last interior face had."""
    n = (8, 5)
    rng = np.random.default_rng(11)
    ux = 1.0 + 0.2 * rng.standard_normal(n)
    uy = 0.1 * rng.standard_normal(n)
    uout = 1.0 + 0.2 * rng.standard_normal(n[1])
    U0 = 1.3
    u, uo, lo, hi, U = _channel(n, ux, uy, uout, U0)
    _, Rout = M.rhs(u, uo, lo, hi, U, 0.02)
    dt = 1.0 / U0
    np.testing.assert_allclose(uout + dt * Rout, ux[-1], rtol=0, atol=1e-14)


@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_outflow_ghosts_extend_an_x_independent_field(sign):
    """A field that does not vary along x (uniform u_x, tangential v(y))
    must see the same x-fluxes at the exit as in the middle of the channel:
    the zero-gradient ghosts beyond the outflow face extend it unchanged.
    With sign = -1 the flow runs back in through the exit, so the upwind
    stencil reaches the second ghost layer."""
    n = (12, 8)
    y = np.arange(n[1], dtype=float)
    ux = np.full(n, sign * 0.9)
    uy = np.ones(n[0])[:, None] * (0.3 * np.sin(2 * np.pi * y / n[1]) + 0.1 * np.cos(
        4 * np.pi * y / n[1]))[None, :]
    uout = np.full(n[1], sign * 0.9)
    u, uo, lo, hi, U = _channel(n, ux, uy, uout, sign * 0.9)
    R, Rout = M.rhs(u, uo, lo, hi, U, 0.03)
    mid = n[0] // 2
    for i in range(mid, n[0]):
        np.testing.assert_allclose(R[1][i], R[1][mid], rtol=0, atol=1e-14)
        np.testing.assert_allclose(R[0][i], R[0][mid], rtol=0, atol=1e-14)
    np.testing.assert_allclose(Rout, 0.0, atol=1e-15)


def _perturbed_channel(n, seed, bc_y):
    """Channel state with a non-uniform outlet: smooth interior perturbation
    of a uniform stream plus an outflow plane that does not carry the
    inflow flux."""
    rng = np.random.default_rng(seed)
    X = np.meshgrid(*[np.arange(m, dtype=float) for m in n], indexing="ij")
    ky = 2 * np.pi / n[1]
    ux = 1.0 + 0.15 * np.sin(ky * (X[1] + 0.5)) * np.exp(-((X[0] - 0.7 * n[0]) / 4.0) ** 2)
    uy = 0.1 * np.cos(ky * X[1]) * np.exp(-((X[0] + 0.5 - 0.7 * n[0]) / 4.0) ** 2)
    ux[0] = 1.0
    if bc_y == WALL:
        uy[:, 0] = 0.0
    uout = 1.0 + 0.2 * np.sin(ky * (np.arange(n[1]) + 0.5)) + 0.05 + 0.01 * rng.standard_normal(
        n[1])
    return ux, uy, uout


@pytest.mark.parametrize("bc_y", [PERIODIC, WALL])
def test_step_balances_exit_flux_and_leaves_a_divergence_free_field(bc_y):
    """Global mass conservation: the discrete divergence telescopes to
    (exit flux - inflow flux), so the pressure system with Neumann
    boundaries is solvable only if the two balance.  After a step from a
    state whose outlet carries 5 % too much flux: the outflow plane carries
    the inflow flux exactly, the projection right-hand side sums to zero over
    the active cells, and a tight solve leaves max |div u| <= 1e-10."""
    n = (24, 12)
    ux, uy, uout = _perturbed_channel(n, 3, bc_y)
    sim = S.Sim(n, [INFLOW, bc_y], [OUTFLOW, bc_y], (1.0, 0.0), 0.02, tol=1e-13,
                max_vcycles=300)
    sim.u = [ux, uy]
    sim._set_boundary(sim.u)
    sim.uout = uout
    dt = 0.3
    # one predictor stage by hand, to see the right-hand side it solves
    R, Rout = M.rhs(sim.u, sim.uout, sim.bc_lo, sim.bc_hi, sim.U, sim.nu)
    f = sim._set_boundary([sim.u[i] + dt * R[i] for i in range(2)])
    fout = M.exit_flux_correct(f, sim.uout + dt * Rout, sim.bc_lo, sim.bc_hi)
    assert fout.sum() == pytest.approx(f[0][0].sum(), rel=1e-14)
    sigma = S.divergence(f, fout, sim.bc_lo, sim.bc_hi, sim.U)
    assert abs(sigma.sum()) <= 1e-12 * np.abs(sigma).sum()
    assert np.ptp(fout - (sim.uout + dt * Rout)) < 1e-14       # a uniform shift
    sim.step(dt)
    assert sim.uout.sum() == pytest.approx(sim.u[0][0].sum(), rel=1e-14)
    div = S.divergence(sim.u, sim.uout, sim.bc_lo, sim.bc_hi, sim.U)
    assert np.abs(div).max() <= 1e-10


def test_perturbation_is_carried_out_through_the_exit():
    """A y-varying disturbance of the outlet leaves the domain with the
    stream: after the flow has crossed the last cells many times the
    outflow plane is uniform to a small fraction of the initial disturbance.
    A frozen plane (no convective rule) keeps its shape; a reversed rule is
    unstable and grows."""
    n = (24, 12)
    ux, uy, uout = _perturbed_channel(n, 5, PERIODIC)
    ux[:] = 1.0
    uy[:] = 0.0
    sim = S.Sim(n, [INFLOW, PERIODIC], [OUTFLOW, PERIODIC], (1.0, 0.0), 0.02, tol=1e-10)
    sim.u = [ux, uy]
    sim.uout = uout
    amp0 = np.ptp(uout)
    for _ in range(30):
        sim.step()
    assert np.ptp(sim.uout) < 0.05 * amp0


def test_cfl_takes_the_largest_per_cell_outflow_total():
    """Hand-worked per-cell outflow totals on a non-uniform periodic field.
    Cell A = (5, 2, 3) at the upper x boundary: its upper x face wraps to
    face 0.  Its faces: u_x lower -0.3 (out), upper +0.5 (out); u_y lower
    -0.2 (out), upper +0.1 (out); u_z lower +0.4 (in), upper +0.05 (out):
    total 0.8 + 0.3 + 0.05 = 1.15.  Elsewhere a lone u_x = 0.95 face gives
    its lower neighbour 0.95.  dt = cfl / (1.15 + 2 d nu)."""
    n = (6, 5, 7)
    per = [PERIODIC] * 3
    u = [np.zeros(n) for _ in range(3)]
    A = (5, 2, 3)
    u[0][5, 2, 3] = -0.3
    u[0][0, 2, 3] = 0.5                       # upper x face of A (wrapped)
    u[1][5, 2, 3] = -0.2
    u[1][5, 3, 3] = 0.1
    u[2][5, 2, 3] = 0.4
    u[2][5, 2, 4] = 0.05
    u[0][2, 0, 0] = 0.95
    nu = 0.01
    dt = M.cfl_dt(u, None, per, per, (0, 0, 0), nu, 0.5)
    assert dt == pytest.approx(0.5 / (1.15 + 6 * nu), rel=1e-14)
    assert A[0] == n[0] - 1


def test_cfl_counts_the_outflow_plane():
    """Non-periodic x: the last cell's upper x face is the outflow plane.
    Last cell (7, 1): u_x lower -0.25 (out), outflow plane +0.6 (out),
    u_y lower -0.1 (out), upper -0.3 (in): total 0.95; the inflow face
    (U = 0.5) gives the first cell at most 0.5 + its other outflows."""
    n = (8, 4)
    u = [np.full(n, 0.0), np.zeros(n)]
    u[0][0] = 0.5
    u[0][7, 1] = -0.25
    u[1][7, 1] = -0.1
    u[1][7, 2] = -0.3
    uout = np.zeros(4)
    uout[1] = 0.6
    nu = 0.005
    dt = M.cfl_dt(u, uout, [INFLOW, PERIODIC], [OUTFLOW, PERIODIC], (0.5, 0.0), nu, 0.5)
    assert dt == pytest.approx(0.5 / (0.95 + 4 * nu), rel=1e-14)
