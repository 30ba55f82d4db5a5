"""Pins of the convection-diffusion / CFL / BDIM / BC oracle (no GPU)."""

import numpy as np
import pytest

from oracle import geometry as G
from oracle import momentum as M
from oracle.grid import INFLOW, OUTFLOW, PERIODIC, WALL


def test_interpolant_is_third_order_on_cell_averages():
    """kappa = 1/3 reproduces the face value of a quadratic from its cell
    averages (monotone data, so the limiter is inactive)."""
    # q(x) = 1 + 2x + 0.3x^2 on cells [-2,-1], [-1,0], [0,1]; face at x = 0
    avg = lambda a, b: (b - a) + (b * b - a * a) + 0.1 * (b ** 3 - a ** 3)  # noqa: E731
    a, c, b = avg(-2, -1), avg(-1, 0), avg(0, 1)
    assert M.face_value(np.array(a), np.array(c), np.array(b)) == pytest.approx(1.0, abs=1e-14)


def test_limiter_is_tvd_and_first_order_at_extrema():
    rng = np.random.default_rng(0)
    a, c, b = rng.standard_normal((3, 10000))
    phi = M.face_value(a, c, b)
    lo, hi = np.minimum(c, b), np.maximum(c, b)
    assert np.all(phi >= lo - 1e-15) and np.all(phi <= hi + 1e-15)
    ext = (c - a) * (b - c) <= 0.0                      # c is a local extremum
    np.testing.assert_array_equal(phi[ext], c[ext])
    mono = (a < c) & (c < b)                            # normalised TVD bound
    assert np.all(phi[mono] - c[mono] <= np.minimum(c - a, b - c)[mono] + 1e-15)


def _rand_periodic_u(rng, n):
    return [rng.standard_normal(n) for _ in n]


@pytest.mark.parametrize("n", [(12, 10), (8, 6, 10)])
def test_free_stream_preservation_and_conservation(n):
    d = len(n)
    per = [PERIODIC] * d
    U = tuple(np.linspace(-0.7, 0.9, d))
    u = [np.full(n, U[i]) for i in range(d)]
    R, _ = M.rhs(u, None, per, per, U, 0.03)
    for Ri in R:
        assert np.abs(Ri).max() < 1e-15
    u = _rand_periodic_u(np.random.default_rng(1), n)
    R, _ = M.rhs(u, None, per, per, U, 0.03)
    for Ri in R:
        assert abs(Ri.sum()) < 1e-12 * np.abs(Ri).sum()


def test_mirror_symmetry_of_the_flux():
    n = (10, 8, 6)
    per = [PERIODIC] * 3
    rng = np.random.default_rng(2)
    u = _rand_periodic_u(rng, n)
    # mirror x -> -x: cell I -> n-1-I, lower x-face I -> (n - I) mod n, u_x -> -u_x
    def mirror(v):
        w = [None] * 3
        w[0] = -np.roll(v[0][::-1], 1, axis=0)
        w[1] = v[1][::-1]
        w[2] = v[2][::-1]
        return w
    R, _ = M.rhs(u, None, per, per, (0, 0, 0), 0.05)
    Rm, _ = M.rhs(mirror(u), None, per, per, (0, 0, 0), 0.05)
    for a, b in zip(mirror(R), Rm):
        np.testing.assert_allclose(a, b, atol=1e-13)


def test_pure_diffusion_is_the_discrete_laplacian():
    n = (9, 7)
    per = [PERIODIC] * 2
    rng = np.random.default_rng(3)
    # with u_y = 0 and u_x independent of x the convective fluxes vanish
    u = [np.repeat(rng.standard_normal((1, 7)), 9, axis=0), np.zeros(n)]
    nu = 0.2
    R, _ = M.rhs(u, None, per, per, (0, 0), nu)
    lap = np.roll(u[0], 1, 1) - 2 * u[0] + np.roll(u[0], -1, 1)
    np.testing.assert_allclose(R[0], nu * lap, atol=1e-14)
    assert np.abs(R[1]).max() < 1e-15


def test_cfl_closed_form_for_uniform_flow():
    n = (8, 8, 8)
    per = [PERIODIC] * 3
    for U in (1.0, -2.5):
        u = [np.full(n, U), np.zeros(n), np.zeros(n)]
        dt = M.cfl_dt(u, None, per, per, (U, 0, 0), 0.01, 0.5)
        assert dt == 0.5 / (abs(U) + 6 * 0.01)
    with pytest.raises(ValueError):
        M.cfl_dt([np.zeros(n)] * 3, None, per, per, (0, 0, 0), 0.0, 0.5)


def test_ghost_rules():
    n = (6, 5)
    u = [np.arange(30.0).reshape(n) + 1.0, np.arange(30.0).reshape(n) * 2 + 1.0]
    uout = np.full(5, 7.0)
    P = M.pad_velocity(u, uout, [INFLOW, WALL], [OUTFLOW, WALL], (1.5, 0.0))
    k = M.PAD
    assert np.all(P[0][k - 1, k:k + 5] == 1.5) and np.all(P[1][k - 2, k:k + 5] == 0.0)
    assert np.all(P[0][k + 6, k:k + 5] == 7.0) and np.all(P[0][k + 7, k:k + 5] == 7.0)
    assert np.all(P[1][k + 6, k:k + 5] == u[1][5])               # zero-gradient tangential
    # free-slip y walls: normal odd about the wall face, tangential even
    np.testing.assert_array_equal(P[1][k:k + 6, k - 1], -u[1][:, 1])
    np.testing.assert_array_equal(P[1][k:k + 6, k + 5], 0.0)
    np.testing.assert_array_equal(P[1][k:k + 6, k + 6], -u[1][:, 4])
    np.testing.assert_array_equal(P[0][k:k + 6, k - 1], u[0][:, 0])
    np.testing.assert_array_equal(P[0][k:k + 6, k - 2], u[0][:, 1])
    np.testing.assert_array_equal(P[0][k:k + 6, k + 5], u[0][:, 4])


def test_bdim_limits():
    n = (20, 20)
    body = dict(centre=(10.0, 10.0), radius=5.0)
    mu0, mu1n, _ = G.measure(n, [PERIODIC] * 2, body)
    rng = np.random.default_rng(4)
    f = [rng.standard_normal(n) for _ in range(2)]
    us = M.bdim(f, mu0, mu1n, [PERIODIC] * 2, [PERIODIC] * 2, (0, 0))
    for i in range(2):
        X = G.face_centres(n, i)
        dist, _ = G.sphere_sdf(X, body["centre"], body["radius"])
        assert np.all(us[i][dist <= -1.0] == 0.0)
        np.testing.assert_array_equal(us[i][dist >= 1.0], f[i][dist >= 1.0])


def test_bdim_blend_equals_kernel_convolution_for_linear_wall_profile():
    """First-order BDIM is the kernel-weighted average of the fluid velocity
    across the band.  For a velocity that grows linearly with the distance d
    from the wall (f = d) the expansion is exact: the convolution
    int_{-eps}^{d} K(s) (d - s) ds equals d mu0(d) + mu1(d); check the blend
    against that quadrature (the residual is the O(1/R) curvature of |x - c|
    and the central difference)."""
    n = (64, 64)
    body = dict(centre=(31.6, 32.3), radius=20.0)
    mu0, mu1n, _ = G.measure(n, [PERIODIC] * 2, body)
    f, dist = [], []
    for i in range(2):
        X = G.face_centres(n, i)
        dd, _ = G.sphere_sdf(X, body["centre"], body["radius"])
        dist.append(dd)
        f.append(dd.copy())
    us = M.bdim(f, mu0, mu1n, [PERIODIC] * 2, [PERIODIC] * 2, (0, 0))
    s = np.linspace(-1.0, 1.0, 4001)
    for i in range(2):
        band = np.abs(dist[i]) < 1.0
        for dv, got in zip(dist[i][band][::7], us[i][band][::7]):
            m = s <= dv
            integrand = G.kernel(s[m]) * (dv - s[m])
            conv = np.trapezoid(integrand, s[m]) if m.sum() > 1 else 0.0
            assert got == pytest.approx(conv, abs=0.02)
