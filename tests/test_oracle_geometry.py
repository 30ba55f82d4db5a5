"""Pins of the BDIM geometry oracle (closed forms and invariants, no GPU)."""

import math

import numpy as np
import pytest

from oracle import geometry as G
from oracle.grid import PERIODIC, WALL


def test_moment_closed_form_values():
    assert G.mu0(0.0) == pytest.approx(0.5, abs=1e-15)
    assert G.mu0(1.0) == 1.0 and G.mu0(-1.0) == 0.0
    assert G.mu0(5.0) == 1.0 and G.mu0(-5.0) == 0.0
    assert G.mu1(0.0) == pytest.approx(0.25 - 1.0 / math.pi ** 2, abs=1e-15)
    assert G.mu1(0.999999) == pytest.approx(0.0, abs=1e-10)
    assert G.mu1(-0.999999) == pytest.approx(0.0, abs=1e-10)
    assert G.mu1(2.0) == 0.0
    # half-width scaling: mu1 scales with eps, mu0 depends on d/eps only
    assert G.mu1(0.0, eps=2.0) == pytest.approx(2.0 * (0.25 - 1.0 / math.pi ** 2), abs=1e-15)
    assert G.mu0(0.6, eps=2.0) == pytest.approx(G.mu0(0.3), abs=1e-15)


def test_kernel_is_normalised_and_moments_integrate_it():
    s = np.linspace(-1.0, 1.0, 200001)
    k = G.kernel(s)
    w = np.full_like(s, s[1] - s[0])
    w[0] *= 0.5
    w[-1] *= 0.5
    assert np.sum(k * w) == pytest.approx(1.0, abs=1e-9)
    # mu0(d) = int_{-1}^{d} K,  mu1(d) = int_d^{1} s K(s) ds, checked by quadrature
    for d in (-0.7, -0.2, 0.0, 0.35, 0.9):
        m = s <= d
        assert np.sum((k * w)[m]) == pytest.approx(float(G.mu0(d)), abs=2e-5)
        m = s >= d
        assert np.sum((s * k * w)[m]) == pytest.approx(float(G.mu1(d)), abs=2e-5)


def test_moment_derivatives_match_kernel():
    d = np.linspace(-0.95, 0.95, 39)
    h = 1e-6
    dmu0 = (G.mu0(d + h) - G.mu0(d - h)) / (2 * h)
    dmu1 = (G.mu1(d + h) - G.mu1(d - h)) / (2 * h)
    np.testing.assert_allclose(dmu0, G.kernel(d), atol=1e-8)
    np.testing.assert_allclose(dmu1, -d * G.kernel(d), atol=1e-8)


def test_mu0_is_c2_at_band_edges():
    h = 1e-4
    for e in (-1.0, 1.0):
        # value, slope and curvature continuous across the edge of the band
        left = G.mu0(np.array([e - 2 * h, e - h, e]))
        right = G.mu0(np.array([e, e + h, e + 2 * h]))
        d1l = (left[2] - left[1]) / h
        d1r = (right[1] - right[0]) / h
        assert abs(d1l - d1r) < 1e-6
        d2l = (left[2] - 2 * left[1] + left[0]) / h ** 2
        d2r = (right[2] - 2 * right[1] + right[0]) / h ** 2
        assert abs(d2l - d2r) < 1e-2


@pytest.mark.parametrize("radius", [6.0, 12.0])
def test_excluded_volume_matches_circle_and_sphere(radius):
    n2 = (64, 64)
    est = G.body_volume_estimate(n2, dict(centre=(32.3, 31.7), radius=radius))
    exact = G.exact_body_volume(2, radius)
    assert abs(est - exact) / exact < 0.6 / radius ** 2 + 1e-3
    n3 = (40, 40, 40)
    est = G.body_volume_estimate(n3, dict(centre=(20.2, 19.9, 20.4), radius=radius))
    exact = G.exact_body_volume(3, radius)
    assert abs(est - exact) / exact < 1.5 / radius ** 2 + 2e-3


def test_measure_limits_and_boundary_faces():
    n = (24, 20, 16)
    body = dict(centre=(12.0, 10.0, 8.0), radius=5.0)
    mu0, mu1n, L = G.measure(n, [WALL, PERIODIC, WALL], body)
    for i in range(3):
        X = G.face_centres(n, i)
        dist, _ = G.sphere_sdf(X, body["centre"], body["radius"])
        deep, far = dist <= -1.0, dist >= 1.0
        assert np.all(mu0[i][deep] == 0.0) and np.all(mu0[i][far] == 1.0)
        for j in range(3):
            assert np.all(mu1n[i][j][deep | far] == 0.0)
    # non-periodic lower boundary faces carry L = 0, periodic ones do not
    assert np.all(L[0][0] == 0.0) and np.all(L[2][:, :, 0] == 0.0)
    assert np.all(L[1][:, 0, :] == mu0[1][:, 0, :])
    # the normal is a unit vector wherever mu1 is non-zero
    m = G.mu1(G.sphere_sdf(G.face_centres(n, 0), body["centre"], body["radius"])[0])
    nrm = np.sqrt(sum(mu1n[0][j] ** 2 for j in range(3)))
    np.testing.assert_allclose(nrm, np.abs(m), atol=1e-15)


@pytest.mark.parametrize("a,R,n", [(3.0, 9.0, (16, 32, 32)), (6.0, 12.0, (24, 48, 48))])
def test_torus_excluded_volume_matches_pappus(a, R, n):
    # sum(1 - mu0) against 2 pi^2 R a^2; the BDIM smoothing of the curved tube
    # leaves a relative excess of about 0.13 / a^2 (cell units)
    body = dict(kind="torus", centre=(n[0] / 2 + 0.2, n[1] / 2 - 0.1, n[2] / 2 + 0.3),
                radius=R, radius2=a)
    est = G.body_volume_estimate(n, body)
    exact = G.exact_torus_volume(R, a)
    assert abs(est - exact) / exact < 0.2 / a ** 2 + 1e-3


def test_torus_sdf_exact_points_and_normals():
    c, R, a = (10.0, 20.0, 21.0), 8.0, 3.0
    pts = {  # point relative to c: (distance, outward normal)
        (0.0, 0.0, 0.0): (R - a, (0.0, 0.0, 0.0)),          # on the axis
        (3.5, R, 0.0): (3.5 - a, (1.0, 0.0, 0.0)),          # beside the tube, along x
        (0.0, 0.0, R + 5.0): (5.0 - a, (0.0, 0.0, 1.0)),    # outside the ring
        (0.0, R - 2.0, 0.0): (2.0 - a, (0.0, -1.0, 0.0)),   # inside the tube, towards the hole
        (0.0, -(R + 1.0), 0.0): (1.0 - a, (0.0, -1.0, 0.0)),
    }
    X = [np.array([c[j] + p[j] for p in pts]) for j in range(3)]
    d, nrm = G.torus_sdf(X, c, R, a)
    for m, (p, (dx, nx)) in enumerate(pts.items()):
        assert abs(d[m] - dx) < 1e-12, p
        assert np.allclose([nrm[j][m] for j in range(3)], nx, atol=1e-12), p


def test_torus_normal_is_unit_gradient_of_distance():
    rng = np.random.default_rng(7)
    c, R, a = (0.0, 0.0, 0.0), 6.0, 2.0
    X = [rng.uniform(-10.0, 10.0, 400) for _ in range(3)]
    d, nrm = G.torus_sdf(X, c, R, a)
    h = 1e-5
    for j in range(3):
        Xp = [x + (h if k == j else 0.0) for k, x in enumerate(X)]
        Xm = [x - (h if k == j else 0.0) for k, x in enumerate(X)]
        fd = (G.torus_sdf(Xp, c, R, a)[0] - G.torus_sdf(Xm, c, R, a)[0]) / (2 * h)
        assert np.max(np.abs(fd - nrm[j])) < 1e-6
    assert np.allclose(sum(x * x for x in nrm), 1.0)


def test_measure_accepts_a_torus_and_limits_hold():
    n = (16, 24, 24)
    body = dict(kind="torus", centre=(8.0, 12.0, 12.0), radius=6.0, radius2=2.5)
    mu0, mu1n, L = G.measure(n, [WALL] * 3, body)
    # the tube's centre circle is deep inside, the axis far outside
    assert mu0[0][8, 12 + 6, 12] == 0.0 and mu0[0][8, 12, 12] == 1.0
    assert all(np.all((m >= 0.0) & (m <= 1.0)) for m in mu0)
    assert np.all(L[0][0] == 0.0) and np.all(L[1][:, 0] == 0.0)
