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
