"""Body immersion geometry: SDF -> BDIM moments and Poisson coefficients (oracle).

Paper, Sec. 2: the immersed body is given by a signed-distance function; the
Boundary Data Immersion Method (BDIM) enforces its boundary condition and
modifies the pressure-Poisson matrix.  The paper does not print the BDIM
formulas, so the following READINGS (first-order BDIM with a cosine kernel)
are the contract:

  * kernel K(s) = (1 + cos(pi s / eps)) / (2 eps) for |s| < eps, else 0, with
    half-width eps = 1 cell;
  * zeroth moment mu0(d) = integral of K from -eps to d
                         = (1 + r + sin(pi r)/pi) / 2,  r = d/eps, |r| < 1;
                           1 for r >= 1, 0 for r <= -1;
  * first moment  mu1(d) = integral of s K(s) from d to eps
                         = eps [ (1 - r^2)/4 - r sin(pi r)/(2 pi)
                                 - (1 + cos(pi r))/(2 pi^2) ],  |r| < 1; else 0;
  * sphere / circle SDF d(x) = |x - c| - R (positive in the fluid), outward
    normal n = (x - c)/|x - c| (zero at the centre);
  * torus (the donut of Sec. 3, 3D), axis along x through c, major radius R,
    tube radius a: with rho the distance of x - c from the axis,
    d(x) = sqrt((x-c)_x^2 + (rho - R)^2) - a, n = grad d (the tube's own
    radial direction; zero on the tube's centre circle or the axis);
  * per face (component i, cell I), evaluated at the face centre:
      mu0_i = mu0(d),  (mu1 n)_ij = mu1(d) n_j,  L_i = mu0_i,
    and L_i = 0 on non-periodic domain-boundary faces (Neumann pressure).

Moving bodies.  Sec. 2 defines a body by its signed-distance function and a
coordinate map.  READING for rigid motion: the map takes x to the body frame
xi = R(t)^T (x - X(t)), so d(x, t) = d0(xi), with
  X(t) = c + V t + A sin(omega t)   (centre path: drift plus oscillation),
  R(t) = rotation by |Omega| t about Omega (a constant spin),
and the body velocity is the map's velocity field,
  V_b(x, t) = dX/dt + Omega x (x - X(t)),  dX/dt = V + A omega cos(omega t),
whose gradient is dV_b,i/dx_j = eps_ikj Omega_k.  Spin is read for spheres
and circles only (their SDF does not change under rotation about the
centre; only V_b does); a scalar spin turns about z.  The body is
re-measured at every step.

Pins: closed-form values of mu0/mu1 at 0 and +-eps, derivative identities
mu0' = K, mu1' = -d K (finite differences), the excluded volume
sum(1 - mu0) -> body volume (sphere 4/3 pi R^3, torus 2 pi^2 R a^2), the
deep-inside / far-outside limits, and for the torus SDF: exact distances at
points whose nearest surface point is known, |n| = 1, n = finite-difference
gradient of d.
"""

import math

import numpy as np

from .grid import PERIODIC


def kernel(d, eps=1.0):
    d = np.asarray(d, dtype=np.float64)
    r = d / eps
    inside = np.abs(r) < 1.0
    return np.where(inside, (1.0 + np.cos(np.pi * r)) / (2.0 * eps), 0.0)


def mu0(d, eps=1.0):
    d = np.asarray(d, dtype=np.float64)
    r = d / eps
    val = 0.5 * (1.0 + r + np.sin(np.pi * r) / np.pi)
    return np.where(r >= 1.0, 1.0, np.where(r <= -1.0, 0.0, val))


def mu1(d, eps=1.0):
    d = np.asarray(d, dtype=np.float64)
    r = d / eps
    val = eps * ((1.0 - r * r) / 4.0 - r * np.sin(np.pi * r) / (2.0 * np.pi)
                 - (1.0 + np.cos(np.pi * r)) / (2.0 * np.pi ** 2))
    return np.where(np.abs(r) < 1.0, val, 0.0)


def face_centres(n, comp):
    """Coordinates of the lower comp-faces of every cell, one array per axis."""
    d = len(n)
    axes = []
    for j in range(d):
        c = np.arange(n[j], dtype=np.float64)
        if j != comp:
            c = c + 0.5
        axes.append(c)
    return np.meshgrid(*axes, indexing="ij")


def cell_centres(n):
    axes = [np.arange(m, dtype=np.float64) + 0.5 for m in n]
    return np.meshgrid(*axes, indexing="ij")


def sphere_sdf(X, centre, radius):
    """Signed distance and outward unit normal of a sphere (circle in 2D)."""
    d = len(X)
    rel = [X[j] - centre[j] for j in range(d)]
    dist = np.sqrt(sum(r * r for r in rel))
    safe = np.where(dist > 0.0, dist, 1.0)
    normal = [np.where(dist > 0.0, r / safe, 0.0) for r in rel]
    return dist - radius, normal


def torus_sdf(X, centre, radius, radius2):
    """Signed distance and outward unit normal of a torus about the x axis."""
    rel = [X[j] - centre[j] for j in range(3)]
    rho = np.sqrt(rel[1] ** 2 + rel[2] ** 2)
    qr = rho - radius
    q = np.sqrt(rel[0] ** 2 + qr ** 2)
    qs = np.where(q > 0.0, q, 1.0)
    rs = np.where(rho > 0.0, rho, 1.0)
    radial = np.where(q > 0.0, qr / qs, 0.0)
    normal = [np.where(q > 0.0, rel[0] / qs, 0.0),
              np.where(rho > 0.0, radial * rel[1] / rs, 0.0),
              np.where(rho > 0.0, radial * rel[2] / rs, 0.0)]
    return q - radius2, normal


def is_moving(body):
    if body is None:
        return False
    keys = ("velocity", "amplitude", "spin")
    return any(np.any(np.asarray(body.get(k, 0.0), dtype=np.float64) != 0.0) for k in keys)


def _vec3(v):
    a = np.zeros(3)
    v = np.atleast_1d(np.asarray(v, dtype=np.float64))
    a[:v.size] = v
    return a


def _spin3(body):
    """Angular velocity as a 3-vector; a scalar spin is about z (2D bodies)."""
    w = np.asarray(body.get("spin", 0.0), dtype=np.float64)
    return np.array([0.0, 0.0, float(w)]) if w.ndim == 0 else _vec3(w)


def body_motion(body, t):
    """Centre X(t), translation velocity dX/dt and angular velocity Omega
    (3-vectors) of a rigidly moving body."""
    c = _vec3(body["centre"])
    V = _vec3(body.get("velocity", 0.0))
    A = _vec3(body.get("amplitude", 0.0))
    w = float(body.get("omega", 0.0))
    spin = _spin3(body)
    X = c + V * t + A * math.sin(w * t)
    Xdot = V + A * w * math.cos(w * t)
    return X, Xdot, spin


def body_at(body, t):
    """The body as placed at time t (its centre moved along the path)."""
    if body is None or not is_moving(body):
        return body
    X, _, _ = body_motion(body, t)
    out = dict(body)
    out["centre"] = tuple(X[:len(body["centre"])])
    return out


def body_velocity(X, body, t):
    """V_b(x, t) = dX/dt + Omega x (x - X(t)) at the points X (one array per axis)."""
    d = len(X)
    Xc, Xdot, W = body_motion(body, t)
    r = [X[j] - Xc[j] for j in range(d)] + [np.zeros_like(X[0])] * (3 - d)
    cross = [W[1] * r[2] - W[2] * r[1], W[2] * r[0] - W[0] * r[2], W[0] * r[1] - W[1] * r[0]]
    return [Xdot[i] + cross[i] for i in range(d)]


def body_velocity_gradient(body, d):
    """G_ij = dV_b,i / dx_j = eps_ikj Omega_k (constant for rigid motion)."""
    W = _spin3(body)
    G = np.array([[0.0, -W[2], W[1]], [W[2], 0.0, -W[0]], [-W[1], W[0], 0.0]])
    return G[:d, :d]


def body_sdf(X, body):
    """SDF and normal of a body dict: a sphere/circle, or kind="torus" (radius2 = tube)."""
    if body.get("kind", "sphere") == "torus":
        return torus_sdf(X, body["centre"], body["radius"], body["radius2"])
    return sphere_sdf(X, body["centre"], body["radius"])


def measure(n, bc_lo, body=None, eps=1.0, t=0.0):
    """BDIM moments and fine-level Poisson coefficients.

    body: None, dict(centre=(..), radius=R), or dict(kind="torus", centre, radius,
    radius2), optionally with motion (velocity, amplitude, omega, spin; the
    body is then measured where it is at time t).  Returns (mu0[i], mu1n[i][j],
    L[i]) with every array shaped like the grid.  Without a body mu0 = 1,
    mu1n = 0.
    """
    d = len(n)
    body = body_at(body, t)
    m0, m1n, L = [], [], []
    for i in range(d):
        if body is None:
            a0 = np.ones(n)
            a1 = [np.zeros(n) for _ in range(d)]
        else:
            X = face_centres(n, i)
            dist, normal = body_sdf(X, body)
            a0 = mu0(dist, eps)
            m = mu1(dist, eps)
            a1 = [m * normal[j] for j in range(d)]
        Li = a0.copy()
        if bc_lo[i] != PERIODIC:
            idx = [slice(None)] * d
            idx[i] = 0
            Li[tuple(idx)] = 0.0
        m0.append(a0)
        m1n.append(a1)
        L.append(Li)
    return m0, m1n, L


def body_volume_estimate(n, body, eps=1.0):
    """sum over cells of (1 - mu0(d_cell)): the excluded volume seen by BDIM."""
    X = cell_centres(n)
    dist, _ = body_sdf(X, body)
    return float(np.sum(1.0 - mu0(dist, eps)))


def exact_body_volume(d, radius):
    return math.pi * radius ** 2 if d == 2 else 4.0 / 3.0 * math.pi * radius ** 3


def exact_torus_volume(radius, radius2):
    """Pappus: the tube's cross-section pi a^2 swept round a circle of length 2 pi R."""
    return 2.0 * math.pi ** 2 * radius * radius2 ** 2
