"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module only builds inputs (analytic initial fields sampled on the
staggered grid, seeded random right-hand sides, configuration records).  It
holds none of the solver's arithmetic and imports neither the oracle nor the
GPU library.

Array convention: numpy float64 indexed a[x, y] / a[x, y, z] (axis i =
direction i).  The velocity component u_i sits on the lower i-face of each
cell, so it is sampled at x_i = I_i (times the grid spacing) and at cell
centres I_j + 1/2 in the other directions.
"""

import math

import numpy as np

PERIODIC, INFLOW, OUTFLOW, WALL = 0, 1, 2, 3


def staggered_coords(n, comp, h=1.0):
    axes = []
    for j, m in enumerate(n):
        c = np.arange(m, dtype=np.float64)
        if j != comp:
            c = c + 0.5
        axes.append(c * h)
    return np.meshgrid(*axes, indexing="ij")


def tgv3d(N, Re=1600.0):
    """Triply periodic 3D Taylor-Green vortex on [0, 2 pi)^3 with N cells a side.

    u = sin x cos y cos z, v = -cos x sin y cos z, w = 0 (unit velocity scale).
    Returns (u, v, w, nu_grid) with nu_grid = (N / 2 pi) / Re.
    """
    h = 2.0 * math.pi / N
    n = (N, N, N)
    X = staggered_coords(n, 0, h)
    u = np.sin(X[0]) * np.cos(X[1]) * np.cos(X[2])
    X = staggered_coords(n, 1, h)
    v = -np.cos(X[0]) * np.sin(X[1]) * np.cos(X[2])
    w = np.zeros(n)
    return u, v, w, (N / (2.0 * math.pi)) / Re


def periodic_modes3d(n, seed=2304, modes=4):
    """Smooth triply periodic 3D velocity field on an n[0] x n[1] x n[2] grid of
    any shape: per component a sum of `modes` Fourier modes (wave numbers 1..2
    per direction, amplitudes N(0, 1), random phases; seeded), sampled at the
    staggered face positions.  Not divergence-free (a step projects it)."""
    rng = np.random.default_rng(seed)
    out = []
    for comp in range(3):
        X = staggered_coords(n, comp)
        f = np.zeros(tuple(n))
        for _ in range(modes):
            k = rng.integers(1, 3, size=3)
            ph = rng.uniform(0.0, 2.0 * math.pi, size=3)
            a = rng.standard_normal()
            term = np.full(tuple(n), a)
            for d in range(3):
                term = term * np.cos(2.0 * math.pi * k[d] * X[d] / n[d] + ph[d])
            f += term
        out.append(f)
    return out


def tgv2d(N, nu_phys, t_phys=0.0):
    """2D Taylor-Green vortex on [0, 2 pi)^2 (closed-form solution at t_phys).

    u = sin x cos y F, v = -cos x sin y F, p = (cos 2x + cos 2y) F^2 / 4,
    F = exp(-2 nu t).  Returns (u, v, p, nu_grid) in grid units (velocity scale
    1, nu_grid = nu_phys N / 2 pi); p is sampled at cell centres.
    """
    h = 2.0 * math.pi / N
    n = (N, N)
    F = math.exp(-2.0 * nu_phys * t_phys)
    X = staggered_coords(n, 0, h)
    u = np.sin(X[0]) * np.cos(X[1]) * F
    X = staggered_coords(n, 1, h)
    v = -np.cos(X[0]) * np.sin(X[1]) * F
    xc = (np.arange(N) + 0.5) * h
    XC, YC = np.meshgrid(xc, xc, indexing="ij")
    p = 0.25 * (np.cos(2 * XC) + np.cos(2 * YC)) * F * F
    return u, v, p, nu_phys * N / (2.0 * math.pi)


def random_rhs(n, seed=2304):
    """i.i.d. N(0, 1) right-hand side, FP64, from numpy's default_rng(seed)."""
    return np.random.default_rng(seed).standard_normal(tuple(n))


def cylinder_config():
    """2D flow past a circle: 128 x 64, D = 16 at (32, 32), U = 1, Re = 250."""
    D = 16.0
    return dict(n=(128, 64), bc_lo=[INFLOW, WALL], bc_hi=[OUTFLOW, WALL],
                U=(1.0, 0.0), nu=1.0 * D / 250.0,
                body=dict(centre=(32.0, 32.0), radius=D / 2), levels=4,
                tol=1e-8, cfl=0.5, steps=100)


def sphere_flow_config(offset=(0.0, 0.0, 0.0)):
    """3D flow past a sphere: 128 x 64 x 64, r = 8 at (32, 32, 32), Re = 100."""
    r = 8.0
    c = tuple(32.0 + o for o in offset)
    return dict(n=(128, 64, 64), bc_lo=[INFLOW, WALL, WALL], bc_hi=[OUTFLOW, WALL, WALL],
                U=(1.0, 0.0, 0.0), nu=1.0 * 2 * r / 100.0,
                body=dict(centre=c, radius=r), levels=0, tol=1e-8, cfl=0.5, steps=50)


def donut_config(p=4, Re=1000.0):
    """Flow past a torus (the donut of Sec. 3): N = (2^(p+1), 2^p, 2^p), inflow U = 1
    in x, convective outflow, free-slip side walls.  The paper gives no radii: the
    torus axis is the x direction through (N_x/4, N_y/2, N_z/2), major radius
    R = N_y/4, tube radius R/4, Re on the major diameter 2R."""
    m = 2 ** p
    R = m / 4.0
    return dict(n=(2 * m, m, m), bc_lo=[INFLOW, WALL, WALL], bc_hi=[OUTFLOW, WALL, WALL],
                U=(1.0, 0.0, 0.0), nu=2.0 * R / Re,
                body=dict(kind="torus", centre=(m / 2.0, m / 2.0, m / 2.0), radius=R,
                          radius2=R / 4.0),
                levels=0, tol=1e-5, cfl=0.5)


def poisson_sphere_config(n=(256, 256, 256), radius=32.0):
    """Neumann box with a centred sphere (BDIM coefficients), N(0,1) RHS."""
    return dict(n=tuple(n), bc_lo=[WALL] * 3, bc_hi=[WALL] * 3,
                body=dict(centre=tuple(m / 2.0 for m in n), radius=radius))
