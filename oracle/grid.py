"""Grid conventions, boundary codes and shift helpers (oracle; test-only).

The paper solves on a uniform Cartesian background grid (Sec. 2).  Spacing is
one grid unit.  Boundary codes per domain face:

  PERIODIC  wrap-around (must be set on both faces of a direction)
  INFLOW    prescribed uniform velocity U (lower x face in the configs)
  OUTFLOW   convective outflow (upper x face)
  WALL      free-slip wall (zero normal velocity, zero tangential stress)

For the pressure every non-periodic face is homogeneous Neumann, carried by a
zero Poisson coefficient on the boundary face.
"""

import numpy as np

PERIODIC, INFLOW, OUTFLOW, WALL = 0, 1, 2, 3


def is_periodic(bc_lo, axis):
    return bc_lo[axis] == PERIODIC


def shift(a, axis, k, periodic, fill=0.0):
    """b[I] = a[I + k*delta_axis]; wraps if periodic, else `fill` outside."""
    if periodic:
        return np.roll(a, -k, axis=axis)
    b = np.full_like(a, fill)
    n = a.shape[axis]
    src = [slice(None)] * a.ndim
    dst = [slice(None)] * a.ndim
    if k >= 0:
        src[axis] = slice(k, n)
        dst[axis] = slice(0, n - k)
    else:
        src[axis] = slice(0, n + k)
        dst[axis] = slice(-k, n)
    b[tuple(dst)] = a[tuple(src)]
    return b


def auto_levels(n, levels=0):
    """Number of multigrid levels.

    READING (the paper gives no GMG constants, Sec. 2): coarsen by two in every
    direction while every direction is even and the coarse grid keeps at least
    4 cells per direction; an explicit level count overrides that limit but a
    level is only formed when every direction is even.
    """
    n = list(n)
    count = 1
    while True:
        if levels and count >= levels:
            break
        if any(m % 2 for m in n):
            break
        if not levels and any(m // 2 < 4 for m in n):
            break
        n = [m // 2 for m in n]
        count += 1
    return count


def level_shapes(n, nlev):
    shapes = [tuple(n)]
    for _ in range(nlev - 1):
        shapes.append(tuple(m // 2 for m in shapes[-1]))
    return shapes
