"""Convection-diffusion, CFL time step, BDIM blend and boundary rules (oracle).

Paper, Sec. 2: third-order finite-volume convection-diffusion with implicit
LES (the scheme's own dissipation, no subgrid model), explicit adaptive time
stepping, and BDIM immersion.  Sec. 3 / Table 2 name the routines convdiff!,
BDIM!, BC! and CFL!.  The formulas are not printed, so these READINGS are the
contract:

Flux (convdiff!).  For the i-momentum control volume of face I, the flux
through its lower j-face is
    F_ij(I) = ubar * phi - nu (u_i(I) - u_i(I - delta_j)),
    ubar    = (u_j(I) + u_j(I - delta_i)) / 2,
with phi the upwind-biased face value of u_i between u_i(I-delta_j) and
u_i(I): for ubar >= 0 take upwind c = u_i(I-delta_j), far-upwind
a = u_i(I-2 delta_j), downwind b = u_i(I); otherwise mirror
(c = u_i(I), a = u_i(I+delta_j), b = u_i(I-delta_j)).  The third-order
kappa = 1/3 interpolant (5c + 2b - a)/6 is bounded by the Koren TVD limiter:
phi = median((5c + 2b - a)/6, c, median(2c - a, c, b)).  At a local extremum
this returns c (first-order upwind), which is the implicit-LES dissipation.
R_i(I) = -sum_j [F_ij(I + delta_j) - F_ij(I)].

CFL!.  dt = cfl / (max_I sum_i [max(u_i(I+delta_i), 0) - min(u_i(I), 0)]
                   + 2 d nu),
the per-cell total outflow velocity plus the explicit viscous limit.

BDIM!.  u*_i = mu0_i f_i + (1 - mu0_i) V_b,i
               + sum_j (mu1 n)_ij [(f_i(I+delta_j) - f_i(I-delta_j))/2 - G_ij]
on interior faces: the first-order blend of the fluid and body velocities
with the normal-derivative correction mu1 d/dn (f - V_b), V_b the body
velocity at the face and G_ij = dV_b,i/dx_j (constant for rigid motion); a
body at rest has V_b = 0, G = 0.

BC!.  Ghost values with two layers per side:
  periodic wrap; INFLOW ghosts (all components) = U; free-slip WALL: normal
  component odd about the wall face (boundary face value 0), tangential
  components even about the wall; OUTFLOW (upper x): the boundary face carries
  its own unknown (a plane array `uout`) advanced by the convective rule
  d(uout)/dt = -U_x (uout - u_x(n-1)), ghosts beyond it zero-gradient.
  After each stage the outflow plane is shifted uniformly so that its total
  flux equals the inflow plane's (FP64 plane sums).
Boundary faces (index 0 of a non-periodic normal direction) are not updated;
they hold U_i (inflow) or 0 (wall).

Pins: free-stream preservation, discrete momentum conservation, mirror
symmetry, third-order exactness of the interpolant on cell averages of
quadratics, TVD bounds of the limiter, closed-form CFL for uniform flow,
deep-inside / far-outside BDIM limits.
"""

import numpy as np

from .grid import INFLOW, OUTFLOW, PERIODIC, WALL

PAD = 2


def median3(a, b, c):
    return np.maximum(np.minimum(a, b), np.minimum(np.maximum(a, b), c))


def face_value(a, c, b):
    """Limited third-order face value (upwind c, far-upwind a, downwind b)."""
    phik = (5.0 * c + 2.0 * b - a) / 6.0
    return median3(phik, c, median3(2.0 * c - a, c, b))


def _sl(axis, ndim, idx):
    s = [slice(None)] * ndim
    s[axis] = idx
    return tuple(s)


def pad_velocity(u, uout, bc_lo, bc_hi, U):
    """Padded copies (PAD ghost layers per side) of every velocity component.

    Index k of a padded axis holds grid index k - PAD.  Directions are filled
    one after another (x, y, z), each over the full padded extent of the
    directions before it, so corner ghosts are defined (they only feed
    boundary faces whose update is discarded).
    """
    d = len(u)
    n = u[0].shape
    out = []
    for c in range(d):
        P = np.zeros(tuple(m + 2 * PAD for m in n))
        P[tuple(slice(PAD, PAD + m) for m in n)] = u[c]
        for j in range(d):
            m = n[j]
            g = lambda k: _sl(j, d, PAD + k)          # noqa: E731  grid index k along j
            if bc_lo[j] == PERIODIC:
                for k in (-2, -1):
                    P[g(k)] = P[g(k + m)]
                for k in (m, m + 1):
                    P[g(k)] = P[g(k - m)]
                continue
            lo, hi = bc_lo[j], bc_hi[j]
            if c == j:                                 # normal component
                if lo == INFLOW:
                    P[g(-1)] = U[c]
                    P[g(-2)] = U[c]
                elif lo == WALL:
                    P[g(-1)] = -P[g(1 if m > 1 else 0)]
                    P[g(-2)] = -P[g(2 if m > 2 else 0)]
                else:
                    raise ValueError("unsupported lower boundary")
                if hi == OUTFLOW:
                    plane = uout if uout is not None else 0.0
                    P[g(m)] = _pad_plane(plane, j, n, d)
                    P[g(m + 1)] = P[g(m)]
                elif hi == WALL:
                    P[g(m)] = 0.0
                    P[g(m + 1)] = -P[g(max(m - 1, 0))]
                else:
                    raise ValueError("unsupported upper boundary")
            else:                                      # tangential component
                if lo == INFLOW:
                    P[g(-1)] = U[c]
                    P[g(-2)] = U[c]
                elif lo == WALL:
                    P[g(-1)] = P[g(0)]
                    P[g(-2)] = P[g(min(1, m - 1))]
                else:
                    raise ValueError("unsupported lower boundary")
                if hi == OUTFLOW:
                    P[g(m)] = P[g(m - 1)]
                    P[g(m + 1)] = P[g(m - 1)]
                elif hi == WALL:
                    P[g(m)] = P[g(m - 1)]
                    P[g(m + 1)] = P[g(max(m - 2, 0))]
                else:
                    raise ValueError("unsupported upper boundary")
        out.append(P)
    return out


def _pad_plane(plane, j, n, d):
    """Embed an interior plane (shape n without axis j) into the padded plane."""
    shp = [m + 2 * PAD for k, m in enumerate(n) if k != j]
    Q = np.zeros(shp)
    if np.isscalar(plane):
        Q[...] = plane
        return Q
    inner = tuple(slice(PAD, PAD + m) for k, m in enumerate(n) if k != j)
    Q[inner] = plane
    # zero-gradient extension into the corner ghosts of the plane
    for a in range(Q.ndim):
        m = plane.shape[a]
        for k in (-2, -1):
            Q[_sl(a, Q.ndim, PAD + k)] = Q[_sl(a, Q.ndim, PAD)]
        for k in (m, m + 1):
            Q[_sl(a, Q.ndim, PAD + k)] = Q[_sl(a, Q.ndim, PAD + m - 1)]
    return Q


def _view(P, n, offs):
    """Interior-shaped window of a padded array shifted by offs (per axis)."""
    return P[tuple(slice(PAD + o, PAD + o + m) for m, o in zip(n, offs))]


def _ext_view(P, n, offs, j):
    """Like _view but n_j + 1 entries along axis j (faces 0..n_j)."""
    sl = []
    for a, (m, o) in enumerate(zip(n, offs)):
        extra = 1 if a == j else 0
        sl.append(slice(PAD + o, PAD + o + m + extra))
    return P[tuple(sl)]


def rhs(u, uout, bc_lo, bc_hi, U, nu):
    """R(u) on every stored face (boundary faces included; callers mask them)
    and the outflow-plane tendency R_out (None without an outflow)."""
    d = len(u)
    n = u[0].shape
    Pd = pad_velocity(u, uout, bc_lo, bc_hi, U)
    R = []
    for i in range(d):
        Ri = np.zeros(n)
        for j in range(d):
            dj = [1 if a == j else 0 for a in range(d)]
            di = [1 if a == i else 0 for a in range(d)]
            # fluxes on lower j-faces for face index 0..n_j along j
            ui_0 = _ext_view(Pd[i], n, [0] * d, j)                          # u_i(I)
            ui_m1 = _ext_view(Pd[i], n, [-x for x in dj], j)                # u_i(I - dj)
            ui_m2 = _ext_view(Pd[i], n, [-2 * x for x in dj], j)            # u_i(I - 2dj)
            ui_p1 = _ext_view(Pd[i], n, dj, j)                              # u_i(I + dj)
            uj_0 = _ext_view(Pd[j], n, [0] * d, j)                          # u_j(I)
            uj_mi = _ext_view(Pd[j], n, [-x for x in di], j)                # u_j(I - di)
            ubar = 0.5 * (uj_0 + uj_mi)
            pos = ubar >= 0.0
            c = np.where(pos, ui_m1, ui_0)
            b = np.where(pos, ui_0, ui_m1)
            a = np.where(pos, ui_m2, ui_p1)
            F = ubar * face_value(a, c, b) - nu * (ui_0 - ui_m1)
            lo = F[_sl(j, d, slice(0, n[j]))]
            hi = F[_sl(j, d, slice(1, n[j] + 1))]
            Ri -= hi - lo
        R.append(Ri)
    Rout = None
    if bc_hi[0] == OUTFLOW:
        Rout = -U[0] * (uout - u[0][-1])
    return R, Rout


def boundary_face_mask(n, bc_lo, i):
    """True on stored faces of component i that are domain-boundary faces."""
    d = len(n)
    m = np.zeros(n, dtype=bool)
    if bc_lo[i] != PERIODIC:
        m[_sl(i, d, 0)] = True
    return m


def boundary_value(bc_lo, U, i):
    return U[i] if bc_lo[i] == INFLOW else 0.0


def cfl_dt(u, uout, bc_lo, bc_hi, U, nu, cfl):
    d = len(u)
    n = u[0].shape
    Pd = pad_velocity(u, uout, bc_lo, bc_hi, U)
    s = np.zeros(n)
    for i in range(d):
        di = [1 if a == i else 0 for a in range(d)]
        up = _view(Pd[i], n, di)
        s += np.maximum(up, 0.0) - np.minimum(u[i], 0.0)
    denom = float(s.max()) + 2.0 * d * nu
    if denom <= 0.0:
        raise ValueError("CFL: zero velocity and zero viscosity")
    return cfl / denom


def bdim(f, mu0, mu1n, bc_lo, bc_hi, U, fout=None, Vb=None, G=None):
    """First-order BDIM blend of the stage velocity f.  Vb: body velocity per
    component at the faces (None: at rest); G: its constant gradient."""
    d = len(f)
    n = f[0].shape
    Pf = pad_velocity(f, fout, bc_lo, bc_hi, U)
    out = []
    for i in range(d):
        g = mu0[i] * f[i]
        if Vb is not None:
            g = g + (1.0 - mu0[i]) * Vb[i]
        for j in range(d):
            dj = [1 if a == j else 0 for a in range(d)]
            fp = _view(Pf[i], n, dj)
            fm = _view(Pf[i], n, [-x for x in dj])
            dn = 0.5 * (fp - fm)
            if G is not None:
                dn = dn - G[i][j]
            g = g + mu1n[i][j] * dn
        out.append(g)
    return out


def exit_flux_correct(u, uout, bc_lo, bc_hi):
    """Shift the outflow plane so its flux equals the inflow plane's."""
    if bc_hi[0] != OUTFLOW:
        return uout
    inflow = float(np.sum(u[0][0]))
    outflow = float(np.sum(uout))
    return uout + (inflow - outflow) / uout.size
