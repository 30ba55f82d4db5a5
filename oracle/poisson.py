"""Pressure Poisson operator and geometric multigrid (oracle; test-only).

Paper, Sec. 2: the pressure system (with the BDIM-modified matrix) is solved
by geometric multigrid whose cost grows linearly with the cell count; the
projection kernel u[I,i] -= coeff[I,i]*(p[I]-p[I-del(i)]) fixes the face
gradient and its coefficient.  The operator is therefore

  (A p)(I) = sum_i  L_i(I+delta_i) (p(I+delta_i) - p(I))
                  - L_i(I)         (p(I) - p(I-delta_i)),

the L-weighted divergence of the face gradient.  A is symmetric negative
semi-definite with A 1 = 0.  A cell whose 2d face coefficients are all zero is
INACTIVE (fully solid).

"Exact" solution = minimum-norm solution of A p = b_proj, where b_proj is b
with inactive cells zeroed and the active-set mean removed.

READINGS for the constants the paper leaves open (it names only GMG and,
for smoothing, kernel-friendly non-ordered relaxation):
  * smoother: damped Jacobi x <- x + w (b - A x)/diag(A), w = 2d/(2d+1),
    inactive cells held at zero; nu1 = nu2 = 2 sweeps (symmetric V-cycle);
  * restriction: coarse RHS = sum of the 2^d child residuals;
  * prolongation: cell-centred (bi/tri)linear interpolation, direction by
    direction: a fine cell takes 3/4 of its parent and 1/4 of the parent's
    neighbour on the fine cell's side (wrapped on periodic directions; at a
    non-periodic domain face the missing neighbour is the parent itself, the
    even reflection of the homogeneous Neumann condition).  With the sum
    restriction (transfer orders 2 + 1 > 2, the order rule for a second-order
    operator) the V-cycle contraction does not degrade with the grid size,
    which Sec. 2's linear-time claim needs; piecewise-constant prolongation
    (orders 1 + 1) measurably does (asymptotic rate 0.42 / 0.50 / 0.58 at
    32^3 / 64^3 / 128^3 against 0.25 for all three with linear
    interpolation).  The V-cycle is then not a symmetric operator; nothing
    relies on that (the adjoint treats each pressure solve as exact);
  * coarse coefficient: half the sum of the 2^(d-1) fine faces a coarse face
    covers (the unit-spacing rediscretisation of the integrated operator);
  * coarsest level: minimum-norm least squares (a library routine);
  * V-cycles until ||b - A x||_2 / ||b||_2 <= tol, tested before each cycle.

Smoother "cg" (the paper's own choice, Sec. 2: conjugate-gradient smoothing
within the GMG levels, because relaxations that visit points in order cannot
be written as kernels).  READINGS: each smoothing step is a fresh run of
Jacobi-preconditioned CG on the level's system from the current iterate
(nu1 = nu2 = 2 iterations, the counts of the Jacobi smoother), on the
positive semi-definite M = -A with the preconditioner D = -diag(A)
(inactive cells, D = 0, stay at zero); the coarsest level is solved exactly
as with Jacobi.
"""

import numpy as np

from .grid import PERIODIC, shift

NU1 = 2
NU2 = 2


def omega(d):
    return 2.0 * d / (2.0 * d + 1.0)


def periodic_flags(bc_lo):
    return [b == PERIODIC for b in bc_lo]


def apply_A(L, p, per):
    d = p.ndim
    out = np.zeros_like(p)
    for i in range(d):
        g = L[i] * (p - shift(p, i, -1, per[i]))        # face gradient * L at lower faces
        out += shift(g, i, 1, per[i]) - g                # upper face minus lower face
    return out


def diag_A(L, per):
    d = L[0].ndim
    D = np.zeros_like(L[0])
    for i in range(d):
        D += L[i] + shift(L[i], i, 1, per[i])
    return -D


def active_mask(L, per):
    return diag_A(L, per) != 0.0


def project_rhs(b, active):
    b = np.where(active, b, 0.0)
    if active.any():
        b = b - np.where(active, b[active].mean(), 0.0)
    return b


def remove_mean(x, active):
    if not active.any():
        return x
    return np.where(active, x - x[active].mean(), 0.0)


def jacobi(L, x, b, per, diag=None):
    d = x.ndim
    if diag is None:
        diag = diag_A(L, per)
    r = b - apply_A(L, x, per)
    safe = np.where(diag != 0.0, diag, 1.0)
    return np.where(diag != 0.0, x + omega(d) * r / safe, 0.0)


def pcg_smooth(L, x, b, per, iters, diag=None, history=None):
    """`iters` Jacobi-preconditioned conjugate-gradient iterations on A x = b
    from x, written for M = -A, c = -b (M positive semi-definite) with the
    preconditioner D = -diag(A):

        r = P(c - M x),  z = r / D,  p = z
        repeat: q = M p, alpha = (r.z) / (p.q), x += alpha p, r = P(r - alpha q),
                z' = r / D, beta = (r.z') / (r.z)_old, p = z' + beta p,

    P removing the mean over the active cells.  P keeps the residual in the
    range of M (orthogonal to its null vector, the constant on the active
    cells); in exact arithmetic it changes nothing (b is mean-free, and
    1.M v = 0 for every v), in rounding it keeps iterations past the
    solution's rounding floor from diverging (READING: CG on the singular
    system restricted to the range of M).  Stops early when r.z or p.q
    vanishes (the iterate is then exact).  With `history` (a list) each
    iteration's (r, z, p) before the update is appended, for the conjugacy
    pins."""
    if diag is None:
        diag = diag_A(L, per)
    D = -diag
    act = D > 0.0
    safe = np.where(act, D, 1.0)

    def M(v):
        return -apply_A(L, v, per)

    x = np.where(act, x, 0.0)
    r = remove_mean(np.where(act, -b - M(x), 0.0), act)
    z = np.where(act, r / safe, 0.0)
    p = z.copy()
    rz = float(np.sum(r * z))
    for _ in range(iters):
        if rz == 0.0:
            break
        q = M(p)
        pq = float(np.sum(p * q))
        if pq == 0.0:
            break
        if history is not None:
            history.append((r.copy(), z.copy(), p.copy()))
        alpha = rz / pq
        x = x + alpha * p
        r = remove_mean(r - alpha * q, act)
        z = np.where(act, r / safe, 0.0)
        rz_new = float(np.sum(r * z))
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x


def restrict(r):
    d = r.ndim
    shp = []
    for m in r.shape:
        shp += [m // 2, 2]
    return r.reshape(shp).sum(axis=tuple(range(1, 2 * d, 2)))


def prolong(xc, per):
    """Cell-centred linear interpolation onto the grid twice as fine.

    Along each direction, fine cells 2I and 2I+1 sit a quarter of a coarse
    cell below and above the centre of coarse cell I, so linear interpolation
    gives them 3/4 x_c(I) + 1/4 x_c(I-1) and 3/4 x_c(I) + 1/4 x_c(I+1).
    Periodic directions wrap; on a non-periodic direction the outside
    neighbour is x_c(I) itself (zero normal gradient).
    """
    x = xc
    for ax in range(xc.ndim):
        n = x.shape[ax]
        lower = shift(x, ax, -1, per[ax])
        upper = shift(x, ax, 1, per[ax])
        if not per[ax]:
            first = [slice(None)] * x.ndim
            first[ax] = 0
            last = [slice(None)] * x.ndim
            last[ax] = n - 1
            lower[tuple(first)] = x[tuple(first)]
            upper[tuple(last)] = x[tuple(last)]
        shp = list(x.shape)
        shp[ax] = 2 * n
        fine = np.empty(shp)
        even = [slice(None)] * x.ndim
        even[ax] = slice(0, None, 2)
        odd = [slice(None)] * x.ndim
        odd[ax] = slice(1, None, 2)
        fine[tuple(even)] = 0.75 * x + 0.25 * lower
        fine[tuple(odd)] = 0.75 * x + 0.25 * upper
        x = fine
    return x


def coarsen_L(L):
    """Coarse face coefficient = 1/2 * sum of the fine faces it covers."""
    d = L[0].ndim
    out = []
    for i in range(d):
        idx = [slice(None)] * d
        idx[i] = slice(0, None, 2)                       # fine faces on coarse face planes
        a = L[i][tuple(idx)]
        for j in range(d):
            if j == i:
                continue
            shp = list(a.shape)
            shp[j:j + 1] = [shp[j] // 2, 2]
            a = a.reshape(shp).sum(axis=j + 1)
        out.append(0.5 * a)
    return out


def dense_matrix(L, per):
    """Assemble A densely, face by face (graph-Laplacian assembly).

    Independent of apply_A: every interior face between cells a and b with
    coefficient c contributes +c to A[a,b], A[b,a] and -c to A[a,a], A[b,b].
    """
    shape = L[0].shape
    d = len(shape)
    N = int(np.prod(shape))
    A = np.zeros((N, N))
    flat = np.arange(N).reshape(shape)
    for i in range(d):
        for I in np.ndindex(*shape):
            c = L[i][I]
            if c == 0.0:
                continue
            J = list(I)
            J[i] -= 1
            if J[i] < 0:
                if not per[i]:
                    continue
                J[i] += shape[i]
            a, b = flat[I], flat[tuple(J)]
            A[a, b] += c
            A[b, a] += c
            A[a, a] -= c
            A[b, b] -= c
    return A


class Hierarchy:
    """Coefficients of every level plus the coarsest pseudo-inverse (cached).
    smoother: "jacobi" (damped Jacobi sweeps) or "cg" (Jacobi-preconditioned
    CG iterations), NU1 before and NU2 after the coarse correction."""

    def __init__(self, L, nlev, per, smoother="jacobi"):
        if smoother not in ("jacobi", "cg"):
            raise ValueError("smoother must be 'jacobi' or 'cg'")
        self.smoother = smoother
        self.per = list(per)
        self.L = [list(L)]
        for _ in range(nlev - 1):
            self.L.append(coarsen_L(self.L[-1]))
        self.diag = [diag_A(Ll, self.per) for Ll in self.L]
        self.active = [dg != 0.0 for dg in self.diag]
        self._pinv = None

    @property
    def nlev(self):
        return len(self.L)

    def coarse_solve(self, b):
        """Minimum-norm least-squares solution on the coarsest level."""
        if self._pinv is None:
            self._pinv = np.linalg.pinv(dense_matrix(self.L[-1], self.per))
        return (self._pinv @ b.reshape(-1)).reshape(b.shape)


def vcycle(h, lev, x, b):
    L, per, diag = h.L[lev], h.per, h.diag[lev]
    if lev == h.nlev - 1:
        return h.coarse_solve(b)
    if h.smoother == "cg":
        x = pcg_smooth(L, x, b, per, NU1, diag)
    else:
        for _ in range(NU1):
            x = jacobi(L, x, b, per, diag)
    r = b - apply_A(L, x, per)
    xc = vcycle(h, lev + 1, np.zeros(tuple(m // 2 for m in x.shape)), restrict(r))
    x = x + prolong(xc, per)
    if h.smoother == "cg":
        x = pcg_smooth(L, x, b, per, NU2, diag)
    else:
        for _ in range(NU2):
            x = jacobi(L, x, b, per, diag)
    return x


def solve(h, b, x0=None, tol=1e-8, max_vcycles=100, force_vcycles=None, atol=0.0):
    """GMG solve of A x = b on hierarchy h.

    Stops before a V-cycle once ||b - A x||_2 <= tol ||b||_2 or
    ||b - A x||_2 <= atol (both norms over the projected b).  Returns
    (x, vcycles, rel_resid_history, converged).  With force_vcycles the
    stopping test is replaced by exactly that many V-cycles (replay mode).
    """
    L, per = h.L[0], h.per
    active = h.active[0]
    b = project_rhs(np.asarray(b, dtype=np.float64), active)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0 and force_vcycles is None:
        return np.zeros_like(b), 0, [0.0], True
    hist = []
    k = 0
    while True:
        res = np.linalg.norm(b - apply_A(L, x, per))
        rel = res / (bnorm if bnorm > 0 else 1.0)
        hist.append(rel)
        if force_vcycles is not None:
            if k == force_vcycles:
                return x, k, hist, True
        else:
            if rel <= tol or res <= atol:
                return x, k, hist, True
            if k == max_vcycles:
                return x, k, hist, False
        x = vcycle(h, 0, x, b)
        k += 1


def min_norm_solution(L, per, b):
    """Exact minimum-norm solution of A x = b_proj by dense least squares."""
    active = active_mask(L, per)
    bp = project_rhs(b, active)
    x, *_ = np.linalg.lstsq(dense_matrix(L, per), bp.reshape(-1), rcond=None)
    return x.reshape(b.shape)
