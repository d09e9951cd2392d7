"""Eigenvalue and eigenfunction errors against the exact Laplace eigenpairs.

Test infrastructure only (see the package docstring).

Follows Sec. 2 of arXiv 2009.08167: the exact eigenpairs of the Dirichlet
Laplacian on the unit square and cube (Eq. exact), the L2 and energy norms
of the eigenfunction error (Eq. norms), the normalised errors EVerr, EFerr_L2
and EFerr_E (Eq. eigerrors) and the Pythagorean relation between them (Eq.
Pythagorean); and Sec. 8, which compares eigenfunctions only for the
diagonal modes (i = j), the others being degenerate.

Readings (the paper is silent on them):
* EVerr pairs the n-th computed eigenvalue with the n-th exact one, both in
  ascending order with multiplicity.
* The computed eigenfunction compared with the exact diagonal mode m is the
  one with the largest |(u_h, u_e)| (L2 inner product) among those given;
  its sign is the one that gives the smaller L2 error.
* Integrals use a Gauss--Legendre rule of ``q`` points per direction and
  element (the exact eigenfunctions are not piecewise polynomials, so the
  rule is not exact; ``q = p + 6`` by default).

Everything is evaluated from the definitions on the full tensor grid of
quadrature points: u_h(x) = sum_a c_a B_a(x) with the coefficients of the
interior functions (zero on the boundary ones), u_e from Eq. exact.
"""
import itertools
import math

import numpy as np

from . import assembly


def default_q(p):
    return p + 6


def exact_eigenvalues(dim, count):
    """The ``count`` smallest pi^2 (i^2 + j^2 [+ k^2]), i, j, k >= 1, in
    ascending order with multiplicity (Eq. exact)."""
    n = 4
    while True:
        vals = np.sort(np.sum(np.array(list(itertools.product(range(1, n + 1), repeat=dim))) ** 2, axis=1))
        # every tuple with an index above n has a value >= (n+1)^2 + dim - 1
        if len(vals) >= count and vals[count - 1] < (n + 1) ** 2 + dim - 1:
            return math.pi ** 2 * vals[:count].astype(np.float64)
        n *= 2


def everr(dim, lam_h):
    """EVerr of Eq. eigerrors for ascending computed eigenvalues."""
    lam_h = np.asarray(lam_h, dtype=np.float64)
    lam_e = exact_eigenvalues(dim, len(lam_h))
    return (lam_h - lam_e) / lam_e


def exact_mode(idx, x):
    """u_e and its derivative along one direction for index ``idx``:
    sqrt(2) sin(i pi x) (the 2D/3D mode of Eq. exact is the product of one
    such factor per direction)."""
    return (math.sqrt(2.0) * np.sin(idx * math.pi * x),
            math.sqrt(2.0) * idx * math.pi * np.cos(idx * math.pi * x))


def _grid(spaces):
    """Per direction: basis values and derivatives at the quadrature points
    of every element, flattened (n_functions, ne * q), the points and the
    weights (weights include the element Jacobian)."""
    out = []
    for sp1 in spaces:
        out.append((sp1.B.reshape(sp1.n, -1), sp1.dB.reshape(sp1.n, -1),
                    sp1.pts.ravel(), sp1.wts.ravel()))
    return out


def _coeff_tensor(spaces, u):
    """Interior coefficients (x fastest) -> full tensor C[z][y][x] with zero
    boundary functions."""
    ns = [sp1.n for sp1 in spaces]
    C = np.zeros(ns[::-1])
    inner = u.reshape([n - 2 for n in ns[::-1]])
    C[tuple(slice(1, n - 1) for n in ns[::-1])] = inner
    return C


def _evaluate(spaces, grid, u):
    """u_h and its gradient on the tensor grid (arrays indexed [z][y][x])."""
    dim = len(spaces)
    C = _coeff_tensor(spaces, u)
    if dim == 2:
        (Bx, dBx, _, _), (By, dBy, _, _) = grid
        val = By.T @ C @ Bx
        gx = By.T @ C @ dBx
        gy = dBy.T @ C @ Bx
        return val, (gx, gy)
    (Bx, dBx, _, _), (By, dBy, _, _), (Bz, dBz, _, _) = grid
    ev = lambda Z, Y, X: np.einsum('zyx,zk,yj,xi->kji', C, Z, Y, X, optimize=True)
    return ev(Bz, By, Bx), (ev(Bz, By, dBx), ev(Bz, dBy, Bx), ev(dBz, By, Bx))


def _exact_on_grid(grid, mode):
    """u_e and its gradient for the tensor mode (i, j[, k]) on the grid."""
    dim = len(grid)
    f = [exact_mode(mode[d], grid[d][2]) for d in range(dim)]
    if dim == 2:
        (fx, dfx), (fy, dfy) = f
        return np.outer(fy, fx), (np.outer(fy, dfx), np.outer(dfy, fx))
    (fx, dfx), (fy, dfy), (fz, dfz) = f
    t = lambda Z, Y, X: np.einsum('k,j,i->kji', Z, Y, X)
    return t(fz, fy, fx), (t(fz, fy, dfx), t(fz, dfy, fx), t(dfz, fy, fx))


def _weights(grid):
    dim = len(grid)
    if dim == 2:
        return np.outer(grid[1][3], grid[0][3])
    return np.einsum('k,j,i->kji', grid[2][3], grid[1][3], grid[0][3])


def overlaps(dim, ne, p, s, U, modes, q=None):
    """G[n, m] = (u_h,n , u_e,m) for computed eigenvectors U [nvec, N]
    (interior coefficients, x fastest) and exact modes ``modes`` [nm, dim]."""
    q = default_q(p) if q is None else q
    spaces = assembly.make_spaces(dim, ne, p, s, q)
    grid = _grid(spaces)
    W = _weights(grid)
    U = np.atleast_2d(np.asarray(U, dtype=np.float64))
    G = np.zeros((U.shape[0], len(modes)))
    for n in range(U.shape[0]):
        uh, _ = _evaluate(spaces, grid, U[n])
        for m, mode in enumerate(modes):
            ue, _ = _exact_on_grid(grid, mode)
            G[n, m] = np.sum(W * uh * ue)
    return G


def mode_errors(dim, ne, p, s, lam_h, U, modes, q=None):
    """For each exact mode: the matched computed eigenpair, its overlap, and
    EFerr_L2, EFerr_E (Eq. eigerrors) with the energy norm integrated
    directly (not taken from the Pythagorean relation), plus EVerr of the
    matched pair against the mode's exact eigenvalue.

    Returns dict of arrays: match, overlap, l2, energy, ev.
    """
    q = default_q(p) if q is None else q
    spaces = assembly.make_spaces(dim, ne, p, s, q)
    grid = _grid(spaces)
    W = _weights(grid)
    U = np.atleast_2d(np.asarray(U, dtype=np.float64))
    G = overlaps(dim, ne, p, s, U, modes, q)
    out = {k: np.zeros(len(modes)) for k in ("overlap", "l2", "energy", "ev")}
    out["match"] = np.zeros(len(modes), dtype=np.int64)
    for m, mode in enumerate(modes):
        n = int(np.argmax(np.abs(G[:, m])))
        uh, guh = _evaluate(spaces, grid, U[n])
        ue, gue = _exact_on_grid(grid, mode)
        lam_e = math.pi ** 2 * float(np.sum(np.asarray(mode) ** 2))
        best = None
        for sign in (1.0, -1.0):
            l2 = float(np.sum(W * (uh - sign * ue) ** 2))
            en = float(sum(np.sum(W * (g - sign * ge) ** 2) for g, ge in zip(guh, gue)))
            if best is None or l2 < best[0]:
                best = (l2, en)
        out["match"][m] = n
        out["overlap"][m] = G[n, m]
        out["l2"][m] = best[0]
        out["energy"][m] = best[1] / lam_e
        out["ev"][m] = (lam_h[n] - lam_e) / lam_e
    return out


def diagonal_modes(dim, count):
    """The first ``count`` diagonal modes (i, i[, i]), i = 1..count."""
    return np.array([[i] * dim for i in range(1, count + 1)], dtype=np.int64)


def linear_fem_eigenvalues_1d(ne, count):
    """Closed form of the 1D Dirichlet Laplacian's eigenvalues with linear
    elements on a uniform mesh (p = 1): 6/h^2 (1 - cos(k pi h)) / (2 + cos(k pi h)).
    A textbook result (consistent mass), used to pin EVerr."""
    h = 1.0 / ne
    k = np.arange(1, count + 1)
    c = np.cos(k * math.pi * h)
    return 6.0 / h ** 2 * (1.0 - c) / (2.0 + c)
