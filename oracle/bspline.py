"""Knot vectors, Cox--de Boor basis evaluation and Gauss--Legendre rules.

Test infrastructure only (see the package docstring).

Follows Sec. 3.1 (Eqs. U and N) and Sec. 3.2 of arXiv 2009.08167.
"""
import numpy as np


def knot_vector(ne, p, s):
    """Open knot vector on [0, 1] for ``ne`` uniform elements of degree ``p``.

    Sec. 3.1, Eq. U: ``p+1`` repeated knots at each end, simple interior knots
    (maximum continuity C^{p-1}).  Sec. 3.2: rIGA raises the multiplicity of
    the knots at macro-element boundaries "up to the degree", i.e. to ``p``,
    which makes the basis C^0 there.  ``s`` is the macro-element size in
    elements (``s = 0`` means plain IGA); interior knot ``k/ne`` gets
    multiplicity ``p`` when ``s > 0`` and ``k % s == 0``.  For ``ne`` not a
    multiple of ``s`` the last macro-element is simply shorter.
    """
    kv = [0.0] * (p + 1)
    for k in range(1, ne):
        mult = p if (s > 0 and k % s == 0) else 1
        kv += [k / ne] * mult
    kv += [1.0] * (p + 1)
    return np.array(kv, dtype=np.float64)


def n_functions(kv, p):
    """Number of B-splines of degree ``p`` on knot vector ``kv``."""
    return len(kv) - p - 1


def _ratio(num, den):
    # Cox--de Boor convention: a term whose knot span is empty is 0 (0/0 := 0).
    out = np.zeros_like(num)
    if den != 0.0:
        out = num / den
    return out


def basis_all(kv, p, x):
    """Values of every B-spline B_{i,p} at the points ``x``.

    Direct transcription of the Cox--de Boor recursion (Eq. N): degree-0
    indicators of the half-open spans [xi_i, xi_{i+1}), then raise the degree
    one step at a time.  Returns an array of shape (n_functions, len(x)).
    """
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    m = len(kv) - 1
    B = np.array([((kv[i] <= x) & (x < kv[i + 1])).astype(np.float64) for i in range(m)])
    for d in range(1, p + 1):
        Bn = np.zeros((m - d, x.size))
        for i in range(m - d):
            left = _ratio(x - kv[i], kv[i + d] - kv[i])
            right = _ratio(kv[i + d + 1] - x, kv[i + d + 1] - kv[i + 1])
            Bn[i] = left * B[i] + right * B[i + 1]
        B = Bn
    return B


def basis_deriv_all(kv, p, x):
    """First derivatives of every B_{i,p} at ``x`` (shape (n, len(x))).

    The paper does not print the derivative; this is the textbook formula
    B'_{i,p} = p/(xi_{i+p}-xi_i) B_{i,p-1} - p/(xi_{i+p+1}-xi_{i+1}) B_{i+1,p-1},
    with the same 0/0 := 0 convention.
    """
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    if p == 0:
        return np.zeros((len(kv) - 1, x.size))
    Bl = basis_all(kv, p - 1, x)  # n+1 functions of degree p-1
    n = len(kv) - p - 1
    dB = np.zeros((n, x.size))
    for i in range(n):
        a = p / (kv[i + p] - kv[i]) if kv[i + p] != kv[i] else 0.0
        b = p / (kv[i + p + 1] - kv[i + 1]) if kv[i + p + 1] != kv[i + 1] else 0.0
        dB[i] = a * Bl[i] - b * Bl[i + 1]
    return dB


def support(kv, p, i):
    """Closed support [xi_i, xi_{i+p+1}] of B_{i,p}."""
    return kv[i], kv[i + p + 1]


def elements(kv):
    """Element (non-empty knot span) boundaries: the distinct knots."""
    return np.unique(kv)


def gauss_legendre(q, a=-1.0, b=1.0):
    """``q``-point Gauss--Legendre rule mapped to [a, b].

    The paper does not state its quadrature; p+1 points per direction
    integrate the piecewise polynomial integrands (degree <= 2p) exactly.
    """
    t, w = np.polynomial.legendre.leggauss(q)
    return 0.5 * (b - a) * t + 0.5 * (a + b), 0.5 * (b - a) * w
