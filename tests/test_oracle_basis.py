"""Pins of the oracle's knot vectors, Cox--de Boor evaluation and quadrature.

Each test checks the oracle against something other than itself: partition
of unity, finite differences, polynomial exactness, the continuity the knot
multiplicity dictates (Sec. 3.2), and the DOF count of Eq. dofs.
"""
import numpy as np
import pytest

from oracle import bspline


@pytest.mark.parametrize("p,s", [(1, 0), (2, 0), (3, 0), (3, 4), (4, 2), (5, 1)])
def test_partition_of_unity_and_nonnegativity(p, s):
    kv = bspline.knot_vector(8, p, s)
    x = np.linspace(0.0, 1.0, 1001)[:-1]
    B = bspline.basis_all(kv, p, x)
    assert np.allclose(B.sum(axis=0), 1.0, atol=1e-14)
    assert (B >= -1e-15).all()


@pytest.mark.parametrize("p,s", [(2, 0), (3, 0), (3, 2), (4, 4)])
def test_derivative_matches_finite_differences(p, s):
    kv = bspline.knot_vector(8, p, s)
    # points away from the knots, where every B is a smooth polynomial
    x = (np.arange(8)[:, None] + np.array([0.21, 0.5, 0.77])[None, :]).ravel() / 8
    h = 1e-6
    fd = (bspline.basis_all(kv, p, x + h) - bspline.basis_all(kv, p, x - h)) / (2 * h)
    dB = bspline.basis_deriv_all(kv, p, x)
    assert np.allclose(dB, fd, atol=1e-6)


def test_derivatives_sum_to_zero():
    kv = bspline.knot_vector(10, 3, 5)
    x = np.linspace(0.013, 0.987, 77)
    assert np.allclose(bspline.basis_deriv_all(kv, 3, x).sum(axis=0), 0.0, atol=1e-12)


@pytest.mark.parametrize("q", [1, 2, 3, 4, 5, 6])
def test_gauss_legendre_exact_to_degree_2q_minus_1(q):
    x, w = bspline.gauss_legendre(q, 0.25, 0.75)
    for deg in range(2 * q):
        exact = (0.75 ** (deg + 1) - 0.25 ** (deg + 1)) / (deg + 1)
        assert abs(np.sum(w * x ** deg) - exact) < 1e-14


@pytest.mark.parametrize("p", [2, 3, 4])
def test_continuity_follows_multiplicity(p):
    """Sec. 3.2: raising a knot's multiplicity to p leaves the basis C^0
    there; a simple knot keeps C^{p-1}.  Check the first-derivative jump of
    a spline with random coefficients at a simple knot (none) and at a C^0
    knot (generically non-zero)."""
    ne, s = 8, 4
    kv = bspline.knot_vector(ne, p, s)
    rng = np.random.default_rng(1)
    c = rng.standard_normal(bspline.n_functions(kv, p))
    eps = 1e-9

    def djump(x0):
        dl = bspline.basis_deriv_all(kv, p, [x0 - eps]).ravel() @ c
        dr = bspline.basis_deriv_all(kv, p, [x0 + eps]).ravel() @ c
        return abs(dr - dl)

    def vjump(x0):
        vl = bspline.basis_all(kv, p, [x0 - eps]).ravel() @ c
        vr = bspline.basis_all(kv, p, [x0 + eps]).ravel() @ c
        return abs(vr - vl)

    assert djump(3 / 8) < 1e-5            # simple knot: C^{p-1}, p >= 2
    assert djump(4 / 8) > 1e-2            # multiplicity p: only C^0
    assert vjump(4 / 8) < 1e-6            # still continuous
    # exactly one function is non-zero at a C^0 knot (it interpolates there)
    vals = bspline.basis_all(kv, p, [0.5]).ravel()
    assert np.count_nonzero(np.abs(vals) > 1e-14) == 1


def test_function_count_sec31():
    """Sec. 3.1: maximum continuity gives n = ne + p functions per direction."""
    for ne in (1, 2, 8, 33):
        for p in (1, 2, 3, 5):
            assert bspline.n_functions(bspline.knot_vector(ne, p, 0), p) == ne + p


@pytest.mark.parametrize("dim", [1, 2, 3])
@pytest.mark.parametrize("ne", [8, 16, 32, 256])
@pytest.mark.parametrize("p", [2, 3, 4, 5])
def test_dof_count_eq_dofs(dim, ne, p):
    """Eq. dofs: IGA (ne+p-2)^d; rIGA at partition level l (2^l blocks of
    blocksize 2^{s-l} per direction) [ne + 2^l (p-1) - 1]^d."""
    n_iga = (bspline.n_functions(bspline.knot_vector(ne, p, 0), p) - 2) ** dim
    assert n_iga == (ne + p - 2) ** dim
    s_exp = int(np.log2(ne))
    for l in range(1, s_exp + 1):
        bs = 2 ** (s_exp - l)
        n = (bspline.n_functions(bspline.knot_vector(ne, p, bs), p) - 2) ** dim
        assert n == (ne + 2 ** l * (p - 1) - 1) ** dim
    # l = s is C^0 FEA: (ne p - 1)^d interior functions
    n_fea = (bspline.n_functions(bspline.knot_vector(ne, p, 1), p) - 2) ** dim
    assert n_fea == (ne * p - 1) ** dim
