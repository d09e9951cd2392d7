"""Pins of the oracle's Gram-Schmidt pass (Sec. 4.2, full
M-reorthogonalisation): with W = M B for an M-orthonormal B, the result is
M-orthogonal to every column of B (the property the pass exists for), the
pass is a projection (a second pass changes nothing), a vector in the span
of B is removed, one orthogonal to it is untouched, and c holds the
M-coordinates."""
import numpy as np
import scipy.linalg as sla

import workloads
from oracle import assembly, lanczos


def _mb(seed=3, m=7):
    w = workloads.small(2, 10, 2, 3, 5, 0.4)
    kappa, rho = w.coefficients()
    _, M = assembly.assemble(w.dim, w.ne, w.p, w.s, kappa, rho)
    M = M.toarray()
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((M.shape[0], m))
    # M-orthonormal basis by a Cholesky of the Gram matrix
    G = X.T @ M @ X
    R = sla.cholesky(G, lower=False)
    B = sla.solve_triangular(R, X.T, trans="T", lower=False).T
    return M, B, rng


def test_result_is_m_orthogonal_and_a_projection():
    M, B, rng = _mb()
    assert np.abs(B.T @ M @ B - np.eye(B.shape[1])).max() < 1e-12
    W = M @ B
    x = rng.standard_normal(M.shape[0])
    c, y = lanczos.cgs_pass(W, B, x)
    assert np.abs(B.T @ (M @ y)).max() <= 1e-12 * np.abs(x).max() * np.abs(M).max() * M.shape[0]
    c2, y2 = lanczos.cgs_pass(W, B, y)
    assert np.abs(c2).max() <= 1e-12 * np.abs(c).max()
    assert np.allclose(y2, y, rtol=0, atol=1e-12 * np.abs(y).max())


def test_span_removed_and_orthogonal_kept():
    M, B, rng = _mb(m=5)
    W = M @ B
    a = rng.standard_normal(B.shape[1])
    c, y = lanczos.cgs_pass(W, B, B @ a)
    assert np.allclose(c, a, rtol=0, atol=1e-12 * np.abs(a).max())
    assert np.abs(y).max() <= 1e-12 * np.abs(B @ a).max()
    z = rng.standard_normal(M.shape[0])
    z = lanczos.cgs_pass(W, B, z)[1]           # now M-orthogonal to B
    c, z2 = lanczos.cgs_pass(W, B, z)
    assert np.abs(c).max() <= 1e-12 * np.abs(z).max()
    assert np.allclose(z2, z, rtol=0, atol=1e-12 * np.abs(z).max())


def test_inputs_untouched_and_coordinates_are_m_inner_products():
    M, B, rng = _mb(m=4)
    W = M @ B
    x = rng.standard_normal(M.shape[0])
    x0, B0 = x.copy(), B.copy()
    c, _ = lanczos.cgs_pass(W, B, x)
    assert np.array_equal(x, x0) and np.array_equal(B, B0)
    for j in range(B.shape[1]):
        assert abs(c[j] - B[:, j] @ (M @ x)) <= 1e-12 * np.abs(c).max()
