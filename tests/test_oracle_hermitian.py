"""Pins of the complex Hermitian source (oracle/hermitian.py: the magnetic
Laplacian with a constant potential, the Hermitian case of Eq. GHEP of
arXiv 2009.08167) against what the mathematics fixes:

* Hermitian symmetry of K (antisymmetric imaginary part), real M;
* A = 0 gives the real oracle's K exactly;
* the Kronecker form of the same matrices from 1D integrals, 2D and 3D (a different
  route from the element-by-element tensor assembly);
* gauge invariance of the limit: the eigenvalues approach pi^2 (i^2 + j^2)
  from above at the rate of the real problem, h^(2p);
* the sign of the magnetic term: the lowest eigenvector is the real one
  times exp(+i A.x) (its phase, read at the Greville points, has slope A;
  the conjugate form would give -A with the same eigenvalues);
* the real-equivalent pencil has every eigenvalue twice and commutes with J.
"""
import math

import numpy as np
import scipy.sparse as sp

from oracle import accuracy, assembly, eigen, hermitian


def _g1d(ne, p, s):
    """1D matrix G[a, b] = int B_a B_b' (full), by the 1D Gauss rule."""
    s1 = assembly.Space1D(ne, p, s)
    G = np.zeros((s1.n, s1.n))
    for e in range(ne):
        a = s1.active[e]
        G[np.ix_(a, a)] += np.einsum('ap,bp,p->ab', s1.B[a, e, :], s1.dB[a, e, :], s1.wts[e])
    return G


def test_hermitian_structure():
    for dim, ne, p, s, A in ((2, 6, 2, 3, (0.9, -1.7)), (3, 3, 2, 0, (0.4, 1.1, -0.6))):
        K, M = hermitian.assemble_magnetic(dim, ne, p, s, A)
        Kd, Md = K.toarray(), M.toarray()
        scale = np.abs(Kd).max()
        assert np.abs(Kd - Kd.conj().T).max() <= 1e-14 * scale
        assert np.abs(Kd.imag + Kd.imag.T).max() <= 1e-14 * scale
        assert np.abs(Kd.imag).max() > 1e-3 * scale  # the magnetic term is there
        assert np.isrealobj(Md) or np.abs(Md.imag).max() == 0.0
        assert np.abs(Md - Md.T).max() <= 1e-15 * np.abs(Md).max()
        K2, M2 = hermitian.real_equivalent(K, M)
        assert abs(K2 - K2.T).max() <= 1e-14 * scale


def test_zero_potential_is_the_real_problem():
    for dim, ne, p, s in ((2, 7, 3, 2), (3, 3, 2, 1)):
        K, M = hermitian.assemble_magnetic(dim, ne, p, s, np.zeros(dim))
        Kr, Mr = assembly.assemble(dim, ne, p, s)
        assert np.abs(K.imag).max() == 0.0
        assert abs(K.real - Kr).max() <= 1e-13 * abs(Kr).max()
        assert abs(M - Mr).max() <= 1e-15 * abs(Mr).max()


def test_kronecker_form():
    """2D, x fastest: K = My (x) Kx + Ky (x) Mx + |A|^2 M
    + i (Ax My (x) (Gx - Gx^T) + Ay (Gy - Gy^T) (x) Mx)."""
    ne, p, s, A = 6, 3, 3, np.array([1.3, -0.45])
    K, M = hermitian.assemble_magnetic(2, ne, p, s, A)
    K1, M1 = assembly.matrices_1d(ne, p, s)
    G1 = _g1d(ne, p, s)
    K1, M1, G1 = K1[1:-1, 1:-1], M1[1:-1, 1:-1], G1[1:-1, 1:-1]
    S1 = G1 - G1.T
    Mk = np.kron(M1, M1)
    Kk = (np.kron(M1, K1) + np.kron(K1, M1) + (A @ A) * Mk
          + 1j * (A[0] * np.kron(M1, S1) + A[1] * np.kron(S1, M1)))
    assert np.abs(K.toarray() - Kk).max() <= 1e-12 * np.abs(Kk).max()
    assert np.abs(M.toarray() - Mk).max() <= 1e-14 * np.abs(Mk).max()


def test_kronecker_form_3d():
    """3D, x fastest: each direction's factor (stiffness, or the magnetic
    S = G - G^T times that component of A) between the other two masses."""
    ne, p, s, A = 4, 2, 2, np.array([0.7, -1.2, 0.35])
    K, M = hermitian.assemble_magnetic(3, ne, p, s, A)
    K1, M1 = assembly.matrices_1d(ne, p, s)
    G1 = _g1d(ne, p, s)
    K1, M1, G1 = K1[1:-1, 1:-1], M1[1:-1, 1:-1], G1[1:-1, 1:-1]
    S1 = G1 - G1.T

    def k3(z, y, x):
        return np.kron(np.kron(z, y), x)

    Mk = k3(M1, M1, M1)
    Kk = (k3(M1, M1, K1) + k3(M1, K1, M1) + k3(K1, M1, M1) + (A @ A) * Mk
          + 1j * (A[0] * k3(M1, M1, S1) + A[1] * k3(M1, S1, M1) + A[2] * k3(S1, M1, M1)))
    assert np.abs(K.toarray() - Kk).max() <= 1e-12 * np.abs(Kk).max()
    assert np.abs(M.toarray() - Mk).max() <= 1e-14 * np.abs(Mk).max()


def test_gauge_invariant_limit_and_rate():
    """Lowest eigenvalue 2 pi^2 for every A: approached from above at h^(2p)."""
    p, A = 2, (1.3, -0.7)
    err = []
    for ne in (8, 16):
        K, M = hermitian.assemble_magnetic(2, ne, p, 0, A)
        lam, _ = hermitian.dense_eigh_hermitian(K, M)
        ex = accuracy.exact_eigenvalues(2, 10)
        rel = (lam[:10] - ex) / ex
        assert rel.min() >= -1e-12, rel  # Courant--Fischer: upper bounds
        err.append(rel[0])
    ratio = err[0] / err[1]
    assert 0.75 * 2 ** (2 * p) <= ratio <= 1.3 * 2 ** (2 * p), ratio


def test_phase_of_the_lowest_mode_has_slope_A():
    """u_h ~ exp(i A.x) w_h: the phase of the lowest eigenvector relative to
    the real (A = 0) one, read at the Greville points of the interior
    functions, is A.x + const (least squares, weighted by |w|)."""
    ne, p, s, A = 12, 3, 4, np.array([1.1, -0.6])
    K, M = hermitian.assemble_magnetic(2, ne, p, s, A)
    lam, U = hermitian.dense_eigh_hermitian(K, M)
    K0, M0 = assembly.assemble(2, ne, p, s)
    lam0, U0 = eigen.dense_eigh(K0, M0)
    assert abs(lam[0] - lam0[0]) / lam0[0] < 1e-2
    s1 = assembly.Space1D(ne, p, s)
    kv = s1.kv
    grev = np.array([kv[i + 1:i + p + 1].mean() for i in range(s1.n)])[1:-1]
    X, Y = np.meshgrid(grev, grev)  # x fastest in the flattened order
    x, y = X.ravel(), Y.ravel()
    u, w = U[:, 0], U0[:, 0]
    c = np.argmax(np.abs(w))
    phase = np.angle(u * np.conj(u[c]) * np.sign(w) * np.sign(w[c]))
    wt = np.abs(w)
    Amat = np.stack([x - x[c], y - y[c]], axis=1) * wt[:, None]
    slope, *_ = np.linalg.lstsq(Amat, phase * wt, rcond=None)
    assert np.abs(slope - A).max() <= 0.05 * np.abs(A).max(), slope


def test_real_equivalent_doubles_the_spectrum_and_commutes_with_J():
    ne, p, s, A = 5, 2, 0, (0.8, 1.9)
    K, M = hermitian.assemble_magnetic(2, ne, p, s, A)
    lam, _ = hermitian.dense_eigh_hermitian(K, M)
    K2, M2 = hermitian.real_equivalent(K, M)
    lam2, _ = eigen.dense_eigh(K2, M2)
    assert np.abs(lam2[0::2] - lam).max() <= 1e-10 * lam.max()
    assert np.abs(lam2[1::2] - lam).max() <= 1e-10 * lam.max()
    n = K.shape[0]
    I = sp.identity(n, format='csr')
    J = sp.bmat([[None, -I], [I, None]]).tocsr()
    assert abs(J @ K2 - K2 @ J).max() <= 1e-14 * abs(K2).max()
    assert abs(J @ M2 - M2 @ J).max() == 0.0
    assert math.isclose(lam[0], 2 * math.pi ** 2, rel_tol=0.05)
