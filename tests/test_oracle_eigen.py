"""Pins of the oracle's eigen-solves (Eq. GHEP, Sec. 4).

Checked against: the exact Laplace spectrum (Eq. exact) and its convergence
order, Kronecker sums of 1D spectra (Eq. 2Dmatrix), the closed-form linear
FEM spectrum, the min-max ordering that nested spaces imply (rIGA encloses
IGA, Sec. 3.2), Sylvester inertia counts, coefficient scaling, and the
sparse shift-and-invert path against the dense one.
"""
import os

import numpy as np
import pytest
import scipy.linalg as sla

import workloads
from oracle import assembly, eigen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _kron_sum_spectrum(dim, ne, p, s):
    """Exact discrete spectrum at kappa = rho = 1 from 1D generalized
    eigenvalues: spec(K, M) = {mu_i + mu_j (+ mu_k)} (Eq. 2Dmatrix)."""
    K1, M1 = assembly.matrices_1d(ne, p, s)
    mu = sla.eigh(K1[1:-1, 1:-1], M1[1:-1, 1:-1], eigvals_only=True)
    lam = mu
    for _ in range(dim - 1):
        lam = (lam[:, None] + mu[None, :]).ravel()
    return np.sort(lam)


def test_c1_against_exact_laplace_spectrum():
    """Eq. exact: the lowest 10 eigenvalues of the 16x16 p=2 problem lie just
    above pi^2 (i^2 + j^2) (Galerkin eigenvalues bound from above)."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "c1_exact_spectrum.txt"))
            if l.strip() and not l.startswith("#")]
    exact = np.array([float(r[1]) for r in rows]) * np.pi ** 2
    K, M = assembly.assemble(2, 16, 2, 0)
    lam, U = eigen.dense_eigh(K, M)
    lam = lam[:10]
    assert (lam >= exact * (1 - 1e-13)).all()
    assert np.max((lam - exact) / exact) < 1e-3


@pytest.mark.parametrize("dim,ne,p,s", [(2, 8, 2, 0), (2, 8, 3, 4), (3, 4, 2, 2), (2, 10, 3, 3)])
def test_dense_matches_kronecker_sums(dim, ne, p, s):
    K, M = assembly.assemble(dim, ne, p, s)
    lam, U = eigen.dense_eigh(K, M)
    ref = _kron_sum_spectrum(dim, ne, p, s)
    assert np.max(np.abs(lam - ref) / ref) < 1e-11
    assert np.max(eigen.residual(K, M, lam, U)) < 1e-12
    assert np.abs(U.T @ (M @ U) - np.eye(len(lam))).max() < 1e-10


@pytest.mark.parametrize("p", [1, 2, 3])
def test_convergence_order_2p(p):
    """Eigenvalue error of the first mode decays like h^{2p}."""
    errs = []
    for ne in (4, 8, 16):
        K, M = assembly.assemble(1, ne, p, 0)
        lam, _ = eigen.dense_eigh(K, M)
        errs.append(lam[0] - np.pi ** 2)
    assert all(e > 0 for e in errs)
    rate = np.log2(errs[-2] / errs[-1])
    assert abs(rate - 2 * p) < 0.25


def test_linear_fem_closed_form():
    """p = 1 (rIGA = IGA = FEA): lambda_k = (6/h^2)(1 - cos k pi h)/(2 + cos k pi h)."""
    ne = 20
    h = 1.0 / ne
    K, M = assembly.assemble(1, ne, 1, 0)
    lam, _ = eigen.dense_eigh(K, M)
    k = np.arange(1, ne)
    ref = 6 / h ** 2 * (1 - np.cos(k * np.pi * h)) / (2 + np.cos(k * np.pi * h))
    assert np.max(np.abs(lam - ref) / ref) < 1e-13


def test_minmax_ordering_of_nested_spaces():
    """IGA subset rIGA(l) subset rIGA(l+1) subset FEA (Sec. 3.2), so by
    min-max lambda_exact <= lambda_FEA <= lambda_rIGA(l+1) <= lambda_rIGA(l)
    <= lambda_IGA for every index the IGA space has."""
    ne, p = 32, 3
    spectra = []
    for bs in (0, 16, 8, 4, 2, 1):
        K, M = assembly.assemble(1, ne, p, bs)
        spectra.append(eigen.dense_eigh(K, M)[0])
    n = len(spectra[0])
    exact = (np.arange(1, n + 1) * np.pi) ** 2
    for coarse, fine in zip(spectra[:-1], spectra[1:]):
        assert (fine[:n] <= coarse[:n] * (1 + 1e-12)).all()
    assert (spectra[-1][:n] >= exact * (1 - 1e-12)).all()


@pytest.mark.parametrize("dim,ne,p,s", [(2, 10, 2, 0), (2, 10, 3, 5), (3, 5, 2, 0)])
def test_inertia_counts_eigenvalues_below_shift(dim, ne, p, s):
    """Remark on inertia: nu(K - sigma M) = #{lambda < sigma}."""
    K, M = assembly.assemble(dim, ne, p, s)
    lam, _ = eigen.dense_eigh(K, M)
    for i in (0, 3, 17, 40, len(lam) // 2):
        sigma = 0.5 * (lam[i] + lam[i + 1]) if lam[i + 1] > lam[i] * (1 + 1e-9) else lam[i] * 0.999
        assert eigen.inertia(K, M, sigma) == np.count_nonzero(lam < sigma)


def test_coefficient_scaling():
    """kappa = c, rho = d everywhere: lambda = (c/d) lambda(1,1),
    u = u(1,1)/sqrt(d) for M-normalised u."""
    dim, ne, p, s = 2, 8, 2, 4
    n_el = ne ** dim
    c, d = 3.0, 0.7
    K1, M1 = assembly.assemble(dim, ne, p, s)
    Kc, Mc = assembly.assemble(dim, ne, p, s, c * np.ones(n_el), d * np.ones(n_el))
    l1, U1 = eigen.dense_eigh(K1, M1)
    lc, Uc = eigen.dense_eigh(Kc, Mc)
    assert np.max(np.abs(lc - c / d * l1) / lc) < 1e-12
    simple = np.where((np.diff(l1[:8]) > 1e-6 * l1[1:8]))[0]
    i = int(simple[0])                       # first mode is simple
    assert np.abs(Uc[:, i] - U1[:, i] / np.sqrt(d)).max() < 1e-9


def test_sparse_shift_invert_matches_dense():
    rng = np.random.default_rng(3)
    dim, ne, p, s = 2, 20, 2, 5
    n_el = ne ** dim
    kappa = np.exp(0.5 * rng.standard_normal(n_el))
    rho = np.exp(0.5 * rng.standard_normal(n_el))
    K, M = assembly.assemble(dim, ne, p, s, kappa, rho)
    lam, U = eigen.dense_eigh(K, M)
    ls, Us = eigen.sparse_eigs(K, M, 12, sigma=0.0)
    assert np.max(np.abs(ls - lam[:12]) / lam[:12]) < 1e-11
    assert np.max(eigen.residual(K, M, ls, Us)) < 1e-12
    # simple eigenvalues: same vectors after the shared sign convention
    assert np.abs(np.abs(Us[:, 0]) - np.abs(U[:, 0])).max() < 1e-8
    # the completeness-checked driver gives the same lowest pairs
    lw, Uw = eigen.lowest(K, M, 10, dense_limit=0)
    assert np.max(np.abs(lw - lam[:10]) / lam[:10]) < 1e-11


def test_residual_detects_wrong_pair():
    K, M = assembly.assemble(2, 8, 2, 0)
    lam, U = eigen.dense_eigh(K, M)
    assert eigen.residual(K, M, lam[:1], U[:, :1])[0] < 1e-13
    assert eigen.residual(K, M, lam[:1] * (1 + 1e-6), U[:, :1])[0] > 1e-9


def test_inertia_many_equals_inertia():
    """The pooled counts are the same factorisations as the serial ones."""
    w = workloads.small(2, 12, 3, 4, 10, 0.4)
    kappa, rho = w.coefficients()
    K, M = assembly.assemble(w.dim, w.ne, w.p, w.s, kappa, rho)
    lam = eigen.dense_eigh(K, M)[0]
    sig = [0.5 * (lam[i] + lam[i + 1]) for i in (0, 4, 17, 40)]
    assert eigen.inertia_many(K, M, sig, workers=2) == [eigen.inertia(K, M, x) for x in sig] == [1, 5, 18, 41]
