"""Pins of the oracle's adjoint eigenvalue gradient.

Checked against central finite differences of eigenvalues (each perturbed
problem re-solved by the dense oracle) and the Euler identities that
degree-1 homogeneity of lambda in kappa and degree -1 in rho imply:
sum_e kappa_e d lambda/d kappa_e = lambda, sum_e rho_e d lambda/d rho_e = -lambda.
"""
import numpy as np

from oracle import assembly, eigen, grad


def _problem(seed=11):
    dim, ne, p, s = 2, 6, 2, 3
    rng = np.random.default_rng(seed)
    n_el = ne ** dim
    kappa = np.exp(0.5 * rng.standard_normal(n_el))
    rho = np.exp(0.5 * rng.standard_normal(n_el))
    return dim, ne, p, s, kappa, rho


def test_euler_identities():
    dim, ne, p, s, kappa, rho = _problem()
    K, M = assembly.assemble(dim, ne, p, s, kappa, rho)
    lam, U = eigen.dense_eigh(K, M)
    for i in range(5):
        gk, gr = grad.eig_grad(dim, ne, p, s, lam[i:i + 1], U[:, i:i + 1], [1.0])
        assert abs(kappa @ gk - lam[i]) < 1e-11 * lam[i]
        assert abs(rho @ gr + lam[i]) < 1e-11 * lam[i]


def test_central_finite_differences():
    dim, ne, p, s, kappa, rho = _problem()
    K, M = assembly.assemble(dim, ne, p, s, kappa, rho)
    lam, U = eigen.dense_eigh(K, M)
    nev = 6
    w = np.linspace(0.2, 1.0, nev)
    gk, gr = grad.eig_grad(dim, ne, p, s, lam[:nev], U[:, :nev], w)
    h = 1e-5
    for e in (0, 7, 20, 35):
        for which in ("k", "r"):
            vals = []
            for sgn in (1, -1):
                kp, rp = kappa.copy(), rho.copy()
                (kp if which == "k" else rp)[e] *= 1 + sgn * h
                Kp, Mp = assembly.assemble(dim, ne, p, s, kp, rp)
                vals.append(w @ eigen.dense_eigh(Kp, Mp)[0][:nev])
            base = kappa[e] if which == "k" else rho[e]
            fd = (vals[0] - vals[1]) / (2 * h * base)
            adj = gk[e] if which == "k" else gr[e]
            assert abs(adj - fd) <= 1e-6 * abs(fd) + 1e-7, (e, which, adj, fd)
