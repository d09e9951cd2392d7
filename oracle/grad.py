"""Adjoint gradient of a weighted eigenvalue sum with respect to per-element
coefficients.

Test infrastructure only (see the package docstring).

Not in the paper.  For a simple eigenpair of the symmetric pencil K(kappa) u =
lambda M(rho) u with u^T M u = 1, first-order perturbation gives
d lambda = u^T (dK - lambda dM) u.  With K = sum_e kappa_e K0_e and
M = sum_e rho_e M0_e (K0_e, M0_e the unit-coefficient element matrices,
restricted to the interior functions):

    d lambda / d kappa_e =  u^T K0_e u,
    d lambda / d rho_e   = -lambda u^T M0_e u.

For the loss L = sum_i w_i lambda_i the gradient is the w-weighted sum.
"""
import itertools

import numpy as np

from . import assembly


def eig_grad(dim, ne, p, s, lam, U, w, q=None):
    """Gradient of sum_i w_i lam_i w.r.t. (kappa_e, rho_e), x-fastest elements.

    ``U`` holds M-normalised interior eigenvectors (columns)."""
    spaces = assembly.make_spaces(dim, ne, p, s, q)
    ns = [s1.n for s1 in spaces]
    nes = [s1.ne for s1 in spaces]
    interior = assembly.interior_index(spaces)
    full_to_int = -np.ones(int(np.prod(ns)), dtype=np.int64)
    full_to_int[interior] = np.arange(interior.size)
    U = np.atleast_2d(U.T).T
    lam = np.atleast_1d(lam)
    w = np.atleast_1d(w)
    n_el = int(np.prod(nes))
    gk = np.zeros(n_el)
    gr = np.zeros(n_el)
    estrides = np.cumprod([1] + nes[:-1])
    for eidx in itertools.product(*[range(n) for n in reversed(nes)]):
        eidx = eidx[::-1]
        e = int(np.dot(eidx, estrides))
        k0, m0, gidx = assembly.element_unit_matrices(spaces, eidx)
        loc = full_to_int[gidx]
        ul = np.zeros((gidx.size, U.shape[1]))
        keep = loc >= 0                      # Dirichlet functions are zero
        ul[keep] = U[loc[keep]]
        qk = np.einsum('ai,ab,bi->i', ul, k0, ul)
        qm = np.einsum('ai,ab,bi->i', ul, m0, ul)
        gk[e] = np.sum(w * qk)
        gr[e] = -np.sum(w * lam * qm)
    return gk, gr
