"""Pins of the oracle's accuracy study (oracle/accuracy.py) against what the
mathematics fixes: the exact spectrum by enumeration, the closed-form
linear-element spectrum, the Courant--Fischer upper bound, the Pythagorean
eigenvalue-error relation (Eq. Pythagorean of arXiv 2009.08167), the
h-convergence rates of smooth modes, and the direction of an anisotropic
mode (which a transposed x/y would flip)."""
import math

import numpy as np
import scipy.linalg as sla

from oracle import accuracy, assembly, eigen


def _dense_pairs(dim, ne, p, s):
    K, M = assembly.assemble(dim, ne, p, s)
    lam, U = eigen.dense_eigh(K, M)
    return lam, U.T  # U rows: eigenvectors


def test_exact_eigenvalues_by_enumeration():
    two = accuracy.exact_eigenvalues(2, 12) / math.pi ** 2
    assert np.allclose(two, [2, 5, 5, 8, 10, 10, 13, 13, 17, 17, 18, 20])
    three = accuracy.exact_eigenvalues(3, 11) / math.pi ** 2
    assert np.allclose(three, [3, 6, 6, 6, 9, 9, 9, 11, 11, 11, 12])
    # brute force over a generous box
    big = np.sort([(i * i + j * j) for i in range(1, 80) for j in range(1, 80)])[:3000]
    assert np.allclose(accuracy.exact_eigenvalues(2, 3000) / math.pi ** 2, big)


def test_linear_elements_closed_form_and_everr():
    ne = 10
    K1, M1 = assembly.matrices_1d(ne, 1, 0)
    mu = sla.eigh(K1[1:-1, 1:-1], M1[1:-1, 1:-1], eigvals_only=True)
    closed = accuracy.linear_fem_eigenvalues_1d(ne, ne - 1)
    assert np.abs(mu - closed).max() <= 1e-10 * closed.max()
    # 2D: the discrete spectrum is the sorted sums mu_i + mu_j
    lam, _ = _dense_pairs(2, ne, 1, 0)
    sums = np.sort((closed[:, None] + closed[None, :]).ravel())
    assert np.abs(lam - sums).max() <= 1e-9 * sums.max()
    ev = accuracy.everr(2, lam)
    ex = accuracy.exact_eigenvalues(2, len(lam))
    assert np.allclose(ev, (sums - ex) / ex, rtol=1e-9, atol=1e-12)


def test_galerkin_eigenvalues_bound_the_exact_ones():
    for p, s in ((2, 0), (2, 2), (3, 4)):
        lam, _ = _dense_pairs(2, 8, p, s)
        assert accuracy.everr(2, lam).min() >= -1e-12, (p, s)


def test_pythagorean_relation_and_overlap_consistency():
    """Eq. Pythagorean: EFerr_E = EVerr + EFerr_L2 for a Galerkin pair, with
    the energy norm integrated directly; and ||u_h - u_e||^2 = 2 - 2|(u_h, u_e)|
    for unit-norm functions (the overlap is computed separately)."""
    for dim, ne, p, s, nm in ((2, 12, 2, 0, 6), (2, 12, 3, 4, 6), (3, 5, 2, 0, 3)):
        lam, U = _dense_pairs(dim, ne, p, s)
        modes = accuracy.diagonal_modes(dim, nm)
        r = accuracy.mode_errors(dim, ne, p, s, lam, U, modes)
        lam_e = math.pi ** 2 * dim * np.arange(1, nm + 1) ** 2
        assert np.allclose(lam[r["match"]], lam_e * (1 + r["ev"]), rtol=1e-12)
        gap = np.abs(r["energy"] - (r["ev"] + r["l2"]))
        assert (gap <= 1e-13 + 1e-10 * r["energy"]).all(), (dim, p, s, gap, r["energy"])
        assert np.abs(r["l2"] - (2 - 2 * np.abs(r["overlap"]))).max() <= 1e-11
        assert (r["ev"] >= -1e-12).all() and (r["l2"] >= 0).all()
        # matched eigenvectors are distinct and strongly aligned
        assert len(set(r["match"].tolist())) == nm
        assert np.abs(r["overlap"]).min() > 0.9


def test_convergence_rates_of_the_lowest_mode():
    """Mode (1,1), p = 2: EVerr ~ h^(2p), EFerr_L2 = ||e||^2 ~ h^(2p+2)."""
    p = 2
    res = []
    for ne in (8, 16):
        lam, U = _dense_pairs(2, ne, p, 0)
        res.append(accuracy.mode_errors(2, ne, p, 0, lam, U, accuracy.diagonal_modes(2, 1)))
    ev_ratio = res[0]["ev"][0] / res[1]["ev"][0]
    l2_ratio = res[0]["l2"][0] / res[1]["l2"][0]
    assert 0.75 * 2 ** (2 * p) <= ev_ratio <= 1.3 * 2 ** (2 * p), ev_ratio
    assert 0.75 * 2 ** (2 * p + 2) <= l2_ratio <= 1.3 * 2 ** (2 * p + 2), l2_ratio


def test_anisotropic_mesh_separates_the_two_orientations():
    """ne = (8, 6): the discrete modes (2,1) and (1,2) differ; each aligns
    with its own exact mode and is orthogonal to the other."""
    ne, p = [8, 6], 2
    K, M = assembly.assemble(2, ne, p, 0)
    lam, U = eigen.dense_eigh(K, M)
    U = U.T
    G = accuracy.overlaps(2, ne, p, 0, U[:6], np.array([[2, 1], [1, 2]]))
    n21, n12 = np.argmax(np.abs(G[:, 0])), np.argmax(np.abs(G[:, 1]))
    assert n21 != n12
    assert abs(G[n21, 0]) > 0.99 and abs(G[n21, 1]) < 1e-6
    assert abs(G[n12, 1]) > 0.99 and abs(G[n12, 0]) < 1e-6
    # the coarser direction (y, 6 elements) carries the larger error
    assert lam[n12] > lam[n21]
