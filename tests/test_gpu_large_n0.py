"""Many shifts: requests of 1,500 (2D) and 600 (3D) eigenpairs, where the
Lanczos runs deflate only against the locked pairs of a window below the
shift (and all above it).  Checked against the exact discrete spectrum of
the Kronecker sums (kappa = rho = 1: sorted sums of the 1D eigenvalues,
Eq. 2Dmatrix and its 3D analogue), M-orthonormality of every returned
vector with the oracle's Kronecker M (a pair locked twice or a lost
direction would break it), and the same spectrum with the window switched
off (RIGA_DEFLATE_ALL=1)."""
import os
import sys

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import assembly

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _riga():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_08167_amd import riga
    riga.lib()
    return riga


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _kron_spectrum(dim, ne, p, s, count):
    K1, M1 = assembly.matrices_1d(ne, p, s)
    mu = sla.eigh(K1[1:-1, 1:-1], M1[1:-1, 1:-1], eigvals_only=True)
    lam = mu
    for _ in range(dim - 1):
        lam = (lam[:, None] + mu[None, :]).ravel()
    return np.sort(lam)[:count]


@pytest.mark.parametrize("case", [(2, 64, 3, 8, 1500), (3, 16, 2, 4, 600)],
                         ids=["2d_64_p3_s8_1500", "3d_16_p2_s4_600"])
def test_many_shifts_window_deflation(case):
    riga = _riga()
    dim, ne, p, s, nev = case
    _say("many shifts", case)
    pr = riga.assemble(dim, ne, p, s)
    lam, U, res, st = pr.eigs(nev)
    _say("stats", st)
    assert len(lam) == nev and res.max() <= 1e-9
    exact = _kron_spectrum(dim, ne, p, s, nev)
    rel = np.abs(lam - exact) / exact
    _say("max rel vs Kronecker spectrum", rel.max())
    assert rel.max() <= 1e-10
    Ko, Mo = assembly.kronecker_interior(dim, ne, p, s)
    Uh = U.cpu().numpy()
    G = Uh.T @ (Mo @ Uh)
    D = np.abs(G - np.eye(nev))
    orth = D.max()
    i, j = np.unravel_index(np.argmax(D), D.shape)
    _say("max |U^T M U - I|", orth, "at", (i, j), "lambda", lam[i], lam[j],
         "rel gap", abs(lam[i] - lam[j]) / lam[i], "residuals", res[i], res[j])
    worst = np.argsort(D.ravel())[::-1][:12]
    for q in worst:
        a, b = np.unravel_index(q, D.shape)
        if a <= b:
            _say("  pair", (a, b), D[a, b], lam[a], lam[b], res[a], res[b])
    assert orth <= 1e-10
    old = os.environ.get("RIGA_DEFLATE_ALL")
    os.environ["RIGA_DEFLATE_ALL"] = "1"
    try:
        lam_all, _, res_all, st_all = pr.eigs(nev, vectors=False)
    finally:
        if old is None:
            del os.environ["RIGA_DEFLATE_ALL"]
        else:
            os.environ["RIGA_DEFLATE_ALL"] = old
    _say("full deflation stats", st_all)
    assert np.abs(lam_all - lam).max() <= 1e-10 * lam.max()


def test_high_degree_iga_4096_pairs():
    """2D 256^2 p = 4 IGA, the 4096 lowest pairs: Ritz pairs of high-degree
    IGA at about lambda = 3e4 can stall at residuals of 1-6e-9, just above
    the 1e-9 tolerance (the FP64 solve's own error); the solver then refines
    its solves (stats n_ir > 0) and finishes.  Whether a run stalls depends
    on rounding details, so only the outcome is checked: eigenvalues against
    the Kronecker-sum spectrum, residuals, and M-orthonormality of 64 sampled
    eigenvectors with the oracle's Kronecker M."""
    riga = _riga()
    dim, ne, p, s, nev = 2, 256, 4, 0, 4096
    _say("high-degree IGA", dim, ne, p, nev)
    pr = riga.assemble(dim, ne, p, s)
    lam, U, res, st = pr.eigs(nev)
    _say("stats", st)
    assert len(lam) == nev and res.max() <= 1e-9
    exact = _kron_spectrum(dim, ne, p, s, nev)
    rel = np.abs(lam - exact) / exact
    _say("max rel vs Kronecker spectrum", rel.max())
    assert rel.max() <= 1e-10
    Ko, Mo = assembly.kronecker_interior(dim, ne, p, s)
    pick = np.random.default_rng(7).choice(nev, 64, replace=False)
    Us = U[:, torch.tensor(pick, device=U.device)].cpu().numpy()
    G = Us.T @ (Mo @ Us)
    orth = np.abs(G - np.eye(64)).max()
    _say("sampled max |U^T M U - I|", orth)
    assert orth <= 1e-10
