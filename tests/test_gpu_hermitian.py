"""GPU parity of complex Hermitian pencils (Eq. GHEP read with conjugate
transposes; Sec. 4 solves generalized Hermitian eigenproblems) against the
oracle's magnetic Laplacian (oracle/hermitian.py, pinned by Hermitian
symmetry, the real limit, the Kronecker form, gauge-invariant convergence and
the eigenvector phase).

The library solves the real-equivalent pencil [[Re K, -Im K], [Im K, Re K]],
diag(M, M) with the two parts of a DOF interleaved, locking J u (times i)
with every converged u.  Checked: the assembled real-equivalent matrices
against the oracle's (re-ordered to the interleaved layout), the complex
eigenvalues against the oracle's dense Hermitian solve (1e-10 relative),
residuals with the oracle's complex K and M (1e-9), M-orthonormality of the
complex eigenvectors (1e-10) and containment in the oracle's eigenspaces
(1e-8), inertia counts (twice the complex count), and the refusals."""
import sys

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import eigen, hermitian

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


CASES = [(2, 10, 2, 5, (0.9, -1.7), 20), (2, 12, 3, 0, (2.5, 0.7), 24), (3, 4, 2, 2, (0.4, 1.1, -0.6), 16),
         (2, 13, 4, 4, (-1.3, 3.1), 30), (2, 40, 3, 8, (1.7, -0.4), 40),
         (3, 8, 2, 4, (0.6, -0.9, 1.2), 24)]


def _interleave(N):
    """Index map: interleaved unknown 2d + t -> block-ordered t N + d."""
    d = np.arange(N)
    perm = np.empty(2 * N, dtype=np.int64)
    perm[0::2] = d
    perm[1::2] = N + d
    return perm


@pytest.mark.parametrize("case", CASES, ids=lambda c: "%dd_%d_p%d_s%d" % c[:4])
def test_assembly_real_equivalent(case):
    riga = _riga()
    dim, ne, p, s, A, _ = case
    pr = riga.assemble(dim, ne, p, s, potential=A)
    K2, M2 = pr.matrices()
    Kc, Mc = hermitian.assemble_magnetic(dim, ne, p, s, A)
    Kb, Mb = hermitian.real_equivalent(Kc, Mc)
    P = _interleave(Kc.shape[0])
    Ko = Kb[P][:, P]
    Mo = Mb[P][:, P]
    _say("hermitian assembly", case, "N", Kc.shape[0])
    assert K2.shape == Ko.shape
    assert abs(K2 - Ko).max() <= 1e-13 * abs(Ko).max()
    assert abs(M2 - Mo).max() <= 1e-13 * abs(Mo).max()
    # the stored pattern holds every 2 x 2 block of a scalar coupling
    assert K2.nnz == 4 * Kc.nnz


@pytest.mark.parametrize("case", CASES, ids=lambda c: "%dd_%d_p%d_s%d" % c[:4])
def test_eigs_match_dense_hermitian_oracle(case):
    riga = _riga()
    dim, ne, p, s, A, nev = case
    pr = riga.assemble(dim, ne, p, s, potential=A)
    Kc, Mc = hermitian.assemble_magnetic(dim, ne, p, s, A)
    lr, Ur = hermitian.dense_eigh_hermitian(Kc, Mc)
    _say("hermitian eigs", case, "N", Kc.shape[0])
    for prec in (riga.RIGA_FP64, riga.RIGA_MIXED):
        lam, U, res, st = pr.eigs(nev, precision=prec, per_shift=12)
        _say("precision", prec, "stats", st)
        assert len(lam) == nev and U.shape == (Kc.shape[0], nev) and U.is_complex()
        rel = np.abs(lam - lr[:nev]) / lr[:nev]
        if rel.max() > 1e-10:
            _say("returned", lam, "\noracle", lr[:nev + 4])
        assert rel.max() <= 1e-10, rel.max()
        Uh = U.cpu().numpy()
        Kd, Md = Kc.toarray(), Mc.toarray()
        nK = np.abs(Kd).sum(axis=0).max()
        R = Kd @ Uh - (Md @ Uh) * lam[None, :]
        r = np.linalg.norm(R, axis=0) / (nK * np.linalg.norm(Uh, axis=0))
        assert r.max() <= 1e-9, r.max()
        G = Uh.conj().T @ Md @ Uh
        assert np.abs(G - np.eye(nev)).max() <= 1e-10
        # eigenvectors lie in the oracle's eigenspace, compared as one
        # subspace within a cluster: the discrete pencil splits the
        # Laplacian's double eigenvalues only slightly (relative gaps down to
        # 5.5e-8 at p = 4), and a vector's error is its residual over the gap
        for i in range(nev):
            cl = np.where(np.abs(lr - lr[i]) <= 1e-5 * abs(lr[i]))[0]
            Q = Ur[:, cl]
            u = Uh[:, i]
            d = u - Q @ (Q.conj().T @ (Md @ u))
            assert np.sqrt(abs(d.conj() @ (Md @ d))) <= 1e-8, (i, cl)


def test_inertia_counts_twice():
    """The real-equivalent pencil counts every complex eigenvalue twice."""
    riga = _riga()
    dim, ne, p, s, A, _ = CASES[0]
    pr = riga.assemble(dim, ne, p, s, potential=A)
    Kc, Mc = hermitian.assemble_magnetic(dim, ne, p, s, A)
    lr = hermitian.dense_eigh_hermitian(Kc, Mc)[0]
    for i in (0, 3, 11, 40):
        sigma = 0.5 * (lr[i] + lr[i + 1])
        neg, st = pr.factor(sigma)
        assert neg == 2 * (i + 1), (sigma, neg)


def test_complex_pencil_refusals():
    riga = _riga()
    with pytest.raises(riga.RigaError) as e:
        riga.assemble(2, 8, 2, 4, kappa=np.ones(64), rho=np.ones(64), potential=(1.0, 0.5))
    assert e.value.code == riga.RIGA_EUNSUPPORTED
    pr = riga.assemble(2, 8, 2, 4, potential=(1.0, 0.5))
    lam, U, res, st = pr.eigs(4)
    with pytest.raises(riga.RigaError) as e:
        pr.eig_grad(lam, torch.view_as_real(U).reshape(pr.n_dof, 4).contiguous(), np.ones(4))
    assert e.value.code == riga.RIGA_EUNSUPPORTED
