"""GPU parity of the accuracy study (riga_mode_errors): eigenfunction errors
of computed eigenpairs against the exact Laplace modes (Eqs. exact, norms,
eigerrors of arXiv 2009.08167; diagonal modes as in Sec. 8).

* Parity: the oracle's dense eigenpairs go to both the GPU entry point and
  the oracle (oracle/accuracy.py), which compute the same integrals with the
  same Gauss rule; the matched indices must agree exactly, the overlaps,
  EFerr_L2 and EFerr_E to summation-order rounding.
* Whole path: eigenpairs from the GPU solver of a larger problem, checked
  through what holds at any size: the Pythagorean relation EFerr_E = EVerr +
  EFerr_L2 (energy norm integrated directly), the Courant--Fischer bound
  EVerr >= 0 against the sorted exact spectrum, distinct matches, and the
  L2 error against 2 - 2 |overlap|.
"""
import sys

import numpy as np
import pytest

from oracle import accuracy, assembly, eigen

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


CASES = [(2, 12, 2, 0, 6, 0), (2, 12, 3, 4, 6, 0), (2, 9, 4, 3, 5, 12), (3, 5, 2, 0, 3, 0),
         (3, 6, 3, 2, 2, 5)]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "%dd_%d_p%d_s%d_q%d" % (c[0], c[1], c[2], c[3], c[5]))
def test_mode_errors_match_oracle(case):
    dim, ne, p, s, nm, q = case
    riga = _riga()
    _say("mode errors", case)
    K, M = assembly.assemble(dim, ne, p, s)
    lam, U = eigen.dense_eigh(K, M)
    nvec = min(len(lam), 60)
    lam, U = lam[:nvec], U[:, :nvec]
    modes = accuracy.diagonal_modes(dim, nm)
    qq = q if q else accuracy.default_q(p)
    ref = accuracy.mode_errors(dim, ne, p, s, lam, U.T, modes, qq)
    pr = riga.assemble(dim, ne, p, s)
    got = pr.mode_errors(lam, U, modes, nquad=q)
    _say("match", got["match"], "l2", got["l2"])
    assert np.array_equal(got["match"], ref["match"])
    assert np.abs(got["overlap"] - ref["overlap"]).max() <= 1e-13
    for key in ("l2", "energy"):
        err = np.abs(got[key] - ref[key])
        assert (err <= 1e-10 * ref[key] + 1e-18).all(), (key, got[key], ref[key])
    assert np.allclose(got["ev"], ref["ev"], rtol=1e-12, atol=1e-15)


def test_single_vector_single_mode_and_bad_arguments():
    riga = _riga()
    K, M = assembly.assemble(2, 8, 2, 4)
    lam, U = eigen.dense_eigh(K, M)
    pr = riga.assemble(2, 8, 2, 4)
    got = pr.mode_errors(lam[:1], U[:, :1], np.array([[1, 1]]))
    ref = accuracy.mode_errors(2, 8, 2, 4, lam[:1], U[:, :1].T, np.array([[1, 1]]))
    assert got["match"][0] == 0 and ref["match"][0] == 0
    assert abs(got["l2"][0] - ref["l2"][0]) <= 1e-10 * ref["l2"][0]
    with pytest.raises(riga.RigaError):
        pr.mode_errors(lam[:2], U[:, :2], np.array([[0, 1]]))
    with pytest.raises(riga.RigaError):
        pr.mode_errors(lam[:2], U[:, :2], np.array([[1, 1]]), nquad=17)


@pytest.mark.parametrize("s", [0, 8], ids=["iga", "riga8"])
def test_solver_pairs_satisfy_the_error_relations(s):
    """2D 48^2, p = 3: the 300 lowest pairs from the GPU solver."""
    riga = _riga()
    dim, ne, p, nev, nm = 2, 48, 3, 300, 12
    pr = riga.assemble(dim, ne, p, s)
    lam, U, res, st = pr.eigs(nev)
    _say("solver pairs", s, st["n_fb"])
    ev_all = (lam - riga.exact_eigenvalues(dim, nev)) / riga.exact_eigenvalues(dim, nev)
    assert ev_all.min() >= -1e-12
    r = pr.mode_errors(lam, U, accuracy.diagonal_modes(dim, nm))
    _say("ev", r["ev"], "l2", r["l2"], "energy", r["energy"])
    assert len(set(r["match"].tolist())) == nm
    gap = np.abs(r["energy"] - (r["ev"] + r["l2"]))
    assert (gap <= 1e-11 + 1e-8 * r["energy"]).all(), gap
    assert np.abs(r["l2"] - (2 - 2 * np.abs(r["overlap"]))).max() <= 1e-10
    assert (r["ev"] >= -1e-12).all() and (r["ev"] < 0.1).all()
