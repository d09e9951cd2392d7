"""GPU tests of the adjoint eigenvalue gradient (riga_eig_grad) and its
torch.autograd.Function, on the 2D 128x128 p=3 rIGA (blocksize 16) workload
with log-normal(0, 0.5) coefficients and loss weights w ~ U(0, 1)^20.

Not in the paper: for simple M-normalised pairs, d lambda / d kappa_e =
u^T K0_e u and d lambda / d rho_e = -lambda u^T M0_e u.  Checked against the
oracle's gradient of the oracle's own eigenpairs, against central finite
differences of the GPU eigenvalues, and through autograd.
"""
import sys

import numpy as np
import pytest

import workloads
from oracle import assembly, eigen, grad

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


@pytest.fixture(scope="module")
def c5_problem():
    riga = _riga()
    w = workloads.c5()
    kappa, rho = w.coefficients()
    pr = riga.assemble(w.dim, w.ne, w.p, w.s, kappa, rho)
    lam, U, res, st = pr.eigs(w.nev)
    return riga, w, kappa, rho, pr, lam, U


def test_gradient_full_size_against_oracle(c5_problem):
    riga, w, kappa, rho, pr, lam, U = c5_problem
    _say("grad vs oracle", w.name)
    wts = w.extra["weights"]
    gk, gr = pr.eig_grad(lam, U, wts)
    gk, gr = gk.cpu().numpy(), gr.cpu().numpy()
    Ko, Mo = assembly.assemble(w.dim, w.ne, w.p, w.s, kappa, rho)
    lo, Uo = eigen.sparse_eigs(Ko, Mo, w.nev + 4, sigma=0.0)
    lo, Uo = lo[:w.nev], Uo[:, :w.nev]
    assert np.max(np.abs(lam - lo) / lo) <= 1e-10
    gko, gro = grad.eig_grad(w.dim, w.ne, w.p, w.s, lo, Uo, wts)
    assert np.abs(gk - gko).max() <= 1e-8 * np.abs(gko).max()
    assert np.abs(gr - gro).max() <= 1e-8 * np.abs(gro).max()
    # Euler identities
    L = wts @ lam
    assert abs(kappa @ gk - L) <= 1e-10 * L
    assert abs(rho @ gr + L) <= 1e-10 * L


@pytest.mark.timeout(600)
def test_gradient_central_differences(c5_problem):
    """Central FD, h = 1e-6 relative, on all 50 seeded elements, for kappa
    and rho (200 perturbed solves).  Accept |g_adj - g_FD| <= 1e-4 |g_FD| +
    10 dL / h, with dL the spread of repeated solves of the unperturbed
    problem (at least 1e-13 L)."""
    riga, w, kappa, rho, pr, lam, U = c5_problem
    wts = w.extra["weights"]
    gk, gr = pr.eig_grad(lam, U, wts)
    gk, gr = gk.cpu().numpy(), gr.cpu().numpy()
    L0 = wts @ lam
    reps = [wts @ pr.eigs(w.nev, vectors=False, seed=s)[0] for s in (1, 2)]
    dL = max(max(abs(r - L0) for r in reps), 1e-13 * L0)
    h = 1e-6
    kd = torch.tensor(kappa, dtype=torch.float64, device="cuda")
    rd = torch.tensor(rho, dtype=torch.float64, device="cuda")
    assert len(w.extra["fd_elements"]) == 50
    worst = 0.0
    for e in w.extra["fd_elements"]:
        for which in ("k", "r"):
            vals = []
            for sgn in (1, -1):
                kp, rp = kd.clone(), rd.clone()
                (kp if which == "k" else rp)[e] *= 1 + sgn * h
                pr.update_coefficients(kp, rp)
                vals.append(wts @ pr.eigs(w.nev, vectors=False)[0])
            base = kappa[e] if which == "k" else rho[e]
            fd = (vals[0] - vals[1]) / (2 * h * base)
            adj = gk[e] if which == "k" else gr[e]
            tol = 1e-4 * abs(fd) + 10 * dL / (h * base)
            worst = max(worst, abs(adj - fd) / tol)
            assert abs(adj - fd) <= tol, (e, which, adj, fd, tol)
    _say("FD on 50 elements x (kappa, rho): worst |adj - fd| / tol", worst)
    pr.update_coefficients(kd, rd)


def test_eigsum_autograd(c5_problem):
    riga, w, kappa, rho, pr, lam, U = c5_problem
    from paper_2009_08167_amd import EigSum
    wts = w.extra["weights"]
    kt = torch.tensor(kappa, dtype=torch.float64, device="cuda", requires_grad=True)
    rt = torch.tensor(rho, dtype=torch.float64, device="cuda", requires_grad=True)
    wt = torch.tensor(wts, dtype=torch.float64, device="cuda")
    loss = EigSum.apply(kt, rt, wt, w.dim, w.ne, w.p, w.s)
    assert abs(loss.item() - wts @ lam) <= 1e-10 * abs(wts @ lam)
    loss.backward()
    gk, gr = pr.eig_grad(lam, U, wts)
    assert torch.allclose(kt.grad, gk, rtol=1e-9, atol=1e-12 * gk.abs().max().item())
    assert torch.allclose(rt.grad, gr, rtol=1e-9, atol=1e-12 * gr.abs().max().item())
    # d L / d w_i = lambda_i
    wt2 = wt.clone().requires_grad_(True)
    loss2 = EigSum.apply(kt.detach(), rt.detach(), wt2, w.dim, w.ne, w.p, w.s)
    loss2.backward()
    assert np.allclose(wt2.grad.cpu().numpy(), lam, rtol=1e-12, atol=0)


def test_eigsum_rejects_a_loss_cut_through_a_multiple_eigenvalue():
    """kappa = rho = 1 on the square: lambda_2 = lambda_3 (modes (1,2) and
    (2,1)); a loss over the two lowest cuts that pair, has no gradient, and
    is refused with RIGA_EDEGENERATE."""
    riga = _riga()
    from paper_2009_08167_amd import EigSum
    ne = 16
    k = torch.ones(ne * ne, dtype=torch.float64, device="cuda", requires_grad=True)
    r = torch.ones(ne * ne, dtype=torch.float64, device="cuda", requires_grad=True)
    wt = torch.tensor([1.0, 0.5], dtype=torch.float64, device="cuda")
    with pytest.raises(riga.RigaError) as e:
        EigSum.apply(k, r, wt, 2, ne, 2, 0)
    assert e.value.code == riga.RIGA_EDEGENERATE


def test_gradient_rejects_degenerate_pairs():
    riga = _riga()
    pr = riga.assemble(2, 16, 2, 0)                  # kappa = rho = 1: lambda_2 = lambda_3
    lam, U, res, st = pr.eigs(3)
    with pytest.raises(riga.RigaError) as e:
        pr.eig_grad(lam, U, np.ones(3))
    assert e.value.code == riga.RIGA_EDEGENERATE
