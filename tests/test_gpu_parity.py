"""GPU parity tests: the HIP path through the C ABI against the CPU oracle on
the same seeded inputs (workloads.py).

Bars (from the rounding of each computation): assembled K, M entries within 1e-13 relative
to the matrix max; solves with backward error <= 1e-12; inertia exact;
eigenvalues within 1e-10 relative, residuals <= 1e-9, M-orthonormality
within 1e-10, eigenvectors of a cluster inside the oracle's cluster
subspace within 1e-8 (M-norm).
"""
import sys

import numpy as np
import pytest
import scipy.sparse as sp

import workloads
from oracle import assembly, eigen, grad

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _riga():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_08167_amd import riga
    riga.lib()  # raises if the library is missing: no fallback
    return riga


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


ASM_CASES = [workloads.c1(), workloads.small(2, 24, 3, 8, 10, 0.5),
             workloads.small(3, 6, 2, 3, 10, 0.4), workloads.small(2, 19, 4, 5, 10, 0.5),
             workloads.small(2, 12, 1, 0, 10, 0.2)]


@pytest.mark.parametrize("w", ASM_CASES, ids=lambda w: w.name)
def test_assembly_matches_oracle(w):
    riga = _riga()
    _say("assembly", w.name)
    kappa, rho = w.coefficients()
    pr = riga.assemble(w.dim, w.ne, w.p, w.s, kappa, rho)
    K, M = pr.matrices()
    Ko, Mo = assembly.assemble(w.dim, w.ne, w.p, w.s, kappa, rho)
    assert abs(K - Ko).max() <= 1e-13 * abs(Ko).max()
    assert abs(M - Mo).max() <= 1e-13 * abs(Mo).max()


def test_spmv_matches_oracle():
    riga = _riga()
    w = workloads.small(2, 20, 3, 5, 10, 0.5)
    _say("spmv", w.name)
    kappa, rho = w.coefficients()
    pr = riga.assemble(w.dim, w.ne, w.p, w.s, kappa, rho)
    Ko, Mo = assembly.assemble(w.dim, w.ne, w.p, w.s, kappa, rho)
    x = np.random.default_rng(5).standard_normal(pr.n_dof)
    xd = torch.tensor(x, dtype=torch.float64, device="cuda")
    for which, A in ((riga.RIGA_MAT_K, Ko), (riga.RIGA_MAT_M, Mo)):
        y = pr.spmv(which, xd).cpu().numpy()
        yo = A @ x
        assert np.abs(y - yo).max() <= 1e-13 * np.abs(yo).max()


FACT_CASES = [workloads.small(2, 16, 2, 0, 10, 0.3), workloads.small(2, 24, 3, 8, 10, 0.5),
              workloads.small(3, 6, 2, 3, 10, 0.3), workloads.small(2, 40, 3, 8, 10, 0.3),
              workloads.small(3, 10, 2, 0, 10, 0.3), workloads.small(2, 64, 3, 0, 10, 0.3),
              workloads.small(2, 96, 2, 16, 10, 0.3)]


@pytest.mark.parametrize("w", FACT_CASES, ids=lambda w: w.name)
def test_factor_inertia_and_solve(w):
    riga = _riga()
    kappa, rho = w.coefficients()
    pr = riga.assemble(w.dim, w.ne, w.p, w.s, kappa, rho, leaf_dofs=32)
    Ko, Mo = assembly.assemble(w.dim, w.ne, w.p, w.s, kappa, rho)
    lam = eigen.dense_eigh(Ko, Mo)[0] if Ko.shape[0] <= 2500 else None
    rng = np.random.default_rng(9)
    b = rng.standard_normal(pr.n_dof)
    bd = torch.tensor(b, dtype=torch.float64, device="cuda")
    for i in (0, 5, 30, 120):
        if lam is not None:
            if i + 1 >= len(lam):
                continue
            sigma = 0.5 * (lam[i] + lam[i + 1]) if i > 0 else 0.0
            expect = int(np.count_nonzero(lam < sigma))
        else:
            sigma = [0.0, 400.0, 2500.0, 9000.0][[0, 5, 30, 120].index(i)]
            expect = eigen.inertia(Ko, Mo, sigma)
        _say("factor", w.name, "sigma", sigma)
        neg, st = pr.factor(sigma)
        assert neg == expect, (sigma, neg, expect)
        x = pr.solve(bd).cpu().numpy()
        A = (Ko - sigma * Mo).tocsr()
        r = b - A @ x
        berr = np.linalg.norm(r) / (sp.linalg.norm(A, 1) * np.linalg.norm(x) + np.linalg.norm(b))
        assert berr <= 1e-12, (sigma, berr)


def _check_pairs(Ko, Mo, lam_ref, U_ref, lam, U, res, nev, tol_val=1e-10):
    """Eigenvalues index by index, residuals, M-orthonormality, and
    containment of each vector in the oracle's eigenspace of its cluster."""
    assert len(lam) == nev
    rel = np.abs(lam - lam_ref[:nev]) / np.abs(lam_ref[:nev])
    assert rel.max() <= tol_val, rel.max()
    r = eigen.residual(Ko, Mo, lam, U)
    assert r.max() <= 1e-9, r.max()
    assert np.abs(res - r).max() <= 1e-9
    G = U.T @ (Mo @ U)
    assert np.abs(G - np.eye(nev)).max() <= 1e-10
    # cluster subspaces from the reference (relative gap 1e-8)
    for i in range(nev):
        cl = np.where(np.abs(lam_ref - lam_ref[i]) <= 1e-8 * abs(lam_ref[i]))[0]
        Q = U_ref[:, cl]
        u = U[:, i]
        proj = Q @ (Q.T @ (Mo @ u))
        d = u - proj
        assert np.sqrt(d @ (Mo @ d)) <= 1e-8, (i, cl)


def test_eigs_c1_lowest_10():
    riga = _riga()
    w = workloads.c1()
    _say("eigs", w.name)
    kappa, rho = w.coefficients()
    pr = riga.assemble(w.dim, w.ne, w.p, w.s, kappa, rho)
    lam, U, res, st = pr.eigs(w.nev)
    Ko, Mo = assembly.assemble(w.dim, w.ne, w.p, w.s, kappa, rho)
    lr, Ur = eigen.dense_eigh(Ko, Mo)
    _check_pairs(Ko, Mo, lr, Ur, lam, U.cpu().numpy(), res, w.nev)
    _say("stats", st)


EIG_CASES = [workloads.small(2, 24, 3, 8, 40, 0.5), workloads.small(3, 6, 2, 3, 30, 0.0),
             workloads.small(2, 30, 2, 0, 60, 0.3), workloads.small(2, 20, 4, 5, 25, 0.5)]


@pytest.mark.parametrize("w", EIG_CASES, ids=lambda w: w.name)
def test_eigs_small_against_dense_oracle(w):
    riga = _riga()
    _say("eigs", w.name)
    kappa, rho = w.coefficients()
    pr = riga.assemble(w.dim, w.ne, w.p, w.s, kappa, rho, leaf_dofs=32)
    lam, U, res, st = pr.eigs(w.nev, per_shift=16)
    _say("stats", st)
    Ko, Mo = assembly.assemble(w.dim, w.ne, w.p, w.s, kappa, rho)
    lr, Ur = eigen.dense_eigh(Ko, Mo)
    _check_pairs(Ko, Mo, lr, Ur, lam, U.cpu().numpy(), res, w.nev)


def test_eigs_interval():
    """[lo, hi) with both ends finite: exactly the eigenvalues inside."""
    riga = _riga()
    w = workloads.small(2, 20, 2, 5, 200, 0.4)
    kappa, rho = w.coefficients()
    Ko, Mo = assembly.assemble(w.dim, w.ne, w.p, w.s, kappa, rho)
    lr, Ur = eigen.dense_eigh(Ko, Mo)
    lo = 0.5 * (lr[9] + lr[10])
    hi = 0.5 * (lr[29] + lr[30])
    pr = riga.assemble(w.dim, w.ne, w.p, w.s, kappa, rho)
    lam, U, res, st = pr.eigs(200, lo=lo, hi=hi, per_shift=8)
    assert len(lam) == 20
    assert np.max(np.abs(lam - lr[10:30]) / lr[10:30]) <= 1e-10


def test_eigs_deterministic():
    riga = _riga()
    w = workloads.small(2, 24, 3, 8, 20, 0.5)
    kappa, rho = w.coefficients()
    pr = riga.assemble(w.dim, w.ne, w.p, w.s, kappa, rho)
    a = pr.eigs(w.nev, per_shift=12)
    b = pr.eigs(w.nev, per_shift=12)
    assert np.array_equal(a[0], b[0])
    assert torch.equal(a[1], b[1])


def test_eigs_deterministic_with_two_slices_and_lookahead():
    """A request large enough to split into two spectrum slices (two host
    threads, two streams, each with its look-ahead factorisation): repeated
    solves return bitwise the same eigenvalues and vectors."""
    riga = _riga()
    w = workloads.small(2, 64, 3, 16, 160, 0.3)
    kappa, rho = w.coefficients()
    pr = riga.assemble(w.dim, w.ne, w.p, w.s, kappa, rho)
    a = pr.eigs(w.nev)
    b = pr.eigs(w.nev)
    c = pr.eigs(w.nev)
    _say("two slices", a[3]["n_shift"], a[3]["n_fb"])
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[0], c[0])
    assert torch.equal(a[1], b[1]) and torch.equal(a[1], c[1])


def test_gradient_matches_oracle():
    riga = _riga()
    w = workloads.small(2, 16, 3, 8, 8, 0.5)
    _say("grad", w.name)
    kappa, rho = w.coefficients()
    pr = riga.assemble(w.dim, w.ne, w.p, w.s, kappa, rho)
    wts = np.linspace(0.3, 1.0, w.nev)
    # the oracle's own eigenpairs go to both sides
    Ko, Mo = assembly.assemble(w.dim, w.ne, w.p, w.s, kappa, rho)
    lo, Uo = eigen.dense_eigh(Ko, Mo)
    lo, Uo = lo[:w.nev], Uo[:, :w.nev]
    gk, gr = pr.eig_grad(lo, torch.tensor(Uo, device="cuda"), wts)
    gko, gro = grad.eig_grad(w.dim, w.ne, w.p, w.s, lo, Uo, wts)
    gk, gr = gk.cpu().numpy(), gr.cpu().numpy()
    assert np.abs(gk - gko).max() <= 1e-12 * np.abs(gko).max()
    assert np.abs(gr - gro).max() <= 1e-12 * np.abs(gro).max()
    # the solver's own pairs: Euler identities (degree-1 homogeneity in
    # kappa, -1 in rho), which hold at any size
    lam, U, res, st = pr.eigs(w.nev)
    gk, gr = pr.eig_grad(lam, U, wts)
    gk, gr = gk.cpu().numpy(), gr.cpu().numpy()
    assert abs(kappa @ gk - wts @ lam) <= 1e-10 * (wts @ lam)
    assert abs(rho @ gr + wts @ lam) <= 1e-10 * (wts @ lam)


MIXED_CASES = [workloads.small(2, 24, 3, 8, 10, 0.5), workloads.small(3, 10, 2, 5, 10, 0.0),
               workloads.small(2, 64, 2, 16, 10, 0.3)]


@pytest.mark.parametrize("w", MIXED_CASES, ids=lambda w: w.name)
def test_mixed_factor_inertia_and_refined_solve(w):
    """FP32 fronts: same inertia as FP64; FP64 iterative refinement brings
    the solve to backward error <= 1e-13 relative residual."""
    riga = _riga()
    _say("mixed factor", w.name)
    kappa, rho = w.coefficients()
    pr = riga.assemble(w.dim, w.ne, w.p, w.s, kappa, rho, leaf_dofs=32)
    Ko, Mo = assembly.assemble(w.dim, w.ne, w.p, w.s, kappa, rho)
    rng = np.random.default_rng(4)
    b = rng.standard_normal(pr.n_dof)
    bd = torch.tensor(b, dtype=torch.float64, device="cuda")
    for sigma in (0.0, 350.0, 1200.0):
        n64, _ = pr.factor(sigma, riga.RIGA_FP64)
        n32, _ = pr.factor(sigma, riga.RIGA_MIXED)
        assert n32 == n64, (sigma, n32, n64)
        x0 = pr.solve(bd, max_ir=0).cpu().numpy()
        x = pr.solve(bd, max_ir=30).cpu().numpy()
        A = (Ko - sigma * Mo).tocsr()
        r0 = np.linalg.norm(b - A @ x0) / np.linalg.norm(b)
        for it in (1, 2, 3, 4):
            xi = pr.solve(bd, max_ir=it).cpu().numpy()
            _say("  ir", it, np.linalg.norm(b - A @ xi) / np.linalg.norm(b))
        r = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
        _say("sigma", sigma, "fp32 solve residual", r0, "refined", r)
        assert r0 < 1e-2
        assert r <= 1e-12, r


@pytest.mark.parametrize("w", [workloads.small(2, 24, 3, 8, 30, 0.5),
                               workloads.small(3, 8, 2, 4, 24, 0.0)], ids=lambda w: w.name)
def test_mixed_eigs_match_fp64_bar(w):
    riga = _riga()
    _say("mixed eigs", w.name)
    kappa, rho = w.coefficients()
    pr = riga.assemble(w.dim, w.ne, w.p, w.s, kappa, rho, leaf_dofs=32)
    lam, U, res, st = pr.eigs(w.nev, precision=riga.RIGA_MIXED, per_shift=16)
    _say("stats", st)
    assert st["n_ir"] > 0
    Ko, Mo = assembly.assemble(w.dim, w.ne, w.p, w.s, kappa, rho)
    lr, Ur = eigen.dense_eigh(Ko, Mo)
    _check_pairs(Ko, Mo, lr, Ur, lam, U.cpu().numpy(), res, w.nev)


def test_budget_exhausted_returns_only_verified_pairs():
    """With a tiny restart budget on a spectrum with 3- and 6-fold
    multiplicities (3D, kappa = rho = 1), the solver may stop early; every
    pair it returns must then be exactly the lowest eigenvalues (no gap), as
    the inertia count at its last completed shift guarantees."""
    riga = _riga()
    w = workloads.small(3, 6, 2, 3, 60, 0.0)
    _say("budget", w.name)
    pr = riga.assemble(w.dim, w.ne, w.p, w.s, leaf_dofs=32)
    lam, U, res, st = pr.eigs(w.nev, per_shift=8, max_basis=20, max_restarts=1, allow_partial=True)
    _say("found", len(lam), "stats", st)
    Ko, Mo = assembly.assemble(w.dim, w.ne, w.p, w.s)
    lr = eigen.dense_eigh(Ko, Mo)[0]
    n = len(lam)
    if n:
        assert np.max(np.abs(lam - lr[:n]) / lr[:n]) <= 1e-10
        assert res.max() <= 1e-9


def test_solve_multi_matches_solve():
    """riga_solve_multi queues the sweeps back to back: every column equals
    riga_solve's result bit for bit, FP64 and refined mixed precision."""
    riga = _riga()
    w = workloads.small(2, 40, 3, 8, 10, 0.3)
    _say("solve_multi", w.name)
    kappa, rho = w.coefficients()
    pr = riga.assemble(w.dim, w.ne, w.p, w.s, kappa, rho, leaf_dofs=32)
    B = torch.randn(5, pr.n_dof, dtype=torch.float64, device="cuda")
    for prec, ir in ((riga.RIGA_FP64, 0), (riga.RIGA_MIXED, 3)):
        pr.factor(650.0, prec)
        X = pr.solve_multi(B, max_ir=ir)
        for i in range(B.shape[0]):
            x = pr.solve(B[i].contiguous(), max_ir=ir)
            assert torch.equal(X[i], x), (prec, i)
    assert pr.solve_multi(B[:0]).shape[0] == 0


@pytest.mark.parametrize("w", [workloads.small(2, 64, 3, 0, 10, 0.3), workloads.small(3, 10, 2, 0, 10, 0.3)],
                         ids=lambda w: w.name)
def test_blocked_fronts_checked_and_unchecked_agree(w, monkeypatch):
    """The blocked (multi-workgroup) fronts run their predicted panel steps
    without host checks; RIGA_FACTOR_CHECKED=1 makes the host check every
    level.  Both give the same inertia and bitwise the same solve."""
    riga = _riga()
    _say("checked vs unchecked", w.name)
    kappa, rho = w.coefficients()
    pr = riga.assemble(w.dim, w.ne, w.p, w.s, kappa, rho)
    b = torch.randn(pr.n_dof, dtype=torch.float64, device="cuda")
    for sigma in (0.0, 900.0):
        for prec in (riga.RIGA_FP64, riga.RIGA_MIXED):
            monkeypatch.delenv("RIGA_FACTOR_CHECKED", raising=False)
            n0, _ = pr.factor(sigma, prec)
            x0 = pr.solve(b)
            monkeypatch.setenv("RIGA_FACTOR_CHECKED", "1")
            n1, _ = pr.factor(sigma, prec)
            x1 = pr.solve(b)
            assert n0 == n1
            assert torch.equal(x0, x1), (sigma, prec)


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "mixed"])
def test_two_slices_match_one(prec, monkeypatch):
    """An open-ended request for many pairs is split, once the inertia at its
    lower end is known, into two slices solved at once (the second starting
    inside its interval); the result equals the single-slice
    solve and the dense oracle (eigenvalues <= 1e-10, residuals <= 1e-9,
    M-orthonormality across the two slices' vectors <= 1e-10)."""
    riga = _riga()
    w = workloads.small(2, 40, 3, 8, 140, 0.3)
    kappa, rho = w.coefficients()
    pr = riga.assemble(w.dim, w.ne, w.p, w.s, kappa, rho, leaf_dofs=32)
    _say("slices", w.name, "N", pr.n_dof, "nev", w.nev)
    Ko, Mo = assembly.assemble(w.dim, w.ne, w.p, w.s, kappa, rho)
    lr, Ur = eigen.dense_eigh(Ko, Mo)
    monkeypatch.setenv("RIGA_SLICES", "1")
    l1, U1, r1, s1 = pr.eigs(w.nev, precision=prec)
    monkeypatch.delenv("RIGA_SLICES")
    l2, U2, r2, s2 = pr.eigs(w.nev, precision=prec)
    _say("one slice", s1, "two slices", s2)
    assert s2["n_shift"] >= 2
    for lam, U, res in ((l1, U1, r1), (l2, U2, r2)):
        _check_pairs(Ko, Mo, lr, Ur, lam, U.cpu().numpy(), res, w.nev)


def test_two_slices_above_a_lower_bound():
    """An open-ended request above lo > 0: the split estimate counts from the
    inertia at lo, and the pairs returned are the oracle's 31st to 170th."""
    riga = _riga()
    w = workloads.small(2, 40, 3, 8, 140, 0.3)
    kappa, rho = w.coefficients()
    Ko, Mo = assembly.assemble(w.dim, w.ne, w.p, w.s, kappa, rho)
    lr, Ur = eigen.dense_eigh(Ko, Mo)
    k = 30
    lo = 0.5 * (lr[k - 1] + lr[k])
    pr = riga.assemble(w.dim, w.ne, w.p, w.s, kappa, rho, leaf_dofs=32)
    _say("lower bound", w.name, "lo", lo)
    lam, U, res, st = pr.eigs(w.nev, lo=lo)
    _say("stats", st)
    assert st["n_shift"] >= 3
    _check_pairs(Ko, Mo, lr[k:], Ur[:, k:], lam, U.cpu().numpy(), res, w.nev)


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "mixed"])
def test_two_slices_with_high_contrast_coefficients(prec):
    """rho = 1e4 on a 4 x 4 block of elements in a corner, 1 elsewhere
    (kappa = 1): the block holds most of the weight in Weyl's leading term
    but, being small, few of the low modes, so the split's estimate (the
    scaled Dirichlet-Laplace spectrum) puts 65 pairs below the split point
    where the oracle has 25.  Each slice counts its own pairs by inertia, so
    the result still equals the oracle's."""
    riga = _riga()
    dim, ne, p, s, nev = 2, 40, 3, 8, 130
    e = np.arange(ne * ne)
    kappa = np.ones(ne * ne)
    rho = np.where((e % ne < 4) & (e // ne < 4), 1e4, 1.0)
    Ko, Mo = assembly.assemble(dim, ne, p, s, kappa, rho)
    lr, Ur = eigen.dense_eigh(Ko, Mo)
    pr = riga.assemble(dim, ne, p, s, kappa, rho, leaf_dofs=32)
    _say("high contrast", prec)
    lam, U, res, st = pr.eigs(nev, precision=prec)
    _say("stats", st)
    _check_pairs(Ko, Mo, lr, Ur, lam, U.cpu().numpy(), res, nev)
