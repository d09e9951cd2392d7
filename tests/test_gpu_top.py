"""GPU parity of the top block (explicit inverse of the top tree levels used
by the forward/backward sweeps) at every cut height, against the oracle's
matrices and inertia, and against the level-by-level sweeps.

The cut is read from RIGA_TOP_CUT when a problem is assembled: "0" sweeps
every level, c >= 1 takes the fronts at heights >= c into the top block.
Bars: inertia exact; FP64 solves with backward error <= 1e-12 and within
1e-10 (relative, max norm) of the level-by-level solve, or within the
perturbation bound of the two solves' backward errors where the shift makes
that larger; mixed-precision
solves refined to a relative residual <= 1e-12; eigenpairs as in
test_gpu_parity.
"""
import sys

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import workloads
from oracle import assembly, eigen

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


CASES = [workloads.small(2, 40, 3, 8, 10, 0.3), workloads.small(3, 10, 2, 0, 10, 0.3),
         workloads.small(2, 64, 3, 16, 10, 0.4), workloads.small(2, 33, 2, 0, 10, 0.3)]


def _berr(A, b, x):
    return np.linalg.norm(b - A @ x) / (sp.linalg.norm(A, 1) * np.linalg.norm(x) + np.linalg.norm(b))


def _agree(A, b, x, xr):
    """Two backward-stable solves agree to the condition number times their
    backward errors (first-order perturbation bound, a factor 4 for the mixed
    norms), and to 1e-10 when that is smaller: at shifts near an eigenvalue
    (kappa_1 = 5e4 at sigma = 4000 on 2D 64^2 p = 3) rounding-order changes
    alone move the solution by more than 1e-10."""
    lu = spla.splu(A.tocsc())
    op = spla.LinearOperator(A.shape, matvec=lu.solve, rmatvec=lambda v: lu.solve(v, trans="T"))
    kappa = spla.onenormest(op) * sp.linalg.norm(A, 1)
    bar = max(1e-10, 4.0 * kappa * (_berr(A, b, x) + _berr(A, b, xr)))
    return np.abs(x - xr).max() / np.abs(xr).max(), bar


def _problem(riga, w, cut, monkeypatch):
    monkeypatch.setenv("RIGA_TOP_CUT", str(cut))
    kappa, rho = w.coefficients()
    return riga.assemble(w.dim, w.ne, w.p, w.s, kappa, rho, leaf_dofs=32)


@pytest.mark.parametrize("w", CASES, ids=lambda w: w.name)
def test_top_block_every_cut_solves(w, monkeypatch):
    riga = _riga()
    kappa, rho = w.coefficients()
    Ko, Mo = assembly.assemble(w.dim, w.ne, w.p, w.s, kappa, rho)
    base = _problem(riga, w, 0, monkeypatch)
    height = base.info["tree_height"]
    _say("top block", w.name, "N", base.n_dof, "height", height)
    rng = np.random.default_rng(17)
    b = rng.standard_normal(base.n_dof)
    bd = torch.tensor(b, dtype=torch.float64, device="cuda")
    sigmas = (0.0, 700.0, 4000.0)
    ref = {}
    for sigma in sigmas:
        neg, _ = base.factor(sigma)
        assert neg == eigen.inertia(Ko, Mo, sigma)
        ref[sigma] = (neg, base.solve(bd).cpu().numpy())
    for cut in range(1, height):
        pr = _problem(riga, w, cut, monkeypatch)
        for sigma in sigmas:
            _say("  cut", cut, "sigma", sigma)
            neg, _ = pr.factor(sigma)
            assert neg == ref[sigma][0]
            x = pr.solve(bd).cpu().numpy()
            A = (Ko - sigma * Mo).tocsr()
            berr = np.linalg.norm(b - A @ x) / (sp.linalg.norm(A, 1) * np.linalg.norm(x)
                                                + np.linalg.norm(b))
            assert berr <= 1e-12, (cut, sigma, berr)
            d, bar = _agree(A, b, x, ref[sigma][1])
            assert d <= bar, (cut, sigma, d, bar)
            neg32, _ = pr.factor(sigma, riga.RIGA_MIXED)
            assert neg32 == ref[sigma][0]
            x32 = pr.solve(bd, max_ir=30).cpu().numpy()
            r = np.linalg.norm(b - A @ x32) / np.linalg.norm(b)
            assert r <= 1e-12, (cut, sigma, r)
        del pr


@pytest.mark.parametrize("cut", [1, 2, 3])
def test_top_block_eigs(cut, monkeypatch):
    riga = _riga()
    w = workloads.small(2, 24, 3, 8, 30, 0.5)
    pr = _problem(riga, w, cut, monkeypatch)
    _say("top block eigs", w.name, "cut", cut, "height", pr.info["tree_height"])
    kappa, rho = w.coefficients()
    Ko, Mo = assembly.assemble(w.dim, w.ne, w.p, w.s, kappa, rho)
    lr, Ur = eigen.dense_eigh(Ko, Mo)
    for prec in (riga.RIGA_FP64, riga.RIGA_MIXED):
        lam, U, res, st = pr.eigs(w.nev, precision=prec, per_shift=8)
        U = U.cpu().numpy()
        rel = np.abs(lam - lr[:w.nev]) / lr[:w.nev]
        assert rel.max() <= 1e-10, rel.max()
        assert eigen.residual(Ko, Mo, lam, U).max() <= 1e-9
        assert np.abs(U.T @ (Mo @ U) - np.eye(w.nev)).max() <= 1e-10


def _problem_fused(riga, w, cut, nh, monkeypatch):
    monkeypatch.setenv("RIGA_TOP_CUT", str(cut))
    monkeypatch.setenv("RIGA_SUBTREE_HEIGHTS", str(nh))
    kappa, rho = w.coefficients()
    return riga.assemble(w.dim, w.ne, w.p, w.s, kappa, rho, leaf_dofs=32)


@pytest.mark.parametrize("w", CASES, ids=lambda w: w.name)
def test_fused_bottom_heights_solves(w, monkeypatch):
    """The bottom heights swept in one launch per direction (one workgroup
    per subtree) give the level-by-level solve: every fused height count,
    with and without a top block; FP64 to 1e-10 of the unfused solve and a
    backward error <= 1e-12, mixed refined to 1e-12; the default choice is
    reported by the problem info."""
    riga = _riga()
    kappa, rho = w.coefficients()
    Ko, Mo = assembly.assemble(w.dim, w.ne, w.p, w.s, kappa, rho)
    base = _problem_fused(riga, w, 0, 0, monkeypatch)
    assert base.info["fused_heights"] == 0 and base.info["top_cut"] == -1
    height = base.info["tree_height"]
    rng = np.random.default_rng(23)
    b = rng.standard_normal(base.n_dof)
    bd = torch.tensor(b, dtype=torch.float64, device="cuda")
    sigmas = (0.0, 900.0)
    ref = {}
    for sigma in sigmas:
        neg, _ = base.factor(sigma)
        ref[sigma] = (neg, base.solve(bd).cpu().numpy())
    del base
    configs = [(0, nh) for nh in range(2, height + 1)] + [(c, nh) for c in (2, height - 2) if c >= 2
                                                         for nh in range(2, c + 1)]
    for cut, nh in configs:
        pr = _problem_fused(riga, w, cut, nh, monkeypatch)
        _say("fused", w.name, "cut", cut, "heights", nh, "->", pr.info["fused_heights"],
             "subtrees", pr.info["fused_subtrees"], "top", pr.info["top_cut"])
        # a forced count is taken unless a subtree exceeds the 64 KB LDS
        # budget (the whole tree of a larger problem)
        assert pr.info["fused_heights"] in (nh, 0)
        assert pr.info["fused_heights"] == nh or nh >= height - 1
        for sigma in sigmas:
            neg, _ = pr.factor(sigma)
            assert neg == ref[sigma][0]
            x = pr.solve(bd).cpu().numpy()
            A = (Ko - sigma * Mo).tocsr()
            berr = np.linalg.norm(b - A @ x) / (sp.linalg.norm(A, 1) * np.linalg.norm(x)
                                                + np.linalg.norm(b))
            assert berr <= 1e-12, (cut, nh, sigma, berr)
            d, bar = _agree(A, b, x, ref[sigma][1])
            assert d <= bar, (cut, nh, sigma, d, bar)
            pr.factor(sigma, riga.RIGA_MIXED)
            x32 = pr.solve(bd, max_ir=30).cpu().numpy()
            r = np.linalg.norm(b - A @ x32) / np.linalg.norm(b)
            assert r <= 1e-12, (cut, nh, sigma, r)
        del pr
    monkeypatch.delenv("RIGA_TOP_CUT")
    monkeypatch.setenv("RIGA_SUBTREE_HEIGHTS", "auto")
    pr = riga.assemble(w.dim, w.ne, w.p, w.s, kappa, rho, leaf_dofs=32)
    _say("automatic", w.name, "top", pr.info["top_cut"], "fused", pr.info["fused_heights"],
         "subtrees", pr.info["fused_subtrees"])
    for sigma in sigmas:
        pr.factor(sigma)
        x = pr.solve(bd).cpu().numpy()
        A = (Ko - sigma * Mo).tocsr()
        assert _berr(A, b, x) <= 1e-12
        d, bar = _agree(A, b, x, ref[sigma][1])
        assert d <= bar, (sigma, d, bar)


def test_fused_heights_eigs_and_default(monkeypatch):
    """Eigenpairs through the fused sweeps; fusion is off by default, and
    the automatic rule on the 2D 256^2 p = 3 rIGA workload's tree takes
    three heights, 256 subtrees, below a top block from height 3."""
    riga = _riga()
    w = workloads.small(2, 24, 3, 8, 30, 0.5)
    kappa, rho = w.coefficients()
    Ko, Mo = assembly.assemble(w.dim, w.ne, w.p, w.s, kappa, rho)
    lr, _ = eigen.dense_eigh(Ko, Mo)
    monkeypatch.setenv("RIGA_TOP_CUT", "0")
    for nh in (2, 4):
        monkeypatch.setenv("RIGA_SUBTREE_HEIGHTS", str(nh))
        pr = riga.assemble(w.dim, w.ne, w.p, w.s, kappa, rho, leaf_dofs=32)
        assert pr.info["fused_heights"] == nh
        for prec in (riga.RIGA_FP64, riga.RIGA_MIXED):
            lam, U, res, st = pr.eigs(w.nev, precision=prec, per_shift=8)
            U = U.cpu().numpy()
            assert np.abs(lam - lr[:w.nev]).max() <= 1e-10 * lr[w.nev - 1]
            assert eigen.residual(Ko, Mo, lam, U).max() <= 1e-9
            assert np.abs(U.T @ (Mo @ U) - np.eye(w.nev)).max() <= 1e-10
        del pr
    monkeypatch.delenv("RIGA_TOP_CUT")
    monkeypatch.delenv("RIGA_SUBTREE_HEIGHTS")
    big = workloads.c2()
    pr = riga.assemble(big.dim, big.ne, big.p, big.s)
    assert (pr.info["top_cut"], pr.info["fused_heights"], pr.info["fused_subtrees"]) == (3, 0, 0)
    del pr
    monkeypatch.setenv("RIGA_SUBTREE_HEIGHTS", "auto")
    pr = riga.assemble(big.dim, big.ne, big.p, big.s)
    _say("main workload", pr.info["top_cut"], pr.info["fused_heights"], pr.info["fused_subtrees"])
    assert (pr.info["top_cut"], pr.info["fused_heights"], pr.info["fused_subtrees"]) == (3, 3, 256)
