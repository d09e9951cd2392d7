"""GPU parity of the top block (explicit inverse of the top tree levels used
by the forward/backward sweeps) at every cut height, against the oracle's
matrices and inertia, and against the level-by-level sweeps.

The cut is read from RIGA_TOP_CUT when a problem is assembled: "0" sweeps
every level, c >= 1 takes the fronts at heights >= c into the top block.
Bars: inertia exact; FP64 solves with backward error <= 1e-12 and within
1e-10 (relative, max norm) of the level-by-level solve; mixed-precision
solves refined to a relative residual <= 1e-12; eigenpairs as in
test_gpu_parity.
"""
import sys

import numpy as np
import pytest
import scipy.sparse as sp

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
            xr = ref[sigma][1]
            assert np.abs(x - xr).max() <= 1e-10 * np.abs(xr).max(), (cut, sigma)
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
