"""GPU parity at the full benchmark sizes, in the configuration bench.py times.

The oracle cannot redo these solves in seconds, so each test checks what it
can compute one piece at a time (see the oracle's pins in test_oracle_*.py):

* 2D 256x256 p=3 rIGA (blocks of 16), log-normal(0, 0.3), 200 lowest, FP64:
  every returned pair's residual and M-orthonormality with the oracle's own
  K and M; the 20 lowest against ARPACK shift-and-invert; the oracle's
  inertia count (Remark on inertia) at shifts it picks from its own lowest
  eigenvalues equals the number of returned pairs below each (no pair
  missed or repeated); every one of the 200 eigenvalues bracketed to 1e-10
  relative by the oracle's inertia counts just below and above it.
* 3D 32^3 p=2 rIGA (blocks of 8) and IGA, kappa = rho = 1, 100 lowest, FP64
  and mixed precision: every eigenvalue against the exact discrete spectrum of
  Kronecker sums (Eq. 2Dmatrix and its 3D analogue), compared as a sorted
  multiset (the 100th cuts a six-fold cluster), residuals with the
  oracle's Kronecker K and M.
* 64 uneven 2D rIGA instances solved together (mixed precision, as the
  batched bench line): three sampled instances checked like the 2D case.
"""
import sys

import numpy as np
import pytest
import scipy.linalg as sla

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


def _bracket_every_eigenvalue(Ko, Mo, lam, tag, rel=1e-10):
    """Every returned eigenvalue pinned to `rel` by the oracle's own inertia
    counts (Remark on inertia): for each group of returned eigenvalues whose
    brackets [lam (1 - rel), lam (1 + rel)) overlap, the oracle's count below
    the group's lower bracket end equals the number of returned pairs below
    the group, and its count below the upper end adds the group's size.
    So the oracle's pencil has exactly those eigenvalues in the brackets, and
    none between them: no pair missed, repeated, or off by more than rel."""
    groups = [[0, 1]]
    for i in range(1, len(lam)):
        if lam[i] * (1 - rel) <= lam[i - 1] * (1 + rel):
            groups[-1][1] = i + 1
        else:
            groups.append([i, i + 1])
    pts = []
    for a, b in groups:
        pts += [lam[a] * (1 - rel), lam[b - 1] * (1 + rel)]
    cnt = eigen.inertia_many(Ko, Mo, pts)
    bad = [(a, b, cnt[2 * g], cnt[2 * g + 1]) for g, (a, b) in enumerate(groups)
           if cnt[2 * g] != a or cnt[2 * g + 1] != b]
    _say(tag, "eigenvalues bracketed by the oracle's inertia at rel", rel, ":", len(lam),
         "in", len(groups), "groups; mismatches", bad[:5])
    assert not bad


def _sampled_checks(Ko, Mo, lam, U, n_sample, eigsh_k, tag):
    """Residuals, M-orthonormality, inertia between sampled neighbours, and
    the lowest eigsh_k eigenvalues against ARPACK."""
    n = len(lam)
    assert np.all(np.diff(lam) >= 0)
    r = eigen.residual(Ko, Mo, lam, U)
    _say(tag, "max residual (oracle K, M)", r.max())
    assert r.max() <= 1e-9
    G = U.T @ (Mo @ U)
    orth = np.abs(G - np.eye(n)).max()
    _say(tag, "max |U^T M U - I|", orth)
    assert orth <= 1e-10
    lo, _ = eigen.sparse_eigs(Ko, Mo, eigsh_k, sigma=0.0)
    rel = np.abs(lam[:eigsh_k] - lo) / lo
    _say(tag, "lowest", eigsh_k, "vs ARPACK max rel", rel.max())
    assert rel.max() <= 1e-10
    # inertia at shifts the oracle picks itself: spread up to 45% of a
    # Weyl-law extrapolation (eigenvalue ~ index in 2D) of its own lowest
    # pairs to the n-th; the oracle's count below each must equal the number
    # of returned eigenvalues below it
    top = 0.45 * lo[-1] * n / eigsh_k
    assert top < lam[-1]
    for sigma in np.linspace(0.5 * (lo[0] + lo[1]), top, n_sample):
        cnt = eigen.inertia(Ko, Mo, sigma)
        below = int(np.sum(lam < sigma))
        _say(tag, "inertia below", sigma, cnt, "returned below", below)
        assert cnt == below


@pytest.mark.timeout(600)
def test_2d_256_p3_riga16_full_size():
    riga = _riga()
    w = workloads.c2(True)
    _say("full size", w.name)
    kappa, rho = w.coefficients()
    kd = torch.tensor(kappa, dtype=torch.float64, device="cuda")
    rd = torch.tensor(rho, dtype=torch.float64, device="cuda")
    pr = riga.assemble(w.dim, w.ne, w.p, w.s, kd, rd)
    lam, U, res, st = pr.eigs(w.nev)
    _say("stats", st)
    assert len(lam) == w.nev and res.max() <= 1e-9
    Ko, Mo = assembly.assemble(w.dim, w.ne, w.p, w.s, kappa, rho)
    _sampled_checks(Ko, Mo, lam, U.cpu().numpy(), 6, 20, w.name)
    _bracket_every_eigenvalue(Ko, Mo, lam, w.name)


def _kron_spectrum(dim, ne, p, s, count):
    K1, M1 = assembly.matrices_1d(ne, p, s)
    mu = sla.eigh(K1[1:-1, 1:-1], M1[1:-1, 1:-1], eigvals_only=True)
    lam = mu
    for _ in range(dim - 1):
        lam = (lam[:, None] + mu[None, :]).ravel()
    return np.sort(lam)[:count]


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
@pytest.mark.parametrize("refined", [True, False], ids=["riga8", "iga"])
def test_3d_32_p2_full_size(refined, precision):
    """IGA in mixed precision stalls with two refinement steps per solve and
    needs the solver's escalation to finish."""
    riga = _riga()
    w = workloads.c3(refined)
    _say("full size", w.name, "precision", precision)
    pr = riga.assemble(w.dim, w.ne, w.p, w.s)
    lam, U, res, st = pr.eigs(w.nev, precision=precision)
    _say("stats", st)
    assert len(lam) == w.nev and res.max() <= 1e-9
    exact = _kron_spectrum(w.dim, w.ne, w.p, w.s, w.nev)
    rel = np.abs(lam - exact) / exact
    _say("max rel error vs Kronecker spectrum", rel.max())
    assert rel.max() <= 1e-10
    Ko, Mo = assembly.kronecker_interior(w.dim, w.ne, w.p, w.s)
    r = eigen.residual(Ko, Mo, lam, U.cpu().numpy())
    _say("max residual (oracle K, M)", r.max())
    assert r.max() <= 1e-9


@pytest.mark.timeout(600)
def test_batched_64_instances_sampled():
    riga = _riga()
    ws = workloads.c4()
    _say("batch of", len(ws))
    probs = []
    for w in ws:
        kappa, rho = w.coefficients()
        probs.append(riga.assemble(w.dim, w.ne, w.p, w.s, kappa, rho))
    res = riga.eigs_batched(probs, ws[0].nev, precision=riga.RIGA_MIXED)
    sizes = [p.n_dof for p in probs]
    order = np.argsort(sizes)
    picks = [order[0], order[len(order) // 2], order[-1]]
    for i in picks:
        w = ws[i]
        lam, U, r, st = res[i]
        _say("instance", w.name, "ne", w.ne, "p", w.p, "s", w.s, "N", sizes[i], "stats", st)
        assert len(lam) == w.nev and r.max() <= 1e-9
        kappa, rho = w.coefficients()
        Ko, Mo = assembly.assemble(w.dim, w.ne, w.p, w.s, kappa, rho)
        _sampled_checks(Ko, Mo, lam, U.cpu().numpy(), 3, w.nev, w.name)
        _bracket_every_eigenvalue(Ko, Mo, lam, w.name)
