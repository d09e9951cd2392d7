"""CPU tests of the library's host-side analysis (no GPU): exported symbols,
DOF maps and sparsity pattern against the oracle's assembly, and the
symbolic factorisation against a brute-force symbolic elimination."""
import ctypes
import os
import re

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import assembly

riga = pytest.importorskip("paper_2009_08167_amd.riga")
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib_or_skip():
    if not os.path.exists(riga.LIB_PATH):
        pytest.skip("libriga.so not built")
    return riga.lib()


def test_exports_every_header_symbol():
    L = _lib_or_skip()
    text = open(os.path.join(ROOT, "include", "riga.h")).read()
    names = set(re.findall(r"^(?:riga_status|void|const char\s*\*)\s*(riga_\w+)\s*\(", text,
                           re.M))
    assert {"riga_assemble", "riga_eigs", "riga_eig_grad"} <= names
    for n in sorted(names):
        assert hasattr(L, n), n
    assert set(riga.EXPORTED) == names


def test_invalid_descriptors_rejected():
    _lib_or_skip()
    for args in [(4, 8, 2, 0), (2, 8, 0, 0), (2, 8, 2, -1), (2, 0, 2, 0), (2, 8, 9, 0)]:
        with pytest.raises(riga.RigaError) as e:
            riga.analyze(*args)
        assert e.value.code == riga.RIGA_EINVAL


CASES = [(2, 16, 2, 0), (2, 16, 3, 4), (2, 20, 2, 6), (2, 13, 4, 5), (3, 6, 2, 0), (3, 8, 2, 4),
         (2, 24, 1, 0), (2, 9, 3, 1)]


@pytest.mark.parametrize("dim,ne,p,s", CASES)
def test_pattern_matches_oracle(dim, ne, p, s):
    _lib_or_skip()
    pr = riga.analyze(dim, ne, p, s)
    K, M = assembly.assemble(dim, ne, p, s)
    assert pr.n_dof == K.shape[0]
    rp, ci = pr.pattern()
    P = sp.csr_matrix((np.ones(len(ci)), ci, rp), shape=K.shape)
    # structural pattern: the oracle's non-zeros (mass entries are > 0 on
    # the whole support overlap) equal the library's stored pattern
    Mo = (abs(M) > 0).astype(float)
    assert (P != Mo).nnz == 0
    for r in range(0, pr.n_dof, max(1, pr.n_dof // 50)):
        row = ci[rp[r]:rp[r + 1]]
        assert (np.diff(row) > 0).all()


def _fronts(t):
    offs = np.concatenate([[0], np.cumsum(t["f"])])
    return [t["rows"][offs[i]:offs[i + 1]] for i in range(len(t["f"]))]


@pytest.mark.parametrize("dim,ne,p,s", CASES)
def test_tree_is_a_valid_elimination_tree(dim, ne, p, s):
    _lib_or_skip()
    pr = riga.analyze(dim, ne, p, s, leaf_dofs=16)
    t = pr.tree()
    perm = t["perm"]
    assert sorted(perm) == list(range(pr.n_dof))
    fronts = _fronts(t)
    nf = len(fronts)
    # post-order, heights, each DOF fully summed in exactly one front
    owner = -np.ones(pr.n_dof, np.int64)
    start = 0
    for F in range(nf):
        par = t["parent"][F]
        assert par == -1 or par > F
        k = t["k"][F]
        fs = fronts[F][:k]
        assert (perm[fs] == np.arange(start, start + k)).all()
        start += k
        assert (owner[fs] == -1).all()
        owner[fs] = F
        # contribution-block rows are eliminated later, ascending
        cb = perm[fronts[F][k:]]
        assert (cb >= start).all() and (np.diff(cb) > 0).all()
        if par >= 0:
            assert set(fronts[F][k:]) <= set(fronts[par])
            assert t["height"][par] >= t["height"][F] + 1
    assert (owner >= 0).all()
    # every matrix entry lies in the front of its earlier-eliminated index
    rp, ci = pr.pattern()
    fsets = [set(f) for f in fronts]
    for r in range(pr.n_dof):
        for c in ci[rp[r]:rp[r + 1]]:
            a, b = (r, c) if perm[r] <= perm[c] else (c, r)
            assert b in fsets[owner[a]]


@pytest.mark.parametrize("dim,ne,p,s,split", [(2, 12, 2, 0, 0), (2, 16, 3, 4, 0), (3, 6, 2, 3, 0),
                                               (2, 10, 4, 5, 0), (2, 16, 3, 4, 6), (3, 6, 2, 3, 8)])
def test_fronts_contain_exact_fill(dim, ne, p, s, split, monkeypatch):
    """Brute force: the symbolic Cholesky of P A P^T (SuperLU, natural order
    on the permuted matrix, no pivoting) never fills outside the fronts, and
    the supernodal count nnz(L) is at least the exact fill; also with
    separators split into chains (split > 0)."""
    _lib_or_skip()
    monkeypatch.setenv("RIGA_SPLIT_FS", str(split))
    pr = riga.analyze(dim, ne, p, s, leaf_dofs=24)
    if split:
        assert pr.tree()["k"].max() <= split
    t = pr.tree()
    perm = t["perm"]
    K, M = assembly.assemble(dim, ne, p, s)
    A = (K + M).tocsr()                    # SPD, same pattern
    n = A.shape[0]
    Pm = sp.csr_matrix((np.ones(n), (perm, np.arange(n))), shape=(n, n))
    Ap = (Pm @ A @ Pm.T).tocsc()
    lu = spla.splu(Ap, permc_spec="NATURAL", diag_pivot_thresh=0.0,
                   options=dict(SymmetricMode=True))
    assert (lu.perm_r == np.arange(n)).all()
    L = sp.tril(lu.L, -1).tocoo()
    fronts = _fronts(t)
    iperm = np.argsort(perm)
    owner = np.zeros(n, np.int64)
    for F, fr in enumerate(fronts):
        owner[perm[fr[:t["k"][F]]]] = F
    fsets = [set(perm[f]) for f in fronts]
    for i, j in zip(L.row, L.col):
        assert i in fsets[owner[j]]
    nnz_exact = L.nnz + n
    assert pr.info["nnz_l"] >= nnz_exact
    # the library's own exact count (row subtrees of its elimination tree)
    assert pr.info["nnz_l_exact"] == nnz_exact
    cc = np.bincount(L.col, minlength=n).astype(float)
    assert pr.info["flops_fact_exact"] == pytest.approx(float(np.sum(cc * (cc + 1))), rel=1e-15)
    assert pr.info["flops_fact_exact"] <= pr.info["flops_fact"] * (1 + 1e-12)
    del iperm


def test_riga_separators_are_single_layers():
    """With rIGA the top separators cut at C^0 knots: one layer of DOFs
    (Sec. 3.2), so the root fully-summed block is one line of the grid."""
    _lib_or_skip()
    pr = riga.analyze(2, 64, 3, 16)
    t = pr.tree()
    root = len(t["k"]) - 1
    assert t["parent"][root] == -1
    assert t["k"][root] == pr.info["n1"][1]
    pr_iga = riga.analyze(2, 64, 3, 0)
    t2 = pr_iga.tree()
    assert t2["k"][-1] == 3 * pr_iga.info["n1"][1]   # p layers at a simple knot
    assert pr.info["flops_fact"] < pr_iga.info["flops_fact"]


def test_analysis_is_deterministic():
    _lib_or_skip()
    a = riga.analyze(2, 40, 3, 8).tree()
    b = riga.analyze(2, 40, 3, 8).tree()
    for k in a:
        assert np.array_equal(a[k], b[k])


def test_exact_eigenvalues_host_enumeration_matches_oracle():
    """riga_exact_eigenvalues (host code of the library) against the
    oracle's enumeration of Eq. exact, 2D and 3D, with multiplicities."""
    from oracle import accuracy
    for dim, count in ((2, 1), (2, 37), (2, 5000), (3, 1), (3, 400)):
        got = riga.exact_eigenvalues(dim, count)
        ref = accuracy.exact_eigenvalues(dim, count)
        assert np.array_equal(got, ref), (dim, count)
    with pytest.raises(riga.RigaError):
        riga.exact_eigenvalues(1, 5)


@pytest.mark.parametrize("dim,ne,p,s,split", [(2, 128, 3, 0, 288), (3, 12, 2, 0, 64), (2, 40, 3, 8, 16)])
def test_supernode_splitting_keeps_order_fill_and_flops(dim, ne, p, s, split, monkeypatch):
    """Separators larger than the split size become chains: the elimination
    order is that of the unsplit tree; nnz(L) and the factorisation flops are
    at most its (a supernode counts its fully-summed block as dense, the
    chain pieces only the structure elimination creates); every
    fully-summed block is at most the split size; a split front's parent is
    the next piece of the same separator (consecutive pivots)."""
    _lib_or_skip()
    monkeypatch.setenv("RIGA_SPLIT_FS", "0")
    whole = riga.analyze(dim, ne, p, s)
    tw = whole.tree()
    monkeypatch.setenv("RIGA_SPLIT_FS", str(split))
    part = riga.analyze(dim, ne, p, s)
    tp = part.tree()
    assert tw["k"].max() > split  # the case exercises the split
    assert tp["k"].max() <= split
    assert np.array_equal(tw["perm"], tp["perm"])
    assert part.info["nnz_l"] <= whole.info["nnz_l"]
    assert part.info["flops_fact"] <= whole.info["flops_fact"] * (1 + 1e-12)
    assert len(tp["k"]) > len(tw["k"])
    # pieces of one separator: consecutive pivot ranges linked child -> parent
    starts = np.concatenate(([0], np.cumsum(tp["k"])[:-1]))
    for F in range(len(tp["k"])):
        P = tp["parent"][F]
        if P == F + 1 and tp["k"][F] == split:
            assert starts[P] == starts[F] + split


@pytest.mark.parametrize("dim,ne,p,s,A", [(2, 10, 2, 5, (0.9, -1.7)), (3, 4, 2, 2, (0.4, 1.1, -0.6)),
                                          (2, 12, 3, 0, (2.5, 0.7))])
def test_complex_pencil_analysis(dim, ne, p, s, A):
    """The complex Hermitian pencil in real-equivalent form: the pattern is
    the scalar one with every coupling a 2 x 2 block (real and imaginary
    parts of a DOF adjacent); the same tree with doubled fronts is a valid
    elimination tree of it, its fronts contain the exact fill of the
    real-equivalent matrix (SuperLU, natural order on the permuted matrix),
    and the library's exact-fill count equals SuperLU's."""
    _lib_or_skip()
    from oracle import hermitian
    pr = riga.analyze(dim, ne, p, s, potential=A)
    sc = riga.analyze(dim, ne, p, s)
    assert pr.hermitian and pr.n_dof == 2 * sc.n_dof
    rp, ci = pr.pattern()
    rps, cis = sc.pattern()
    n = pr.n_dof
    P = sp.csr_matrix((np.ones(len(ci)), ci, rp), shape=(n, n))
    S = sp.csr_matrix((np.ones(len(cis)), cis, rps), shape=(n // 2, n // 2))
    assert (P != sp.kron(S, np.ones((2, 2)), format="csr")).nnz == 0
    t = pr.tree()
    perm = t["perm"]
    assert sorted(perm) == list(range(n))
    assert (perm[0::2] % 2 == 0).all() and (perm[1::2] == perm[0::2] + 1).all()
    fronts = _fronts(t)
    owner = -np.ones(n, np.int64)
    start = 0
    for F in range(len(fronts)):
        k = t["k"][F]
        assert k % 2 == 0 and t["f"][F] % 2 == 0
        fs = fronts[F][:k]
        assert (perm[fs] == np.arange(start, start + k)).all()
        start += k
        owner[fs] = F
    # the stored pattern is the oracle's real-equivalent matrix's, plus the
    # diagonal blocks' off-diagonal entries (Im K is antisymmetric: zero there)
    Kc, Mc = hermitian.assemble_magnetic(dim, ne, p, s, A)
    K2, M2 = hermitian.real_equivalent(Kc + Mc, Mc)
    N = Kc.shape[0]
    il = np.empty(2 * N, dtype=np.int64)
    il[0::2] = np.arange(N)
    il[1::2] = N + np.arange(N)
    Ko = (abs(K2[il][:, il]) > 0).astype(float)
    assert (Ko.multiply(P) != Ko).nnz == 0
    # exact fill of the stored pattern: SuperLU without pivoting on a
    # diagonally dominant matrix with that pattern (no cancellation)
    Ai = (P + (P.sum(axis=1).max() + 1.0) * sp.identity(n)).tocsr()
    Pm = sp.csr_matrix((np.ones(n), (perm, np.arange(n))), shape=(n, n))
    Ap = (Pm @ Ai @ Pm.T).tocsc()
    lu = spla.splu(Ap, permc_spec="NATURAL", diag_pivot_thresh=0.0, options=dict(SymmetricMode=True))
    assert (lu.perm_r == np.arange(n)).all()
    L = sp.tril(lu.L, -1).tocoo()
    iperm = np.argsort(perm)
    fsets = [set(perm[f]) for f in fronts]
    for i, j in zip(L.row, L.col):
        assert i in fsets[owner[iperm[j]]]
    assert pr.info["nnz_l_exact"] == L.nnz + n
