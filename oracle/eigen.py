"""Generalized symmetric eigenproblem K u = lambda M u (Eq. GHEP).

Test infrastructure only (see the package docstring).

The method under test (shift-and-invert Lanczos with exact LDL^T solves,
Secs. 4.1--4.2) returns eigenpairs of the discrete pencil; its plain
definition is "the eigenpairs of (K, M)", which is what this module computes
directly:

* ``dense_eigh``  -- the Cholesky reduction of Sec. 4.1 (M = L L^T, eigen-
  decomposition of L^{-1} K L^{-T}, u = L^{-T} w), for small N.
* ``sparse_eigs`` -- ARPACK in shift-and-invert mode (Eq. ST_GHEP) with a
  SuperLU factorisation of K - sigma M, for larger N.
* ``inertia``     -- Sylvester's law of inertia (Remark on inertia): the number
  of eigenvalues below sigma equals the number of negative pivots of an
  LDL^T factorisation of K - sigma M (``inertia_many``: the same at many
  shifts, in worker processes).
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def normalize(M, U):
    """Scale each column to u^T M u = 1 and fix its sign so that the entry of
    largest magnitude is positive (ties: the lowest index)."""
    U = np.array(U, dtype=np.float64, copy=True)
    for i in range(U.shape[1]):
        u = U[:, i]
        u /= np.sqrt(u @ (M @ u))
        j = int(np.argmax(np.abs(u)))
        if u[j] < 0:
            u *= -1.0
        U[:, i] = u
    return U


def dense_eigh(K, M):
    """All eigenpairs by the Cholesky reduction of Sec. 4.1.

    Returns (lam ascending, U with M-normalised columns)."""
    Kd = K.toarray() if sp.issparse(K) else np.asarray(K)
    Md = M.toarray() if sp.issparse(M) else np.asarray(M)
    L = np.linalg.cholesky(Md)
    X = sla.solve_triangular(L, Kd, lower=True)          # L^{-1} K
    C = sla.solve_triangular(L, X.T, lower=True)         # L^{-1} K L^{-T}
    C = 0.5 * (C + C.T)
    lam, W = np.linalg.eigh(C)
    U = sla.solve_triangular(L.T, W, lower=False)        # u = L^{-T} w
    return lam, normalize(Md, U)


def sparse_eigs(K, M, k, sigma=0.0):
    """The ``k`` eigenpairs nearest ``sigma`` by ARPACK shift-and-invert
    (Eq. ST_GHEP: the largest |theta| = 1/|lambda - sigma|).  Sorted by
    lambda, M-normalised."""
    lam, U = spla.eigsh(K.tocsc(), k=k, M=M.tocsc(), sigma=sigma, which='LM',
                        tol=0.0)
    order = np.argsort(lam)
    lam, U = lam[order], U[:, order]
    return lam, normalize(M, U)


def inertia(K, M, sigma):
    """Number of eigenvalues of (K, M) strictly below ``sigma``.

    Remark on inertia: factor A = K - sigma M = P^T L D L^T P symmetrically
    (SuperLU in symmetric mode with a fill-reducing symmetric ordering and no
    row pivoting, so that U = D L^T) and count the negative entries of D.
    """
    A = (K - sigma * M).tocsc()
    lu = spla.splu(A, permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.0,
                   options=dict(SymmetricMode=True))
    if not np.array_equal(lu.perm_r, lu.perm_c):
        raise RuntimeError("SuperLU pivoted off the diagonal; inertia undefined")
    return int(np.count_nonzero(lu.U.diagonal() < 0))


_pool_KM = None


def _pool_init(K, M):
    global _pool_KM
    _pool_KM = (K, M)


def _pool_count(sigma):
    return inertia(_pool_KM[0], _pool_KM[1], sigma)


def inertia_many(K, M, sigmas, workers=8):
    """``inertia(K, M, sigma)`` for every sigma, in a pool of fresh worker
    processes (each gets its own copy of K and M; the counts are independent
    factorisations, so only the wall time changes)."""
    import multiprocessing as mp
    sigmas = [float(x) for x in sigmas]
    if workers <= 1 or len(sigmas) < 2:
        return [inertia(K, M, x) for x in sigmas]
    ctx = mp.get_context("spawn")
    with ctx.Pool(min(workers, len(sigmas)), initializer=_pool_init, initargs=(K.tocsr(), M.tocsr())) as pool:
        return pool.map(_pool_count, sigmas, chunksize=1)


def residual(K, M, lam, U):
    """Relative residuals ||K u - lam M u||_2 / (||K||_1 ||u||_2), one per pair."""
    U = np.atleast_2d(U.T).T
    lam = np.atleast_1d(lam)
    nK = sp.linalg.norm(K, 1) if sp.issparse(K) else np.linalg.norm(K, 1)
    R = K @ U - (M @ U) * lam[None, :]
    return np.linalg.norm(R, axis=0) / (nK * np.linalg.norm(U, axis=0))


def lowest(K, M, nev, dense_limit=4000, margin=8):
    """The ``nev`` lowest eigenpairs: dense Cholesky reduction for small N,
    otherwise shift-and-invert at sigma = 0 (K is SPD after Dirichlet
    elimination) with a margin of extra pairs, checked for completeness by
    the inertia count just above the last returned eigenvalue."""
    n = K.shape[0]
    if n <= dense_limit:
        lam, U = dense_eigh(K, M)
        return lam[:nev], U[:, :nev]
    k = min(nev + margin, n - 2)
    lam, U = sparse_eigs(K, M, k, sigma=0.0)
    top = lam[nev - 1]
    gap_hi = lam[nev] if nev < k else top * (1 + 1e-6)
    cut = 0.5 * (top + gap_hi) if gap_hi > top * (1 + 1e-12) else top * (1 + 1e-9)
    cnt = inertia(K, M, cut)
    if cnt != int(np.count_nonzero(lam < cut)):
        raise RuntimeError("shift-and-invert missed eigenvalues below %g" % cut)
    return lam[:nev], U[:, :nev]
