"""Complex Hermitian pencils: a synthetic source with a known spectrum.

Test infrastructure only (see the package docstring).

The paper's eigenproblem (Eq. GHEP) allows K and M to be Hermitian, with
every transpose in its solver read as the conjugate transpose (Sec. on
solving generalized Hermitian eigenproblems), but its experiments are all
real.  The complex source used here is the magnetic Laplacian with a
constant vector potential A on the unit square or cube,

    -(grad - i A) . (grad - i A) u = lambda u,   u = 0 on the boundary,

whose Galerkin form on the B-spline space of ``assembly`` gives

    K_ab = int (grad B_b - i A B_b) . conj(grad B_a - i A B_a)
         = int grad B_a . grad B_b + |A|^2 B_a B_b
           + i int (B_a A . grad B_b - B_b A . grad B_a),
    M_ab = int B_a B_b,

K Hermitian (its imaginary part antisymmetric), M real.  For constant A the
gauge map u = exp(i A . x) w turns the problem into the Dirichlet Laplacian,
so the exact eigenvalues are pi^2 (i^2 + j^2 [+ k^2]) for every A; the
discrete ones are not gauge invariant (exp(i A . x) w_h leaves the space) and
approach them from above, at the order of the real problem.

The real-equivalent pencil of size 2N, [[Kr, -Ki], [Ki, Kr]] and
diag(M, M), is real symmetric, has every eigenvalue of the complex pencil
twice, and commutes with J = [[0, -I], [I, 0]]: the form in which a real
solver handles the complex pencil.
"""
import itertools

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .assembly import dirichlet, element_unit_matrices, make_spaces


def element_magnetic_matrix(spaces, e_multi, A):
    """Element matrix of the magnetic form (complex, Hermitian) and the
    full-space indices of the active functions on element ``e_multi``,
    integrated with the tensor Gauss rule at every active pair."""
    dim = len(spaces)
    act = [spaces[d].active[e_multi[d]] for d in range(dim)]
    vals, wq = None, None
    grads = None
    for d in range(dim):
        Bd = spaces[d].B[act[d], e_multi[d], :]
        dBd = spaces[d].dB[act[d], e_multi[d], :]
        wd = spaces[d].wts[e_multi[d]]
        if vals is None:
            vals, wq = Bd, wd
            grads = [dBd]
        else:
            nv = np.einsum('ap,bq->bapq', vals, Bd).reshape(-1, vals.shape[1] * Bd.shape[1])
            grads = [np.einsum('ap,bq->bapq', g, Bd).reshape(nv.shape) for g in grads]
            grads.append(np.einsum('ap,bq->bapq', vals, dBd).reshape(nv.shape))
            vals = nv
            wq = np.einsum('p,q->qp', wq, wd).ravel()
    # D B_b = grad B_b - i A B_b, one array per direction
    D = [grads[d] - 1j * A[d] * vals for d in range(dim)]
    ke = sum(np.einsum('ap,bp,p->ab', np.conj(D[d]), D[d], wq) for d in range(dim))
    _, _, gidx = element_unit_matrices(spaces, e_multi)
    return ke, gidx


def assemble_magnetic(dim, ne, p, s, A, q=None):
    """Interior K (complex Hermitian, CSR) and M (real, CSR) of the magnetic
    Laplacian with constant potential ``A`` (length ``dim``), Dirichlet
    functions deleted as in ``assembly``."""
    A = np.asarray(A, dtype=np.float64)
    assert A.shape == (dim,)
    spaces = make_spaces(dim, ne, p, s, q)
    nes = [s1.ne for s1 in spaces]
    nt = int(np.prod([s1.n for s1 in spaces]))
    rows, cols, kv, mv = [], [], [], []
    for eidx in itertools.product(*[range(n) for n in reversed(nes)]):
        eidx = eidx[::-1]
        ke, gidx = element_magnetic_matrix(spaces, eidx, A)
        _, m0, _ = element_unit_matrices(spaces, eidx)
        rr, cc = np.meshgrid(gidx, gidx, indexing='ij')
        rows.append(rr.ravel())
        cols.append(cc.ravel())
        kv.append(ke.ravel())
        mv.append(m0.ravel())
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    K = sp.coo_matrix((np.concatenate(kv), (r, c)), shape=(nt, nt)).tocsr()
    M = sp.coo_matrix((np.concatenate(mv), (r, c)), shape=(nt, nt)).tocsr()
    K.sum_duplicates()
    M.sum_duplicates()
    return dirichlet(K, M, spaces)


def real_equivalent(K, M):
    """The real symmetric pencil of size 2N equivalent to (K, M):
    [[Kr, -Ki], [Ki, Kr]] and diag(M, M), unknowns (Re u, Im u)."""
    Kr, Ki = sp.csr_matrix(K.real), sp.csr_matrix(K.imag)
    Mr = sp.csr_matrix(M.real)
    K2 = sp.bmat([[Kr, -Ki], [Ki, Kr]]).tocsr()
    M2 = sp.block_diag([Mr, Mr]).tocsr()
    return K2, M2


def dense_eigh_hermitian(K, M):
    """All eigenpairs of the Hermitian pencil (dense LAPACK: Cholesky of M,
    then the Hermitian standard problem); eigenvectors M-orthonormal."""
    Kd = K.toarray() if sp.issparse(K) else np.asarray(K)
    Md = M.toarray() if sp.issparse(M) else np.asarray(M)
    lam, U = sla.eigh(Kd, Md.astype(Kd.dtype))
    return lam, U
