"""Galerkin stiffness and mass matrices on the unit square / cube.

Test infrastructure only (see the package docstring).

The model problem is the Dirichlet Laplace eigenproblem (Sec. 2.1, Eq.
helmholtz); its Galerkin form (Eqs. weakform--weakform3) gives K_ab = a(B_a,
B_b) and M_ab = (B_a, B_b).  We assemble the generalisation
``-div(kappa grad u) = lambda rho u`` with ``kappa``, ``rho`` constant on each
element (``kappa = rho = 1`` is the paper's problem).  Each element integral
is evaluated by a full tensor Gauss rule with q points per direction at every
basis function that is non-zero on the element -- the weak form written out,
with no use of the Kronecker structure, so that Eq. 2Dmatrix can serve as an
independent check.

Degrees of freedom are the tensor-product functions (Eq. u, Remark on
Tensor(u)) ordered lexicographically with x fastest.  Dirichlet conditions
(H^1_0, Eq. helmholtz) are imposed by deleting the first and last function in
each direction (the paper does not say how it imposes them; with an open knot
vector those are the only functions that do not vanish on the boundary).
"""
import itertools

import numpy as np
import scipy.sparse as sp

from . import bspline


class Space1D:
    """One direction of the tensor-product space: knots, elements, tables."""

    def __init__(self, ne, p, s, q=None):
        self.ne, self.p, self.s = ne, p, s
        self.q = q if q else p + 1
        self.kv = bspline.knot_vector(ne, p, s)
        self.n = bspline.n_functions(self.kv, p)
        self.edges = bspline.elements(self.kv)
        assert len(self.edges) == ne + 1
        pts, wts, self.active = [], [], []
        for e in range(ne):
            a, b = self.edges[e], self.edges[e + 1]
            x, w = bspline.gauss_legendre(self.q, a, b)
            pts.append(x)
            wts.append(w)
            # B_{i,p} is non-zero on (a, b) iff its support [xi_i, xi_{i+p+1}]
            # contains the element.
            act = [i for i in range(self.n)
                   if self.kv[i] <= a and self.kv[i + p + 1] >= b]
            self.active.append(np.array(act))
        self.pts = np.array(pts)            # (ne, q)
        self.wts = np.array(wts)            # (ne, q)
        flat = self.pts.ravel()
        self.B = bspline.basis_all(self.kv, p, flat).reshape(self.n, ne, self.q)
        self.dB = bspline.basis_deriv_all(self.kv, p, flat).reshape(self.n, ne, self.q)


def make_spaces(dim, ne, p, s, q=None):
    ne = [ne] * dim if np.isscalar(ne) else list(ne)
    return [Space1D(ne[d], p, s, q) for d in range(dim)]


def n_interior(spaces):
    return int(np.prod([sp1.n - 2 for sp1 in spaces]))


def assemble_full(spaces, kappa=None, rho=None):
    """Full (boundary functions included) K and M as CSR matrices.

    ``kappa``/``rho``: per-element coefficients, x-fastest element order, or
    None for 1.  Loops over elements; on each one integrates
    kappa_e * grad B_a . grad B_b and rho_e * B_a B_b with the tensor Gauss
    rule at all active function pairs.
    """
    dim = len(spaces)
    nes = [s1.ne for s1 in spaces]
    ns = [s1.n for s1 in spaces]
    n_el = int(np.prod(nes))
    kappa = np.ones(n_el) if kappa is None else np.asarray(kappa, dtype=np.float64)
    rho = np.ones(n_el) if rho is None else np.asarray(rho, dtype=np.float64)
    rows, cols, kv, mv = [], [], [], []
    estrides = np.cumprod([1] + nes[:-1])
    for eidx in itertools.product(*[range(n) for n in reversed(nes)]):
        eidx = eidx[::-1]                       # (ex, ey, ez), x fastest
        e = int(np.dot(eidx, estrides))
        k0, m0, gidx = element_unit_matrices(spaces, eidx)
        rr, cc = np.meshgrid(gidx, gidx, indexing='ij')
        rows.append(rr.ravel())
        cols.append(cc.ravel())
        kv.append((kappa[e] * k0).ravel())
        mv.append((rho[e] * m0).ravel())
    nt = int(np.prod(ns))
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    K = sp.coo_matrix((np.concatenate(kv), (r, c)), shape=(nt, nt)).tocsr()
    M = sp.coo_matrix((np.concatenate(mv), (r, c)), shape=(nt, nt)).tocsr()
    K.sum_duplicates()
    M.sum_duplicates()
    return K, M


def interior_index(spaces):
    """Full-space indices of the interior (Dirichlet-free) functions, in the
    interior lexicographic order (x fastest)."""
    ns = [s1.n for s1 in spaces]
    strides = np.cumprod([1] + ns[:-1])
    idx = np.zeros(1, dtype=np.int64)
    for d in range(len(spaces)):
        idx = (np.arange(1, ns[d] - 1)[:, None] * strides[d] + idx[None, :]).ravel()
    return idx


def dirichlet(K, M, spaces):
    """Delete the boundary functions (first/last per direction)."""
    idx = interior_index(spaces)
    return K[idx][:, idx].tocsr(), M[idx][:, idx].tocsr()


def assemble(dim, ne, p, s, kappa=None, rho=None, q=None):
    """Interior K, M (CSR, FP64) of the Dirichlet problem."""
    spaces = make_spaces(dim, ne, p, s, q)
    Kf, Mf = assemble_full(spaces, kappa, rho)
    return dirichlet(Kf, Mf, spaces)


def matrices_1d(ne, p, s, q=None):
    """1D stiffness and mass matrices of Eq. 1Dmatrix (full, dense)."""
    s1 = Space1D(ne, p, s, q)
    K = np.zeros((s1.n, s1.n))
    M = np.zeros((s1.n, s1.n))
    for e in range(ne):
        a = s1.active[e]
        B = s1.B[a, e, :]
        dB = s1.dB[a, e, :]
        w = s1.wts[e]
        K[np.ix_(a, a)] += np.einsum('ap,bp,p->ab', dB, dB, w)
        M[np.ix_(a, a)] += np.einsum('ap,bp,p->ab', B, B, w)
    return K, M


def kronecker_interior(dim, ne, p, s, q=None):
    """Interior K, M from the Kronecker formulas of Eq. 2Dmatrix (kappa=rho=1).

    2D: K = My (x) Kx + Ky (x) Mx, M = My (x) Mx; 3D analogously.  Built
    from the Dirichlet-reduced 1D matrices, so the x-fastest ordering means
    the y factor is on the left of the Kronecker product.
    """
    K1, M1 = matrices_1d(ne, p, s, q)
    K1, M1 = K1[1:-1, 1:-1], M1[1:-1, 1:-1]
    K1s, M1s = sp.csr_matrix(K1), sp.csr_matrix(M1)
    if dim == 1:
        return K1s, M1s
    if dim == 2:
        K = sp.kron(M1s, K1s) + sp.kron(K1s, M1s)
        M = sp.kron(M1s, M1s)
    else:
        K = (sp.kron(sp.kron(M1s, M1s), K1s) + sp.kron(sp.kron(M1s, K1s), M1s)
             + sp.kron(sp.kron(K1s, M1s), M1s))
        M = sp.kron(sp.kron(M1s, M1s), M1s)
    return K.tocsr(), M.tocsr()


def element_unit_matrices(spaces, e_multi):
    """Unit-coefficient element matrices (K0_e, M0_e) and the full-space
    indices of the active functions on element ``e_multi`` (tuple)."""
    dim = len(spaces)
    ns = [s1.n for s1 in spaces]
    strides = np.cumprod([1] + ns[:-1])
    act = [spaces[d].active[e_multi[d]] for d in range(dim)]
    vals, gl, wq = None, None, None
    for d in range(dim):
        Bd = spaces[d].B[act[d], e_multi[d], :]
        dBd = spaces[d].dB[act[d], e_multi[d], :]
        wd = spaces[d].wts[e_multi[d]]
        if vals is None:
            vals, wq = Bd, wd
            gl = [dBd if dd == 0 else Bd for dd in range(dim)]
        else:
            vals = np.einsum('ap,bq->bapq', vals, Bd).reshape(-1, vals.shape[1] * Bd.shape[1])
            gl = [np.einsum('ap,bq->bapq', gl[dd], dBd if dd == d else Bd).reshape(vals.shape)
                  for dd in range(dim)]
            # quadrature points of the directions so far (p) slowest, this
            # direction's (q) fastest: the same order as vals and gl
            wq = np.einsum('p,q->pq', wq, wd).ravel()
    k0 = sum(np.einsum('ap,bp,p->ab', g, g, wq) for g in gl)
    m0 = np.einsum('ap,bp,p->ab', vals, vals, wq)
    gidx = np.zeros(1, dtype=np.int64)
    for d in range(dim):
        gidx = (act[d][:, None] * strides[d] + gidx[None, :]).ravel()
    return k0, m0, gidx
