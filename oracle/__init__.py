"""CPU FP64 oracle for the rIGA shift-and-invert eigensolver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library, its
Python binding) may import, call or link anything in this package; only the
tests, the smoke check and the CPU-baseline leg of the benchmark do.  It
shares no code with the GPU path: it has its own knot vectors, its own
Cox--de Boor evaluation, its own quadrature loop and its own eigen-solves,
all written in plain NumPy/SciPy, slow and obviously correct.

Modules (each function cites the passage of Hashemian, Pardo & Calo,
"Refined isogeometric analysis for generalized Hermitian eigenproblems",
arXiv 2009.08167, that it follows):

* ``bspline``  -- knot vectors (Eq. U, Sec. 3.2), Cox--de Boor (Eq. N),
  Gauss--Legendre rules.
* ``assembly`` -- Galerkin stiffness and mass matrices of the weak form
  (Eqs. weakform--weakform3) with per-element coefficients, Dirichlet
  elimination, and the 1D matrices / Kronecker construction (Eqs. 1Dmatrix,
  2Dmatrix).
* ``eigen``    -- the generalized eigenproblem (Eq. GHEP): dense
  Cholesky-reduced solve (Sec. 4.1), sparse shift-and-invert solve (Eq.
  ST_GHEP), inertia counts (Remark on inertia), residuals, normalisation.
* ``accuracy`` -- EVerr, EFerr_L2, EFerr_E against the exact eigenpairs
  (Eqs. exact, norms, eigerrors; diagonal modes as in Sec. 8).
* ``hermitian`` -- a complex Hermitian source for the Hermitian case of Eq.
  GHEP: the magnetic Laplacian with a constant potential (gauge-equivalent
  to the Laplacian), its real-equivalent pencil and a dense Hermitian solve.
* ``lanczos``  -- one classical Gram-Schmidt pass of the full M-
  reorthogonalisation (Sec. 4.2): c = W^T x, x - B c with W = M B.
* ``grad``     -- adjoint eigenvalue gradient with respect to per-element
  coefficients (not in the paper: first-order perturbation theory of a
  simple eigenpair of a symmetric pencil).

Every function here is pinned by the ``-m "not gpu"`` tests against closed
forms, invariants and brute force; see ``tests/test_oracle_*.py``.
"""
