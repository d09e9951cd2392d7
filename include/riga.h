/*
 * riga.h -- C ABI of the rIGA shift-and-invert eigensolver for one MI355X.
 *
 * Computes eigenpairs of the generalized symmetric eigenproblem
 *     K u = lambda M u                                   (Eq. GHEP, Sec. 3.1)
 * where K and M are the Galerkin stiffness and mass matrices of the Dirichlet
 * problem -div(kappa grad u) = lambda rho u on the unit square or cube
 * (Eqs. helmholtz, weakform--weakform3; kappa = rho = 1 is the paper's
 * Laplace problem), discretised with tensor-product B-splines of degree p on
 * a uniform mesh (Eqs. u, U, N), optionally refined into rIGA
 * macro-elements by knots of multiplicity p every `sep_spacing` elements
 * (Sec. 3.2).  The solver is shift-and-invert Lanczos (Eqs. ST_GHEP,
 * Lanczos--LanczosAlphaBeta) on LDL^T factorisations of K - sigma M ordered
 * by the tree of separators, with spectrum slicing driven by inertia
 * (Remark on inertia) and Ritz extraction (Eqs. LanczosRitz, RitzValues).
 *
 * Conventions shared by every call:
 *  - Every call returns riga_status (RIGA_OK = 0).  No C++ exception crosses
 *    the ABI.  On error, riga_last_error() returns a thread-local message.
 *  - Degrees of freedom are the interior tensor-product functions (the first
 *    and last function in each direction are removed by the Dirichlet
 *    condition), ordered lexicographically with x fastest (the vectorised
 *    control tensor of the Remark on Tensor(u)).  Elements are ordered x
 *    fastest as well.
 *  - "_dev" pointers are device (HBM) pointers; "_host" pointers are host
 *    memory.  The caller owns every buffer it passes; the library copies
 *    what it keeps.  Work is ordered on the hipStream_t passed as `stream`
 *    (NULL = the null stream); calls synchronise that stream before they
 *    return host results.  The stream in riga_mesh_desc is the problem's
 *    own: buffers the problem keeps are allocated on it, riga_destroy
 *    synchronises it, and it must stay valid until then.  A stream passed to
 *    any other call is used by that call only and is not remembered.
 *  - A riga_problem is owned by the caller until riga_destroy().  It must not
 *    be used from two threads at once.
 */
#ifndef RIGA_H
#define RIGA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RIGA_OK = 0,
  RIGA_EINVAL = -1,        /* invalid argument or descriptor */
  RIGA_ENOMEM = -2,        /* device or host allocation failed */
  RIGA_EDEVICE = -3,       /* a HIP call failed (message names it) */
  RIGA_ENOCONV = -4,       /* not all requested pairs converged; n_found holds the rest */
  RIGA_ESINGULAR = -5,     /* K - sigma M singular to working precision (a pivot was perturbed) */
  RIGA_EDEGENERATE = -6,   /* gradient requested for an eigenvalue that is not simple */
  RIGA_EUNSUPPORTED = -7   /* valid request outside what the library implements */
} riga_status;

enum { RIGA_FP64 = 0, RIGA_MIXED = 1 };            /* riga_eigs_opts.precision */
enum { RIGA_MAT_K = 0, RIGA_MAT_M = 1, RIGA_MAT_A = 2 }; /* riga_spmv: K, M, K - sigma M */

typedef struct riga_problem riga_problem;

/* Mesh and coefficients (Sec. 3.1--3.2). */
typedef struct {
  int32_t dim;            /* 2 or 3 */
  int32_t ne[3];          /* elements per direction (unused entries ignored) */
  int32_t p;              /* B-spline degree, 1..6 */
  int32_t sep_spacing;    /* 0: maximum-continuity IGA; s > 0: knot multiplicity p at
                             every element boundary k with k % s == 0 (rIGA, Sec. 3.2) */
  int32_t nquad;          /* Gauss points per direction; 0 -> p + 1 */
  const double* kappa;    /* [n_elem] per-element stiffness coefficient, > 0; NULL -> 1 */
  const double* rho;      /* [n_elem] per-element mass coefficient, > 0; NULL -> 1 */
  int32_t coeffs_on_device; /* kappa/rho are device pointers (1) or host pointers (0) */
  int32_t leaf_dofs;      /* nested-dissection leaf size in DOFs; 0 -> default */
  void* stream;           /* hipStream_t */
  int32_t hermitian;      /* 0: the real pencil above.  1: the complex Hermitian pencil of
                             the magnetic Laplacian -(grad - iA).(grad - iA) u = lambda u with
                             the constant vector potential `potential` (kappa = rho = 1 only):
                             K_ab = int (grad B_b - iA B_b).conj(grad B_a - iA B_a),
                             M_ab = int B_a B_b (Eq. GHEP read with conjugate transposes).
                             It is solved in its real-equivalent form [[Re K, -Im K],
                             [Im K, Re K]], diag(M, M), with the real and imaginary parts
                             of DOF d at unknowns 2d and 2d + 1: riga_problem_info's n_dof
                             counts those 2N unknowns, riga_spmv / riga_factor / riga_solve
                             act on that real system, and riga_eigs returns each complex
                             eigenvalue once with its eigenvector as N complex numbers
                             (2N doubles, real and imaginary parts interleaved) */
  double potential[3];    /* A, per direction (unused entries ignored) */
} riga_mesh_desc;

/* Eigen-solve request (Sec. 4.1: eigenvalues in [lambda_s, lambda_e]). */
typedef struct {
  double lo;              /* interval start (inclusive) */
  double hi;              /* interval end (exclusive); +INFINITY -> the nev lowest >= lo */
  int32_t nev;            /* number of pairs wanted, returned ascending */
  int32_t precision;      /* RIGA_FP64, or RIGA_MIXED: FP32 fronts and solves refined in FP64
                             (2 steps per solve, doubled up to 8 when a run stalls) */
  double tol;             /* accept a pair when ||K u - lambda M u||_2 / (||K||_1 ||u||_2) <= tol;
                             0 -> 1e-9 */
  int32_t max_basis;      /* Lanczos basis size per run; 0 -> max(160, 4 per_shift + 32) */
  int32_t max_restarts;   /* Lanczos runs per shift; 0 -> 10 */
  int32_t per_shift;      /* eigenpairs targeted per shift; 0 -> 32 */
  uint64_t seed;          /* start vectors (counter-based hash of seed and index) */
  void* stream;           /* hipStream_t */
} riga_eigs_opts;

/* Counters of the operation classes of Table matvecs, and timings (seconds). */
typedef struct {
  int32_t n_shift;        /* shifts used (N_sh) */
  int32_t n_fact;         /* numeric factorisations (N_fa) */
  int32_t n_fb;           /* forward/backward eliminations (N_fb) */
  int32_t n_mv;           /* sparse matrix-vector products (N_mv), M, K and A */
  int32_t n_it;           /* Lanczos runs (restarts included) */
  int32_t n_ir;           /* iterative-refinement corrections (mixed precision) */
  int32_t n_perturbed_pivots; /* pivots replaced by a perturbation (static pivoting) */
  int32_t n_2x2_pivots;   /* Bunch-Kaufman 2x2 pivots taken */
  /* host wall times; t_fact counts only the time the solve waited for a
   * factorisation (one made ahead on a second stream while the Lanczos runs
   * at the current shift proceed counts only the wait at its end) */
  double t_fact, t_fb, t_mv, t_orth, t_proj, t_ritz, t_total;
  double flops_fact;      /* algorithmic flops of one factorisation */
  double bytes_fb;        /* algorithmic bytes of one forward+backward elimination */
  int32_t n_thick;        /* Lanczos runs continued from a thick-restart basis (Sec. 4.2,
                             Eq. LanczosRestart: a run whose basis filled up keeps its
                             unconverged Ritz vectors nearest the shift, up to half the
                             basis, and its last Lanczos vector) */
} riga_stats;

/* Static facts about an assembled problem (host-side analysis). */
typedef struct {
  int64_t n_dof;          /* interior DOFs N */
  int64_t n_elem;         /* elements */
  int64_t nnz;            /* structural non-zeros of K (= of M) */
  int32_t n1[3];          /* interior functions per direction */
  int32_t n_fronts;       /* nodes of the separator tree */
  int32_t tree_height;    /* levels of the tree (leaves = 0) */
  int32_t max_front;      /* largest front order */
  int32_t max_fs;         /* largest fully-summed block */
  int64_t nnz_l;          /* entries of L (lower, diagonal included) as the supernodal
                             fronts store them (fully-summed blocks dense) */
  double flops_fact;      /* flops of one factorisation of those fronts: sum over their
                             columns of c (c + 1), c = rows below the diagonal */
  int64_t front_pool;     /* entries of the dense front pool */
  int64_t nnz_l_exact;    /* entries of L for the same elimination order without
                             pivoting (exact structural fill, diagonal included) */
  double flops_fact_exact; /* sum over the columns of that L of c (c + 1) */
  int32_t components;     /* 1: real pencil; 2: complex pencil (n_dof = 2 x complex DOFs) */
  double sweep_bytes_stored; /* FP64 factor bytes one forward + backward elimination reads
                             as stored (partitioned-inverse blocks of the levels below
                             the top block, both copies of the top block's inverse);
                             0 before riga_assemble */
  int32_t top_cut;        /* height from which the sweeps use the top block's explicit
                             inverse; -1: none (or before riga_assemble) */
  int32_t fused_heights;  /* bottom heights swept in one launch per direction (one
                             workgroup per subtree); 0: none */
  int32_t fused_subtrees; /* workgroups of those launches */
  int32_t tuned;          /* 1: top_cut and fused_heights are a measured choice
                             (riga_tune, or its cache at assembly) */
} riga_problem_info_t;

/* Allocation hooks (e.g. torch's caching allocator).  Optional. */
typedef struct {
  void* ctx;
  void* (*alloc)(void* ctx, size_t bytes, void* stream);
  void (*free)(void* ctx, void* ptr, void* stream);
} riga_allocator;

/* riga_set_allocator: route the library's device allocations through `a`
 * (copied; NULL restores hipMalloc/hipFree).  Affects allocations made after
 * the call, also those of existing problems; each buffer is released by the
 * allocator that made it, so hooks may be replaced while problems live (the
 * hook's ctx and functions must stay valid until its buffers are freed).
 * alloc(ctx, bytes, stream) returns device memory usable on `stream` or
 * NULL, which makes the calling entry point return RIGA_ENOMEM; nothing
 * leaks (a failed call releases its own buffers; a problem's buffers go
 * with riga_destroy).  alloc and free may be called from any thread of the
 * library.  RIGA_EINVAL if either function is NULL. */
riga_status riga_set_allocator(const riga_allocator* a);

/* riga_analyze: host-only analysis of a mesh (no device needed): knot
 * vectors and DOF maps (Sec. 3.1--3.2), the sparsity pattern, the tree of
 * separators and the supernodal symbolic factorisation (Sec. 5, one symbolic
 * factorisation per pattern).  *out receives a problem handle without device
 * data; riga_problem_info and riga_tree_export work on it, the solver
 * calls return RIGA_EINVAL.  Errors: RIGA_EINVAL for a bad descriptor. */
riga_status riga_analyze(const riga_mesh_desc* desc, riga_problem** out);

/* riga_assemble: riga_analyze, then assemble K and M on the device with
 * Gauss quadrature (Eqs. 1Dmatrix/2Dmatrix generalised to per-element
 * kappa, rho).  `desc->kappa/rho` are copied.  *out is owned by the caller.
 * Errors: RIGA_EINVAL (descriptor, non-positive coefficient), RIGA_ENOMEM,
 * RIGA_EDEVICE. */
riga_status riga_assemble(const riga_mesh_desc* desc, riga_problem** out);

/* riga_update_coefficients: replace kappa/rho (n_elem each; NULL -> 1) and
 * re-assemble K and M on the device, reusing the analysis of the pattern.
 * `on_device`: the arrays are device (1) or host (0) pointers; both are
 * copied.  Invalidates the current factorisation.  Errors: RIGA_EINVAL
 * (problem without device data, non-positive host coefficient),
 * RIGA_EDEVICE. */
riga_status riga_update_coefficients(riga_problem* pr, const double* kappa, const double* rho,
                                     int32_t on_device, void* stream);

riga_status riga_problem_info(const riga_problem* pr, riga_problem_info_t* info);

/* riga_tree_export: copy the symbolic analysis to host arrays (any may be
 * NULL).  perm[n_dof]: new (elimination) position of each DOF.
 * front_k/front_f/front_parent/front_height[n_fronts]: fully-summed size,
 * front order, parent (-1 = root) and height of each tree node, in
 * elimination (post-)order.  front_rows: concatenated front index lists
 * (original DOF indices, fully-summed first), sum(front_f) entries. */
riga_status riga_tree_export(const riga_problem* pr, int32_t* perm, int32_t* front_k,
                             int32_t* front_f, int32_t* front_parent, int32_t* front_height,
                             int32_t* front_rows);

/* riga_get_matrices: copy the assembled CSR matrices to the host (row_ptr
 * [n_dof+1], col_idx [nnz], k_vals/m_vals [nnz]; any may be NULL).  Column
 * indices ascending within a row. */
riga_status riga_get_matrices(const riga_problem* pr, int64_t* row_ptr, int32_t* col_idx,
                              double* k_vals, double* m_vals);

/* riga_spmv: y = K x, M x or (K - sigma M) x for the last factorised sigma
 * (Sec. 5.1 "mat-vec").  x_dev, y_dev: [n_dof] device FP64, not
 * overlapping.  Queued on `stream`; returns without waiting for it. */
riga_status riga_spmv(riga_problem* pr, int32_t which, const double* x_dev, double* y_dev,
                      void* stream);

/* riga_factor: numeric LDL^T factorisation of K - sigma M with Bunch-Kaufman
 * pivoting inside fronts (Sec. 5: one numeric factorisation per shift), in
 * FP64 or (precision = RIGA_MIXED) FP32.  *neg_pivots (may be NULL) receives
 * the inertia nu(K - sigma M), the number of eigenvalues below sigma (Remark
 * on inertia).  The factorisation stays in the problem for riga_solve.
 * A pivot smaller than 1e-20 (||K||_1 + |sigma| ||M||_1) in magnitude is
 * replaced by that value with its sign (zero counts as positive) and counted
 * in stats->n_perturbed_pivots; the call then returns RIGA_ESINGULAR (sigma
 * lies on an eigenvalue to working precision) with *neg_pivots and *stats
 * filled and the perturbed factorisation kept: solves with it are not
 * meaningful. */
riga_status riga_factor(riga_problem* pr, double sigma, int32_t precision,
                        int64_t* neg_pivots, riga_stats* stats);

/* riga_factor_batched: riga_factor of `count` independent problems at once,
 * problem i at sigmas[i] (host array), all in `precision` (Sec. 5's one
 * numeric factorisation per shift, for many instances): the fronts of one
 * tree height of every problem go in one launch per kernel (assembly,
 * LDS-resident fronts, the blocked fronts' panel, update and finishing
 * kernels), heights in order from the leaves.  Each front gets the same
 * arithmetic as in riga_factor, so every factorisation, inertia and later
 * riga_solve result is identical bit for bit to riga_factor's at the same
 * shift.  probs: `count` distinct problems assembled on the current device.
 * neg_pivots [count] (host, may be NULL): the inertias; stats [count] (may
 * be NULL): as riga_factor's.  The call waits for earlier work on each
 * problem's stream, runs on a stream of its own and returns when all are
 * done.  A problem with perturbed pivots is handled as in riga_factor: the
 * call returns RIGA_ESINGULAR (riga_last_error() names the first such
 * instance) with every output filled and every factorisation kept.
 * count = 0 is a no-op; a repeated problem, another device or a
 * non-finite shift is RIGA_EINVAL. */
riga_status riga_factor_batched(riga_problem* const* probs, int32_t count, const double* sigmas,
                                int32_t precision, int64_t* neg_pivots, riga_stats* stats);

/* riga_tune: measured choice of how the forward/backward elimination of
 * `pr` is decomposed (Sec. 4.2's sweeps, applied once per Lanczos step):
 * the height from which the top tree levels are swept through their
 * explicit inverse (-1: none); the bottom heights swept in one launch per
 * subtree are left off (0).  Every cut within the size limits, and none, is
 * timed on the problem itself -- the best
 * of two factorisations at sigma = 0 in `precision` and the median of
 * `reps` sweep pairs (reps <= 0: 20), each after a 320 MB write that takes
 * the factor out of the caches as the eigensolver's Gram-Schmidt passes
 * do -- and the fastest by sweep pair + factorisation / 70, if it beats the
 * configuration in place by more than 3%, is applied to the problem and
 * stored in
 * the tuning cache under a key of the device (architecture, compute units)
 * and of the elimination tree.  Problems assembled later with the same key
 * take the stored choice, unless RIGA_TOP_CUT or RIGA_SUBTREE_HEIGHTS is
 * set.  The cache is the text file named by RIGA_TUNE_CACHE, else
 * $XDG_CACHE_HOME/riga/tune.txt, else $HOME/.cache/riga/tune.txt
 * (RIGA_TUNE_CACHE="" keeps choices in the problem only).  Choices differ
 * in the order of the same operations: results differ between them by
 * rounding only.  The problem's factorisations are discarded: factorise
 * again before riga_solve.  out (host, may be NULL) receives the choice,
 * its times and those of the configuration in place before the call. */
typedef struct riga_tune_result {
  int32_t top_cut;              /* chosen cut height (-1: no top block) */
  int32_t fused_heights;        /* chosen fused bottom heights (0: none) */
  int32_t candidates;           /* configurations timed */
  int32_t before_top_cut;       /* the configuration before the call */
  int32_t before_fused_heights;
  double sweep_us;              /* chosen: one forward + backward elimination, us */
  double fact_us;               /* chosen: one factorisation (host clock), us */
  double before_sweep_us;
  double before_fact_us;
} riga_tune_result;
riga_status riga_tune(riga_problem* pr, int32_t precision, int32_t reps, riga_tune_result* out);

/* riga_solve: x = (K - sigma M)^{-1} b with the last factorisation (one
 * forward/backward elimination; in RIGA_MIXED the FP32 solve is refined in
 * FP64 until ||b - A x|| <= 1e-13 ||b|| or `max_ir` corrections).  b_dev,
 * x_dev: [n_dof] device FP64, may not alias. */
riga_status riga_solve(riga_problem* pr, const double* b_dev, double* x_dev, int32_t max_ir,
                       void* stream);

/* riga_solve_multi: X(:, i) = (K - sigma M)^{-1} B(:, i), i < nrhs, with the
 * last factorisation: one forward/backward elimination per column, queued on
 * `stream` one after another with no host synchronisation between them (the
 * call returns when the last is done).  In RIGA_MIXED with max_ir > 0 each
 * column is refined as in riga_solve.  B_dev, X_dev: device FP64,
 * column-major with leading dimension ld >= n_dof, not overlapping.
 * nrhs = 0 is a no-op; nrhs < 0 or ld < n_dof is RIGA_EINVAL. */
riga_status riga_solve_multi(riga_problem* pr, const double* B_dev, double* X_dev, int32_t nrhs,
                             int64_t ld, int32_t max_ir, void* stream);

/* riga_project: one classical Gram-Schmidt pass of the full
 * M-reorthogonalisation of the Lanczos vectors (Sec. 4.2, Eqs. Lanczos and
 * LanczosAlphaBeta with a fully reorthogonalised basis):
 *     c = W^T x,   x <- x - B c,
 * where B = [b_1 .. b_m] is a basis and W = M B (so c holds the
 * M-inner products).  W_dev, B_dev: [n x m] column-major device FP64
 * (leading dimension n); x_dev [n] device FP64, updated in place; c_dev [m]
 * device FP64 output.  x and c may not overlap W or B.  The reductions over
 * rows run in a fixed order (results are bitwise reproducible).  A device
 * workspace of ceil(n / 4096) * m doubles is allocated for the call (the
 * allocator hook, else hipMalloc) and released before it returns; the call
 * waits for `stream`.  RIGA_EINVAL unless n >= 1 and
 * 1 <= m <= RIGA_PROJECT_MAX_COLS. */
#define RIGA_PROJECT_MAX_COLS 8192
riga_status riga_project(int64_t n, int32_t m, const double* W_dev, const double* B_dev, double* x_dev,
                         double* c_dev, void* stream);

/* riga_project_noalloc: riga_project for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments and results (bitwise),
 * but the workspace is a fixed scratch array of 2^20 doubles (8 MiB) per
 * GPU, held by the library until the process ends: RIGA_EINVAL when
 * ceil(n / 4096) * m exceeds it (or as riga_project).  Allocates nothing
 * and does not wait: the work is queued on `stream` and the call returns.
 * Every call on a GPU uses that GPU's one scratch array, so calls that
 * overlap on one GPU (other streams, other threads) race; nothing in the
 * scratch needs to start at zero. */
riga_status riga_project_noalloc(int64_t n, int32_t m, const double* W_dev, const double* B_dev,
                                 double* x_dev, double* c_dev, void* stream);

/* riga_eigs: the nev lowest eigenpairs with lambda in [lo, hi) (Sec. 4).
 * Spectrum slicing with inertia counts (Sec. 4.1): the factorisation at a
 * guess of the next shift runs on a second HIP stream of the library's own
 * (and a second host thread) while the Lanczos runs at the current shift
 * proceed; the call returns only after both are done.  An open-ended
 * request (hi = +inf) for at least 4 * per_shift pairs is split in two
 * spectrum slices solved at once, the upper one on a further host thread
 * and HIP stream with its own factorisations, when the device's free memory
 * holds its storage; the split point only balances the work, each slice
 * counts its own pairs by inertia.  Not reentrant for one problem: calls on
 * the same problem must not overlap.
 * evals_host[nev]: ascending eigenvalues (Rayleigh quotients).
 * evecs_dev: [n_dof * nev] column-major device buffer for M-normalised
 * eigenvectors, or NULL.  resid_host[nev] (or NULL): relative residuals
 * ||K u - lambda M u||_2 / (||K||_1 ||u||_2).  *n_found: pairs returned.
 * stats (or NULL): counters and timings.  Returns RIGA_ENOCONV when the
 * restart budget ran out; then n_found < nev and the pairs returned are the
 * complete set of eigenvalues in [lo, sigma) for the last shift sigma whose
 * inertia count they matched.
 * Ends and singular shifts: the ends are moved down by 1e-9 relative before
 * they are factorised, so an eigenvalue within 1e-9 |lo| below lo is
 * returned and one within 1e-9 |hi| below hi is not (an eigenvalue on an
 * end, to rounding, counts as lying at lo or at hi).  A shift whose
 * factorisation perturbs a pivot is moved down by 1e-9 relative and
 * factorised again (shift perturbation, counted in n_fact); RIGA_ESINGULAR
 * if three moves do not help. */
riga_status riga_eigs(riga_problem* pr, const riga_eigs_opts* opts, int32_t* n_found,
                      double* evals_host, double* evecs_dev, double* resid_host,
                      riga_stats* stats);

/* riga_eigs_batched: riga_eigs on `count` independent assembled problems at
 * once (instances of uneven size run concurrently on the device: a pool of
 * `workers` host threads, 0 -> 16, each with its own HIP stream; opts->stream
 * is ignored and the call returns when all instances are done).  Per
 * instance i: n_found[i], evals_host[i] ([nev] host), evecs_dev[i] ([n_dof_i
 * * nev] device, or NULL; evecs_dev itself may be NULL), resid_host[i] (or
 * NULL), stats[i] (stats may be NULL).  Each problem must appear once.
 * Returns RIGA_OK, or the first error (RIGA_ENOCONV only if no other error)
 * with riga_last_error() naming the instance. */
riga_status riga_eigs_batched(riga_problem* const* probs, int32_t count, const riga_eigs_opts* opts,
                              int32_t workers, int32_t* n_found, double* const* evals_host,
                              double* const* evecs_dev, double* const* resid_host,
                              riga_stats* stats);

/* riga_eig_grad: gradient of L = sum_i w_i lambda_i with respect to the
 * per-element coefficients, for M-normalised simple eigenpairs (not in the
 * paper; first-order perturbation: d lambda/d kappa_e = u^T K0_e u,
 * d lambda/d rho_e = -lambda u^T M0_e u).  evals_host[k], w_host[k] host;
 * evecs_dev [n_dof * k] column-major device; dkappa_dev, drho_dev [n_elem]
 * device outputs.  RIGA_EDEGENERATE if two of the eigenvalues are within
 * 1e-8 relative of each other. */
riga_status riga_eig_grad(riga_problem* pr, int32_t k, const double* evals_host,
                          const double* evecs_dev, const double* w_host, double* dkappa_dev,
                          double* drho_dev, void* stream);

/* riga_mode_errors: eigenfunction errors of computed eigenpairs against the
 * exact eigenpairs of the Dirichlet Laplacian on the unit square or cube
 * (Eq. exact: lambda_e = pi^2 (i^2 + j^2 [+ k^2]), u_e = 2^(d/2) prod
 * sin(i pi x)), as the accuracy study of Sec. 8 uses them (Eqs. norms,
 * eigerrors).  Meaningful for a problem assembled with kappa = rho = 1.
 * n_vec computed pairs: lam_host [n_vec] (host), U_dev [n_vec][n_dof]
 * device FP64, M-normalised (the layout riga_eigs returns).  modes_host
 * [n_modes][dim] 1-based mode indices (Sec. 8 uses the diagonal ones).
 * nquad: Gauss points per direction and element for the integrals (0 ->
 * p + 6, at most 16).  Outputs per mode, host [n_modes]:
 *   match    index of the computed eigenvector with the largest |(u_h, u_e)|
 *   overlap  that (u_h, u_e) (L2 inner product)
 *   ef_l2    EFerr_L2 = ||u_h - s u_e||^2, s = +-1 giving the smaller value
 *   ef_e     EFerr_E = a(u_h - s u_e, u_h - s u_e) / lambda_e (integrated
 *            directly; equals EVerr + EFerr_L2 for a Galerkin pair)
 *   ev       (lam_host[match] - lambda_e) / lambda_e
 * Runs on `stream` (U_dev must be ready there) and returns when the results
 * are on the host.  RIGA_EINVAL on a mode index below 1 or nquad above 16. */
riga_status riga_mode_errors(riga_problem* pr, int32_t n_vec, const double* lam_host,
                             const double* U_dev, int32_t n_modes, const int32_t* modes_host,
                             int32_t nquad, int32_t* match, double* overlap, double* ef_l2,
                             double* ef_e, double* ev, void* stream);

/* riga_exact_eigenvalues: the `count` smallest exact eigenvalues of the
 * Dirichlet Laplacian on the unit square (dim 2) or cube (dim 3), Eq. exact,
 * ascending with multiplicity, into out_host [count].  Host only; EVerr of
 * the n-th computed eigenvalue is (lambda_h,n - out_host[n]) / out_host[n]. */
riga_status riga_exact_eigenvalues(int32_t dim, int32_t count, double* out_host);

void riga_destroy(riga_problem* pr);
const char* riga_status_string(riga_status s);
const char* riga_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* RIGA_H */
