// Shift-and-invert Lanczos with full M-reorthogonalisation, explicit
// restarts with locking, and spectrum slicing driven by inertia
// (arXiv 2009.08167, Sec. 4: Eqs. ST_GHEP, Lanczos--RitzValues, Remark on
// inertia, Eq. LanczosRestart and the deflation paragraph after it).
//
// The host only orchestrates: every vector operation, the factorisation,
// the solves and the projected eigensolve run in the HIP kernels.  The host
// reads back a few scalars per convergence check (Ritz values and the last
// row of the projected eigenvectors) and the inertia of each factorisation.
//
// Storage: B = [U_locked | V] and W = M B, column-major N x (lock cap +
// basis cap + 1), so one transposed product c = W^T x gives the M-inner
// products against the locked vectors and the Lanczos basis together.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <thread>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <limits>
#include <memory>
#include <numeric>
#include <string>

#include "problem.h"

namespace riga {


namespace {

using clk = std::chrono::steady_clock;

// refinement steps per mixed-precision solve after escalation (2 at start)
constexpr int MAX_IR_ESCALATED = 8;

// refinement steps per FP64 solve after escalation (none at start)
constexpr int MAX_IR_FP64 = 2;

// deflation window, in intervals between consecutive shifts below the shift
constexpr double DEFLATE_SPACINGS = 4.0;

// Candidate Ritz vectors are projected once against the locked pairs when
// N * (locked pairs) * ceil(candidates / 8) is at most this (the block
// projection reads the locked block once per 8 candidates): every 4096-pair
// request up to 2D 1024^2 (about 1.7e10) is covered
constexpr double LOCK_PROJECT_MAX = 17179869184.0;

// A shift whose factorisation had to perturb a pivot (K - sigma M singular
// to working precision: the shift sits on an eigenvalue) is moved down by
// this much, relative, and factorised again, at most SHIFT_MOVES times.
constexpr double SHIFT_NUDGE = 1e-9;
constexpr int SHIFT_MOVES = 3;

// The ends of a requested interval are moved down by this much, relative,
// so that an eigenvalue lying on an end within rounding is counted by the
// inertia at the end the same way the locking test classifies it: such an
// eigenvalue counts as lying at lo (returned) or at hi (not returned).
constexpr double END_SHIFT = 1e-9;

// spectrum slices solved at once at most (each with a host thread, a HIP
// stream and a solve context of the problem)
constexpr int MAX_SLICES = 8;

// RIGA_DEFLATE_ALL=1 projects every Lanczos vector against all locked pairs
// (no window); read per call
bool deflate_window_on() {
  const char* v = std::getenv("RIGA_DEFLATE_ALL");
  return !(v && *v && *v != '0');
}

// Thick restarts (RIGA_THICK_RESTART=0 switches them off: a run whose basis
// fills up then restarts from a fresh vector, as a run that found its pairs).
bool thick_restart_on() {
  const char* v = std::getenv("RIGA_THICK_RESTART");
  return !(v && *v == '0');
}

// Lanczos steps replayed from a HIP graph captured once per run
// (RIGA_GRAPH=1).  Off by default: bitwise the eager results, but measured
// slower on one MI355X (2D 256^2 p=3 rIGA 2,239 against 2,305 eigenpairs/s,
// its IGA 1,398 against 1,576): the launches of a step are not host-bound
// here, and each run pays its capture and instantiation.
bool graph_on() {
  const char* v = std::getenv("RIGA_GRAPH");
  return v && *v == '1';
}

// A restart basis for thick-restart Lanczos (Sec. 4.2, Eq. LanczosRestart):
// with Ritz pairs (theta_i, s_i) of T_m kept and b_i = beta_{m+1} s_i[m-1],
// the projection on [V S, v_{m+1}] is the arrowhead [[diag(theta), b],
// [b^T, .]].  Lanczos on diag(theta) from b / |b| (full re-orthogonalisation,
// in FP64 on the host) gives an orthonormal Q, its columns reversed so that
// the last one is b / |b|, with Q^T diag(theta) Q tridiagonal: on
// [V S Q, v_{m+1}] the projection is tridiagonal with coupling |b| between
// the last kept vector and v_{m+1}, and the recurrence continues unchanged.
// Returns Q (c x c', column-major) with c' <= c (fewer when the Krylov space
// of diag(theta) and b is smaller), alpha[0..c'), beta[1..c'] (beta[c'] = |b|).
struct ThickBasis {
  int c = 0;
  std::vector<double> Q, alpha, beta;
};

ThickBasis thick_basis(const std::vector<double>& theta, const std::vector<double>& b) {
  ThickBasis T;
  const int c = (int)theta.size();
  double nb = 0.0, tmax = 0.0;
  for (int i = 0; i < c; ++i) {
    nb += b[i] * b[i];
    tmax = std::max(tmax, std::fabs(theta[i]));
  }
  nb = std::sqrt(nb);
  if (c == 0 || !(nb > 0.0)) return T;
  std::vector<double> U, a, g(1, 0.0);  // U: c x t, column-major
  std::vector<double> u(c), w(c);
  for (int i = 0; i < c; ++i) u[i] = b[i] / nb;
  for (int t = 0; t < c; ++t) {
    U.insert(U.end(), u.begin(), u.end());
    double at = 0.0;
    for (int i = 0; i < c; ++i) {
      w[i] = theta[i] * u[i];
      at += u[i] * w[i];
    }
    a.push_back(at);
    // w -= U (U^T w), twice
    for (int pass = 0; pass < 2; ++pass)
      for (int q = 0; q <= t; ++q) {
        const double* uq = &U[(size_t)q * c];
        double d = 0.0;
        for (int i = 0; i < c; ++i) d += uq[i] * w[i];
        for (int i = 0; i < c; ++i) w[i] -= d * uq[i];
      }
    double gn = 0.0;
    for (int i = 0; i < c; ++i) gn += w[i] * w[i];
    gn = std::sqrt(gn);
    if (t + 1 == c || gn <= 1e-12 * tmax) break;  // invariant subspace
    g.push_back(gn);
    for (int i = 0; i < c; ++i) u[i] = w[i] / gn;
  }
  const int cp = (int)a.size();
  T.c = cp;
  T.Q.resize((size_t)c * cp);
  T.alpha.resize(cp);
  T.beta.assign(cp + 1, 0.0);
  for (int q = 0; q < cp; ++q) {
    const int t = cp - 1 - q;
    std::memcpy(&T.Q[(size_t)q * c], &U[(size_t)t * c], c * sizeof(double));
    T.alpha[q] = a[t];
    if (q >= 1) T.beta[q] = g[cp - q];
  }
  T.beta[cp] = nb;
  return T;
}

// RIGA_LOG=1 prints one line per Lanczos run and per shift to stderr.
bool log_on() {
  static const bool on = [] {
    const char* v = std::getenv("RIGA_LOG");
    return v && *v && *v != '0';
  }();
  return on;
}
double secs(clk::time_point a, clk::time_point b) {
  return std::chrono::duration<double>(b - a).count();
}

// Factorises K - sigma M into F with shift perturbation: while a pivot had
// to be perturbed, the shift moves down by SHIFT_NUDGE relative and the
// factorisation is repeated.  F.sigma holds the shift used, F.refactored
// the repeats.  RIGA_ESINGULAR if SHIFT_MOVES moves do not help.
void factor_shift(riga_problem* pr, Factor& F, double sigma, int precision, hipStream_t s) {
  int moves = 0;
  while (true) {
    factor_numeric(pr, F, sigma, precision, s);
    F.refactored = moves;
    if (F.perturbed == 0) return;
    if (moves == SHIFT_MOVES)
      throw Error(RIGA_ESINGULAR, "K - sigma M singular at sigma = " + std::to_string(sigma) +
                                      " and at " + std::to_string(SHIFT_MOVES) + " shifts below it");
    sigma -= SHIFT_NUDGE * std::max(std::fabs(sigma), std::numeric_limits<double>::min());
    ++moves;
  }
}

struct Locked {
  double lam;
  double resid;
  int col;       // column in B / W
  bool partner = false;  // the J (times i) copy of a complex pencil's pair
};

struct Solver {
  riga_problem* pr;
  hipStream_t s;
  int64_t N;
  int lock_cap, mb, ncols;
  double lo, hi, tol;
  uint64_t seed;
  int per_shift;
  int max_restarts;
  int precision;
  // a complex Hermitian pencil in real-equivalent form: every eigenvalue is
  // double, its eigenspace {u, J u} (J: times i); both are locked together
  bool cplx = false;
  int max_ir;
  int max_ir_fp64 = 0;   // refinement steps of an FP64 solve (raised on a stall)
  int dim = 2;           // spatial dimension (eigenvalue-count growth)
  int64_t nu_lo = 0;     // eigenvalues below lo
  DBuf<double> B, W, x, y, c1, c2, partial, dotp, alpha, beta, scal;
  DBuf<int32_t> flag;
  DBuf<int32_t> dstep;   // the step index j read by a replayed step
  DBuf<double> rhs;      // the replayed step's right-hand side (M v_j)
  hipGraphExec_t gexec = nullptr;
  hipStream_t cap = nullptr;  // capture only (the solve's own stream may be the null stream)
  int32_t hstep = 0;     // host copy of the step index uploaded before replays
  DBuf<double> chk, S, Sh, Ub, KU, MU, res3, rqn, lam, rpart, bpart;
  double* theta = nullptr;  // in chk: theta[mb + 1], est[mb + 1], beta_m, flag
  double* tdest = nullptr;
  double* chk_extra = nullptr;
  DBuf<int32_t> sel;
  DBuf<double> ir_r, ir_d;
  std::vector<Locked> locked;
  int nl = 0;            // locked columns
  // deflation window of the current run: the locked columns from c_win on
  // hold every locked pair with eigenvalue >= win_lo; only they are
  // projected out, and only candidates >= win_lo are locked
  int c_win = 0;
  double win_lo = -INFINITY;
  int n_evicted = 0;
  uint64_t run_id = 0;
  riga_stats st{};
  clk::time_point t0;

  double* Bc(int j) { return B.p + (int64_t)j * N; }
  double* Wc(int j) { return W.p + (int64_t)j * N; }

  void alloc() {
    ncols = lock_cap + mb + 1;
    B.alloc((size_t)N * ncols, s);
    W.alloc((size_t)N * ncols, s);
    x.alloc(N, s);
    y.alloc(N, s);
    c1.alloc(ncols, s);
    c2.alloc(ncols, s);
    partial.alloc((size_t)proj_row_blocks(N) * ncols, s);
    dotp.alloc(spmv_dot_blocks(pr), s);
    alpha.alloc(mb + 1, s);
    beta.alloc(mb + 2, s);
    scal.alloc(8, s);
    flag.alloc(4, s);
    chk.alloc(2 * (mb + 1) + 2, s);
    theta = chk.p;
    tdest = chk.p + (mb + 1);
    chk_extra = chk.p + 2 * (mb + 1);
    S.alloc((size_t)(mb + 1) * (mb + 1), s);
    sel.alloc(2 * (mb + 2), s);
    const int umax = mb + 1;
    Sh.alloc((size_t)(mb + 1) * umax, s);
    Ub.alloc((size_t)N * umax, s);
    KU.alloc((size_t)N * umax, s);
    MU.alloc((size_t)N * umax, s);
    rqn.alloc(umax, s);
    res3.alloc(3 * (size_t)umax, s);  // u^T M u, ||K u - lam M u||^2, ||u||^2
    lam.alloc(umax, s);
    rpart.alloc(residual_partials(N, umax), s);
    ir_r.alloc(N, s);
    ir_d.alloc(N, s);
    dstep.alloc(1, s);
    rhs.alloc(N, s);
  }

  ~Solver() {
    drop_graph();
    if (cap) (void)hipStreamDestroy(cap);
  }

  void drop_graph() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    gexec = nullptr;
  }

  SolveCtx* ctx = nullptr;  // the solve's factorisations and sweep scratch
  Factor& cur() { return ctx->current(); }

  // counts one factorisation (in place or look-ahead) in the statistics
  void count_factor(const Factor& F) {
    st.n_fact += 1 + F.refactored;
    st.n_perturbed_pivots += F.perturbed;
    st.n_2x2_pivots += F.two;
  }

  // factorises K - sigma M in place of the current factorisation (at a
  // shift moved down if sigma is singular; cur().sigma holds the one used)
  void factor(double sigma, int prec = -1) {
    if (prec < 0) prec = precision;
    // the solve's first factorisation may have been made ahead together
    // with other problems' (riga_eigs_batched): the same arithmetic, used
    // as it is when shift and precision match
    Factor& P = cur();
    if (P.pre && P.factored && P.sigma == sigma && P.precision == prec && P.perturbed == 0) {
      P.pre = false;
      P.refactored = 0;
      count_factor(P);
      return;
    }
    P.pre = false;
    auto a = clk::now();
    factor_reserve(pr, cur(), prec, pr->home);
    factor_shift(pr, cur(), sigma, prec, s);
    st.t_fact += secs(a, clk::now());
    count_factor(cur());
  }

  // x = A^{-1} b (FP64), or FP32 solve + FP64 refinement (mixed); FP64
  // solves are refined too once a stall has raised max_ir_fp64
  int ir_steps() { return cur().precision == RIGA_MIXED ? max_ir : max_ir_fp64; }

  // the launches of one application of (K - sigma M)^{-1} (with its
  // refinement steps); counts them when `count`
  void apply_inverse(const double* b, double* out, bool count = true) {
    const Factor& F = cur();
    solve_fb(pr, F, b, out, s);
    const int nir = ir_steps();
    for (int it = 0; it < nir; ++it) {
      // r = b - A x
      launch_spmv(pr, F.av.p, out, ir_r.p, nullptr, s);
      axpy_launch(-1.0, ir_r.p, b, ir_r.p);
      solve_fb(pr, F, ir_r.p, ir_d.p, s);
      axpy_launch(1.0, ir_d.p, out, out);
    }
    if (count) {
      st.n_fb += 1 + nir;
      st.n_mv += nir;
      st.n_ir += nir;
    }
  }

  // One Lanczos step with every quantity that depends on the step index j
  // read from dstep (and dstep advanced at its end): the same launches as
  // step(j), captured once per run into a HIP graph and replayed for each
  // step of it (the basis columns, the locked window, the factorisation and
  // the refinement count are fixed within a run).
  void enqueue_step_dyn(int maxm) {
    launch_copy_col_dyn(rhs.p, Wc(nl), N, dstep.p, s);
    apply_inverse(rhs.p, x.p, false);
    const int m1 = nl + 1 - c_win;
    launch_project(Wc(c_win), Bc(c_win), N, m1, x.p, partial.p, c1.p + c_win, nullptr, nullptr, s, dstep.p,
                   m1 + maxm - 1);
    launch_project(Wc(nl), Bc(nl), N, 1, x.p, partial.p, c2.p + nl, alpha.p, c1.p + nl, s, dstep.p, maxm);
    if (cplx) {
      launch_jrot(x.p, N, 1.0, s);
      launch_project(Wc(nl), Bc(nl), N, 1, x.p, partial.p, c2.p + nl, nullptr, nullptr, s, dstep.p, maxm);
      launch_jrot(x.p, N, -1.0, s);
    }
    launch_spmv(pr, pr->mv.p, x.p, y.p, dotp.p, s);
    launch_scale2(x.p, y.p, dotp.p, spmv_dot_blocks(pr), Bc(nl + 1), Wc(nl + 1), N, beta.p + 1, flag.p, s,
                  dstep.p);
    launch_step_advance(dstep.p, s);
  }

  // The step's launches recorded on a stream of the solver's own (nothing
  // runs during a capture; the graph is launched on the solve's stream).
  void capture_step_graph(int maxm) {
    drop_graph();
    if (!cap) HIPCHECK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    const hipStream_t run_s = s;
    HIPCHECK(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
    s = cap;
    try {
      enqueue_step_dyn(maxm);
    } catch (...) {
      s = run_s;
      (void)hipStreamEndCapture(cap, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    s = run_s;
    HIPCHECK(hipStreamEndCapture(cap, &g));
    const hipError_t e = hipGraphInstantiate(&gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      gexec = nullptr;
      throw Error(RIGA_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
  }

  // the launches of step j, replayed from the run's graph
  void replay_step() {
    HIPCHECK(hipGraphLaunch(gexec, s));
    const int nir = ir_steps();
    st.n_fb += 1 + nir;
    st.n_mv += nir + 1;
    st.n_ir += nir;
  }

  // out = a * u + v
  void axpy_launch(double a, const double* u, const double* v, double* out) {
    launch_axpby(a, u, v, out, N, s);
  }

  // c[c0:m] = W[:, c0:m]^T x ; x -= B[:, c0:m] c[c0:m]; with alpha_out,
  // also *alpha_out = *addend + c[m - 1]
  void project_out(int m, double* c, int c0 = 0, double* alpha_out = nullptr,
                   const double* addend = nullptr) {
    if (m <= c0) return;
    launch_project(Wc(c0), Bc(c0), N, m - c0, x.p, partial.p, c + c0, alpha_out, addend, s);
  }

  // M-normalise x into column j of B (and M x into W); returns false on breakdown
  void normalize_into(int col, double* beta_out) {
    launch_spmv(pr, pr->mv.p, x.p, y.p, dotp.p, s);
    st.n_mv++;
    launch_scale2(x.p, y.p, dotp.p, spmv_dot_blocks(pr), Bc(col), Wc(col), N, beta_out, flag.p, s);
  }

  void start_vector(const double* init /* may be null */) {
    HIPCHECK(hipMemsetAsync(flag.p, 0, 4 * sizeof(int32_t), s));
    if (init) launch_copy(x.p, init, N, s);
    else launch_fill_random(x.p, N, seed, ++run_id, s);
    // against every locked pair, window or not: a start vector with
    // components along the pairs below the window would pass them into the
    // Ritz vectors (inside a multiple eigenvalue's eigenspace no residual
    // shows them), while the steps only keep the Krylov space clear of the
    // pairs near the shift, whose components the operator amplifies
    if (nl > 0) {
      project_out(nl, c1.p);
      project_out(nl, c2.p);
    }
    normalize_into(nl, scal.p + 1);
  }

  // one Lanczos step: column nl+j -> nl+j+1; alpha[j], beta[j+1]
  void step(int j) {
    const int col = nl + j;
    apply_inverse(Wc(col), x.p);
    auto a = clk::now();
    // Classical Gram-Schmidt against [U_locked (window) | V], then a second
    // pass against V only: x = (K - sigma M)^{-1} M v_j starts M-orthogonal
    // to the locked eigenvectors up to rounding and their residuals, so the
    // first pass removes those components without cancellation; the
    // cancellation the second pass repairs comes from the large components
    // along v_j and v_{j-1}.
    project_out(col + 1, c1.p, c_win);
    project_out(col + 1, c2.p, nl, alpha.p + j, c1.p + col);
    if (cplx) {
      // Lanczos on the real-equivalent form is Hermitian Lanczos only while
      // V stays M-orthogonal to J V (in exact arithmetic the recurrence
      // keeps it so: M (K - sigma M)^{-1} M commutes with J, and J is
      // M-skew); rounding lets J V components grow, and the copy J u of a
      // pair locked with u would then converge a second time.  Projecting
      // x against J V is projecting J x against V and rotating back:
      // x - J V (J V)^T M x = J^{-1} (J x - V W^T J x).
      launch_jrot(x.p, N, 1.0, s);
      project_out(col + 1, c2.p, nl);
      launch_jrot(x.p, N, -1.0, s);
    }
    normalize_into(col + 1, beta.p + j + 1);
    st.t_orth += secs(a, clk::now());
  }

  struct Ritz {
    std::vector<double> theta;    // all Ritz values of T_m, ascending
    std::vector<double> est;      // Ritz estimates |beta_{m+1} s_m|
    double beta_m = 0.0;
    int m = 0;
  };

  // Convergence check: eigenvalues of T_m and their Ritz estimates.
  Ritz check(int m) {
    auto a = clk::now();
    Ritz r;
    r.m = m;
    launch_ritz_check(alpha.p, beta.p, m, theta, tdest, flag.p, chk_extra, s);
    // one read-back: theta, estimates, beta_m and the breakdown flag
    std::vector<double> h(chk.n);
    HIPCHECK(hipMemcpyAsync(h.data(), chk.p, chk.n * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    r.theta.assign(h.begin(), h.begin() + m);
    r.est.assign(h.begin() + (mb + 1), h.begin() + (mb + 1) + m);
    r.beta_m = h[2 * (mb + 1)];
    const bool fl = h[2 * (mb + 1) + 1] != 0.0;
    if (fl) {
      r.beta_m = 0.0;
      std::fill(r.est.begin(), r.est.end(), 0.0);
    }
    st.t_proj += secs(a, clk::now());
    return r;
  }

  static bool converged(const Ritz& r, int i) { return r.est[i] <= 1e-10 * std::fabs(r.theta[i]); }

  // Unit eigenvectors of T_m for the Ritz values theta[idx] (idx ascending),
  // returned column by column (m x idx.size()).
  std::vector<double> vectors(const Ritz& r, const std::vector<int>& idx) {
    const int m = r.m, n = (int)idx.size();
    std::vector<double> Sv((size_t)m * n);
    if (n == 0) return Sv;
    std::vector<int32_t> ix(idx.begin(), idx.end());
    // clusters: consecutive selected eigenvalues closer than 1e-3 relative
    // when adjacent in T's spectrum, or closer than 1e-8 relative across
    // unselected ones (copies of a multiple eigenvalue, some not converged
    // and left out, must still be orthogonalised against each other)
    std::vector<int32_t> cl{0};
    for (int i = 1; i < n; ++i) {
      const double t0 = r.theta[idx[i - 1]], t1 = r.theta[idx[i]];
      const double gap = std::fabs(t1 - t0), scale = std::max(std::fabs(t0), std::fabs(t1));
      const bool close = (idx[i] == idx[i - 1] + 1 && gap <= 1e-3 * scale) || gap <= 1e-8 * scale;
      if (!close) cl.push_back(i);
    }
    cl.push_back(n);
    const int ncl = (int)cl.size() - 1;
    ix.insert(ix.end(), cl.begin(), cl.end());
    HIPCHECK(hipMemcpyAsync(sel.p, ix.data(), ix.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    launch_ritz_vectors(alpha.p, beta.p, m, theta, sel.p, sel.p + n, ncl, S.p, s);
    HIPCHECK(hipMemcpyAsync(Sv.data(), S.p, Sv.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    return Sv;
  }

  // Ritz vectors V s_q of the pairs `which` (columns of Sv) plus, if
  // `restart_from` is not empty, the sum of those columns as a restart
  // vector; lock the pairs that pass the residual test.  Returns the number
  // locked.
  // With a thick restart (`thick`: cz = thick->c columns of Z = S_kept Q,
  // m x cz), also V Z and W Z (its M images) into columns nw + 1 .. nw + cz
  // of Ub and MU, and v_{m+1}, M v_{m+1} into column nw + 1 + cz: they are
  // formed before the locked pairs overwrite the basis, and copied into the
  // new basis by the caller.
  int lock_pairs(const Ritz& r, double sigma, const std::vector<double>& Sv,
                 const std::vector<int>& which, const std::vector<int>& restart_from,
                 const std::vector<double>& lam_ritz, bool* have_restart,
                 const std::vector<double>* Z = nullptr, int cz = 0) {
    auto a = clk::now();
    const int m = r.m;
    const int nw = (int)which.size();
    const int nc = nw + (restart_from.empty() ? 0 : 1);
    *have_restart = !restart_from.empty();
    (void)lam_ritz;
    if (cz > 0) {
      // (column nw is the restart vector's, present whenever cz > 0)
      const int z0 = nw + 1;
      HIPCHECK(hipMemcpyAsync(Sh.p + (size_t)z0 * m, Z->data(), (size_t)m * cz * sizeof(double),
                              hipMemcpyHostToDevice, s));
      launch_gemm_nn(Bc(nl), N, m, Sh.p + (size_t)z0 * m, m, cz, Ub.p + (int64_t)z0 * N, s);
      launch_gemm_nn(Wc(nl), N, m, Sh.p + (size_t)z0 * m, m, cz, MU.p + (int64_t)z0 * N, s);
      launch_copy(Ub.p + (int64_t)(z0 + cz) * N, Bc(nl + m), N, s);
      launch_copy(MU.p + (int64_t)(z0 + cz) * N, Wc(nl + m), N, s);
    }
    if (nc == 0) return 0;
    std::vector<double> Sh_h((size_t)m * nc, 0.0);
    for (int i = 0; i < nw; ++i)
      std::memcpy(&Sh_h[(size_t)i * m], &Sv[(size_t)which[i] * m], m * sizeof(double));
    if (!restart_from.empty())
      for (int q : restart_from)
        for (int t = 0; t < m; ++t) Sh_h[(size_t)nw * m + t] += Sv[(size_t)q * m + t];
    HIPCHECK(hipMemcpyAsync(Sh.p, Sh_h.data(), Sh_h.size() * sizeof(double), hipMemcpyHostToDevice, s));
    // U = V S (the restart combination lands in column nw)
    launch_gemm_nn(Bc(nl), N, m, Sh.p, m, nc, Ub.p, s);
    // The candidates are projected once against every locked pair before
    // the residual test.  The steps of this run were projected only against
    // the deflation window, and each FP64 solve leaves components of
    // relative size ~ (its backward error) ||A|| / |lambda_j - sigma| along
    // the eigenvectors below it, which the steps neither amplify nor remove;
    // and a pair locked earlier with a residual near the tolerance carries
    // components of that size along eigenvectors found later.  Either way
    // the locked set would lose M-orthogonality at ~1e-10; one block
    // projection of the candidates (U -= B (W^T U)) keeps it at rounding.
    if (nw > 0 && nl > 0 && (double)N * nl * ((nw + 7) / 8) <= LOCK_PROJECT_MAX) {
      if (bpart.n == 0) bpart.alloc(block_project_partials(N, (int)lam.n), s);
      launch_block_project(W.p, B.p, N, nl, Ub.p, nw, bpart.p, s);
    }
    int nlocked = 0;
    if (nw > 0) {
      launch_spmm_km(pr, Ub.p, nw, KU.p, MU.p, s);
      st.n_mv += 2 * nw;
      const int umax = (int)lam.n;
      double* rqd = res3.p;
      double* rn2 = res3.p + umax;
      double* un2 = res3.p + 2 * (size_t)umax;
      launch_residuals(KU.p, MU.p, Ub.p, N, nw, rqn.p, rqd, rn2, un2, lam.p, rpart.p, s);
      // M-normalise on the device: u /= sqrt(u^T M u), and M u with it
      launch_scale_cols_rsqrt(Ub.p, MU.p, N, nw, rqd, s);
      // one read-back (on the solve's own stream: the null stream would not
      // order it after the kernels, and could wait on unrelated streams)
      std::vector<double> h3(3 * (size_t)umax), h_lam(nw);
      HIPCHECK(hipMemcpyAsync(h3.data(), res3.p, h3.size() * sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHECK(hipMemcpyAsync(h_lam.data(), lam.p, nw * sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHECK(hipStreamSynchronize(s));
      const double* h_rn2 = h3.data() + umax;
      const double* h_un2 = h3.data() + 2 * (size_t)umax;
      // candidates: residual below tol, eigenvalue in [lo, hi); locked in
      // ascending order.  When the locked set is full, a candidate replaces
      // the largest locked eigenvalue above the shift if it is smaller.
      std::vector<int> cand;
      for (int i = 0; i < nw; ++i) {
        const double res = std::sqrt(h_rn2[i]) / (pr->normK1 * std::sqrt(h_un2[i]));
        if (res <= tol && h_lam[i] >= lo && h_lam[i] >= win_lo && h_lam[i] < hi) cand.push_back(i);
        else if (std::getenv("RIGA_LOG_LOCKS"))
          std::fprintf(stderr, "[riga] not locked lambda=%.12g res=%.3e sigma=%.6g\n", h_lam[i], res, sigma);
      }
      std::sort(cand.begin(), cand.end(), [&](int a, int b) { return h_lam[a] < h_lam[b]; });
      if (*have_restart) launch_copy(y.p, Ub.p + (int64_t)nw * N, N, s);
      int appended = 0;
      std::vector<int> dst_col, src_col;  // a column evicted twice keeps the last copy
      std::vector<int> jdst, jsrc;  // J copies (complex pencils)
      for (int i : cand) {
        const double res = std::sqrt(h_rn2[i]) / (pr->normK1 * std::sqrt(h_un2[i]));
        int col = -1;
        if (cplx) {
          // u and J u (same eigenvalue, residual and M-norm; M-orthogonal)
          if (nl + appended + 2 > lock_cap) break;
          col = nl + appended;
          appended += 2;
          locked.push_back(Locked{h_lam[i], res, col, false});
          locked.push_back(Locked{h_lam[i], res, col + 1, true});
          jdst.push_back(col + 1);
          jsrc.push_back(i);
        } else if (nl + appended < lock_cap) {
          col = nl + appended;
          ++appended;
          locked.push_back(Locked{h_lam[i], res, col});
        } else {
          int worst = -1;
          for (int t = 0; t < (int)locked.size(); ++t)
            if (locked[t].lam > sigma && (worst < 0 || locked[t].lam > locked[worst].lam)) worst = t;
          if (worst < 0 || locked[worst].lam <= h_lam[i]) break;
          col = locked[worst].col;
          locked[worst] = Locked{h_lam[i], res, col};
          ++n_evicted;
        }
        if (std::getenv("RIGA_LOG_LOCKS"))
          std::fprintf(stderr, "[riga] lock lambda=%.12g col=%d sigma=%.6g\n", h_lam[i], col, sigma);
        const auto it = std::find(dst_col.begin(), dst_col.end(), col);
        if (it != dst_col.end()) src_col[it - dst_col.begin()] = i;
        else {
          dst_col.push_back(col);
          src_col.push_back(i);
        }
        nlocked += cplx ? 2 : 1;
      }
      launch_copy_cols(dst_col, src_col, N, B.p, Ub.p, W.p, MU.p, s);
      if (!jdst.empty()) launch_copy_cols(jdst, jsrc, N, B.p, Ub.p, W.p, MU.p, s, true);
      nl += appended;

    } else if (*have_restart) {
      launch_copy(y.p, Ub.p, N, s);
      HIPCHECK(hipStreamSynchronize(s));  // Sh_h (pageable) must outlive its upload
    }
    (void)sigma;
    st.t_ritz += secs(a, clk::now());
    return nlocked;
  }

  // Deflation window of the Lanczos steps for runs at sigma when every
  // eigenvalue below `verified` (the previous shift) is locked: the locked
  // pairs above sigma - DEFLATE_SPACINGS (sigma - verified), i.e. those of
  // the last few shift intervals and all above sigma (the clusters that
  // straddle shifts).  A locked pair further down has |1 / (lambda - sigma)|
  // below 1 / DEFLATE_SPACINGS of every missing pair's, so the operator does
  // not amplify its components (the start vector is cleared of all locked
  // pairs); were one to converge, it lies below win_lo and is not locked
  // again.
  void set_window(double sigma, double verified) {
    win_lo = -INFINITY;
    c_win = 0;
    if (!deflate_window_on() || !(sigma > verified)) return;
    win_lo = sigma - DEFLATE_SPACINGS * (sigma - verified);
    c_win = nl;
    for (auto& L : locked)
      if (L.lam >= win_lo) c_win = std::min(c_win, L.col);
  }

  int count_locked(double a, double b) const {
    int c = 0;
    for (auto& L : locked)
      if (L.lam >= a && L.lam < b) ++c;
    return c;
  }

  // One Lanczos run at the current factorisation.  Stops when the
  // converged pairs cover the needs or the basis is full.  Returns the
  // final Ritz data (for shift placement).
  // on_check (optional) sees the Ritz data of every convergence check.
  Ritz run(double sigma, int need_below, int need_above, const double* init, int* n_new,
           const std::function<void(const Ritz&)>& on_check = nullptr) {
    // a run at the shift of a run whose basis filled up continues from its
    // thick-restart basis (columns 0 .. thick_c of V, T's entries uploaded)
    int j = 0;
    if (thick_c > 0 && init == nullptr && sigma == thick_sigma) {
      HIPCHECK(hipMemsetAsync(flag.p, 0, 4 * sizeof(int32_t), s));
      j = thick_c;
      st.n_thick++;
    } else {
      start_vector(init);
    }
    thick_c = 0;
    const int maxm = (int)std::min<int64_t>(mb, N - nl - 1);
    const bool graph = graph_on() && maxm > j;
    if (graph) {
      hstep = j;
      HIPCHECK(hipMemcpyAsync(dstep.p, &hstep, sizeof(int32_t), hipMemcpyHostToDevice, s));
      capture_step_graph(maxm);
    }
    Ritz r;
    int next_check = std::min(maxm, std::max(16, std::min(need_below + need_above, maxm)));
    bool met = false, breakdown = false;
    while (true) {
      if (graph) replay_step();
      else step(j);
      ++j;
      if (j < next_check && j < maxm) continue;
      r = check(j);
      if (on_check) on_check(r);
      // (a converged Ritz value of a complex pencil locks two pairs)
      int cb = 0, ca = 0;
      const int per = cplx ? 2 : 1;
      for (int i = 0; i < j; ++i) {
        if (!converged(r, i)) continue;
        const double l = sigma + 1.0 / r.theta[i];
        if (l < sigma) cb += per; else ca += per;
      }
      breakdown = r.beta_m == 0.0;
      met = cb >= need_below && ca >= need_above;
      if (met || j >= maxm || breakdown) break;
      next_check = std::min(maxm, j + 8);
    }
    st.n_it++;
    // lock every converged pair; restart from the nearest unconverged ones
    std::vector<int> conv, unc;
    for (int i = 0; i < j; ++i) (converged(r, i) ? conv : unc).push_back(i);
    std::sort(unc.begin(), unc.end(), [&](int a, int b) {
      return std::fabs(r.theta[a]) > std::fabs(r.theta[b]);
    });
    // Thick restart (Sec. 4.2, Eq. LanczosRestart) when the basis filled up
    // before the pairs this run is after converged: keep the unconverged
    // Ritz vectors nearest the shift, up to half the basis, and the last
    // Lanczos vector.  (A run that found its pairs but left some missing --
    // further copies of a multiple eigenvalue, which its Krylov space cannot
    // reach -- restarts from a fresh vector instead.)
    std::vector<int> keep;
    if (thick_restart_on() && !met && !breakdown && j >= maxm && unc.size() >= 2) {
      const int c = std::min<int>((int)unc.size() - 1, maxm / 2);
      keep.assign(unc.begin(), unc.begin() + c);
    }
    if (unc.size() > 8) unc.resize(8);
    std::vector<int> idx = conv;
    for (int q : keep)
      if (std::find(unc.begin(), unc.end(), q) == unc.end()) idx.push_back(q);
    idx.insert(idx.end(), unc.begin(), unc.end());
    std::sort(idx.begin(), idx.end());
    auto a = clk::now();
    std::vector<double> Sv = vectors(r, idx);
    st.t_proj += secs(a, clk::now());
    std::vector<int> which, rest, kpos;
    for (size_t q = 0; q < idx.size(); ++q) {
      if (converged(r, idx[q])) which.push_back((int)q);
      else if (std::find(unc.begin(), unc.end(), idx[q]) != unc.end()) rest.push_back((int)q);
    }
    for (int q : keep) kpos.push_back((int)(std::lower_bound(idx.begin(), idx.end(), q) - idx.begin()));
    // the restart basis: Z = S_kept Q (m x c')
    ThickBasis TB;
    std::vector<double> Z;
    if (!keep.empty()) {
      const int m = r.m;
      std::vector<double> th(keep.size()), bb(keep.size());
      for (size_t i = 0; i < keep.size(); ++i) {
        th[i] = r.theta[keep[i]];
        bb[i] = r.beta_m * Sv[(size_t)kpos[i] * m + (m - 1)];
      }
      TB = thick_basis(th, bb);
      Z.assign((size_t)m * TB.c, 0.0);
      for (int q = 0; q < TB.c; ++q)
        for (size_t i = 0; i < keep.size(); ++i) {
          const double w = TB.Q[(size_t)q * keep.size() + i];
          const double* sv = &Sv[(size_t)kpos[i] * m];
          double* z = &Z[(size_t)q * m];
          for (int t = 0; t < m; ++t) z[t] += w * sv[t];
        }
      if (rest.empty()) TB.c = 0;  // (unreachable: keep is a superset of rest)
    }
    bool have_restart = false;
    *n_new = lock_pairs(r, sigma, Sv, which, rest, r.theta, &have_restart, TB.c > 0 ? &Z : nullptr, TB.c);
    restart_valid = have_restart && r.beta_m != 0.0;
    if (TB.c > 0) {
      // V := [V Z, v_{m+1}] after the locked columns, T's leading block
      // := the re-tridiagonalised arrowhead
      const int cz = TB.c, z0 = (int)which.size() + 1;
      std::vector<int> dst, src;
      for (int q = 0; q <= cz; ++q) {
        dst.push_back(nl + q);
        src.push_back(z0 + q);
      }
      launch_copy_cols(dst, src, N, B.p, Ub.p, W.p, MU.p, s);
      HIPCHECK(hipMemcpyAsync(alpha.p, TB.alpha.data(), cz * sizeof(double), hipMemcpyHostToDevice, s));
      HIPCHECK(hipMemcpyAsync(beta.p, TB.beta.data(), (cz + 1) * sizeof(double), hipMemcpyHostToDevice, s));
      HIPCHECK(hipStreamSynchronize(s));  // the host arrays must outlive their uploads
      thick_c = cz;
      thick_sigma = sigma;
    }
    if (log_on())
      std::fprintf(stderr, "[riga] run sigma=%.6g steps=%d need=(%d,%d) converged=%zu locked=%d total_locked=%d "
                   "window=[%.6g, from column %d]\n",
                   sigma, j, need_below, need_above, which.size(), *n_new, nl, win_lo, c_win);
    return r;
  }
  bool restart_valid = false;
  // thick-restart basis for the next run at thick_sigma: columns 0 .. thick_c
  // of V (0 when there is none)
  int thick_c = 0;
  double thick_sigma = 0.0;
};


// Moves cand to the middle of the gap between estimated eigenvalues above
// top that contains it (estimates: the locked values and the Ritz values of
// run r, made at shift sigma); clamps to hi.
// Increase of lambda above `top` (n eigenvalues below it) that adds `add`
// eigenvalues, with the count growing like lambda^{dim/2} (Weyl's law for
// second-order operators); 0 when top or n is not positive.
double weyl_step(double top, int64_t n, int add, int dim) {
  if (!(top > 0) || n <= 0) return 0.0;
  return top * (std::pow((double)(n + add) / (double)n, 2.0 / dim) - 1.0);
}

double place_in_gap(const Solver& sv, const Solver::Ritz& r, double sigma, double top, double cand,
                    double step, double hi) {
  std::vector<double> est;
  for (auto& L : sv.locked) est.push_back(L.lam);
  for (int i = 0; i < (int)r.theta.size(); ++i)
    if (r.theta[i] != 0.0) est.push_back(sigma + 1.0 / r.theta[i]);
  std::sort(est.begin(), est.end());
  // the gap containing cand (estimates above top only)
  double below = top, above = std::numeric_limits<double>::infinity();
  for (double e : est) {
    if (e <= top) continue;
    if (e <= cand) below = std::max(below, e);
    else { above = std::min(above, e); }
  }
  if (std::isfinite(above)) {
    // a wide gap (estimates missing, e.g. copies of a multiple eigenvalue
    // that the last Krylov space did not resolve) is not crossed: cand only
    // keeps half a step from its lower end
    if (above - below <= 2.0 * step) cand = 0.5 * (below + above);
    else cand = std::min(std::max(cand, below + 0.5 * step), above - 0.5 * step);
  } else if (below > top) {
    cand = std::max(cand, below + 0.5 * step);
  }
  if (std::isfinite(hi) && cand >= hi) cand = hi;
  return cand;
}


// Places the next shift above the eigenvalues locked so far: far enough
// that the new slice holds about `target` eigenvalues (the count below the
// top locked eigenvalue extrapolated with Weyl's law, linearly in 2D), then
// moved into the nearest gap between estimated eigenvalues so that
// K - sigma M stays well conditioned (the paper gives no rule for choosing
// shifts; Sec. 4.1).
double next_shift(const Solver& sv, const Solver::Ritz& r, double sigma, double lo, double hi,
                  int target) {
  double top = sigma;
  int cnt = 0;
  for (auto& L : sv.locked)
    if (L.lam >= lo && L.lam < hi) {
      top = std::max(top, L.lam);
      ++cnt;
    }
  double step = weyl_step(top, sv.nu_lo + cnt, target, sv.dim);
  if (!(step > 0)) {
    const double width = top - lo;
    step = (cnt > 0 && width > 0) ? target * width / cnt : std::max(std::fabs(top), 1.0) * 0.5;
  }
  return place_in_gap(sv, r, sigma, top, top + step, step, hi);
}

// Once at least nev pairs of the slice are locked, a shift just above the
// nev-th lowest of them, v, verifies them by inertia alone: with nothing
// missing below it, it needs no run.  The shift goes to the middle of the
// gap above v to the next estimate (a locked value or a Ritz value of run r,
// made at shift r_sigma), gaps narrower than a relative 1e-4 (copies of a
// multiple eigenvalue) skipped, and at most half of Weyl's spacing for one
// more eigenvalue above the gap's lower end.  NaN when fewer are locked or
// the shift would leave (sigma, hi).
double verify_shift(const Solver& sv, const Solver::Ritz& r, double r_sigma, double lo, double hi,
                    int nev, double sigma) {
  const double none = std::numeric_limits<double>::quiet_NaN();
  std::vector<double> lk;
  for (auto& L : sv.locked)
    if (L.lam >= lo && L.lam < hi) lk.push_back(L.lam);
  if (nev < 1 || (int)lk.size() < nev) return none;
  std::sort(lk.begin(), lk.end());
  const double v = lk[nev - 1];
  std::vector<double> est(lk.begin() + (nev - 1), lk.end());
  for (int i = 0; i < (int)r.theta.size(); ++i)
    if (r.theta[i] != 0.0) {
      const double e = r_sigma + 1.0 / r.theta[i];
      if (e > v) est.push_back(e);
    }
  std::sort(est.begin(), est.end());
  for (size_t i = 1; i < est.size(); ++i) {
    const double a = est[i - 1], b = est[i];
    if (b - a < 1e-4 * std::fabs(a)) continue;
    double cand = 0.5 * (a + b);
    const double space = weyl_step(a, sv.nu_lo + nev + (int64_t)(i - 1), 1, sv.dim);
    if (space > 0) cand = std::min(cand, a + 0.5 * space);
    if (!(cand > sigma) || (std::isfinite(hi) && cand >= hi)) return none;
    return cand;
  }
  return none;
}

// Look-ahead guess of the shift that next_shift will choose once the runs at
// sigma have finished, made before they start: those runs lock about
// `per_above` eigenvalues above sigma, so the top of the locked set moves to
// about sigma + per_above / density; the guess lies `target` eigenvalues
// beyond, in a gap of the estimates known now (locked values and the Ritz
// values of the last run, made at shift r_sigma).  Returns NaN when the
// locked set gives no density yet.
double predict_shift(const Solver& sv, const Solver::Ritz& r, double r_sigma, double sigma,
                     double lo, double hi, int per_above, int target) {
  double top = sigma;
  int cnt = 0;
  for (auto& L : sv.locked)
    if (L.lam >= lo && L.lam < hi) {
      top = std::max(top, L.lam);
      ++cnt;
    }
  if (cnt == 0 || !(top > lo)) return std::numeric_limits<double>::quiet_NaN();
  int64_t n_top = sv.nu_lo + cnt;
  // pairs locked above sigma already count towards the runs' target
  const int64_t n_sigma = sv.nu_lo + sv.count_locked(lo, sigma);
  if (sv.count_locked(sigma, hi) < per_above && n_sigma + per_above > n_top) {
    const double up = weyl_step(sigma, n_sigma, per_above, sv.dim);
    if (!(up > 0)) return std::numeric_limits<double>::quiet_NaN();
    top = std::max(top, sigma + up);
    n_top = n_sigma + per_above;
  }
  const double step = weyl_step(top, n_top, target, sv.dim);
  if (!(step > 0)) return std::numeric_limits<double>::quiet_NaN();
  return place_in_gap(sv, r, r_sigma, top, top + step, step, hi);
}

// The same guess made during the first run at the lowest shift, before
// anything is locked: the converged Ritz values of a convergence check
// stand in for the locked eigenvalues.  NaN while fewer than 8 have
// converged.
double predict_from_ritz(const Solver& sv, const Solver::Ritz& r, double sigma, double lo, double hi,
                         int per_above, int target, int dim) {
  int cnt = 0, above = 0;
  double top = sigma;
  for (int i = 0; i < (int)r.theta.size(); ++i) {
    if (r.theta[i] == 0.0 || !Solver::converged(r, i)) continue;
    const double l = sigma + 1.0 / r.theta[i];
    if (l < lo || l >= hi) continue;
    ++cnt;
    if (l >= sigma) ++above;
    top = std::max(top, l);
  }
  if (cnt < 8 || !(top > lo)) return std::numeric_limits<double>::quiet_NaN();
  const int add = std::max(0, per_above - above) + target;
  const double step = weyl_step(top, sv.nu_lo + cnt, add, dim);
  if (!(step > 0)) return std::numeric_limits<double>::quiet_NaN();
  return place_in_gap(sv, r, sigma, top, top + step, step, hi);
}

// A factorisation at a predicted shift made on a second host thread and
// stream into the spare Factor, while the Lanczos runs at the current shift
// use the other one.  The destructor waits for it, so no exit path leaves
// the thread writing into the problem.
struct LookAhead {
  riga_problem* pr = nullptr;
  SolveCtx* ctx = nullptr;
  hipStream_t s2 = nullptr;
  std::thread th;
  bool active = false;
  double sigma = 0.0;
  std::string err;
  riga_status code = RIGA_OK;

  ~LookAhead() {
    if (th.joinable()) th.join();
    if (s2) (void)hipStreamDestroy(s2);
  }

  Factor& spare() { return ctx->spare(); }

  // s: the stream of the Lanczos runs, whose work on the spare Factor (if
  // it was the current one before) must be finished before it is reused
  void start(double sig, int precision, hipStream_t s) {
    factor_reserve(pr, spare(), precision, pr->home);
    HIPCHECK(hipStreamSynchronize(s));
    if (!s2) HIPCHECK(hipStreamCreateWithFlags(&s2, hipStreamNonBlocking));
    sigma = sig;
    err.clear();
    code = RIGA_OK;
    active = true;
    const int dev = pr->device;
    th = std::thread([this, dev, precision] {
      try {
        HIPCHECK(hipSetDevice(dev));
        factor_shift(pr, spare(), sigma, precision, s2);
      } catch (const Error& e) {
        code = e.code;
        err = e.what();
      } catch (const std::exception& e) {
        code = RIGA_EDEVICE;
        err = e.what();
      }
    });
  }

  // waits for the factorisation; rethrows its error.  Afterwards `sigma`
  // is the shift used (moved down if the guess was singular).
  void join() {
    if (th.joinable()) th.join();
    active = false;
    if (code != RIGA_OK) throw Error(code, "look-ahead factorisation: " + err);
    sigma = spare().sigma;
  }
};

// RIGA_LOOKAHEAD=0 factorises every shift in place, after its runs.
bool lookahead_on() {
  static const bool on = [] {
    const char* v = std::getenv("RIGA_LOOKAHEAD");
    return !(v && *v == '0');
  }();
  return on;
}

}  // namespace

namespace {

// One slice of the spectrum: the nev lowest eigenpairs in [lo, hi) found by
// shift-and-invert Lanczos with spectrum slicing (Sec. 4.1) on its own
// Solver (basis storage, stream, factorisations).  `nu_base` >= 0 makes the
// slice find nev - (nu(lo) - nu_base) pairs instead (the pairs of a lower
// slice ending at lo are counted by the inertia at lo).  `after_lo`, if
// set, runs once the inertia at lo is known and may lower hi (the split of
// run_eigs: the rest goes to another slice).  A finite `first_shift` above
// lo makes the first runs start there, inside the slice, rather than at lo.
struct Slice {
  Solver sv;
  double lo = 0.0, hi = 0.0;
  int nev = 0;
  int64_t nu_base = -1;
  double first_shift = std::numeric_limits<double>::quiet_NaN();
  riga_status status = RIGA_OK;
  double verified = 0.0;
  bool requested_ends = true;  // lo and a finite hi are the request's (not a split point)
  bool serial_first = false;   // factorise the first shift after lo, not beside it (memory)
  bool count_hi_first = true;  // a finite hi is counted before the runs (else reached by the shifts)
  std::function<void(Slice&)> after_lo;
};

void setup_solver(Solver& sv, riga_problem* pr, SolveCtx* ctx, const riga_eigs_opts* o, hipStream_t s,
                  int nev_cap) {
  sv.pr = pr;
  sv.ctx = ctx;
  sv.s = s;
  sv.N = pr->an.N;
  sv.t0 = clk::now();
  sv.tol = o->tol > 0 ? o->tol : 1e-9;
  sv.seed = o->seed;
  sv.precision = o->precision;
  sv.max_ir = 2;
  if (const char* v = std::getenv("RIGA_MAX_IR")) sv.max_ir = std::max(0, std::atoi(v));
  // RIGA_FP64_IR=n refines every FP64 solve n times from the start (the
  // refinement a stall switches on; n at most MAX_IR_FP64)
  if (const char* v = std::getenv("RIGA_FP64_IR"))
    sv.max_ir_fp64 = std::min(MAX_IR_FP64, std::max(0, std::atoi(v)));
  sv.per_shift = o->per_shift > 0 ? o->per_shift : 32;
  sv.max_restarts = o->max_restarts > 0 ? o->max_restarts : 10;
  int mb = o->max_basis > 0 ? o->max_basis : std::max(160, 4 * sv.per_shift + 32);
  mb = (int)std::min<int64_t>(std::min(mb, 1000), sv.N - 1);
  sv.mb = mb;
  sv.lock_cap = (int)std::min<int64_t>(nev_cap + 2 * sv.per_shift + 32, sv.N);
  sv.dim = pr->an.dim;
  sv.cplx = pr->an.components == 2;
  sv.alloc();
}

void run_slice(Slice& S) {
  Solver& sv = S.sv;
  riga_problem* pr = sv.pr;
  // the ends in use: moved down when a factorisation there is singular
  double lo = S.lo, hi = S.hi;
  int nev = S.nev;
  LookAhead la;
  la.pr = pr;
  la.ctx = sv.ctx;
  // an open-ended slice with a first shift inside it factorises there on
  // the look-ahead stream while the factorisation at lo proceeds
  const bool first_ahead = lookahead_on() && !S.serial_first && (!std::isfinite(hi) || !S.count_hi_first) &&
                           !S.after_lo &&
                           std::isfinite(S.first_shift) && S.first_shift > lo;
  if (first_ahead) la.start(S.first_shift, sv.precision, sv.s);
  // the counts at the ends decide which eigenvalues the slice returns: in
  // mixed precision a nonzero end of the request is factorised in FP64, as
  // an FP32 count cannot resolve an eigenvalue within the end's offset (K is
  // positive definite, so an end at 0 has no eigenvalue near it).  The
  // split point between two slices is counted in the solver's precision by
  // both, so that the two counts there agree.
  auto end_prec = [&](double x) {
    return (x == 0.0 || !S.requested_ends) ? sv.precision : (int)RIGA_FP64;
  };
  int64_t nu_lo = 0;
  if (std::isfinite(hi) && S.count_hi_first) {
    sv.factor(hi, end_prec(hi));
    hi = sv.cur().sigma;
    const int64_t nu_hi = sv.cur().inertia;
    sv.factor(lo, end_prec(lo));
    lo = std::min(sv.cur().sigma, hi);
    nu_lo = sv.cur().inertia;
    nev = (int)std::min<int64_t>(nev, std::max<int64_t>(0, nu_hi - nu_lo));
  } else {
    sv.factor(lo, end_prec(lo));
    lo = sv.cur().sigma;
    nu_lo = sv.cur().inertia;
  }
  S.lo = lo;
  S.hi = hi;
  sv.lo = lo;
  sv.hi = hi;
  if (S.nu_base >= 0) nev = (int)std::max<int64_t>(0, nev - (nu_lo - S.nu_base));
  S.nev = nev;
  sv.nu_lo = nu_lo;
  sv.st.n_shift = 1;
  double hi_now = hi;  // the split may lower it
  if (S.after_lo) {
    S.after_lo(S);
    hi_now = S.hi;
    sv.hi = hi_now;
  }
  riga_status status = RIGA_OK;
  double sigma = lo;
  int64_t known = 0;  // eigenvalues in [lo, sigma)
  // a first shift inside the slice locks pairs on both of its sides; one
  // that turns out to lie past more eigenvalues than a run is sized for
  // (a poor estimate) is given up for lo
  bool inside = false;
  if (la.active) {
    auto a = clk::now();
    la.join();
    sv.st.t_fact += secs(a, clk::now());
    sv.count_factor(la.spare());
  }
  if (nev > 0 && std::isfinite(S.first_shift) && S.first_shift > lo && S.first_shift < hi_now) {
    int64_t k = 0;
    double fs = S.first_shift;
    if (first_ahead) {
      // the factorisation at lo stays current if the first shift is given up
      fs = la.sigma;
      k = la.spare().inertia - nu_lo;
      if (k <= sv.per_shift) sv.ctx->cur = 1 - sv.ctx->cur;
    } else {
      sv.factor(S.first_shift);
      fs = sv.cur().sigma;
      k = sv.cur().inertia - nu_lo;
      if (k > sv.per_shift) {
        sv.factor(lo);
        sv.st.n_shift++;
      }
    }
    sv.st.n_shift++;
    if (k <= sv.per_shift && fs > lo) {
      sigma = fs;
      known = k;
      inside = true;
    } else if (first_ahead && k <= sv.per_shift) {
      sv.ctx->cur = 1 - sv.ctx->cur;  // moved below lo: keep the factorisation at lo
    }
    if (log_on())
      std::fprintf(stderr, "[riga] first shift %.10g: count above lo=%lld (%s)\n", S.first_shift,
                   (long long)k, inside ? "kept" : "given up");
  }
  double verified = lo;  // every eigenvalue in [lo, verified) is locked
  const double* init = nullptr;
  Solver::Ritz last;        // final Ritz data of the last run
  double last_sigma = sigma;  // its shift
  for (int shift = 0; nev > 0 && shift < 400; ++shift) {
    int runs = 0;
    const int per_above = (shift == 0 && !inside) ? sv.per_shift : std::max(1, sv.per_shift / 2);
    const int64_t target = std::max<int64_t>(1, std::min<int64_t>(sv.per_shift / 2, nev - known));
    // factorise at the guessed next shift while the runs at this one proceed
    if (lookahead_on() && shift > 0 && known < nev && !(std::isfinite(hi_now) && sigma >= hi_now)) {
      const double guess = predict_shift(sv, last, last_sigma, sigma, lo, hi_now, per_above, (int)target);
      if (std::isfinite(guess) && guess > sigma) la.start(guess, sv.precision, sv.s);
    }
    do {
      const int below = sv.count_locked(lo, sigma);
      const int need_below = (int)std::max<int64_t>(0, known - below);
      const int above = sv.count_locked(sigma, hi_now);
      // none above the slice's upper end (a split slice's last shift)
      const int need_above = (std::isfinite(hi_now) && sigma >= hi_now)
                                 ? 0
                                 : (int)std::max<int64_t>(
                                       0, std::min<int64_t>(per_above, nev - known - above));
      // a shift with every eigenvalue below it locked and enough locked
      // above (a split slice's last shift, a verifying shift) needs no run
      if (need_below == 0 && need_above == 0) break;
      int n_new = 0;
      // a repeated run at the same shift means eigenvalues are missing that
      // the previous Krylov space did not reach (e.g. further copies of a
      // multiple eigenvalue): start it from a fresh random vector.  At the
      // lowest shift the look-ahead starts from the first run's convergence
      // checks
      std::function<void(const Solver::Ritz&)> hook;
      if (shift == 0 && lookahead_on() && !la.active && !(std::isfinite(hi_now) && sigma >= hi_now))
        hook = [&](const Solver::Ritz& r) {
          if (la.active) return;
          const double guess =
              predict_from_ritz(sv, r, sigma, lo, hi_now, per_above, (int)target, pr->an.dim);
          if (std::isfinite(guess) && guess > sigma) la.start(guess, sv.precision, sv.s);
        };
      sv.set_window(sigma, verified);
      last = sv.run(sigma, need_below, need_above, runs == 0 ? init : nullptr, &n_new, hook);
      // A run that locks under an eighth of what is missing, or a repeated
      // run at this shift that locks none of the pairs missing below it, has
      // reached the accuracy the solve allows: the Ritz values converge but
      // their FP64 residuals stay above the tolerance (an FP32 factor, or an
      // FP64 one of an ill-conditioned K - sigma M).  Refine the solves more
      // from here on.
      // (a run continued by a thick restart ran out of basis, not accuracy)
      const bool stalled = sv.thick_c == 0 &&
                           (8 * n_new < need_below + need_above ||
                            (runs >= 1 && need_below > 0 && sv.count_locked(lo, sigma) == below));
      if (stalled) {
        if (sv.precision == RIGA_MIXED && sv.max_ir < MAX_IR_ESCALATED) {
          sv.max_ir = std::min(MAX_IR_ESCALATED, std::max(1, 2 * sv.max_ir));
          if (log_on()) std::fprintf(stderr, "[riga] refinement steps raised to %d\n", sv.max_ir);
        } else if (sv.precision != RIGA_MIXED && sv.max_ir_fp64 < MAX_IR_FP64) {
          ++sv.max_ir_fp64;
          if (log_on()) std::fprintf(stderr, "[riga] FP64 refinement steps raised to %d\n", sv.max_ir_fp64);
        }
      }
      last_sigma = sigma;
      init = sv.restart_valid ? sv.y.p : nullptr;
      ++runs;
    } while (sv.count_locked(lo, sigma) < known && runs < sv.max_restarts);
    if (sv.count_locked(lo, sigma) < known) {
      status = RIGA_ENOCONV;
      break;
    }
    verified = sigma;
    if (known >= nev) break;
    if (std::isfinite(hi_now) && sigma >= hi_now) break;
    double next = next_shift(sv, last, sigma, lo, hi_now, (int)target);
    const double check = verify_shift(sv, last, last_sigma, lo, hi_now, nev, sigma);
    const bool verify = std::isfinite(check);
    if (verify) next = check;
    bool taken = false;
    if (la.active) {
      // the look-ahead factorisation replaces the one at `next` when it
      // moves past this shift and leaves no more eigenvalues below it to
      // find than one run is sized for
      auto a = clk::now();
      la.join();
      sv.st.t_fact += secs(a, clk::now());
      const Factor& F = la.spare();
      sv.count_factor(F);
      const int64_t known_g = F.inertia - nu_lo;
      const int64_t missing = known_g - sv.count_locked(lo, la.sigma);
      // (a verifying shift is preferred unless this one verifies as well)
      taken = la.sigma > sigma && known_g > known && missing <= sv.per_shift &&
              !(std::isfinite(hi_now) && la.sigma > hi_now) && (!verify || (missing == 0 && known_g >= nev));
      if (log_on())
        std::fprintf(stderr, "[riga] look-ahead sigma=%.10g (placed after the runs: %.10g): %s\n",
                     la.sigma, next, taken ? "taken" : "discarded");
      if (taken) {
        sv.ctx->cur = 1 - sv.ctx->cur;
        next = la.sigma;
      }
    }
    if (!taken) {
      sv.factor(next);
      next = sv.cur().sigma;
    }
    sv.st.n_shift++;
    known = sv.cur().inertia - nu_lo;
    if (log_on())
      std::fprintf(stderr, "[riga] shift %d: sigma=%.10g count below=%lld locked below=%d\n",
                   shift + 1, next, (long long)known, sv.count_locked(lo, next));
    if (sv.count_locked(lo, next) > known) {
      status = RIGA_ENOCONV;  // more pairs locked than exist: inconsistent
      break;
    }
    sigma = next;
  }
  S.status = status;
  S.verified = verified;
}

// The slice's pairs to return: those in [lo, hi) (only below the last
// verified shift if the budget ran out), ascending, at most its nev.
std::vector<Locked> slice_pairs(const Slice& S) {
  const double top = S.status == RIGA_OK ? S.hi : std::min(S.hi, S.verified);
  std::vector<Locked> in;
  for (auto& L : S.sv.locked)
    if (L.lam >= S.lo && L.lam < top) in.push_back(L);
  std::sort(in.begin(), in.end(), [](const Locked& a, const Locked& b) { return a.lam < b.lam; });
  if ((int)in.size() > S.nev) in.resize(S.nev);
  return in;
}

void add_stats(riga_stats& a, const riga_stats& b) {
  a.n_shift += b.n_shift;
  a.n_fact += b.n_fact;
  a.n_fb += b.n_fb;
  a.n_mv += b.n_mv;
  a.n_it += b.n_it;
  a.n_ir += b.n_ir;
  a.n_perturbed_pivots += b.n_perturbed_pivots;
  a.n_2x2_pivots += b.n_2x2_pivots;
  a.n_thick += b.n_thick;
  a.t_fact += b.t_fact;
  a.t_fb += b.t_fb;
  a.t_mv += b.t_mv;
  a.t_orth += b.t_orth;
  a.t_proj += b.t_proj;
  a.t_ritz += b.t_ritz;
}

// Estimates of the `count` lowest eigenvalues made before any shift: those
// of the Dirichlet Laplacian on the unit square or cube (pi^2 times sums of
// squared integers) divided by the mean of (rho/kappa)^(dim/2) to the power
// 2/dim, the factor by which variable coefficients scale the leading term of
// Weyl's law for -div(kappa grad u) = lambda rho u.
std::vector<double> spectrum_estimates(riga_problem* pr, int count, hipStream_t s) {
  const int64_t ne = pr->an.n_elem;
  const int dim = pr->an.dim;
  std::vector<double> kap(pr->kappa.p ? ne : 0), rho(pr->rho.p ? ne : 0);
  if (!kap.empty())
    HIPCHECK(hipMemcpyAsync(kap.data(), pr->kappa.p, ne * sizeof(double), hipMemcpyDeviceToHost, s));
  if (!rho.empty())
    HIPCHECK(hipMemcpyAsync(rho.data(), pr->rho.p, ne * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  double acc = 0.0;
  for (int64_t e = 0; e < ne; ++e) {
    const double q = (rho.empty() ? 1.0 : rho[e]) / (kap.empty() ? 1.0 : kap[e]);
    acc += std::pow(q, 0.5 * dim);
  }
  const double scale = std::pow(acc / (double)ne, 2.0 / dim);
  std::vector<double> est(count);
  exact_eigenvalues(dim, count, est.data());
  for (double& v : est) v /= scale;
  return est;
}

// Spectrum slices of an open-ended request (RIGA_SLICES=n, at most
// MAX_SLICES; default 2): every slice gets at least two runs' worth of pairs.
int slices_wanted() {
  const char* v = std::getenv("RIGA_SLICES");
  if (v && *v) return std::max(1, std::min(MAX_SLICES, std::atoi(v)));
  return 2;
}

}  // namespace

riga_status run_eigs(riga_problem* pr, const riga_eigs_opts* o, int32_t* n_found, double* evals,
                     double* evecs, double* resid, riga_stats* stats_out) {
  const hipStream_t s = o->stream ? (hipStream_t)o->stream : pr->home;
  StreamBind bind(pr, s);
  const auto t0 = clk::now();
  *n_found = 0;
  // slices[0] runs on this thread and stream; slices[i > 0] each on a host
  // thread, HIP stream and solve context of their own.  Destruction order:
  // the threads are joined first, the slices' buffers are freed next, their
  // streams are destroyed last.
  std::vector<hipStream_t> streams;
  struct StreamGuard {
    std::vector<hipStream_t>& st;
    ~StreamGuard() {
      for (hipStream_t x : st)
        if (x) (void)hipStreamDestroy(x);
    }
  } stream_guard{streams};
  std::vector<std::unique_ptr<Slice>> slices;
  slices.emplace_back(new Slice);
  std::vector<std::string> errs(MAX_SLICES);
  std::vector<riga_status> codes(MAX_SLICES, RIGA_OK);
  std::vector<std::thread> threads;
  struct Joiner {
    std::vector<std::thread>& t;
    ~Joiner() {
      for (auto& x : t)
        if (x.joinable()) x.join();
    }
  } joiner{threads};
  Slice& A = *slices[0];
  // a complex pencil's eigenvalues are double in its real-equivalent form:
  // the slice counts and locks pairs of the real system (u and J u)
  const int comp = pr->an.components;
  setup_solver(A.sv, pr, &pr->ctx[0], o, s, o->nev * comp);
  A.lo = o->lo - END_SHIFT * std::fabs(o->lo);
  A.hi = std::isfinite(o->hi) ? o->hi - END_SHIFT * std::fabs(o->hi) : o->hi;
  if (!(A.hi > A.lo)) {
    A.lo = o->lo;
    A.hi = o->hi;
  }
  A.nev = o->nev * comp;
  const int per_shift = o->per_shift > 0 ? o->per_shift : 32;
  const int nsl = (std::isfinite(o->hi) || comp > 1)
                      ? 1
                      : std::max(1, std::min(slices_wanted(), o->nev / (2 * per_shift)));
  if (nsl > 1) {
    A.after_lo = [&](Slice& a) {
      // split where the estimates put equal shares of the pairs; each later
      // slice's first runs start half a run's worth of pairs above its lower
      // end, so that they lock pairs on both sides of their shift
      Solver& sv = a.sv;
      const int w = std::max(2, per_shift / 8);
      const int64_t t_last = sv.nu_lo + (int64_t)a.nev * (nsl - 1) / nsl + per_shift / 2;
      if (t_last + w + 1 > (int64_t)1 << 22) return;
      const std::vector<double> est = spectrum_estimates(pr, (int)(t_last + w + 1), s);
      // the middle of the widest gap between neighbouring estimates around
      // index c (the count of estimates below it lies within c -/+ w)
      auto gap_mid = [&](int64_t c) {
        int64_t best = std::max<int64_t>(1, c - w);
        for (int64_t i = best + 1; i <= c + w; ++i)
          if (est[i] - est[i - 1] > est[best] - est[best - 1]) best = i;
        return 0.5 * (est[best] + est[best - 1]);
      };
      std::vector<double> b(nsl), s1(nsl);
      b[0] = a.lo;
      for (int i = 1; i < nsl; ++i) {
        const int64_t t = sv.nu_lo + (int64_t)a.nev * i / nsl;
        b[i] = gap_mid(t);
        s1[i] = gap_mid(t + per_shift / 2);
        if (!(b[i] > b[i - 1]) || !(s1[i] > b[i]) || !std::isfinite(s1[i])) return;
      }
      for (int i = 1; i + 1 < nsl; ++i)
        if (!(s1[i] < b[i + 1])) return;
      // every later slice brings its own Lanczos storage (room for all nev
      // pairs: how many lie in it is not known yet) and two more
      // factorisations: split only when the device holds them with room to
      // spare (fewer slices are the same computation, serial)
      const int cap_b = o->nev;
      const double n = (double)sv.N;
      const double cols = (double)std::min<int64_t>(cap_b + 2 * sv.per_shift + 32, sv.N) + sv.mb + 1;
      const double umax = (double)sv.mb + 1.0;
      const Analysis& an = pr->an;
      const TopDev& td = pr->top;
      const double fact = (double)an.h_size + (double)td.e_row + (double)td.e_col + (double)td.e_cb +
                          4.0 * (double)n + (double)pr->kv.n;
      // (a further factorisation's worth of margin per slice: the first
      // slice's look-ahead factorisation may not be allocated yet.  The
      // front pool is per slice, shared by its factorisations, plus a
      // second one while its first two factorisations overlap.)
      const double need = 8.0 * (nsl - 1) * (2.0 * n * cols + 3.0 * n * umax + 3.0 * fact +
                                             2.0 * (double)an.pool_size);
      // without the overlap of a slice's first two factorisations, one
      // pool per slice
      const double need_serial = need - 8.0 * (nsl - 1) * (double)an.pool_size;
      size_t free_b = 0, total_b = 0;
      HIPCHECK(hipMemGetInfo(&free_b, &total_b));
      bool serial_first = false;
      if (need * 1.15 > (double)free_b) {
        if (need_serial * 1.15 > (double)free_b) {
          if (log_on())
            std::fprintf(stderr, "[riga] no split: %d more slices need %.1f GB, %.1f GB free\n", nsl - 1,
                         need_serial * 1e-9, (double)free_b * 1e-9);
          return;
        }
        serial_first = true;
      }
      a.hi = b[1];
      const int dev = pr->device;
      for (int i = 1; i < nsl; ++i) {
        hipStream_t si = nullptr;
        HIPCHECK(hipStreamCreateWithFlags(&si, hipStreamNonBlocking));
        streams.push_back(si);
        slices.emplace_back(new Slice);
        Slice& S = *slices.back();
        S.lo = b[i];
        S.hi = i + 1 < nsl ? b[i + 1] : o->hi;
        S.requested_ends = false;
        S.count_hi_first = false;
        S.serial_first = serial_first;
        S.nev = o->nev;
        S.nu_base = i + 1 < nsl ? -1 : sv.nu_lo;
        S.first_shift = s1[i];
        if (log_on())
          std::fprintf(stderr, "[riga] slice %d: [%.10g, %.10g), first shift %.10g\n", i, S.lo, S.hi, s1[i]);
      }
      for (int i = 1; i < nsl; ++i) {
        Slice* S = slices[i].get();
        hipStream_t si = streams[i - 1];
        threads.emplace_back([&, S, si, i, dev, cap_b] {
          try {
            HIPCHECK(hipSetDevice(dev));
            setup_solver(S->sv, pr, &pr->ctx[i], o, si, cap_b);
            run_slice(*S);
          } catch (const Error& e) {
            codes[i] = e.code;
            errs[i] = e.what();
          } catch (const std::exception& e) {
            codes[i] = RIGA_EDEVICE;
            errs[i] = e.what();
          }
        });
      }
    };
  }
  run_slice(A);
  for (auto& t : threads)
    if (t.joinable()) t.join();
  for (int i = 1; i < (int)slices.size(); ++i)
    if (codes[i] != RIGA_OK) throw Error(codes[i], "spectrum slice " + std::to_string(i) + ": " + errs[i]);
  // Slices lock their pairs without seeing each other's: a pair's overlap
  // with an eigenvector of another slice is bounded only by its residual
  // over the gap (at the 1e-9 tolerance, up to a few 1e-10 in 3D).  One
  // block Gram-Schmidt pass of each slice's locked vectors against every
  // lower slice's (their intervals are disjoint) brings that overlap to
  // rounding level; it changes the residuals at the level of the removed
  // overlap times the gap, within the tolerance.
  if (evecs && slices.size() > 1) {
    for (auto si : streams) HIPCHECK(hipStreamSynchronize(si));
    const int64_t n = A.sv.N;
    constexpr int CROSS_COLS = 128;
    DBuf<double> part;
    part.alloc(block_project_partials(n, CROSS_COLS), s);
    for (size_t i = 1; i < slices.size(); ++i) {
      Solver& cur = slices[i]->sv;
      for (size_t k = 0; k < i; ++k) {
        const Solver& low = slices[k]->sv;
        for (int a = 0; a < cur.nl; a += CROSS_COLS)
          launch_block_project(low.W.p, low.B.p, n, low.nl, cur.B.p + (int64_t)a * n,
                               std::min(CROSS_COLS, cur.nl - a), part.p, s);
      }
    }
  }
  // results: the slices' pairs in order, up to the first slice that did not
  // complete (the pairs above it would leave a gap)
  riga_status status = RIGA_OK;
  int nf = 0;
  for (int i = 0; i < (int)slices.size() && nf < o->nev; ++i) {
    const Slice& S = *slices[i];
    const std::vector<Locked> pairs = slice_pairs(S);
    std::vector<int> out, in;
    for (size_t q = 0; q < pairs.size() && nf < o->nev; ++q) {
      if (pairs[q].partner) continue;  // J u of a complex pair: returned once
      if (evals) evals[nf] = pairs[q].lam;
      if (resid) resid[nf] = pairs[q].resid;
      out.push_back(nf);
      in.push_back(pairs[q].col);
      ++nf;
    }
    if (evecs && !out.empty()) {
      if (i > 0) HIPCHECK(hipStreamSynchronize(streams[i - 1]));
      launch_copy_cols(out, in, S.sv.N, evecs, S.sv.B.p, nullptr, nullptr, s);
    }
    if (S.status != RIGA_OK) {
      status = S.status;
      break;
    }
  }
  HIPCHECK(hipStreamSynchronize(s));
  *n_found = nf;
  const bool split = slices.size() > 1;
  const int wanted = split ? o->nev : A.nev / comp;
  if (nf < wanted && status == RIGA_OK) status = RIGA_ENOCONV;
  riga_stats st = A.sv.st;
  for (int i = 1; i < (int)slices.size(); ++i) add_stats(st, slices[i]->sv.st);
  st.t_total = secs(t0, clk::now());
  st.flops_fact = pr->an.flops_fact;
  st.bytes_fb = (double)pr->an.nnz_l * 2.0 * (o->precision == RIGA_MIXED ? 4.0 : 8.0);
  if (stats_out) *stats_out = st;
  pr->stats = st;
  return status;
}

namespace {

// RIGA_BATCH_FACTOR=0: every batched instance makes its first
// factorisation itself
bool batch_factor_on() {
  const char* v = std::getenv("RIGA_BATCH_FACTOR");
  return !(v && *v == '0');
}

// The shift and precision of the first factorisation of run_eigs (the
// first slice's finite upper end, counted first, else its lower end; an
// end other than 0 in FP64).
void first_factorisation(const riga_eigs_opts* o, double* sigma, int* prec) {
  double lo = o->lo - END_SHIFT * std::fabs(o->lo);
  double hi = std::isfinite(o->hi) ? o->hi - END_SHIFT * std::fabs(o->hi) : o->hi;
  if (!(hi > lo)) {
    lo = o->lo;
    hi = o->hi;
  }
  *sigma = std::isfinite(hi) ? hi : lo;
  *prec = *sigma == 0.0 ? o->precision : (int)RIGA_FP64;
}

// The instances' first factorisations, all at once (one launch per kernel
// and tree height over every instance), marked for their solves to use.
void prefactor(riga_problem* const* probs, int count, const riga_eigs_opts* o) {
  double sigma = 0.0;
  int prec = 0;
  first_factorisation(o, &sigma, &prec);
  std::vector<riga_problem*> prs(probs, probs + count);
  std::vector<Factor*> Fs(count);
  std::vector<double> sg(count, sigma);
  for (int i = 0; i < count; ++i) {
    Fs[i] = &prs[i]->ctx[0].current();
    factor_reserve(prs[i], *Fs[i], prec, prs[i]->home);
  }
  for (int i = 0; i < count; ++i) HIPCHECK(hipStreamSynchronize(prs[i]->home));
  hipStream_t s = nullptr;
  HIPCHECK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  struct Destroy {
    hipStream_t s;
    ~Destroy() { (void)hipStreamDestroy(s); }
  } destroy{s};
  factor_numeric_batched(prs, Fs, sg, prec, s);
  for (Factor* F : Fs) F->pre = true;
}

}  // namespace

// Many independent problems at once: the instances' first factorisations
// in one batched factorisation, then a pool of host threads, each with its
// own HIP stream, takes instances in order and runs the rest of the solve
// on its stream, so the kernels of different instances overlap on the
// device.
riga_status run_eigs_batched(riga_problem* const* probs, int count, const riga_eigs_opts* o,
                             int32_t* n_found, double* const* evals, double* const* evecs,
                             double* const* resid, riga_stats* stats, int workers,
                             std::string* first_error) {
  // (16 threads: 4-5% above 8 on the 64-instance 2D batch, the instances'
  // host-side checks and read-backs overlapping more of each other's work)
  if (workers <= 0) workers = 16;
  workers = std::max(1, std::min(workers, count));
  int dev = 0;
  HIPCHECK(hipGetDevice(&dev));
  std::atomic<int> next(0);
  std::vector<riga_status> status(count, RIGA_OK);
  std::vector<std::string> errs(count);
  std::vector<std::string> worker_err(workers);
  for (int i = 0; i < count; ++i) n_found[i] = 0;
  // kernel attributes are per device and process: set them once here, not
  // from the workers while others launch
  set_kernel_attributes();
  // a factorisation made ahead and not used (a solve that failed before
  // its first factorisation) is not left for later calls
  struct ClearPre {
    riga_problem* const* p;
    int n;
    ~ClearPre() {
      for (int i = 0; i < n; ++i)
        for (Factor& F : p[i]->ctx[0].fac) F.pre = false;
    }
  } clear_pre{probs, count};
  if (batch_factor_on()) prefactor(probs, count, o);
  std::vector<std::thread> pool;
  for (int w = 0; w < workers; ++w) {
    pool.emplace_back([&, w] {
      hipStream_t st = nullptr;
      try {
        HIPCHECK(hipSetDevice(dev));
        HIPCHECK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
      } catch (const std::exception& e) {
        worker_err[w] = e.what();
        return;
      }
      for (int i = next++; i < count; i = next++) {
        riga_eigs_opts oi = *o;
        oi.stream = st;
        try {
          status[i] = run_eigs(probs[i], &oi, &n_found[i], evals[i], evecs ? evecs[i] : nullptr,
                               resid ? resid[i] : nullptr, stats ? &stats[i] : nullptr);
        } catch (const Error& e) {
          status[i] = e.code;
          errs[i] = e.what();
        } catch (const std::exception& e) {
          status[i] = RIGA_EINVAL;
          errs[i] = e.what();
        }
      }
      (void)hipStreamDestroy(st);
    });
  }
  for (auto& t : pool) t.join();
  riga_status worst = RIGA_OK;
  int done = next.load() >= count ? count : next.load();
  for (int w = 0; w < workers; ++w)
    if (!worker_err[w].empty()) {
      *first_error = "worker set-up: " + worker_err[w];
      if (done < count) return RIGA_EDEVICE;
    }
  for (int i = 0; i < count; ++i) {
    if (status[i] == RIGA_OK) continue;
    if (worst == RIGA_OK || (worst == RIGA_ENOCONV && status[i] != RIGA_ENOCONV)) {
      worst = status[i];
      *first_error = "instance " + std::to_string(i) + ": " +
                     (errs[i].empty() ? std::string("not converged") : errs[i]);
    }
  }
  return worst;
}

}  // namespace riga
