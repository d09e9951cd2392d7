// The C ABI (include/riga.h): argument checks, error mapping, handle
// lifetime.  No exception crosses this boundary.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>

#include "problem.h"

namespace riga {
void set_allocator(const riga_allocator* a);
void setup_device(riga_problem* pr, const riga_mesh_desc* desc);
void load_and_assemble(riga_problem* pr, const double* kappa, const double* rho, int on_device,
                       hipStream_t s);
riga_status run_eigs(riga_problem* pr, const riga_eigs_opts* o, int32_t* n_found, double* evals,
                     double* evecs, double* resid, riga_stats* stats_out);
riga_status run_eigs_batched(riga_problem* const* probs, int count, const riga_eigs_opts* o,
                             int32_t* n_found, double* const* evals, double* const* evecs,
                             double* const* resid, riga_stats* stats, int workers,
                             std::string* first_error);
}  // namespace riga

namespace {

thread_local std::string g_err;

riga_status fail(riga_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

template <class F>
riga_status guarded(F&& f) {
  try {
    g_err.clear();
    return f();
  } catch (const riga::Error& e) {
    return fail(e.code, e.what());
  } catch (const std::bad_alloc&) {
    return fail(RIGA_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(RIGA_EINVAL, e.what());
  } catch (...) {
    return fail(RIGA_EINVAL, "unknown error");
  }
}

riga_status do_analyze(const riga_mesh_desc* d, riga_problem** out) {
  if (!d || !out) return fail(RIGA_EINVAL, "null descriptor or output");
  *out = nullptr;
  auto* pr = new riga_problem();
  if (d->hermitian != 0 && d->hermitian != 1) {
    delete pr;
    return fail(RIGA_EINVAL, "hermitian must be 0 or 1");
  }
  if (d->hermitian && (d->kappa || d->rho)) {
    delete pr;
    return fail(RIGA_EUNSUPPORTED, "the complex Hermitian pencil takes kappa = rho = 1 (NULL coefficients)");
  }
  std::string err = riga::analyze(d->dim, d->ne, d->p, d->sep_spacing, d->nquad, d->leaf_dofs, pr->an,
                                  d->hermitian ? 2 : 1);
  for (int q = 0; q < 3; ++q) pr->potential[q] = (d->hermitian && q < d->dim) ? d->potential[q] : 0.0;
  if (!err.empty()) {
    delete pr;
    return fail(RIGA_EINVAL, err);
  }
  *out = pr;
  return RIGA_OK;
}

bool need_device(const riga_problem* pr) { return pr && pr->has_device; }

}  // namespace

extern "C" {

riga_status riga_set_allocator(const riga_allocator* a) {
  return guarded([&] {
    riga::set_allocator(a);
    return RIGA_OK;
  });
}

riga_status riga_analyze(const riga_mesh_desc* desc, riga_problem** out) {
  return guarded([&] { return do_analyze(desc, out); });
}

riga_status riga_assemble(const riga_mesh_desc* desc, riga_problem** out) {
  return guarded([&]() -> riga_status {
    riga_status s = do_analyze(desc, out);
    if (s != RIGA_OK) return s;
    try {
      riga::setup_device(*out, desc);
    } catch (...) {
      delete *out;
      *out = nullptr;
      throw;
    }
    return RIGA_OK;
  });
}

riga_status riga_update_coefficients(riga_problem* pr, const double* kappa, const double* rho,
                                     int32_t on_device, void* stream) {
  return guarded([&]() -> riga_status {
    if (!need_device(pr)) return fail(RIGA_EINVAL, "problem has no device data");
    riga::StreamBind bind(pr, (hipStream_t)stream);
    riga::load_and_assemble(pr, kappa, rho, on_device, pr->stream);
    return RIGA_OK;
  });
}

riga_status riga_problem_info(const riga_problem* pr, riga_problem_info_t* info) {
  if (!pr || !info) return fail(RIGA_EINVAL, "null argument");
  const riga::Analysis& a = pr->an;
  info->n_dof = a.N;
  info->n_elem = a.n_elem;
  info->nnz = a.row_ptr.empty() ? 0 : a.row_ptr[a.N];
  for (int d = 0; d < 3; ++d) info->n1[d] = a.n1[d];
  info->n_fronts = a.n_fronts;
  info->tree_height = a.height;
  info->max_front = a.max_front;
  info->max_fs = a.max_fs;
  info->nnz_l = a.nnz_l;
  info->flops_fact = a.flops_fact;
  info->front_pool = a.pool_size;
  info->nnz_l_exact = a.nnz_l_exact;
  info->flops_fact_exact = a.flops_exact;
  info->components = a.components;
  info->sweep_bytes_stored = 0.0;
  info->top_cut = pr->has_device ? pr->top.cut : -1;
  info->fused_heights = pr->has_device ? pr->sub.nh : 0;
  info->fused_subtrees = pr->has_device ? pr->sub.n_sub : 0;
  info->tuned = pr->has_device && pr->tuned ? 1 : 0;
  if (pr->has_device) {
    const int cut = pr->top.cut >= 0 ? pr->top.cut : a.height;
    double e = (double)pr->top.e_row + (double)pr->top.e_col;
    for (int F = 0; F < a.n_fronts; ++F)
      if (a.f_height[F] < cut) e += 2.0 * (double)a.f_f[F] * (double)a.f_k[F];
    info->sweep_bytes_stored = 8.0 * e;
  }
  return RIGA_OK;
}

riga_status riga_tree_export(const riga_problem* pr, int32_t* perm, int32_t* front_k,
                             int32_t* front_f, int32_t* front_parent, int32_t* front_height,
                             int32_t* front_rows) {
  if (!pr) return fail(RIGA_EINVAL, "null problem");
  const riga::Analysis& a = pr->an;
  if (perm) std::memcpy(perm, a.perm.data(), a.N * sizeof(int32_t));
  if (front_k) std::memcpy(front_k, a.f_k.data(), a.n_fronts * sizeof(int32_t));
  if (front_f) std::memcpy(front_f, a.f_f.data(), a.n_fronts * sizeof(int32_t));
  if (front_parent) std::memcpy(front_parent, a.f_parent.data(), a.n_fronts * sizeof(int32_t));
  if (front_height) std::memcpy(front_height, a.f_height.data(), a.n_fronts * sizeof(int32_t));
  if (front_rows) std::memcpy(front_rows, a.rows.data(), a.rows.size() * sizeof(int32_t));
  return RIGA_OK;
}

riga_status riga_get_matrices(const riga_problem* pr, int64_t* row_ptr, int32_t* col_idx,
                              double* k_vals, double* m_vals) {
  return guarded([&]() -> riga_status {
    if (!pr) return fail(RIGA_EINVAL, "null problem");
    const riga::Analysis& a = pr->an;
    const int64_t nnz = a.row_ptr[a.N];
    if (row_ptr) std::memcpy(row_ptr, a.row_ptr.data(), (a.N + 1) * sizeof(int64_t));
    if (col_idx) std::memcpy(col_idx, a.col_idx.data(), nnz * sizeof(int32_t));
    if (k_vals || m_vals) {
      if (!need_device(pr)) return fail(RIGA_EINVAL, "problem has no device data (use riga_assemble)");
      if (k_vals) HIPCHECK(hipMemcpy(k_vals, pr->kv.p, nnz * sizeof(double), hipMemcpyDeviceToHost));
      if (m_vals) HIPCHECK(hipMemcpy(m_vals, pr->mv.p, nnz * sizeof(double), hipMemcpyDeviceToHost));
    }
    return RIGA_OK;
  });
}

riga_status riga_spmv(riga_problem* pr, int32_t which, const double* x, double* y, void* stream) {
  return guarded([&]() -> riga_status {
    if (!need_device(pr) || !x || !y) return fail(RIGA_EINVAL, "bad problem or vectors");
    hipStream_t s = (hipStream_t)stream;
    const double* vals = nullptr;
    if (which == RIGA_MAT_K) vals = pr->kv.p;
    else if (which == RIGA_MAT_M) vals = pr->mv.p;
    else if (which == RIGA_MAT_A) {
      riga::Factor& F = pr->ctx[0].current();
      if (!F.factored) return fail(RIGA_EINVAL, "no shift factorised yet");
      if (F.av.n < pr->kv.n) F.av.alloc(pr->kv.n, pr->home);
      riga::launch_axpby_vals(pr->kv.p, pr->mv.p, F.sigma, F.av.p, (int64_t)pr->kv.n, s);
      vals = F.av.p;
    } else return fail(RIGA_EINVAL, "which must be RIGA_MAT_K, _M or _A");
    riga::launch_spmv(pr, vals, x, y, nullptr, s);
    return RIGA_OK;
  });
}

riga_status riga_factor(riga_problem* pr, double sigma, int32_t precision, int64_t* neg_pivots,
                        riga_stats* stats) {
  return guarded([&]() -> riga_status {
    if (!need_device(pr)) return fail(RIGA_EINVAL, "problem has no device data");
    if (!std::isfinite(sigma)) return fail(RIGA_EINVAL, "sigma must be finite");
    if (precision != RIGA_FP64 && precision != RIGA_MIXED) return fail(RIGA_EINVAL, "bad precision");
    riga::Factor& F = pr->ctx[0].current();
    riga::factor_reserve(pr, F, precision, pr->home);
    riga::factor_numeric(pr, F, sigma, precision, pr->home);
    if (neg_pivots) *neg_pivots = F.inertia;
    if (stats) {
      std::memset(stats, 0, sizeof(*stats));
      stats->n_fact = 1;
      stats->n_perturbed_pivots = F.perturbed;
      stats->n_2x2_pivots = F.two;
      stats->flops_fact = pr->an.flops_fact;
    }
    if (F.perturbed > 0)
      return fail(RIGA_ESINGULAR, std::to_string(F.perturbed) +
                                      " pivot(s) perturbed: K - sigma M is singular to working precision");
    return RIGA_OK;
  });
}

riga_status riga_tune(riga_problem* pr, int32_t precision, int32_t reps, riga_tune_result* out) {
  return guarded([&]() -> riga_status {
    if (!need_device(pr)) return fail(RIGA_EINVAL, "problem has no device data");
    if (precision != RIGA_FP64 && precision != RIGA_MIXED) return fail(RIGA_EINVAL, "bad precision");
    riga::StreamBind bind(pr, pr->home);
    riga::tune_problem(pr, precision, reps > 0 ? reps : 20, out);
    pr->tuned = true;
    return RIGA_OK;
  });
}

riga_status riga_factor_batched(riga_problem* const* probs, int32_t count, const double* sigmas,
                                int32_t precision, int64_t* neg_pivots, riga_stats* stats) {
  return guarded([&]() -> riga_status {
    if (!probs || count < 0 || (count > 0 && !sigmas)) return fail(RIGA_EINVAL, "bad arguments");
    if (precision != RIGA_FP64 && precision != RIGA_MIXED) return fail(RIGA_EINVAL, "bad precision");
    if (count == 0) return RIGA_OK;
    int dev = 0;
    HIPCHECK(hipGetDevice(&dev));
    std::vector<riga_problem*> prs(probs, probs + count);
    std::vector<riga::Factor*> Fs(count);
    std::vector<double> sg(sigmas, sigmas + count);
    for (int i = 0; i < count; ++i) {
      if (!need_device(prs[i])) return fail(RIGA_EINVAL, "instance without device data");
      if (prs[i]->device != dev) return fail(RIGA_EINVAL, "instances must be on the current device");
      if (!std::isfinite(sg[i])) return fail(RIGA_EINVAL, "sigma must be finite");
      for (int j = 0; j < i; ++j)
        if (prs[j] == prs[i]) return fail(RIGA_EINVAL, "an instance appears twice");
    }
    for (int i = 0; i < count; ++i) {
      Fs[i] = &prs[i]->ctx[0].current();
      riga::factor_reserve(prs[i], *Fs[i], precision, prs[i]->home);
    }
    // the buffers (and earlier work on the problems) are ready before the
    // batched launches, which run on a stream of this call
    for (int i = 0; i < count; ++i) HIPCHECK(hipStreamSynchronize(prs[i]->home));
    hipStream_t s = nullptr;
    HIPCHECK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    struct Destroy {
      hipStream_t s;
      ~Destroy() { (void)hipStreamDestroy(s); }
    } destroy{s};
    riga::factor_numeric_batched(prs, Fs, sg, precision, s);
    int singular = 0;
    for (int i = 0; i < count; ++i) {
      const riga::Factor& F = *Fs[i];
      if (neg_pivots) neg_pivots[i] = F.inertia;
      if (stats) {
        std::memset(&stats[i], 0, sizeof(stats[i]));
        stats[i].n_fact = 1;
        stats[i].n_perturbed_pivots = F.perturbed;
        stats[i].n_2x2_pivots = F.two;
        stats[i].flops_fact = prs[i]->an.flops_fact;
      }
      if (F.perturbed > 0 && singular++ == 0)
        g_err = "instance " + std::to_string(i) + ": " + std::to_string(F.perturbed) +
                " pivot(s) perturbed: K - sigma M is singular to working precision";
    }
    return singular ? RIGA_ESINGULAR : RIGA_OK;
  });
}

namespace {

// x = A^{-1} b with the current factorisation; in mixed precision refined in
// FP64 (r = b - A x, x += A32^{-1} r) until ||r|| <= 1e-13 ||b|| or max_ir
// corrections.  Returns without synchronising when no refinement runs.
void solve_one(riga_problem* pr, const riga::Factor& F, const double* b, double* x, int32_t max_ir,
               hipStream_t s) {
  riga::solve_fb(pr, F, b, x, s);
  if (F.precision != RIGA_MIXED || max_ir <= 0) return;
  const int64_t N = pr->an.N;
  if (pr->ir_r.n < (size_t)N) {
    pr->ir_r.alloc(N, pr->home);
    pr->ir_d.alloc(N, pr->home);
  }
  riga::DBuf<double> part, nr;
  part.alloc(256, s);
  nr.alloc(2, s);
  double h[2] = {0.0, 0.0};
  riga::launch_dot(b, b, N, part.p, nr.p, s);
  HIPCHECK(hipMemcpyAsync(&h[0], nr.p, sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  const double bn2 = h[0];
  for (int it = 0; it < max_ir; ++it) {
    riga::launch_spmv(pr, F.av.p, x, pr->ir_r.p, nullptr, s);
    riga::launch_axpby(-1.0, pr->ir_r.p, b, pr->ir_r.p, N, s);
    riga::launch_dot(pr->ir_r.p, pr->ir_r.p, N, part.p, nr.p + 1, s);
    HIPCHECK(hipMemcpyAsync(&h[1], nr.p + 1, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    if (h[1] <= 1e-26 * bn2) break;
    riga::solve_fb(pr, F, pr->ir_r.p, pr->ir_d.p, s);
    riga::launch_axpby(1.0, pr->ir_d.p, x, x, N, s);
  }
}

}  // namespace

riga_status riga_solve(riga_problem* pr, const double* b, double* x, int32_t max_ir, void* stream) {
  return guarded([&]() -> riga_status {
    if (!need_device(pr) || !b || !x || b == x) return fail(RIGA_EINVAL, "bad problem or vectors");
    const riga::Factor& F = pr->ctx[0].current();
    if (!F.factored) return fail(RIGA_EINVAL, "no factorisation");
    hipStream_t s = (hipStream_t)stream;
    solve_one(pr, F, b, x, max_ir, s);
    HIPCHECK(hipStreamSynchronize(s));
    return RIGA_OK;
  });
}

riga_status riga_solve_multi(riga_problem* pr, const double* B, double* X, int32_t nrhs, int64_t ld,
                             int32_t max_ir, void* stream) {
  return guarded([&]() -> riga_status {
    if (!need_device(pr) || nrhs < 0) return fail(RIGA_EINVAL, "bad problem or nrhs");
    if (nrhs == 0) return RIGA_OK;
    if (!B || !X || ld < pr->an.N) return fail(RIGA_EINVAL, "bad blocks or leading dimension");
    const int64_t span = ld * (int64_t)(nrhs - 1) + pr->an.N;
    if (B < X + span && X < B + span) return fail(RIGA_EINVAL, "B and X overlap");
    const riga::Factor& F = pr->ctx[0].current();
    if (!F.factored) return fail(RIGA_EINVAL, "no factorisation");
    hipStream_t s = (hipStream_t)stream;
    for (int32_t i = 0; i < nrhs; ++i) solve_one(pr, F, B + ld * i, X + ld * i, max_ir, s);
    HIPCHECK(hipStreamSynchronize(s));
    return RIGA_OK;
  });
}

riga_status riga_project(int64_t n, int32_t m, const double* W, const double* B, double* x, double* c,
                         void* stream) {
  return guarded([&]() -> riga_status {
    if (n < 1 || m < 1 || m > RIGA_PROJECT_MAX_COLS || !W || !B || !x || !c)
      return fail(RIGA_EINVAL, "need n >= 1, 1 <= m <= RIGA_PROJECT_MAX_COLS and non-null blocks");
    hipStream_t s = (hipStream_t)stream;
    riga::DBuf<double> partial;
    partial.alloc((size_t)riga::proj_row_blocks(n) * m, s);
    riga::launch_project(W, B, n, m, x, partial.p, c, nullptr, nullptr, s);
    HIPCHECK(hipStreamSynchronize(s));
    return RIGA_OK;
  });
}

riga_status riga_project_noalloc(int64_t n, int32_t m, const double* W, const double* B, double* x,
                                 double* c, void* stream) {
  return guarded([&]() -> riga_status {
    if (n < 1 || m < 1 || m > RIGA_PROJECT_MAX_COLS || !W || !B || !x || !c)
      return fail(RIGA_EINVAL, "need n >= 1, 1 <= m <= RIGA_PROJECT_MAX_COLS and non-null blocks");
    const size_t need = (size_t)riga::proj_row_blocks(n) * (size_t)m;
    if (need > riga::NOALLOC_SCRATCH_DOUBLES)
      return fail(RIGA_EINVAL, "ceil(n / 4096) * m = " + std::to_string(need) +
                                   " exceeds the fixed scratch of " +
                                   std::to_string(riga::NOALLOC_SCRATCH_DOUBLES) + " doubles");
    double* partial = riga::noalloc_scratch();
    riga::launch_project(W, B, n, m, x, partial, c, nullptr, nullptr, (hipStream_t)stream);
    return RIGA_OK;
  });
}

riga_status riga_eigs(riga_problem* pr, const riga_eigs_opts* o, int32_t* n_found, double* evals,
                      double* evecs, double* resid, riga_stats* stats) {
  return guarded([&]() -> riga_status {
    if (!need_device(pr) || !o || !n_found) return fail(RIGA_EINVAL, "bad problem or options");
    if (o->nev < 1) return fail(RIGA_EINVAL, "nev must be >= 1");
    if ((int64_t)o->nev * pr->an.components > pr->an.N) return fail(RIGA_EINVAL, "nev exceeds the number of DOFs");
    if (!std::isfinite(o->lo) || !(o->hi > o->lo)) return fail(RIGA_EINVAL, "need finite lo < hi");
    if (o->precision != RIGA_FP64 && o->precision != RIGA_MIXED) return fail(RIGA_EINVAL, "bad precision");
    if (!evals) return fail(RIGA_EINVAL, "evals_host required");
    riga_status st = riga::run_eigs(pr, o, n_found, evals, evecs, resid, stats);
    if (st == RIGA_ENOCONV) g_err = "not all requested eigenpairs converged";
    return st;
  });
}

riga_status riga_eigs_batched(riga_problem* const* probs, int32_t count, const riga_eigs_opts* o,
                              int32_t workers, int32_t* n_found, double* const* evals,
                              double* const* evecs, double* const* resid, riga_stats* stats) {
  return guarded([&]() -> riga_status {
    if (!probs || count < 1 || !o || !n_found || !evals) return fail(RIGA_EINVAL, "bad arguments");
    for (int i = 0; i < count; ++i) {
      if (!need_device(probs[i])) return fail(RIGA_EINVAL, "instance without device data");
      if (!evals[i]) return fail(RIGA_EINVAL, "evals_host[i] required");
      if ((int64_t)o->nev * probs[i]->an.components > probs[i]->an.N)
        return fail(RIGA_EINVAL, "nev exceeds an instance's DOFs");
      for (int j = 0; j < i; ++j)
        if (probs[j] == probs[i]) return fail(RIGA_EINVAL, "an instance appears twice");
    }
    if (o->nev < 1 || !std::isfinite(o->lo) || !(o->hi > o->lo)) return fail(RIGA_EINVAL, "bad options");
    std::string err;
    riga_status st = riga::run_eigs_batched(probs, count, o, n_found, evals, evecs, resid, stats,
                                            workers, &err);
    if (st != RIGA_OK) g_err = err;
    return st;
  });
}

riga_status riga_eig_grad(riga_problem* pr, int32_t k, const double* evals, const double* evecs,
                          const double* w, double* dkappa, double* drho, void* stream) {
  return guarded([&]() -> riga_status {
    if (!need_device(pr) || k < 1 || !evals || !evecs || !w || !dkappa || !drho)
      return fail(RIGA_EINVAL, "bad arguments");
    if (pr->an.components != 1) return fail(RIGA_EUNSUPPORTED, "gradient of a complex pencil");
    for (int i = 0; i < k; ++i)
      for (int j = i + 1; j < k; ++j)
        if (std::fabs(evals[i] - evals[j]) <= 1e-8 * std::max(std::fabs(evals[i]), std::fabs(evals[j])))
          return fail(RIGA_EDEGENERATE, "eigenvalues " + std::to_string(i) + " and " +
                                            std::to_string(j) + " are not simple");
    hipStream_t s = (hipStream_t)stream;
    riga::DBuf<double> lam, ww;
    lam.alloc(k, s);
    ww.alloc(k, s);
    HIPCHECK(hipMemcpyAsync(lam.p, evals, k * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHECK(hipMemcpyAsync(ww.p, w, k * sizeof(double), hipMemcpyHostToDevice, s));
    riga::launch_eig_grad(pr, k, evecs, lam.p, ww.p, dkappa, drho, s);
    HIPCHECK(hipStreamSynchronize(s));
    return RIGA_OK;
  });
}

riga_status riga_mode_errors(riga_problem* pr, int32_t n_vec, const double* lam_host,
                             const double* U_dev, int32_t n_modes, const int32_t* modes_host,
                             int32_t nquad, int32_t* match, double* overlap, double* ef_l2,
                             double* ef_e, double* ev, void* stream) {
  return guarded([&]() -> riga_status {
    if (!need_device(pr) || n_vec < 1 || n_modes < 1 || !lam_host || !U_dev || !modes_host || !match ||
        !overlap || !ef_l2 || !ef_e || !ev || nquad < 0)
      return fail(RIGA_EINVAL, "bad arguments");
    if (pr->an.components != 1) return fail(RIGA_EUNSUPPORTED, "mode errors of a complex pencil");
    riga::mode_errors(pr, n_vec, lam_host, U_dev, n_modes, modes_host, nquad, match, overlap, ef_l2,
                      ef_e, ev, (hipStream_t)stream);
    return RIGA_OK;
  });
}

riga_status riga_exact_eigenvalues(int32_t dim, int32_t count, double* out_host) {
  return guarded([&]() -> riga_status {
    if ((dim != 2 && dim != 3) || count < 1 || count > (1 << 24) || !out_host)
      return fail(RIGA_EINVAL, "bad arguments");
    riga::exact_eigenvalues(dim, count, out_host);
    return RIGA_OK;
  });
}

void riga_destroy(riga_problem* pr) {
  if (!pr) return;
  try {
    if (pr->has_device) (void)hipStreamSynchronize(pr->home);
  } catch (...) {
  }
  delete pr;
}

const char* riga_status_string(riga_status s) {
  switch (s) {
    case RIGA_OK: return "ok";
    case RIGA_EINVAL: return "invalid argument";
    case RIGA_ENOMEM: return "out of memory";
    case RIGA_EDEVICE: return "device error";
    case RIGA_ENOCONV: return "not converged";
    case RIGA_ESINGULAR: return "singular shifted matrix";
    case RIGA_EDEGENERATE: return "degenerate eigenvalue";
    case RIGA_EUNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

const char* riga_last_error(void) { return g_err.c_str(); }

}  // extern "C"
