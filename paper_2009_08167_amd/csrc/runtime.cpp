// Device set-up of a problem: upload of the analysis, assembly of K and M,
// norms, the per-level front lists; allocation helpers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

#include "problem.h"

namespace riga {

static riga_allocator g_alloc{};
static bool g_alloc_set = false;
static std::mutex g_alloc_mu;

void set_allocator(const riga_allocator* a) {
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  if (a) {
    g_alloc = *a;
    g_alloc_set = true;
  } else {
    g_alloc_set = false;
  }
}

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess)
    throw Error(e == hipErrorOutOfMemory ? RIGA_ENOMEM : RIGA_EDEVICE,
                std::string(what) + ": " + hipGetErrorString(e));
}

void* dmalloc(size_t bytes, hipStream_t s) {
  void* p = nullptr;
  if (g_alloc_set && g_alloc.alloc) {
    p = g_alloc.alloc(g_alloc.ctx, bytes, (void*)s);
    if (!p) throw Error(RIGA_ENOMEM, "allocator hook returned NULL");
    return p;
  }
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) throw Error(RIGA_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  return p;
}

void dfree(void* p, hipStream_t s) {
  if (!p) return;
  if (g_alloc_set && g_alloc.free) {
    g_alloc.free(g_alloc.ctx, p, (void*)s);
    return;
  }
  (void)hipFree(p);
}

// Copies the per-element coefficients (host values are checked positive)
// and assembles K and M on the device.
void load_and_assemble(riga_problem* pr, const double* kappa, const double* rho, int on_device,
                       hipStream_t s) {
  const Analysis& an = pr->an;
  auto load_coef = [&](const double* src, DBuf<double>& dst, const char* name) {
    if (!src) {
      dst.reset();
      return;
    }
    if (dst.n != (size_t)an.n_elem) dst.alloc(an.n_elem, s);
    if (on_device) {
      HIPCHECK(hipMemcpyAsync(dst.p, src, an.n_elem * sizeof(double), hipMemcpyDeviceToDevice, s));
    } else {
      for (int64_t e = 0; e < an.n_elem; ++e)
        if (!(src[e] > 0.0) || !std::isfinite(src[e]))
          throw Error(RIGA_EINVAL, std::string(name) + " must be positive and finite");
      HIPCHECK(hipMemcpyAsync(dst.p, src, an.n_elem * sizeof(double), hipMemcpyHostToDevice, s));
    }
  };
  load_coef(kappa, pr->kappa, "kappa");
  load_coef(rho, pr->rho, "rho");
  launch_assemble(pr);
  compute_norms(pr);
  pr->factored = false;
}

void setup_device(riga_problem* pr, const riga_mesh_desc* desc) {
  Analysis& an = pr->an;
  hipStream_t s = (hipStream_t)desc->stream;
  pr->stream = s;
  HIPCHECK(hipGetDevice(&pr->device));
  const int64_t N = an.N, nnz = an.row_ptr[N];
  pr->row_ptr.upload(an.row_ptr, s);
  pr->col_idx.upload(an.col_idx, s);
  pr->kv.alloc(nnz, s);
  pr->mv.alloc(nnz, s);
  launch_basis_tables(pr);
  load_and_assemble(pr, desc->kappa, desc->rho, desc->coeffs_on_device, s);
  const double avg = (double)nnz / (double)N;
  int g = 4;
  while (g < 64 && g * 3 < avg) g *= 2;
  pr->spmv_group = g;

  // symbolic factorisation
  pr->d_rows.upload(an.rows, s);
  pr->d_fk.upload(an.f_k, s);
  pr->d_ff.upload(an.f_f, s);
  pr->d_fstart.upload(an.f_start, s);
  pr->d_child_ptr.upload(an.child_ptr, s);
  pr->d_child_list.upload(an.child_list, s);
  pr->d_inv.upload(an.inv, s);
  pr->d_rows_off.upload(an.f_rows_off, s);
  pr->d_pool_off.upload(an.f_pool_off, s);
  pr->d_cb_off.upload(an.f_cb_off, s);
  pr->d_inv_off.upload(an.inv_off, s);
  pr->d_amap_ptr.upload(an.amap_ptr, s);
  pr->d_amap_row.upload(an.amap_row, s);
  pr->d_amap_val.upload(an.amap_val, s);
  pr->levels.clear();
  pr->levels.resize(an.height);
  for (int h = 0; h < an.height; ++h) {
    std::vector<int32_t> fr = an.levels[h];
    std::stable_sort(fr.begin(), fr.end(), [&](int a, int b) { return an.f_f[a] < an.f_f[b]; });
    LevelDev& L = pr->levels[h];
    L.n = (int)fr.size();
    std::vector<int64_t> pref(fr.size() + 1, 0);
    L.host_f.clear();
    for (size_t i = 0; i < fr.size(); ++i) {
      pref[i + 1] = pref[i] + an.f_f[fr[i]];
      L.max_f = std::max(L.max_f, an.f_f[fr[i]]);
      L.max_k = std::max(L.max_k, an.f_k[fr[i]]);
      L.host_f.push_back(an.f_f[fr[i]]);
    }
    L.cols = pref.back();
    L.fronts.upload(fr, s);
    L.col_prefix.upload(pref, s);
  }
  pr->piv_perm.alloc(N, s);
  pr->piv_type.alloc(N, s);
  pr->front_stat.alloc((size_t)an.n_fronts * 4, s);
  pr->cbvec.alloc(std::max<int64_t>(an.cb_size, 1), s);
  pr->fwd.alloc(N, s);
  HIPCHECK(hipStreamSynchronize(s));
  pr->has_device = true;
}

}  // namespace riga
