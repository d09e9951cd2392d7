// Device set-up of a problem: upload of the analysis, assembly of K and M,
// norms, the per-level front lists; allocation helpers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <mutex>

#include "problem.h"

namespace riga {

static riga_allocator g_alloc{};
static bool g_alloc_set = false;
static std::mutex g_alloc_mu;

void set_allocator(const riga_allocator* a) {
  if (a && (!a->alloc || !a->free)) throw Error(RIGA_EINVAL, "allocator needs both alloc and free");
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

void* dmalloc(size_t bytes, hipStream_t s, Release* how) {
  void* p = nullptr;
  riga_allocator a{};
  {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    if (g_alloc_set) a = g_alloc;
  }
  if (a.alloc) {
    p = a.alloc(a.ctx, bytes, (void*)s);
    if (!p) throw Error(RIGA_ENOMEM, "allocator hook returned NULL for " + std::to_string(bytes) + " bytes");
    how->ctx = a.ctx;
    how->free = a.free;
    return p;
  }
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw Error(RIGA_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  *how = Release{};
  return p;
}

void dfree(void* p, hipStream_t s, const Release& how) {
  if (!p) return;
  if (how.free) {
    how.free(how.ctx, p, (void*)s);
    return;
  }
  (void)hipFree(p);
}

void set_front_attributes();
void set_solve_attributes();
void set_inverse_attributes();
void set_bigfront_attributes();
void set_tridiag_attributes();
void set_top_attributes();

void set_kernel_attributes() {
  static std::once_flag once;
  std::call_once(once, [] {
    set_front_attributes();
    set_solve_attributes();
    set_inverse_attributes();
    set_bigfront_attributes();
    set_tridiag_attributes();
    set_top_attributes();
  });
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
  for (SolveCtx& c : pr->ctx) c.fac[0].factored = c.fac[1].factored = false;
}

void setup_device(riga_problem* pr, const riga_mesh_desc* desc) {
  Analysis& an = pr->an;
  hipStream_t s = (hipStream_t)desc->stream;
  // before the first launch of any problem: raising a kernel's LDS limit
  // while another thread launches kernels is a race in the runtime (the
  // batched solves once crashed in a launch while workers set attributes)
  set_kernel_attributes();
  pr->home = s;
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
  // solve descriptors and the flattened gather map: for each front position,
  // the absolute index in the update vectors of each child's contribution
  {
    int gs = 1;
    for (int F = 0; F < an.n_fronts; ++F) gs = std::max(gs, an.child_ptr[F + 1] - an.child_ptr[F]);
    if (gs > 4) throw Error(RIGA_EUNSUPPORTED, "a separator-tree node has more than 4 children");
    pr->gstride = gs;
    std::vector<FrontDesc> desc(an.n_fronts);
    std::vector<int32_t> gmap((size_t)an.f_rows_off[an.n_fronts] * gs, -1);
    for (int F = 0; F < an.n_fronts; ++F) {
      FrontDesc& d = desc[F];
      d.f = an.f_f[F];
      d.k = an.f_k[F];
      d.start = an.f_start[F];
      d.ldh = h_ld(d.f);
      d.pool_off = an.f_pool_off[F];
      d.h_off = an.f_h_off[F];
      d.rows_off = an.f_rows_off[F];
      d.cb_off = an.f_cb_off[F];
      d.gmap_off = an.f_rows_off[F] * gs;
      for (int ci = an.child_ptr[F]; ci < an.child_ptr[F + 1]; ++ci) {
        const int slot = ci - an.child_ptr[F], C = an.child_list[ci];
        for (int i = 0; i < d.f; ++i) {
          const int c = an.inv[an.inv_off[ci] + i];
          if (c >= 0) gmap[d.gmap_off + (int64_t)i * gs + slot] = (int32_t)(an.f_cb_off[C] + c);
        }
      }
    }
    pr->d_desc.upload(desc, s);
    pr->d_gmap.upload(gmap, s);
    std::vector<int32_t> front_of(N);
    for (int F = 0; F < an.n_fronts; ++F)
      for (int t = 0; t < an.f_k[F]; ++t) front_of[an.f_start[F] + t] = F;
    pr->d_front_of.upload(front_of, s);
  }
  pr->levels.clear();
  pr->levels.resize(an.height);
  for (int h = 0; h < an.height; ++h) {
    std::vector<int32_t> fr = an.levels[h];
    std::stable_sort(fr.begin(), fr.end(), [&](int a, int b) { return an.f_f[a] < an.f_f[b]; });
    LevelDev& L = pr->levels[h];
    L.n = (int)fr.size();
    std::vector<int64_t> pref(fr.size() + 1, 0);
    L.host_f.clear();
    L.host_k.clear();
    int lvl_max_f = 1;
    for (int F : fr) lvl_max_f = std::max(lvl_max_f, an.f_f[F]);
    L.asm_cols = std::max(1, std::min(ASM_COLS, ASM_LDS / (lvl_max_f * (int)sizeof(double))));
    if ((size_t)lvl_max_f * sizeof(double) > (size_t)ASM_LDS)
      throw Error(RIGA_EUNSUPPORTED, "front too large for the assembly kernel's LDS");
    for (size_t i = 0; i < fr.size(); ++i) {
      pref[i + 1] = pref[i] + (an.f_f[fr[i]] + L.asm_cols - 1) / L.asm_cols;
      L.max_f = std::max(L.max_f, an.f_f[fr[i]]);
      L.max_k = std::max(L.max_k, an.f_k[fr[i]]);
      L.host_f.push_back(an.f_f[fr[i]]);
      L.host_k.push_back(an.f_k[fr[i]]);
    }
    L.cols = pref.back();
    L.fronts.upload(fr, s);
    L.col_prefix.upload(pref, s);
    // sweep work units, largest fronts first
    std::vector<WorkUnit> fu, bu;
    int64_t nu_f = 0, nu_b = 0;
    for (int F : fr) {
      nu_f += (an.f_f[F] + SWEEP_ROWS - 1) / SWEEP_ROWS;
      nu_b += (an.f_k[F] + SWEEP_COLS - 1) / SWEEP_COLS;
    }
    L.fwd_thin = nu_f < SWEEP_THIN_BELOW;
    L.bwd_thin = nu_b < SWEEP_THIN_BELOW;
    const int rw = L.fwd_thin ? SWEEP_ROWS_THIN : SWEEP_ROWS;
    const int cw = L.bwd_thin ? SWEEP_COLS_THIN : SWEEP_COLS;
    auto unit = [&](int F, int lo, int hi) {
      WorkUnit w{};
      w.front = F;
      w.lo = lo;
      w.hi = hi;
      w.f = an.f_f[F];
      w.k = an.f_k[F];
      w.start = an.f_start[F];
      w.ldh = h_ld(an.f_f[F]);
      w.h_off = an.f_h_off[F];
      w.rows_off = an.f_rows_off[F];
      w.cb_off = an.f_cb_off[F];
      w.gmap_off = an.f_rows_off[F] * pr->gstride;
      return w;
    };
    // All units of one front go to one XCD (workgroups are dispatched to the
    // 8 XCDs round-robin by index), so the gathers that every unit of a
    // front repeats hit that XCD's L2; fronts are spread over the XCDs
    // largest first, and empty slots (front -1) pad the interleave.
    auto xcd_order = [&](bool rows_split, int width) {
      std::vector<std::vector<WorkUnit>> q(XCDS);
      std::vector<int64_t> load(XCDS, 0);
      for (auto it = fr.rbegin(); it != fr.rend(); ++it) {
        const int F = *it, f = an.f_f[F], k = an.f_k[F];
        const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        const int n = rows_split ? f : k;
        for (int a = 0; a < n; a += width) q[x].push_back(unit(F, a, std::min(n, a + width)));
        load[x] += (n + width - 1) / width;
      }
      size_t len = 0;
      for (auto& v : q) len = std::max(len, v.size());
      std::vector<WorkUnit> out;
      WorkUnit none{};
      none.front = -1;
      for (size_t i = 0; i < len; ++i)
        for (int x = 0; x < XCDS; ++x) out.push_back(i < q[x].size() ? q[x][i] : none);
      while (!out.empty() && out.back().front < 0) out.pop_back();
      return out;
    };
    fu = xcd_order(true, rw);
    bu = xcd_order(false, cw);
    L.n_fwd = (int)fu.size();
    L.n_bwd = (int)bu.size();
    L.fwd_units.upload(fu, s);
    L.bwd_units.upload(bu, s);
  }
  // inverse work units: row blocks of every front, most panels first
  {
    std::vector<int> order(an.n_fronts);
    for (int F = 0; F < an.n_fronts; ++F) order[F] = F;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return an.f_k[a] > an.f_k[b]; });
    std::vector<WorkUnit> iu;
    for (int F : order)
      for (int r = 0; r < an.f_f[F]; r += 64) {
        WorkUnit w{};
        w.front = F;
        w.lo = r;
        w.hi = std::min(an.f_f[F], r + 64);
        iu.push_back(w);
      }
    pr->n_inv_units = (int)iu.size();
    pr->inv_units.upload(iu, s);
  }
  if (an.max_fs > bigfront_max_k())
    throw Error(RIGA_EUNSUPPORTED, "fully-summed block too large for the panel kernel");
  if (front_inverse_lds(an.max_fs) > 159 * 1024)
    throw Error(RIGA_EUNSUPPORTED, "fully-summed block too large for the inverse kernel's LDS");
  setup_top(pr);
  HIPCHECK(hipStreamSynchronize(s));
  pr->has_device = true;
}

}  // namespace riga
