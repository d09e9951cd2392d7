// Device set-up of a problem: upload of the analysis, assembly of K and M,
// norms, the per-level front lists; allocation helpers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cmath>
#include <cstdint>
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
  {
    // fronts whose one child's update block is the front row for row (the
    // chains of split separators): assembled by contiguous copies
    std::vector<int32_t> ident(std::max(an.n_fronts, 1), 0);
    for (int F = 0; F < an.n_fronts; ++F) {
      if (an.child_ptr[F + 1] - an.child_ptr[F] != 1) continue;
      const int ci = an.child_ptr[F], C = an.child_list[ci];
      if (an.f_f[C] - an.f_k[C] != an.f_f[F]) continue;
      bool same = true;
      for (int i = 0; i < an.f_f[F] && same; ++i) same = an.inv[an.inv_off[ci] + i] == i;
      ident[F] = same ? 1 : 0;
    }
    pr->d_asm_ident.upload(ident, s);
  }
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
    // A front of more than XCD_PIECE units (the tall fronts of split
    // separators, alone on their level) is dealt out in pieces of that many
    // consecutive units, so that one front does not leave seven XCDs idle.
    auto xcd_order = [&](bool rows_split, int width) {
      std::vector<std::vector<WorkUnit>> q(XCDS);
      std::vector<int64_t> load(XCDS, 0);
      for (auto it = fr.rbegin(); it != fr.rend(); ++it) {
        const int F = *it, f = an.f_f[F], k = an.f_k[F];
        const int n = rows_split ? f : k;
        for (int a0 = 0; a0 < n; a0 += XCD_PIECE * width) {
          const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
          const int a1 = std::min(n, a0 + XCD_PIECE * width);
          for (int a = a0; a < a1; a += width) q[x].push_back(unit(F, a, std::min(n, a + width)));
          load[x] += (a1 - a0 + width - 1) / width;
        }
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
  // a measured choice of the sweep decomposition for this device and tree
  // (riga_tune's cache), unless the environment fixes either part
  int cut = TOP_CUT_MODEL, fused = SUB_FROM_ENV;
  const char* env_cut = std::getenv("RIGA_TOP_CUT");
  const char* env_sub = std::getenv("RIGA_SUBTREE_HEIGHTS");
  pr->tuned = false;
  if (!(env_cut && *env_cut) && !(env_sub && *env_sub) && tune_lookup(pr, &cut, &fused)) pr->tuned = true;
  setup_top(pr, cut);
  setup_subtrees(pr, fused);
  HIPCHECK(hipStreamSynchronize(s));
  pr->has_device = true;
}

// Fused sweeps of the bottom heights.  Every launch of a level sweep pays a
// chain of dependent memory round trips (unit record, gather indices, the
// gathered values, H) whatever its data; the fronts of the bottom heights
// form many independent subtrees, so one workgroup per subtree can sweep
// them all in one launch per direction, keeping the vectors passed between
// the subtree's fronts in LDS and loading the next round's H while the
// current one is reduced.  The fused heights are the most that keep at
// least SUB_MIN_SUBTREES subtrees (a workgroup per CU) or subtrees of at
// most SUB_MAX_BYTES of H each (small problems, where latency is all there
// is); at least two heights, below the top block, and every subtree within
// the LDS budget.  Off by default: on the 2D 256^2 p = 3 rIGA workload the
// fused launches take as long as the level launches they replace (24.2 and
// 35.0 us against 24.3 and 35.4 us per sweep pair: each round of a subtree
// still waits out a memory latency), and during an eigen-solve their
// CU-wide workgroups slow the other spectrum slice's kernels.
// RIGA_SUBTREE_HEIGHTS=n fuses n heights; "auto" applies the rule above.
void setup_subtrees(riga_problem* pr, int forced) {
  constexpr int SUB_MIN_SUBTREES = 256;
  constexpr double SUB_MAX_BYTES = 262144.0;
  constexpr size_t SUB_LDS_MAX = 64 * 1024;
  const Analysis& an = pr->an;
  hipStream_t s = pr->home;
  pr->sub = SubtreeDev{};
  const int nl = pr->top.cut >= 0 ? pr->top.cut : an.height;
  const int nf = an.n_fronts;
  struct Plan {
    int nh = 0;
    std::vector<int> subs;        // roots, heaviest first
    std::vector<int> first;       // per root: its first front (post-order)
    int max_units = 0, max_np = 0, max_ncb = 0, max_k = 0, max_f = 0;
    size_t lds_fwd = 0, lds_bwd = 0;
    double max_bytes = 0.0;
  };
  // the plan for nh fused heights; false if a subtree is not a post-order
  // range or does not fit the LDS budget
  auto plan = [&](int nh, Plan& P) {
    P = Plan{};
    P.nh = nh;
    std::vector<int> root(nf, -1), lo(nf, -1);
    std::vector<double> bytes(nf, 0.0);
    std::vector<int> units(nf, 0), cnt(nf, 0);
    for (int F = 0; F < nf; ++F) {
      if (an.f_height[F] >= nh) continue;
      int R = F;
      while (an.f_parent[R] >= 0 && an.f_height[an.f_parent[R]] < nh) R = an.f_parent[R];
      root[F] = R;
      if (lo[R] < 0) lo[R] = F;
      ++cnt[R];
      bytes[R] += (double)an.f_f[F] * an.f_k[F] * 8.0;
      units[R] += std::max((an.f_f[F] + SUB_ROWS - 1) / SUB_ROWS, (an.f_k[F] + SUB_COLS - 1) / SUB_COLS);
      P.max_k = std::max(P.max_k, an.f_k[F]);
      P.max_f = std::max(P.max_f, an.f_f[F]);
    }
    for (int R = 0; R < nf; ++R) {
      if (root[R] != R) continue;
      if (cnt[R] != R - lo[R] + 1) return false;  // not a post-order range
      P.subs.push_back(R);
      const int np = an.f_start[R] + an.f_k[R] - an.f_start[lo[R]];
      const int64_t ncb = an.f_cb_off[R + 1] - an.f_cb_off[lo[R]];
      if (ncb > INT32_MAX) return false;
      P.max_units = std::max(P.max_units, units[R]);
      P.max_np = std::max(P.max_np, np);
      P.max_ncb = std::max(P.max_ncb, (int)ncb);
      P.max_bytes = std::max(P.max_bytes, bytes[R]);
    }
    std::stable_sort(P.subs.begin(), P.subs.end(), [&](int a, int b) { return bytes[a] > bytes[b]; });
    for (int R : P.subs) P.first.push_back(lo[R]);
    const size_t ucache = (size_t)P.max_units * sizeof(WorkUnit);
    P.lds_fwd = ucache + sizeof(double) * ((size_t)P.max_np + P.max_ncb + (size_t)SUB_GROUPS * (P.max_k + 256));
    P.lds_bwd = ucache + sizeof(double) * (2 * (size_t)P.max_np + (size_t)SUB_GROUPS * P.max_f);
    return P.lds_fwd <= SUB_LDS_MAX && P.lds_bwd <= SUB_LDS_MAX;
  };
  Plan best, P;
  int want = forced;
  if (want == SUB_FROM_ENV) {
    const char* env = std::getenv("RIGA_SUBTREE_HEIGHTS");
    if (!env || !*env) return;
    want = std::strcmp(env, "auto") == 0 ? SUB_AUTO : std::atoi(env);
  }
  if (want == 0) return;
  if (want != SUB_AUTO) {
    const int nh = std::max(0, std::min(want, nl));
    if (nh >= 2 && plan(nh, P)) best = std::move(P);
  } else {
    for (int c = 2; c <= nl; ++c)
      if (plan(c, P) && ((int)P.subs.size() >= SUB_MIN_SUBTREES || P.max_bytes <= SUB_MAX_BYTES))
        best = std::move(P);
  }
  if (best.nh < 2) return;
  const int nh = best.nh, n_sub = (int)best.subs.size();
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
    // `pad` marks the subtree's root: its update vector is also the
    // input of the sweep above the fused heights
    w.pad = an.f_parent[F] < 0 || an.f_height[an.f_parent[F]] >= nh;
    return w;
  };
  std::vector<WorkUnit> fu, bu;
  std::vector<int32_t> fo, bo;
  std::vector<SubInfo> info;
  for (int i = 0; i < n_sub; ++i) {
    const int R = best.subs[i], F0 = best.first[i];
    SubInfo si{};
    si.p0 = an.f_start[F0];
    si.np = an.f_start[R] + an.f_k[R] - si.p0;
    si.cb0 = (int32_t)an.f_cb_off[F0];
    si.ncb = (int32_t)(an.f_cb_off[R + 1] - an.f_cb_off[F0]);
    info.push_back(si);
    for (int h = 0; h <= nh; ++h) {
      fo.push_back((int32_t)fu.size());
      bo.push_back((int32_t)bu.size());
      if (h == nh) break;
      for (int F = F0; F <= R; ++F) {
        if (an.f_height[F] != h) continue;
        for (int a = 0; a < an.f_f[F]; a += SUB_ROWS) fu.push_back(unit(F, a, std::min(an.f_f[F], a + SUB_ROWS)));
        for (int a = 0; a < an.f_k[F]; a += SUB_COLS) bu.push_back(unit(F, a, std::min(an.f_k[F], a + SUB_COLS)));
      }
    }
  }
  SubtreeDev& S = pr->sub;
  S.nh = nh;
  S.n_sub = n_sub;
  S.max_units = best.max_units;
  S.max_np = best.max_np;
  S.max_ncb = best.max_ncb;
  S.grp_fwd = best.max_k + 256;
  S.grp_bwd = std::max(best.max_f, 1);
  S.lds_fwd = best.lds_fwd;
  S.lds_bwd = best.lds_bwd;
  S.fwd_units.upload(fu, s);
  S.bwd_units.upload(bu, s);
  S.fwd_off.upload(fo, s);
  S.bwd_off.upload(bo, s);
  S.info.upload(info, s);
}

}  // namespace riga
