// Forward/backward elimination with the multifrontal LDL^T factors: one
// application of (K - sigma M)^{-1} per Lanczos step (the "f/b elimination"
// of Sec. 5.1 and Table matvecs of arXiv 2009.08167).
//
// The sweeps use the partitioned inverse H = [L11^{-1}; L21 L11^{-1}] of each
// front (formed after the factorisation, see k_inverse.hip), so that a
// front's share of a sweep is one dense product with no serial chain:
//
// Forward, leaves to root.  y = P b(front's FS variables) (+) children's
// update vectors (extend-add);
//     z      = L11^{-1} y_FS                 (rows 0..k-1 of H, unit diagonal)
//     u_CB   = y_CB - (L21 L11^{-1}) y_FS    (rows k..f-1 of H)
// z is kept per fully-summed variable, u_CB is the update vector passed to
// the parent.  Row blocks of one front go to different workgroups.
// Backward, root to leaves.  w = D^{-1} z (1x1 and 2x2 blocks);
//     x_FS = L11^{-T} (w - L21^T x_CB) = (L11^{-1})^T w - (L21 L11^{-1})^T x_CB
// one dot product per column of H; column blocks go to different
// workgroups, and x(FS variables) = P^T x_FS.
// Every vector entry is written by one thread (no atomics); the children of
// a front and the partial sums are added in a fixed order, so results are
// bitwise reproducible.
#include <hip/hip_runtime.h>

#include <mutex>

#include "problem.h"

namespace riga {
namespace {

struct SolveArgs {
  const int32_t* gmap;      // per front position: children's update indices
  int gstride;              // children slots per position (<= 4)
  const int32_t* rows;
  const int32_t* piv_type;  // 1: 1x1 pivot, 2/3: first/second of a 2x2 block
  const int32_t* piv_dof;   // DOF of each pivot
  const int32_t* piv_gmap;  // children's update indices of each pivot
  const double* dc;         // [N * 3] D^{-1} by pivot: w_n = c0 z_n + c+ z_{n+1} + c- z_{n-1}
  double* cbvec;            // update vectors, one per front (f - k entries)
  double* fwd;              // z of the forward sweep, by new (pivot-order) index
};

// Forward sweep: RW rows of one front per workgroup, lanes over rows (the
// column-major H is read coalesced), 256 / RW thread groups over interleaved
// columns (RW = 16 on levels with few fronts, for more loads in flight per
// row).  The first 16 loads of H are issued before the gather of y so that
// both latencies overlap.
template <class T, int RW>
__global__ void __launch_bounds__(256) fwd_kernel(SolveArgs sa, const T* __restrict__ H,
                                                  const WorkUnit* __restrict__ units,
                                                  const double* __restrict__ b) {
  constexpr int G = 256 / RW;
  extern __shared__ double smem[];
  const WorkUnit u = units[blockIdx.x];
  if (u.front < 0) return;  // padding slot of the XCD interleave
  const int k = u.k, start = u.start, ldh = u.ldh;
  const int lo = u.lo, hi = u.hi;
  double* y = smem;          // k: permuted fully-summed right-hand side
  double* psum = y + k;      // G x RW partial sums
  const int gs = sa.gstride;
  const int tid = threadIdx.x, rl = tid % RW, g = tid / RW;
  const int i = lo + rl;
  const bool row = i < hi;
  const int jend = row ? (i < k ? i : k) : 0;
  const T* hc = H + u.h_off + i;
  // the first 16 columns of this thread (predicated), before the gather
  double hv[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int j = g + G * q;
    hv[q] = j < jend ? (double)hc[(int64_t)j * ldh] : 0.0;
  }
  // the (i, i-1) slot of a 2x2 pivot block holds D, not L11^{-1} (= 0)
  const int skip = (row && i < k && i > 0 && sa.piv_type[start + i] == 3) ? i - 1 : -1;
  // update rows: the children's contributions at this position
  double ycb = 0.0;
  if (g == 0 && row && i >= k) {
    const int32_t* gm = sa.gmap + u.gmap_off + (int64_t)i * gs;
    int c[4];
#pragma unroll
    for (int sl = 0; sl < 4; ++sl) c[sl] = sl < gs ? gm[sl] : -1;
#pragma unroll
    for (int sl = 0; sl < 4; ++sl)
      if (c[sl] >= 0) ycb += sa.cbvec[c[sl]];
  }
  // the top rows need y_FS up to their own index, the update rows all of it
  const int kn = hi <= k ? hi : k;
  for (int t = tid; t < kn; t += 256) {
    const int n = start + t;
    int c[4];
#pragma unroll
    for (int sl = 0; sl < 4; ++sl) c[sl] = sl < gs ? sa.piv_gmap[(int64_t)n * gs + sl] : -1;
    double v = b[sa.piv_dof[n]];
#pragma unroll
    for (int sl = 0; sl < 4; ++sl)
      if (c[sl] >= 0) v += sa.cbvec[c[sl]];
    y[t] = v;
  }
  __syncthreads();
  double s = 0.0;
  for (int jb = g;;) {
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int j = jb + G * q;
      if (j < jend && j != skip) s += hv[q] * y[j];
    }
    jb += 16 * G;
    if (jb >= jend) break;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int j = jb + G * q;
      hv[q] = j < jend ? (double)hc[(int64_t)j * ldh] : 0.0;
    }
  }
  psum[g * RW + rl] = s;
  __syncthreads();
  if (g == 0 && row) {
    double tot = 0.0;
#pragma unroll
    for (int q = 0; q < G; ++q) tot += psum[q * RW + rl];
    if (i < k) sa.fwd[start + i] = y[i] + tot;
    else sa.cbvec[u.cb_off + i - k] = ycb - tot;
  }
}

// Backward sweep: 4 CPW columns of one front per workgroup; wave w takes
// columns lo + w + 4c (c < CPW), lanes over rows, 16 loads in flight per
// lane (16 / CPW row chunks of 64 per iteration; CPW = 1 on levels with few
// fronts).  The first iteration's loads are issued before the gather of v.
template <class T, int CPW>
__global__ void __launch_bounds__(256) bwd_kernel(SolveArgs sa, const T* __restrict__ H,
                                                  const WorkUnit* __restrict__ units, double* x) {
  constexpr int RCH = 16 / CPW;
  extern __shared__ double smem[];
  const WorkUnit u = units[blockIdx.x];
  if (u.front < 0) return;  // padding slot of the XCD interleave
  const int f = u.f, k = u.k, start = u.start, ldh = u.ldh;
  const int lo = u.lo, hi = u.hi;
  const T* Hf = H + u.h_off;
  const int32_t* rows = sa.rows + u.rows_off;
  double* v = smem;  // v[i - lo], i in [lo, f): D^{-1} z on the FS rows, -x below
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int jc[CPW];
  bool two[CPW];
  double acc[CPW];
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    jc[c] = lo + wave + 4 * c;
    two[c] = jc[c] < hi && sa.piv_type[start + jc[c]] == 2;
    acc[c] = 0.0;
  }
  double hv[RCH][CPW];
  // the 2x2 slot (j + 1, j) holds D: loaded like the rest, zeroed at use,
  // so that the loads do not wait for the pivot types
  auto load = [&](int i0) {
#pragma unroll
    for (int r = 0; r < RCH; ++r) {
      const int i = i0 + 64 * r + lane;
#pragma unroll
      for (int c = 0; c < CPW; ++c) {
        const int j = jc[c];
        const bool use = j < hi && i < f && i > j;
        hv[r][c] = use ? (double)Hf[(int64_t)j * ldh + i] : 0.0;
      }
    }
  };
  // row chunks start on a 16-row boundary (whole cache lines); rows at or
  // above a column's diagonal are masked
  const int ibeg = (lo + 1) & ~15;
  if (ibeg < f) load(ibeg);
  for (int i = lo + tid; i < f; i += 256) {
    double val;
    if (i < k) {
      // neighbours inside the front's own pivots (a 2x2 block never
      // crosses a front); their coefficient is zero otherwise
      const int n = start + i;
      const double* c3 = sa.dc + 3 * (int64_t)n;
      val = c3[0] * sa.fwd[n] + c3[1] * sa.fwd[start + min(i + 1, k - 1)] +
            c3[2] * sa.fwd[start + max(i - 1, 0)];
    } else {
      val = -x[rows[i]];
    }
    v[i - lo] = val;
  }
  __syncthreads();
  for (int i0 = ibeg; i0 < f; i0 += 64 * RCH) {
    if (i0 != ibeg) load(i0);
#pragma unroll
    for (int r = 0; r < RCH; ++r) {
      const int i = i0 + 64 * r + lane;
      const double vv = (i > lo && i < f) ? v[i - lo] : 0.0;
#pragma unroll
      for (int c = 0; c < CPW; ++c) acc[c] += (two[c] && i == jc[c] + 1) ? 0.0 : hv[r][c] * vv;
    }
  }
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    double s = acc[c];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    const int j = jc[c];
    if (lane == 0 && j < hi) x[sa.piv_dof[start + j]] = v[j - lo] + s;
  }
}

// Pivot-order copies of the forward gather maps: DOF and children's update
// indices of every pivot (the pivot order changes with each factorisation).
__global__ void pivot_maps_kernel(const FrontDesc* __restrict__ desc,
                                  const int32_t* __restrict__ front_of,
                                  const int32_t* __restrict__ piv_perm,
                                  const int32_t* __restrict__ rows, const int32_t* __restrict__ gmap,
                                  int gs, int64_t N, int32_t* piv_dof, int32_t* piv_gmap) {
  const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (n >= N) return;
  const FrontDesc d = desc[front_of[n]];
  const int pos = piv_perm[n];
  piv_dof[n] = rows[d.rows_off + pos];
  for (int sl = 0; sl < gs; ++sl) piv_gmap[n * gs + sl] = gmap[d.gmap_off + (int64_t)pos * gs + sl];
}

// D^{-1} by pivot (per factorisation): w_n = c0 z_n + c+ z_{n+1} + c- z_{n-1},
// the neighbours non-zero only inside a 2x2 block.
__global__ void dinv_coef_kernel(const int32_t* __restrict__ piv_type, const double* __restrict__ dd,
                                 const double* __restrict__ dsub, int64_t N, double* dc) {
  const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (n >= N) return;
  const int ty = piv_type[n];
  double c0, cp = 0.0, cm = 0.0;
  if (ty == 1) {
    c0 = 1.0 / dd[n];
  } else if (ty == 2) {
    const double d11 = dd[n], d21 = dsub[n], d22 = dd[n + 1];
    const double det = d11 * d22 - d21 * d21;
    c0 = d22 / det;
    cp = -d21 / det;
  } else {
    const double d11 = dd[n - 1], d21 = dsub[n - 1], d22 = dd[n];
    const double det = d11 * d22 - d21 * d21;
    c0 = d11 / det;
    cm = -d21 / det;
  }
  dc[3 * n] = c0;
  dc[3 * n + 1] = cp;
  dc[3 * n + 2] = cm;
}

SolveArgs solve_args(riga_problem* pr, const Factor& F) {
  SolveArgs sa{};
  sa.gmap = pr->d_gmap.p;
  sa.gstride = pr->gstride;
  sa.rows = pr->d_rows.p;
  sa.piv_type = F.piv_type.p;
  sa.piv_dof = F.piv_dof.p;
  sa.piv_gmap = F.piv_gmap.p;
  sa.dc = F.dcoef.p;
  sa.cbvec = F.cbvec.p;
  sa.fwd = F.fwd.p;
  return sa;
}

template <class T>
void apply_solve_attrs() {
  const void* ks[] = {(const void*)fwd_kernel<T, SWEEP_ROWS>, (const void*)fwd_kernel<T, SWEEP_ROWS_THIN>,
                      (const void*)bwd_kernel<T, SWEEP_COLS / 4>,
                      (const void*)bwd_kernel<T, SWEEP_COLS_THIN / 4>};
  for (const void* k : ks)
    HIPCHECK(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, 159 * 1024));
}

// One launch per tree level and direction.
// One launch per tree level and direction below the top block (all levels
// when there is none), three for the top block.
template <class T>
void solve_levels(riga_problem* pr, const Factor& F, const T* H, const T* trow, const T* tcol,
                  const double* b, double* x, hipStream_t s) {
  SolveArgs sa = solve_args(pr, F);
  const int nl = pr->top.cut >= 0 ? pr->top.cut : (int)pr->levels.size();
  for (int h = 0; h < nl; ++h) {
    const LevelDev& L = pr->levels[h];
    if (L.n_fwd == 0) continue;
    const size_t lds = (size_t)(L.max_k + 256) * sizeof(double);
    if (L.fwd_thin) fwd_kernel<T, SWEEP_ROWS_THIN><<<L.n_fwd, 256, lds, s>>>(sa, H, L.fwd_units.p, b);
    else fwd_kernel<T, SWEEP_ROWS><<<L.n_fwd, 256, lds, s>>>(sa, H, L.fwd_units.p, b);
  }
  if (pr->top.cut >= 0) sweep_top<T>(pr, F, trow, tcol, b, x, s);
  for (int h = nl - 1; h >= 0; --h) {
    const LevelDev& L = pr->levels[h];
    if (L.n_bwd == 0) continue;
    const size_t lds = (size_t)L.max_f * sizeof(double);
    if (L.bwd_thin) bwd_kernel<T, SWEEP_COLS_THIN / 4><<<L.n_bwd, 256, lds, s>>>(sa, H, L.bwd_units.p, x);
    else bwd_kernel<T, SWEEP_COLS / 4><<<L.n_bwd, 256, lds, s>>>(sa, H, L.bwd_units.p, x);
  }
  HIPCHECK(hipGetLastError());
}

}  // namespace

void set_solve_attributes() {
  apply_solve_attrs<double>();
  apply_solve_attrs<float>();
}

void launch_pivot_maps(riga_problem* pr, Factor& F, hipStream_t s) {
  const int64_t N = pr->an.N;
  if (N == 0) return;
  pivot_maps_kernel<<<(unsigned)((N + 255) / 256), 256, 0, s>>>(
      pr->d_desc.p, pr->d_front_of.p, F.piv_perm.p, pr->d_rows.p, pr->d_gmap.p, pr->gstride, N,
      F.piv_dof.p, F.piv_gmap.p);
  dinv_coef_kernel<<<(unsigned)((N + 255) / 256), 256, 0, s>>>(F.piv_type.p, F.d_diag.p, F.d_sub.p, N,
                                                             F.dcoef.p);
  HIPCHECK(hipGetLastError());
}

void solve_fb(riga_problem* pr, const Factor& F, const double* b, double* x, hipStream_t s) {
  if (!F.factored) throw Error(RIGA_EINVAL, "solve before factorisation");
  set_kernel_attributes();
  if (F.precision == RIGA_MIXED) solve_levels<float>(pr, F, F.h32.p, F.trow32.p, F.tcol32.p, b, x, s);
  else solve_levels<double>(pr, F, F.h64.p, F.trow64.p, F.tcol64.p, b, x, s);
}

}  // namespace riga
