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
  const FrontDesc* desc;  // packed per-front record
  const int32_t* gmap;    // per front position: children's update indices
  int gstride;            // children slots per position (<= 4)
  const int32_t* rows;
  const int32_t* piv_perm;
  const int32_t* piv_type;
  double* cbvec;          // update vectors, one per front (f - k entries)
  double* fwd;            // z of the forward sweep, by new (pivot-order) index
};

// Forward sweep: 64 rows of one front per workgroup, lanes over rows (the
// column-major H is read coalesced), the four waves over interleaved columns.
template <class T>
__global__ void __launch_bounds__(256) fwd_kernel(SolveArgs sa, const T* __restrict__ H,
                                                  const WorkUnit* __restrict__ units,
                                                  const double* __restrict__ b) {
  extern __shared__ double smem[];
  const WorkUnit u = units[blockIdx.x];
  const FrontDesc d = sa.desc[u.front];
  const int f = d.f, k = d.k, start = d.start;
  const int lo = u.lo, hi = u.hi;
  double* y = smem;          // k: permuted fully-summed right-hand side
  double* psum = y + k;      // 4 x 64 partial sums
  const int32_t* rows = sa.rows + d.rows_off;
  const int32_t* gm = sa.gmap + d.gmap_off;
  const int gs = sa.gstride;
  const int tid = threadIdx.x, lane = tid & 63, g = tid >> 6;
  // the top rows need y_FS up to their own index, the update rows all of it
  const int kn = hi <= k ? hi : k;
  for (int t = tid; t < kn; t += 256) {
    const int pos = sa.piv_perm[start + t];
    int c[4];
#pragma unroll
    for (int sl = 0; sl < 4; ++sl) c[sl] = sl < gs ? gm[(int64_t)pos * gs + sl] : -1;
    double v = b[rows[pos]];
#pragma unroll
    for (int sl = 0; sl < 4; ++sl)
      if (c[sl] >= 0) v += sa.cbvec[c[sl]];
    y[t] = v;
  }
  __syncthreads();
  const int i = lo + lane;
  double s = 0.0;
  if (i < hi) {
    const int jend = i < k ? i : k;
    // the (i, i-1) slot of a 2x2 pivot block holds D, not L11^{-1} (= 0)
    const int skip = (i < k && i > 0 && sa.piv_type[start + i] == 3) ? i - 1 : -1;
    const T* hc = H + d.h_off + i;
    int j = g;
    for (; j + 60 < jend; j += 64) {
      double hv[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) hv[q] = (double)hc[(int64_t)(j + 4 * q) * f];
#pragma unroll
      for (int q = 0; q < 16; ++q) s += (j + 4 * q == skip ? 0.0 : hv[q]) * y[j + 4 * q];
    }
    for (; j < jend; j += 4)
      if (j != skip) s += (double)hc[(int64_t)j * f] * y[j];
  }
  psum[g * 64 + lane] = s;
  __syncthreads();
  if (g == 0 && i < hi) {
    const double tot = (psum[lane] + psum[64 + lane]) + (psum[128 + lane] + psum[192 + lane]);
    if (i < k) {
      sa.fwd[start + i] = y[i] + tot;
    } else {
      int c[4];
#pragma unroll
      for (int sl = 0; sl < 4; ++sl) c[sl] = sl < gs ? gm[(int64_t)i * gs + sl] : -1;
      double ycb = 0.0;
#pragma unroll
      for (int sl = 0; sl < 4; ++sl)
        if (c[sl] >= 0) ycb += sa.cbvec[c[sl]];
      sa.cbvec[d.cb_off + i - k] = ycb - tot;
    }
  }
}

// Backward sweep: 16 columns of one front per workgroup; wave w takes
// columns lo + w + 4c (c < 4), lanes over rows, 16 loads in flight per lane.
template <class T>
__global__ void __launch_bounds__(256) bwd_kernel(SolveArgs sa, const T* __restrict__ H,
                                                  const WorkUnit* __restrict__ units, double* x) {
  extern __shared__ double smem[];
  const WorkUnit u = units[blockIdx.x];
  const FrontDesc d = sa.desc[u.front];
  const int f = d.f, k = d.k, start = d.start;
  const int lo = u.lo, hi = u.hi;
  const T* Hf = H + d.h_off;
  const int32_t* rows = sa.rows + d.rows_off;
  double* v = smem;  // v[i - lo], i in [lo, f): D^{-1} z on the FS rows, -x below
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int i = lo + tid; i < f; i += 256) {
    double val;
    if (i < k) {
      const int ty = sa.piv_type[start + i];
      const double zi = sa.fwd[start + i];
      const double dii = (double)Hf[(int64_t)i * f + i];
      if (ty == 1) {
        val = zi / dii;
      } else if (ty == 2) {
        const double d21 = (double)Hf[(int64_t)i * f + i + 1];
        const double d22 = (double)Hf[(int64_t)(i + 1) * f + i + 1];
        val = (d22 * zi - d21 * sa.fwd[start + i + 1]) / (dii * d22 - d21 * d21);
      } else {
        const double d11 = (double)Hf[(int64_t)(i - 1) * f + i - 1];
        const double d21 = (double)Hf[(int64_t)(i - 1) * f + i];
        val = (d11 * zi - d21 * sa.fwd[start + i - 1]) / (d11 * dii - d21 * d21);
      }
    } else {
      val = -x[rows[i]];
    }
    v[i - lo] = val;
  }
  __syncthreads();
  int jc[4];
  bool two[4];
  double acc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    jc[c] = lo + wave + 4 * c;
    two[c] = jc[c] < hi && sa.piv_type[start + jc[c]] == 2;
    acc[c] = 0.0;
  }
  for (int i0 = lo + 1; i0 < f; i0 += 256) {
    double hv[4][4], vv[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = i0 + 64 * r + lane;
      vv[r] = i < f ? v[i - lo] : 0.0;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int j = jc[c];
        const bool use = j < hi && i < f && i > j && !(two[c] && i == j + 1);
        hv[r][c] = use ? (double)Hf[(int64_t)j * f + i] : 0.0;
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[c] += hv[r][c] * vv[r];
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    double s = acc[c];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    const int j = jc[c];
    if (lane == 0 && j < hi) x[rows[sa.piv_perm[start + j]]] = v[j - lo] + s;
  }
}

SolveArgs solve_args(riga_problem* pr) {
  SolveArgs sa{};
  sa.desc = pr->d_desc.p;
  sa.gmap = pr->d_gmap.p;
  sa.gstride = pr->gstride;
  sa.rows = pr->d_rows.p;
  sa.piv_perm = pr->piv_perm.p;
  sa.piv_type = pr->piv_type.p;
  sa.cbvec = pr->cbvec.p;
  sa.fwd = pr->fwd.p;
  return sa;
}

template <class T>
void apply_solve_attrs() {
  const void* ks[] = {(const void*)fwd_kernel<T>, (const void*)bwd_kernel<T>};
  for (const void* k : ks)
    HIPCHECK(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, 159 * 1024));
}

void attrs_once() {
  static std::once_flag once;
  std::call_once(once, [] { set_kernel_attributes(); });
}

// One launch per tree level and direction.
template <class T>
void solve_levels(riga_problem* pr, const T* H, const double* b, double* x, hipStream_t s) {
  SolveArgs sa = solve_args(pr);
  const int nl = (int)pr->levels.size();
  for (int h = 0; h < nl; ++h) {
    const LevelDev& L = pr->levels[h];
    if (L.n_fwd == 0) continue;
    fwd_kernel<T><<<L.n_fwd, 256, (size_t)(L.max_k + 256) * sizeof(double), s>>>(sa, H, L.fwd_units.p, b);
  }
  for (int h = nl - 1; h >= 0; --h) {
    const LevelDev& L = pr->levels[h];
    if (L.n_bwd == 0) continue;
    bwd_kernel<T><<<L.n_bwd, 256, (size_t)L.max_f * sizeof(double), s>>>(sa, H, L.bwd_units.p, x);
  }
  HIPCHECK(hipGetLastError());
}

}  // namespace

void set_solve_attributes() {
  apply_solve_attrs<double>();
  apply_solve_attrs<float>();
}

void solve_fb(riga_problem* pr, const double* b, double* x, hipStream_t s) {
  if (!pr->factored) throw Error(RIGA_EINVAL, "solve before factorisation");
  attrs_once();
  if (pr->fact_precision == RIGA_MIXED) solve_levels<float>(pr, pr->h32.p, b, x, s);
  else solve_levels<double>(pr, pr->h64.p, b, x, s);
}

}  // namespace riga
