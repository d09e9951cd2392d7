// Forward/backward elimination with the multifrontal LDL^T factors: one
// application of (K - sigma M)^{-1} per Lanczos step (the "f/b elimination"
// of Sec. 5.1 and Table matvecs of arXiv 2009.08167).
//
// Forward sweep, leaves to root, one workgroup per front:
//   y = b(front FS variables) (+) children's update vectors (extend-add)
//   z = P y_FS;  L11 z' = z;  y_CB -= L21 z';  w = D^{-1} z'
//   w is kept per fully-summed variable, y_CB becomes the update vector
//   passed to the parent.
// Backward sweep, root to leaves:
//   v = w - L21^T x_CB;  L11^T x' = v;  x(FS variables) = P^T x'.
// Every vector entry is written by one thread (no atomics); the children
// of a front are summed in a fixed order.
#include <hip/hip_runtime.h>

#include "problem.h"

namespace riga {
namespace {

struct SolveArgs {
  const int32_t* fk;
  const int32_t* ff;
  const int32_t* fstart;
  const int64_t* pool_off;
  const int64_t* rows_off;
  const int32_t* rows;
  const int64_t* cb_off;
  const int32_t* child_ptr;
  const int32_t* child_list;
  const int64_t* inv_off;
  const int32_t* inv;
  const int32_t* piv_perm;
  const int32_t* piv_type;
  double* cbvec;
  double* fwd;
};

template <class T>
__global__ void __launch_bounds__(256) fwd_kernel(SolveArgs sa, const T* pool,
                                                const int32_t* fronts, const double* b) {
  extern __shared__ double y[];  // f + k doubles
  const int F = fronts[blockIdx.x];
  const int f = sa.ff[F], k = sa.fk[F], start = sa.fstart[F];
  const T* L = pool + sa.pool_off[F];
  const int32_t* rows = sa.rows + sa.rows_off[F];
  double* z = y + f;
  for (int i = threadIdx.x; i < f; i += blockDim.x) {
    double v = i < k ? b[rows[i]] : 0.0;
    for (int ci = sa.child_ptr[F]; ci < sa.child_ptr[F + 1]; ++ci) {
      const int c = sa.inv[sa.inv_off[ci] + i];
      if (c >= 0) v += sa.cbvec[sa.cb_off[sa.child_list[ci]] + c];
    }
    y[i] = v;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < k; t += blockDim.x) z[t] = y[sa.piv_perm[start + t]];
  __syncthreads();
  for (int t = threadIdx.x; t < k; t += blockDim.x) y[t] = z[t];
  __syncthreads();
  int t = 0;
  while (t < k) {
    const int ty = sa.piv_type[start + t];
    if (ty == 2) {
      const double z0 = y[t], z1 = y[t + 1];
      const T* c0 = L + (int64_t)t * f;
      const T* c1 = L + (int64_t)(t + 1) * f;
      for (int i = t + 2 + threadIdx.x; i < f; i += blockDim.x)
        y[i] -= (double)c0[i] * z0 + (double)c1[i] * z1;
      t += 2;
    } else {
      const double z0 = y[t];
      const T* c0 = L + (int64_t)t * f;
      for (int i = t + 1 + threadIdx.x; i < f; i += blockDim.x) y[i] -= (double)c0[i] * z0;
      t += 1;
    }
    __syncthreads();
  }
  for (int t2 = threadIdx.x; t2 < k; t2 += blockDim.x) {
    const int ty = sa.piv_type[start + t2];
    const double d = (double)L[(int64_t)t2 * f + t2];
    if (ty == 1) {
      sa.fwd[start + t2] = y[t2] / d;
    } else if (ty == 2) {
      const double d21 = (double)L[(int64_t)t2 * f + t2 + 1];
      const double d22 = (double)L[(int64_t)(t2 + 1) * f + t2 + 1];
      const double det = d * d22 - d21 * d21;
      sa.fwd[start + t2] = (d22 * y[t2] - d21 * y[t2 + 1]) / det;
      sa.fwd[start + t2 + 1] = (d * y[t2 + 1] - d21 * y[t2]) / det;
    }
  }
  for (int c = threadIdx.x; c < f - k; c += blockDim.x) sa.cbvec[sa.cb_off[F] + c] = y[k + c];
}

template <class T>
__global__ void __launch_bounds__(256) bwd_kernel(SolveArgs sa, const T* pool,
                                                const int32_t* fronts, double* x) {
  extern __shared__ double v[];  // k + (f - k) doubles
  const int F = fronts[blockIdx.x];
  const int f = sa.ff[F], k = sa.fk[F], start = sa.fstart[F];
  const T* L = pool + sa.pool_off[F];
  const int32_t* rows = sa.rows + sa.rows_off[F];
  double* xcb = v + k;
  for (int c = threadIdx.x; c < f - k; c += blockDim.x) xcb[c] = x[rows[k + c]];
  __syncthreads();
  // v_t = w_t - L21(:, t)^T x_CB : one wave per column
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int t = wave; t < k; t += nw) {
    const T* col = L + (int64_t)t * f + k;
    double s = 0.0;
    for (int c = lane; c < f - k; c += 64) s += (double)col[c] * xcb[c];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0) v[t] = sa.fwd[start + t] - s;
  }
  __syncthreads();
  // L11^T x' = v, last row first; a 2x2 pivot block has no L coupling
  for (int i = k - 1; i >= 0; --i) {
    const double xi = v[i];
    const int skip = sa.piv_type[start + i] == 3 ? i - 1 : -1;
    for (int s2 = threadIdx.x; s2 < i; s2 += blockDim.x)
      if (s2 != skip) v[s2] -= (double)L[(int64_t)s2 * f + i] * xi;
    __syncthreads();
  }
  for (int t = threadIdx.x; t < k; t += blockDim.x) x[rows[sa.piv_perm[start + t]]] = v[t];
}

SolveArgs solve_args(riga_problem* pr) {
  SolveArgs sa{};
  sa.fk = pr->d_fk.p;
  sa.ff = pr->d_ff.p;
  sa.fstart = pr->d_fstart.p;
  sa.pool_off = pr->d_pool_off.p;
  sa.rows_off = pr->d_rows_off.p;
  sa.rows = pr->d_rows.p;
  sa.cb_off = pr->d_cb_off.p;
  sa.child_ptr = pr->d_child_ptr.p;
  sa.child_list = pr->d_child_list.p;
  sa.inv_off = pr->d_inv_off.p;
  sa.inv = pr->d_inv.p;
  sa.piv_perm = pr->piv_perm.p;
  sa.piv_type = pr->piv_type.p;
  sa.cbvec = pr->cbvec.p;
  sa.fwd = pr->fwd.p;
  return sa;
}

template <class T>
void solve_levels(riga_problem* pr, const T* pool, const double* b, double* x, hipStream_t s) {
  SolveArgs sa = solve_args(pr);
  const int H = (int)pr->levels.size();
  for (int h = 0; h < H; ++h) {
    const LevelDev& L = pr->levels[h];
    if (L.n == 0) continue;
    fwd_kernel<T><<<L.n, 256, (size_t)(L.max_f + L.max_k) * sizeof(double), s>>>(sa, pool,
                                                                                 L.fronts.p, b);
  }
  for (int h = H - 1; h >= 0; --h) {
    const LevelDev& L = pr->levels[h];
    if (L.n == 0) continue;
    bwd_kernel<T><<<L.n, 256, (size_t)L.max_f * sizeof(double), s>>>(sa, pool, L.fronts.p, x);
  }
  HIPCHECK(hipGetLastError());
}

}  // namespace

void solve_fb(riga_problem* pr, const double* b, double* x, hipStream_t s) {
  if (!pr->factored) throw Error(RIGA_EINVAL, "solve before factorisation");
  if (pr->fact_precision == RIGA_MIXED)
    solve_levels<float>(pr, pr->pool32.p, b, x, s);
  else
    solve_levels<double>(pr, pr->pool64.p, b, x, s);
}

}  // namespace riga
