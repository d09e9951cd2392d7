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

constexpr int PB = 64;  // panel width of the blocked triangular solves

// Loads the diagonal block L(p0:p0+pw, p0:p0+pw) (unit lower, strict part)
// into LDS `blk` (row-major, ld PB+1), zeroing the D entry of 2x2 pivot
// blocks, which is not part of L.
template <class T>
__device__ __forceinline__ void load_diag_block(const T* L, int f, int p0, int pw,
                                                const int32_t* type, double* blk) {
  for (int e = threadIdx.x; e < PB * PB; e += blockDim.x) {
    const int c = e / PB, r = e % PB;
    double v = 0.0;
    if (r < pw && c < pw && r > c) {
      v = (double)L[(int64_t)(p0 + c) * f + p0 + r];
      if (r == c + 1 && type[p0 + c] == 2) v = 0.0;
    }
    blk[r * (PB + 1) + c] = v;
  }
}

template <class T>
__device__ void fwd_front(const SolveArgs& sa, const T* pool, int F, const double* b,
                          double* smem) {
  double* blk = smem;                     // PB x (PB+1)
  double* y = smem + PB * (PB + 1);       // f
  const int f = sa.ff[F], k = sa.fk[F], start = sa.fstart[F];
  const T* L = pool + sa.pool_off[F];
  const int32_t* rows = sa.rows + sa.rows_off[F];
  const int32_t* type = sa.piv_type + start;
  const int32_t* perm = sa.piv_perm + start;
  double* z = y + f;                      // k (permutation scratch)
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // gather: own right-hand side entries plus the children's updates
  for (int i = threadIdx.x; i < f; i += blockDim.x) {
    double v = i < k ? b[rows[i]] : 0.0;
    for (int ci = sa.child_ptr[F]; ci < sa.child_ptr[F + 1]; ++ci) {
      const int c = sa.inv[sa.inv_off[ci] + i];
      if (c >= 0) v += sa.cbvec[sa.cb_off[sa.child_list[ci]] + c];
    }
    y[i] = v;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < k; t += blockDim.x) z[t] = y[perm[t]];
  __syncthreads();
  for (int t = threadIdx.x; t < k; t += blockDim.x) y[t] = z[t];
  // panels of the fully-summed block; a 2x2 pivot block never straddles two
  int p0 = 0;
  while (p0 < k) {
    int pw = min(PB, k - p0);
    if (pw > 1 && p0 + pw < k && type[p0 + pw - 1] == 2) --pw;
    __syncthreads();
    load_diag_block(L, f, p0, pw, type, blk);
    __syncthreads();
    if (wave == 0) {
      double yl = lane < pw ? y[p0 + lane] : 0.0;
      for (int t = 0; t < pw; ++t) {
        const double zt = __shfl(yl, t);
        if (lane > t) yl -= blk[lane * (PB + 1) + t] * zt;
      }
      if (lane < pw) y[p0 + lane] = yl;
    }
    __syncthreads();
    // rows below the panel: y_r -= L(r, panel) z_panel (16 loads in flight)
    for (int r = p0 + pw + threadIdx.x; r < f; r += blockDim.x) {
      const T* lr = L + (int64_t)p0 * f + r;
      double s = 0.0;
      int t = 0;
      for (; t + 16 <= pw; t += 16) {
        double lv[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) lv[u] = (double)lr[(int64_t)(t + u) * f];
#pragma unroll
        for (int u = 0; u < 16; ++u) s += lv[u] * y[p0 + t + u];
      }
      for (; t < pw; ++t) s += (double)lr[(int64_t)t * f] * y[p0 + t];
      y[r] -= s;
    }
    p0 += pw;
  }
  __syncthreads();
  for (int t2 = threadIdx.x; t2 < k; t2 += blockDim.x) {
    const int ty = type[t2];
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
__global__ void __launch_bounds__(256) fwd_kernel(SolveArgs sa, const T* pool,
                                                const int32_t* fronts, const double* b) {
  extern __shared__ double smem[];
  fwd_front<T>(sa, pool, fronts[blockIdx.x], b, smem);
}

template <class T>
__device__ void bwd_front(const SolveArgs& sa, const T* pool, int F, double* x, double* smem) {
  double* blk = smem;                     // PB x (PB+1)
  double* xv = smem + PB * (PB + 1);      // f: v/x of the FS block, then x_CB
  const int f = sa.ff[F], k = sa.fk[F], start = sa.fstart[F];
  const T* L = pool + sa.pool_off[F];
  const int32_t* rows = sa.rows + sa.rows_off[F];
  const int32_t* type = sa.piv_type + start;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int c = threadIdx.x; c < f - k; c += blockDim.x) xv[k + c] = x[rows[k + c]];
  for (int t = threadIdx.x; t < k; t += blockDim.x) xv[t] = sa.fwd[start + t];
  // panels from the bottom: v_panel -= L(below, panel)^T x_below, then the
  // transposed unit-triangular solve of the diagonal block
  int p1 = k;
  while (p1 > 0) {
    int p0 = max(0, p1 - PB);
    if (p0 > 0 && type[p0] == 3) ++p0;   // keep 2x2 pivot blocks whole
    const int pw = p1 - p0;
    __syncthreads();
    // each wave takes 16 panel columns at once (independent loads), lanes
    // over the rows below the panel
    for (int t0 = wave * 16; t0 < pw; t0 += nw * 16) {
      double acc[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) acc[u] = 0.0;
      for (int r = p1 + lane; r < f; r += 64) {
        const double xr = xv[r];
        const T* lr = L + (int64_t)(p0 + t0) * f + r;
#pragma unroll
        for (int u = 0; u < 16; ++u)
          if (t0 + u < pw) acc[u] += (double)lr[(int64_t)u * f] * xr;
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        double s = acc[u];
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
        if (lane == 0 && t0 + u < pw) xv[p0 + t0 + u] -= s;
      }
    }
    load_diag_block(L, f, p0, pw, type, blk);
    __syncthreads();
    if (wave == 0) {
      double vl = lane < pw ? xv[p0 + lane] : 0.0;
      for (int j = pw - 1; j >= 0; --j) {
        const double xj = __shfl(vl, j);
        if (lane < j) vl -= blk[j * (PB + 1) + lane] * xj;
      }
      if (lane < pw) xv[p0 + lane] = vl;
    }
    p1 = p0;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < k; t += blockDim.x) x[rows[sa.piv_perm[start + t]]] = xv[t];
}

template <class T>
__global__ void __launch_bounds__(256) bwd_kernel(SolveArgs sa, const T* pool,
                                                const int32_t* fronts, double* x) {
  extern __shared__ double smem[];
  bwd_front<T>(sa, pool, fronts[blockIdx.x], x, smem);
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
void set_solve_attrs() {
  static bool done = false;
  if (done) return;
  HIPCHECK(hipFuncSetAttribute((const void*)fwd_kernel<T>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, 159 * 1024));
  HIPCHECK(hipFuncSetAttribute((const void*)bwd_kernel<T>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, 159 * 1024));
  done = true;
}

// Level-by-level sweeps: one launch per tree level and direction.
template <class T>
void solve_levels(riga_problem* pr, const T* pool, const double* b, double* x, hipStream_t s) {
  SolveArgs sa = solve_args(pr);
  const int H = (int)pr->levels.size();
  for (int h = 0; h < H; ++h) {
    const LevelDev& L = pr->levels[h];
    if (L.n == 0) continue;
    fwd_kernel<T><<<L.n, 256, (size_t)(PB * (PB + 1) + L.max_f + L.max_k) * sizeof(double), s>>>(
        sa, pool, L.fronts.p, b);
  }
  for (int h = H - 1; h >= 0; --h) {
    const LevelDev& L = pr->levels[h];
    if (L.n == 0) continue;
    bwd_kernel<T><<<L.n, 256, (size_t)(PB * (PB + 1) + L.max_f) * sizeof(double), s>>>(
        sa, pool, L.fronts.p, x);
  }
  HIPCHECK(hipGetLastError());
}

}  // namespace

void solve_fb(riga_problem* pr, const double* b, double* x, hipStream_t s) {
  if (!pr->factored) throw Error(RIGA_EINVAL, "solve before factorisation");
  if (pr->fact_precision == RIGA_MIXED) {
    set_solve_attrs<float>();
    solve_levels<float>(pr, pr->pool32.p, b, x, s);
  } else {
    set_solve_attrs<double>();
    solve_levels<double>(pr, pr->pool64.p, b, x, s);
  }
}

}  // namespace riga
