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

#include <mutex>

#include "problem.h"

namespace riga {
namespace {

struct SolveArgs {
  const FrontDesc* desc;   // packed per-front record
  const int32_t* gmap;     // per front position: children's update indices
  int gstride;             // children slots per position
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

// Value of `v` in lane `l` of the wave (l uniform): a scalar-register read,
// far cheaper than an LDS permute on the serial path of the panel solves.
__device__ __forceinline__ double lane_value(double v, int l) {
  const long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(bits & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Loads the diagonal block L(p0:p0+pw, p0:p0+pw) (unit lower, strict part)
// into LDS `blk` (row-major, ld PB+1), zeroing the D entry of 2x2 pivot
// blocks, which is not part of L.  Each thread issues all its loads before
// its first LDS store, so the loads are in flight together.
template <class T, int NT>
__device__ __forceinline__ void load_diag_block(const T* L, int f, int p0, int pw,
                                                const int32_t* type, double* blk) {
  constexpr int PER = PB * PB / NT;
  double v[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = threadIdx.x + u * NT;
    const int c = e / PB, r = e % PB;
    v[u] = (r < pw && c < pw && r > c) ? (double)L[(int64_t)(p0 + c) * f + p0 + r] : 0.0;
  }
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = threadIdx.x + u * NT;
    const int c = e / PB, r = e % PB;
    if (r == c + 1 && c < pw && type[p0 + c] == 2) v[u] = 0.0;
    blk[r * (PB + 1) + c] = v[u];
  }
}

// Work split of the panel updates: NT threads = 256 row lanes x CG column
// groups (CG = NT / 256), so that a big front's workgroup keeps NT loads in
// flight; partial sums of the column groups are added in a fixed order.
template <class T, int NT>
__device__ void fwd_front(const SolveArgs& sa, const T* pool, int F, const double* b,
                          double* smem) {
  constexpr int CG = NT / 256;
  double* blk = smem;                     // PB x (PB+1)
  double* y = smem + PB * (PB + 1);       // f
  const FrontDesc d = sa.desc[F];
  const int f = d.f, k = d.k, start = d.start;
  const T* L = pool + d.pool_off;
  const int32_t* rows = sa.rows + d.rows_off;
  const int32_t* gm = sa.gmap + d.gmap_off;
  double* z = y + f;                      // k (permutation scratch)
  double* psum = z + k;                   // CG x 256 partial sums (CG > 1)
  int32_t* type = (int32_t*)(psum + (CG > 1 ? CG * 256 : 0));  // k pivot types
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // gather: own right-hand side entries plus the children's updates (all
  // index loads first, then the values), pivot types to LDS
  for (int i = threadIdx.x; i < f; i += blockDim.x) {
    const int ri = i < k ? rows[i] : -1;
    int g[4];
#pragma unroll
    for (int sl = 0; sl < 4; ++sl) g[sl] = sl < sa.gstride ? gm[(int64_t)i * sa.gstride + sl] : -1;
    double v = ri >= 0 ? b[ri] : 0.0;
#pragma unroll
    for (int sl = 0; sl < 4; ++sl)
      if (g[sl] >= 0) v += sa.cbvec[g[sl]];
    y[i] = v;
  }
  for (int t = threadIdx.x; t < k; t += blockDim.x) type[t] = sa.piv_type[start + t];
  __syncthreads();
  for (int t = threadIdx.x; t < k; t += blockDim.x) z[t] = y[sa.piv_perm[start + t]];
  __syncthreads();
  for (int t = threadIdx.x; t < k; t += blockDim.x) y[t] = z[t];
  // panels of the fully-summed block; a 2x2 pivot block never straddles two
  int p0 = 0;
  while (p0 < k) {
    int pw = min(PB, k - p0);
    if (pw > 1 && p0 + pw < k && type[p0 + pw - 1] == 2) --pw;
    __syncthreads();
    load_diag_block<T, NT>(L, f, p0, pw, type, blk);
    __syncthreads();
    if (wave == 0) {
      double yl = lane < pw ? y[p0 + lane] : 0.0;
#pragma unroll 8
      for (int t = 0; t < pw; ++t) {
        const double lt = blk[lane * (PB + 1) + t];
        const double zt = lane_value(yl, t);
        if (lane > t) yl -= lt * zt;
      }
      if (lane < pw) y[p0 + lane] = yl;
    }
    __syncthreads();
    // rows below the panel: y_r -= L(r, panel) z_panel, 16 loads in flight
    // per thread; column group cg takes panel columns [cg*cw, (cg+1)*cw);
    // rows go in chunks of 256, the groups' partial sums are added in a
    // fixed order
    {
      const int rl = threadIdx.x & 255, cg = threadIdx.x >> 8;
      const int cw = (pw + CG - 1) / CG;
      const int c0 = min(pw, cg * cw), c1 = min(pw, c0 + cw);
      for (int rb = p0 + pw; rb < f; rb += 256) {
        const int r = rb + rl;
        double s = 0.0;
        if (r < f) {
          const T* lr = L + (int64_t)p0 * f + r;
          int t = c0;
          for (; t + 16 <= c1; t += 16) {
            double lv[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) lv[u] = (double)lr[(int64_t)(t + u) * f];
#pragma unroll
            for (int u = 0; u < 16; ++u) s += lv[u] * y[p0 + t + u];
          }
          for (; t < c1; ++t) s += (double)lr[(int64_t)t * f] * y[p0 + t];
        }
        if (CG == 1) {
          if (r < f) y[r] -= s;
        } else {
          psum[cg * 256 + rl] = s;
          __syncthreads();
          if (cg == 0 && r < f) {
            double tot = 0.0;
#pragma unroll
            for (int g = 0; g < CG; ++g) tot += psum[g * 256 + rl];
            y[r] -= tot;
          }
          __syncthreads();
        }
      }
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
  for (int c = threadIdx.x; c < f - k; c += blockDim.x) sa.cbvec[d.cb_off + c] = y[k + c];
}

template <class T, int NT>
__global__ void __launch_bounds__(NT) fwd_kernel(SolveArgs sa, const T* pool,
                                               const int32_t* fronts, const double* b) {
  extern __shared__ double smem[];
  fwd_front<T, NT>(sa, pool, fronts[blockIdx.x], b, smem);
}

template <class T, int NT>
__device__ void bwd_front(const SolveArgs& sa, const T* pool, int F, double* x, double* smem) {
  constexpr int RG = NT / 256;            // row groups of the panel products
  double* blk = smem;                     // PB x (PB+1)
  double* xv = smem + PB * (PB + 1);      // f: v/x of the FS block, then x_CB
  const FrontDesc d = sa.desc[F];
  const int f = d.f, k = d.k, start = d.start;
  double* psum = xv + f;                  // RG x PB partial sums
  int32_t* type = (int32_t*)(psum + RG * PB);  // k pivot types
  const T* L = pool + d.pool_off;
  const int32_t* rows = sa.rows + d.rows_off;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int c = threadIdx.x; c < f - k; c += blockDim.x) xv[k + c] = x[rows[k + c]];
  for (int t = threadIdx.x; t < k; t += blockDim.x) {
    xv[t] = sa.fwd[start + t];
    type[t] = sa.piv_type[start + t];
  }
  __syncthreads();
  // panels from the bottom: v_panel -= L(below, panel)^T x_below, then the
  // transposed unit-triangular solve of the diagonal block
  int p1 = k;
  while (p1 > 0) {
    int p0 = max(0, p1 - PB);
    if (p0 > 0 && type[p0] == 3) ++p0;   // keep 2x2 pivot blocks whole
    const int pw = p1 - p0;
    __syncthreads();
    // waves: 4 column groups of 16 panel columns x RG row groups; 16 loads
    // in flight per lane; row-group partial sums added in a fixed order
    {
      const int cgi = wave & 3, rg = wave >> 2;
      const int t0 = cgi * 16;
      double acc[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) acc[u] = 0.0;
      if (t0 < pw) {
        for (int r = p1 + rg * 64 + lane; r < f; r += 64 * RG) {
          const double xr = xv[r];
          const T* lr = L + (int64_t)(p0 + t0) * f + r;
#pragma unroll
          for (int u = 0; u < 16; ++u)
            if (t0 + u < pw) acc[u] += (double)lr[(int64_t)u * f] * xr;
        }
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        double s = acc[u];
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
        if (lane == 0 && t0 + u < pw) {
          if (RG == 1) xv[p0 + t0 + u] -= s;
          else psum[rg * PB + t0 + u] = s;
        }
      }
      if (RG > 1) {
        __syncthreads();
        for (int t = threadIdx.x; t < pw; t += NT) {
          double s = 0.0;
#pragma unroll
          for (int g = 0; g < RG; ++g) s += psum[g * PB + t];
          xv[p0 + t] -= s;
        }
      }
    }
    load_diag_block<T, NT>(L, f, p0, pw, type, blk);
    __syncthreads();
    if (wave == 0) {
      double vl = lane < pw ? xv[p0 + lane] : 0.0;
#pragma unroll 8
      for (int j = pw - 1; j >= 0; --j) {
        const double lj = blk[j * (PB + 1) + lane];
        const double xj = lane_value(vl, j);
        if (lane < j) vl -= lj * xj;
      }
      if (lane < pw) xv[p0 + lane] = vl;
    }
    p1 = p0;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < k; t += blockDim.x) x[rows[sa.piv_perm[start + t]]] = xv[t];
}

template <class T, int NT>
__global__ void __launch_bounds__(NT) bwd_kernel(SolveArgs sa, const T* pool,
                                               const int32_t* fronts, double* x) {
  extern __shared__ double smem[];
  bwd_front<T, NT>(sa, pool, fronts[blockIdx.x], x, smem);
}

SolveArgs solve_args(riga_problem* pr) {
  SolveArgs sa{};
  sa.desc = pr->d_desc.p;
  sa.gmap = pr->d_gmap.p;
  sa.gstride = pr->gstride;
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

// Fronts above this order use 1024-thread workgroups in the sweeps.
constexpr int SOLVE_BIG_F = 256;

template <class T>
void apply_solve_attrs() {
  const void* ks[] = {(const void*)fwd_kernel<T, 256>, (const void*)fwd_kernel<T, 1024>,
                      (const void*)bwd_kernel<T, 256>, (const void*)bwd_kernel<T, 1024>};
  for (const void* k : ks)
    HIPCHECK(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, 159 * 1024));
}

template <class T>
void set_solve_attrs() {
  static std::once_flag once;
  std::call_once(once, [] { set_kernel_attributes(); });
}

// Level-by-level sweeps: per tree level and direction one launch for the
// fronts of order <= SOLVE_BIG_F (256 threads each) and one for the larger
// ones (1024 threads each).
template <class T>
void solve_levels(riga_problem* pr, const T* pool, const double* b, double* x, hipStream_t s) {
  SolveArgs sa = solve_args(pr);
  const int H = (int)pr->levels.size();
  for (int h = 0; h < H; ++h) {
    const LevelDev& L = pr->levels[h];
    if (L.n == 0) continue;
    const int ns = L.n_upto(SOLVE_BIG_F);
    const int fs = ns > 0 ? L.host_f[ns - 1] : 0;
    if (ns > 0)
      fwd_kernel<T, 256><<<ns, 256, (size_t)(PB * (PB + 1) + fs + fs + fs / 2 + 1) * sizeof(double), s>>>(
          sa, pool, L.fronts.p, b);
    if (L.n > ns)
      fwd_kernel<T, 1024><<<L.n - ns, 1024,
                            (size_t)(PB * (PB + 1) + 2 * L.max_f + 4 * 256 + L.max_f / 2 + 1) * sizeof(double), s>>>(
          sa, pool, L.fronts.p + ns, b);
  }
  for (int h = H - 1; h >= 0; --h) {
    const LevelDev& L = pr->levels[h];
    if (L.n == 0) continue;
    const int ns = L.n_upto(SOLVE_BIG_F);
    const int fs = ns > 0 ? L.host_f[ns - 1] : 0;
    if (ns > 0)
      bwd_kernel<T, 256><<<ns, 256, (size_t)(PB * (PB + 1) + fs + PB + fs / 2 + 1) * sizeof(double), s>>>(
          sa, pool, L.fronts.p, x);
    if (L.n > ns)
      bwd_kernel<T, 1024><<<L.n - ns, 1024,
                            (size_t)(PB * (PB + 1) + L.max_f + 4 * PB + L.max_f / 2 + 1) * sizeof(double), s>>>(
          sa, pool, L.fronts.p + ns, x);
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
  if (pr->fact_precision == RIGA_MIXED) {
    set_solve_attrs<float>();
    solve_levels<float>(pr, pr->pool32.p, b, x, s);
  } else {
    set_solve_attrs<double>();
    solve_levels<double>(pr, pr->pool64.p, b, x, s);
  }
}

}  // namespace riga
