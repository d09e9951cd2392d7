// Eigenpairs of the projected Lanczos matrix T_m (Eqs. LanczosTm,
// LanczosRitz, RitzValues of arXiv 2009.08167; "any method" for the
// symmetric tridiagonal eigenproblem is admissible, Sec. 4.2).
//
// Two kernels, FP64:
//  ritz_check: every eigenvalue by Sturm-count multisection (one wave per
//     eigenvalue) and the last component of its unit eigenvector from a
//     twisted factorisation; the Ritz estimate of Eq. Lanczos is
//     |beta_{m+1} s_m|.  Used at every convergence check.
//  ritz_vectors: eigenvectors of the eigenvalues the host selected, by
//     inverse iteration with a tridiagonal LU with partial pivoting, one
//     wave per cluster of close eigenvalues, the members of a cluster
//     Gram-Schmidt orthogonalised against each other at every iteration.
//     Used once per Lanczos run.
#include <hip/hip_runtime.h>

#include <cmath>

#include "problem.h"

namespace riga {
namespace {

constexpr int TD_MAX = 1024;

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

struct Bounds {
  double lo, hi, tnorm, pivmin;
};

// Gershgorin interval, norm and pivot floor of T (computed per thread).
__device__ Bounds tridiag_bounds(const double* a, const double* b, int m) {
  double lo = 1e300, hi = -1e300, bm = 0.0;
  for (int i = 0; i < m; ++i) {
    const double bi = i > 0 ? b[i] : 0.0;
    const double bn = i + 1 < m ? b[i + 1] : 0.0;
    const double r = fabs(bi) + fabs(bn);
    lo = fmin(lo, a[i] - r);
    hi = fmax(hi, a[i] + r);
    bm = fmax(bm, bi * bi);
  }
  Bounds B;
  B.tnorm = fmax(fabs(lo), fabs(hi));
  B.pivmin = 2.2250738585072014e-308 * fmax(1.0, bm);
  const double eps = 2.220446049250313e-16;
  B.lo = lo - 2.0 * eps * B.tnorm - 2.0 * B.pivmin;
  B.hi = hi + 2.0 * eps * B.tnorm + 2.0 * B.pivmin;
  return B;
}

// Number of eigenvalues of T below x (Sturm count of the LDL^T pivots).
__device__ __forceinline__ int sturm_count(const double* a, const double* b, int m, double x,
                                           double pivmin) {
  int cnt = 0;
  double q = a[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  cnt += q < 0.0;
  for (int i = 1; i < m; ++i) {
    q = a[i] - x - b[i] * b[i] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += q < 0.0;
  }
  return cnt;
}

// The t-th smallest eigenvalue, one wave: multisection of the bracket into 65
// parts per step (each lane one Sturm count), down to a relative width of
// 2 eps.
__device__ double multisect(const double* a, const double* b, int m, int t, const Bounds& B,
                            int lane) {
  const double eps = 2.220446049250313e-16;
  double l = B.lo, h = B.hi;
  for (int it = 0; it < 64; ++it) {
    if (h - l <= 2.0 * eps * fmax(fabs(l), fabs(h)) + B.pivmin) break;
    const double w = h - l;
    const double x = l + w * (double)(lane + 1) / 65.0;
    const int cnt = sturm_count(a, b, m, x, B.pivmin);
    const unsigned long long above = __ballot(cnt > t);
    double nl, nh;
    if (above == 0ull) {
      nl = l + w * 64.0 / 65.0;
      nh = h;
    } else {
      const int first = __ffsll((long long)above) - 1;
      nh = l + w * (double)(first + 1) / 65.0;
      nl = first > 0 ? l + w * (double)first / 65.0 : l;
    }
    if (nl == l && nh == h) break;
    l = nl;
    h = nh;
  }
  return 0.5 * (l + h);
}

// Ritz values and estimates, one wave per eigenvalue t of T_m (two per
// workgroup).  The estimate needs the last component s_m of the unit
// eigenvector, from a twisted factorisation of T - theta I: bottom-up
// T - theta I = U D- U^T (lane 0) and top-down L D+ L^T (lane 1) in LDS, twist
// index r = argmin |gamma_k|, gamma_k = D+_k + D-_k - (a_k - theta) (the
// eigenvector's largest entry, which makes the twisted solve stable).  With
// x_r = 1: x_i = -l_i x_{i+1} above r, x_{i+1} = -u_i x_i below r, so
// ||x||^2 = Q+_r + P-_r - 1 and x_m = R-_r.  est = |beta_{m+1} s_m|.
__global__ void __launch_bounds__(128) ritz_check_kernel(const double* alpha, const double* beta,
                                                       int m, double* theta_out, double* est,
                                                       const int32_t* flag, double* extra) {
  extern __shared__ double sm[];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    extra[0] = beta[m];
    extra[1] = (double)flag[0];
  }
  double* a = sm;
  double* b = sm + m;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double* Dm = sm + 2 * m + (size_t)wave * 5 * m;
  double* Pm = Dm + m;
  double* Rm = Pm + m;
  double* Dp = Rm + m;
  double* Qp = Dp + m;
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    a[i] = alpha[i];
    b[i] = i > 0 ? beta[i] : 0.0;
  }
  __syncthreads();
  const int t = blockIdx.x * 2 + wave;
  const bool active = t < m;
  const Bounds B = tridiag_bounds(a, b, m);
  const double th = active ? multisect(a, b, m, t, B, lane) : 0.0;
  const double big = 1e300;
  if (active && lane == 0) {
    double dm = a[m - 1] - th, pm = 1.0, rm = 1.0;
    Dm[m - 1] = dm;
    Pm[m - 1] = pm;
    Rm[m - 1] = rm;
    for (int k = m - 2; k >= 0; --k) {
      if (fabs(dm) < B.pivmin) dm = dm < 0.0 ? -B.pivmin : B.pivmin;
      const double u = b[k + 1] / dm;
      dm = a[k] - th - u * b[k + 1];
      pm = fmin(1.0 + u * u * pm, big);
      rm = fmax(fmin(-u * rm, big), -big);
      Dm[k] = dm;
      Pm[k] = pm;
      Rm[k] = rm;
    }
  } else if (active && lane == 1) {
    double dp = a[0] - th, qp = 1.0;
    for (int k = 0; k < m; ++k) {
      Dp[k] = dp;
      Qp[k] = qp;
      if (k + 1 < m) {
        if (fabs(dp) < B.pivmin) dp = dp < 0.0 ? -B.pivmin : B.pivmin;
        const double l = b[k + 1] / dp;
        dp = a[k + 1] - th - l * b[k + 1];
        qp = fmin(1.0 + l * l * qp, big);
      }
    }
  }
  __syncthreads();
  if (!active) return;
  double best = 1e308;
  int r = m;
  for (int k = lane; k < m; k += 64) {
    const double g = fabs(Dp[k] + Dm[k] - (a[k] - th));
    if (g < best) { best = g; r = k; }
  }
  for (int off = 32; off > 0; off >>= 1) {
    const double ob = __shfl_xor(best, off);
    const int orr = __shfl_xor(r, off);
    if (ob < best || (ob == best && orr < r)) { best = ob; r = orr; }
  }
  if (lane == 0) {
    const double nrm2 = Qp[r] + Pm[r] - 1.0;
    theta_out[t] = th;
    est[t] = fabs(beta[m]) * fabs(Rm[r]) / sqrt(fmax(nrm2, 1.0));
  }
}

// Eigenvectors of selected eigenvalues by inverse iteration, one wave per
// cluster of close eigenvalues (relative gap below 1e-3, adjacent indices):
// LU with partial pivoting of T - shift I and the solves run on lane 0 with
// the work arrays in LDS; start vector, Gram-Schmidt against the cluster's
// earlier members (twice) and normalisation use all lanes.  Members of a
// cluster get shifts at least 10 eps apart.
__global__ void __launch_bounds__(64) ritz_vectors_kernel(const double* alpha, const double* beta,
                                                        int m, const double* theta,
                                                        const int32_t* sel,
                                                        const int32_t* cl_start, double* S) {
  extern __shared__ double sm[];
  double* a = sm;
  double* bb = a + m;
  double* dl = bb + m;
  double* d = dl + m;
  double* du = d + m;
  double* du2 = du + m;
  double* piv = du2 + m;
  double* x = piv + m;
  const int lane = threadIdx.x;
  for (int i = lane; i < m; i += 64) {
    a[i] = alpha[i];
    bb[i] = i > 0 ? beta[i] : 0.0;
  }
  __syncthreads();
  const Bounds B = tridiag_bounds(a, bb, m);
  const double eps = 2.220446049250313e-16;
  const double tiny = eps * B.tnorm + B.pivmin;
  const int c0 = cl_start[blockIdx.x], c1 = cl_start[blockIdx.x + 1];
  double prev_shift = 0.0;
  for (int mem = c0; mem < c1; ++mem) {
    const int idx = sel[mem];
    double shift = theta[idx];
    if (mem > c0 && shift - prev_shift < 10.0 * eps * fabs(shift))
      shift = prev_shift + 10.0 * eps * fabs(shift);
    prev_shift = shift;
    for (int i = lane; i < m; i += 64) {
      d[i] = a[i] - shift;
      dl[i] = i + 1 < m ? bb[i + 1] : 0.0;
      du[i] = dl[i];
      du2[i] = 0.0;
      piv[i] = 0.0;
      const uint64_t hsh = mix64(0x5DEECE66Dull * (uint64_t)(idx + 1) + (uint64_t)i);
      x[i] = (double)(hsh >> 11) * (2.0 / 9007199254740992.0) - 1.0;
    }
    __syncthreads();
    if (lane == 0) {
      for (int i = 0; i + 1 < m; ++i) {
        if (fabs(d[i]) >= fabs(dl[i])) {
          if (d[i] == 0.0) d[i] = tiny;
          const double fct = dl[i] / d[i];
          dl[i] = fct;
          d[i + 1] -= fct * du[i];
        } else {
          const double fct = d[i] / dl[i];
          d[i] = dl[i];
          dl[i] = fct;
          const double tmp = du[i];
          du[i] = d[i + 1];
          d[i + 1] = tmp - fct * d[i + 1];
          if (i + 2 < m) {
            du2[i] = du[i + 1];
            du[i + 1] = -fct * du[i + 1];
          }
          piv[i] = 1.0;
        }
      }
      if (d[m - 1] == 0.0) d[m - 1] = tiny;
    }
    __syncthreads();
    for (int it = 0; it < 4; ++it) {
      if (lane == 0) {
        for (int i = 0; i + 1 < m; ++i) {
          if (piv[i] != 0.0) {
            const double t0 = x[i];
            x[i] = x[i + 1];
            x[i + 1] = t0 - dl[i] * x[i];
          } else {
            x[i + 1] -= dl[i] * x[i];
          }
        }
        x[m - 1] /= d[m - 1];
        if (m >= 2) x[m - 2] = (x[m - 2] - du[m - 2] * x[m - 1]) / d[m - 2];
        for (int i = m - 3; i >= 0; --i)
          x[i] = (x[i] - du[i] * x[i + 1] - du2[i] * x[i + 2]) / d[i];
      }
      __syncthreads();
      for (int pass = 0; pass < 2; ++pass) {
        for (int o = c0; o < mem; ++o) {
          const double* so = S + (int64_t)o * m;
          double dot = 0.0;
          for (int i = lane; i < m; i += 64) dot += so[i] * x[i];
          for (int off = 32; off > 0; off >>= 1) dot += __shfl_xor(dot, off);
          for (int i = lane; i < m; i += 64) x[i] -= dot * so[i];
          __syncthreads();
        }
      }
      double nrm = 0.0;
      for (int i = lane; i < m; i += 64) nrm += x[i] * x[i];
      for (int off = 32; off > 0; off >>= 1) nrm += __shfl_xor(nrm, off);
      const double inv = nrm > 0.0 ? 1.0 / sqrt(nrm) : 0.0;
      for (int i = lane; i < m; i += 64) x[i] *= inv;
      __syncthreads();
    }
    double* so = S + (int64_t)mem * m;
    for (int i = lane; i < m; i += 64) so[i] = x[i];
    __syncthreads();
  }
}

}  // namespace

void launch_ritz_check(const double* alpha, const double* beta, int m, double* theta, double* est,
                       const int32_t* flag, double* extra, hipStream_t s) {
  if (m > TD_MAX) throw Error(RIGA_EUNSUPPORTED, "Lanczos basis larger than 1024");
  const size_t lds = (size_t)12 * m * sizeof(double);
  ritz_check_kernel<<<(m + 1) / 2, 128, lds, s>>>(alpha, beta, m, theta, est, flag, extra);
  HIPCHECK(hipGetLastError());
}

void launch_ritz_vectors(const double* alpha, const double* beta, int m, const double* theta,
                         const int32_t* sel, const int32_t* cl_start, int ncl, double* S,
                         hipStream_t s) {
  if (m > TD_MAX) throw Error(RIGA_EUNSUPPORTED, "Lanczos basis larger than 1024");
  if (ncl <= 0) return;
  const size_t lds = (size_t)8 * m * sizeof(double);
  ritz_vectors_kernel<<<ncl, 64, lds, s>>>(alpha, beta, m, theta, sel, cl_start, S);
  HIPCHECK(hipGetLastError());
}

void set_tridiag_attributes() {
  HIPCHECK(hipFuncSetAttribute((const void*)ritz_check_kernel,
                               hipFuncAttributeMaxDynamicSharedMemorySize, 12 * TD_MAX * (int)sizeof(double)));
  HIPCHECK(hipFuncSetAttribute((const void*)ritz_vectors_kernel,
                               hipFuncAttributeMaxDynamicSharedMemorySize, 8 * TD_MAX * (int)sizeof(double)));
}

}  // namespace riga
