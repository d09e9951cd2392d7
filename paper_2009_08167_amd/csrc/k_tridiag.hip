// Eigenpairs of the projected Lanczos matrix T_m (Eqs. LanczosTm,
// LanczosRitz, RitzValues of arXiv 2009.08167; "any method" for the
// symmetric tridiagonal eigenproblem is admissible, Sec. 4.2).
//
// One workgroup, FP64:
//  1. every eigenvalue by Sturm-count bisection (one thread per eigenvalue);
//  2. the `nvec` eigenvalues of largest |theta| -- the ones nearest the
//     shift after the spectral transformation -- are selected;
//  3. their eigenvectors by inverse iteration with a tridiagonal LU with
//     partial pivoting, one thread per cluster of close eigenvalues, the
//     members of a cluster Gram-Schmidt orthogonalised against each other at
//     every iteration.
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

__global__ void __launch_bounds__(512) tridiag_eig_kernel(const double* alpha, const double* beta,
                                                        int m, double* theta_out, double* S,
                                                        int nvec, int32_t* sel_out,
                                                        double* work) {
  __shared__ double a[TD_MAX], b2[TD_MAX], bb[TD_MAX], th[TD_MAX];
  __shared__ int sel[TD_MAX];
  __shared__ int cl_start[TD_MAX + 1];
  __shared__ int n_cl;
  __shared__ double s_lo[512], s_hi[512], s_bmax[512];
  const int tid = threadIdx.x, nt = blockDim.x;
  double lo = 1e300, hi = -1e300, bm = 0.0;
  for (int i = tid; i < m; i += nt) {
    a[i] = alpha[i];
    const double bi = i > 0 ? beta[i] : 0.0;
    const double bn = i + 1 < m ? beta[i + 1] : 0.0;
    bb[i] = bi;
    b2[i] = bi * bi;
    const double r = fabs(bi) + fabs(bn);
    lo = fmin(lo, alpha[i] - r);
    hi = fmax(hi, alpha[i] + r);
    bm = fmax(bm, bi * bi);
  }
  s_lo[tid] = lo;
  s_hi[tid] = hi;
  s_bmax[tid] = bm;
  __syncthreads();
  for (int w = nt / 2; w > 0; w >>= 1) {
    if (tid < w) {
      s_lo[tid] = fmin(s_lo[tid], s_lo[tid + w]);
      s_hi[tid] = fmax(s_hi[tid], s_hi[tid + w]);
      s_bmax[tid] = fmax(s_bmax[tid], s_bmax[tid + w]);
    }
    __syncthreads();
  }
  const double gl = s_lo[0], gu = s_hi[0];
  const double tnorm = fmax(fabs(gl), fabs(gu));
  const double pivmin = 2.2250738585072014e-308 * fmax(1.0, s_bmax[0]);
  const double eps = 2.220446049250313e-16;
  // widen the Gershgorin interval slightly
  const double wlo = gl - 2.0 * eps * tnorm - 2.0 * pivmin;
  const double whi = gu + 2.0 * eps * tnorm + 2.0 * pivmin;
  // ---- 1. bisection: eigenvalue index t in ascending order
  for (int t = tid; t < m; t += nt) {
    double l = wlo, h = whi;
    for (int it = 0; it < 200; ++it) {
      const double mid = 0.5 * (l + h);
      if (h - l <= 2.0 * eps * fmax(fabs(l), fabs(h)) + pivmin || mid == l || mid == h) break;
      int cnt = 0;
      double q = a[0] - mid;
      if (fabs(q) < pivmin) q = -pivmin;
      cnt += q < 0.0;
      for (int i = 1; i < m; ++i) {
        q = a[i] - mid - b2[i] / q;
        if (fabs(q) < pivmin) q = -pivmin;
        cnt += q < 0.0;
      }
      if (cnt <= t) l = mid; else h = mid;
    }
    th[t] = 0.5 * (l + h);
  }
  __syncthreads();
  for (int t = tid; t < m; t += nt) theta_out[t] = th[t];
  // ---- 2. selection of the nvec largest |theta|, then clusters
  if (tid == 0) {
    int l = 0, r = m - 1, c = 0;
    while (c < nvec && l <= r) {
      if (fabs(th[l]) >= fabs(th[r])) sel[c++] = l++;
      else sel[c++] = r--;
    }
    // ascending index order (insertion sort; c <= 1024, called rarely)
    for (int i = 1; i < c; ++i) {
      const int v = sel[i];
      int jj = i - 1;
      while (jj >= 0 && sel[jj] > v) { sel[jj + 1] = sel[jj]; --jj; }
      sel[jj + 1] = v;
    }
    int k = 0;
    cl_start[k++] = 0;
    for (int i = 1; i < c; ++i) {
      const double t0 = th[sel[i - 1]], t1 = th[sel[i]];
      const bool close = sel[i] == sel[i - 1] + 1 &&
                         fabs(t1 - t0) <= 1e-3 * fmax(fabs(t0), fabs(t1));
      if (!close) cl_start[k++] = i;
    }
    cl_start[k] = c;
    n_cl = k;
  }
  __syncthreads();
  for (int i = tid; i < nvec; i += nt) sel_out[i] = sel[i];
  // ---- 3. inverse iteration, one thread per cluster
  for (int c = tid; c < n_cl; c += nt) {
    double* dl = work + (int64_t)c * 6 * m;
    double* d = dl + m;
    double* du = d + m;
    double* du2 = du + m;
    double* piv = du2 + m;
    double* x = piv + m;
    double prev_shift = 0.0;
    for (int mem = cl_start[c]; mem < cl_start[c + 1]; ++mem) {
      const int idx = sel[mem];
      double shift = th[idx];
      if (mem > cl_start[c] && shift - prev_shift < 10.0 * eps * fabs(shift))
        shift = prev_shift + 10.0 * eps * fabs(shift);
      prev_shift = shift;
      // LU with partial pivoting of T - shift I
      for (int i = 0; i < m; ++i) {
        d[i] = a[i] - shift;
        if (i + 1 < m) { dl[i] = bb[i + 1]; du[i] = bb[i + 1]; }
        du2[i] = 0.0;
        piv[i] = 0.0;
      }
      const double tiny = eps * tnorm + pivmin;
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
      // start vector
      for (int i = 0; i < m; ++i) {
        const uint64_t h = mix64(0x5DEECE66Dull * (uint64_t)(idx + 1) + (uint64_t)i);
        x[i] = (double)(h >> 11) * (2.0 / 9007199254740992.0) - 1.0;
      }
      for (int it = 0; it < 5; ++it) {
        // solve (T - shift I) y = x in place
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
        // orthogonalise against the cluster members already computed (twice)
        for (int pass = 0; pass < 2; ++pass) {
          for (int o = cl_start[c]; o < mem; ++o) {
            const double* so = S + (int64_t)o * m;
            double dot = 0.0;
            for (int i = 0; i < m; ++i) dot += so[i] * x[i];
            for (int i = 0; i < m; ++i) x[i] -= dot * so[i];
          }
        }
        double nrm = 0.0;
        for (int i = 0; i < m; ++i) nrm += x[i] * x[i];
        nrm = sqrt(nrm);
        const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
        for (int i = 0; i < m; ++i) x[i] *= inv;
      }
      double* so = S + (int64_t)mem * m;
      for (int i = 0; i < m; ++i) so[i] = x[i];
    }
  }
}

}  // namespace

void launch_tridiag_eig(const double* alpha, const double* beta, int m, double* theta, double* S,
                        int nvec, int32_t* sel_out, double* work, hipStream_t s) {
  if (m > TD_MAX) throw Error(RIGA_EUNSUPPORTED, "Lanczos basis larger than 1024");
  if (nvec > m) nvec = m;
  tridiag_eig_kernel<<<1, 512, 0, s>>>(alpha, beta, m, theta, S, nvec,
                                       sel_out, work);
  HIPCHECK(hipGetLastError());
}

}  // namespace riga
