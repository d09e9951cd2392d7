// Eigenpairs of the projected Lanczos matrix T_m (Eqs. LanczosTm,
// LanczosRitz, RitzValues of arXiv 2009.08167; "any method" for the
// symmetric tridiagonal eigenproblem is admissible, Sec. 4.2).
//
// Two kernels, FP64:
//  ritz_check: every eigenvalue by Sturm-count bisection (one thread per
//     eigenvalue) and the last component of its unit eigenvector from the
//     top-down factorisation T - theta I = L D L^T: the eigenvector with
//     x_m = 1 satisfies x_i = -l_i x_{i+1}, so ||x||^2 follows from one
//     forward recurrence without storage, and |s_m| = 1/||x||.  The Ritz
//     estimate of Eq. Lanczos is |beta_{m+1} s_m|.  Used at every
//     convergence check.
//  ritz_vectors: eigenvectors of the eigenvalues the host selected, by
//     inverse iteration with a tridiagonal LU with partial pivoting, one
//     thread per cluster of close eigenvalues, the members of a cluster
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

// The t-th smallest eigenvalue by bisection on the Sturm count.
__device__ double bisect(const double* a, const double* b, int m, int t, const Bounds& B) {
  const double eps = 2.220446049250313e-16;
  double l = B.lo, h = B.hi;
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (l + h);
    if (h - l <= 2.0 * eps * fmax(fabs(l), fabs(h)) + B.pivmin || mid == l || mid == h) break;
    int cnt = 0;
    double q = a[0] - mid;
    if (fabs(q) < B.pivmin) q = -B.pivmin;
    cnt += q < 0.0;
    for (int i = 1; i < m; ++i) {
      q = a[i] - mid - b[i] * b[i] / q;
      if (fabs(q) < B.pivmin) q = -B.pivmin;
      cnt += q < 0.0;
    }
    if (cnt <= t) l = mid; else h = mid;
  }
  return 0.5 * (l + h);
}

// Ritz estimate of eigenvalue t from a twisted factorisation of
// T - theta I: bottom-up T - theta I = U D- U^T and top-down = L D+ L^T,
// twist index r = argmin |gamma_k|, gamma_k = D+_k + D-_k - (a_k - theta)
// (the eigenvector's largest entry, which makes the twisted solve stable).
// With x_r = 1: x_i = -l_i x_{i+1} above r, x_{i+1} = -u_i x_i below r, so
// ||x||^2 = Q+_r + P-_r - 1 and x_m = R-_r from the running sums below.
// Per-thread streams (D-, P-, R-) are stored interleaved across threads so
// that a wave's accesses are coalesced.
__global__ void __launch_bounds__(64) ritz_check_kernel(const double* alpha, const double* beta,
                                                      int m, double* theta_out, double* est,
                                                      double* work, int nthreads) {
  __shared__ double a[TD_MAX], b[TD_MAX];
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    a[i] = alpha[i];
    b[i] = i > 0 ? beta[i] : 0.0;
  }
  __syncthreads();
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m) return;
  const Bounds B = tridiag_bounds(a, b, m);
  const double th = bisect(a, b, m, t, B);
  const double big = 1e300;
  double* Dm = work;
  double* Pm = work + (int64_t)m * nthreads;
  double* Rm = work + 2 * (int64_t)m * nthreads;
  auto at = [&](int k) { return (int64_t)k * nthreads + t; };
  // bottom-up
  double dm = a[m - 1] - th, pm = 1.0, rm = 1.0;
  Dm[at(m - 1)] = dm;
  Pm[at(m - 1)] = pm;
  Rm[at(m - 1)] = rm;
  for (int k = m - 2; k >= 0; --k) {
    if (fabs(dm) < B.pivmin) dm = dm < 0.0 ? -B.pivmin : B.pivmin;
    const double u = b[k + 1] / dm;
    dm = a[k] - th - u * b[k + 1];
    pm = fmin(1.0 + u * u * pm, big);
    rm = fmax(fmin(-u * rm, big), -big);
    Dm[at(k)] = dm;
    Pm[at(k)] = pm;
    Rm[at(k)] = rm;
  }
  // top-down with the twist search
  double dp = a[0] - th, qp = 1.0;
  double best = 1e308, nrm2 = 1.0, xm = 1.0;
  for (int k = 0; k < m; ++k) {
    const double dmk = Dm[at(k)];
    const double g = dp + dmk - (a[k] - th);
    if (fabs(g) < best) {
      best = fabs(g);
      nrm2 = qp + Pm[at(k)] - 1.0;
      xm = Rm[at(k)];
    }
    if (k + 1 < m) {
      if (fabs(dp) < B.pivmin) dp = dp < 0.0 ? -B.pivmin : B.pivmin;
      const double l = b[k + 1] / dp;
      dp = a[k + 1] - th - l * b[k + 1];
      qp = fmin(1.0 + l * l * qp, big);
    }
  }
  theta_out[t] = th;
  est[t] = fabs(beta[m]) * fabs(xm) / sqrt(fmax(nrm2, 1.0));
}

__global__ void __launch_bounds__(256) ritz_vectors_kernel(const double* alpha, const double* beta,
                                                         int m, const double* theta,
                                                         const int32_t* sel, int nsel, double* S,
                                                         double* work) {
  __shared__ double a[TD_MAX], bb[TD_MAX];
  __shared__ int cl_start[TD_MAX + 1];
  __shared__ int n_cl;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int i = tid; i < m; i += nt) {
    a[i] = alpha[i];
    bb[i] = i > 0 ? beta[i] : 0.0;
  }
  __syncthreads();
  const Bounds B = tridiag_bounds(a, bb, m);
  const double eps = 2.220446049250313e-16;
  const double tnorm = B.tnorm, pivmin = B.pivmin;
  if (tid == 0) {
    // clusters of adjacent selected eigenvalues closer than 1e-3 relative
    int k = 0;
    cl_start[k++] = 0;
    for (int i = 1; i < nsel; ++i) {
      const double t0 = theta[sel[i - 1]], t1 = theta[sel[i]];
      const bool close = sel[i] == sel[i - 1] + 1 &&
                         fabs(t1 - t0) <= 1e-3 * fmax(fabs(t0), fabs(t1));
      if (!close) cl_start[k++] = i;
    }
    cl_start[k] = nsel;
    n_cl = k;
  }
  __syncthreads();
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
      double shift = theta[idx];
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

void launch_ritz_check(const double* alpha, const double* beta, int m, double* theta, double* est,
                       double* work, hipStream_t s) {
  if (m > TD_MAX) throw Error(RIGA_EUNSUPPORTED, "Lanczos basis larger than 1024");
  const int nb = (m + 63) / 64;
  ritz_check_kernel<<<nb, 64, 0, s>>>(alpha, beta, m, theta, est, work, nb * 64);
  HIPCHECK(hipGetLastError());
}

void launch_ritz_vectors(const double* alpha, const double* beta, int m, const double* theta,
                         const int32_t* sel, int nsel, double* S, double* work, hipStream_t s) {
  if (m > TD_MAX) throw Error(RIGA_EUNSUPPORTED, "Lanczos basis larger than 1024");
  if (nsel <= 0) return;
  ritz_vectors_kernel<<<1, 256, 0, s>>>(alpha, beta, m, theta, sel, nsel, S, work);
  HIPCHECK(hipGetLastError());
}

}  // namespace riga
