// Sparse mat-vec and the dense vector kernels of the Lanczos recurrence
// (Eqs. Lanczos--LanczosAlphaBeta of arXiv 2009.08167, with full
// M-reorthogonalisation, Eq. LanczosRestart and the paragraph after it).
//
// All reductions are two-stage with a fixed summation order, so results are
// bitwise reproducible from run to run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include <vector>

#include "problem.h"

namespace riga {
namespace {

// y = A x with CSR (G lanes per row, grid-stride over row groups); with
// dot_partial, also one partial of x^T y per workgroup (fixed order).
template <int G>
__global__ void __launch_bounds__(256) spmv_kernel(const int64_t* __restrict__ row_ptr,
                                                 const int32_t* __restrict__ col,
                                                 const double* __restrict__ val,
                                                 const double* __restrict__ x,
                                                 double* __restrict__ y, int64_t N,
                                                 double* dot_partial) {
  __shared__ double red[256 / G];
  const int sub = threadIdx.x % G;
  double d = 0.0;
  for (int64_t r0 = (int64_t)blockIdx.x * (256 / G); r0 < N; r0 += (int64_t)gridDim.x * (256 / G)) {
    const int64_t r = r0 + threadIdx.x / G;
    double s = 0.0;
    if (r < N) {
      // four entries per thread in flight: indices and values first, then
      // the gathers of x (a masked entry reads x[0] with value 0)
      const int64_t e1 = row_ptr[r + 1];
      for (int64_t eb = row_ptr[r] + sub; eb < e1; eb += 4 * G) {
        int c[4];
        double v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int64_t e = eb + q * G;
          const bool ok = e < e1;
          c[q] = ok ? col[e] : 0;
          v[q] = ok ? val[e] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) s += v[q] * x[c[q]];
      }
    }
    for (int off = G / 2; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (sub == 0 && r < N) {
      y[r] = s;
      d += s * x[r];
    }
  }
  if (dot_partial) {
    if (sub == 0) red[threadIdx.x / G] = d;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int i = 0; i < 256 / G; ++i) t += red[i];
      dot_partial[blockIdx.x] = t;
    }
  }
}

// KU = K U and MU = M U for NV columns of U per workgroup row (CSR pattern
// and both value arrays read once per NV columns), G lanes per row.
template <int G, int NV>
__global__ void __launch_bounds__(256) spmm_km_kernel(const int64_t* __restrict__ row_ptr,
                                                    const int32_t* __restrict__ col,
                                                    const double* __restrict__ kv,
                                                    const double* __restrict__ mv,
                                                    const double* __restrict__ U, int nw,
                                                    double* __restrict__ KU,
                                                    double* __restrict__ MU, int64_t N) {
  const int sub = threadIdx.x % G;
  const int64_t r = (int64_t)blockIdx.x * (256 / G) + threadIdx.x / G;
  const int v0 = blockIdx.y * NV;
  double sk[NV], sm[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) sk[q] = sm[q] = 0.0;
  if (r < N) {
    const int64_t e1 = row_ptr[r + 1];
    for (int64_t e = row_ptr[r] + sub; e < e1; e += G) {
      const int64_t c = col[e];
      const double a = kv[e], b = mv[e];
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        const double xv = v0 + q < nw ? U[(int64_t)(v0 + q) * N + c] : 0.0;
        sk[q] += a * xv;
        sm[q] += b * xv;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < NV; ++q)
    for (int off = G / 2; off > 0; off >>= 1) {
      sk[q] += __shfl_xor(sk[q], off);
      sm[q] += __shfl_xor(sm[q], off);
    }
  if (sub == 0 && r < N) {
#pragma unroll
    for (int q = 0; q < NV; ++q)
      if (v0 + q < nw) {
        KU[(int64_t)(v0 + q) * N + r] = sk[q];
        MU[(int64_t)(v0 + q) * N + r] = sm[q];
      }
  }
}

__global__ void axpby_vals_kernel(const double* k, const double* m, double sigma, double* a,
                                  int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = k[i] - sigma * m[i];
}

constexpr int GEMV_RB = 1024;  // rows per block of the column-pair reductions

// Projection x -= B (W^T x) of one Gram-Schmidt pass, in two launches:
// proj_t_kernel forms partial sums of c = W^T x over row blocks of PROJ_RB
// rows (2 columns per workgroup, the rows split over its 4 waves); every
// workgroup of proj_n_kernel sums the partials of all columns in the same
// fixed order, so c needs no launch of its own, and subtracts B c.
constexpr int PROJ_RB = 4096;  // rows per partial sum (1024 per wave)

__global__ void __launch_bounds__(256) proj_t_kernel(const double* __restrict__ W, int64_t n, int m,
                                                   const double* __restrict__ x,
                                                   double* __restrict__ partial,
                                                   const int32_t* __restrict__ dj) {
  // workgroup: 2 columns x PROJ_RB rows; wave w takes rows
  // [rb * PROJ_RB + w * PROJ_RB / 4, ...), 16 per lane, all loads issued first
  // (with dj, a replayed launch: m + *dj columns, the grid sized for the most)
  __shared__ double red[2][4];
  if (dj) m += *dj;
  const int rb = blockIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j0 = blockIdx.y * 2;
  if (j0 >= m) return;
  const bool two = j0 + 1 < m;
  const int64_t r0 = (int64_t)rb * PROJ_RB + (int64_t)wave * (PROJ_RB / 4);
  const int64_t r1 = min((int64_t)rb * PROJ_RB + PROJ_RB, n);
  const double* c0 = W + (int64_t)j0 * n;
  const double* c1 = W + (int64_t)(two ? j0 + 1 : j0) * n;
  constexpr int RPL = PROJ_RB / 4 / 64;
  double xv[RPL], a0[RPL], a1[RPL];
#pragma unroll
  for (int u = 0; u < RPL; ++u) {
    const int64_t r = r0 + lane + 64 * u;
    const bool ok = r < r1;
    xv[u] = ok ? x[r] : 0.0;
    a0[u] = ok ? c0[r] : 0.0;
    a1[u] = ok ? c1[r] : 0.0;
  }
  double s0 = 0.0, s1 = 0.0;
#pragma unroll
  for (int u = 0; u < RPL; ++u) {
    s0 += a0[u] * xv[u];
    s1 += a1[u] * xv[u];
  }
  for (int off = 32; off > 0; off >>= 1) {
    s0 += __shfl_xor(s0, off);
    s1 += __shfl_xor(s1, off);
  }
  if (lane == 0) {
    red[0][wave] = s0;
    red[1][wave] = s1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    partial[(int64_t)rb * m + j0] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
    if (two) partial[(int64_t)rb * m + j0 + 1] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
  }
}

// c = sum of the nrb partials (rb ascending, eight loads in flight);
// x -= B c.  Workgroup 0 also stores c and, with alpha_out,
// *alpha_out = *addend + c[m - 1].
__global__ void __launch_bounds__(256) proj_n_kernel(const double* __restrict__ B, int64_t n, int m,
                                                   const double* __restrict__ partial, int nrb,
                                                   double* c_out, double* alpha_out,
                                                   const double* addend, double* __restrict__ x,
                                                   const int32_t* __restrict__ dj) {
  extern __shared__ double cs[];
  if (dj) {
    // a replayed launch: m + *dj columns, alpha_out and addend advanced by *dj
    const int d = *dj;
    m += d;
    if (alpha_out) alpha_out += d;
    if (addend) addend += d;
  }
  for (int j = threadIdx.x; j < m; j += blockDim.x) {
    double sj = 0.0;
    for (int rb = 0; rb < nrb; rb += 8) {
      double v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = rb + q < nrb ? partial[(int64_t)(rb + q) * m + j] : 0.0;
#pragma unroll
      for (int q = 0; q < 8; ++q) sj += v[q];
    }
    cs[j] = sj;
    if (blockIdx.x == 0) {
      c_out[j] = sj;
      if (alpha_out && j == m - 1) *alpha_out = *addend + sj;
    }
  }
  __syncthreads();
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  // 16 column loads in flight per thread (the last batch predicated)
  double s = 0.0;
  for (int j = 0; j < m; j += 16) {
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = j + u < m ? B[(int64_t)(j + u) * n + r] : 0.0;
#pragma unroll
    for (int u = 0; u < 16; ++u) s += j + u < m ? v[u] * cs[j + u] : 0.0;
  }
  x[r] -= s;
}

__global__ void reduce_partials_kernel(const double* partial, int nblk, double* out) {
  __shared__ double sm[256];
  double s = 0.0;
  // fixed assignment of partials to threads, then a fixed tree
  for (int i = threadIdx.x; i < nblk; i += 256) s += partial[i];
  sm[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sm[0];
}

// Counter-based generator: splitmix64 of (seed, stream, index) -> U(-1, 1).
__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void fill_random_kernel(double* x, int64_t n, uint64_t seed, uint64_t sid) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t h = splitmix64(seed ^ splitmix64(sid * 0x632BE59BD9B4E019ull + (uint64_t)i));
  x[i] = (double)(h >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// v = x / beta, w = y / beta, beta^2 = sum of the np partials (each
// workgroup adds them in the same fixed order); writes beta; flags breakdown
__global__ void __launch_bounds__(256) scale2_kernel(const double* x, const double* y,
                                                   const double* partial, int np, double* v,
                                                   double* w, int64_t n, double* beta_out,
                                                   int32_t* flag, const int32_t* __restrict__ dj) {
  __shared__ double sm[4];
  if (dj) {
    // a replayed launch: columns and beta advanced by *dj
    const int d = *dj;
    v += (int64_t)d * n;
    w += (int64_t)d * n;
    if (beta_out) beta_out += d;
  }
  // every workgroup sums all partials: eight loads in flight per thread,
  // then the wave and workgroup reductions (fixed order)
  double t = 0.0;
  for (int i0 = threadIdx.x; i0 < np; i0 += 8 * 256) {
    double pv[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) pv[q] = i0 + q * 256 < np ? partial[i0 + q * 256] : 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) t += pv[q];
  }
  for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off);
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = t;
  __syncthreads();
  const double b2 = (sm[0] + sm[1]) + (sm[2] + sm[3]);
  const bool ok = b2 > 0.0 && isfinite(b2);
  const double b = ok ? sqrt(b2) : 0.0;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    if (beta_out) *beta_out = b;
    if (!ok && flag) *flag = 1;
  }
  if (i >= n || !ok) return;
  const double ib = 1.0 / b;
  v[i] = x[i] * ib;
  w[i] = y[i] * ib;
}

// U(n x m) = V(n x k) S(k x m), S column-major with leading dimension lds.
// S is staged through LDS in chunks of GEMM_KC rows.
constexpr int GEMM_CB = 16;
constexpr int GEMM_KC = 128;
__global__ void __launch_bounds__(256) gemm_nn_kernel(const double* __restrict__ V, int64_t n,
                                                    int k, const double* __restrict__ S, int lds,
                                                    int m, double* __restrict__ U, int sub) {
  __shared__ double ss[GEMM_KC * GEMM_CB];
  const int c0 = blockIdx.y * GEMM_CB;
  const int nc = min(GEMM_CB, m - c0);
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double acc[GEMM_CB];
#pragma unroll
  for (int q = 0; q < GEMM_CB; ++q) acc[q] = 0.0;
  for (int k0 = 0; k0 < k; k0 += GEMM_KC) {
    const int kc = min(GEMM_KC, k - k0);
    __syncthreads();
    for (int e = threadIdx.x; e < GEMM_KC * GEMM_CB; e += blockDim.x) {
      const int t = e % GEMM_KC, q = e / GEMM_KC;
      ss[e] = (q < nc && t < kc) ? S[(int64_t)(c0 + q) * lds + k0 + t] : 0.0;
    }
    __syncthreads();
    if (r < n) {
      for (int t = 0; t < kc; ++t) {
        const double v = V[(int64_t)(k0 + t) * n + r];
#pragma unroll
        for (int q = 0; q < GEMM_CB; ++q) acc[q] += v * ss[q * GEMM_KC + t];
      }
    }
  }
  if (r < n) {
    if (sub)
      for (int q = 0; q < nc; ++q) U[(int64_t)(c0 + q) * n + r] -= acc[q];
    else
      for (int q = 0; q < nc; ++q) U[(int64_t)(c0 + q) * n + r] = acc[q];
  }
}

// Partial sums of C = W^T U over row blocks of TN_RB rows, for a tile of
// TN_T columns of W and TN_T columns of U per workgroup: each thread keeps
// the TN_T x TN_T products of its rows, the waves reduce them with
// shuffles, and partial[(rb * c + i) * m + q] takes the workgroup's sum.
constexpr int TN_T = 8;
constexpr int TN_RB = 4096;

__global__ void __launch_bounds__(256) gemm_tn_partial_kernel(const double* __restrict__ W, int64_t n, int c,
                                                            const double* __restrict__ U, int m,
                                                            double* __restrict__ partial) {
  __shared__ double red[4][TN_T * TN_T];
  const int rb = blockIdx.x;
  const int i0 = blockIdx.y * TN_T, q0 = blockIdx.z * TN_T;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t r1 = min((int64_t)(rb + 1) * TN_RB, n);
  double acc[TN_T][TN_T];
#pragma unroll
  for (int a = 0; a < TN_T; ++a)
#pragma unroll
    for (int b = 0; b < TN_T; ++b) acc[a][b] = 0.0;
  for (int64_t r = (int64_t)rb * TN_RB + threadIdx.x; r < r1; r += 256) {
    double w[TN_T], u[TN_T];
#pragma unroll
    for (int a = 0; a < TN_T; ++a) {
      w[a] = i0 + a < c ? W[(int64_t)(i0 + a) * n + r] : 0.0;
      u[a] = q0 + a < m ? U[(int64_t)(q0 + a) * n + r] : 0.0;
    }
#pragma unroll
    for (int a = 0; a < TN_T; ++a)
#pragma unroll
      for (int b = 0; b < TN_T; ++b) acc[a][b] += w[a] * u[b];
  }
#pragma unroll
  for (int a = 0; a < TN_T; ++a)
#pragma unroll
    for (int b = 0; b < TN_T; ++b) {
      double v = acc[a][b];
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
      if (lane == 0) red[wave][a * TN_T + b] = v;
    }
  __syncthreads();
  if (threadIdx.x < TN_T * TN_T) {
    const int a = threadIdx.x / TN_T, b = threadIdx.x % TN_T;
    const double v = (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
    if (i0 + a < c && q0 + b < m) partial[((int64_t)rb * c + i0 + a) * m + q0 + b] = v;
  }
}

// C(i, q) = sum over row blocks (ascending) of the partials; C column-major
// with leading dimension c.
__global__ void gemm_tn_reduce_kernel(const double* __restrict__ partial, int nrb, int c, int m,
                                      double* __restrict__ C) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= c * m) return;
  const int i = e % c, q = e / c;
  double s = 0.0;
  for (int rb = 0; rb < nrb; ++rb) s += partial[((int64_t)rb * c + i) * m + q];
  C[(int64_t)q * c + i] = s;
}

// Per column q of the n x m blocks: mode 0 -> partial sums of (u^T K u,
// u^T M u); mode 1 -> partial sums of (||K u - lam_q M u||^2, ||u||^2).
__global__ void __launch_bounds__(256) colpair_kernel(const double* KU, const double* MU,
                                                    const double* U, int64_t n, int m,
                                                    const double* lam, int mode,
                                                    double* partial) {
  const int rb = blockIdx.x;
  const int q = blockIdx.y;
  const int64_t r0 = (int64_t)rb * GEMV_RB, r1 = min(r0 + GEMV_RB, n);
  double s0 = 0.0, s1 = 0.0;
  const double* ku = KU + (int64_t)q * n;
  const double* mu = MU + (int64_t)q * n;
  const double* u = U + (int64_t)q * n;
  const double lq = mode ? lam[q] : 0.0;
  for (int64_t r = r0 + threadIdx.x; r < r1; r += 256) {
    if (mode == 0) {
      s0 += u[r] * ku[r];
      s1 += u[r] * mu[r];
    } else {
      const double d = ku[r] - lq * mu[r];
      s0 += d * d;
      s1 += u[r] * u[r];
    }
  }
  __shared__ double a0[256], a1[256];
  a0[threadIdx.x] = s0;
  a1[threadIdx.x] = s1;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      a0[threadIdx.x] += a0[threadIdx.x + w];
      a1[threadIdx.x] += a1[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[((int64_t)rb * m + q) * 2 + 0] = a0[0];
    partial[((int64_t)rb * m + q) * 2 + 1] = a1[0];
  }
}

__global__ void colpair_reduce_kernel(const double* partial, int nrb, int m, double* out0,
                                      double* out1) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= m) return;
  double s0 = 0.0, s1 = 0.0;
  for (int rb = 0; rb < nrb; ++rb) {
    s0 += partial[((int64_t)rb * m + q) * 2];
    s1 += partial[((int64_t)rb * m + q) * 2 + 1];
  }
  out0[q] = s0;
  out1[q] = s1;
}

__global__ void ratio_kernel(const double* a, const double* b, double* out, int m) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < m) out[q] = a[q] / b[q];
}

__global__ void copy_kernel(double* dst, const double* src, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

__global__ void scale_cols_kernel(double* U, int64_t n, int m, const double* scale) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int q = blockIdx.y;
  if (i < n && q < m) U[(int64_t)q * n + i] *= scale[q];
}

// U(:, q) and V(:, q) scaled by 1 / sqrt(d[q])
__global__ void scale_cols_rsqrt_kernel(double* U, double* V, int64_t n, int m, const double* d) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int q = blockIdx.y;
  if (i >= n || q >= m) return;
  const double sc = 1.0 / sqrt(d[q]);
  U[(int64_t)q * n + i] *= sc;
  V[(int64_t)q * n + i] *= sc;
}

// Column copies dst(:, dcol[q]) = src(:, scol[q]) for up to COLS_PER_COPY
// pairs, for two matrices at once (the second pair may be null).
// jmul: the column times i of a complex vector stored as interleaved real
// and imaginary parts (J u: (re, im) -> (-im, re)); n even then.
__global__ void copy_cols_kernel(ColCopy cc, int64_t n, double* d0, const double* s0, double* d1,
                                 const double* s1, int jmul) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int q = blockIdx.y;
  if (i >= n || q >= cc.count) return;
  const int64_t src = jmul ? (i ^ 1) : i;
  const double sg = (jmul && !(i & 1)) ? -1.0 : 1.0;
  d0[(int64_t)cc.dst[q] * n + i] = sg * s0[(int64_t)cc.src[q] * n + src];
  if (d1) d1[(int64_t)cc.dst[q] * n + i] = sg * s1[(int64_t)cc.src[q] * n + src];
}

// x <- sg J x in place, J: (re, im) -> (-im, re) on interleaved pairs
// (sg = -1: the inverse rotation); one thread per pair, n even.
__global__ void jrot_kernel(double* x, int64_t pairs, double sg) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= pairs) return;
  const double2 v = reinterpret_cast<const double2*>(x)[k];
  reinterpret_cast<double2*>(x)[k] = make_double2(-sg * v.y, sg * v.x);
}

__global__ void axpby_kernel(double a, const double* u, const double* v, double* out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a * u[i] + v[i];
}

__global__ void __launch_bounds__(256) dot_partial_kernel(const double* a, const double* b,
                                                        int64_t n, double* partial) {
  __shared__ double sm[256];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    s += a[i] * b[i];
  sm[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sm[0];
}

}  // namespace

void launch_axpby(double a, const double* u, const double* v, double* out, int64_t n,
                  hipStream_t s) {
  axpby_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(a, u, v, out, n);
  HIPCHECK(hipGetLastError());
}

constexpr int DOT_BLOCKS = 256;

// out[0] = a^T b (two-stage, fixed order); partial holds DOT_BLOCKS doubles
void launch_dot(const double* a, const double* b, int64_t n, double* partial, double* out,
                hipStream_t s) {
  dot_partial_kernel<<<DOT_BLOCKS, 256, 0, s>>>(a, b, n, partial);
  reduce_partials_kernel<<<1, 256, 0, s>>>(partial, DOT_BLOCKS, out);
  HIPCHECK(hipGetLastError());
}

int spmv_blocks(const riga_problem* pr) {
  const int G = pr->spmv_group;
  return (int)((pr->an.N + (256 / G) - 1) / (256 / G));
}

int spmv_dot_blocks(const riga_problem* pr) { return spmv_blocks(pr); }

void launch_spmv(const riga_problem* pr, const double* vals, const double* x, double* y,
                 double* dot_partial, hipStream_t s) {
  const int64_t N = pr->an.N;
  const int nb = dot_partial ? spmv_dot_blocks(pr) : spmv_blocks(pr);
  auto* rp = pr->row_ptr.p;
  auto* ci = pr->col_idx.p;
  switch (pr->spmv_group) {
    case 4: spmv_kernel<4><<<nb, 256, 0, s>>>(rp, ci, vals, x, y, N, dot_partial); break;
    case 8: spmv_kernel<8><<<nb, 256, 0, s>>>(rp, ci, vals, x, y, N, dot_partial); break;
    case 16: spmv_kernel<16><<<nb, 256, 0, s>>>(rp, ci, vals, x, y, N, dot_partial); break;
    case 32: spmv_kernel<32><<<nb, 256, 0, s>>>(rp, ci, vals, x, y, N, dot_partial); break;
    default: spmv_kernel<64><<<nb, 256, 0, s>>>(rp, ci, vals, x, y, N, dot_partial); break;
  }
  HIPCHECK(hipGetLastError());
}

void launch_spmm_km(const riga_problem* pr, const double* U, int nw, double* KU, double* MU,
                    hipStream_t s) {
  if (nw <= 0) return;
  constexpr int NV = 8;
  const int64_t N = pr->an.N;
  const dim3 grid((unsigned)spmv_blocks(pr), (nw + NV - 1) / NV);
  auto* rp = pr->row_ptr.p;
  auto* ci = pr->col_idx.p;
  auto* k = pr->kv.p;
  auto* m = pr->mv.p;
  switch (pr->spmv_group) {
    case 4: spmm_km_kernel<4, NV><<<grid, 256, 0, s>>>(rp, ci, k, m, U, nw, KU, MU, N); break;
    case 8: spmm_km_kernel<8, NV><<<grid, 256, 0, s>>>(rp, ci, k, m, U, nw, KU, MU, N); break;
    case 16: spmm_km_kernel<16, NV><<<grid, 256, 0, s>>>(rp, ci, k, m, U, nw, KU, MU, N); break;
    case 32: spmm_km_kernel<32, NV><<<grid, 256, 0, s>>>(rp, ci, k, m, U, nw, KU, MU, N); break;
    default: spmm_km_kernel<64, NV><<<grid, 256, 0, s>>>(rp, ci, k, m, U, nw, KU, MU, N); break;
  }
  HIPCHECK(hipGetLastError());
}

void launch_axpby_vals(const double* k, const double* m, double sigma, double* a, int64_t n,
                       hipStream_t s) {
  axpby_vals_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(k, m, sigma, a, n);
  HIPCHECK(hipGetLastError());
}

int gemv_row_blocks(int64_t n) { return (int)((n + GEMV_RB - 1) / GEMV_RB); }

int proj_row_blocks(int64_t n) { return (int)((n + PROJ_RB - 1) / PROJ_RB); }

void launch_project(const double* W, const double* B, int64_t n, int m, double* x, double* partial,
                    double* c, double* alpha_out, const double* addend, hipStream_t s,
                    const int32_t* dj, int m_max) {
  if (m <= 0 && !dj) return;
  const int mg = dj ? m_max : m;
  const int nrb = proj_row_blocks(n);
  dim3 grid(nrb, (mg + 1) / 2);
  proj_t_kernel<<<grid, 256, 0, s>>>(W, n, m, x, partial, dj);
  proj_n_kernel<<<(unsigned)((n + 255) / 256), 256, (size_t)mg * sizeof(double), s>>>(
      B, n, m, partial, nrb, c, alpha_out, addend, x, dj);
  HIPCHECK(hipGetLastError());
}

// dst = src + *dj n (a column chosen by the step index; n entries)
__global__ void copy_col_dyn_kernel(double* dst, const double* src, int64_t n, const int32_t* dj) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[(int64_t)(*dj) * n + i];
}

__global__ void step_advance_kernel(int32_t* dj) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dj += 1;
}

void launch_copy_col_dyn(double* dst, const double* src, int64_t n, const int32_t* dj, hipStream_t s) {
  copy_col_dyn_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(dst, src, n, dj);
  HIPCHECK(hipGetLastError());
}

void launch_step_advance(int32_t* dj, hipStream_t s) {
  step_advance_kernel<<<1, 64, 0, s>>>(dj);
  HIPCHECK(hipGetLastError());
}

void launch_reduce_partials(const double* partial, int nblk, double* out, hipStream_t s) {
  reduce_partials_kernel<<<1, 256, 0, s>>>(partial, nblk, out);
  HIPCHECK(hipGetLastError());
}

void launch_fill_random(double* x, int64_t n, uint64_t seed, uint64_t sid, hipStream_t s) {
  fill_random_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(x, n, seed, sid);
  HIPCHECK(hipGetLastError());
}

void launch_scale2(const double* x, const double* y, const double* partial, int np, double* v,
                   double* w, int64_t n, double* beta_out, int32_t* flag, hipStream_t s,
                   const int32_t* dj) {
  scale2_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(x, y, partial, np, v, w, n, beta_out, flag, dj);
  HIPCHECK(hipGetLastError());
}

void launch_gemm_nn(const double* V, int64_t n, int k, const double* S, int lds, int m, double* U,
                    hipStream_t s) {
  if (m <= 0 || k <= 0) return;
  dim3 grid((unsigned)((n + 255) / 256), (m + GEMM_CB - 1) / GEMM_CB);
  gemm_nn_kernel<<<grid, 256, 0, s>>>(V, n, k, S, lds, m, U, 0);
  HIPCHECK(hipGetLastError());
}

constexpr int BP_CHUNK = 512;  // columns of W, B per block-projection pass

static int tn_row_blocks(int64_t n) { return (int)((n + TN_RB - 1) / TN_RB); }

size_t block_project_partials(int64_t n, int m) {
  return (size_t)tn_row_blocks(n) * (size_t)BP_CHUNK * (size_t)m + (size_t)BP_CHUNK * (size_t)m;
}

void launch_block_project(const double* W, const double* B, int64_t n, int c, double* U, int m,
                          double* partial, hipStream_t s) {
  if (c <= 0 || m <= 0) return;
  const int nrb = tn_row_blocks(n);
  for (int a = 0; a < c; a += BP_CHUNK) {
    const int cc = std::min(BP_CHUNK, c - a);
    const double* Wa = W + (int64_t)a * n;
    const double* Ba = B + (int64_t)a * n;
    double* C = partial + (size_t)nrb * cc * m;
    dim3 g1((unsigned)nrb, (unsigned)((cc + TN_T - 1) / TN_T), (unsigned)((m + TN_T - 1) / TN_T));
    gemm_tn_partial_kernel<<<g1, 256, 0, s>>>(Wa, n, cc, U, m, partial);
    gemm_tn_reduce_kernel<<<(unsigned)((cc * m + 255) / 256), 256, 0, s>>>(partial, nrb, cc, m, C);
    dim3 g2((unsigned)((n + 255) / 256), (m + GEMM_CB - 1) / GEMM_CB);
    gemm_nn_kernel<<<g2, 256, 0, s>>>(Ba, n, cc, C, cc, m, U, 1);
  }
  HIPCHECK(hipGetLastError());
}

// Rayleigh quotients lam = u^T K u / u^T M u, then ||K u - lam M u||^2 and ||u||^2.
int residual_partials(int64_t n, int m) { return gemv_row_blocks(n) * m * 2; }

void launch_residuals(const double* KU, const double* MU, const double* U, int64_t n, int m,
                      double* out_rq_num, double* out_rq_den, double* out_rnorm2,
                      double* out_unorm2, double* lam, double* partial, hipStream_t s) {
  const int nrb = gemv_row_blocks(n);
  dim3 grid(nrb, m);
  colpair_kernel<<<grid, 256, 0, s>>>(KU, MU, U, n, m, nullptr, 0, partial);
  colpair_reduce_kernel<<<(m + 127) / 128, 128, 0, s>>>(partial, nrb, m, out_rq_num, out_rq_den);
  ratio_kernel<<<(m + 127) / 128, 128, 0, s>>>(out_rq_num, out_rq_den, lam, m);
  colpair_kernel<<<grid, 256, 0, s>>>(KU, MU, U, n, m, lam, 1, partial);
  colpair_reduce_kernel<<<(m + 127) / 128, 128, 0, s>>>(partial, nrb, m, out_rnorm2, out_unorm2);
  HIPCHECK(hipGetLastError());
}

void launch_scale_cols_rsqrt(double* U, double* V, int64_t n, int m, const double* d, hipStream_t s) {
  if (m <= 0) return;
  dim3 grid((unsigned)((n + 255) / 256), m);
  scale_cols_rsqrt_kernel<<<grid, 256, 0, s>>>(U, V, n, m, d);
  HIPCHECK(hipGetLastError());
}

void launch_copy_cols(const std::vector<int>& dst, const std::vector<int>& src, int64_t n, double* d0,
                      const double* s0, double* d1, const double* s1, hipStream_t s, bool jmul) {
  if (jmul && (n & 1)) throw Error(RIGA_EINVAL, "J copy of an odd-length column");
  for (size_t q0 = 0; q0 < dst.size(); q0 += COLS_PER_COPY) {
    ColCopy cc{};
    cc.count = (int)std::min<size_t>(COLS_PER_COPY, dst.size() - q0);
    for (int q = 0; q < cc.count; ++q) {
      cc.dst[q] = dst[q0 + q];
      cc.src[q] = src[q0 + q];
    }
    dim3 grid((unsigned)((n + 255) / 256), cc.count);
    copy_cols_kernel<<<grid, 256, 0, s>>>(cc, n, d0, s0, d1, s1, jmul ? 1 : 0);
    HIPCHECK(hipGetLastError());
  }
}

void launch_jrot(double* x, int64_t n, double sg, hipStream_t s) {
  if (n & 1) throw Error(RIGA_EINVAL, "launch_jrot: odd length");
  const int64_t pairs = n / 2;
  if (pairs == 0) return;
  jrot_kernel<<<(unsigned)((pairs + 255) / 256), 256, 0, s>>>(x, pairs, sg);
  HIPCHECK(hipGetLastError());
}

void launch_copy(double* dst, const double* src, int64_t n, hipStream_t s) {
  copy_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(dst, src, n);
  HIPCHECK(hipGetLastError());
}

void launch_scale_cols(double* U, int64_t n, int m, const double* scale, hipStream_t s) {
  if (m <= 0) return;
  dim3 grid((unsigned)((n + 255) / 256), m);
  scale_cols_kernel<<<grid, 256, 0, s>>>(U, n, m, scale);
  HIPCHECK(hipGetLastError());
}

}  // namespace riga
