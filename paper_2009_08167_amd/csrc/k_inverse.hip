// Partitioned inverse of the front factors, formed once per factorisation so
// that every forward/backward elimination of the Lanczos steps (Sec. 5.1:
// the f/b eliminations dominate the cost on small and mid-size problems) is
// a pair of dense matrix-vector products per front instead of a chain of
// triangular panel solves.
//
// For a front of order f with k fully-summed variables, the factorisation
// leaves L = [L11; L21] (f x k, unit lower L11, pivot order) and the block
// diagonal D.  This kernel writes, in a separate pool, column-major with the
// leading dimension ldh (f rounded up to 32 elements, every column starting
// on a 128-byte boundary),
//     H = [I; L21] * L11^{-1}   =  [ L11^{-1} ; L21 L11^{-1} ]
// except on the diagonal of the top k x k block, which keeps D(i, i), and on
// the (t+1, t) slot of every 2x2 pivot block, which keeps D(t+1, t) (both
// entries of L11^{-1} there are known: 1 and 0).  The strict upper triangle
// of the top block is never written or read.  D is also copied, by pivot
// index, into two compact FP64 arrays (diagonal; (t+1, t) entry of 2x2
// blocks) for the backward sweep.
//
// Rows of H are independent (row i solves h L11 = r_i with r_i = e_i or the
// row of L21), so a workgroup takes a block of up to 64 rows and walks the
// columns from the right in 64-wide panels:
//     Hp = R(:, panel) - H(:, right of panel) * L11(right of panel, panel)
//     (a GEMM on the matrix cores in the factor's precision, operands
//     staged in LDS; the panel Hp then takes the LDS of the GEMM's first
//     operand, so that two workgroups fit in a compute unit), then the
//     unit-triangular solve with the panel's diagonal block of L11.
// The columns to the right were written by the same workgroup earlier; the
// workgroup barrier orders those global writes before the reads.
#include <hip/hip_runtime.h>

#include "mfma_tile.h"
#include "problem.h"

namespace riga {
namespace {

constexpr int IB = 64;       // panel width and row block
constexpr int LDP = IB + 1;  // padded LDS leading dimension

__device__ __forceinline__ double lane_bcast(double v, int l) {
  const long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(bits & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// L(m, c) of the unit lower factor, m > c: the (c+1, c) slot of a 2x2 pivot
// block holds D, and L is zero there.
template <class T>
__device__ __forceinline__ double l_entry(const T* L, int f, int m, int c, const int32_t* type) {
  if (m == c + 1 && type[c] == 2) return 0.0;
  return (double)L[(int64_t)c * f + m];
}

template <class T>
__global__ void __launch_bounds__(256, 2) front_inverse_kernel(const FrontDesc* __restrict__ desc,
                                                            const WorkUnit* __restrict__ units,
                                                            const T* __restrict__ pool, T* H,
                                                            const int32_t* __restrict__ piv_type,
                                                            double* dd, double* dsub) {
  extern __shared__ double smem[];
  double* Ac = smem;              // Ac[mm * LDP + ii] = H(r0 + ii, m0 + mm)
  double* Bc = Ac + IB * LDP;     // Bc[mm * LDP + c]  = L(m0 + mm, j0 + c)
  double* Hp = Ac;                // Hp[ii * LDP + c]  = H(r0 + ii, j0 + c), after the GEMM
  int32_t* type = (int32_t*)(Bc + IB * LDP);
  const WorkUnit u = units[blockIdx.x];
  const FrontDesc d = desc[u.front];
  const int f = d.f, k = d.k, ldh = d.ldh;
  const int r0 = u.lo, nr = u.hi - u.lo;
  const T* L = pool + d.pool_off;
  T* Hf = H + d.h_off;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int t = tid; t < k; t += 256) type[t] = piv_type[d.start + t];
  __syncthreads();
  // a block of rows of the top (inverse) part has zeros right of its last row
  int qlast = (k - 1) / IB;
  if (r0 + nr <= k) qlast = min(qlast, (r0 + nr - 1) / IB);
  const int nrt = (nr + 15) / 16;
  for (int q = qlast; q >= 0; --q) {
    const int j0 = q * IB, pw = min(IB, k - j0), j1 = j0 + pw;
    // Hp -= H(:, j1:k) * L11(j1:k, panel), 64-deep chunks on the MFMA units
    Tile16<T> acc[4];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) acc[rt].zero();
    if (j1 < k) {
      for (int m0 = j1; m0 < k; m0 += IB) {
        const int mw = min(IB, k - m0);
        double ar[IB * IB / 256], br[IB * IB / 256];
#pragma unroll
        for (int q = 0; q < IB * IB / 256; ++q) {
          const int e = tid + 256 * q;
          const int ii = e & 63, mm = e >> 6;
          double a = 0.0;
          if (ii < nr && mm < mw) {
            const int i = r0 + ii, m = m0 + mm;
            if (i >= k) a = (double)Hf[(int64_t)m * ldh + i];
            else if (m == i) a = 1.0;
            else if (m < i && !(m == i - 1 && type[m] == 2)) a = (double)Hf[(int64_t)m * ldh + i];
          }
          ar[q] = a;
          const int mb = e & 63, cb = e >> 6;
          br[q] = (mb < mw && cb < pw) ? l_entry(L, f, m0 + mb, j0 + cb, type) : 0.0;
        }
#pragma unroll
        for (int q = 0; q < IB * IB / 256; ++q) {
          const int e = tid + 256 * q;
          Ac[(e >> 6) * LDP + (e & 63)] = ar[q];
          Bc[(e & 63) * LDP + (e >> 6)] = br[q];
        }
        __syncthreads();
        const int cl = wave * 16 + (lane & 15);
#pragma unroll 4
        for (int kk = 0; kk < IB; kk += 4) {
          const int kr = kk + (lane >> 4);
          const double bv = Bc[kr * LDP + cl];
#pragma unroll
          for (int rt = 0; rt < 4; ++rt)
            if (rt < nrt) {
              const double av = Ac[kr * LDP + rt * 16 + (lane & 15)];
              acc[rt].step(av, bv);
            }
        }
        __syncthreads();
      }
    }
    // right-hand side rows: e_i in the top block, L21 rows below (every
    // load of the thread's share issued before the LDS stores), into the
    // LDS of the GEMM's first operand: the GEMM's last barrier is behind
    {
      double rv[IB * IB / 256];
#pragma unroll
      for (int q = 0; q < IB * IB / 256; ++q) {
        const int e = tid + 256 * q;
        const int ii = e & 63, c = e >> 6;
        double v = 0.0;
        if (ii < nr && c < pw) {
          const int i = r0 + ii, j = j0 + c;
          v = i < k ? (i == j ? 1.0 : 0.0) : (double)L[(int64_t)j * f + i];
        }
        rv[q] = v;
      }
#pragma unroll
      for (int q = 0; q < IB * IB / 256; ++q) {
        const int e = tid + 256 * q;
        Hp[(e & 63) * LDP + (e >> 6)] = rv[q];
      }
    }
    __syncthreads();
    if (j1 < k) {
      // lane holds the product at row Tile16::row(lane, r) of the row
      // tile, column lane & 15 of this wave's column tile
#pragma unroll
      for (int rt = 0; rt < 4; ++rt)
        if (rt < nrt) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int ii = rt * 16 + Tile16<T>::row(lane, r);
            Hp[ii * LDP + wave * 16 + (lane & 15)] -= acc[rt].get(r);
          }
        }
    }
    // diagonal block of the panel: Bc[m * LDP + c] = L11(j0 + m, j0 + c), m > c
    {
      double dr[IB * IB / 256];
#pragma unroll
      for (int q = 0; q < IB * IB / 256; ++q) {
        const int e = tid + 256 * q;
        const int m = e & 63, c = e >> 6;
        dr[q] = (m > c && m < pw) ? l_entry(L, f, j0 + m, j0 + c, type) : 0.0;
      }
#pragma unroll
      for (int q = 0; q < IB * IB / 256; ++q) {
        const int e = tid + 256 * q;
        Bc[(e & 63) * LDP + (e >> 6)] = dr[q];
      }
    }
    __syncthreads();
    // h(:, c) for c from the right: once h(i, m) is final, remove its share
    // h(i, m) L(m, c) from every column c < m.  Wave w takes rows w, w+4, ...
    {
      double val[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int ii = wave + 4 * r;
        val[r] = ii < nr ? Hp[ii * LDP + lane] : 0.0;
      }
      for (int m = pw - 1; m >= 1; --m) {
        const double lm = Bc[m * LDP + lane];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const double h = lane_bcast(val[r], m);
          if (lane < m) val[r] -= h * lm;
        }
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int ii = wave + 4 * r;
        if (ii < nr) Hp[ii * LDP + lane] = val[r];
      }
    }
    __syncthreads();
    // panel out: below the diagonal the computed entries, on the diagonal
    // and in 2x2 slots the D entries of the factor
    for (int e = tid; e < IB * IB; e += 256) {
      const int ii = e & 63, c = e >> 6;
      if (ii < nr && c < pw) {
        const int i = r0 + ii, j = j0 + c;
        const int64_t o = (int64_t)j * ldh + i, ol = (int64_t)j * f + i;
        if (i >= k) {
          Hf[o] = (T)Hp[ii * LDP + c];
        } else if (j == i) {
          Hf[o] = L[ol];
          dd[d.start + i] = (double)L[ol];
        } else if (j == i - 1 && type[j] == 2) {
          Hf[o] = L[ol];
          dsub[d.start + j] = (double)L[ol];
        } else if (j < i) {
          Hf[o] = (T)Hp[ii * LDP + c];
        }
      }
    }
    __syncthreads();
  }
}

constexpr size_t INV_LDS_FIXED = (size_t)2 * IB * LDP * sizeof(double);

}  // namespace

size_t front_inverse_lds(int max_k) { return INV_LDS_FIXED + (size_t)max_k * sizeof(int32_t); }

void set_inverse_attributes() {
  HIPCHECK(hipFuncSetAttribute((const void*)front_inverse_kernel<double>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, 159 * 1024));
  HIPCHECK(hipFuncSetAttribute((const void*)front_inverse_kernel<float>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, 159 * 1024));
}

template <class T>
void launch_front_inverse(riga_problem* pr, Factor& F, const T* pool, T* h, hipStream_t s) {
  if (pr->n_inv_units == 0) return;
  front_inverse_kernel<T><<<pr->n_inv_units, 256, front_inverse_lds(pr->an.max_fs), s>>>(
      pr->d_desc.p, pr->inv_units.p, pool, h, F.piv_type.p, F.d_diag.p, F.d_sub.p);
  HIPCHECK(hipGetLastError());
}

template void launch_front_inverse<double>(riga_problem*, Factor&, const double*, double*, hipStream_t);
template void launch_front_inverse<float>(riga_problem*, Factor&, const float*, float*, hipStream_t);

}  // namespace riga
