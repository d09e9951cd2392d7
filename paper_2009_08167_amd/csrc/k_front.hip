// Multifrontal LDL^T of A = K - sigma M over the tree of separators, with
// Bunch-Kaufman pivoting inside each front's fully-summed block and the
// inertia count of the Remark on inertia (arXiv 2009.08167, Sec. 4.2) --
// the numeric factorisation that Sec. 5 performs once per shift.
//
// Per tree level (all fronts of one height are independent):
//  1. front_assemble: one workgroup per front column gathers the children's
//     contribution blocks (extend-add through the parent->child position
//     maps) and adds the entries of A of the fully-summed columns.
//     Deterministic: every front entry is written by exactly one thread, the
//     children are summed in a fixed order.
//  2. front_factor: partial LDL^T of the fully-summed block (1x1 and 2x2
//     Bunch-Kaufman pivots chosen among the fully-summed rows), L21 and the
//     Schur-complement update of the contribution block.  Fronts up to
//     LDS_FRONT_MAX are factorised entirely in LDS by one workgroup; larger
//     fronts use the blocked multi-workgroup path of k_bigfront.hip.
//
// Fronts are dense column-major f x f blocks in one pool (lower triangle
// used).  After factorisation, column t < k holds L(:, t) below the
// diagonal and D on it (a 2x2 block keeps its off-diagonal in (t+1, t));
// rows/cols >= k hold the contribution block for the parent.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <mutex>

#include "problem.h"

namespace riga {
namespace {

struct FrontArgs {
  const int32_t* fk;
  const int32_t* ff;
  const int32_t* fstart;
  const int64_t* pool_off;
  const int32_t* child_ptr;
  const int32_t* child_list;
  const int64_t* inv_off;
  const int32_t* inv;
  const int64_t* amap_ptr;
  const int32_t* amap_row;
  const int32_t* amap_val;
  const double* kv;
  const double* mv;
  int32_t* piv_perm;
  int32_t* piv_type;
  int32_t* stat;   // per front: negative pivots, perturbed pivots, 2x2 pivots
};

template <class T>
__global__ void __launch_bounds__(64 * ASM_COLS) front_assemble_kernel(FrontArgs fa, T* pool,
                                                                     const int32_t* fronts,
                                                                     const int64_t* col_prefix,
                                                                     int nf, int cpw, double sigma) {
  // workgroup: cpw consecutive columns of one front, one wave each,
  // lanes over rows; the column is built in LDS and written once
  extern __shared__ double cols[];
  const int64_t gid = blockIdx.x;
  int lo = 0, hi = nf;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (col_prefix[mid] <= gid) lo = mid; else hi = mid;
  }
  const int F = fronts[lo];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j = (int)(gid - col_prefix[lo]) * cpw + wave;
  const int f = fa.ff[F], k = fa.fk[F];
  double* col = cols + (size_t)wave * f;
  T* front = pool + fa.pool_off[F];
  const int c0 = fa.child_ptr[F], nc = fa.child_ptr[F + 1] - c0;
  if (j < f) {
    // children's contributions: positions of column j in each child first
    int cc[4], kc[4], fc[4];
    int64_t po[4];
    const int32_t* inv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      cc[q] = -1;
      if (q < nc) {
        inv[q] = fa.inv + fa.inv_off[c0 + q];
        const int C = fa.child_list[c0 + q];
        kc[q] = fa.fk[C];
        fc[q] = fa.ff[C];
        po[q] = fa.pool_off[C];
        cc[q] = inv[q][j];
      }
    }
    for (int r0 = j; r0 < f; r0 += 64 * 4) {
      double v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int r = r0 + lane + 64 * u;
        double t = 0.0;
        if (r < f) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            if (cc[q] >= 0) {
              const int cr = inv[q][r];
              if (cr >= 0) t += (double)pool[po[q] + (int64_t)(kc[q] + cc[q]) * fc[q] + (kc[q] + cr)];
            }
          }
        }
        v[u] = t;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int r = r0 + lane + 64 * u;
        if (r < f) col[r] = v[u];
      }
    }
  }
  __syncthreads();
  if (j < k) {
    const int g = fa.fstart[F] + j;
    for (int64_t e = fa.amap_ptr[g] + lane; e < fa.amap_ptr[g + 1]; e += 64) {
      const int r = fa.amap_row[e];
      const int v = fa.amap_val[e];
      col[r] += fa.kv[v] - sigma * fa.mv[v];
    }
  }
  __syncthreads();
  if (j < f)
    for (int r = j + lane; r < f; r += 64) front[(int64_t)j * f + r] = (T)col[r];
}

constexpr double BK_ALPHA = 0.6403882032022076;  // (1 + sqrt(17)) / 8

// Shared decision of one pivot step.
struct PivotStep {
  int kind;     // 1: 1x1, 2: 2x2
  int swap_a;   // position to swap with swap_b (-1: none)
  int swap_b;
  int perturbed;
};

// Partial LDL^T of the front `a` (f x f, ld = f, lower), fully-summed block
// of order k.  NT threads.  `lbuf` holds 2 f doubles of scratch, `perm` k
// ints, `dec` the broadcast decision.  Works for `a` in LDS or in global
// memory.
template <class T, int NT, class Acc>
__device__ __forceinline__ void ldlt_partial(Acc A, int f, int k, double* lbuf, int* perm,
                                             PivotStep* dec, double pivtol, int* n_neg,
                                             int* n_pert, int* n_2x2, int32_t* type_out) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  constexpr int NW = NT / 64;
  for (int t = tid; t < k; t += NT) perm[t] = t;
  int neg = 0, pert = 0, two = 0;
  __syncthreads();
  int j = 0;
  while (j < k) {
    // ---- pivot decision (wave 0)
    if (wave == 0) {
      double cmax = 0.0;
      int r = -1;
      for (int i = j + 1 + lane; i < k; i += 64) {
        const double v = fabs((double)A(i, j));
        if (v > cmax) { cmax = v; r = i; }
      }
      for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(cmax, off);
        const int orr = __shfl_xor(r, off);
        if (ov > cmax || (ov == cmax && orr >= 0 && (r < 0 || orr < r))) { cmax = ov; r = orr; }
      }
      const double akk = fabs((double)A(j, j));
      int kind = 1, sa = -1, sb = -1, pz = 0;
      if (cmax == 0.0 || akk >= BK_ALPHA * cmax) {
        kind = 1;
      } else {
        // largest off-diagonal magnitude in row/column r of the remaining
        // fully-summed block
        double rmax = 0.0;
        for (int i = j + lane; i < k; i += 64) {
          if (i == r) continue;
          const double v = i < r ? fabs((double)A(r, i)) : fabs((double)A(i, r));
          rmax = fmax(rmax, v);
        }
        for (int off = 32; off > 0; off >>= 1) rmax = fmax(rmax, __shfl_xor(rmax, off));
        const double arr = fabs((double)A(r, r));
        if (akk * rmax >= BK_ALPHA * cmax * cmax) {
          kind = 1;
        } else if (arr >= BK_ALPHA * rmax) {
          kind = 1;
          sa = j;
          sb = r;
        } else {
          kind = 2;
          if (r != j + 1) { sa = j + 1; sb = r; }
        }
      }
      if (lane == 0) {
        dec->kind = kind;
        dec->swap_a = sa;
        dec->swap_b = sb;
        dec->perturbed = pz;
      }
    }
    __syncthreads();
    const int kind = dec->kind;
    const int p = dec->swap_a, q = dec->swap_b;  // p < q
    // ---- symmetric interchange of indices p and q (lower storage)
    if (p >= 0) {
      for (int c = tid; c < f; c += NT) {
        if (c < p) {
          T tmp = A(p, c); A(p, c) = A(q, c); A(q, c) = tmp;
        } else if (c == p) {
          T tmp = A(p, p); A(p, p) = A(q, q); A(q, q) = tmp;
        } else if (c < q) {
          T tmp = A(c, p); A(c, p) = A(q, c); A(q, c) = tmp;
        } else if (c > q) {
          T tmp = A(c, p); A(c, p) = A(c, q); A(c, q) = tmp;
        }
      }
      if (tid == 0) { int tp = perm[p]; perm[p] = perm[q]; perm[q] = tp; }
    }
    __syncthreads();
    if (kind == 1) {
      double d = (double)A(j, j);
      if (fabs(d) < pivtol) {
        d = d < 0.0 ? -pivtol : pivtol;
        if (tid == 0) { A(j, j) = (T)d; ++pert; }
      }
      if (tid == 0) {
        if (d < 0.0) ++neg;
        type_out[j] = 1;
      }
      const double dinv = 1.0 / d;
      for (int i = j + 1 + tid; i < f; i += NT) {
        const double u = (double)A(i, j);
        lbuf[i] = u * dinv;     // L(i, j)
        lbuf[f + i] = u;        // unscaled column
      }
      __syncthreads();
      // trailing update a(i,m) -= L(i,j) * a(m,j), j < m <= i, on the
      // fully-summed columns only (the contribution block is updated once,
      // after the last pivot)
      for (int m = j + 1 + wave; m < k; m += NW) {
        const double um = lbuf[f + m];
        for (int i = m + lane; i < f; i += 64) A(i, m) = (T)((double)A(i, m) - lbuf[i] * um);
      }
      __syncthreads();
      for (int i = j + 1 + tid; i < f; i += NT) A(i, j) = (T)lbuf[i];
      j += 1;
    } else {
      const double d11 = (double)A(j, j), d21 = (double)A(j + 1, j), d22 = (double)A(j + 1, j + 1);
      const double det = d11 * d22 - d21 * d21;
      if (tid == 0) {
        if (det < 0.0) neg += 1;
        else if (d11 < 0.0) neg += 2;
        ++two;
        type_out[j] = 2;
        type_out[j + 1] = 3;
      }
      const double idet = 1.0 / det;
      // lbuf[i] = L(i, j), lbuf[f + i] = L(i, j+1); keep the unscaled
      // columns in place until the update is done
      for (int i = j + 2 + tid; i < f; i += NT) {
        const double u1 = (double)A(i, j), u2 = (double)A(i, j + 1);
        lbuf[i] = (u1 * d22 - u2 * d21) * idet;
        lbuf[f + i] = (u2 * d11 - u1 * d21) * idet;
      }
      __syncthreads();
      for (int m = j + 2 + wave; m < k; m += NW) {
        const double u1 = (double)A(m, j), u2 = (double)A(m, j + 1);
        for (int i = m + lane; i < f; i += 64)
          A(i, m) = (T)((double)A(i, m) - lbuf[i] * u1 - lbuf[f + i] * u2);
      }
      __syncthreads();
      for (int i = j + 2 + tid; i < f; i += NT) {
        A(i, j) = (T)lbuf[i];
        A(i, j + 1) = (T)lbuf[f + i];
      }
      j += 2;
    }
    __syncthreads();
  }
  // contribution block: C(i, m) -= sum_t L(i, t) W(m, t), k <= m <= i < f,
  // with W = L21 D (D block diagonal: 1x1 and 2x2 pivots).  Each thread
  // owns 4 x 4 tiles of the lower triangle of C, entries in registers.
  const int fk = f - k;
  const int nt = (fk + 3) >> 2, ntiles = nt * (nt + 1) / 2;
  for (int tl = tid; tl < ntiles; tl += NT) {
    int ti = (int)((sqrt(8.0 * tl + 1.0) - 1.0) * 0.5);
    while (ti * (ti + 1) / 2 > tl) --ti;
    while ((ti + 1) * (ti + 2) / 2 <= tl) ++ti;
    const int mi = tl - ti * (ti + 1) / 2;
    const int i0 = k + 4 * ti, m0 = k + 4 * mi;
    double acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
    int t = 0;
    while (t < k) {
      if (type_out[t] == 2) {
        const double d11 = (double)A(t, t), d21 = (double)A(t + 1, t), d22 = (double)A(t + 1, t + 1);
        double li0[4], li1[4], w0[4], w1[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          const int i = min(i0 + a, f - 1), m = min(m0 + a, f - 1);
          li0[a] = (double)A(i, t);
          li1[a] = (double)A(i, t + 1);
          const double lm0 = (double)A(m, t), lm1 = (double)A(m, t + 1);
          w0[a] = lm0 * d11 + lm1 * d21;
          w1[a] = lm0 * d21 + lm1 * d22;
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) acc[a][b] += li0[a] * w0[b] + li1[a] * w1[b];
        t += 2;
      } else {
        const double d = (double)A(t, t);
        double li[4], w[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          li[a] = (double)A(min(i0 + a, f - 1), t);
          w[a] = (double)A(min(m0 + a, f - 1), t) * d;
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) acc[a][b] += li[a] * w[b];
        t += 1;
      }
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int i = i0 + a, m = m0 + b;
        if (i < f && m <= i) A(i, m) = (T)((double)A(i, m) - acc[a][b]);
      }
  }
  __syncthreads();
  if (tid == 0) { *n_neg = neg; *n_pert = pert; *n_2x2 = two; }
}

// The front in LDS as a packed lower triangle (column j holds rows j..f-1),
// f (f + 1) / 2 entries, so that two workgroups fit on a CU.
template <class T, int MAXF>
__global__ void __launch_bounds__(256) front_factor_lds_kernel(FrontArgs fa, T* pool,
                                                             const int32_t* fronts,
                                                             double pivtol) {
  __shared__ T sa[MAXF * (MAXF + 1) / 2];
  __shared__ double lbuf[2 * MAXF];
  __shared__ int perm[MAXF];
  __shared__ int32_t type[MAXF];
  __shared__ PivotStep dec;
  const int F = fronts[blockIdx.x];
  const int f = fa.ff[F], k = fa.fk[F];
  T* g = pool + fa.pool_off[F];
  auto pk = [f](int i, int j) { return j * f - ((j * (j - 1)) >> 1) + (i - j); };
  const int n2 = f * f;
  // eight loads in flight per thread before their LDS stores
  for (int e0 = threadIdx.x; e0 < n2; e0 += 8 * 256) {
    T v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = e0 + 256 * q;
      v[q] = e < n2 && (e % f) >= (e / f) ? g[e] : (T)0;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = e0 + 256 * q;
      const int c = e / f, r = e % f;
      if (e < n2 && r >= c) sa[pk(r, c)] = v[q];
    }
  }
  __syncthreads();
  int neg = 0, pert = 0, two = 0;
  auto A = [&](int i, int j) -> T& { return sa[pk(i, j)]; };
  ldlt_partial<T, 256>(A, f, k, lbuf, perm, &dec, pivtol, &neg, &pert, &two, type);
  __syncthreads();
  for (int e = threadIdx.x; e < n2; e += blockDim.x) {
    const int c = e / f, r = e % f;
    if (r >= c) g[e] = sa[pk(r, c)];
  }
  const int start = fa.fstart[F];
  for (int t = threadIdx.x; t < k; t += blockDim.x) {
    fa.piv_perm[start + t] = perm[t];
    fa.piv_type[start + t] = type[t];
  }
  if (threadIdx.x == 0) {
    fa.stat[4 * F + 0] = neg;
    fa.stat[4 * F + 1] = pert;
    fa.stat[4 * F + 2] = two;
  }
}

FrontArgs front_args(riga_problem* pr, Factor& F) {
  FrontArgs fa{};
  fa.fk = pr->d_fk.p;
  fa.ff = pr->d_ff.p;
  fa.fstart = pr->d_fstart.p;
  fa.pool_off = pr->d_pool_off.p;
  fa.child_ptr = pr->d_child_ptr.p;
  fa.child_list = pr->d_child_list.p;
  fa.inv_off = pr->d_inv_off.p;
  fa.inv = pr->d_inv.p;
  fa.amap_ptr = pr->d_amap_ptr.p;
  fa.amap_row = pr->d_amap_row.p;
  fa.amap_val = pr->d_amap_val.p;
  fa.kv = pr->kv.p;
  fa.mv = pr->mv.p;
  fa.piv_perm = F.piv_perm.p;
  fa.piv_type = F.piv_type.p;
  fa.stat = F.front_stat.p;
  return fa;
}

template <class T, int MAXF>
void factor_levels(riga_problem* pr, Factor& F, T* pool, T* hpool, double sigma, bool checked,
                   hipStream_t s) {
  FrontArgs fa = front_args(pr, F);
  // a pivot below pivtol is replaced by +-pivtol and counted (static
  // pivoting); RIGA_PIVTOL_REL overrides the relative threshold 1e-20
  double rel = 1e-20;
  if (const char* v = std::getenv("RIGA_PIVTOL_REL")) rel = std::atof(v);
  const double pivtol = rel * (pr->normK1 + fabs(sigma) * pr->normM1);
  set_kernel_attributes();
  for (size_t h = 0; h < pr->levels.size(); ++h) {
    LevelDev& L = pr->levels[h];
    if (L.n == 0) continue;
    front_assemble_kernel<T><<<(unsigned)L.cols, 64 * L.asm_cols,
                               (size_t)L.asm_cols * L.max_f * sizeof(double), s>>>(
        fa, pool, L.fronts.p, L.col_prefix.p, L.n, L.asm_cols, sigma);
    HIPCHECK(hipGetLastError());
    const int ns = L.n_upto(MAXF);
    if (ns > 0) {
      front_factor_lds_kernel<T, MAXF><<<ns, 256, 0, s>>>(fa, pool, L.fronts.p, pivtol);
      HIPCHECK(hipGetLastError());
    }
    if (L.n > ns) {
      std::vector<int> bf(L.host_f.begin() + ns, L.host_f.end());
      std::vector<int> bk(L.host_k.begin() + ns, L.host_k.end());
      factor_big_fronts<T>(pr, F, pool, L.fronts.p + ns, bf, bk, pivtol, (int)h, checked, s);
    }
  }
  launch_front_inverse<T>(pr, F, pool, hpool, s);
  launch_pivot_maps(pr, F, s);
}

}  // namespace

void set_front_attributes() {
  HIPCHECK(hipFuncSetAttribute((const void*)front_assemble_kernel<double>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, ASM_LDS));
  HIPCHECK(hipFuncSetAttribute((const void*)front_assemble_kernel<float>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, ASM_LDS));
}

void factor_reserve(riga_problem* pr, Factor& F, int precision, hipStream_t s) {
  const Analysis& an = pr->an;
  const int64_t N = an.N;
  const size_t gs = (size_t)pr->gstride;
  if (F.piv_perm.n < (size_t)N) {
    F.piv_perm.alloc(N, s);
    F.piv_type.alloc(N, s);
    F.piv_dof.alloc(N, s);
    F.piv_gmap.alloc((size_t)N * gs, s);
    F.piv_inv.alloc(N, s);
    F.rows_piv.alloc(std::max<int64_t>(an.f_rows_off[an.n_fronts], 1), s);
    F.d_diag.alloc(N, s);
    F.d_sub.alloc(N, s);
    F.dcoef.alloc((size_t)N * 3, s);
    F.front_stat.alloc((size_t)an.n_fronts * 4, s);
    F.cbvec.alloc(std::max<int64_t>(an.cb_size, 1), s);
    F.fwd.alloc(N, s);
  }
  if (F.av.n < pr->kv.n) F.av.alloc(pr->kv.n, s);
  if (precision == RIGA_MIXED) {
    if (F.pool32.n < (size_t)an.pool_size) F.pool32.alloc(an.pool_size, s);
    if (F.h32.n < (size_t)an.h_size) F.h32.alloc(an.h_size, s);
    bigfront_reserve(pr, F, LDS_FRONT_MAX_F32, s);
  } else {
    if (F.pool64.n < (size_t)an.pool_size) F.pool64.alloc(an.pool_size, s);
    if (F.h64.n < (size_t)an.h_size) F.h64.alloc(an.h_size, s);
    bigfront_reserve(pr, F, LDS_FRONT_MAX_F64, s);
  }
  top_reserve(pr, F, precision, s);
}

void factor_numeric(riga_problem* pr, Factor& F, double sigma, int precision, hipStream_t s) {
  const Analysis& an = pr->an;
  F.factored = false;
  if (F.av.n < pr->kv.n) throw Error(RIGA_EINVAL, "factorisation buffers not reserved");
  if (precision == RIGA_MIXED) {
    if (F.pool32.n < (size_t)an.pool_size || F.h32.n < (size_t)an.h_size)
      throw Error(RIGA_EINVAL, "factorisation buffers not reserved");
  } else if (F.pool64.n < (size_t)an.pool_size || F.h64.n < (size_t)an.h_size) {
    throw Error(RIGA_EINVAL, "factorisation buffers not reserved");
  }
  const size_t nlev = pr->levels.size();
  std::vector<int32_t> st((size_t)an.n_fronts * 4), pend(nlev, 0);
  // the blocked fronts run their predicted panel steps without waiting for
  // the host; in the rare case that a front needed more, the whole
  // factorisation is repeated with the host checking every level
  // (RIGA_FACTOR_CHECKED=1 checks every level from the start)
  const char* ev = std::getenv("RIGA_FACTOR_CHECKED");
  const int first = (ev && *ev == '1') ? 1 : 0;
  for (int pass = first; pass < 2; ++pass) {
    const bool checked = pass == 1;
    if (nlev) HIPCHECK(hipMemsetAsync(F.big_pend.p, 0, nlev * sizeof(int32_t), s));
    if (precision == RIGA_MIXED) {
      factor_levels<float, LDS_FRONT_MAX_F32>(pr, F, F.pool32.p, F.h32.p, sigma, checked, s);
      build_top<float>(pr, F, F.h32.p, F.trow32.p, F.tcol32.p, s);
    } else {
      factor_levels<double, LDS_FRONT_MAX_F64>(pr, F, F.pool64.p, F.h64.p, sigma, checked, s);
      build_top<double>(pr, F, F.h64.p, F.trow64.p, F.tcol64.p, s);
    }
    // K - sigma M for the refinement residuals (mixed precision, and FP64
    // solves refined after a stall)
    launch_axpby_vals(pr->kv.p, pr->mv.p, sigma, F.av.p, (int64_t)pr->kv.n, s);
    HIPCHECK(hipMemcpyAsync(st.data(), F.front_stat.p, st.size() * sizeof(int32_t),
                            hipMemcpyDeviceToHost, s));
    if (nlev)
      HIPCHECK(hipMemcpyAsync(pend.data(), F.big_pend.p, nlev * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    if (std::all_of(pend.begin(), pend.end(), [](int32_t v) { return v == 0; })) break;
  }
  int64_t neg = 0;
  int pert = 0, two = 0;
  for (int f = 0; f < an.n_fronts; ++f) {
    neg += st[4 * f];
    pert += st[4 * f + 1];
    two += st[4 * f + 2];
  }
  F.inertia = neg;
  F.perturbed = pert;
  F.two = two;
  F.sigma = sigma;
  F.precision = precision;
  F.factored = true;
}

}  // namespace riga
