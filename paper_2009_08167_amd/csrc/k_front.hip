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
#include <cstring>
#include <memory>
#include <mutex>

#include "problem.h"
#include "wave_reduce.h"

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
  const int32_t* ident;  // per front: 1 if its one child's update block is the front, row for row
};

// workgroup gid of an assembly launch: cpw consecutive columns of one front,
// one wave each, lanes over rows; the column is built in LDS and written once
template <class T>
__device__ __forceinline__ void front_assemble_body(const FrontArgs& fa, T* pool, const int32_t* fronts,
                                                    const int64_t* col_prefix, int nf, int cpw,
                                                    double sigma, int64_t gid) {
  extern __shared__ double cols[];
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
  if (j < f && nc == 1 && fa.ident[F]) {
    // (a front of a split separator's chain: its child's update block,
    // column j, rows j.. are contiguous in the child's pool slot)
    const int C = fa.child_list[c0];
    const int kc = fa.fk[C], fc = fa.ff[C];
    const T* src = pool + fa.pool_off[C] + (int64_t)(kc + j) * fc + kc;
    for (int r0 = j; r0 < f; r0 += 64 * 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int r = r0 + lane + 64 * u;
        v[u] = r < f ? (double)src[r] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int r = r0 + lane + 64 * u;
        if (r < f) col[r] = v[u];
      }
    }
  } else if (j < f) {
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
    // per child holding column j (a wave-uniform test): the map entries of
    // AU rows, then their values, each batch of loads in flight together;
    // the children are added in their fixed order
    constexpr int AU = 8;
    for (int r0 = j; r0 < f; r0 += 64 * AU) {
      double t[AU];
#pragma unroll
      for (int u = 0; u < AU; ++u) t[u] = 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (cc[q] < 0) continue;
        const T* src = pool + po[q] + (int64_t)(kc[q] + cc[q]) * fc[q] + kc[q];
        int cr[AU];
#pragma unroll
        for (int u = 0; u < AU; ++u) {
          const int r = r0 + lane + 64 * u;
          cr[u] = r < f ? inv[q][r] : -1;
        }
        double v[AU];
#pragma unroll
        for (int u = 0; u < AU; ++u) v[u] = cr[u] >= 0 ? (double)src[cr[u]] : 0.0;
#pragma unroll
        for (int u = 0; u < AU; ++u)
          if (cr[u] >= 0) t[u] += v[u];
      }
#pragma unroll
      for (int u = 0; u < AU; ++u) {
        const int r = r0 + lane + 64 * u;
        if (r < f) col[r] = t[u];
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

template <class T>
__global__ void __launch_bounds__(64 * ASM_COLS) front_assemble_kernel(FrontArgs fa, T* pool,
                                                                     const int32_t* fronts,
                                                                     const int64_t* col_prefix,
                                                                     int nf, int cpw, double sigma) {
  front_assemble_body<T>(fa, pool, fronts, col_prefix, nf, cpw, sigma, blockIdx.x);
}

// One height of several problems: job j owns workgroups [g0, next job's g0).
struct AsmJob {
  FrontArgs fa;
  void* pool;
  const int32_t* fronts;
  const int64_t* col_prefix;
  int64_t g0;
  double sigma;
  int32_t nf, cpw;
};

template <class T>
__global__ void __launch_bounds__(64 * ASM_COLS) front_assemble_batched_kernel(const AsmJob* jobs, int njobs) {
  const int64_t gid = blockIdx.x;
  int lo = 0, hi = njobs;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (jobs[mid].g0 <= gid) lo = mid; else hi = mid;
  }
  const AsmJob& J = jobs[lo];
  front_assemble_body<T>(J.fa, static_cast<T*>(J.pool), J.fronts, J.col_prefix, J.nf, J.cpw, J.sigma,
                         gid - J.g0);
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
// of order k.  NT threads.  `perm` holds k ints, `dec` the broadcast
// decision.  Works for `a` in LDS or in global memory.
template <class T, int NT, class Acc>
__device__ __forceinline__ void ldlt_partial(Acc A, int f, int k, int* perm,
                                             PivotStep* dec, double pivtol, int* n_neg,
                                             int* n_pert, int* n_2x2, int32_t* type_out) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  constexpr int NW = NT / 64;
  for (int t = tid; t < k; t += NT) perm[t] = t;
  int neg = 0, pert = 0, two = 0;
  __syncthreads();
  int j = 0;
  // The column(s) of a pivot are scaled into L lazily, by waves 1.. while
  // wave 0 takes the next decision (which reads later columns only); the
  // rank-1/2 update uses the unscaled columns.  Two barriers per pivot (one
  // more with an interchange).
  int pj = -1, pkind = 0;
  double p11 = 0.0, p21 = 0.0, p22 = 0.0;
  auto scale_pending = [&](int t0, int nt) {
    if (pkind == 1) {
      const double dinv = 1.0 / p11;
      for (int i = pj + 1 + t0; i < f; i += nt) A(i, pj) = (T)((double)A(i, pj) * dinv);
    } else if (pkind == 2) {
      const double idet = 1.0 / (p11 * p22 - p21 * p21);
      for (int i = pj + 2 + t0; i < f; i += nt) {
        const double u1 = (double)A(i, pj), u2 = (double)A(i, pj + 1);
        A(i, pj) = (T)((u1 * p22 - u2 * p21) * idet);
        A(i, pj + 1) = (T)((u2 * p11 - u1 * p21) * idet);
      }
    }
  };
  while (j < k) {
    // ---- pivot decision (wave 0); the previous pivot's scaling (others)
    if (wave == 0) {
      double cmax = 0.0;
      int r = -1;
      for (int i = j + 1 + lane; i < k; i += 64) {
        const double v = fabs((double)A(i, j));
        if (v > cmax) { cmax = v; r = i; }
      }
      wave_argmax(cmax, r);
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
        rmax = wave_max(rmax);
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
    } else {
      scale_pending(tid - 64, NT - 64);
    }
    __syncthreads();
    pkind = 0;
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
      __syncthreads();
    }
    if (kind == 1) {
      double d = (double)A(j, j);
      const bool small = fabs(d) < pivtol;
      if (small) d = d < 0.0 ? -pivtol : pivtol;
      if (tid == 0) {
        if (small) ++pert;
        if (d < 0.0) ++neg;
        type_out[j] = 1;
      }
      // trailing update a(i,m) -= a(i,j) a(m,j) / d, j < m <= i, on the
      // fully-summed columns only (the contribution block is updated once,
      // after the last pivot)
      const double dinv = 1.0 / d;
      for (int m = j + 1 + wave; m < k; m += NW) {
        const double um = (double)A(m, j) * dinv;
        for (int i = m + lane; i < f; i += 64) A(i, m) = (T)((double)A(i, m) - (double)A(i, j) * um);
      }
      __syncthreads();
      if (tid == 0 && small) A(j, j) = (T)d;
      pj = j;
      pkind = 1;
      p11 = d;
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
      // a(i,m) -= [a_ij a_ij+1] D^{-1} [a_mj; a_mj+1] with the unscaled columns
      for (int m = j + 2 + wave; m < k; m += NW) {
        const double u1 = (double)A(m, j), u2 = (double)A(m, j + 1);
        const double w1 = (u1 * d22 - u2 * d21) * idet, w2 = (u2 * d11 - u1 * d21) * idet;
        for (int i = m + lane; i < f; i += 64)
          A(i, m) = (T)((double)A(i, m) - ((double)A(i, j) * w1 + (double)A(i, j + 1) * w2));
      }
      __syncthreads();
      pj = j;
      pkind = 2;
      p11 = d11;
      p21 = d21;
      p22 = d22;
      j += 2;
    }
  }
  // the last pivot's column(s)
  scale_pending(tid, NT);
  __syncthreads();
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

// bytes of the packed lower triangle of a front of order f
template <class T>
constexpr size_t lds_front_bytes(int f) { return (size_t)f * (f + 1) / 2 * sizeof(T); }

// The front in LDS as a packed lower triangle (column j holds rows j..f-1),
// f (f + 1) / 2 entries in dynamic LDS sized by the launch's largest front,
// so that two workgroups fit on a CU at the largest orders and more on the
// levels of small fronts.
template <class T, int MAXF>
__device__ __forceinline__ void front_factor_lds_body(const FrontArgs& fa, T* pool, const int32_t* fronts,
                                                      double pivtol, int blk) {
  extern __shared__ double lds_front[];
  T* sa = reinterpret_cast<T*>(lds_front);
  __shared__ int perm[MAXF];
  __shared__ int32_t type[MAXF];
  __shared__ PivotStep dec;
  const int F = fronts[blk];
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
  ldlt_partial<T, 256>(A, f, k, perm, &dec, pivtol, &neg, &pert, &two, type);
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

template <class T, int MAXF>
__global__ void __launch_bounds__(256) front_factor_lds_kernel(FrontArgs fa, T* pool,
                                                             const int32_t* fronts,
                                                             double pivtol) {
  front_factor_lds_body<T, MAXF>(fa, pool, fronts, pivtol, blockIdx.x);
}

// One height of several problems: job j owns workgroups [y0, next job's y0).
struct LdsJob {
  FrontArgs fa;
  void* pool;
  const int32_t* fronts;
  double pivtol;
  int64_t y0;
};

template <class T, int MAXF>
__global__ void __launch_bounds__(256) front_factor_lds_batched_kernel(const LdsJob* jobs, int njobs) {
  const int64_t y = blockIdx.x;
  int lo = 0, hi = njobs;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (jobs[mid].y0 <= y) lo = mid; else hi = mid;
  }
  const LdsJob& J = jobs[lo];
  front_factor_lds_body<T, MAXF>(J.fa, static_cast<T*>(J.pool), J.fronts, J.pivtol, (int)(y - J.y0));
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
  fa.ident = pr->d_asm_ident.p;
  return fa;
}

// a pivot below the tolerance is replaced by +-tolerance and counted (static
// pivoting); RIGA_PIVTOL_REL overrides the relative threshold 1e-20
double pivot_tolerance(const riga_problem* pr, double sigma) {
  double rel = 1e-20;
  if (const char* v = std::getenv("RIGA_PIVTOL_REL")) rel = std::atof(v);
  return rel * (pr->normK1 + fabs(sigma) * pr->normM1);
}

template <class T, int MAXF>
void factor_levels(riga_problem* pr, Factor& F, T* pool, double sigma, bool checked, hipStream_t s) {
  FrontArgs fa = front_args(pr, F);
  const double pivtol = pivot_tolerance(pr, sigma);
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
      front_factor_lds_kernel<T, MAXF><<<ns, 256, lds_front_bytes<T>(L.host_f[ns - 1]), s>>>(
          fa, pool, L.fronts.p, pivtol);
      HIPCHECK(hipGetLastError());
    }
    if (L.n > ns) {
      std::vector<int> bf(L.host_f.begin() + ns, L.host_f.end());
      std::vector<int> bk(L.host_k.begin() + ns, L.host_k.end());
      factor_big_fronts<T>(pr, F, pool, L.fronts.p + ns, bf, bk, pivtol, (int)h, checked, s);
    }
  }
}

}  // namespace

void set_front_attributes() {
  HIPCHECK(hipFuncSetAttribute((const void*)front_factor_lds_kernel<double, 128>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_front_bytes<double>(128)));
  HIPCHECK(hipFuncSetAttribute((const void*)front_factor_lds_kernel<float, 176>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_front_bytes<float>(176)));
  HIPCHECK(hipFuncSetAttribute((const void*)front_factor_lds_batched_kernel<double, 128>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_front_bytes<double>(128)));
  HIPCHECK(hipFuncSetAttribute((const void*)front_factor_lds_batched_kernel<float, 176>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_front_bytes<float>(176)));
  HIPCHECK(hipFuncSetAttribute((const void*)front_assemble_kernel<double>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, ASM_LDS));
  HIPCHECK(hipFuncSetAttribute((const void*)front_assemble_kernel<float>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, ASM_LDS));
  HIPCHECK(hipFuncSetAttribute((const void*)front_assemble_batched_kernel<double>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, ASM_LDS));
  HIPCHECK(hipFuncSetAttribute((const void*)front_assemble_batched_kernel<float>,
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
    if (F.h32.n < (size_t)an.h_size) F.h32.alloc(an.h_size, s);
    bigfront_reserve(pr, F, LDS_FRONT_MAX_F32, s);
  } else {
    if (F.h64.n < (size_t)an.h_size) F.h64.alloc(an.h_size, s);
    bigfront_reserve(pr, F, LDS_FRONT_MAX_F64, s);
  }
  top_reserve(pr, F, precision, s);
}

namespace {

void check_reserved(const riga_problem* pr, const Factor& F, int precision) {
  const Analysis& an = pr->an;
  if (F.av.n < pr->kv.n) throw Error(RIGA_EINVAL, "factorisation buffers not reserved");
  if (precision == RIGA_MIXED) {
    if (F.h32.n < (size_t)an.h_size) throw Error(RIGA_EINVAL, "factorisation buffers not reserved");
  } else if (F.h64.n < (size_t)an.h_size) {
    throw Error(RIGA_EINVAL, "factorisation buffers not reserved");
  }
}

// A second pool slot up to this size stays allocated for the next overlap
constexpr size_t POOL_KEEP_BYTES = (size_t)1 << 30;

SolveCtx& ctx_of(riga_problem* pr, const Factor& F) {
  for (SolveCtx& c : pr->ctx)
    if (&F == &c.fac[0] || &F == &c.fac[1]) return c;
  throw Error(RIGA_EINVAL, "factorisation outside the problem's solve contexts");
}

// The front pool of one factorisation of F: a free slot of F's context,
// sized on first use; held until destruction, which waits for the
// factorisation's stream first.
struct PoolLease {
  SolveCtx* c = nullptr;
  int slot = -1;
  hipStream_t s = nullptr;
  void* p = nullptr;
  size_t bytes = 0;
  bool mixed = false;
  PoolLease(riga_problem* pr, Factor& F, int precision, hipStream_t st) : s(st) {
    c = &ctx_of(pr, F);
    {
      std::lock_guard<std::mutex> lk(c->pool_mu);
      for (int i = 0; i < 2 && slot < 0; ++i)
        if (!c->pool_busy[i]) {
          c->pool_busy[i] = true;
          slot = i;
        }
    }
    if (slot < 0) throw Error(RIGA_EDEVICE, "more than two factorisations at once in one solve context");
    const size_t n = (size_t)pr->an.pool_size;
    mixed = precision == RIGA_MIXED;
    // (allocated on the problem's own stream, as its other persistent
    // buffers: a factorisation's stream may not outlive the pool)
    try {
      if (mixed) {
        if (c->pool32[slot].n < n) c->pool32[slot].alloc(n, pr->home);
        p = c->pool32[slot].p;
        bytes = n * sizeof(float);
      } else {
        if (c->pool64[slot].n < n) c->pool64[slot].alloc(n, pr->home);
        p = c->pool64[slot].p;
        bytes = n * sizeof(double);
      }
    } catch (...) {
      std::lock_guard<std::mutex> lk(c->pool_mu);
      c->pool_busy[slot] = false;
      throw;
    }
  }
  PoolLease(const PoolLease&) = delete;
  PoolLease& operator=(const PoolLease&) = delete;
  template <class T>
  T* get() const { return static_cast<T*>(p); }
  ~PoolLease() {
    if (slot < 0) return;
    (void)hipStreamSynchronize(s);
    if (slot == 1 && bytes > POOL_KEEP_BYTES) {
      if (mixed) c->pool32[1].reset();
      else c->pool64[1].reset();
    }
    std::lock_guard<std::mutex> lk(c->pool_mu);
    c->pool_busy[slot] = false;
  }
};

// after the levels: partitioned inverses, sweep maps, the top block and
// K - sigma M for the refinement residuals (mixed precision, and FP64
// solves refined after a stall); queues the copies of the per-front counts
// and the pending counters into st and pend
void factor_tail(riga_problem* pr, Factor& F, const PoolLease& pool, double sigma, int precision,
                 std::vector<int32_t>& st, std::vector<int32_t>& pend, hipStream_t s) {
  const size_t nlev = pr->levels.size();
  if (precision == RIGA_MIXED) {
    launch_front_inverse<float>(pr, F, pool.get<float>(), F.h32.p, s);
    launch_pivot_maps(pr, F, s);
    build_top<float>(pr, F, F.h32.p, F.trow32.p, F.tcol32.p, s);
  } else {
    launch_front_inverse<double>(pr, F, pool.get<double>(), F.h64.p, s);
    launch_pivot_maps(pr, F, s);
    build_top<double>(pr, F, F.h64.p, F.trow64.p, F.tcol64.p, s);
  }
  launch_axpby_vals(pr->kv.p, pr->mv.p, sigma, F.av.p, (int64_t)pr->kv.n, s);
  st.assign((size_t)pr->an.n_fronts * 4, 0);
  pend.assign(nlev, 0);
  HIPCHECK(hipMemcpyAsync(st.data(), F.front_stat.p, st.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  if (nlev) HIPCHECK(hipMemcpyAsync(pend.data(), F.big_pend.p, nlev * sizeof(int32_t), hipMemcpyDeviceToHost, s));
}

// inertia and pivot counts from the per-front counts (after synchronising)
void factor_done(riga_problem* pr, Factor& F, double sigma, int precision, const std::vector<int32_t>& st) {
  int64_t neg = 0;
  int pert = 0, two = 0;
  for (int f = 0; f < pr->an.n_fronts; ++f) {
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

bool all_zero(const std::vector<int32_t>& v) {
  return std::all_of(v.begin(), v.end(), [](int32_t x) { return x == 0; });
}

}  // namespace

void factor_numeric(riga_problem* pr, Factor& F, double sigma, int precision, hipStream_t s) {
  F.factored = false;
  F.pre = false;
  check_reserved(pr, F, precision);
  const size_t nlev = pr->levels.size();
  std::vector<int32_t> st, pend;
  const PoolLease pool(pr, F, precision, s);
  // the blocked fronts run their predicted panel steps without waiting for
  // the host; in the rare case that a front needed more, the whole
  // factorisation is repeated with the host checking every level
  // (RIGA_FACTOR_CHECKED=1 checks every level from the start)
  const char* ev = std::getenv("RIGA_FACTOR_CHECKED");
  const int first = (ev && *ev == '1') ? 1 : 0;
  for (int pass = first; pass < 2; ++pass) {
    const bool checked = pass == 1;
    if (nlev) HIPCHECK(hipMemsetAsync(F.big_pend.p, 0, nlev * sizeof(int32_t), s));
    if (precision == RIGA_MIXED)
      factor_levels<float, LDS_FRONT_MAX_F32>(pr, F, pool.get<float>(), sigma, checked, s);
    else
      factor_levels<double, LDS_FRONT_MAX_F64>(pr, F, pool.get<double>(), sigma, checked, s);
    factor_tail(pr, F, pool, sigma, precision, st, pend, s);
    HIPCHECK(hipStreamSynchronize(s));
    if (all_zero(pend)) break;
  }
  factor_done(pr, F, sigma, precision, st);
}

namespace {

// The argument blocks of one batched factorisation, every height's in one
// device table: per height, the assembly jobs grouped by columns per
// workgroup, the LDS jobs and the blocked-front jobs.
struct BatchHeight {
  struct AsmGroup {
    size_t off;  // byte offset of the AsmJob array
    int njobs, cpw;
    int64_t blocks;
    size_t lds;
  };
  std::vector<AsmGroup> asm_groups;
  size_t lds_off = 0;
  int lds_jobs = 0;
  int64_t lds_blocks = 0;
  int lds_max_f = 0;  // largest front of the LDS jobs
  size_t big_off = 0, big_ystart_off = 0;
  int big_jobs = 0;
  BigPlan big;
};

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

template <class T, int MAXF>
void factor_levels_batched(const std::vector<riga_problem*>& prs, const std::vector<Factor*>& Fs,
                           const std::vector<double>& sigmas, const std::vector<T*>& pools,
                           std::vector<uint8_t>& tab, DBuf<uint8_t>& dtab, hipStream_t s) {
  const int count = (int)prs.size();
  size_t H = 0;
  for (riga_problem* pr : prs) H = std::max(H, pr->levels.size());
  std::vector<double> pivtol(count);
  std::vector<FrontArgs> fas(count);
  for (int i = 0; i < count; ++i) {
    pivtol[i] = pivot_tolerance(prs[i], sigmas[i]);
    fas[i] = front_args(prs[i], *Fs[i]);
  }
  // host image of the table
  tab.clear();
  auto put = [&](const void* src, size_t bytes) {
    const size_t off = align_up(tab.size());
    tab.resize(off + bytes);
    std::memcpy(tab.data() + off, src, bytes);
    return off;
  };
  const size_t big_bytes = big_args_bytes();
  std::vector<BatchHeight> hts(H);
  for (size_t h = 0; h < H; ++h) {
    BatchHeight& B = hts[h];
    // assembly: one group per columns-per-workgroup value
    std::vector<std::pair<int, std::vector<AsmJob>>> groups;
    std::vector<LdsJob> lds;
    std::vector<uint8_t> bigs;
    std::vector<int32_t> ystart(1, 0);
    std::vector<int> all_f, all_k;
    for (int i = 0; i < count; ++i) {
      riga_problem* pr = prs[i];
      if (h >= pr->levels.size()) continue;
      LevelDev& L = pr->levels[h];
      if (L.n == 0) continue;
      auto g = std::find_if(groups.begin(), groups.end(), [&](const auto& x) { return x.first == L.asm_cols; });
      if (g == groups.end()) {
        groups.emplace_back(L.asm_cols, std::vector<AsmJob>());
        g = groups.end() - 1;
      }
      AsmJob aj{};
      aj.fa = fas[i];
      aj.pool = pools[i];
      aj.fronts = L.fronts.p;
      aj.col_prefix = L.col_prefix.p;
      aj.g0 = 0;  // set below, once the group is complete
      aj.sigma = sigmas[i];
      aj.nf = L.n;
      aj.cpw = L.asm_cols;
      g->second.push_back(aj);
      const int ns = L.n_upto(MAXF);
      if (ns > 0) {
        LdsJob lj{};
        lj.fa = fas[i];
        lj.pool = pools[i];
        lj.fronts = L.fronts.p;
        lj.pivtol = pivtol[i];
        lj.y0 = B.lds_blocks;
        lds.push_back(lj);
        B.lds_blocks += ns;
        B.lds_max_f = std::max(B.lds_max_f, L.host_f[ns - 1]);
      }
      if (L.n > ns) {
        std::vector<int> bf(L.host_f.begin() + ns, L.host_f.end());
        std::vector<int> bk(L.host_k.begin() + ns, L.host_k.end());
        const BigPlan P = big_plan(bf, bk);
        const size_t o = bigs.size();
        bigs.resize(o + big_bytes);
        big_args_fill(pr, *Fs[i], pools[i], L.fronts.p + ns, P, pivtol[i], (int)h, bigs.data() + o);
        ystart.push_back(ystart.back() + P.nbig);
        B.big.nbig += P.nbig;
        B.big.steps = std::max(B.big.steps, P.steps);
        B.big.maxk = std::max(B.big.maxk, P.maxk);
        B.big.maxcb = std::max(B.big.maxcb, P.maxcb);
        B.big.max_tiles = std::max(B.big.max_tiles, P.max_tiles);
        B.big.max_cb_tiles = std::max(B.big.max_cb_tiles, P.max_cb_tiles);
      }
    }
    for (auto& g : groups) {
      // workgroup offsets of the group's jobs
      int64_t blocks = 0;
      size_t max_f = 0;
      int q = 0;
      for (int i = 0; i < count; ++i) {
        riga_problem* pr = prs[i];
        if (h >= pr->levels.size()) continue;
        LevelDev& L = pr->levels[h];
        if (L.n == 0 || L.asm_cols != g.first) continue;
        g.second[q].g0 = blocks;
        blocks += L.cols;
        max_f = std::max(max_f, (size_t)L.max_f);
        ++q;
      }
      BatchHeight::AsmGroup ag;
      ag.off = put(g.second.data(), g.second.size() * sizeof(AsmJob));
      ag.njobs = (int)g.second.size();
      ag.cpw = g.first;
      ag.blocks = blocks;
      ag.lds = (size_t)g.first * max_f * sizeof(double);
      B.asm_groups.push_back(ag);
    }
    if (!lds.empty()) {
      B.lds_off = put(lds.data(), lds.size() * sizeof(LdsJob));
      B.lds_jobs = (int)lds.size();
    }
    if (B.big.nbig > 0) {
      B.big_off = put(bigs.data(), bigs.size());
      B.big_ystart_off = put(ystart.data(), ystart.size() * sizeof(int32_t));
      B.big_jobs = (int)ystart.size() - 1;
    }
  }
  if (tab.empty()) return;
  dtab.alloc(tab.size(), s);
  HIPCHECK(hipMemcpyAsync(dtab.p, tab.data(), tab.size(), hipMemcpyHostToDevice, s));
  set_kernel_attributes();
  for (size_t h = 0; h < H; ++h) {
    const BatchHeight& B = hts[h];
    for (const auto& ag : B.asm_groups) {
      front_assemble_batched_kernel<T><<<(unsigned)ag.blocks, 64 * ag.cpw, ag.lds, s>>>(
          reinterpret_cast<const AsmJob*>(dtab.p + ag.off), ag.njobs);
      HIPCHECK(hipGetLastError());
    }
    if (B.lds_jobs > 0) {
      front_factor_lds_batched_kernel<T, MAXF><<<(unsigned)B.lds_blocks, 256,
                                                 lds_front_bytes<T>(B.lds_max_f), s>>>(
          reinterpret_cast<const LdsJob*>(dtab.p + B.lds_off), B.lds_jobs);
      HIPCHECK(hipGetLastError());
    }
    if (B.big_jobs > 0)
      factor_big_fronts_batched<T>(dtab.p + B.big_off, reinterpret_cast<const int32_t*>(dtab.p + B.big_ystart_off),
                                   B.big_jobs, B.big, s);
  }
}

}  // namespace

void factor_numeric_batched(const std::vector<riga_problem*>& prs, const std::vector<Factor*>& Fs,
                            const std::vector<double>& sigmas, int precision, hipStream_t s) {
  const int count = (int)prs.size();
  for (int i = 0; i < count; ++i) {
    Fs[i]->factored = false;
    Fs[i]->pre = false;
    check_reserved(prs[i], *Fs[i], precision);
    const size_t nlev = prs[i]->levels.size();
    if (nlev) HIPCHECK(hipMemsetAsync(Fs[i]->big_pend.p, 0, nlev * sizeof(int32_t), s));
  }
  // the job table (host image and device copy) lives until the
  // synchronisation below
  std::vector<uint8_t> tab;
  DBuf<uint8_t> dtab;
  std::vector<std::unique_ptr<PoolLease>> lease(count);
  for (int i = 0; i < count; ++i) lease[i].reset(new PoolLease(prs[i], *Fs[i], precision, s));
  if (precision == RIGA_MIXED) {
    std::vector<float*> pools(count);
    for (int i = 0; i < count; ++i) pools[i] = lease[i]->get<float>();
    factor_levels_batched<float, LDS_FRONT_MAX_F32>(prs, Fs, sigmas, pools, tab, dtab, s);
  } else {
    std::vector<double*> pools(count);
    for (int i = 0; i < count; ++i) pools[i] = lease[i]->get<double>();
    factor_levels_batched<double, LDS_FRONT_MAX_F64>(prs, Fs, sigmas, pools, tab, dtab, s);
  }
  std::vector<std::vector<int32_t>> st(count), pend(count);
  for (int i = 0; i < count; ++i)
    factor_tail(prs[i], *Fs[i], *lease[i], sigmas[i], precision, st[i], pend[i], s);
  HIPCHECK(hipStreamSynchronize(s));
  lease.clear();  // (a repeat below takes its own)
  for (int i = 0; i < count; ++i) {
    // a blocked front that needed more panel steps than predicted: that
    // problem alone again, checked where needed
    if (all_zero(pend[i])) factor_done(prs[i], *Fs[i], sigmas[i], precision, st[i]);
    else factor_numeric(prs[i], *Fs[i], sigmas[i], precision, s);
  }
}

}  // namespace riga
