// Fronts larger than the LDS-resident limit: right-looking blocked LDL^T
// with Bunch-Kaufman pivoting inside the fully-summed block (the numeric
// factorisation of Sec. 4.1/5.1 of arXiv 2009.08167, per shift), with the
// work of one front spread over many workgroups.  All big fronts of one tree
// level advance together, one panel per step:
//
//  1. big_panel_kernel (one 1024-thread workgroup per front): the panel's
//     fully-summed rows [j0, k) x [j0, j0 + nb) are factorised in LDS.  The
//     1x1 / 2x2 test uses the column maximum over all fully-summed rows; the
//     2x2 partner is taken inside the panel, and when a column needs a
//     partner beyond it the panel ends early (kb < nb factorised columns).
//     Rows p, q of the earlier panels' L are interchanged in global memory.
//  2. big_cbrows_kernel (many workgroups): the update-block rows [k, f) of
//     the panel columns receive the same interchanges and eliminations:
//     lanes hold the panel columns, pivots are broadcast with readlane.
//  3. big_trailing_kernel (many workgroups): the trailing columns
//     [j0 + nb, k) of the fully-summed block, all rows below the diagonal,
//     receive A -= L_p W_p^T, W_p = L_p D_p, in 64 x 64 tiles on the MFMA
//     units (operands staged in LDS, the tile read-modified-written
//     coalesced).
//  After the last panel, big_cbupdate_kernel applies the whole rank-k update
//  to the update block [k, f)^2 at once.
//
// The panel start of each front lives in device memory, so the host issues
// a fixed number of steps computed for panels that never end early, then
// checks once per level whether any front needs more.  No workgroup waits
// for another: each step is three ordinary launches on one stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "mfma_tile.h"
#include "problem.h"
#include "wave_reduce.h"

namespace riga {
namespace {

constexpr int BF_NB = 64;        // widest panel
constexpr int BF_LDS = 18432;    // doubles of the panel kernel's LDS panel
constexpr int BF_TILE = 64;      // trailing-update tile
constexpr double BF_ALPHA = 0.6403882032022076;  // (1 + sqrt(17)) / 8

struct BigState {
  int32_t next;   // first column of the next panel
  int32_t cur;    // first column of the panel of this step
  int32_t kb;     // columns factorised in this step (0: nothing to do)
  int32_t nb;     // panel width of this step
  int32_t neg, pert, two, pad;
};

struct BigArgs {
  const int32_t* fronts;  // this level's big fronts
  const int32_t* ff;
  const int32_t* fk;
  const int32_t* fstart;
  const int64_t* pool_off;
  int32_t* piv_perm;      // by new index: front position of each pivot
  int32_t* piv_type;      // by new index: 1, or 2 / 3 for a 2x2 block
  int32_t* stat;          // per front: negative, perturbed, 2x2 pivots
  int32_t* perm;          // [slot * perm_stride]: running pivot order
  int64_t perm_stride;
  int32_t* lperm;         // [slot * BF_NB]: this step's panel column order
  BigState* st;
  double pivtol;
  void* pool;             // the factor pool (T*), for launches over several problems
  int32_t* pend;          // fronts left unfinished at the end (big_pending_kernel)
  int32_t nbig;
};

// Launches over the big fronts of one height of several problems: front y
// of the grid belongs to job j with ystart[j] <= y < ystart[j + 1] (jobs
// null: a single problem, the arguments passed by value).
struct BigJobs {
  const BigArgs* jobs;
  const int32_t* ystart;
  int njobs;
};

__device__ __forceinline__ int big_job_of(const BigJobs& J, int y) {
  int lo = 0, hi = J.njobs;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (J.ystart[mid] <= y) lo = mid; else hi = mid;
  }
  return lo;
}

// this workgroup's problem and front (y: its front index in the grid)
template <class T>
__device__ __forceinline__ void big_pick(const BigArgs& a0, T* pool0, const BigJobs& J, int y, BigArgs& a,
                                         T*& pool, int& b) {
  if (J.jobs) {
    const int j = big_job_of(J, y);
    a = J.jobs[j];
    pool = reinterpret_cast<T*>(a.pool);
    b = y - J.ystart[j];
  } else {
    a = a0;
    pool = pool0;
    b = y;
  }
}

struct Decision {
  int kind;   // 1 or 2
  int sa, sb; // interchange sa <-> sb (-1: none)
  int end;    // the panel ends before this column
};

// Panel width for a fully-summed remainder of m rows (LDS holds m x nb).
__host__ __device__ inline int panel_width(int m) {
  int nb = BF_LDS / m;
  nb = nb < BF_NB ? nb : BF_NB;
  nb = nb < m ? nb : m;
  return nb < 1 ? 1 : nb;
}

__device__ __forceinline__ double bcast(double v, int l) {
  const long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(bits & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Pivot steps with two workgroup barriers each: the column(s) of a pivot are
// scaled into L lazily, by waves 1.. while wave 0 takes the next decision
// (which reads only later columns); the rank-1/2 update uses the unscaled
// columns.
template <class T>
__global__ void __launch_bounds__(1024) big_panel_kernel(BigArgs a0, T* pool0, BigJobs J) {
  BigArgs a;
  T* pool;
  int b;
  big_pick(a0, pool0, J, blockIdx.x, a, pool, b);
  extern __shared__ double Pn[];
  __shared__ Decision dec;
  __shared__ int lp[BF_NB];
  constexpr int NT = 1024, NW = NT / 64;
  BigState* st = a.st + b;
  const int F = a.fronts[b];
  const int f = a.ff[F], k = a.fk[F], start = a.fstart[F];
  const int j0 = st->next;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (j0 >= k) {
    if (tid == 0) st->kb = 0;
    return;
  }
  T* A = pool + a.pool_off[F];
  int* perm = a.perm + (int64_t)b * a.perm_stride;
  int32_t* type_out = a.piv_type + start;
  const int m = k - j0;
  const int nb = panel_width(m);
  const int pend = j0 + nb;
  auto P = [&](int r, int c) -> double& { return Pn[(c - j0) * m + (r - j0)]; };
  for (int e = tid; e < nb * m; e += NT) {
    const int c = e / m, r = e % m;
    if (r >= c) Pn[e] = (double)A[(int64_t)(j0 + c) * f + j0 + r];
  }
  if (tid < nb) lp[tid] = tid;
  int neg = 0, pert = 0, two = 0;
  // pending scaling of the previous pivot's column(s)
  int pj = -1, pkind = 0;
  double p11 = 0.0, p21 = 0.0, p22 = 0.0;
  auto scale_pending = [&](int t0, int nt) {
    if (pkind == 1) {
      const double dinv = 1.0 / p11;
      for (int r = pj + 1 + t0; r < k; r += nt) P(r, pj) *= dinv;
    } else if (pkind == 2) {
      const double idet = 1.0 / (p11 * p22 - p21 * p21);
      for (int r = pj + 2 + t0; r < k; r += nt) {
        const double u1 = P(r, pj), u2 = P(r, pj + 1);
        P(r, pj) = (u1 * p22 - u2 * p21) * idet;
        P(r, pj + 1) = (u2 * p11 - u1 * p21) * idet;
      }
    }
  };
  __syncthreads();
  int jj = 0;
  while (jj < nb) {
    const int j = j0 + jj;
    if (wave == 0) {
      // column maximum over the fully-summed rows; candidate partner inside
      // the panel
      double cmax = 0.0, rin = 0.0;
      int r = -1;
      for (int i = j + 1 + lane; i < k; i += 64) {
        const double v = fabs(P(i, j));
        cmax = fmax(cmax, v);
        if (i < pend && v > rin) { rin = v; r = i; }
      }
      cmax = wave_max(cmax);
      wave_argmax(rin, r);
      const double ajj = fabs(P(j, j));
      int kind = 1, sa = -1, sb = -1, end = 0;
      if (cmax == 0.0 || ajj >= BF_ALPHA * cmax) {
        kind = 1;
      } else if (r < 0) {
        if (jj > 0) end = 1;   // the partner lies beyond the panel
      } else {
        double rmax = 0.0;
        for (int i = j + lane; i < k; i += 64) {
          if (i == r) continue;
          rmax = fmax(rmax, i < r ? fabs(P(r, i)) : fabs(P(i, r)));
        }
        rmax = wave_max(rmax);
        const double arr = fabs(P(r, r));
        if (ajj * rmax >= BF_ALPHA * cmax * cmax) {
          kind = 1;
        } else if (arr >= BF_ALPHA * rmax) {
          kind = 1;
          sa = j;
          sb = r;
        } else if (jj + 1 < nb) {
          kind = 2;
          if (r != j + 1) { sa = j + 1; sb = r; }
        } else {
          end = jj > 0;        // no room for a 2x2 block in this panel
        }
      }
      if (lane == 0) {
        dec.kind = kind;
        dec.sa = sa;
        dec.sb = sb;
        dec.end = end;
      }
    } else {
      scale_pending(tid - 64, NT - 64);
    }
    __syncthreads();
    pkind = 0;
    if (dec.end) break;
    const int kind = dec.kind;
    const int p = dec.sa, q = dec.sb;  // p < q < pend
    if (p >= 0) {
      // symmetric interchange of p and q: rows p, q of the earlier panels'
      // L in global memory, the panel's fully-summed rows in LDS (the
      // update-block rows follow from the panel column order lp)
      for (int c = tid; c < j0; c += NT) {
        T* col = A + (int64_t)c * f;
        const T t0 = col[p];
        col[p] = col[q];
        col[q] = t0;
      }
      for (int c = j0 + tid; c < k; c += NT) {
        if (c < p) {
          const double t0 = P(p, c); P(p, c) = P(q, c); P(q, c) = t0;
        } else if (c == p) {
          const double t0 = P(p, p); P(p, p) = P(q, q); P(q, q) = t0;
        } else if (c < q) {
          const double t0 = P(c, p); P(c, p) = P(q, c); P(q, c) = t0;
        } else if (c > q) {
          const double t0 = P(c, p); P(c, p) = P(c, q); P(c, q) = t0;
        }
      }
      if (tid == 0) {
        const int tp = perm[p]; perm[p] = perm[q]; perm[q] = tp;
        const int tl = lp[p - j0]; lp[p - j0] = lp[q - j0]; lp[q - j0] = tl;
      }
      __syncthreads();
    }
    if (kind == 1) {
      // every thread computes the same (possibly perturbed) pivot
      const double a0 = P(j, j);
      const double d = fabs(a0) < a.pivtol ? (a0 < 0.0 ? -a.pivtol : a.pivtol) : a0;
      if (tid == 0) {
        if (d != a0) ++pert;
        if (d < 0.0) ++neg;
        type_out[j] = 1;
      }
      const double dinv = 1.0 / d;
      for (int c = j + 1 + wave; c < pend; c += NW) {
        const double uc = P(c, j) * dinv;
        for (int r = c + lane; r < k; r += 64) P(r, c) -= P(r, j) * uc;
      }
      __syncthreads();
      if (tid == 0) P(j, j) = d;
      pj = j;
      pkind = 1;
      p11 = d;
      jj += 1;
    } else {
      const double d11 = P(j, j), d21 = P(j + 1, j), d22 = P(j + 1, j + 1);
      const double det = d11 * d22 - d21 * d21;
      const double idet = 1.0 / det;
      if (tid == 0) {
        if (det < 0.0) neg += 1;
        else if (d11 < 0.0) neg += 2;
        ++two;
        type_out[j] = 2;
        type_out[j + 1] = 3;
      }
      // A(r, c) -= [a_rj a_rj+1] D^{-1} [a_cj; a_cj+1] with the unscaled columns
      for (int c = j + 2 + wave; c < pend; c += NW) {
        const double u1 = P(c, j), u2 = P(c, j + 1);
        const double w1 = (u1 * d22 - u2 * d21) * idet, w2 = (u2 * d11 - u1 * d21) * idet;
        for (int r = c + lane; r < k; r += 64) P(r, c) -= P(r, j) * w1 + P(r, j + 1) * w2;
      }
      __syncthreads();
      pj = j;
      pkind = 2;
      p11 = d11;
      p21 = d21;
      p22 = d22;
      jj += 2;
    }
  }
  // the last pivot's column(s)
  scale_pending(tid, NT);
  __syncthreads();
  const int kb = jj;
  for (int e = tid; e < nb * m; e += NT) {
    const int c = e / m, r = e % m;
    if (r >= c) A[(int64_t)(j0 + c) * f + j0 + r] = (T)Pn[e];
  }
  if (tid < nb) a.lperm[(int64_t)b * BF_NB + tid] = lp[tid];
  if (tid == 0) {
    st->cur = j0;
    st->kb = kb;
    st->nb = nb;
    st->next = j0 + kb;
    st->neg += neg;
    st->pert += pert;
    st->two += two;
  }
}

// Update-block rows of the panel columns: gather them in the panel's column
// order, eliminate with the panel's pivots (l = y (L_pp D)^{-T} on the kb
// factorised columns, the rank-kb update on the other nb - kb), write back.
// One thread per row with the row's nb panel entries in registers (loads and
// stores coalesced across the rows), W(c, t) = (L_pp D)(c, t) read from LDS
// as a broadcast.
template <class T>
__global__ void __launch_bounds__(256) big_cbrows_kernel(BigArgs a0, T* pool0, BigJobs J) {
  BigArgs a;
  T* pool;
  int b;
  big_pick(a0, pool0, J, blockIdx.y, a, pool, b);
  __shared__ double W[BF_NB * BF_NB];   // W[t * BF_NB + c] = (L_pp D)(j0 + c, j0 + t)
  __shared__ double dA[BF_NB], dB[BF_NB], dinv[BF_NB];
  __shared__ int ty[BF_NB], lp[BF_NB];
  const BigState st = a.st[b];
  if (st.kb == 0) return;
  const int F = a.fronts[b];
  const int f = a.ff[F], k = a.fk[F], start = a.fstart[F];
  const int i0 = k + blockIdx.x * 256;
  if (i0 >= f) return;
  const int j0 = st.cur, kb = st.kb, nb = st.nb;
  T* A = pool + a.pool_off[F];
  const int tid = threadIdx.x;
  if (tid < BF_NB) {
    lp[tid] = tid < nb ? a.lperm[(int64_t)b * BF_NB + tid] : 0;
    int tt = 0;
    double da = 1.0, db = 0.0;
    if (tid < kb) {
      tt = a.piv_type[start + j0 + tid];
      da = (double)A[(int64_t)(j0 + tid) * f + j0 + tid];
      if (tt == 2) db = (double)A[(int64_t)(j0 + tid) * f + j0 + tid + 1];
      else if (tt == 3) db = (double)A[(int64_t)(j0 + tid - 1) * f + j0 + tid];
    }
    ty[tid] = tt;
    dA[tid] = da;
    dB[tid] = db;
  }
  __syncthreads();
  if (tid < BF_NB) {
    // 1 / d for 1x1 pivots, 1 / det for the first pivot of a 2x2 block
    const int tt = ty[tid];
    dinv[tid] = tt == 1 ? 1.0 / dA[tid]
                        : (tt == 2 ? 1.0 / (dA[tid] * dA[tid + 1] - dB[tid] * dB[tid]) : 0.0);
  }
  for (int e = tid; e < BF_NB * BF_NB; e += 256) {
    const int c = e & 63, t = e >> 6;
    double w = 0.0;
    if (t < kb && c < nb && c > t) {
      const T* Lc = A + (int64_t)j0 * f + j0 + c;  // row j0 + c
      const int tt = ty[t];
      if (tt == 1) {
        w = (double)Lc[(int64_t)t * f] * dA[t];
      } else if (tt == 2) {
        const double l1 = (double)Lc[(int64_t)t * f];
        const double l2 = c > t + 1 ? (double)Lc[(int64_t)(t + 1) * f] : 0.0;
        w = l1 * dA[t] + l2 * dB[t];
      } else {
        const double l1 = (double)Lc[(int64_t)(t - 1) * f];
        const double l2 = (double)Lc[(int64_t)t * f];
        w = l1 * dB[t] + l2 * dA[t];
      }
    }
    W[t * BF_NB + c] = w;
  }
  __syncthreads();
  const int i = i0 + tid;
  if (i >= f) return;
  double v[BF_NB];
#pragma unroll
  for (int c = 0; c < BF_NB; ++c) v[c] = c < nb ? (double)A[(int64_t)(j0 + lp[c]) * f + i] : 0.0;
#pragma unroll
  for (int t = 0; t < BF_NB; ++t) {
    const int tt = t < kb ? ty[t] : 0;
    if (tt == 1) {
      const double l = v[t] * dinv[t];
      v[t] = l;
#pragma unroll
      for (int c = t + 1; c < BF_NB; ++c) v[c] -= l * W[t * BF_NB + c];
    } else if (tt == 2) {
      const double d11 = dA[t], d21 = dB[t], d22 = dA[t + 1], idet = dinv[t];
      const double y1 = v[t], y2 = v[t + 1];
      const double l1 = (y1 * d22 - y2 * d21) * idet;
      const double l2 = (y2 * d11 - y1 * d21) * idet;
      v[t] = l1;
      v[t + 1] = l2;
#pragma unroll
      for (int c = t + 2; c < BF_NB; ++c)
        v[c] -= l1 * W[t * BF_NB + c] + l2 * W[(t + 1) * BF_NB + c];
    }
    // tt == 3: second pivot of a 2x2 block, done with the first
  }
#pragma unroll
  for (int c = 0; c < BF_NB; ++c)
    if (c < nb) A[(int64_t)(j0 + c) * f + i] = (T)v[c];
}

// Trailing update of one 64 x 64 lower-triangle tile of [j0 + nb, f)^2:
// A(i, c) -= sum_t L(i, t) W(c, t) over the kb factorised panel columns.
template <class T>
__global__ void __launch_bounds__(256) big_trailing_kernel(BigArgs a0, T* pool0, BigJobs J) {
  BigArgs a;
  T* pool;
  int b;
  big_pick(a0, pool0, J, blockIdx.y, a, pool, b);
  __shared__ double La[BF_NB * (BF_TILE + 1)];  // La[t][ii] = L(r0 + ii, j0 + t)
  __shared__ double Wb[BF_NB * (BF_TILE + 1)];  // Wb[t][cc] = W(c0 + cc, j0 + t); tile result later
  __shared__ double dA[BF_NB], dB[BF_NB];
  __shared__ int ty[BF_NB];
  const BigState st = a.st[b];
  if (st.kb == 0) return;
  const int F = a.fronts[b];
  const int f = a.ff[F], k = a.fk[F], start = a.fstart[F];
  const int j0 = st.cur, kb = st.kb, c0 = st.cur + st.nb;
  if (c0 >= f || c0 >= k) return;
  const int nt = (f - c0 + BF_TILE - 1) / BF_TILE;
  const int ntiles = nt * (nt + 1) / 2;
  T* A = pool + a.pool_off[F];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid < kb) {
    const int t = tid;
    const int tt = a.piv_type[start + j0 + t];
    ty[t] = tt;
    dA[t] = (double)A[(int64_t)(j0 + t) * f + j0 + t];
    if (tt == 2) dB[t] = (double)A[(int64_t)(j0 + t) * f + j0 + t + 1];
    else if (tt == 3) dB[t] = (double)A[(int64_t)(j0 + t - 1) * f + j0 + t];
    else dB[t] = 0.0;
  }
  __syncthreads();
  const int kpad = (kb + 3) & ~3;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    int bi = (int)((sqrt(8.0 * tile + 1.0) - 1.0) * 0.5);
    while ((bi + 1) * (bi + 2) / 2 <= tile) ++bi;
    while (bi * (bi + 1) / 2 > tile) --bi;
    const int bj = tile - bi * (bi + 1) / 2;
    const int r0 = c0 + bi * BF_TILE, cb0 = c0 + bj * BF_TILE;
    // the update block's own columns wait for big_cbupdate_kernel
    if (cb0 >= k) continue;
    // stage L rows of the tile and W of its columns (zero beyond kb / f)
    for (int e = tid; e < BF_NB * BF_TILE; e += 256) {
      const int ii = e & 63, t = e >> 6;
      double lv = 0.0, wv = 0.0;
      if (t < kb) {
        const int i = r0 + ii, c = cb0 + ii;
        if (i < f) lv = (double)A[(int64_t)(j0 + t) * f + i];
        if (c < f) {
          const int tt = ty[t];
          if (tt == 1) {
            wv = (double)A[(int64_t)(j0 + t) * f + c] * dA[t];
          } else if (tt == 2) {
            wv = (double)A[(int64_t)(j0 + t) * f + c] * dA[t] +
                 (double)A[(int64_t)(j0 + t + 1) * f + c] * dB[t];
          } else {
            wv = (double)A[(int64_t)(j0 + t - 1) * f + c] * dB[t] +
                 (double)A[(int64_t)(j0 + t) * f + c] * dA[t];
          }
        }
      }
      La[t * (BF_TILE + 1) + ii] = lv;
      Wb[t * (BF_TILE + 1) + ii] = wv;
    }
    __syncthreads();
    // wave w: column block w (16 columns), all four row blocks, on the
    // matrix cores in the factor's precision (FP64, or FP32 for the mixed
    // precision fronts)
    Tile16<T> acc[4];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) acc[rt].zero();
    for (int t0 = 0; t0 < kpad; t0 += 4) {
      const int kr = t0 + (lane >> 4);
      const double bv = Wb[kr * (BF_TILE + 1) + wave * 16 + (lane & 15)];
#pragma unroll
      for (int rt = 0; rt < 4; ++rt) {
        const double av = La[kr * (BF_TILE + 1) + rt * 16 + (lane & 15)];
        acc[rt].step(av, bv);
      }
    }
    __syncthreads();
    // tile product to LDS (reusing Wb as Ct[ii][cc]), then a coalesced
    // read-modify-write of the lower triangle
    double* Ct = Wb;
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int ii = rt * 16 + Tile16<T>::row(lane, r);
        Ct[ii * (BF_TILE + 1) + wave * 16 + (lane & 15)] = acc[rt].get(r);
      }
    __syncthreads();
    for (int e = tid; e < BF_TILE * BF_TILE; e += 256) {
      const int ii = e & 63, cc = e >> 6;
      const int i = r0 + ii, c = cb0 + cc;
      if (i < f && c < k && i >= c) {
        T* ap = A + (int64_t)c * f + i;
        *ap = (T)((double)*ap - Ct[ii * (BF_TILE + 1) + cc]);
      }
    }
    __syncthreads();
  }
}

// W21 = L21 D of every big front of the level (1x1 and 2x2 blocks of D),
// stored transposed in the front's unused upper-right block: W(c, t) at
// A[c f + t] for t < k <= c (column-major, so row t of column c lies above
// the diagonal).  64 x 64 tiles through LDS: L read down its columns, W
// written down the block's columns.
template <class T>
__global__ void __launch_bounds__(256) big_w21_kernel(BigArgs a0, T* pool0, BigJobs J) {
  BigArgs a;
  T* pool;
  int b;
  big_pick(a0, pool0, J, blockIdx.y, a, pool, b);
  __shared__ double Wt[64][65];
  __shared__ double dA[64], dB[64];
  __shared__ int ty[64];
  const int F = a.fronts[b];
  const int f = a.ff[F], k = a.fk[F], start = a.fstart[F];
  if (k >= f) return;
  const int nr = (f - k + 63) / 64, nc = (k + 63) / 64;
  T* A = pool + a.pool_off[F];
  const int tid = threadIdx.x;
  for (int tile = blockIdx.x; tile < nr * nc; tile += gridDim.x) {
    const int c0 = k + (tile / nc) * 64, t0 = (tile % nc) * 64;
    __syncthreads();  // the previous tile's LDS reads are done
    if (tid < 64) {
      const int g = t0 + tid;
      int tt = 1;
      double d = 0.0, e = 0.0;
      if (g < k) {
        tt = a.piv_type[start + g];
        d = (double)A[(int64_t)g * f + g];
        if (tt == 2) e = (double)A[(int64_t)g * f + g + 1];
        else if (tt == 3) e = (double)A[(int64_t)(g - 1) * f + g];
      }
      ty[tid] = tt;
      dA[tid] = d;
      dB[tid] = e;
    }
    __syncthreads();
    // lanes over c: L(c, g) and its 2x2 partner column, coalesced
    for (int e = tid; e < 64 * 64; e += 256) {
      const int cc = e & 63, t = e >> 6;
      const int c = c0 + cc, g = t0 + t;
      double w = 0.0;
      if (c < f && g < k) {
        const double l = (double)A[(int64_t)g * f + c];
        if (ty[t] == 1) w = l * dA[t];
        else if (ty[t] == 2) w = l * dA[t] + (double)A[(int64_t)(g + 1) * f + c] * dB[t];
        else w = (double)A[(int64_t)(g - 1) * f + c] * dB[t] + l * dA[t];
      }
      Wt[cc][t] = w;
    }
    __syncthreads();
    // lanes over t: W(c, g) at A[c f + g]
    for (int e = tid; e < 64 * 64; e += 256) {
      const int t = e & 63, cc = e >> 6;
      const int c = c0 + cc, g = t0 + t;
      if (c < f && g < k) A[(int64_t)c * f + g] = (T)Wt[cc][t];
    }
  }
}

// The update block C = A[k:f, k:f] (lower triangle) receives C -= L21 W21^T,
// W21 = L21 D, over all k fully-summed columns at once after the level's
// last panel step (the panels' trailing updates stop at column k): C is read
// and written once per front instead of once per panel.  A GEMM on the
// matrix cores: 128 x 128 tiles of C (lower-triangle tiles only), a grid of
// waves over each tile (below), the inner dimension in chunks of 16
// columns staged through LDS in two buffers, the next chunk's global loads
// in flight while the current one is multiplied.  The transposed product
// C^T = W L^T is formed, so that a lane's MFMA output column is a row of C:
// sixteen lanes write sixteen consecutive doubles of a column of the
// column-major front.  W21 is read from the front's upper-right block,
// where big_w21_kernel has stored it transposed.
constexpr int CB_T = 128;
constexpr int CB_K = 16;
constexpr int CB_LD = CB_T + 4;
constexpr size_t CB_LDS = 2 * 2 * CB_K * CB_LD * sizeof(double);
// the wave grid of a tile: WR waves down by WC across, each with RT x CT MFMA
// tiles of 16 x 16; FP64 takes sixteen waves of 32 x 32 (few accumulators per
// lane, four waves per SIMD in one workgroup), FP32 eight of 32 x 64 (two
// workgroups per compute unit)
template <class T>
struct CbShape {
  static constexpr int WR = 4, WC = sizeof(T) == 8 ? 4 : 2;
  static constexpr int NT = 64 * WR * WC;          // threads
  static constexpr int RT = CB_T / WR / 16, CT = CB_T / WC / 16;
  static constexpr int SP = NT / CB_T;             // threads per staged row or column
  static constexpr int QS = CB_K * CB_T / NT;      // staged entries of each operand per thread
};

template <class T>
__global__ void __launch_bounds__(CbShape<T>::NT) big_cbupdate_kernel(BigArgs a0, T* pool0, BigJobs J) {
  BigArgs a;
  T* pool;
  int b;
  big_pick(a0, pool0, J, blockIdx.y, a, pool, b);
  extern __shared__ double cbs[];
  // As[buf][t][row] = L(r0 + row, j0 + t), Bs[buf][t][col] = W(c0 + col, j0 + t)
  auto As = [&](int buf, int t, int r) -> double& { return cbs[((buf * 2 + 0) * CB_K + t) * CB_LD + r]; };
  auto Bs = [&](int buf, int t, int r) -> double& { return cbs[((buf * 2 + 1) * CB_K + t) * CB_LD + r]; };
  const int F = a.fronts[b];
  const int f = a.ff[F], k = a.fk[F], start = a.fstart[F];
  if (k >= f) return;
  const int nt = (f - k + CB_T - 1) / CB_T;
  const int ntiles = nt * (nt + 1) / 2;
  const T* A = pool + a.pool_off[F];
  T* Aw = pool + a.pool_off[F];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  using S = CbShape<T>;
  constexpr int QS = S::QS, SP = S::SP, RT = S::RT, CT = S::CT;
  const int wr = wave / S::WC, wc = wave % S::WC;
  const int srow = tid % CB_T, st0 = tid / CB_T;         // staging of L: row, first t
  const int wcol = tid / SP, wt0 = (tid % SP) * QS;      // staging of W: column, first t
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    int bi = (int)((sqrt(8.0 * tile + 1.0) - 1.0) * 0.5);
    while ((bi + 1) * (bi + 2) / 2 <= tile) ++bi;
    while (bi * (bi + 1) / 2 > tile) --bi;
    const int bj = tile - bi * (bi + 1) / 2;
    const int r0 = k + bi * CB_T, c0 = k + bj * CB_T;
    const int i = r0 + srow, c = c0 + wcol;
    T la[QS], wb[QS];
    // chunk j0: L(i, j0 + st0 + SP q) down a column of L21, W(c, j0 + wt0 + q)
    // down a column of the stored W21^T (plain loads: nothing waits on them
    // before the chunk's multiplications)
    auto load = [&](int j0) {
#pragma unroll
      for (int q = 0; q < QS; ++q) {
        const int g = j0 + st0 + SP * q;
        la[q] = (g < k && i < f) ? A[(int64_t)g * f + i] : (T)0;
        const int h = j0 + wt0 + q;
        wb[q] = (h < k && c < f) ? A[(int64_t)c * f + h] : (T)0;
      }
    };
    auto store = [&](int buf) {
#pragma unroll
      for (int q = 0; q < QS; ++q) {
        As(buf, st0 + SP * q, srow) = (double)la[q];
        Bs(buf, wt0 + q, wcol) = (double)wb[q];
      }
    };
    Tile16<T> acc[CT][RT];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) acc[ct][rt].zero();
    __syncthreads();  // the previous tile's LDS reads are done
    load(0);
    store(0);
    __syncthreads();
    int buf = 0;
    for (int j0 = 0; j0 < k; j0 += CB_K) {
      const bool more = j0 + CB_K < k;
      if (more) load(j0 + CB_K);
#pragma unroll
      for (int t0 = 0; t0 < CB_K; t0 += 4) {
        const int kr = t0 + (lane >> 4);
        double av[RT], bv[CT];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) av[rt] = As(buf, kr, (wr * RT + rt) * 16 + (lane & 15));
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) bv[ct] = Bs(buf, kr, (wc * CT + ct) * 16 + (lane & 15));
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
#pragma unroll
          for (int rt = 0; rt < RT; ++rt) acc[ct][rt].step(bv[ct], av[rt]);
      }
      if (more) store(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
    // acc[ct][rt] holds (W L^T)(c, i): c = c0 + (wc CT + ct) 16 + row(lane, q),
    // i = r0 + (wr RT + rt) 16 + (lane & 15)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int cc = c0 + (wc * CT + ct) * 16 + Tile16<T>::row(lane, q);
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
          const int ii = r0 + (wr * RT + rt) * 16 + (lane & 15);
          if (ii < f && cc < f && ii >= cc) {
            T* ap = Aw + (int64_t)cc * f + ii;
            *ap = (T)((double)*ap - acc[ct][rt].get(q));
          }
        }
      }
  }
}

__global__ void big_init_kernel(BigArgs a0, int nbig, BigJobs J) {
  BigArgs a;
  double* pool;
  int b;
  big_pick<double>(a0, nullptr, J, blockIdx.x, a, pool, b);
  if (b >= (J.jobs ? a.nbig : nbig)) return;
  const int k = a.fk[a.fronts[b]];
  int* perm = a.perm + (int64_t)b * a.perm_stride;
  for (int t = threadIdx.x; t < k; t += blockDim.x) perm[t] = t;
  if (threadIdx.x == 0) a.st[b] = BigState{0, 0, 0, 0, 0, 0, 0, 0};
}

// (with jobs: one workgroup per job, each writing its job's count)
__global__ void big_pending_kernel(BigArgs a0, int nbig, int* pending, BigJobs J) {
  BigArgs a = a0;
  if (J.jobs) {
    a = J.jobs[blockIdx.x];
    nbig = a.nbig;
    pending = a.pend;
  }
  int c = 0;
  for (int b = threadIdx.x; b < nbig; b += blockDim.x)
    if (a.st[b].next < a.fk[a.fronts[b]]) ++c;
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
  __shared__ int part[4];
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) *pending = part[0] + part[1] + part[2] + part[3];
}

__global__ void big_finish_kernel(BigArgs a0, int nbig, BigJobs J) {
  BigArgs a;
  double* pool;
  int b;
  big_pick<double>(a0, nullptr, J, blockIdx.x, a, pool, b);
  if (b >= (J.jobs ? a.nbig : nbig)) return;
  const int F = a.fronts[b];
  const int k = a.fk[F], start = a.fstart[F];
  const int* perm = a.perm + (int64_t)b * a.perm_stride;
  for (int t = threadIdx.x; t < k; t += blockDim.x) a.piv_perm[start + t] = perm[t];
  if (threadIdx.x == 0) {
    a.stat[4 * F + 0] = a.st[b].neg;
    a.stat[4 * F + 1] = a.st[b].pert;
    a.stat[4 * F + 2] = a.st[b].two;
  }
}

}  // namespace

void set_bigfront_attributes() {
  HIPCHECK(hipFuncSetAttribute((const void*)big_panel_kernel<double>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, BF_LDS * (int)sizeof(double)));
  HIPCHECK(hipFuncSetAttribute((const void*)big_panel_kernel<float>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, BF_LDS * (int)sizeof(double)));
  HIPCHECK(hipFuncSetAttribute((const void*)big_cbupdate_kernel<double>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)CB_LDS));
  HIPCHECK(hipFuncSetAttribute((const void*)big_cbupdate_kernel<float>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)CB_LDS));
}

int bigfront_max_k() { return BF_LDS; }

namespace {

// The arguments of one problem's blocked fronts at one height.
BigArgs big_args(riga_problem* pr, Factor& F, void* pool, const int32_t* fronts, const BigPlan& P,
                 double pivtol, int level) {
  if (P.maxk > bigfront_max_k())
    throw Error(RIGA_EUNSUPPORTED, "fully-summed block too large for the panel kernel");
  // scratch reserved before the factorisation for the largest level: it is
  // never reallocated while kernels of an earlier level may still use it
  const int64_t stride = P.maxk + 1;
  const size_t need_perm = (size_t)P.nbig * stride, need_lp = (size_t)P.nbig * BF_NB;
  const size_t need_st = (size_t)P.nbig * sizeof(BigState) / sizeof(int32_t) + 1;
  if (F.big_perm.n < need_perm || F.big_lperm.n < need_lp || F.big_state.n < need_st)
    throw Error(RIGA_EINVAL, "blocked-factorisation scratch not reserved");
  if (F.big_pend.n < pr->levels.size()) throw Error(RIGA_EINVAL, "pending counts not reserved");
  BigArgs a{};
  a.fronts = fronts;
  a.ff = pr->d_ff.p;
  a.fk = pr->d_fk.p;
  a.fstart = pr->d_fstart.p;
  a.pool_off = pr->d_pool_off.p;
  a.piv_perm = F.piv_perm.p;
  a.piv_type = F.piv_type.p;
  a.stat = F.front_stat.p;
  a.perm = F.big_perm.p;
  a.perm_stride = stride;
  a.lperm = F.big_lperm.p;
  a.st = reinterpret_cast<BigState*>(F.big_state.p);
  a.pivtol = pivtol;
  a.pool = pool;
  a.pend = F.big_pend.p + level;
  a.nbig = P.nbig;
  return a;
}

// `n` rounds of panel, update-block rows and trailing update over the
// P.nbig fronts of the grid.
template <class T>
void big_rounds(const BigArgs& a, T* pool, const BigJobs& J, const BigPlan& P, int n, hipStream_t s) {
  const int nb = P.nbig;
  const unsigned cb_blocks = (unsigned)std::max(1, (P.maxcb + 255) / 256);
  const unsigned tpf = (unsigned)std::max(1, std::min(P.max_tiles, std::max(1, 2048 / nb)));
  for (int it = 0; it < n; ++it) {
    big_panel_kernel<T><<<nb, 1024, BF_LDS * sizeof(double), s>>>(a, pool, J);
    if (P.maxcb > 0) big_cbrows_kernel<T><<<dim3(cb_blocks, nb), 256, 0, s>>>(a, pool, J);
    big_trailing_kernel<T><<<dim3(tpf, nb), 256, 0, s>>>(a, pool, J);
  }
  HIPCHECK(hipGetLastError());
}

// the update blocks, once every panel of the level is done
template <class T>
void big_cb_update(const BigArgs& a, T* pool, const BigJobs& J, const BigPlan& P, hipStream_t s) {
  if (P.maxcb == 0) return;
  const int nb = P.nbig;
  const unsigned cpf = (unsigned)std::max(1, std::min(P.max_cb_tiles, std::max(1, 4096 / nb)));
  const unsigned wpf = (unsigned)std::max(1, std::min(((P.maxcb + 63) / 64) * ((P.maxk + 63) / 64),
                                                      std::max(1, 2048 / nb)));
  big_w21_kernel<T><<<dim3(wpf, nb), 256, 0, s>>>(a, pool, J);
  big_cbupdate_kernel<T><<<dim3(cpf, nb), CbShape<T>::NT, CB_LDS, s>>>(a, pool, J);
  HIPCHECK(hipGetLastError());
}

// The predicted panel steps plus one (covering a panel that ended early at
// a 2x2 pivot on its edge; the steps of finished fronts return at once),
// the update blocks, the count of unfinished fronts into each problem's
// pending counter and the pivot orders.  A front left unfinished gets an
// incomplete update block and is counted: the caller then repeats the
// factorisation in checked mode.
template <class T>
void big_unchecked(const BigArgs& a, T* pool, const BigJobs& J, const BigPlan& P, hipStream_t s) {
  const int nb = P.nbig;
  big_init_kernel<<<nb, 256, 0, s>>>(a, nb, J);
  HIPCHECK(hipGetLastError());
  big_rounds<T>(a, pool, J, P, P.steps + 1, s);
  big_cb_update<T>(a, pool, J, P, s);
  if (J.jobs) big_pending_kernel<<<J.njobs, 256, 0, s>>>(a, nb, nullptr, J);
  else big_pending_kernel<<<1, 256, 0, s>>>(a, nb, a.pend, J);
  big_finish_kernel<<<nb, 256, 0, s>>>(a, nb, J);
  HIPCHECK(hipGetLastError());
}

}  // namespace

BigPlan big_plan(const std::vector<int>& big_f, const std::vector<int>& big_k) {
  BigPlan P;
  P.nbig = (int)big_f.size();
  for (int i = 0; i < P.nbig; ++i) {
    const int f = big_f[i], k = big_k[i];
    P.maxk = std::max(P.maxk, k);
    P.maxcb = std::max(P.maxcb, f - k);
    int j0 = 0, n = 0;
    while (j0 < k) {
      j0 += panel_width(k - j0);
      ++n;
    }
    P.steps = std::max(P.steps, n);
    const int nb0 = panel_width(k);
    const int nt = (f - nb0 + BF_TILE - 1) / BF_TILE;
    P.max_tiles = std::max(P.max_tiles, nt * (nt + 1) / 2);
    const int ntc = (f - k + CB_T - 1) / CB_T;
    P.max_cb_tiles = std::max(P.max_cb_tiles, ntc * (ntc + 1) / 2);
  }
  return P;
}

size_t big_args_bytes() { return sizeof(BigArgs); }

void big_args_fill(riga_problem* pr, Factor& F, void* pool, const int32_t* fronts, const BigPlan& P,
                   double pivtol, int level, void* out) {
  const BigArgs a = big_args(pr, F, pool, fronts, P, pivtol, level);
  std::memcpy(out, &a, sizeof(a));
}

template <class T>
void factor_big_fronts_batched(const void* jobs, const int32_t* ystart, int njobs, const BigPlan& P,
                               hipStream_t s) {
  if (njobs == 0 || P.nbig == 0) return;
  const BigJobs J{static_cast<const BigArgs*>(jobs), ystart, njobs};
  big_unchecked<T>(BigArgs{}, nullptr, J, P, s);
}

template <class T>
void factor_big_fronts(riga_problem* pr, Factor& F, T* pool, const int32_t* fronts,
                       const std::vector<int>& big_f, const std::vector<int>& big_k,
                       double pivtol, int level, bool checked, hipStream_t s) {
  const BigPlan P = big_plan(big_f, big_k);
  if (P.nbig == 0) return;
  const BigArgs a = big_args(pr, F, pool, fronts, P, pivtol, level);
  if (!checked) {
    big_unchecked<T>(a, pool, BigJobs{}, P, s);
    return;
  }
  const int nbig = P.nbig;
  int32_t* pending = F.big_state.p + (F.big_state.n - 1);
  big_init_kernel<<<nbig, 256, 0, s>>>(a, nbig, BigJobs{});
  HIPCHECK(hipGetLastError());
  big_rounds<T>(a, pool, BigJobs{}, P, P.steps, s);
  // panels that ended early leave columns for further steps
  for (int guard = 0;; ++guard) {
    big_pending_kernel<<<1, 256, 0, s>>>(a, nbig, pending, BigJobs{});
    HIPCHECK(hipGetLastError());
    int left = 0;
    HIPCHECK(hipMemcpyAsync(&left, pending, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    if (left == 0) break;
    if (guard > P.maxk) throw Error(RIGA_EDEVICE, "blocked factorisation made no progress");
    big_rounds<T>(a, pool, BigJobs{}, P, 4, s);
  }
  big_cb_update<T>(a, pool, BigJobs{}, P, s);
  big_finish_kernel<<<nbig, 256, 0, s>>>(a, nbig, BigJobs{});
  HIPCHECK(hipGetLastError());
}

void bigfront_reserve(riga_problem* pr, Factor& F, int lds_max_f, hipStream_t s) {
  size_t need_perm = 0, need_lp = 0, need_st = 0;
  for (const LevelDev& L : pr->levels) {
    const int ns = L.n_upto(lds_max_f);
    const int nbig = L.n - ns;
    if (nbig <= 0) continue;
    int maxk = 0;
    for (int i = ns; i < L.n; ++i) maxk = std::max(maxk, L.host_k[i]);
    need_perm = std::max(need_perm, (size_t)nbig * (size_t)(maxk + 1));
    need_lp = std::max(need_lp, (size_t)nbig * BF_NB);
    need_st = std::max(need_st, (size_t)nbig * sizeof(BigState) / sizeof(int32_t) + 1);
  }
  if (F.big_pend.n < pr->levels.size()) F.big_pend.alloc(pr->levels.size(), s);
  if (need_perm == 0) return;
  // the pending counter takes the last slot of big_state, past every level's states
  if (F.big_perm.n < need_perm) F.big_perm.alloc(need_perm, s);
  if (F.big_lperm.n < need_lp) F.big_lperm.alloc(need_lp, s);
  if (F.big_state.n < need_st) F.big_state.alloc(need_st, s);
}

template void factor_big_fronts<double>(riga_problem*, Factor&, double*, const int32_t*,
                                        const std::vector<int>&, const std::vector<int>&, double,
                                        int, bool, hipStream_t);
template void factor_big_fronts<float>(riga_problem*, Factor&, float*, const int32_t*,
                                       const std::vector<int>&, const std::vector<int>&, double,
                                       int, bool, hipStream_t);
template void factor_big_fronts_batched<double>(const void*, const int32_t*, int, const BigPlan&, hipStream_t);
template void factor_big_fronts_batched<float>(const void*, const int32_t*, int, const BigPlan&, hipStream_t);

}  // namespace riga
