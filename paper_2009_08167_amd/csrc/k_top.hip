// Explicit inverse of the top of the separator tree, for the forward and
// backward eliminations of the Lanczos steps (the f/b eliminations of
// Sec. 5.1 of arXiv 2009.08167).
//
// Near the root the tree has few fronts per level and little data per front,
// so sweeping it level by level costs one kernel launch per level and
// direction, each bound by latency rather than bandwidth.  Instead, the
// fronts at heights >= cut form the top block T, and every factorisation
// also stores L_TT^{-1} (unit lower triangular, T's variables in pivot
// order).  With the update vectors of the fronts below T assembled into
//     r_T = b_T + (the extend-add of every lower front's update entries that
//           lands on a variable of T)
// the top part of a sweep is three launches:
//     forward   w_T = D_TT^{-1} L_TT^{-1} r_T       (rows of D_TT^{-1} L_TT^{-1})
//     backward  x_T = L_TT^{-T} w_T                 (columns of L_TT^{-1})
// after which the lower levels continue as before, reading x_T through
// their update rows.  This extends the per-front partitioned inverse
// H = [I; L21] L11^{-1} over several tree levels (a partitioned inverse of
// the top block).  Row j of L_TT^{-1} is non-zero only in the columns of the
// top variables of the subtree of j's front (a contiguous range in a
// postorder); column j only in the rows of j's front and its ancestors.
//
// Construction (once per factorisation): the block column of top front F
// is the forward sweep of the identity on F's variables, carried up F's
// ancestor chain.  At ancestor P the incoming block (rows of P's front) is
// R = extend-add of the block that P's child on the way passed up (the
// identity on P's own variables when P = F), and
//     X_P  = L11^{-1}(P) R_FS         -> rows of P in L_TT^{-1}(:, F)
//     R_CB = R_CB - (L21 L11^{-1})(P) R_FS   -> passed to P's parent
// with P's partitioned inverse.  Every (P, F) pair of one height is one
// launch of 64 x 64 output tiles on the FP64 matrix units; a last launch
// folds D_TT^{-1} (1x1 and 2x2 blocks) into the row copy.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <map>

#include "mfma_tile.h"
#include "problem.h"
#include "wave_reduce.h"

namespace riga {
namespace {

// Cost model for the choice of the cut (sweep pair, seconds): a tree level
// costs one launch per direction, a fixed latency plus its factor bytes at
// the rate its kernels reach; the top block costs three launches and one
// pass over each of its two copies. Fitted to measured sweep pairs over
// forced cuts of the 2D and 3D workloads.
constexpr double LEVEL_LATENCY = 5.0e-6;
constexpr double LEVEL_BW = 2.0e12;
constexpr double TOP_LATENCY = 5.0e-6;
constexpr double TOP_BW = 2.75e12;
constexpr int64_t TOP_MAX_ENTRIES = int64_t(1) << 27;  // rows + columns + construction blocks
constexpr int TOP_MAX_STACK = 16384;  // stacked rows of a column block (backward kernel's LDS)
constexpr int TOP_MAX_ANC = 64;       // fronts in one ancestor chain

constexpr int TB = 64;        // construction tile
constexpr int TLD = TB + 1;   // padded LDS leading dimension

struct Sizes {
  int64_t e_row = 0, e_col = 0, e_cb = 0;
  int max_h = 0, max_depth = 0;
  int nT = 0;
};

// Sizes of the two copies and the construction blocks for a cut.
Sizes top_sizes(const Analysis& an, int cut) {
  Sizes z;
  const int nf = an.n_fronts;
  std::vector<int> tstart(nf, -1), sub_lo(nf, -1);
  for (int F = 0; F < nf; ++F)
    if (an.f_height[F] >= cut) {
      tstart[F] = z.nT;
      sub_lo[F] = z.nT;
      z.nT += an.f_k[F];
    }
  for (int F = 0; F < nf; ++F)
    if (tstart[F] >= 0 && an.f_parent[F] >= 0)
      sub_lo[an.f_parent[F]] = std::min(sub_lo[an.f_parent[F]], sub_lo[F]);
  for (int F = 0; F < nf; ++F) {
    if (tstart[F] < 0) continue;
    for (int t = 0; t < an.f_k[F]; ++t) z.e_row += ((int64_t)(tstart[F] + t - sub_lo[F] + 1) + 15) & ~int64_t(15);
    int h = 0, depth = 0;
    for (int A = F; A >= 0; A = an.f_parent[A]) {
      h += an.f_k[A];
      ++depth;
      if (an.f_parent[A] >= 0) z.e_cb += (int64_t)(an.f_f[A] - an.f_k[A]) * an.f_k[F];
    }
    z.max_h = std::max(z.max_h, h);
    z.max_depth = std::max(z.max_depth, depth);
    z.e_col += (int64_t)((h + 31) & ~31) * an.f_k[F];
  }
  return z;
}

// a top block from height c up stays within the size limits
bool cut_fits(const Analysis& an, int c) {
  if (c < 1 || c >= an.height) return false;
  const Sizes z = top_sizes(an, c);
  return z.e_row + z.e_col + z.e_cb <= TOP_MAX_ENTRIES && z.max_h <= TOP_MAX_STACK &&
         z.max_depth <= TOP_MAX_ANC;
}

// The cut: `forced` (a measured choice: -1 none, c >= 1 that height), else
// RIGA_TOP_CUT, else the cost model below.
int choose_cut(const Analysis& an, int forced) {
  const int H = an.height;
  if (H < 2) return -1;
  if (forced != TOP_CUT_MODEL) return cut_fits(an, forced) ? forced : -1;
  if (const char* env = std::getenv("RIGA_TOP_CUT")) {
    if (*env) {
      const int c = std::atoi(env);
      return (c >= 1 && c < H) ? c : -1;
    }
  }
  std::vector<double> bytes(H, 0.0);
  for (int F = 0; F < an.n_fronts; ++F) {
    const double f = an.f_f[F], k = an.f_k[F];
    bytes[an.f_height[F]] += (k * (k - 1) / 2 + (f - k) * k) * 8.0;
  }
  auto level = [&](int h) { return 2.0 * (LEVEL_LATENCY + bytes[h] / LEVEL_BW); };
  double all = 0.0;
  for (int h = 0; h < H; ++h) all += level(h);
  double best = 0.95 * all;  // take the top block only for a clear gain
  int cut = -1;
  for (int c = 1; c < H; ++c) {
    if (!cut_fits(an, c)) continue;
    const Sizes z = top_sizes(an, c);
    double t = 3.0 * TOP_LATENCY + (double)(z.e_row + z.e_col) * 8.0 / TOP_BW;
    for (int h = 0; h < c; ++h) t += level(h);
    if (t < best) {
      best = t;
      cut = c;
    }
  }
  return cut;
}

// ---- per factorisation: pivot-order maps ----
__global__ void top_maps_kernel(const int32_t* __restrict__ n_of_j, const int32_t* __restrict__ front_of,
                                const FrontDesc* __restrict__ desc, const int32_t* __restrict__ piv_perm,
                                const int32_t* __restrict__ piv_dof, const int32_t* __restrict__ slist,
                                int nT, int tgs, int32_t* tmap, int32_t* tdof) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= nT) return;
  const int n = n_of_j[j];
  const int slot = j - (n - desc[front_of[n]].start) + piv_perm[n];
  tdof[j] = piv_dof[n];
  for (int s = 0; s < tgs; ++s) tmap[(int64_t)j * tgs + s] = slist[(int64_t)slot * tgs + s];
}

// ---- per factorisation: L_TT^{-1} ----
template <class T>
__global__ void __launch_bounds__(256) top_inverse_kernel(
    const TopTile* __restrict__ tiles, const TopPair* __restrict__ pairs, const T* __restrict__ H,
    const int32_t* __restrict__ piv_perm, const int32_t* __restrict__ piv_type,
    const int32_t* __restrict__ inv, const int64_t* __restrict__ roff, double* cb, T* trow, T* tcol) {
  __shared__ double At[TB * TLD];  // At[u * TLD + r] = A(r0 + r, u0 + u)
  __shared__ double Bt[TB * TLD];  // Bt[u * TLD + c] = R_FS(u0 + u, c0 + c)
  __shared__ int32_t qs[TB], tys[TB];
  const TopTile tl = tiles[blockIdx.x];
  const TopPair p = pairs[tl.pair];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r0 = tl.r0, c0 = tl.c0;
  const int kP = p.kP, fP = p.fP, kF = p.kF;
  const bool self = p.inv_off < 0;  // F = P: R_FS is the identity, R_CB zero
  const T* Hp = H + p.h_off;
  Tile16<T> acc[4];
#pragma unroll
  for (int rt = 0; rt < 4; ++rt) acc[rt].zero();
  // A(r, u): strictly lower L11^{-1} (the 2x2 slots hold D) on the top rows,
  // L21 L11^{-1} below; rows of the top part need u < r only
  const int kmax = (r0 + TB <= kP) ? r0 + TB : kP;
  const int ubeg = self ? c0 : 0;
  const int uend = self ? std::min(kmax, c0 + TB) : kmax;
  for (int u0 = ubeg; u0 < uend; u0 += TB) {
    const int uw = std::min(TB, uend - u0);
    if (tid < TB) {
      int q = -1, ty = 1;
      if (tid < uw) {
        const int n = p.startP + u0 + tid;
        ty = piv_type[n];
        if (!self) q = inv[p.inv_off + piv_perm[n]];
      }
      qs[tid] = q;
      tys[tid] = ty;
    }
    __syncthreads();
    // all 32 loads of this thread's share first, then the LDS stores
    double av[TB * TB / 256], bvv[TB * TB / 256];
#pragma unroll
    for (int q8 = 0; q8 < TB * TB / 256; ++q8) {
      const int e = tid + 256 * q8;
      const int rr = e & 63, uu = e >> 6;
      const int r = r0 + rr, u = u0 + uu;
      double a = 0.0;
      if (uu < uw && r < fP) {
        if (r >= kP || (u < r && !(u == r - 1 && tys[uu] == 2)))
          a = (double)Hp[(int64_t)u * p.ldh + r];
      }
      av[q8] = a;
      const int col = c0 + rr;
      double bv = 0.0;
      if (uu < uw && col < kF) {
        if (self) {
          bv = (u0 + uu == col) ? 1.0 : 0.0;
        } else {
          const int q = qs[uu];
          bv = q >= 0 ? cb[p.cb_in + (int64_t)q * kF + col] : 0.0;
        }
      }
      bvv[q8] = bv;
    }
#pragma unroll
    for (int q8 = 0; q8 < TB * TB / 256; ++q8) {
      const int e = tid + 256 * q8;
      At[(e >> 6) * TLD + (e & 63)] = av[q8];
      Bt[(e >> 6) * TLD + (e & 63)] = bvv[q8];
    }
    __syncthreads();
    const int cl = wave * 16 + (lane & 15);
#pragma unroll 4
    for (int kk = 0; kk < TB; kk += 4) {
      const int kr = kk + (lane >> 4);
      const double bv = Bt[kr * TLD + cl];
#pragma unroll
      for (int rt = 0; rt < 4; ++rt) {
        const double av = At[kr * TLD + rt * 16 + (lane & 15)];
        acc[rt].step(av, bv);
      }
    }
    __syncthreads();
  }
  // lane holds rows Tile16::row(lane, i) of each 16-row tile, column
  // lane & 15 of this wave's 16 columns
  const int col = c0 + wave * 16 + (lane & 15);
  if (col >= kF) return;
#pragma unroll
  for (int rt = 0; rt < 4; ++rt) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = r0 + rt * 16 + Tile16<T>::row(lane, i);
      if (r >= fP) continue;
      if (r < kP) {
        double base;
        if (self) {
          base = r == col ? 1.0 : 0.0;
        } else {
          const int q = inv[p.inv_off + piv_perm[p.startP + r]];
          base = q >= 0 ? cb[p.cb_in + (int64_t)q * kF + col] : 0.0;
        }
        const double out = base + acc[rt].get(i);
        tcol[p.xcol + (int64_t)p.ldF * col + r] = (T)out;
        if (!self || col <= r) trow[roff[p.tstartP + r] + p.colbase + col] = (T)out;
      } else if (p.cb_out >= 0) {
        double base = 0.0;
        if (!self) {
          const int q = inv[p.inv_off + r];
          base = q >= 0 ? cb[p.cb_in + (int64_t)q * kF + col] : 0.0;
        }
        cb[p.cb_out + (int64_t)(r - kP) * kF + col] = base - acc[rt].get(i);
      }
    }
  }
}

// ---- per sweep ----
// r_T: the right-hand side of each top variable plus every lower front's
// update entry on it
__global__ void top_rhs_kernel(const int32_t* __restrict__ tdof, const int32_t* __restrict__ tmap, int nT,
                               int tgs, const double* __restrict__ b, const double* __restrict__ cbvec,
                               double* r) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= nT) return;
  double v = b[tdof[j]];
  // eight map entries, then their update entries, in flight at a time
  for (int s0 = 0; s0 < tgs; s0 += 8) {
    int m[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) m[q] = s0 + q < tgs ? tmap[(int64_t)j * tgs + s0 + q] : -1;
    double c[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) c[q] = m[q] >= 0 ? cbvec[m[q]] : 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) v += c[q];
  }
  r[j] = v;
}

// w_T = D^{-1} L_TT^{-1} r_T by rows: workgroups of 1024 threads, tpr threads per
// row (16, 64, 256 or 1024 by the row's length), each summing every tpr-th
// entry of the row's segment, then a reduction in a fixed order.
constexpr int TOP_FWD_THREADS = 1024;

template <class T>
__global__ void __launch_bounds__(TOP_FWD_THREADS) top_fwd_kernel(const TopRowUnit* __restrict__ units,
                                                                  const int64_t* __restrict__ roff,
                                                                  const int32_t* __restrict__ rlo,
                                                                  const int32_t* __restrict__ rlen,
                                                                  const T* __restrict__ L,
                                                                  const double* __restrict__ r,
                                                                  double* y) {
  __shared__ double red[TOP_FWD_THREADS / 64];
  const TopRowUnit u = units[blockIdx.x];
  const int tid = threadIdx.x, tpr = u.tpr;
  const int row = u.r0 + tid / tpr, ph = tid % tpr;
  double acc = 0.0;
  if (row < u.r1) {
    const int len = rlen[row];
    const T* a = L + roff[row];
    const double* x = r + rlo[row];
    for (int c = ph; c < len; c += 8 * tpr) {
      double av[8], xv[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const bool ok = c + q * tpr < len;
        av[q] = ok ? (double)a[c + q * tpr] : 0.0;
        xv[q] = ok ? x[c + q * tpr] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) acc += av[q] * xv[q];
    }
  }
  const int w = tpr < 64 ? tpr : 64;
  for (int off = w >> 1; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if (tpr > 64) {
    // rows of tpr / 64 waves: wave sums through LDS, in wave order
    if ((tid & 63) == 0) red[tid >> 6] = acc;
    __syncthreads();
    if (ph == 0 && row < u.r1) {
      const int w0 = tid >> 6, nw = tpr >> 6;
      double t = 0.0;
      for (int q = 0; q < nw; ++q) t += red[w0 + q];
      y[row] = t;
    }
  } else if (ph == 0 && row < u.r1) {
    y[row] = acc;
  }
}

// x_T = L_TT^{-T} w_T by columns (w = D^{-1} y from the forward sweep, whose
// rows carry D^{-1}): the workgroup gathers w over the stacked rows of its
// front into LDS, then each wave forms one column's dot product.  The
// column's first loads are issued before the gather.
template <class T>
__global__ void __launch_bounds__(256) top_bwd_kernel(const TopColUnit* __restrict__ units,
                                                      const TopFront* __restrict__ fronts,
                                                      const TopAnc* __restrict__ anc, const T* __restrict__ L,
                                                      const double* __restrict__ w,
                                                      const int32_t* __restrict__ piv_dof, double* x) {
  extern __shared__ double v[];
  __shared__ TopAnc al[TOP_MAX_ANC];
  const TopColUnit u = units[blockIdx.x];
  const TopFront F = fronts[u.tf];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int j = u.c0 + wave;
  const bool col = j < u.c1;
  const T* c = L + F.coff + (int64_t)F.ld * (col ? j : u.c0);
  const int dof = col ? piv_dof[F.start + j] : 0;  // output index, loaded early
  double cv[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) cv[q] = (col && lane + 64 * q < F.h) ? (double)c[lane + 64 * q] : 0.0;
  if (tid < F.n_anc) al[tid] = anc[F.anc_off + tid];
  __syncthreads();
  // eight rows per thread at a time: indices, then all their loads
  int e = 0;
  for (int i0 = tid; i0 < F.h; i0 += 8 * 256) {
    int av[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int i = min(i0 + 256 * q, F.h - 1);
      while (e + 1 < F.n_anc && al[e + 1].rowpos <= i) ++e;
      av[q] = al[e].tstart + (i - al[e].rowpos);
    }
    double wv[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) wv[q] = w[av[q]];
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (i0 + 256 * q < F.h) v[i0 + 256 * q] = wv[q];
  }
  __syncthreads();
  if (!col) return;
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < 8; ++q) s += cv[q] * ((lane + 64 * q < F.h) ? v[lane + 64 * q] : 0.0);
  for (int i = lane + 8 * 64; i < F.h; i += 8 * 64) {
    double cw[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) cw[q] = i + 64 * q < F.h ? (double)c[i + 64 * q] : 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) s += i + 64 * q < F.h ? cw[q] * v[i + 64 * q] : 0.0;
  }
  s = wave_sum(s);
  if (lane == 0) x[dof] = s;
}

// Coefficients of D^{-1} by top row (per factorisation): w_a = c0 y_a +
// c+ y_{a+1} + c- y_{a-1}, non-zero neighbours only inside a 2x2 block.
__global__ void top_dinv_kernel(const int32_t* __restrict__ n_of_j, const int32_t* __restrict__ piv_type,
                                const double* __restrict__ dd, const double* __restrict__ dsub, int nT,
                                double* dc) {
  const int a = blockIdx.x * 256 + threadIdx.x;
  if (a >= nT) return;
  const int n = n_of_j[a];
  const int ty = piv_type[n];
  double c0, cp = 0.0, cm = 0.0;
  if (ty == 1) {
    c0 = 1.0 / dd[n];
  } else if (ty == 2) {
    const double d11 = dd[n], d21 = dsub[n], d22 = dd[n + 1];
    const double det = d11 * d22 - d21 * d21;
    c0 = d22 / det;
    cp = -d21 / det;
  } else {
    const double d11 = dd[n - 1], d21 = dsub[n - 1], d22 = dd[n];
    const double det = d11 * d22 - d21 * d21;
    c0 = d11 / det;
    cm = -d21 / det;
  }
  dc[3 * (int64_t)a] = c0;
  dc[3 * (int64_t)a + 1] = cp;
  dc[3 * (int64_t)a + 2] = cm;
}

// Rows of D^{-1} L_TT^{-1} in place of those of L_TT^{-1} (per
// factorisation, after the construction), so that the forward sweep yields
// w = D^{-1} y directly.  One workgroup per row: a 1x1 pivot's row is
// scaled; the first row a of a 2x2 block combines rows a and a + 1 into both
// (L_TT^{-1} has a zero at (a, a + 1) and (a + 1, a) and a unit diagonal;
// the column a + 1 of row a is its spare slot).  A spare slot not taken is
// cleared.
template <class T>
__global__ void __launch_bounds__(256) top_fold_kernel(const int32_t* __restrict__ n_of_j,
                                                       const int32_t* __restrict__ piv_type,
                                                       const double* __restrict__ dc,
                                                       const int64_t* __restrict__ roff,
                                                       const int32_t* __restrict__ rlo,
                                                       const int32_t* __restrict__ rlen, T* trow) {
  const int j = blockIdx.x;
  const int ty = piv_type[n_of_j[j]];
  const int len = j - rlo[j] + 1;                // entries up to the diagonal
  const bool spare = rlen[j] > len;
  T* a = trow + roff[j];
  if (ty == 3) {  // second row of a 2x2 block: rewritten with the first
    if (spare && threadIdx.x == 0) a[len] = (T)0.0;
    return;
  }
  const double c0 = dc[3 * (int64_t)j];
  if (ty == 1) {
    for (int e = threadIdx.x; e < len; e += 256) a[e] = (T)(c0 * (double)a[e]);
    if (spare && threadIdx.x == 0) a[len] = (T)0.0;
    return;
  }
  // 2x2 block (j, j + 1): w_j = c0 y_j + cp y_{j+1}, w_{j+1} = cm' y_j + c0' y_{j+1}
  const double cp = dc[3 * (int64_t)j + 1];
  const double c0b = dc[3 * (int64_t)(j + 1)], cmb = dc[3 * (int64_t)(j + 1) + 2];
  T* b = trow + roff[j + 1];
  for (int e = threadIdx.x; e <= len; e += 256) {
    const double va = e < len ? (double)a[e] : 0.0;  // L_TT^{-1}(j, j + 1) = 0
    const double vb = (double)b[e];                  // L_TT^{-1}(j + 1, j + 1) = 1
    a[e] = (T)(c0 * va + cp * vb);
    b[e] = (T)(cmb * va + c0b * vb);
  }
}

}  // namespace

std::vector<int> top_cut_candidates(const riga_problem* pr) {
  std::vector<int> c(1, -1);
  for (int h = 1; h < pr->an.height; ++h)
    if (cut_fits(pr->an, h)) c.push_back(h);
  return c;
}

void setup_top(riga_problem* pr, int forced) {
  const Analysis& an = pr->an;
  hipStream_t s = pr->home;
  pr->top = TopDev{};
  TopDev& T = pr->top;
  const int cut = choose_cut(an, forced);
  if (cut < 0) return;
  const int nf = an.n_fronts;
  std::vector<int> tstart(nf, -1), sub_lo(nf, -1), tf_of(nf, -1), Tf;
  int nT = 0;
  for (int F = 0; F < nf; ++F)
    if (an.f_height[F] >= cut) {
      tf_of[F] = (int)Tf.size();
      Tf.push_back(F);
      tstart[F] = sub_lo[F] = nT;
      nT += an.f_k[F];
    }
  if (nT == 0) return;
  for (int F : Tf)
    if (an.f_parent[F] >= 0) sub_lo[an.f_parent[F]] = std::min(sub_lo[an.f_parent[F]], sub_lo[F]);
  // rows
  std::vector<int32_t> n_of_j(nT), rlo(nT), rlen(nT);
  std::vector<int64_t> roff(nT);
  int64_t e_row = 0;
  for (int F : Tf)
    for (int t = 0; t < an.f_k[F]; ++t) {
      const int j = tstart[F] + t;
      n_of_j[j] = an.f_start[F] + t;
      rlo[j] = sub_lo[F];
      // one slot beyond the diagonal when the next pivot is in the same
      // front: the first row of a 2x2 block takes its partner's column
      // once D^{-1} is folded in
      rlen[j] = j - sub_lo[F] + 1 + (t + 1 < an.f_k[F] ? 1 : 0);
      roff[j] = e_row;
      e_row += ((int64_t)rlen[j] + 15) & ~int64_t(15);
    }
  // columns: stacked rows of each top front (itself, then its ancestors)
  std::vector<TopFront> tfr(Tf.size());
  std::vector<TopAnc> anc;
  std::vector<std::map<int, int>> rowpos(Tf.size());
  int64_t e_col = 0;
  int max_h = 0;
  for (size_t i = 0; i < Tf.size(); ++i) {
    const int F = Tf[i];
    TopFront& d = tfr[i];
    d.anc_off = (int)anc.size();
    int h = 0;
    for (int A = F; A >= 0; A = an.f_parent[A]) {
      rowpos[i][A] = h;
      anc.push_back(TopAnc{tstart[A], an.f_start[A], an.f_k[A], h});
      h += an.f_k[A];
    }
    d.n_anc = (int)anc.size() - d.anc_off;
    d.h = h;
    d.ld = (h + 31) & ~31;
    d.k = an.f_k[F];
    d.start = an.f_start[F];
    d.tstart = tstart[F];
    d.coff = e_col;
    e_col += (int64_t)d.ld * d.k;
    max_h = std::max(max_h, h);
    if (d.n_anc > TOP_MAX_ANC) throw Error(RIGA_EUNSUPPORTED, "top block: ancestor chain too long");
  }
  // lower fronts' update entries on top variables, by (front, position)
  std::vector<int> fs_front(an.N, -1), fs_pos(an.N, -1);
  for (int F : Tf)
    for (int i = 0; i < an.f_k[F]; ++i) {
      const int d = an.rows[an.f_rows_off[F] + i];
      fs_front[d] = F;
      fs_pos[d] = i;
    }
  std::vector<std::vector<int32_t>> lists(nT);
  for (int C = 0; C < nf; ++C) {
    const int P = an.f_parent[C];
    if (an.f_height[C] >= cut || P < 0 || an.f_height[P] < cut) continue;
    for (int i = an.f_k[C]; i < an.f_f[C]; ++i) {
      const int d = an.rows[an.f_rows_off[C] + i];
      const int A = fs_front[d];
      if (A < 0) throw Error(RIGA_EINVAL, "top block: update row outside the top block");
      lists[tstart[A] + fs_pos[d]].push_back((int32_t)(an.f_cb_off[C] + i - an.f_k[C]));
    }
  }
  int tgs = 1;
  for (auto& l : lists) tgs = std::max(tgs, (int)l.size());
  std::vector<int32_t> slist((size_t)nT * tgs, -1);
  for (int j = 0; j < nT; ++j)
    for (size_t q = 0; q < lists[j].size(); ++q) slist[(size_t)j * tgs + q] = lists[j][q];
  // forward units: consecutive rows of one width class (up to 12 entries
  // per thread below the widest class)
  std::vector<TopRowUnit> fu;
  for (int j = 0; j < nT;) {
    auto cls = [&](int len) { return len <= 192 ? 16 : (len <= 768 ? 64 : (len <= 3072 ? 256 : 1024)); };
    const int tpr = cls(rlen[j]);
    int j1 = j + 1;
    while (j1 < nT && j1 - j < 1024 / tpr && cls(rlen[j1]) == tpr) ++j1;
    fu.push_back(TopRowUnit{j, j1, tpr, 0});
    j = j1;
  }
  // backward units: four columns (one per wave), tallest column blocks first
  std::vector<int> order(Tf.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return (int64_t)tfr[a].h * tfr[a].k > (int64_t)tfr[b].h * tfr[b].k;
  });
  std::vector<TopColUnit> bu;
  for (int i : order)
    for (int c = 0; c < tfr[i].k; c += 4) bu.push_back(TopColUnit{i, c, std::min(tfr[i].k, c + 4), 0});
  // construction pairs, by height of P
  std::vector<TopPair> pairs;
  std::map<std::pair<int, int>, int64_t> cb_of;  // (P, F) -> block passed to P's parent
  int64_t e_cb = 0;
  const int H = an.height;
  T.tiles.resize(H - cut);
  T.n_tiles.assign(H - cut, 0);
  std::vector<std::vector<TopTile>> tiles(H - cut);
  for (int h = cut; h < H; ++h) {
    for (int P : Tf) {
      if (an.f_height[P] != h) continue;
      const int fP = an.f_f[P], kP = an.f_k[P];
      const bool root = an.f_parent[P] < 0;
      for (int F : Tf) {
        if (tstart[F] < sub_lo[P] || tstart[F] > tstart[P]) continue;  // not in P's subtree
        TopPair q{};
        q.kP = kP;
        q.fP = fP;
        q.startP = an.f_start[P];
        q.tstartP = tstart[P];
        q.kF = an.f_k[F];
        q.ldF = tfr[tf_of[F]].ld;
        q.colbase = tstart[F] - sub_lo[P];
        q.ldh = h_ld(fP);
        q.h_off = an.f_h_off[P];
        q.inv_off = -1;
        q.cb_in = -1;
        if (F != P) {
          int C = F;
          while (an.f_parent[C] != P) C = an.f_parent[C];
          int ci = -1;
          for (int x = an.child_ptr[P]; x < an.child_ptr[P + 1]; ++x)
            if (an.child_list[x] == C) ci = x;
          if (ci < 0) throw Error(RIGA_EINVAL, "top block: child not found");
          q.inv_off = an.inv_off[ci];
          auto it = cb_of.find({C, F});
          if (it == cb_of.end()) throw Error(RIGA_EINVAL, "top block: missing child block");
          q.cb_in = it->second;
        }
        q.cb_out = -1;
        if (!root) {
          q.cb_out = e_cb;
          cb_of[{P, F}] = e_cb;
          e_cb += (int64_t)(fP - kP) * q.kF;
        }
        q.xcol = tfr[tf_of[F]].coff + rowpos[tf_of[F]].at(P);
        const int pi = (int)pairs.size();
        pairs.push_back(q);
        const int rows = root ? kP : fP;
        for (int r0 = 0; r0 < rows; r0 += TB)
          for (int c0 = 0; c0 < q.kF; c0 += TB) tiles[h - cut].push_back(TopTile{pi, r0, c0, 0});
      }
    }
  }
  if (max_h > TOP_MAX_STACK || e_row + e_col + e_cb > TOP_MAX_ENTRIES) return;  // forced cut too low
  T.cut = cut;
  T.nT = nT;
  T.tgs = tgs;
  T.e_row = e_row;
  T.e_col = e_col;
  T.e_cb = e_cb;
  T.max_h = max_h;
  T.n_of_j.upload(n_of_j, s);
  T.slist.upload(slist, s);
  T.roff.upload(roff, s);
  T.rlo.upload(rlo, s);
  T.rlen.upload(rlen, s);
  T.fwd_units.upload(fu, s);
  T.n_fwd = (int)fu.size();
  T.bwd_units.upload(bu, s);
  T.n_bwd = (int)bu.size();
  T.fronts.upload(tfr, s);
  T.anc.upload(anc, s);
  T.pairs.upload(pairs, s);
  for (int l = 0; l < H - cut; ++l) {
    T.tiles[l].upload(tiles[l], s);
    T.n_tiles[l] = (int)tiles[l].size();
  }
  if (const char* v = std::getenv("RIGA_LOG"))
    if (*v && *v != '0')
      std::fprintf(stderr, "[riga] top block: heights >= %d, %d variables, %zu fronts, %.1f MB by rows, "
                   "%.1f MB by columns (FP64)\n", cut, nT, Tf.size(), e_row * 8e-6, e_col * 8e-6);
}

void top_reserve(riga_problem* pr, Factor& F, int precision, hipStream_t s) {
  const TopDev& T = pr->top;
  if (T.cut < 0) return;
  if (precision == RIGA_MIXED) {
    if (F.trow32.n < (size_t)T.e_row) F.trow32.alloc(T.e_row, s);
    if (F.tcol32.n < (size_t)T.e_col) F.tcol32.alloc(T.e_col, s);
  } else {
    if (F.trow64.n < (size_t)T.e_row) F.trow64.alloc(T.e_row, s);
    if (F.tcol64.n < (size_t)T.e_col) F.tcol64.alloc(T.e_col, s);
  }
  if (F.tmap.n < (size_t)T.nT * T.tgs) F.tmap.alloc((size_t)T.nT * T.tgs, s);
  if (F.tdof.n < (size_t)T.nT) F.tdof.alloc(T.nT, s);
  if (F.tdc.n < (size_t)T.nT * 3) F.tdc.alloc((size_t)T.nT * 3, s);
  if (F.tcb.n < (size_t)std::max<int64_t>(T.e_cb, 1)) F.tcb.alloc(std::max<int64_t>(T.e_cb, 1), s);
  if (F.top_r.n < (size_t)T.nT) {
    F.top_r.alloc(T.nT, s);
    F.top_y.alloc(T.nT, s);
  }
}

template <class T>
void build_top(riga_problem* pr, Factor& F, const T* h, T* trow, T* tcol, hipStream_t s) {
  const TopDev& TD = pr->top;
  if (TD.cut < 0) return;
  if (!trow || !tcol || F.tmap.n < (size_t)TD.nT * TD.tgs || F.tdof.n < (size_t)TD.nT ||
      F.tdc.n < (size_t)TD.nT * 3)
    throw Error(RIGA_EINVAL, "top block buffers not reserved");
  top_dinv_kernel<<<(TD.nT + 255) / 256, 256, 0, s>>>(TD.n_of_j.p, F.piv_type.p, F.d_diag.p, F.d_sub.p,
                                                      TD.nT, F.tdc.p);
  top_maps_kernel<<<(TD.nT + 255) / 256, 256, 0, s>>>(TD.n_of_j.p, pr->d_front_of.p, pr->d_desc.p,
                                                      F.piv_perm.p, F.piv_dof.p, TD.slist.p, TD.nT,
                                                      TD.tgs, F.tmap.p, F.tdof.p);
  HIPCHECK(hipGetLastError());
  for (size_t l = 0; l < TD.tiles.size(); ++l) {
    if (TD.n_tiles[l] == 0) continue;
    top_inverse_kernel<T><<<TD.n_tiles[l], 256, 0, s>>>(TD.tiles[l].p, TD.pairs.p, h, F.piv_perm.p,
                                                        F.piv_type.p, pr->d_inv.p, TD.roff.p,
                                                        F.tcb.p, trow, tcol);
    HIPCHECK(hipGetLastError());
  }
  top_fold_kernel<T><<<TD.nT, 256, 0, s>>>(TD.n_of_j.p, F.piv_type.p, F.tdc.p, TD.roff.p, TD.rlo.p,
                                           TD.rlen.p, trow);
  HIPCHECK(hipGetLastError());
}

template <class T>
void sweep_top(riga_problem* pr, const Factor& F, const T* trow, const T* tcol, const double* b,
               double* x, hipStream_t s) {
  const TopDev& TD = pr->top;
  top_rhs_kernel<<<(TD.nT + 255) / 256, 256, 0, s>>>(F.tdof.p, F.tmap.p, TD.nT, TD.tgs, b, F.cbvec.p,
                                                     F.top_r.p);
  top_fwd_kernel<T><<<TD.n_fwd, TOP_FWD_THREADS, 0, s>>>(TD.fwd_units.p, TD.roff.p, TD.rlo.p, TD.rlen.p,
                                                         trow, F.top_r.p, F.top_y.p);
  top_bwd_kernel<T><<<TD.n_bwd, 256, (size_t)TD.max_h * sizeof(double), s>>>(
      TD.bwd_units.p, TD.fronts.p, TD.anc.p, tcol, F.top_y.p, F.piv_dof.p, x);
  HIPCHECK(hipGetLastError());
}

void set_top_attributes() {
  HIPCHECK(hipFuncSetAttribute((const void*)top_bwd_kernel<double>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024));
  HIPCHECK(hipFuncSetAttribute((const void*)top_bwd_kernel<float>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024));
}

template void build_top<double>(riga_problem*, Factor&, const double*, double*, double*, hipStream_t);
template void build_top<float>(riga_problem*, Factor&, const float*, float*, float*, hipStream_t);
template void sweep_top<double>(riga_problem*, const Factor&, const double*, const double*,
                                const double*, double*, hipStream_t);
template void sweep_top<float>(riga_problem*, const Factor&, const float*, const float*, const double*,
                               double*, hipStream_t);

}  // namespace riga
