// Forward/backward elimination with the multifrontal LDL^T factors: one
// application of (K - sigma M)^{-1} per Lanczos step (the "f/b elimination"
// of Sec. 5.1 and Table matvecs of arXiv 2009.08167).
//
// The sweeps use the partitioned inverse H = [L11^{-1}; L21 L11^{-1}] of each
// front (formed after the factorisation, see k_inverse.hip), so that a
// front's share of a sweep is one dense product with no serial chain:
//
// Forward, leaves to root.  y = P b(front's FS variables) (+) children's
// update vectors (extend-add);
//     z      = L11^{-1} y_FS                 (rows 0..k-1 of H, unit diagonal)
//     u_CB   = y_CB - (L21 L11^{-1}) y_FS    (rows k..f-1 of H)
// z is kept per fully-summed variable, u_CB is the update vector passed to
// the parent.  Row blocks of one front go to different workgroups.
// Backward, root to leaves.  w = D^{-1} z (1x1 and 2x2 blocks);
//     x_FS = L11^{-T} (w - L21^T x_CB) = (L11^{-1})^T w - (L21 L11^{-1})^T x_CB
// one dot product per column of H; column blocks go to different
// workgroups, and x(FS variables) = P^T x_FS.
// Every vector entry is written by one thread (no atomics); the children of
// a front and the partial sums are added in a fixed order, so results are
// bitwise reproducible.
#include <hip/hip_runtime.h>

#include <mutex>

#include "problem.h"
#include "wave_reduce.h"

namespace riga {
namespace {

struct SolveArgs {
  const int32_t* gmap;      // per front position: children's update indices
  int gstride;              // children slots per position (<= 4)
  const int32_t* rows;
  const int32_t* piv_type;  // 1: 1x1 pivot, 2/3: first/second of a 2x2 block
  const int32_t* piv_dof;   // DOF of each pivot
  const int32_t* piv_gmap;  // children's update indices of each pivot
  const double* dc;         // [N * 3] D^{-1} by pivot: w_n = c0 z_n + c+ z_{n+1} + c- z_{n-1}
  const int32_t* rows_piv;  // pivot index of the DOF at every front position
  double* cbvec;            // update vectors, one per front (f - k entries)
  double* fwd;              // z of the forward sweep, by new (pivot-order) index
};

// Forward sweep unit: RW rows of one front by 256 threads (tid 0..255),
// lanes over rows (the column-major H is read coalesced), 256 / RW thread
// groups over interleaved columns (RW = 16 on levels with few fronts, for
// more loads in flight per row).  The first 16 loads of H are issued before
// the gather of y so that both latencies overlap.  `smem` holds k + 256
// doubles; two barriers of the whole workgroup, whatever the unit (an empty
// unit, k = 0 and lo = hi = 0, touches no memory).
template <class T, int RW>
__device__ __forceinline__ void fwd_unit(const SolveArgs& sa, const T* __restrict__ H, const WorkUnit& u,
                                         const double* __restrict__ b, double* smem, int tid) {
  constexpr int G = 256 / RW;
  const int k = u.k, start = u.start, ldh = u.ldh;
  const int lo = u.lo, hi = u.hi;
  double* y = smem;          // k: permuted fully-summed right-hand side
  double* psum = y + k;      // G x RW partial sums
  const int gs = sa.gstride;
  const int rl = tid % RW, g = tid / RW;
  const int i = lo + rl;
  const bool row = i < hi;
  const int jend = row ? (i < k ? i : k) : 0;
  const T* hc = H + u.h_off + i;
  // the first 16 columns of this thread (predicated), before the gather
  double hv[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int j = g + G * q;
    hv[q] = j < jend ? (double)hc[(int64_t)j * ldh] : 0.0;
  }
  // the (i, i-1) slot of a 2x2 pivot block holds D, not L11^{-1} (= 0)
  const int skip = (row && i < k && i > 0 && sa.piv_type[start + i] == 3) ? i - 1 : -1;
  // update rows: the children's contributions at this position
  double ycb = 0.0;
  if (g == 0 && row && i >= k) {
    const int32_t* gm = sa.gmap + u.gmap_off + (int64_t)i * gs;
    int c[4];
#pragma unroll
    for (int sl = 0; sl < 4; ++sl) c[sl] = sl < gs ? gm[sl] : -1;
#pragma unroll
    for (int sl = 0; sl < 4; ++sl)
      if (c[sl] >= 0) ycb += sa.cbvec[c[sl]];
  }
  // the top rows need y_FS up to their own index, the update rows all of it
  const int kn = hi <= k ? hi : k;
  for (int t = tid; t < kn; t += 256) {
    const int n = start + t;
    int c[4];
#pragma unroll
    for (int sl = 0; sl < 4; ++sl) c[sl] = sl < gs ? sa.piv_gmap[(int64_t)n * gs + sl] : -1;
    double v = b[sa.piv_dof[n]];
#pragma unroll
    for (int sl = 0; sl < 4; ++sl)
      if (c[sl] >= 0) v += sa.cbvec[c[sl]];
    y[t] = v;
  }
  __syncthreads();
  double s = 0.0;
  for (int jb = g;;) {
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int j = jb + G * q;
      if (j < jend && j != skip) s += hv[q] * y[j];
    }
    jb += 16 * G;
    if (jb >= jend) break;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int j = jb + G * q;
      hv[q] = j < jend ? (double)hc[(int64_t)j * ldh] : 0.0;
    }
  }
  psum[g * RW + rl] = s;
  __syncthreads();
  if (g == 0 && row) {
    double tot = 0.0;
#pragma unroll
    for (int q = 0; q < G; ++q) tot += psum[q * RW + rl];
    if (i < k) sa.fwd[start + i] = y[i] + tot;
    else sa.cbvec[u.cb_off + i - k] = ycb - tot;
  }
}

template <class T, int RW>
__global__ void __launch_bounds__(256) fwd_kernel(SolveArgs sa, const T* __restrict__ H,
                                                  const WorkUnit* __restrict__ units,
                                                  const double* __restrict__ b) {
  extern __shared__ double smem[];
  const WorkUnit u = units[blockIdx.x];
  if (u.front < 0) return;  // padding slot of the XCD interleave
  fwd_unit<T, RW>(sa, H, u, b, smem, threadIdx.x);
}


// Backward sweep: 4 CPW columns of one front per workgroup; wave w takes
// columns lo + w + 4c (c < CPW), lanes over rows, 16 loads in flight per
// lane (16 / CPW row chunks of 64 per iteration; CPW = 1 on levels with few
// fronts).  The first iteration's loads are issued before the gather of v.
// One unit by 256 threads with `smem` of f - lo doubles; one barrier of the
// whole workgroup, whatever the unit (an empty one touches no memory).
template <class T, int CPW>
__device__ __forceinline__ void bwd_unit(const SolveArgs& sa, const T* __restrict__ H, const WorkUnit& u,
                                         double* x, double* smem, int tid) {
  constexpr int RCH = 16 / CPW;
  const int f = u.f, k = u.k, start = u.start, ldh = u.ldh;
  const int lo = u.lo, hi = u.hi;
  const T* Hf = H + u.h_off;
  const int32_t* rows = sa.rows + u.rows_off;
  double* v = smem;  // v[i - lo], i in [lo, f): D^{-1} z on the FS rows, -x below
  const int lane = tid & 63, wave = tid >> 6;
  int jc[CPW];
  bool two[CPW];
  double acc[CPW];
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    jc[c] = lo + wave + 4 * c;
    two[c] = jc[c] < hi && sa.piv_type[start + jc[c]] == 2;
    acc[c] = 0.0;
  }
  double hv[RCH][CPW];
  // the 2x2 slot (j + 1, j) holds D: loaded like the rest, zeroed at use,
  // so that the loads do not wait for the pivot types
  auto load = [&](int i0) {
#pragma unroll
    for (int r = 0; r < RCH; ++r) {
      const int i = i0 + 64 * r + lane;
#pragma unroll
      for (int c = 0; c < CPW; ++c) {
        const int j = jc[c];
        const bool use = j < hi && i < f && i > j;
        hv[r][c] = use ? (double)Hf[(int64_t)j * ldh + i] : 0.0;
      }
    }
  };
  // row chunks start on a 16-row boundary (whole cache lines); rows at or
  // above a column's diagonal are masked
  const int ibeg = (lo + 1) & ~15;
  if (ibeg < f) load(ibeg);
  // v in batches of GB rows per thread: the update rows' indices of a batch,
  // then their values, each set of loads in flight together (the rows of a
  // tall front's update block are many more than the threads)
  constexpr int GB = 4;
  for (int i0 = lo + tid; i0 < f; i0 += 256 * GB) {
    int ri[GB];
#pragma unroll
    for (int g = 0; g < GB; ++g) {
      const int i = i0 + 256 * g;
      ri[g] = (i >= k && i < f) ? rows[i] : -1;
    }
    double xv[GB];
#pragma unroll
    for (int g = 0; g < GB; ++g) xv[g] = ri[g] >= 0 ? x[ri[g]] : 0.0;
#pragma unroll
    for (int g = 0; g < GB; ++g) {
      const int i = i0 + 256 * g;
      if (i >= f) continue;
      double val;
      if (i < k) {
        // neighbours inside the front's own pivots (a 2x2 block never
        // crosses a front); their coefficient is zero otherwise
        const int n = start + i;
        const double* c3 = sa.dc + 3 * (int64_t)n;
        val = c3[0] * sa.fwd[n] + c3[1] * sa.fwd[start + min(i + 1, k - 1)] +
              c3[2] * sa.fwd[start + max(i - 1, 0)];
      } else {
        val = -xv[g];
      }
      v[i - lo] = val;
    }
  }
  __syncthreads();
  for (int i0 = ibeg; i0 < f; i0 += 64 * RCH) {
    if (i0 != ibeg) load(i0);
#pragma unroll
    for (int r = 0; r < RCH; ++r) {
      const int i = i0 + 64 * r + lane;
      const double vv = (i > lo && i < f) ? v[i - lo] : 0.0;
#pragma unroll
      for (int c = 0; c < CPW; ++c) acc[c] += (two[c] && i == jc[c] + 1) ? 0.0 : hv[r][c] * vv;
    }
  }
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    const double s = wave_sum(acc[c]);
    const int j = jc[c];
    if (lane == 0 && j < hi) x[sa.piv_dof[start + j]] = v[j - lo] + s;
  }
}

template <class T, int CPW>
__global__ void __launch_bounds__(256) bwd_kernel(SolveArgs sa, const T* __restrict__ H,
                                                  const WorkUnit* __restrict__ units, double* x) {
  extern __shared__ double smem[];
  const WorkUnit u = units[blockIdx.x];
  if (u.front < 0) return;  // padding slot of the XCD interleave
  bwd_unit<T, CPW>(sa, H, u, x, smem, threadIdx.x);
}


// ---- the bottom heights in one launch per direction ----
//
// One workgroup of SUB_GROUPS 256-thread groups per subtree (a front below
// the fused height whose parent lies above it, with its descendants).  The
// units of one height go to the groups in rounds, heights in order; a group
// without a unit in a round takes the empty one, so every group meets the
// same barriers.  The values passed between the subtree's fronts stay in
// LDS: the update vectors of the forward sweep, the solution of the
// backward sweep.  The barriers order LDS only, so the global loads of the
// next round (index maps, then H), issued before the current round is
// reduced and written, stay in flight across them.

__device__ __forceinline__ WorkUnit empty_unit() {
  WorkUnit u{};
  u.front = -1;
  return u;
}

__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// The rounds of a subtree: height h, round start r (group q takes unit
// r + q if below the height's end o[h + 1]).
__device__ __forceinline__ void round_skip(const int32_t* o, int nh, int& h, int& r) {
  while (h < nh && r >= o[h + 1]) {
    ++h;
    if (h < nh) r = o[h];
  }
}

template <class T>
struct FwdPre {
  T hv[16];      // H(i, g + G q), the first 16 columns of this thread
  int pt;        // pivot type of row i (a 2x2 block's second row skips a column)
  int rc[4];     // children's update entries at update row i
  int yc[4];     // children's update entries of y_FS entry tid
};

template <class T, int RW>
__device__ __forceinline__ void fwd_prefetch(const SolveArgs& sa, const T* __restrict__ H, const WorkUnit& u,
                                             int tid, FwdPre<T>& P) {
  constexpr int G = 256 / RW;
  const int k = u.k, start = u.start, lo = u.lo, hi = u.hi;
  const int rl = tid % RW, g = tid / RW, gs = sa.gstride;
  const int i = lo + rl;
  const bool row = i < hi;
  // Unconditional loads (a lane without an entry reads element 0 and drops
  // it), so the batch issues without branches; index maps first, so that
  // waiting for them does not wait for H.
  const bool own_pt = row && i < k && i > 0;
  const int pt = sa.piv_type[own_pt ? start + i : 0];
  P.pt = own_pt ? pt : 0;
#pragma unroll
  for (int sl = 0; sl < 4; ++sl) {
    const bool own = g == 0 && row && i >= k && sl < gs;
    const int c = sa.gmap[own ? u.gmap_off + (int64_t)i * gs + sl : 0];
    P.rc[sl] = own ? c : -1;
  }
  const int kn = hi <= k ? hi : k;
#pragma unroll
  for (int sl = 0; sl < 4; ++sl) {
    const bool own = tid < kn && sl < gs;
    const int c = sa.piv_gmap[own ? (int64_t)(start + tid) * gs + sl : 0];
    P.yc[sl] = own ? c : -1;
  }
  const int jend = row ? (i < k ? i : k) : 0;
  const T* hc = H + u.h_off + i;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int j = g + G * q;
    const T hvq = *(j < jend ? hc + (int64_t)j * u.ldh : H);
    P.hv[q] = j < jend ? hvq : (T)0;
  }
}

template <class T, int RW>
__global__ void __launch_bounds__(256 * SUB_GROUPS) fwd_subtree_kernel(
    SolveArgs sa, const T* __restrict__ H, const WorkUnit* __restrict__ units, const int32_t* __restrict__ off,
    const SubInfo* __restrict__ infos, int nh, int max_units, int max_np, int max_ncb, int grp_doubles,
    const double* __restrict__ b) {
  constexpr int G = 256 / RW;
  extern __shared__ double smem[];
  const int grp = threadIdx.x >> 8, tid = threadIdx.x & 255;
  const int rl = tid % RW, g = tid / RW, gs = sa.gstride;
  const SubInfo si = infos[blockIdx.x];
  const int32_t* o = off + (int64_t)blockIdx.x * (nh + 1);
  WorkUnit* uc = reinterpret_cast<WorkUnit*>(smem);
  double* yb = smem + (size_t)max_units * (sizeof(WorkUnit) / sizeof(double));  // b by subtree pivot
  double* cbs = yb + max_np;                                                    // update vectors
  double* y = cbs + max_ncb + (size_t)grp * grp_doubles;                        // k: y_FS
  const int u0 = o[0];
  int h = 0, r = u0;
  round_skip(o, nh, h, r);
  WorkUnit cur = (h < nh && r + grp < o[h + 1]) ? units[r + grp] : empty_unit();
  FwdPre<T> P;
  fwd_prefetch<T, RW>(sa, H, cur, tid, P);
  {
    const int64_t* src = reinterpret_cast<const int64_t*>(units + u0);
    int64_t* dst = reinterpret_cast<int64_t*>(uc);
    const int nw = (o[nh] - u0) * (int)(sizeof(WorkUnit) / sizeof(int64_t));
    for (int t = threadIdx.x; t < nw; t += 256 * SUB_GROUPS) dst[t] = src[t];
    for (int t = threadIdx.x; t < si.np; t += 256 * SUB_GROUPS) yb[t] = b[sa.piv_dof[si.p0 + t]];
  }
  lds_barrier();
  while (h < nh) {
    const int k = cur.k, start = cur.start, lo = cur.lo, hi = cur.hi;
    const int i = lo + rl;
    const bool row = i < hi;
    const int jend = row ? (i < k ? i : k) : 0;
    double* psum = y + k;  // G x RW partial sums
    // y_FS and the update rows' children entries, all from LDS
    // (branch-free: an absent entry reads slot 0 and adds zero)
    double ycb = 0.0;
#pragma unroll
    for (int sl = 0; sl < 4; ++sl) {
      const double c = cbs[P.rc[sl] >= 0 ? P.rc[sl] - si.cb0 : 0];
      ycb += P.rc[sl] >= 0 ? c : 0.0;
    }
    const int kn = hi <= k ? hi : k;
    if (tid < kn) {
      double v = yb[start + tid - si.p0];
#pragma unroll
      for (int sl = 0; sl < 4; ++sl) {
        const double c = cbs[P.yc[sl] >= 0 ? P.yc[sl] - si.cb0 : 0];
        v += P.yc[sl] >= 0 ? c : 0.0;
      }
      y[tid] = v;
    }
    for (int t = tid + 256; t < kn; t += 256) {
      double v = yb[start + t - si.p0];
      for (int sl = 0; sl < gs; ++sl) {
        const int c = sa.piv_gmap[(int64_t)(start + t) * gs + sl];
        if (c >= 0) v += cbs[c - si.cb0];
      }
      y[t] = v;
    }
    lds_barrier();
    const int skip = P.pt == 3 ? i - 1 : -1;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int j = g + G * q;
      const bool use = j < jend && j != skip;
      const double yj = y[use ? j : 0];
      s += use ? (double)P.hv[q] * yj : 0.0;
    }
    {
      const T* hc = H + cur.h_off + i;
      for (int jb = g + 16 * G; jb < jend; jb += 8 * G) {
        double hv[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int j = jb + G * q;
          hv[q] = j < jend ? (double)hc[(int64_t)j * cur.ldh] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int j = jb + G * q;
          if (j < jend && j != skip) s += hv[q] * y[j];
        }
      }
    }
    // the next round's loads, in flight while this one is reduced
    int h2 = h, r2 = r + SUB_GROUPS;
    round_skip(o, nh, h2, r2);
    const WorkUnit nx = (h2 < nh && r2 + grp < o[h2 + 1]) ? uc[r2 + grp - u0] : empty_unit();
    fwd_prefetch<T, RW>(sa, H, nx, tid, P);
    psum[g * RW + rl] = s;
    lds_barrier();
    if (g == 0 && row) {
      double tot = 0.0;
#pragma unroll
      for (int q = 0; q < G; ++q) tot += psum[q * RW + rl];
      if (i < k) {
        sa.fwd[start + i] = y[i] + tot;
      } else {
        const double val = ycb - tot;
        sa.cbvec[cur.cb_off + i - k] = val;
        cbs[cur.cb_off + i - k - si.cb0] = val;
      }
    }
    lds_barrier();
    cur = nx;
    h = h2;
    r = r2;
  }
}

template <class T, int CPW>
struct BwdPre {
  T hv[16 / CPW][CPW];  // the first row chunk of each column
  int pt[CPW];          // pivot types of the columns
  int dof[CPW];         // their output indices
  int rp[2], rd[2];     // update rows lo + tid (+ 256): pivot index and DOF
};

template <class T, int CPW>
__device__ __forceinline__ void bwd_prefetch(const SolveArgs& sa, const T* __restrict__ H, const WorkUnit& u,
                                             int tid, BwdPre<T, CPW>& P) {
  constexpr int RCH = 16 / CPW;
  const int f = u.f, k = u.k, start = u.start, lo = u.lo, hi = u.hi;
  const int lane = tid & 63, wave = tid >> 6;
  // unconditional loads from element 0 where a lane has no entry (see
  // fwd_prefetch), index maps first
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    const int j = lo + wave + 4 * c;
    const bool own = j < hi;
    const int pt = sa.piv_type[own ? start + j : 0];
    const int dof = sa.piv_dof[own ? start + j : 0];
    P.pt[c] = own ? pt : 0;
    P.dof[c] = own ? dof : 0;
  }
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const int i = lo + tid + 256 * e;
    const bool cb = i >= k && i < f;
    const int rp = sa.rows_piv[cb ? u.rows_off + i : 0];
    const int rd = sa.rows[cb ? u.rows_off + i : 0];
    P.rp[e] = cb ? rp : -1;
    P.rd[e] = cb ? rd : -1;
  }
  const int ibeg = (lo + 1) & ~15;
  const T* Hf = H + u.h_off;
#pragma unroll
  for (int rr = 0; rr < RCH; ++rr) {
    const int i = ibeg + 64 * rr + lane;
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      const int j = lo + wave + 4 * c;
      const bool use = j < hi && i < f && i > j;
      const T hv = *(use ? Hf + (int64_t)j * u.ldh + i : H);
      P.hv[rr][c] = use ? hv : (T)0;
    }
  }
}

template <class T, int CPW>
__global__ void __launch_bounds__(256 * SUB_GROUPS) bwd_subtree_kernel(
    SolveArgs sa, const T* __restrict__ H, const WorkUnit* __restrict__ units, const int32_t* __restrict__ off,
    const SubInfo* __restrict__ infos, int nh, int max_units, int max_np, int grp_doubles, double* x) {
  constexpr int RCH = 16 / CPW;
  extern __shared__ double smem[];
  const int grp = threadIdx.x >> 8, tid = threadIdx.x & 255;
  const int lane = tid & 63, wave = tid >> 6;
  const SubInfo si = infos[blockIdx.x];
  const int32_t* o = off + (int64_t)blockIdx.x * (nh + 1);
  WorkUnit* uc = reinterpret_cast<WorkUnit*>(smem);
  double* vz = smem + (size_t)max_units * (sizeof(WorkUnit) / sizeof(double));  // D^{-1} z by subtree pivot
  double* xs = vz + max_np;                                                     // x by subtree pivot
  double* v = xs + max_np + (size_t)grp * grp_doubles;                          // v[i - lo], i in [lo, f)
  const int u0 = o[0];
  // heights from the top: round starts within a height ascend
  int h = nh - 1, r = o[nh - 1];
  auto skip_down = [&](int& hh, int& rr) {
    while (hh >= 0 && rr >= o[hh + 1]) {
      --hh;
      if (hh >= 0) rr = o[hh];
    }
  };
  skip_down(h, r);
  WorkUnit cur = (h >= 0 && r + grp < o[h + 1]) ? units[r + grp] : empty_unit();
  BwdPre<T, CPW> P;
  bwd_prefetch<T, CPW>(sa, H, cur, tid, P);
  {
    const int64_t* src = reinterpret_cast<const int64_t*>(units + u0);
    int64_t* dst = reinterpret_cast<int64_t*>(uc);
    const int nw = (o[nh] - u0) * (int)(sizeof(WorkUnit) / sizeof(int64_t));
    for (int t = threadIdx.x; t < nw; t += 256 * SUB_GROUPS) dst[t] = src[t];
    // D^{-1} z of the subtree's pivots (a 2x2 block's partner lies in the
    // same front, and its coefficient is zero otherwise)
    for (int t = threadIdx.x; t < si.np; t += 256 * SUB_GROUPS) {
      const int64_t n = si.p0 + t;
      const double c0 = sa.dc[3 * n], cp = sa.dc[3 * n + 1], cm = sa.dc[3 * n + 2];
      const double z = sa.fwd[n];
      const double zp = cp != 0.0 ? sa.fwd[n + 1] : 0.0;
      const double zm = cm != 0.0 ? sa.fwd[n - 1] : 0.0;
      vz[t] = c0 * z + cp * zp + cm * zm;
    }
  }
  lds_barrier();
  while (h >= 0) {
    const int f = cur.f, k = cur.k, start = cur.start, lo = cur.lo, hi = cur.hi;
    // v: D^{-1} z on the fully-summed rows, -x below (from LDS when the
    // variable is the subtree's, else from the sweep above)
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int i = lo + tid + 256 * e;
      if (i < f) {
        double val;
        if (i < k) {
          val = vz[start + i - si.p0];
        } else {
          const int q = P.rp[e] - si.p0;
          val = -((q >= 0 && q < si.np) ? xs[q] : x[P.rd[e]]);
        }
        v[i - lo] = val;
      }
    }
    for (int i = lo + tid + 512; i < f; i += 256) {
      double val;
      if (i < k) {
        val = vz[start + i - si.p0];
      } else {
        const int q = sa.rows_piv[cur.rows_off + i] - si.p0;
        val = -((q >= 0 && q < si.np) ? xs[q] : x[sa.rows[cur.rows_off + i]]);
      }
      v[i - lo] = val;
    }
    lds_barrier();
    int jc[CPW];
    bool two[CPW];
    double acc[CPW];
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      jc[c] = lo + wave + 4 * c;
      two[c] = P.pt[c] == 2;
      acc[c] = 0.0;
    }
    const int ibeg = (lo + 1) & ~15;
    // rows at or above a column's diagonal were loaded as zero; the 2x2
    // slot (j + 1, j) holds D and is skipped
    if (ibeg < f) {
#pragma unroll
      for (int rr = 0; rr < RCH; ++rr) {
        const int i = ibeg + 64 * rr + lane;
        const bool in = i > lo && i < f;
        const double vl = v[in ? i - lo : 0];
        const double vv = in ? vl : 0.0;
#pragma unroll
        for (int c = 0; c < CPW; ++c) acc[c] += (two[c] && i == jc[c] + 1) ? 0.0 : (double)P.hv[rr][c] * vv;
      }
    }
    {
      const T* Hf = H + cur.h_off;
      for (int i0 = ibeg + 64 * RCH; i0 < f; i0 += 64 * RCH) {
        double hv[RCH][CPW];
#pragma unroll
        for (int rr = 0; rr < RCH; ++rr) {
          const int i = i0 + 64 * rr + lane;
#pragma unroll
          for (int c = 0; c < CPW; ++c) {
            const int j = jc[c];
            const bool use = j < hi && i < f && i > j;
            hv[rr][c] = use ? (double)Hf[(int64_t)j * cur.ldh + i] : 0.0;
          }
        }
#pragma unroll
        for (int rr = 0; rr < RCH; ++rr) {
          const int i = i0 + 64 * rr + lane;
          const double vv = (i > lo && i < f) ? v[i - lo] : 0.0;
#pragma unroll
          for (int c = 0; c < CPW; ++c) acc[c] += (two[c] && i == jc[c] + 1) ? 0.0 : hv[rr][c] * vv;
        }
      }
    }
    int dof[CPW];
#pragma unroll
    for (int c = 0; c < CPW; ++c) dof[c] = P.dof[c];
    // the next round's loads, in flight while this one is reduced
    int h2 = h, r2 = r + SUB_GROUPS;
    skip_down(h2, r2);
    const WorkUnit nx = (h2 >= 0 && r2 + grp < o[h2 + 1]) ? uc[r2 + grp - u0] : empty_unit();
    bwd_prefetch<T, CPW>(sa, H, nx, tid, P);
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      const double sm = wave_sum(acc[c]);
      const int j = jc[c];
      if (lane == 0 && j < hi) {
        const double val = v[j - lo] + sm;
        x[dof[c]] = val;
        xs[start + j - si.p0] = val;
      }
    }
    lds_barrier();
    cur = nx;
    h = h2;
    r = r2;
  }
}

// Pivot-order copies of the forward gather maps: DOF and children's update
// indices of every pivot (the pivot order changes with each factorisation).
__global__ void pivot_maps_kernel(const FrontDesc* __restrict__ desc,
                                  const int32_t* __restrict__ front_of,
                                  const int32_t* __restrict__ piv_perm,
                                  const int32_t* __restrict__ rows, const int32_t* __restrict__ gmap,
                                  int gs, int64_t N, int32_t* piv_dof, int32_t* piv_gmap,
                                  int32_t* piv_inv) {
  const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (n >= N) return;
  const FrontDesc d = desc[front_of[n]];
  const int pos = piv_perm[n];
  const int32_t dof = rows[d.rows_off + pos];
  piv_dof[n] = dof;
  piv_inv[dof] = (int32_t)n;
  for (int sl = 0; sl < gs; ++sl) piv_gmap[n * gs + sl] = gmap[d.gmap_off + (int64_t)pos * gs + sl];
}

// Pivot index of the DOF at every front position (per factorisation: the
// pivoting permutes each front's fully-summed variables).
__global__ void rows_piv_kernel(const int32_t* __restrict__ rows, int64_t n, const int32_t* __restrict__ piv_inv,
                                int32_t* rows_piv) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < n) rows_piv[e] = piv_inv[rows[e]];
}

// D^{-1} by pivot (per factorisation): w_n = c0 z_n + c+ z_{n+1} + c- z_{n-1},
// the neighbours non-zero only inside a 2x2 block.
__global__ void dinv_coef_kernel(const int32_t* __restrict__ piv_type, const double* __restrict__ dd,
                                 const double* __restrict__ dsub, int64_t N, double* dc) {
  const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (n >= N) return;
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
  dc[3 * n] = c0;
  dc[3 * n + 1] = cp;
  dc[3 * n + 2] = cm;
}

SolveArgs solve_args(riga_problem* pr, const Factor& F) {
  SolveArgs sa{};
  sa.gmap = pr->d_gmap.p;
  sa.gstride = pr->gstride;
  sa.rows = pr->d_rows.p;
  sa.piv_type = F.piv_type.p;
  sa.piv_dof = F.piv_dof.p;
  sa.piv_gmap = F.piv_gmap.p;
  sa.rows_piv = F.rows_piv.p;
  sa.dc = F.dcoef.p;
  sa.cbvec = F.cbvec.p;
  sa.fwd = F.fwd.p;
  return sa;
}

template <class T>
void apply_solve_attrs() {
  const void* ks[] = {(const void*)fwd_kernel<T, SWEEP_ROWS>, (const void*)fwd_kernel<T, SWEEP_ROWS_THIN>,
                      (const void*)bwd_kernel<T, SWEEP_COLS / 4>,
                      (const void*)bwd_kernel<T, SWEEP_COLS_THIN / 4>};
  for (const void* k : ks)
    HIPCHECK(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, 159 * 1024));
  const void* ksub[] = {(const void*)fwd_subtree_kernel<T, SUB_ROWS>,
                        (const void*)bwd_subtree_kernel<T, SUB_COLS / 4>};
  for (const void* k : ksub)
    HIPCHECK(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, 159 * 1024));
}

// One launch for the fused bottom heights, one per further tree level and
// direction below the top block (all levels
// when there is none), three for the top block.
template <class T>
void solve_levels(riga_problem* pr, const Factor& F, const T* H, const T* trow, const T* tcol,
                  const double* b, double* x, hipStream_t s) {
  SolveArgs sa = solve_args(pr, F);
  const int nl = pr->top.cut >= 0 ? pr->top.cut : (int)pr->levels.size();
  const SubtreeDev& S = pr->sub;
  if (S.nh > 0)
    fwd_subtree_kernel<T, SUB_ROWS><<<S.n_sub, 256 * SUB_GROUPS, S.lds_fwd, s>>>(
        sa, H, S.fwd_units.p, S.fwd_off.p, S.info.p, S.nh, S.max_units, S.max_np, S.max_ncb, S.grp_fwd, b);
  for (int h = S.nh; h < nl; ++h) {
    const LevelDev& L = pr->levels[h];
    if (L.n_fwd == 0) continue;
    const size_t lds = (size_t)(L.max_k + 256) * sizeof(double);
    if (L.fwd_thin) fwd_kernel<T, SWEEP_ROWS_THIN><<<L.n_fwd, 256, lds, s>>>(sa, H, L.fwd_units.p, b);
    else fwd_kernel<T, SWEEP_ROWS><<<L.n_fwd, 256, lds, s>>>(sa, H, L.fwd_units.p, b);
  }
  if (pr->top.cut >= 0) sweep_top<T>(pr, F, trow, tcol, b, x, s);
  for (int h = nl - 1; h >= S.nh; --h) {
    const LevelDev& L = pr->levels[h];
    if (L.n_bwd == 0) continue;
    const size_t lds = (size_t)L.max_f * sizeof(double);
    if (L.bwd_thin) bwd_kernel<T, SWEEP_COLS_THIN / 4><<<L.n_bwd, 256, lds, s>>>(sa, H, L.bwd_units.p, x);
    else bwd_kernel<T, SWEEP_COLS / 4><<<L.n_bwd, 256, lds, s>>>(sa, H, L.bwd_units.p, x);
  }
  if (S.nh > 0)
    bwd_subtree_kernel<T, SUB_COLS / 4><<<S.n_sub, 256 * SUB_GROUPS, S.lds_bwd, s>>>(
        sa, H, S.bwd_units.p, S.bwd_off.p, S.info.p, S.nh, S.max_units, S.max_np, S.grp_bwd, x);
  HIPCHECK(hipGetLastError());
}

}  // namespace

void set_solve_attributes() {
  apply_solve_attrs<double>();
  apply_solve_attrs<float>();
}

void launch_pivot_maps(riga_problem* pr, Factor& F, hipStream_t s) {
  const int64_t N = pr->an.N;
  if (N == 0) return;
  pivot_maps_kernel<<<(unsigned)((N + 255) / 256), 256, 0, s>>>(
      pr->d_desc.p, pr->d_front_of.p, F.piv_perm.p, pr->d_rows.p, pr->d_gmap.p, pr->gstride, N,
      F.piv_dof.p, F.piv_gmap.p, F.piv_inv.p);
  const int64_t nr = pr->an.f_rows_off[pr->an.n_fronts];
  if (nr > 0)
    rows_piv_kernel<<<(unsigned)((nr + 255) / 256), 256, 0, s>>>(pr->d_rows.p, nr, F.piv_inv.p, F.rows_piv.p);
  dinv_coef_kernel<<<(unsigned)((N + 255) / 256), 256, 0, s>>>(F.piv_type.p, F.d_diag.p, F.d_sub.p, N,
                                                             F.dcoef.p);
  HIPCHECK(hipGetLastError());
}

void solve_fb(riga_problem* pr, const Factor& F, const double* b, double* x, hipStream_t s) {
  if (!F.factored) throw Error(RIGA_EINVAL, "solve before factorisation");
  set_kernel_attributes();
  if (F.precision == RIGA_MIXED) solve_levels<float>(pr, F, F.h32.p, F.trow32.p, F.tcol32.p, b, x, s);
  else solve_levels<double>(pr, F, F.h64.p, F.trow64.p, F.tcol64.p, b, x, s);
}

}  // namespace riga
