// Eigenfunction errors against the exact eigenpairs of the Dirichlet
// Laplacian on the unit square and cube (Eq. exact of arXiv 2009.08167):
// the L2 and energy norms of u_h - u_e (Eq. norms) that define EFerr_L2 and
// EFerr_E (Eq. eigerrors), for the diagonal modes that Sec. 8 compares.
//
// 1. load_1d: g_{m,d}[a] = int B_a(x) sqrt(2) sin(i_{m,d} pi x) dx for every
//    mode m, direction d and interior function a (Gauss rule of q points per
//    element; one thread per entry, summing over the function's support).
// 2. overlap: G[n][m] = (u_h,n , u_e,m) = sum_a U[n][a] prod_d g_{m,d}[a_d]:
//    an exact mode is a product of one factor per direction, so its load
//    vector is the tensor product of the 1D loads.  One workgroup per
//    eigenvector and group of 8 modes; a fixed-order reduction.
// 3. (host) the matched eigenvector of mode m maximises |G[n][m]|.
// 4. err_elem: per mode and element, the integrals of (u_h -/+ u_e)^2 and
//    |grad u_h -/+ grad u_e|^2 over the element's q^d Gauss points, u_h by
//    sum factorisation over the element's (p+1)^d coefficients.  Both signs
//    are kept so that the smaller error is formed without cancellation.
// 5. err_reduce: per mode and quantity, the element sums in a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "problem.h"

namespace riga {
namespace {

constexpr int NP_MAX = 7;   // p <= 6
constexpr int Q_MAX = 16;   // Gauss points per direction and element
constexpr int OV_MODES = 8; // modes per overlap workgroup

struct AccArgs {
  int dim, p, q, nm;
  int ne[3], n1[3], tab_off[3], fn_off[3], nfn[3];
  int64_t N, nel;
  const int* first_fn;
  const int* fe;
  const int* le;
  const double* val;  // basis values at the q-point rule, per direction and element
  const double* der;
  const double* gx;   // Gauss nodes on [-1, 1]
  const double* gw;
  const int32_t* modes;  // [nm][dim], 1-based
  int n1max;
  double* g;          // [nm][dim][n1max]
};

__global__ void load_1d_kernel(AccArgs a) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)a.nm * a.dim * a.n1max;
  if (t >= total) return;
  const int fa = (int)(t % a.n1max);
  const int d = (int)((t / a.n1max) % a.dim);
  const int m = (int)(t / ((int64_t)a.n1max * a.dim));
  double sum = 0.0;
  if (fa < a.n1[d]) {
    const int fn = fa + 1;  // interior function, global index within direction d
    const int np = a.p + 1;
    const double h = 1.0 / a.ne[d];
    const double w = 0.5 * h;
    const double k = (double)a.modes[m * a.dim + d] * M_PI;
    for (int el = a.fe[a.fn_off[d] + fn]; el <= a.le[a.fn_off[d] + fn]; ++el) {
      const int loc = fn - a.first_fn[a.tab_off[d] + el];
      const int64_t o = (int64_t)(a.tab_off[d] + el) * a.q * np + loc;
      for (int qp = 0; qp < a.q; ++qp) {
        const double x = (el + 0.5 * (a.gx[qp] + 1.0)) * h;
        sum += a.gw[qp] * w * a.val[o + (int64_t)qp * np] * (M_SQRT2 * sin(k * x));
      }
    }
  }
  a.g[t] = sum;
}

__global__ void __launch_bounds__(256) overlap_kernel(AccArgs a, const double* __restrict__ U, double* G) {
  __shared__ double red[OV_MODES][256];
  const int n = blockIdx.x;
  const int m0 = blockIdx.y * OV_MODES;
  const int nmb = min(OV_MODES, a.nm - m0);
  const double* u = U + (int64_t)n * a.N;
  double acc[OV_MODES];
#pragma unroll
  for (int k = 0; k < OV_MODES; ++k) acc[k] = 0.0;
  for (int64_t i = threadIdx.x; i < a.N; i += 256) {
    const int ix = (int)(i % a.n1[0]);
    const int iy = (int)((i / a.n1[0]) % a.n1[1]);
    const int iz = a.dim == 3 ? (int)(i / ((int64_t)a.n1[0] * a.n1[1])) : 0;
    const double ui = u[i];
#pragma unroll
    for (int k = 0; k < OV_MODES; ++k) {
      if (k < nmb) {
        const double* gm = a.g + (int64_t)(m0 + k) * a.dim * a.n1max;
        double f = gm[ix] * gm[a.n1max + iy];
        if (a.dim == 3) f *= gm[2 * (int64_t)a.n1max + iz];
        acc[k] += ui * f;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < OV_MODES; ++k) red[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
#pragma unroll
      for (int k = 0; k < OV_MODES; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
    __syncthreads();
  }
  if ((int)threadIdx.x < nmb) G[(int64_t)n * a.nm + m0 + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void __launch_bounds__(128) err_elem_kernel(AccArgs a, const double* __restrict__ U,
                                                       const int32_t* __restrict__ match, double* part) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int m = blockIdx.y;
  if (e >= a.nel) return;
  const int np = a.p + 1, q = a.q;
  const int ei[3] = {(int)(e % a.ne[0]), (int)((e / a.ne[0]) % a.ne[1]),
                     (int)(e / ((int64_t)a.ne[0] * a.ne[1]))};
  const double* u = U + (int64_t)match[m] * a.N;
  const int nz = a.dim == 3 ? np : 1;
  // local coefficients c[az][ay][ax] (zero on the Dirichlet functions)
  int f0[3] = {0, 0, 0};
  for (int d = 0; d < a.dim; ++d) f0[d] = a.first_fn[a.tab_off[d] + ei[d]];
  double c[NP_MAX * NP_MAX * NP_MAX];
  for (int az = 0; az < nz; ++az)
    for (int ay = 0; ay < np; ++ay)
      for (int ax = 0; ax < np; ++ax) {
        const int gx = f0[0] + ax, gy = f0[1] + ay, gz = a.dim == 3 ? f0[2] + az : 1;
        const bool in = gx >= 1 && gx <= a.nfn[0] - 2 && gy >= 1 && gy <= a.nfn[1] - 2 &&
                        (a.dim == 2 || (gz >= 1 && gz <= a.nfn[2] - 2));
        c[(az * np + ay) * np + ax] =
            in ? u[(gx - 1) + (int64_t)a.n1[0] * ((gy - 1) + (int64_t)a.n1[1] * (gz - 1))] : 0.0;
      }
  // exact factors per direction at the element's points
  double sx[3][Q_MAX], dx[3][Q_MAX], wq[3][Q_MAX];
  for (int d = 0; d < 3; ++d)
    for (int qp = 0; qp < q; ++qp) {
      if (d < a.dim) {
        const double h = 1.0 / a.ne[d];
        const double x = (ei[d] + 0.5 * (a.gx[qp] + 1.0)) * h;
        const double k = (double)a.modes[m * a.dim + d] * M_PI;
        sx[d][qp] = M_SQRT2 * sin(k * x);
        dx[d][qp] = M_SQRT2 * k * cos(k * x);
        wq[d][qp] = a.gw[qp] * 0.5 * h;
      } else {
        sx[d][qp] = 1.0;
        dx[d][qp] = 0.0;
        wq[d][qp] = 1.0;
      }
    }
  const double* tv[3];
  const double* td[3];
  for (int d = 0; d < a.dim; ++d) {
    tv[d] = a.val + (int64_t)(a.tab_off[d] + ei[d]) * q * np;
    td[d] = a.der + (int64_t)(a.tab_off[d] + ei[d]) * q * np;
  }
  double lm = 0.0, lp = 0.0, em = 0.0, ep = 0.0;
  const int qz_n = a.dim == 3 ? q : 1;
  for (int qz = 0; qz < qz_n; ++qz) {
    // s0 = sum_az c B_z, s1 = sum_az c B_z'
    double s0[NP_MAX * NP_MAX], s1[NP_MAX * NP_MAX];
    for (int t = 0; t < np * np; ++t) {
      if (a.dim == 3) {
        double v0 = 0.0, v1 = 0.0;
        for (int az = 0; az < np; ++az) {
          v0 += c[az * np * np + t] * tv[2][qz * np + az];
          v1 += c[az * np * np + t] * td[2][qz * np + az];
        }
        s0[t] = v0;
        s1[t] = v1;
      } else {
        s0[t] = c[t];
        s1[t] = 0.0;
      }
    }
    for (int qy = 0; qy < q; ++qy) {
      double t00[NP_MAX], t01[NP_MAX], t10[NP_MAX];
      for (int ax = 0; ax < np; ++ax) {
        double v00 = 0.0, v01 = 0.0, v10 = 0.0;
        for (int ay = 0; ay < np; ++ay) {
          const double by = tv[1][qy * np + ay], dby = td[1][qy * np + ay];
          v00 += s0[ay * np + ax] * by;
          v01 += s0[ay * np + ax] * dby;
          v10 += s1[ay * np + ax] * by;
        }
        t00[ax] = v00;
        t01[ax] = v01;
        t10[ax] = v10;
      }
      for (int qx = 0; qx < q; ++qx) {
        double uh = 0.0, ux = 0.0, uy = 0.0, uz = 0.0;
        for (int ax = 0; ax < np; ++ax) {
          const double bx = tv[0][qx * np + ax], dbx = td[0][qx * np + ax];
          uh += t00[ax] * bx;
          ux += t00[ax] * dbx;
          uy += t01[ax] * bx;
          uz += t10[ax] * bx;
        }
        const double ue = sx[0][qx] * sx[1][qy] * sx[2][qz];
        const double gxe = dx[0][qx] * sx[1][qy] * sx[2][qz];
        const double gye = sx[0][qx] * dx[1][qy] * sx[2][qz];
        const double gze = sx[0][qx] * sx[1][qy] * dx[2][qz];
        const double w = wq[0][qx] * wq[1][qy] * wq[2][qz];
        const double dm = uh - ue, dp = uh + ue;
        lm += w * dm * dm;
        lp += w * dp * dp;
        const double ax_m = ux - gxe, ay_m = uy - gye, az_m = uz - gze;
        const double ax_p = ux + gxe, ay_p = uy + gye, az_p = uz + gze;
        em += w * (ax_m * ax_m + ay_m * ay_m + az_m * az_m);
        ep += w * (ax_p * ax_p + ay_p * ay_p + az_p * az_p);
      }
    }
  }
  double* o = part + ((int64_t)m * a.nel + e) * 4;
  o[0] = lm;
  o[1] = lp;
  o[2] = em;
  o[3] = ep;
}

__global__ void __launch_bounds__(256) err_reduce_kernel(const double* __restrict__ part, int64_t nel,
                                                         double* out) {
  __shared__ double red[256];
  const int m = blockIdx.x >> 2, t = blockIdx.x & 3;
  double s = 0.0;
  for (int64_t e = threadIdx.x; e < nel; e += 256) s += part[((int64_t)m * nel + e) * 4 + t];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

}  // namespace

void mode_errors(riga_problem* pr, int n_vec, const double* lam, const double* U, int nm,
                 const int32_t* modes, int nquad, int32_t* match, double* overlap, double* ef_l2,
                 double* ef_e, double* ev, hipStream_t s) {
  const Analysis& an = pr->an;
  const int dim = an.dim, p = an.p;
  const int q = nquad > 0 ? nquad : p + 6;
  if (p + 1 > NP_MAX) throw Error(RIGA_EUNSUPPORTED, "degree above 6");
  if (q > Q_MAX) throw Error(RIGA_EINVAL, "nquad above 16");
  for (int m = 0; m < nm; ++m)
    for (int d = 0; d < dim; ++d)
      if (modes[m * dim + d] < 1) throw Error(RIGA_EINVAL, "mode indices start at 1");
  DBuf<double> val, der;
  basis_tables_q(pr, q, val, der);  // synchronises the problem's stream
  std::vector<double> gx, gw;
  gauss_legendre(q, gx, gw);
  std::vector<int32_t> hm(modes, modes + (size_t)nm * dim);
  DBuf<double> d_gx, d_gw, g, G, part, out;
  DBuf<int32_t> d_modes, d_match;
  d_gx.upload(gx, s);
  d_gw.upload(gw, s);
  d_modes.upload(hm, s);
  AccArgs a{};
  a.dim = dim;
  a.p = p;
  a.q = q;
  a.nm = nm;
  int n1max = 1;
  for (int d = 0; d < 3; ++d) {
    a.ne[d] = d < dim ? an.ne[d] : 1;
    a.n1[d] = d < dim ? an.n1[d] : 1;
    a.tab_off[d] = pr->tab_off[d];
    a.fn_off[d] = pr->fn_off[d];
    a.nfn[d] = d < dim ? an.sp[d].n : 3;
    if (d < dim) n1max = std::max(n1max, an.n1[d]);
  }
  a.N = an.N;
  a.nel = an.n_elem;
  a.first_fn = pr->first_fn.p;
  a.fe = pr->fe.p;
  a.le = pr->le.p;
  a.val = val.p;
  a.der = der.p;
  a.gx = d_gx.p;
  a.gw = d_gw.p;
  a.modes = d_modes.p;
  a.n1max = n1max;
  g.alloc((size_t)nm * dim * n1max, s);
  a.g = g.p;
  const int64_t ng = (int64_t)nm * dim * n1max;
  load_1d_kernel<<<(unsigned)((ng + 255) / 256), 256, 0, s>>>(a);
  HIPCHECK(hipGetLastError());
  G.alloc((size_t)n_vec * nm, s);
  overlap_kernel<<<dim3(n_vec, (nm + OV_MODES - 1) / OV_MODES), 256, 0, s>>>(a, U, G.p);
  HIPCHECK(hipGetLastError());
  std::vector<double> hG((size_t)n_vec * nm);
  HIPCHECK(hipMemcpyAsync(hG.data(), G.p, hG.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  std::vector<int32_t> hmatch(nm);
  for (int m = 0; m < nm; ++m) {
    int best = 0;
    for (int n = 1; n < n_vec; ++n)
      if (std::fabs(hG[(size_t)n * nm + m]) > std::fabs(hG[(size_t)best * nm + m])) best = n;
    hmatch[m] = best;
  }
  d_match.upload(hmatch, s);
  part.alloc((size_t)nm * an.n_elem * 4, s);
  err_elem_kernel<<<dim3((unsigned)((an.n_elem + 127) / 128), nm), 128, 0, s>>>(a, U, d_match.p, part.p);
  HIPCHECK(hipGetLastError());
  out.alloc((size_t)nm * 4, s);
  err_reduce_kernel<<<nm * 4, 256, 0, s>>>(part.p, an.n_elem, out.p);
  HIPCHECK(hipGetLastError());
  std::vector<double> ho((size_t)nm * 4);
  HIPCHECK(hipMemcpyAsync(ho.data(), out.p, ho.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  for (int m = 0; m < nm; ++m) {
    double sq = 0.0;
    for (int d = 0; d < dim; ++d) sq += (double)hm[m * dim + d] * hm[m * dim + d];
    const double lam_e = M_PI * M_PI * sq;
    const double* o = &ho[(size_t)m * 4];
    const bool minus = o[0] <= o[1];  // the sign that aligns u_h with u_e
    match[m] = hmatch[m];
    overlap[m] = hG[(size_t)hmatch[m] * nm + m];
    ef_l2[m] = minus ? o[0] : o[1];
    ef_e[m] = (minus ? o[2] : o[3]) / lam_e;
    ev[m] = (lam[hmatch[m]] - lam_e) / lam_e;
  }
}

void exact_eigenvalues(int dim, int count, double* out) {
  // every tuple of indices in [1, n]; n grows until no tuple outside the box
  // can be among the `count` smallest (any index above n gives a value of at
  // least (n+1)^2 + dim - 1)
  for (int n = 4;; n *= 2) {
    std::vector<int64_t> v;
    if (dim == 2) {
      for (int i = 1; i <= n; ++i)
        for (int j = 1; j <= n; ++j) v.push_back((int64_t)i * i + (int64_t)j * j);
    } else {
      for (int i = 1; i <= n; ++i)
        for (int j = 1; j <= n; ++j)
          for (int k = 1; k <= n; ++k) v.push_back((int64_t)i * i + (int64_t)j * j + (int64_t)k * k);
    }
    if ((int64_t)v.size() < count) continue;
    std::nth_element(v.begin(), v.begin() + (count - 1), v.end());
    const int64_t top = v[count - 1];
    if (top >= (int64_t)(n + 1) * (n + 1) + dim - 1) continue;
    std::sort(v.begin(), v.begin() + count);
    for (int t = 0; t < count; ++t) out[t] = M_PI * M_PI * (double)v[t];
    return;
  }
}

}  // namespace riga
