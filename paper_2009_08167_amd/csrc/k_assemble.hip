// Gauss-quadrature assembly of the B-spline stiffness and mass matrices
// (Eqs. 1Dmatrix, 2Dmatrix of arXiv 2009.08167, generalised to per-element
// coefficients kappa_e, rho_e; Eqs. weakform--weakform3).
//
// Three kernels:
//  1. basis_tables: the p+1 non-zero B-splines and derivatives at each Gauss
//     point of each element, per direction (Cox--de Boor, Eq. N).
//  2. element_1d: 1D element stiffness / mass matrices (p+1)x(p+1).
//  3. assemble: one thread per stored non-zero (row a, column b) sums the
//     contributions of the <= (p+1)^d elements shared by the supports of
//     B_a and B_b.  Element matrices are tensor products, so each term is
//     kappa_e (My (x) Kx + Ky (x) Mx)[a,b] (3D analogous).  No atomics, each
//     value written once, consecutive threads write consecutive values.
#include <hip/hip_runtime.h>

#include <cmath>

#include "problem.h"

namespace riga {
namespace {

constexpr int PMAX = 7;  // p <= 6

// B_{span-deg+a, deg}(x), a = 0..deg: the degree-`deg` B-splines that are
// non-zero in knot span `span`, obtained by raising the degree one step at a
// time from the degree-0 indicator of the span (Eq. N), keeping only the
// functions whose support contains the span.  A term whose knot difference
// vanishes is zero (0/0 := 0).
__device__ void span_basis(const double* kv, int span, int deg, double x, double* b) {
  double prev[PMAX + 1];
  b[0] = 1.0;
  for (int r = 1; r <= deg; ++r) {
    for (int a = 0; a < r; ++a) prev[a] = b[a];
    for (int a = 0; a <= r; ++a) {
      const int i = span - r + a;
      double v = 0.0;
      if (a >= 1) {  // B_{i,r-1} = prev[a-1]
        const double den = kv[i + r] - kv[i];
        if (den > 0.0) v += (x - kv[i]) / den * prev[a - 1];
      }
      if (a <= r - 1) {  // B_{i+1,r-1} = prev[a]
        const double den = kv[i + r + 1] - kv[i + 1];
        if (den > 0.0) v += (kv[i + r + 1] - x) / den * prev[a];
      }
      b[a] = v;
    }
  }
}

// Values and first derivatives of the p+1 B-splines non-zero in `span`.
// Derivative: B'_{i,p} = p/(k[i+p]-k[i]) B_{i,p-1} - p/(k[i+p+1]-k[i+1]) B_{i+1,p-1}.
__device__ void local_basis(const double* kv, int span, int p, double x, double* val,
                            double* der) {
  double lower[PMAX + 1];
  span_basis(kv, span, p, x, val);
  span_basis(kv, span, p - 1, x, lower);  // B_{span-p+1+a, p-1}
  for (int a = 0; a <= p; ++a) {
    const int i = span - p + a;
    double d = 0.0;
    if (a >= 1) {  // B_{i,p-1} = lower[a-1]
      const double den = kv[i + p] - kv[i];
      if (den > 0.0) d += p / den * lower[a - 1];
    }
    if (a <= p - 1) {  // B_{i+1,p-1} = lower[a]
      const double den = kv[i + p + 1] - kv[i + 1];
      if (den > 0.0) d -= p / den * lower[a];
    }
    der[a] = d;
  }
}

struct TabArgs {
  const double* kv[3];   // knot values per direction
  const int* first_fn;   // concatenated per direction
  int tab_off[3];
  int ne[3];
  int dim, p, q;
  const double* gx;      // Gauss nodes on [-1, 1]
  const double* gw;
  double* val;
  double* der;
  double* ke1;
  double* me1;
  double* ge1;           // optional: int B_a B_b' (derivative on the second index)
};

__global__ void basis_tables_kernel(TabArgs a) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  int d = 0, e = t / a.q, qp = t % a.q;
  int acc = 0;
  for (d = 0; d < a.dim; ++d) {
    if (e < acc + a.ne[d]) break;
    acc += a.ne[d];
  }
  if (d >= a.dim) return;
  const int el = e - acc;
  const int ne = a.ne[d];
  const double h = 1.0 / ne;
  const double x = (el + 0.5 * (a.gx[qp] + 1.0)) * h;
  const int span = a.first_fn[a.tab_off[d] + el] + a.p;
  double val[PMAX + 1], der[PMAX + 1];
  local_basis(a.kv[d], span, a.p, x, val, der);
  const int np = a.p + 1;
  const int64_t o = ((int64_t)(a.tab_off[d] + el) * a.q + qp) * np;
  for (int i = 0; i < np; ++i) {
    a.val[o + i] = val[i];
    a.der[o + i] = der[i];
  }
}

__global__ void element_1d_kernel(TabArgs a, int total_el) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int np = a.p + 1;
  const int e = t / (np * np);
  if (e >= total_el) return;
  const int ab = t % (np * np), ia = ab / np, ib = ab % np;
  int d = 0, acc = 0;
  for (d = 0; d < a.dim; ++d) {
    if (e < acc + a.ne[d]) break;
    acc += a.ne[d];
  }
  const double hw = 0.5 / a.ne[d];  // Jacobian of [-1,1] -> element
  double k = 0.0, m = 0.0, g = 0.0;
  for (int qp = 0; qp < a.q; ++qp) {
    const int64_t o = ((int64_t)e * a.q + qp) * np;
    k += a.gw[qp] * hw * a.der[o + ia] * a.der[o + ib];
    m += a.gw[qp] * hw * a.val[o + ia] * a.val[o + ib];
    g += a.gw[qp] * hw * a.val[o + ia] * a.der[o + ib];
  }
  a.ke1[(int64_t)e * np * np + ab] = k;
  a.me1[(int64_t)e * np * np + ab] = m;
  if (a.ge1) a.ge1[(int64_t)e * np * np + ab] = g;
}

struct AsmArgs {
  const int64_t* row_ptr;
  const int32_t* col;
  int64_t N, nnz;
  int n1[3];
  int ne[3];
  int tab_off[3];
  int fn_off[3];
  const int* fe;
  const int* le;
  const int* first_fn;
  const double* ke1;
  const double* me1;
  const double* ge1;
  const double* kappa;
  const double* rho;
  int dim, p;
  int cplx;              // complex pencil in real-equivalent form (2 x 2 blocks)
  double A[3];           // its vector potential
  double* kv;
  double* mv;
};

__global__ void assemble_kernel(AsmArgs a) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= a.nnz) return;
  // row of entry e: last r with row_ptr[r] <= e
  int64_t lo = 0, hi = a.N;
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (a.row_ptr[mid] <= e) lo = mid; else hi = mid;
  }
  // a complex pencil: unknowns 2d (real part) and 2d + 1 (imaginary part)
  // of scalar DOF d, each scalar coupling a 2 x 2 block [[Kr, -Ki], [Ki, Kr]]
  const int64_t r = a.cplx ? lo >> 1 : lo, c = a.cplx ? (a.col[e] >> 1) : a.col[e];
  const int part_r = a.cplx ? (int)(lo & 1) : 0, part_c = a.cplx ? (a.col[e] & 1) : 0;
  int ri[3], ci[3];
  int64_t rr = r, cc = c;
  for (int d = 0; d < 3; ++d) {
    ri[d] = (int)(rr % a.n1[d]);
    rr /= a.n1[d];
    ci[d] = (int)(cc % a.n1[d]);
    cc /= a.n1[d];
  }
  // per direction: shared element range and, per element, the local indices
  int e0[3] = {0, 0, 0}, e1[3] = {0, 0, 0};
  for (int d = 0; d < a.dim; ++d) {
    const int gr = ri[d] + 1 + a.fn_off[d], gc = ci[d] + 1 + a.fn_off[d];
    e0[d] = max(a.fe[gr], a.fe[gc]);
    e1[d] = min(a.le[gr], a.le[gc]);
  }
  const int np = a.p + 1, np2 = np * np;
  double ksum = 0.0, msum = 0.0, isum = 0.0;
  // the magnetic form: |A|^2 B_a B_b added to the real part, and the
  // imaginary part sum_d A_d int (B_a d_d B_b - B_b d_d B_a)
  const double A2 = a.A[0] * a.A[0] + a.A[1] * a.A[1] + a.A[2] * a.A[2];
  if (a.dim == 2) {
    for (int ey = e0[1]; ey <= e1[1]; ++ey) {
      const int fy = a.first_fn[a.tab_off[1] + ey];
      const int ay = ri[1] + 1 - fy, by = ci[1] + 1 - fy;
      const int64_t oy = (int64_t)(a.tab_off[1] + ey) * np2 + ay * np + by;
      const double Ky = a.ke1[oy], My = a.me1[oy];
      for (int ex = e0[0]; ex <= e1[0]; ++ex) {
        const int fx = a.first_fn[a.tab_off[0] + ex];
        const int ax = ri[0] + 1 - fx, bx = ci[0] + 1 - fx;
        const int64_t ox = (int64_t)(a.tab_off[0] + ex) * np2 + ax * np + bx;
        const double Kx = a.ke1[ox], Mx = a.me1[ox];
        const int64_t el = (int64_t)ex + (int64_t)a.ne[0] * ey;
        const double kap = a.kappa ? a.kappa[el] : 1.0;
        const double rh = a.rho ? a.rho[el] : 1.0;
        ksum += kap * (My * Kx + Ky * Mx);
        msum += rh * (My * Mx);
        if (a.cplx) {
          const int64_t ox_t = (int64_t)(a.tab_off[0] + ex) * np2 + bx * np + ax;
          const int64_t oy_t = (int64_t)(a.tab_off[1] + ey) * np2 + by * np + ay;
          ksum += A2 * (My * Mx);
          isum += a.A[0] * My * (a.ge1[ox] - a.ge1[ox_t]) + a.A[1] * (a.ge1[oy] - a.ge1[oy_t]) * Mx;
        }
      }
    }
  } else {
    for (int ez = e0[2]; ez <= e1[2]; ++ez) {
      const int fz = a.first_fn[a.tab_off[2] + ez];
      const int az = ri[2] + 1 - fz, bz = ci[2] + 1 - fz;
      const int64_t oz = (int64_t)(a.tab_off[2] + ez) * np2 + az * np + bz;
      const double Kz = a.ke1[oz], Mz = a.me1[oz];
      const double Gz = a.cplx ? a.ge1[oz] - a.ge1[(int64_t)(a.tab_off[2] + ez) * np2 + bz * np + az] : 0.0;
      for (int ey = e0[1]; ey <= e1[1]; ++ey) {
        const int fy = a.first_fn[a.tab_off[1] + ey];
        const int ay = ri[1] + 1 - fy, by = ci[1] + 1 - fy;
        const int64_t oy = (int64_t)(a.tab_off[1] + ey) * np2 + ay * np + by;
        const double Ky = a.ke1[oy], My = a.me1[oy];
        const double Gy = a.cplx ? a.ge1[oy] - a.ge1[(int64_t)(a.tab_off[1] + ey) * np2 + by * np + ay] : 0.0;
        for (int ex = e0[0]; ex <= e1[0]; ++ex) {
          const int fx = a.first_fn[a.tab_off[0] + ex];
          const int ax = ri[0] + 1 - fx, bx = ci[0] + 1 - fx;
          const int64_t ox = (int64_t)(a.tab_off[0] + ex) * np2 + ax * np + bx;
          const double Kx = a.ke1[ox], Mx = a.me1[ox];
          const int64_t el = ex + (int64_t)a.ne[0] * (ey + (int64_t)a.ne[1] * ez);
          const double kap = a.kappa ? a.kappa[el] : 1.0;
          const double rh = a.rho ? a.rho[el] : 1.0;
          ksum += kap * (Mz * My * Kx + Mz * Ky * Mx + Kz * My * Mx);
          msum += rh * (Mz * My * Mx);
          if (a.cplx) {
            const double Gx = a.ge1[ox] - a.ge1[(int64_t)(a.tab_off[0] + ex) * np2 + bx * np + ax];
            ksum += A2 * (Mz * My * Mx);
            isum += a.A[0] * Mz * My * Gx + a.A[1] * Mz * Gy * Mx + a.A[2] * Gz * My * Mx;
          }
        }
      }
    }
  }
  if (a.cplx) {
    // block [[Kr, -Ki], [Ki, Kr]] and diag(M, M)
    a.kv[e] = part_r == part_c ? ksum : (part_r == 0 ? -isum : isum);
    a.mv[e] = part_r == part_c ? msum : 0.0;
  } else {
    a.kv[e] = ksum;
    a.mv[e] = msum;
  }
}

// Row sums of |values| (1-norm = inf-norm of a symmetric matrix) and max |entry|.
__global__ void row_abs_sum_kernel(const int64_t* row_ptr, const double* v, int64_t N, double* out) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= N) return;
  double s = 0.0;
  for (int64_t e = row_ptr[r]; e < row_ptr[r + 1]; ++e) s += fabs(v[e]);
  out[r] = s;
}

__global__ void max_reduce_kernel(const double* x, int64_t n, double* out) {
  __shared__ double sm[256];
  double m = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) m = fmax(m, x[i]);
  sm[threadIdx.x] = m;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sm[0];
}

}  // namespace

namespace {

// Knot values and first functions per direction, and the Gauss rule of q
// points, on the device; the tables (and, with ke1/me1, the 1D element
// matrices) at those points.
void basis_tables_at(riga_problem* pr, int q, double* val, double* der, double* ke1, double* me1,
                     double* ge1 = nullptr) {
  const Analysis& an = pr->an;
  const int dim = an.dim, p = an.p, np = p + 1;
  hipStream_t s = pr->stream;
  std::vector<double> kvv;
  std::vector<int> kvoff(3, 0);
  int total_el = 0;
  for (int d = 0; d < dim; ++d) {
    kvoff[d] = (int)kvv.size();
    for (int k : an.sp[d].kv) kvv.push_back((double)k / an.ne[d]);
    total_el += an.ne[d];
  }
  std::vector<double> gx, gw;
  gauss_legendre(q, gx, gw);
  DBuf<double> d_kv, d_gx, d_gw;
  d_kv.upload(kvv, s);
  d_gx.upload(gx, s);
  d_gw.upload(gw, s);
  TabArgs a{};
  for (int d = 0; d < 3; ++d) {
    a.kv[d] = d < dim ? d_kv.p + kvoff[d] : nullptr;
    a.tab_off[d] = pr->tab_off[d];
    a.ne[d] = an.ne[d];
  }
  a.first_fn = pr->first_fn.p;
  a.dim = dim;
  a.p = p;
  a.q = q;
  a.gx = d_gx.p;
  a.gw = d_gw.p;
  a.val = val;
  a.der = der;
  a.ke1 = ke1;
  a.me1 = me1;
  a.ge1 = ge1;
  const int n1 = total_el * q;
  basis_tables_kernel<<<(n1 + 127) / 128, 128, 0, s>>>(a);
  HIPCHECK(hipGetLastError());
  if (ke1) {
    const int n2 = total_el * np * np;
    element_1d_kernel<<<(n2 + 127) / 128, 128, 0, s>>>(a, total_el);
    HIPCHECK(hipGetLastError());
  }
  HIPCHECK(hipStreamSynchronize(s));  // d_kv/d_gx/d_gw are freed on return
}

}  // namespace

void launch_basis_tables(riga_problem* pr) {
  const Analysis& an = pr->an;
  const int dim = an.dim, p = an.p, q = an.nquad, np = p + 1;
  hipStream_t s = pr->stream;
  // first functions and supports per direction
  std::vector<int32_t> ff, fe, le;
  int total_el = 0, total_fn = 0;
  for (int d = 0; d < dim; ++d) {
    pr->tab_off[d] = total_el;
    pr->fn_off[d] = total_fn;
    for (int e = 0; e < an.ne[d]; ++e) ff.push_back(an.sp[d].first_fn[e]);
    for (int i = 0; i < an.sp[d].n; ++i) {
      fe.push_back(an.sp[d].fe[i]);
      le.push_back(an.sp[d].le[i]);
    }
    total_el += an.ne[d];
    total_fn += an.sp[d].n;
  }
  pr->first_fn.upload(ff, s);
  pr->fe.upload(fe, s);
  pr->le.upload(le, s);
  pr->tab_val.alloc((size_t)total_el * q * np, s);
  pr->tab_der.alloc((size_t)total_el * q * np, s);
  pr->ke1.alloc((size_t)total_el * np * np, s);
  pr->me1.alloc((size_t)total_el * np * np, s);
  if (an.components == 2) pr->ge1.alloc((size_t)total_el * np * np, s);
  basis_tables_at(pr, q, pr->tab_val.p, pr->tab_der.p, pr->ke1.p, pr->me1.p,
                  an.components == 2 ? pr->ge1.p : nullptr);
}

void basis_tables_q(riga_problem* pr, int q, DBuf<double>& val, DBuf<double>& der) {
  const Analysis& an = pr->an;
  int total_el = 0;
  for (int d = 0; d < an.dim; ++d) total_el += an.ne[d];
  val.alloc((size_t)total_el * q * (an.p + 1), pr->stream);
  der.alloc((size_t)total_el * q * (an.p + 1), pr->stream);
  basis_tables_at(pr, q, val.p, der.p, nullptr, nullptr);
}

void launch_assemble(riga_problem* pr) {
  const Analysis& an = pr->an;
  AsmArgs a{};
  a.row_ptr = pr->row_ptr.p;
  a.col = pr->col_idx.p;
  a.N = an.N;
  a.nnz = an.row_ptr[an.N];
  for (int d = 0; d < 3; ++d) {
    a.n1[d] = an.n1[d];
    a.ne[d] = an.ne[d];
    a.tab_off[d] = pr->tab_off[d];
    a.fn_off[d] = pr->fn_off[d];
  }
  a.fe = pr->fe.p;
  a.le = pr->le.p;
  a.first_fn = pr->first_fn.p;
  a.ke1 = pr->ke1.p;
  a.me1 = pr->me1.p;
  a.ge1 = pr->ge1.p;
  a.kappa = pr->kappa.p;
  a.rho = pr->rho.p;
  a.dim = an.dim;
  a.p = an.p;
  a.cplx = an.components == 2;
  for (int d = 0; d < 3; ++d) a.A[d] = pr->potential[d];
  a.kv = pr->kv.p;
  a.mv = pr->mv.p;
  const int64_t nb = (a.nnz + 255) / 256;
  assemble_kernel<<<(unsigned)nb, 256, 0, pr->stream>>>(a);
  HIPCHECK(hipGetLastError());
}

void compute_norms(riga_problem* pr) {
  const int64_t N = pr->an.N;
  hipStream_t s = pr->stream;
  DBuf<double> rs, out;
  rs.alloc(N, s);
  out.alloc(2, s);
  row_abs_sum_kernel<<<(unsigned)((N + 255) / 256), 256, 0, s>>>(pr->row_ptr.p, pr->kv.p, N, rs.p);
  max_reduce_kernel<<<1, 256, 0, s>>>(rs.p, N, out.p);
  row_abs_sum_kernel<<<(unsigned)((N + 255) / 256), 256, 0, s>>>(pr->row_ptr.p, pr->mv.p, N, rs.p);
  max_reduce_kernel<<<1, 256, 0, s>>>(rs.p, N, out.p + 1);
  HIPCHECK(hipGetLastError());
  double h[2];
  HIPCHECK(hipMemcpyAsync(h, out.p, sizeof(h), hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  pr->normK1 = h[0];
  pr->normM1 = h[1];
}

}  // namespace riga
