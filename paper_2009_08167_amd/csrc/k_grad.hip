// Adjoint gradient of L = sum_i w_i lambda_i with respect to per-element
// coefficients (an extension; not in arXiv 2009.08167).  For an
// M-normalised simple eigenpair, first-order perturbation of
// K u = lambda M u gives d lambda / d kappa_e = u^T K0_e u and
// d lambda / d rho_e = -lambda u^T M0_e u, with K0_e, M0_e the
// unit-coefficient element matrices -- tensor products of the 1D element
// matrices (Eq. 2Dmatrix restricted to one element).
//
// One thread per element: gathers the (p+1)^d local coefficients of each
// eigenvector (zero at the Dirichlet functions) and evaluates the two
// quadratic forms.  Each output is written once; no atomics.
#include <hip/hip_runtime.h>

#include "problem.h"

namespace riga {
namespace {

constexpr int NPMAX = 7;

struct GradArgs {
  int dim, p;
  int ne[3], n1[3], tab_off[3], nfn[3];
  const int* first_fn;
  const double* ke1;
  const double* me1;
  const double* U;
  int64_t N;
  int k;
  const double* lam;
  const double* w;
  double* gk;
  double* gr;
};

__global__ void __launch_bounds__(128) eig_grad_kernel(GradArgs g) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nel = (int64_t)g.ne[0] * g.ne[1] * g.ne[2];
  if (e >= nel) return;
  const int np = g.p + 1, np2 = np * np;
  int ei[3] = {(int)(e % g.ne[0]), (int)((e / g.ne[0]) % g.ne[1]),
               (int)(e / ((int64_t)g.ne[0] * g.ne[1]))};
  double Kd[3][NPMAX * NPMAX], Md[3][NPMAX * NPMAX];
  int f0[3] = {0, 0, 0};
  for (int d = 0; d < g.dim; ++d) {
    const int64_t o = (int64_t)(g.tab_off[d] + ei[d]) * np2;
    for (int t = 0; t < np2; ++t) {
      Kd[d][t] = g.ke1[o + t];
      Md[d][t] = g.me1[o + t];
    }
    f0[d] = g.first_fn[g.tab_off[d] + ei[d]];
  }
  const int nz = g.dim == 3 ? np : 1;
  double sk = 0.0, sr = 0.0;
  double u[NPMAX * NPMAX * NPMAX];
  for (int i = 0; i < g.k; ++i) {
    const double* ui = g.U + (int64_t)i * g.N;
    // local coefficients u[az][ay][ax]
    for (int az = 0; az < nz; ++az)
      for (int ay = 0; ay < np; ++ay)
        for (int ax = 0; ax < np; ++ax) {
          const int gx = f0[0] + ax, gy = f0[1] + ay, gz = g.dim == 3 ? f0[2] + az : 1;
          const bool in = gx >= 1 && gx <= g.nfn[0] - 2 && gy >= 1 && gy <= g.nfn[1] - 2 &&
                          (g.dim == 2 || (gz >= 1 && gz <= g.nfn[2] - 2));
          double v = 0.0;
          if (in) {
            const int64_t idx = (gx - 1) + (int64_t)g.n1[0] * ((gy - 1) + (int64_t)g.n1[1] * (gz - 1));
            v = ui[idx];
          }
          u[(az * np + ay) * np + ax] = v;
        }
    double qk = 0.0, qm = 0.0;
    if (g.dim == 2) {
      for (int ay = 0; ay < np; ++ay)
        for (int by = 0; by < np; ++by) {
          const double ky = Kd[1][ay * np + by], my = Md[1][ay * np + by];
          for (int ax = 0; ax < np; ++ax) {
            const double ua = u[ay * np + ax];
            double tk = 0.0, tm = 0.0;
            for (int bx = 0; bx < np; ++bx) {
              const double ub = u[by * np + bx];
              tk += Kd[0][ax * np + bx] * ub;
              tm += Md[0][ax * np + bx] * ub;
            }
            qk += ua * (my * tk + ky * tm);
            qm += ua * my * tm;
          }
        }
    } else {
      for (int az = 0; az < np; ++az)
        for (int bz = 0; bz < np; ++bz) {
          const double kz = Kd[2][az * np + bz], mz = Md[2][az * np + bz];
          for (int ay = 0; ay < np; ++ay)
            for (int by = 0; by < np; ++by) {
              const double ky = Kd[1][ay * np + by], my = Md[1][ay * np + by];
              for (int ax = 0; ax < np; ++ax) {
                const double ua = u[(az * np + ay) * np + ax];
                double tk = 0.0, tm = 0.0;
                for (int bx = 0; bx < np; ++bx) {
                  const double ub = u[(bz * np + by) * np + bx];
                  tk += Kd[0][ax * np + bx] * ub;
                  tm += Md[0][ax * np + bx] * ub;
                }
                qk += ua * (mz * my * tk + mz * ky * tm + kz * my * tm);
                qm += ua * mz * my * tm;
              }
            }
        }
    }
    sk += g.w[i] * qk;
    sr -= g.w[i] * g.lam[i] * qm;
  }
  g.gk[e] = sk;
  g.gr[e] = sr;
}

}  // namespace

void launch_eig_grad(const riga_problem* pr, int k, const double* U, const double* lam_dev,
                     const double* w_dev, double* gk, double* gr, hipStream_t s) {
  const Analysis& an = pr->an;
  GradArgs g{};
  g.dim = an.dim;
  g.p = an.p;
  for (int d = 0; d < 3; ++d) {
    g.ne[d] = an.ne[d];
    g.n1[d] = an.n1[d];
    g.tab_off[d] = pr->tab_off[d];
    g.nfn[d] = d < an.dim ? an.sp[d].n : 3;
  }
  g.first_fn = pr->first_fn.p;
  g.ke1 = pr->ke1.p;
  g.me1 = pr->me1.p;
  g.U = U;
  g.N = an.N;
  g.k = k;
  g.lam = lam_dev;
  g.w = w_dev;
  g.gk = gk;
  g.gr = gr;
  const int64_t nel = an.n_elem;
  eig_grad_kernel<<<(unsigned)((nel + 127) / 128), 128, 0, s>>>(g);
  HIPCHECK(hipGetLastError());
}

}  // namespace riga
