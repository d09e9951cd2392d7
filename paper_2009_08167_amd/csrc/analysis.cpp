// Host-side analysis: knot vectors and DOF maps, sparsity pattern, tree of
// separators, supernodal symbolic factorisation.  See analysis.h.
#include "analysis.h"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <functional>
#include <numeric>

namespace riga {

Space1D make_space(int ne, int p, int s) {
  // Open knot vector (Eq. U): p+1 end knots, simple interior knots; rIGA
  // (Sec. 3.2) raises the multiplicity of every s-th interior knot to p.
  Space1D sp;
  sp.ne = ne;
  sp.p = p;
  sp.s = s;
  for (int i = 0; i <= p; ++i) sp.kv.push_back(0);
  for (int k = 1; k < ne; ++k) {
    int m = (s > 0 && k % s == 0) ? p : 1;
    for (int i = 0; i < m; ++i) sp.kv.push_back(k);
  }
  for (int i = 0; i <= p; ++i) sp.kv.push_back(ne);
  sp.n = (int)sp.kv.size() - p - 1;
  sp.mult.assign(ne + 1, 0);
  for (int k : sp.kv) sp.mult[k]++;
  // Support of B_{i,p} is [xi_i, xi_{i+p+1}]: elements kv[i] .. kv[i+p+1]-1.
  sp.fe.resize(sp.n);
  sp.le.resize(sp.n);
  for (int i = 0; i < sp.n; ++i) {
    sp.fe[i] = sp.kv[i];
    sp.le[i] = sp.kv[i + p + 1] - 1;
  }
  // Element e lies in the knot span whose left knot is the last copy of e;
  // the p+1 functions span-p .. span are non-zero on it.
  sp.first_fn.resize(ne);
  for (int e = 0; e < ne; ++e) {
    int span = (int)(std::upper_bound(sp.kv.begin(), sp.kv.end(), e) - sp.kv.begin()) - 1;
    sp.first_fn[e] = span - p;
  }
  // Interior neighbours: functions sharing at least one element.
  int ni = sp.n - 2;
  sp.nb_lo.resize(std::max(ni, 0));
  sp.nb_hi.resize(std::max(ni, 0));
  for (int j = 0; j < ni; ++j) {
    int g = j + 1;
    int lo = g, hi = g;
    while (lo - 1 >= 1 && sp.le[lo - 1] >= sp.fe[g]) --lo;
    while (hi + 1 <= sp.n - 2 && sp.fe[hi + 1] <= sp.le[g]) ++hi;
    sp.nb_lo[j] = lo - 1;
    sp.nb_hi[j] = hi - 1;
  }
  return sp;
}

void gauss_legendre(int q, std::vector<double>& x, std::vector<double>& w) {
  x.assign(q, 0.0);
  w.assign(q, 0.0);
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < q; ++i) {
    double t = std::cos(pi * (i + 0.75) / (q + 0.5));  // Chebyshev-like initial guess
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = t;
      for (int k = 2; k <= q; ++k) {
        double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (q == 1) { p1 = t; p0 = 1.0; }
      double dp = q * (t * p1 - p0) / (t * t - 1.0);
      double dt = p1 / dp;
      t -= dt;
      if (std::fabs(dt) < 1e-16) {
        // final derivative at the converged node for the weight
        double a0 = 1.0, a1 = t;
        for (int k = 2; k <= q; ++k) {
          double a2 = ((2.0 * k - 1.0) * t * a1 - (k - 1.0) * a0) / k;
          a0 = a1;
          a1 = a2;
        }
        if (q == 1) { a1 = t; a0 = 1.0; }
        dp = q * (t * a1 - a0) / (t * t - 1.0);
        w[i] = 2.0 / ((1.0 - t * t) * dp * dp);
        break;
      }
    }
    x[i] = t;
  }
  // ascending order
  std::vector<int> o(q);
  std::iota(o.begin(), o.end(), 0);
  std::sort(o.begin(), o.end(), [&](int a, int b) { return x[a] < x[b]; });
  std::vector<double> xs(q), ws(q);
  for (int i = 0; i < q; ++i) { xs[i] = x[o[i]]; ws[i] = w[o[i]]; }
  x = xs;
  w = ws;
}

namespace {

struct Box {
  int a[3], b[3];    // interior DOF index range per direction
  int e0[3], e1[3];  // element range per direction
};

struct NodeTmp {
  Box slab;                   // the node's own variables
  std::vector<int> children;
};

// Largest fully-summed block of one front; larger separators are split into
// chains.  288 is the largest block whose panels get the full 64 columns
// (the panel kernel's LDS holds 18,432 doubles of remaining rows x panel
// columns).  RIGA_SPLIT_FS overrides (0: no splitting).
constexpr int SPLIT_FS = 288;
int split_fs() {
  if (const char* v = std::getenv("RIGA_SPLIT_FS"))
    if (*v) return std::max(0, std::atoi(v));
  return SPLIT_FS;
}

}  // namespace

std::string analyze(int dim, const int ne_in[3], int p, int s, int nquad, int leaf_dofs,
                    Analysis& A, int components) {
  if (components != 1 && components != 2) return "components must be 1 or 2";
  if (dim < 2 || dim > 3) return "dim must be 2 or 3";
  if (p < 1 || p > 6) return "p must be in 1..6";
  if (s < 0) return "sep_spacing must be >= 0";
  for (int d = 0; d < dim; ++d)
    if (ne_in[d] < 1 || ne_in[d] > 1 << 16) return "ne must be in 1..65536";
  A = Analysis();
  A.dim = dim;
  A.p = p;
  A.s = s;
  A.nquad = nquad > 0 ? nquad : p + 1;
  if (A.nquad > 16) return "nquad must be <= 16";
  // (a complex pencil doubles every front: half the scalar leaf by default,
  // so that its leaf fronts stay within the LDS-resident size)
  if (leaf_dofs <= 0) leaf_dofs = components == 2 ? 32 : 64;
  A.N = 1;
  A.n_elem = 1;
  for (int d = 0; d < 3; ++d) {
    A.ne[d] = d < dim ? ne_in[d] : 1;
    if (d < dim) {
      A.sp[d] = make_space(A.ne[d], p, s);
      A.n1[d] = A.sp[d].n_int();
      if (A.n1[d] < 1) return "mesh has no interior functions";
    } else {
      A.n1[d] = 1;
    }
    A.N *= A.n1[d];
    A.n_elem *= A.ne[d];
  }
  if (A.N * components >= (int64_t)1 << 31) return "too many DOFs";
  int64_t N = A.N;
  const int nx = A.n1[0], ny = A.n1[1], nz = A.n1[2];

  // ---- CSR pattern: row (i,j,k) couples with the tensor product of the
  // 1D neighbour ranges, columns ascending (x fastest).
  A.row_ptr.assign(N + 1, 0);
  for (int64_t r = 0; r < N; ++r) {
    int i = r % nx, j = (r / nx) % ny, k = (int)(r / ((int64_t)nx * ny));
    int64_t c = 1;
    int idx[3] = {i, j, k};
    for (int d = 0; d < dim; ++d) c *= A.sp[d].nb_hi[idx[d]] - A.sp[d].nb_lo[idx[d]] + 1;
    A.row_ptr[r + 1] = A.row_ptr[r] + c;
  }
  if (A.row_ptr[N] * components * components >= (int64_t)1 << 31) return "too many non-zeros";
  A.col_idx.resize(A.row_ptr[N]);
  for (int64_t r = 0; r < N; ++r) {
    int idx[3] = {(int)(r % nx), (int)((r / nx) % ny), (int)(r / ((int64_t)nx * ny))};
    int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int d = 0; d < dim; ++d) {
      lo[d] = A.sp[d].nb_lo[idx[d]];
      hi[d] = A.sp[d].nb_hi[idx[d]];
    }
    int64_t o = A.row_ptr[r];
    for (int c2 = lo[2]; c2 <= hi[2]; ++c2)
      for (int c1 = lo[1]; c1 <= hi[1]; ++c1)
        for (int c0 = lo[0]; c0 <= hi[0]; ++c0)
          A.col_idx[o++] = (int32_t)(c0 + (int64_t)nx * (c1 + (int64_t)ny * c2));
  }

  // ---- Tree of separators: recursive bisection of the element box along
  // its longest direction.  A cut at element boundary c removes the
  // functions whose support straddles c (p + 1 - mult(c) of them per line):
  // one layer at a C^0 knot of rIGA, p layers at a simple knot.  The C^0
  // knot nearest the middle is preferred when one lies in the middle half.
  std::vector<NodeTmp> nodes;
  auto box_count = [&](const Box& b) {
    int64_t c = 1;
    for (int d = 0; d < 3; ++d) c *= std::max(0, b.b[d] - b.a[d]);
    return c;
  };
  std::function<std::vector<int>(const Box&)> build = [&](const Box& bx) -> std::vector<int> {
    int64_t cnt = box_count(bx);
    if (cnt == 0) return {};
    int cut_dim = -1, best = 1;
    if (cnt > leaf_dofs) {
      for (int d = 0; d < dim; ++d) {
        int w = bx.e1[d] - bx.e0[d];
        if (w >= 2 && bx.b[d] > bx.a[d] && w > best) {
          best = w;
          cut_dim = d;
        }
      }
    }
    if (cut_dim < 0) {
      NodeTmp nd;
      nd.slab = bx;
      nodes.push_back(nd);
      return {(int)nodes.size() - 1};
    }
    const int d = cut_dim;
    const Space1D& S = A.sp[d];
    int e0 = bx.e0[d], e1 = bx.e1[d], w = e1 - e0;
    int mid = e0 + w / 2;
    int c = mid;
    int bestdist = 1 << 30;
    for (int cc = e0 + 1; cc < e1; ++cc) {
      if (S.mult[cc] == p && cc >= e0 + w / 4 && cc <= e1 - w / 4) {
        int dist = std::abs(2 * cc - (e0 + e1));
        if (dist < bestdist) {
          bestdist = dist;
          c = cc;
        }
      }
    }
    // separator: interior functions in [a, b) whose support straddles c.
    // fe and le are non-decreasing, so the straddlers are the contiguous
    // range between the functions ending before c and those starting at c.
    int sa = bx.a[d];
    while (sa < bx.b[d] && S.le[sa + 1] < c) ++sa;
    int sb = sa;
    while (sb < bx.b[d] && S.fe[sb + 1] < c) ++sb;
    Box L = bx, R = bx, sep = bx;
    L.b[d] = sa;
    L.e1[d] = c;
    R.a[d] = sb;
    R.e0[d] = c;
    sep.a[d] = sa;
    sep.b[d] = sb;
    std::vector<int> lc = build(L);
    std::vector<int> rc = build(R);
    std::vector<int> ch = lc;
    ch.insert(ch.end(), rc.begin(), rc.end());
    if (box_count(sep) == 0) return ch;
    NodeTmp nd;
    nd.slab = sep;
    nd.children = ch;
    nodes.push_back(nd);
    return {(int)nodes.size() - 1};
  };
  Box root;
  for (int d = 0; d < 3; ++d) {
    root.a[d] = 0;
    root.b[d] = A.n1[d];
    root.e0[d] = 0;
    root.e1[d] = A.ne[d];
  }
  std::vector<int> roots = build(root);
  int nf = (int)nodes.size();
  A.n_fronts = nf;

  // ---- Elimination order: nodes are created in post-order; each node's
  // variables take the next new indices, lexicographic (x fastest) inside.
  A.perm.assign(N, -1);
  A.iperm.assign(N, -1);
  A.f_start.resize(nf);
  A.f_k.resize(nf);
  A.f_parent.assign(nf, -1);
  A.f_height.assign(nf, 0);
  int32_t next = 0;
  for (int f = 0; f < nf; ++f) {
    const Box& b = nodes[f].slab;
    A.f_start[f] = next;
    for (int k = b.a[2]; k < b.b[2]; ++k)
      for (int j = b.a[1]; j < b.b[1]; ++j)
        for (int i = b.a[0]; i < b.b[0]; ++i) {
          int64_t o = i + (int64_t)nx * (j + (int64_t)ny * k);
          if (A.perm[o] != -1) return "internal: DOF in two separators";
          A.perm[o] = next;
          A.iperm[next] = (int32_t)o;
          ++next;
        }
    A.f_k[f] = next - A.f_start[f];
    for (int c : nodes[f].children) {
      if (c >= f) return "internal: tree not in post-order";
      A.f_parent[c] = f;
    }
  }
  if (next != N) return "internal: DOFs not covered by the tree";
  (void)roots;
  A.child_ptr.assign(nf + 1, 0);
  for (int f = 0; f < nf; ++f) A.child_ptr[f + 1] = A.child_ptr[f] + (int)nodes[f].children.size();
  A.child_list.clear();
  for (int f = 0; f < nf; ++f)
    for (int c : nodes[f].children) A.child_list.push_back(c);
  for (int f = 0; f < nf; ++f) {
    int h = 0;
    for (int c : nodes[f].children) h = std::max(h, A.f_height[c] + 1);
    A.f_height[f] = h;
  }

  // ---- Supernode splitting: a separator with more than `split` variables
  // becomes a chain of fronts of at most `split` each, in the same
  // elimination order (same fill, same flops).  The panel kernel holds a
  // front's remaining fully-summed rows of its panel columns in LDS, so a
  // smaller fully-summed block allows wider panels, and the trailing
  // updates become dense rank-(panel width) contractions instead of
  // streaming the update block through HBM a few columns at a time.
  // (in scalar DOFs: a complex pencil doubles every block below)
  const int split = split_fs() / components;
  if (split > 0) {
    int nn = 0;
    std::vector<int> first_new(A.n_fronts), nchunk(A.n_fronts);
    for (int f = 0; f < A.n_fronts; ++f) {
      nchunk[f] = std::max(1, (A.f_k[f] + split - 1) / split);
      first_new[f] = nn;
      nn += nchunk[f];
    }
    if (nn != A.n_fronts) {
      std::vector<int32_t> start(nn), kk(nn), parent(nn, -1);
      std::vector<std::vector<int>> kids(nn);
      for (int f = 0; f < A.n_fronts; ++f) {
        for (int c = 0; c < nchunk[f]; ++c) {
          const int i = first_new[f] + c;
          start[i] = A.f_start[f] + c * split;
          kk[i] = std::min(split, A.f_k[f] - c * split);
          if (c + 1 < nchunk[f]) {
            parent[i] = i + 1;
            kids[i + 1].push_back(i);
          }
        }
        const int last = first_new[f] + nchunk[f] - 1;
        if (A.f_parent[f] >= 0) {
          parent[last] = first_new[A.f_parent[f]];
          kids[first_new[A.f_parent[f]]].push_back(last);
        }
      }
      A.n_fronts = nn;
      A.f_start = start;
      A.f_k = kk;
      A.f_parent = parent;
      A.child_ptr.assign(nn + 1, 0);
      A.child_list.clear();
      for (int i = 0; i < nn; ++i) {
        std::sort(kids[i].begin(), kids[i].end());
        A.child_ptr[i + 1] = A.child_ptr[i] + (int)kids[i].size();
        for (int c : kids[i]) {
          if (c >= i) return "internal: split tree not in post-order";
          A.child_list.push_back(c);
        }
      }
      A.f_height.assign(nn, 0);
      for (int i = 0; i < nn; ++i) {
        int h = 0;
        for (int ci = A.child_ptr[i]; ci < A.child_ptr[i + 1]; ++ci)
          h = std::max(h, A.f_height[A.child_list[ci]] + 1);
        A.f_height[i] = h;
      }
    }
  }
  nf = A.n_fronts;

  // ---- A complex Hermitian pencil K + iK' (M real) is solved in its
  // real-equivalent form [[K, -K'], [K', K]], diag(M, M): every scalar DOF d
  // becomes the two variables 2d (real part) and 2d + 1 (imaginary part),
  // adjacent in the pattern, in the elimination order and in every front,
  // and every scalar coupling becomes a 2 x 2 block.  The tree is the
  // scalar one; everything below is built for the expanded variables.
  A.components = components;
  if (components == 2) {
    const int64_t Ns = N;
    std::vector<int64_t> rp(2 * Ns + 1, 0);
    std::vector<int32_t> ci;
    ci.reserve(4 * A.col_idx.size());
    for (int64_t r = 0; r < Ns; ++r) {
      const int64_t len = A.row_ptr[r + 1] - A.row_ptr[r];
      for (int t = 0; t < 2; ++t) {
        rp[2 * r + t + 1] = rp[2 * r + t] + 2 * len;
        for (int64_t e = A.row_ptr[r]; e < A.row_ptr[r + 1]; ++e) {
          ci.push_back(2 * A.col_idx[e]);
          ci.push_back(2 * A.col_idx[e] + 1);
        }
      }
    }
    A.row_ptr.swap(rp);
    A.col_idx.swap(ci);
    std::vector<int32_t> perm2(2 * Ns), iperm2(2 * Ns);
    for (int64_t d = 0; d < Ns; ++d)
      for (int t = 0; t < 2; ++t) {
        perm2[2 * d + t] = 2 * A.perm[d] + t;
        iperm2[2 * (int64_t)A.perm[d] + t] = (int32_t)(2 * d + t);
      }
    A.perm.swap(perm2);
    A.iperm.swap(iperm2);
    for (int f = 0; f < nf; ++f) {
      A.f_start[f] *= 2;
      A.f_k[f] *= 2;
    }
    A.N = N = 2 * Ns;
  }

  // ---- Supernodal symbolic factorisation.  struct(P) = the variables
  // eliminated after P that are adjacent to P's variables or in a child's
  // structure.  Front = P's variables followed by struct(P) ascending.
  std::vector<std::vector<int32_t>> st(nf);
  std::vector<int32_t> mark(N, -1);
  for (int f = 0; f < nf; ++f) {
    const int32_t beg = A.f_start[f], end = beg + A.f_k[f];
    std::vector<int32_t>& S = st[f];
    for (int32_t g = beg; g < end; ++g) {
      int32_t o = A.iperm[g];
      for (int64_t e = A.row_ptr[o]; e < A.row_ptr[o + 1]; ++e) {
        int32_t g2 = A.perm[A.col_idx[e]];
        if (g2 >= end && mark[g2] != f) {
          mark[g2] = f;
          S.push_back(g2);
        }
      }
    }
    for (int ci = A.child_ptr[f]; ci < A.child_ptr[f + 1]; ++ci) {
      for (int32_t g2 : st[A.child_list[ci]]) {
        if (g2 >= end && mark[g2] != f) {
          mark[g2] = f;
          S.push_back(g2);
        }
      }
    }
    std::sort(S.begin(), S.end());
  }
  A.f_f.resize(nf);
  A.f_rows_off.resize(nf + 1);
  A.f_pool_off.resize(nf + 1);
  A.f_cb_off.resize(nf + 1);
  A.f_h_off.resize(nf + 1);
  A.f_rows_off[0] = A.f_pool_off[0] = A.f_cb_off[0] = A.f_h_off[0] = 0;
  A.nnz_l = 0;
  A.flops_fact = 0.0;
  A.max_front = A.max_fs = 0;
  for (int f = 0; f < nf; ++f) {
    int k = A.f_k[f], fo = k + (int)st[f].size();
    A.f_f[f] = fo;
    A.f_rows_off[f + 1] = A.f_rows_off[f] + fo;
    A.f_pool_off[f + 1] = A.f_pool_off[f] + (int64_t)fo * fo;
    A.f_cb_off[f + 1] = A.f_cb_off[f] + (fo - k);
    A.f_h_off[f + 1] = A.f_h_off[f] + (int64_t)h_ld(fo) * k;
    A.max_front = std::max(A.max_front, fo);
    A.max_fs = std::max(A.max_fs, k);
    A.nnz_l += (int64_t)k * (k + 1) / 2 + (int64_t)k * (fo - k);
    for (int j = 0; j < k; ++j) {
      double c = fo - j - 1;
      A.flops_fact += c * (c + 1.0);
    }
  }
  A.pool_size = A.f_pool_off[nf];
  A.cb_size = A.f_cb_off[nf];
  A.h_size = A.f_h_off[nf];
  A.rows.resize(A.f_rows_off[nf]);
  for (int f = 0; f < nf; ++f) {
    int64_t o = A.f_rows_off[f];
    for (int t = 0; t < A.f_k[f]; ++t) A.rows[o + t] = A.iperm[A.f_start[f] + t];
    for (size_t c = 0; c < st[f].size(); ++c) A.rows[o + A.f_k[f] + c] = A.iperm[st[f][c]];
  }

  // ---- Parent-position -> child contribution-block maps.
  std::vector<int32_t> pos(N, -1);
  A.inv_off.assign(A.child_list.size() + 1, 0);
  for (int f = 0; f < nf; ++f)
    for (int ci = A.child_ptr[f]; ci < A.child_ptr[f + 1]; ++ci)
      A.inv_off[ci + 1] = A.inv_off[ci] + A.f_f[f];
  A.inv.assign(A.inv_off[A.child_list.size()], -1);
  for (int f = 0; f < nf; ++f) {
    const int k = A.f_k[f];
    for (int t = 0; t < k; ++t) pos[A.f_start[f] + t] = t;
    for (size_t c = 0; c < st[f].size(); ++c) pos[st[f][c]] = k + (int)c;
    for (int ci = A.child_ptr[f]; ci < A.child_ptr[f + 1]; ++ci) {
      int ch = A.child_list[ci];
      const std::vector<int32_t>& S = st[ch];
      for (size_t c = 0; c < S.size(); ++c) {
        int32_t g = S[c];
        bool in_front = (g >= A.f_start[f] && g < A.f_start[f] + k) ||
                        std::binary_search(st[f].begin(), st[f].end(), g);
        if (!in_front) return "internal: child structure not inside parent front";
        A.inv[A.inv_off[ci] + pos[g]] = (int32_t)c;
      }
    }
  }
  A.amap_ptr.assign(N + 1, 0);
  // first pass: counts
  for (int f = 0; f < nf; ++f) {
    for (int t = 0; t < A.f_k[f]; ++t) {
      int32_t g = A.f_start[f] + t, o = A.iperm[g];
      int64_t c = 0;
      for (int64_t e = A.row_ptr[o]; e < A.row_ptr[o + 1]; ++e)
        if (A.perm[A.col_idx[e]] >= g) ++c;
      A.amap_ptr[g + 1] = c;
    }
  }
  for (int64_t g = 0; g < N; ++g) A.amap_ptr[g + 1] += A.amap_ptr[g];
  A.amap_row.resize(A.amap_ptr[N]);
  A.amap_val.resize(A.amap_ptr[N]);
  for (int f = 0; f < nf; ++f) {
    const int k = A.f_k[f];
    for (int t = 0; t < k; ++t) pos[A.f_start[f] + t] = t;
    for (size_t c = 0; c < st[f].size(); ++c) pos[st[f][c]] = k + (int)c;
    for (int t = 0; t < k; ++t) {
      int32_t g = A.f_start[f] + t, o = A.iperm[g];
      int64_t w = A.amap_ptr[g];
      for (int64_t e = A.row_ptr[o]; e < A.row_ptr[o + 1]; ++e) {
        int32_t g2 = A.perm[A.col_idx[e]];
        if (g2 >= g) {
          bool own = g2 < A.f_start[f] + k;
          if (!own && !std::binary_search(st[f].begin(), st[f].end(), g2))
            return "internal: matrix entry outside its front";
          A.amap_row[w] = pos[g2];
          A.amap_val[w] = (int32_t)e;
          ++w;
        }
      }
    }
  }

  // ---- Exact fill of the elimination order: the elimination tree of the
  // permuted pattern (ancestors with path compression), then the non-zeros
  // of each row of L as its row subtree, the union of the tree paths from
  // the row's entries left of the diagonal up to the row itself.
  {
    std::vector<int32_t> eparent(N, -1), anc(N, -1), mark(N, -1);
    for (int64_t i = 0; i < N; ++i) {
      const int32_t o = A.iperm[i];
      for (int64_t e = A.row_ptr[o]; e < A.row_ptr[o + 1]; ++e) {
        int32_t r = A.perm[A.col_idx[e]];
        if (r >= i) continue;
        while (anc[r] != -1 && anc[r] != i) {
          const int32_t nx = anc[r];
          anc[r] = (int32_t)i;
          r = nx;
        }
        if (anc[r] == -1) {
          anc[r] = (int32_t)i;
          eparent[r] = (int32_t)i;
        }
      }
    }
    std::vector<int64_t> colcnt(N, 0);
    int64_t below = 0;
    for (int64_t i = 0; i < N; ++i) {
      mark[i] = (int32_t)i;
      const int32_t o = A.iperm[i];
      for (int64_t e = A.row_ptr[o]; e < A.row_ptr[o + 1]; ++e) {
        for (int32_t k = A.perm[A.col_idx[e]]; k < i && mark[k] != i; k = eparent[k]) {
          mark[k] = (int32_t)i;
          ++colcnt[k];
          ++below;
        }
      }
    }
    A.nnz_l_exact = below + N;
    A.flops_exact = 0.0;
    for (int64_t k = 0; k < N; ++k) A.flops_exact += (double)colcnt[k] * (double)(colcnt[k] + 1);
  }

  // ---- Levels by height.
  A.height = 0;
  for (int f = 0; f < nf; ++f) A.height = std::max(A.height, A.f_height[f] + 1);
  A.levels.assign(A.height, {});
  for (int f = 0; f < nf; ++f) A.levels[A.f_height[f]].push_back(f);
  return "";
}

}  // namespace riga
