// Host-side analysis of a tensor-product B-spline discretisation: knot
// vectors and DOF maps (Sec. 3.1--3.2 of arXiv 2009.08167), the sparsity
// pattern of K and M, the tree of separators and the supernodal symbolic
// factorisation that every shift reuses (Sec. 5: one symbolic factorisation
// per pattern, one numeric factorisation per shift).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace riga {

// Leading dimension of a front's partitioned-inverse block: the order rounded
// up to 32 elements, so that every column starts on a 128-byte boundary.
inline int h_ld(int f) { return (f + 31) & ~31; }


// One direction of the tensor-product space.  Knot positions are kept as
// integer element-boundary indices (knot value = index / ne), so that the
// support of every function is an exact element range.
struct Space1D {
  int ne = 0, p = 0, s = 0;
  std::vector<int> kv;       // open knot vector, element-boundary units
  int n = 0;                 // functions, boundary ones included (n = len(kv) - p - 1)
  std::vector<int> first_fn; // [ne]  global index of the first function non-zero on element e
  std::vector<int> fe, le;   // [n]   first / last element of the support of function i
  std::vector<int> mult;     // [ne+1] multiplicity of each element boundary
  // interior functions j = 0..n-3 are the global functions j+1
  std::vector<int> nb_lo, nb_hi;  // [n-2] interior neighbours (share an element), inclusive
  int n_int() const { return n - 2; }
};

Space1D make_space(int ne, int p, int s);

// Gauss--Legendre rule on [-1, 1] (Newton iteration on P_q).
void gauss_legendre(int q, std::vector<double>& x, std::vector<double>& w);

struct Analysis {
  int dim = 0;
  int p = 0, s = 0, nquad = 0;
  Space1D sp[3];
  int n1[3] = {1, 1, 1};     // interior functions per direction
  int ne[3] = {1, 1, 1};
  int64_t N = 0;             // unknowns: interior DOFs, twice that for a complex pencil
  int64_t n_elem = 0;
  int components = 1;        // 1: real pencil; 2: complex Hermitian pencil in real-equivalent
                             // form (unknowns 2d, 2d + 1 = real, imaginary part of DOF d)

  // CSR pattern of K and M in original (lexicographic, x fastest) order.
  std::vector<int64_t> row_ptr;
  std::vector<int32_t> col_idx;

  // Elimination order.
  std::vector<int32_t> perm;   // original -> new
  std::vector<int32_t> iperm;  // new -> original

  // Separator tree in post-order (children before parents).
  int n_fronts = 0;
  std::vector<int32_t> f_start;   // first new index of the node's variables
  std::vector<int32_t> f_k;       // fully-summed (own) variables
  std::vector<int32_t> f_f;       // front order = k + |structure|
  std::vector<int32_t> f_parent;  // -1 for roots
  std::vector<int32_t> f_height;  // 0 for leaves
  std::vector<int64_t> f_rows_off;   // offset into rows[] (sum f)
  std::vector<int32_t> rows;          // front index lists, ORIGINAL DOF indices
  std::vector<int64_t> f_pool_off;   // offset of the dense f x f front in the pool
  std::vector<int64_t> f_cb_off;     // offset of the contribution vector (sum of f-k)
  std::vector<int64_t> f_h_off;      // offset of the h_ld(f) x k partitioned inverse
  int64_t pool_size = 0;             // sum f^2
  int64_t h_size = 0;                // sum f k
  int64_t cb_size = 0;               // sum (f-k)
  // Children, and for each (parent, child) pair the map from parent front
  // position to child contribution-block position (-1 if none).
  std::vector<int32_t> child_ptr;    // [n_fronts+1]
  std::vector<int32_t> child_list;
  std::vector<int64_t> inv_off;      // [child_list.size()] offset into inv[]
  std::vector<int32_t> inv;
  // Original-matrix entries of each fully-summed column, by new column
  // index: (front row position, CSR value index), rows >= the column.
  std::vector<int64_t> amap_ptr;     // [N+1]
  std::vector<int32_t> amap_row;
  std::vector<int32_t> amap_val;

  int height = 0;                    // number of levels
  std::vector<std::vector<int32_t>> levels;  // fronts by height
  int max_front = 0, max_fs = 0;
  int64_t nnz_l = 0;                 // lower factor entries, diagonal included
  double flops_fact = 0.0;
  // exact fill of the same elimination order (no pivoting): the entries of
  // L, diagonal included, and sum over columns of c (c + 1), c = column
  // count below the diagonal; the supernodal counts above treat every
  // fully-summed block as dense
  int64_t nnz_l_exact = 0;
  double flops_exact = 0.0;
};

// Builds everything above.  Returns "" on success, else an error message.
std::string analyze(int dim, const int ne[3], int p, int s, int nquad, int leaf_dofs,
                    Analysis& out, int components = 1);

}  // namespace riga
