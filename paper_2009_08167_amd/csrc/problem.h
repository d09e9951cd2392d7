// Internal state of a riga_problem and the launchers of the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/riga.h"
#include "analysis.h"

namespace riga {

// Error carrying a riga_status; converted to a return code at the ABI.
struct Error : std::runtime_error {
  riga_status code;
  Error(riga_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

void hip_check(hipError_t e, const char* what);
#define RIGA_STR2(x) #x
#define RIGA_STR(x) RIGA_STR2(x)
#define HIPCHECK(x) ::riga::hip_check((x), __FILE__ ":" RIGA_STR(__LINE__) ": " #x)

// Device allocation through the optional allocator hook.  The release
// function of the allocator that made an allocation (none: hipFree) travels
// with it, so replacing the hook never frees a buffer through another one.
struct Release {
  void* ctx = nullptr;
  void (*free)(void* ctx, void* ptr, void* stream) = nullptr;
};
void* dmalloc(size_t bytes, hipStream_t s, Release* how);
void dfree(void* p, hipStream_t s, const Release& how);

template <class T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;
  hipStream_t s = nullptr;
  Release how;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept : p(o.p), n(o.n), s(o.s), how(o.how) { o.p = nullptr; o.n = 0; }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) {
      reset();
      p = o.p; n = o.n; s = o.s; how = o.how;
      o.p = nullptr; o.n = 0;
    }
    return *this;
  }
  ~DBuf() { reset(); }
  void alloc(size_t count, hipStream_t st) {
    reset();
    s = st;
    if (count) p = (T*)dmalloc(count * sizeof(T), st, &how);
    n = count;
  }
  void reset() {
    if (p) dfree(p, s, how);
    p = nullptr;
    n = 0;
  }
  void upload(const std::vector<T>& v, hipStream_t st) {
    alloc(v.size(), st);
    if (!v.empty()) HIPCHECK(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
  }
};

// Front columns assembled per workgroup (one wave each), at most; fewer
// where ASM_COLS columns of the level's largest front exceed ASM_LDS bytes.
constexpr int ASM_COLS = 8;
constexpr int ASM_LDS = 150 * 1024;

// Fronts at or below this order are factorised in LDS by one workgroup.
constexpr int LDS_FRONT_MAX_F64 = 128;
constexpr int LDS_FRONT_MAX_F32 = 176;

// Packed per-front record read once by the inverse and solve kernels.
struct FrontDesc {
  int32_t f, k, start, ldh;  // ldh: leading dimension of the front's H block
  int64_t pool_off;  // front in the factor pool (f x f, column-major)
  int64_t h_off;     // partitioned inverse in the H pool (f x k, column-major)
  int64_t rows_off, cb_off, gmap_off;
};

// Rows per forward-sweep work unit and columns per backward-sweep unit;
// the thin shapes serve tree levels with few fronts (more workgroups and
// more loads in flight per row or column).
constexpr int SWEEP_ROWS = 64;
constexpr int SWEEP_COLS = 16;
constexpr int SWEEP_ROWS_THIN = 16;
constexpr int SWEEP_COLS_THIN = 4;
constexpr int SWEEP_THIN_BELOW = 512;  // units of the default shape
constexpr int XCD_PIECE = 16;          // sweep units of one front kept on one XCD
constexpr int XCDS = 8;                // accelerator complex dies of an MI355X
// Fused sweeps of the bottom heights (one workgroup per subtree): four
// 256-thread groups, forward units of SUB_ROWS rows, backward units of
// SUB_COLS columns (8 per wave).
constexpr int SUB_GROUPS = 4;
constexpr int SUB_ROWS = 64;
constexpr int SUB_COLS = 32;

// One workgroup's share of a front: rows [lo, hi) (forward sweep, inverse)
// or columns [lo, hi) (backward sweep), with the front's record inlined so a
// sweep workgroup starts from a single scalar load.
struct WorkUnit {
  int32_t front, lo, hi, f;
  int32_t k, start, ldh, pad;
  int64_t h_off, rows_off, cb_off, gmap_off;
};

// The bottom heights 0..nh-1 swept in one launch per direction: subtree
// `s` (its root at height < nh, its parent at height >= nh or none) has the
// units of its fronts at height h in [off[s (nh + 1) + h], off[s (nh + 1) +
// h + 1]) of fwd_units / bwd_units.  Its fronts are consecutive in the
// post-order, so their pivots and update-vector entries are two ranges.
struct SubInfo {
  int32_t p0, np;    // pivots [p0, p0 + np)
  int32_t cb0, ncb;  // update-vector entries [cb0, cb0 + ncb)
};

struct SubtreeDev {
  int nh = 0;                 // fused heights; 0: none
  int n_sub = 0;
  int max_units = 0;          // units of one subtree, either direction
  int max_np = 0, max_ncb = 0;
  int grp_fwd = 0, grp_bwd = 0;  // doubles of LDS per 256-thread group
  size_t lds_fwd = 0, lds_bwd = 0;  // bytes of LDS per workgroup
  DBuf<WorkUnit> fwd_units, bwd_units;
  DBuf<int32_t> fwd_off, bwd_off;
  DBuf<SubInfo> info;
};

struct LevelDev {
  int n = 0;                 // fronts at this height
  int64_t cols = 0;          // assembly workgroups: sum of ceil(f / asm_cols)
  int asm_cols = 1;          // columns per assembly workgroup
  int max_f = 0, max_k = 0;
  std::vector<int> host_f;   // front orders, ascending (same order as `fronts`)
  std::vector<int> host_k;   // their fully-summed orders
  DBuf<int32_t> fronts;      // front ids sorted by order
  DBuf<int64_t> col_prefix;  // [n+1] prefix sums of ceil(f / asm_cols)
  DBuf<WorkUnit> fwd_units;  // forward sweep: row blocks of this level's fronts
  DBuf<WorkUnit> bwd_units;  // backward sweep: column blocks
  int n_fwd = 0, n_bwd = 0;
  bool fwd_thin = false, bwd_thin = false;
  int n_upto(int fmax) const {  // fronts of order <= fmax (a prefix)
    return (int)(std::upper_bound(host_f.begin(), host_f.end(), fmax) - host_f.begin());
  }
};

// ---- explicit inverse of the top of the separator tree ----
// The fronts at heights >= cut (closed under taking parents) form the top
// block T; its variables are numbered 0..nT-1 in pivot order (a postorder,
// so the top fronts of any subtree hold a contiguous range ending with the
// subtree's root).  Each factorisation also stores L_TT^{-1} (unit lower)
// twice: by rows (row j holds columns [rlo_j, j], the top variables of the
// subtree of j's front) for the forward sweep, and by columns (one block per
// top front F: rows = the variables of F and of its ancestors, stacked) for
// the backward sweep.
struct TopRowUnit {  // forward: rows [r0, r1), tpr threads per row
  int32_t r0, r1, tpr, pad;
};
struct TopColUnit {  // backward: columns [c0, c1) of top front tf
  int32_t tf, c0, c1, pad;
};
struct TopFront {
  int64_t coff;                // column block (ld x k, column-major)
  int32_t ld, h, k, start;     // h: stacked rows (own and ancestors'), ld >= h
  int32_t tstart, anc_off, n_anc, pad;
};
struct TopAnc {  // one front of a top front's stacked rows
  int32_t tstart, start, k, rowpos;
};
// Construction: the block of L_TT^{-1} with the rows of top front P and the
// columns of top front F (F in the subtree of P), from P's partitioned
// inverse and the block that the child of P on the way to F passed up.
struct TopPair {
  int32_t kP, fP, startP, tstartP;
  int32_t kF, ldF, colbase, ldh;  // colbase: F's first column in P's row segments
  int64_t h_off;                  // P's partitioned inverse
  int64_t inv_off;                // position map of that child (-1 if F == P)
  int64_t cb_in;                  // its (f_C - k_C) x kF block, row-major (-1 if F == P)
  int64_t cb_out;                 // (fP - kP) x kF block for P's parent (-1 at a root)
  int64_t xcol;                   // column block of F at P's stacked rows
};
struct TopTile {  // 64 x 64 output tile of a pair
  int32_t pair, r0, c0, pad;
};
struct TopDev {
  int cut = -1;  // -1: no top block, every level is swept by level
  int nT = 0, tgs = 0;
  int64_t e_row = 0, e_col = 0, e_cb = 0;
  int max_h = 0;
  DBuf<int32_t> n_of_j;   // [nT] pivot index of each top variable
  DBuf<int32_t> slist;    // [nT * tgs] update-vector entries of each (front, position)
  DBuf<int64_t> roff;     // [nT] row offsets
  DBuf<int32_t> rlo, rlen;
  DBuf<TopRowUnit> fwd_units;
  DBuf<TopColUnit> bwd_units;
  int n_fwd = 0, n_bwd = 0;
  DBuf<TopFront> fronts;
  DBuf<TopAnc> anc;
  DBuf<TopPair> pairs;
  std::vector<DBuf<TopTile>> tiles;  // per height, cut upwards
  std::vector<int> n_tiles;
};

// One numeric factorisation of K - sigma M and everything the sweeps read
// from it.  A problem holds two, so that the factorisation at the next shift
// can proceed on another stream while the sweeps use the current one.
struct Factor {
  DBuf<double> h64;                    // partitioned inverses (the fronts: SolveCtx pools)
  DBuf<float> h32;                     // the same in FP32 (mixed precision)
  DBuf<int32_t> piv_perm, piv_type;    // by new index
  DBuf<int32_t> front_stat;            // [n_fronts * 4]: neg, perturbed, 2x2, spare
  DBuf<int32_t> piv_dof, piv_gmap;     // pivot-order gather maps of the sweeps
  DBuf<int32_t> piv_inv;               // [N] pivot index of each DOF (inverse of piv_dof)
  DBuf<int32_t> rows_piv;              // [sum f] pivot index of every front position's DOF
  DBuf<double> d_diag, d_sub;          // D by pivot index: diagonal, (t+1, t) of 2x2 blocks
  DBuf<double> dcoef;                  // [N * 3] D^{-1} by pivot (see dinv_coef_kernel)
  DBuf<double> av;                     // K - sigma M values (refinement residuals)
  DBuf<int32_t> big_perm, big_lperm, big_state;  // blocked-factorisation scratch
  DBuf<int32_t> big_pend;              // per level: fronts left unfinished (0 when complete)
  DBuf<double> trow64, tcol64;         // L_TT^{-1} by rows and by columns
  DBuf<float> trow32, tcol32;
  DBuf<int32_t> tmap, tdof;            // top gather maps in pivot order
  DBuf<double> tdc;                    // [nT * 3] D^{-1} coefficients of the top rows
  DBuf<double> tcb;                    // top block construction blocks [e_cb]
  // sweep scratch: sweeps with this factorisation run one at a time
  DBuf<double> cbvec, fwd;             // update vectors [cb_size], forward z [N]
  DBuf<double> top_r, top_y;           // top block right-hand side and w = D^{-1} y [nT]
  bool factored = false;
  int precision = 0;
  double sigma = 0.0;
  int64_t inertia = 0;
  int perturbed = 0, two = 0;
  int refactored = 0;  // repeats at a shift moved off a singular one (riga_eigs)
  bool pre = false;    // made ahead by a batched call for the solve's first factorisation
};

// The mutable state of one solve: two factorisations (the current one and
// the one made ahead), each with its own sweep scratch, and the dense front
// pools (one f x f block per front) their factorisations work in.  A pool
// is needed only while a factorisation runs -- the sweeps read the
// partitioned inverses H, D and the top block -- so the two factorisations
// share pool slot 0; slot 1 serves a factorisation that overlaps another
// one of the same context (the first shift made ahead beside the one at the
// slice's lower end) and is given back to the allocator afterwards when it
// is large.  A problem has several, so that slices of the spectrum can be
// solved at once.
struct SolveCtx {
  Factor fac[2];
  int cur = 0;
  DBuf<double> pool64[2];
  DBuf<float> pool32[2];
  std::mutex pool_mu;
  bool pool_busy[2] = {false, false};
  Factor& current() { return fac[cur]; }
  Factor& spare() { return fac[1 - cur]; }
};

}  // namespace riga

struct riga_problem {
  riga::Analysis an;
  bool has_device = false;
  // `home` is the stream given at assembly and the one persistent buffers are
  // allocated on; `stream` is the stream of the call in progress (equal to
  // `home` between calls).
  hipStream_t home = nullptr;
  hipStream_t stream = nullptr;
  int device = 0;

  // coefficients and assembled matrices
  riga::DBuf<double> kappa, rho;
  riga::DBuf<int64_t> row_ptr;
  riga::DBuf<int32_t> col_idx;
  riga::DBuf<double> kv, mv;        // K and M values (CSR order)
  riga::DBuf<double> tab_val, tab_der;  // basis tables per direction
  riga::DBuf<double> ke1, me1;          // 1D element matrices per direction
  riga::DBuf<double> ge1;               // 1D element integrals of B_a B_b' (complex pencils)
  double potential[3] = {0.0, 0.0, 0.0}; // vector potential of a complex pencil
  riga::DBuf<int32_t> fe, le, first_fn; // 1D maps per direction (concatenated)
  int tab_off[3] = {0, 0, 0};       // element offset of each direction in the tables
  int fn_off[3] = {0, 0, 0};        // function offset of each direction in fe/le
  double normK1 = 0.0, normM1 = 0.0, maxabsA = 0.0;
  int spmv_group = 8;

  // symbolic factorisation on the device
  riga::DBuf<int32_t> d_rows, d_fk, d_ff, d_fstart, d_child_ptr, d_child_list, d_inv;
  riga::DBuf<int64_t> d_rows_off, d_pool_off, d_cb_off, d_inv_off, d_amap_ptr;
  riga::DBuf<int32_t> d_amap_row, d_amap_val;
  riga::DBuf<int32_t> d_asm_ident;  // per front: one child whose update block maps row for row
  std::vector<riga::LevelDev> levels;

  // numeric factorisations: ctx[0].current() is the one riga_factor /
  // riga_solve use; ctx[i] serves the i-th further slice of the spectrum
  // (buffers are allocated on first use)
  riga::SolveCtx ctx[8];
  riga::DBuf<riga::WorkUnit> inv_units;     // row blocks of every front
  int n_inv_units = 0;

  // solve descriptors
  riga::DBuf<riga::FrontDesc> d_desc;
  riga::DBuf<int32_t> d_front_of;           // front of each new (pivot-order) index
  riga::DBuf<int32_t> d_gmap;               // [sum f * gstride] children's update indices
  int gstride = 1;
  riga::TopDev top;                         // explicit inverse of the top levels
  riga::SubtreeDev sub;                     // fused sweeps of the bottom heights
  bool tuned = false;                       // top and sub from a measured choice
  riga::DBuf<double> ir_r, ir_x, ir_d;      // iterative refinement vectors

  riga_stats stats{};
};

namespace riga {

// ---- launchers (kernels in k_*.hip) ----
void launch_basis_tables(riga_problem* pr);
void launch_assemble(riga_problem* pr);
void compute_norms(riga_problem* pr);

void launch_axpby_vals(const double* k, const double* m, double sigma, double* a, int64_t n,
                       hipStream_t s);
// y = A x (A one of kv/mv/av); with dot_partial, also spmv_dot_blocks()
// partial sums of x^T y.
void launch_spmv(const riga_problem* pr, const double* vals, const double* x, double* y,
                 double* dot_partial, hipStream_t s);
int spmv_blocks(const riga_problem* pr);
int spmv_dot_blocks(const riga_problem* pr);
// KU = K U, MU = M U for the nw columns of U (N x nw, column-major).
void launch_spmm_km(const riga_problem* pr, const double* U, int nw, double* KU, double* MU,
                    hipStream_t s);

// Factorises K - sigma M into F on stream s (host-synchronous: returns with
// F complete, its inertia read back).  Reads only the problem's symbolic
// data and matrices, so it may run on another thread and stream while the
// sweeps use the other Factor.
void factor_numeric(riga_problem* pr, Factor& F, double sigma, int precision, hipStream_t s);
// factor_numeric of several problems (each Fs[i] reserved for `precision`)
// with every tree height of all of them in one launch per kernel: the same
// per-front arithmetic as one problem alone, so the factorisations are
// identical bit for bit.  Problems of different heights share the launches
// of the heights they have.  Synchronises s.
void factor_numeric_batched(const std::vector<riga_problem*>& prs, const std::vector<Factor*>& Fs,
                            const std::vector<double>& sigmas, int precision, hipStream_t s);
// Allocates every buffer factor_numeric(F, precision) writes (a no-op once
// done): call it on the thread and stream that own the problem before a
// factorisation runs on another stream.
void factor_reserve(riga_problem* pr, Factor& F, int precision, hipStream_t s);
// H = [I; L21] L11^{-1} for every front (D kept on the diagonal), from the
// factor pool into the H pool.
template <class T>
void launch_front_inverse(riga_problem* pr, Factor& F, const T* pool, T* h, hipStream_t s);
size_t front_inverse_lds(int max_k);
// Fronts above the LDS limit of one tree level (`fronts`, orders big_f,
// fully-summed orders big_k): blocked LDL^T spread over many workgroups.
// Without `checked`, the predicted number of panel steps plus one is
// launched and the count of unfinished fronts is left in F.big_pend[level]
// for the caller to test after its own synchronisation; with `checked`, the
// host waits for that count and launches further steps until it is zero.
template <class T>
void factor_big_fronts(riga_problem* pr, Factor& F, T* pool, const int32_t* fronts,
                       const std::vector<int>& big_f, const std::vector<int>& big_k,
                       double pivtol, int level, bool checked, hipStream_t s);
int bigfront_max_k();
// Launch shape of the blocked fronts of one height: fronts in the grid,
// panel steps predicted for the widest, largest fully-summed and update
// orders, trailing and update-block tiles of the largest front.
struct BigPlan {
  int nbig = 0, steps = 0, maxk = 0, maxcb = 0, max_tiles = 0, max_cb_tiles = 0;
};
BigPlan big_plan(const std::vector<int>& big_f, const std::vector<int>& big_k);
// The device argument block of one problem's blocked fronts at one height
// (big_args_bytes() bytes, written to host memory at `out`).
size_t big_args_bytes();
void big_args_fill(riga_problem* pr, Factor& F, void* pool, const int32_t* fronts, const BigPlan& P,
                   double pivtol, int level, void* out);
// The blocked fronts of one height of several problems in one launch per
// kernel: `jobs` (device) holds njobs argument blocks, ystart[j] (device,
// njobs + 1 entries) the first grid front of job j; P merges the jobs'
// plans (nbig: their sum, the rest: maxima).  Unchecked: each job's count of
// unfinished fronts goes to its own pending counter.
template <class T>
void factor_big_fronts_batched(const void* jobs, const int32_t* ystart, int njobs, const BigPlan& P,
                               hipStream_t s);
// Allocates the blocked-factorisation scratch of F for every level (fronts
// above lds_max_f), so that no level reallocates it mid-factorisation.
void bigfront_reserve(riga_problem* pr, Factor& F, int lds_max_f, hipStream_t s);
// Pivot-order gather maps of the sweeps (after each factorisation).
void launch_pivot_maps(riga_problem* pr, Factor& F, hipStream_t s);
// Top block: chooses the cut and builds its static maps (at set-up); builds
// L_TT^{-1} of factorisation F from its partitioned inverses h; runs the
// top part of a forward/backward sweep.
// forced = TOP_CUT_MODEL: RIGA_TOP_CUT, else the cost model; -1: no top
// block; c >= 1: the cut at height c (none if it exceeds the size limits).
constexpr int TOP_CUT_MODEL = -1000;
void setup_top(riga_problem* pr, int forced = TOP_CUT_MODEL);
// the cuts within the size limits, and -1 (no top block)
std::vector<int> top_cut_candidates(const riga_problem* pr);
// Fused bottom heights of the sweeps: forced = SUB_FROM_ENV reads
// RIGA_SUBTREE_HEIGHTS (unset: none); 0: none; SUB_AUTO: the automatic
// choice; n >= 2: n heights where they fit.
constexpr int SUB_FROM_ENV = -1000, SUB_AUTO = -1;
void setup_subtrees(riga_problem* pr, int forced = SUB_FROM_ENV);
// The measured choice for this problem's device and tree in the tuning
// cache, if any (tune.cpp).
bool tune_lookup(const riga_problem* pr, int* cut, int* fused);
// Times the candidate decompositions, applies and caches the fastest;
// the problem's factorisations are invalidated.
void tune_problem(riga_problem* pr, int precision, int reps, riga_tune_result* out);
void top_reserve(riga_problem* pr, Factor& F, int precision, hipStream_t s);
template <class T>
void build_top(riga_problem* pr, Factor& F, const T* h, T* trow, T* tcol, hipStream_t s);
template <class T>
void sweep_top(riga_problem* pr, const Factor& F, const T* trow, const T* tcol, const double* b,
               double* x, hipStream_t s);
// Binds a call's stream to the problem for the duration of the call only, so
// no stream handle outlives the call that passed it.
struct StreamBind {
  riga_problem* pr;
  hipStream_t prev;
  StreamBind(riga_problem* p, hipStream_t s) : pr(p), prev(p->stream) { p->stream = s; }
  ~StreamBind() { pr->stream = prev; }
  StreamBind(const StreamBind&) = delete;
  StreamBind& operator=(const StreamBind&) = delete;
};

// Raises the dynamic-LDS limit of the kernels that need more than 64 KB;
// runs once per process (later calls return at once).
void set_kernel_attributes();
void solve_fb(riga_problem* pr, const Factor& F, const double* b, double* x, hipStream_t s);

// Fixed per-device scratch of the entry points that allocate nothing
// (8 MiB; scratch.hip): its device address on the current device.
constexpr size_t NOALLOC_SCRATCH_DOUBLES = (size_t)1 << 20;
double* noalloc_scratch();

// BLAS-like helpers on column-major N x m blocks (ld = N).
int gemv_row_blocks(int64_t n);
// One Gram-Schmidt pass: c = W^T x, then x -= B c (W, B: n x m column-major,
// ld = n); partial holds proj_row_blocks(n) * m doubles.  With alpha_out,
// also *alpha_out = *addend + c[m - 1].  With dj (a launch captured once
// and replayed for every Lanczos step of a run), the pass covers m + *dj
// columns (at most m_max: partial holds proj_row_blocks(n) * m_max) and
// alpha_out, addend are advanced by *dj.
int proj_row_blocks(int64_t n);
void launch_project(const double* W, const double* B, int64_t n, int m, double* x, double* partial,
                    double* c, double* alpha_out, const double* addend, hipStream_t s,
                    const int32_t* dj = nullptr, int m_max = 0);
// dst = column *dj of the n-row block src
void launch_copy_col_dyn(double* dst, const double* src, int64_t n, const int32_t* dj, hipStream_t s);
// *dj += 1
void launch_step_advance(int32_t* dj, hipStream_t s);
void launch_reduce_partials(const double* partial, int nblk, double* out, hipStream_t s);
void launch_fill_random(double* x, int64_t n, uint64_t seed, uint64_t stream_id, hipStream_t s);
// v = x / beta, w = y / beta with beta^2 the sum of partial[0..np).  With
// dj, v, w and beta_out are advanced by *dj columns / entries.
void launch_scale2(const double* x, const double* y, const double* partial, int np, double* v,
                   double* w, int64_t n, double* beta_out, int32_t* flag, hipStream_t s,
                   const int32_t* dj = nullptr);
void launch_gemm_nn(const double* V, int64_t n, int k, const double* S, int lds, int m,
                    double* U, hipStream_t s);
// U -= B (W^T U) for the n x c blocks W, B and the n x m block U (all
// column-major, ld = n), in passes of at most 512 columns of W and B;
// partial holds block_project_partials(n, m) doubles of scratch.
size_t block_project_partials(int64_t n, int m);
void launch_block_project(const double* W, const double* B, int64_t n, int c, double* U, int m,
                          double* partial, hipStream_t s);
// partial: residual_partials(n, m) doubles of scratch
int residual_partials(int64_t n, int m);
void launch_residuals(const double* KU, const double* MU, const double* U, int64_t n, int m,
                      double* out_rq_num, double* out_rq_den, double* out_rnorm2,
                      double* out_unorm2, double* lam_in, double* partial, hipStream_t s);
// U(:, q), V(:, q) *= 1 / sqrt(d[q]) for q < m
void launch_scale_cols_rsqrt(double* U, double* V, int64_t n, int m, const double* d, hipStream_t s);
// d0(:, dst[q]) = s0(:, src[q]) and, if d1, d1(:, dst[q]) = s1(:, src[q])
constexpr int COLS_PER_COPY = 32;
struct ColCopy {
  int32_t count;
  int32_t dst[COLS_PER_COPY], src[COLS_PER_COPY];
};
// with jmul: d0(:, dst[q]) = J s0(:, src[q]) (and d1 from s1), J the
// multiplication by i of interleaved complex columns: (re, im) -> (-im, re)
void launch_copy_cols(const std::vector<int>& dst, const std::vector<int>& src, int64_t n, double* d0,
                      const double* s0, double* d1, const double* s1, hipStream_t s, bool jmul = false);
void launch_copy(double* dst, const double* src, int64_t n, hipStream_t s);
// x <- sg J x in place for interleaved complex storage (J multiplies by i)
void launch_jrot(double* x, int64_t n, double sg, hipStream_t s);
void launch_axpby(double a, const double* u, const double* v, double* out, int64_t n,
                  hipStream_t s);
// out[0] = a^T b; partial: 256 doubles of scratch
void launch_dot(const double* a, const double* b, int64_t n, double* partial, double* out,
                hipStream_t s);
void launch_scale_cols(double* U, int64_t n, int m, const double* scale, hipStream_t s);

// Projected (tridiagonal) eigenproblem of T_m: diagonal alpha[0..m),
// off-diagonal beta[1..m) (beta[j] couples j-1 and j), residual beta[m].
// ritz_check: theta[m] all eigenvalues ascending, est[m] Ritz estimates
// |beta[m] s_m|.  ritz_vectors: unit eigenvectors S[m x nsel]
// of the eigenvalues theta[sel[q]] (sel ascending), grouped in ncl clusters
// [cl_start[c], cl_start[c+1]) of close eigenvalues.
// ritz_check also stores beta[m] and the breakdown flag at extra[0], extra[1]
void launch_ritz_check(const double* alpha, const double* beta, int m, double* theta, double* est,
                       const int32_t* flag, double* extra, hipStream_t s);
void launch_ritz_vectors(const double* alpha, const double* beta, int m, const double* theta,
                         const int32_t* sel, const int32_t* cl_start, int ncl, double* S,
                         hipStream_t s);

// basis values and derivatives at a q-point Gauss rule per element and
// direction (same layout as tab_val/tab_der); synchronises pr->stream
void basis_tables_q(riga_problem* pr, int q, DBuf<double>& val, DBuf<double>& der);
// eigenfunction errors against the exact Laplace modes (k_accuracy.hip)
void mode_errors(riga_problem* pr, int n_vec, const double* lam, const double* U, int nm,
                 const int32_t* modes, int nquad, int32_t* match, double* overlap, double* ef_l2,
                 double* ef_e, double* ev, hipStream_t s);
void exact_eigenvalues(int dim, int count, double* out);
void launch_eig_grad(const riga_problem* pr, int k, const double* U, const double* lam_w_dev,
                     const double* w_dev, double* gk, double* gr, hipStream_t s);

}  // namespace riga
