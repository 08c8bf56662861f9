// Internal declarations of the HIP H-MLE library (not part of the public ABI).
//
// Data layout in HBM (all FP64, column-major, rows in tree order):
//   * A "panel set" is an n x (levels*kc) matrix; column block d-1 holds the
//     depth-d panels F_c of every node c at depth d (the nodes of one depth
//     partition the rows, so one n x kc block holds all of them).
//   * Leaf blocks are stored leaf-major: leaf L occupies nl*nl contiguous
//     doubles (column-major nl x nl) at offset L*nl*nl.
//   * Per-node small matrices are stored by heap index (root 0, children of
//     x are 2x+1 and 2x+2) with a fixed stride per node.
#pragma once
#include <hip/hip_runtime.h>
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/hmle.h"

namespace hm {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
void set_error(const std::string& msg);
const char* get_error();

#define HM_HIP(call)                                                              \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess) {                                                       \
      hm::set_error(std::string("HIP error ") + hipGetErrorString(e_) + " at " + \
                    __FILE__ + ":" + std::to_string(__LINE__));                   \
      return HM_E_DEVICE;                                                         \
    }                                                                             \
  } while (0)

#define HM_CHECK(st)                 \
  do {                               \
    hm_status s_ = (st);             \
    if (s_ != HM_OK) return s_;      \
  } while (0)

#define HM_LAUNCH_CHECK() HM_HIP(hipGetLastError())

// device-side status flags (bit mask), read back at scalar-returning calls
enum DevFlag : int { DF_NOT_SPD_LEAF = 1, DF_NOT_SPD_NODE = 2, DF_QR_FAIL = 4, DF_NONFINITE = 8,
                     DF_JACOBI = 16 };

// ---------------------------------------------------------------------------
// model, sketch, H
// ---------------------------------------------------------------------------
// Kernel-family instrumentation (roofline measurement): launches of the enabled
// family are timed by HIP events on the model stream; each record carries the
// launch's algorithmic flop and byte counts.  The expand family passes its events to
// the launch itself (hipExtLaunchKernel), which sets them to the kernel's own start
// and end, with no marker packets between the kernels; the other families record
// the events before and after their launches.
enum ProfFamily : int { PF_NONE = -1, PF_EXPAND = 0, PF_REDUCE = 1, PF_DST = 2, PF_GEMM = 3, PF_LEAFGEMM = 4,
                        PF_COUNT = 5 };
struct ProfRec {
  hipEvent_t a, b;
  double flops, bytes;
  bool by_launch;   // a and b are set by the kernel launch
};

// Grid point (x, y) -> tree position, the closed form of the uniform bisection
// (splits alternate x, y, x, ... from the root; leaves wl x hl): the leaf index
// interleaves the bits of x / wl and y / hl in split order, and
//   t = leaf * nl + (x mod wl) + (y mod hl) * wl.
// One-dimensional models keep grid order.  The quotients use reciprocal
// multipliers ceil(2^32 / w), exact for coordinates and extents up to 2^16.
// A tree with leaves of unequal size (odd sides, left child floor(side/2)) has no
// closed form: then tab holds the position of every grid point (y N + x).
struct TreeIdx {
  int two, wl, hl, nl, sx, sy;
  unsigned mx, my;
  const int* tab;
  int N;
  __host__ __device__ static unsigned spread(unsigned v) {   // bit b -> bit 2b (16 bits)
    v &= 0xFFFFu;
    v = (v | (v << 8)) & 0x00FF00FFu;
    v = (v | (v << 4)) & 0x0F0F0F0Fu;
    v = (v | (v << 2)) & 0x33333333u;
    v = (v | (v << 1)) & 0x55555555u;
    return v;
  }
  __device__ __forceinline__ int operator()(int x, int y) const {
    if (tab) return tab[y * N + x];
    if (!two) return x;
    const unsigned xh = __umulhi((unsigned)x, mx), yh = __umulhi((unsigned)y, my);
    const unsigned L = (spread(xh) << sx) | (spread(yh) << sy);
    return (int)(L * (unsigned)nl + ((unsigned)x - xh * wl) + ((unsigned)y - yh * hl) * wl);
  }
};
TreeIdx make_tree_idx(int dim, int N, int levels);

// Workgroup placement over the XCDs.  A launch's workgroups go to the eight XCDs in
// turn by linear id (x fastest, then y, then z), and each XCD has its own L2.
// xcd_order() renumbers the linear ids so that every XCD receives one contiguous
// range of logical ids, and tile_block() turns the logical id back into (x, y, z)
// with x fastest.  Tiles that are neighbours in that order share operand blocks
// (the row tiles of one column tile; the column tiles, depths and row chunks of one
// leaf), which then come from one L2 instead of being fetched once per XCD.  The
// renumbering is a bijection: it moves work between XCDs and changes nothing else.
constexpr int kXcds = 8;
__host__ __device__ inline int xcd_order(int b, int n) {
  const int per = n / kXcds, rem = n % kXcds;
  const int x = b % kXcds, loc = b / kXcds;
  return (x < rem ? x * (per + 1) : rem * (per + 1) + (x - rem) * per) + loc;
}
struct TileIdx {
  int x, y, z;
};
__device__ __forceinline__ TileIdx tile_block() {
  const int nx = (int)gridDim.x, ny = (int)gridDim.y;
  const int n = nx * ny * (int)gridDim.z;
  const int l = xcd_order((int)blockIdx.x + nx * ((int)blockIdx.y + ny * (int)blockIdx.z), n);
  return TileIdx{l % nx, (l / nx) % ny, l / (nx * ny)};
}

// Device memory of a model and of its sketches and H handles comes from the
// context's allocator callbacks (e.g. a caching allocator of the caller's framework);
// without callbacks, hipMalloc / hipFree.
struct Ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  hm_alloc_fn alloc = nullptr;
  hm_free_fn release = nullptr;
  void* uctx = nullptr;
};
void* dev_alloc(const Ctx* c, size_t bytes);
void dev_free(const Ctx* c, void* p);

// Counters of the work done through one model (read by hm_stats).
struct ModelCounters {
  long long kcols_value = 0;   // columns of K applied
  long long kcols_deriv = 0;   // columns of dK/dkappa and dK/dalpha applied
  long long kapply_calls = 0;
};

struct Model {
  Ctx* ctx = nullptr;       // allocator and default stream (own_ctx unless the caller gave one)
  Ctx own_ctx;
  ModelCounters cnt;
  int device = 0;
  hipStream_t stream = nullptr;
  // n: rows of the tree-ordered layout.  The leaves are stored uniformly, nl rows each
  // (n = nleaves nl); with leaves of unequal size (non-uniform bisection) each leaf is
  // padded to the largest, and the padding ("ghost") rows are identically zero in
  // every panel, sample and vector, identity in the leaf blocks of K~ and zero in
  // those of every derivative matrix.  n_real: grid points (the model's dimension).
  int dim = 2, N = 0, n = 0, levels = 0, nl = 0, nleaves = 0;
  int n_real = 0;
  int nl_min = 0;           // smallest leaf (real rows)
  // variables per location: 2 for the bivariate model, whose natural index is
  // v * nsplit + location (rows with natural index >= nsplit belong to variable 2 and
  // take the second nugget, theta_full[4]); 1 otherwise (nsplit = n_real)
  int nvars = 1;
  long nsplit = 0;
  bool uniform = true;
  // caller-supplied operator (hm_model_create_op): K = sigma2 K_op + tau2 I, applied
  // through op in the caller's point order; d_opws: its reductions' scratch
  hm_op_fn op = nullptr;
  void* op_ctx = nullptr;
  double* d_opws = nullptr;
  bool op_builtin = false;                 // a library operator: its status and message pass through
  void (*op_release)(Model*) = nullptr;    // frees a library operator's state
  // a library operator's own vector-Jacobian product: per-mode weights accumulated into
  // wmode by op_vjp, turned into the four sums of kvjp (see there) by op_vjp_final
  hm_status (*op_vjp)(Model*, const double* theta, const double* X, int ldx, const double* Yb, int ldb, int c,
                      double* wmode) = nullptr;
  hm_status (*op_vjp_final)(Model*, const double* theta, const double* wmode, double* out4) = nullptr;
  long op_wmode = 0;        // doubles of per-mode weights op_vjp needs, if above the default 3 n + 8
  double h = 0.0;
  int* d_perm = nullptr;    // tree position -> grid index (-1 for a padding row)
  int* d_iperm = nullptr;   // grid index -> tree position
  int* d_pad2tree = nullptr;  // non-uniform: tree position -> index among the real rows (-1 padding)
  TreeIdx tix{};            // closed form of iperm for the transforms
  double* d_dst = nullptr;  // N x N orthonormal DST-I
  double* d_dsth = nullptr; // N even: its even/odd halves P0, P1, Q0, Q1 (each N/2 x N/2)
  double* d_mu = nullptr;   // N eigenvalues of the 1D -Laplacian
  double* d_lam = nullptr;  // per-mode multipliers of K, dK/dkappa, dK/dalpha (3 * n)
  double lam_key[4] = {-1.0, -1.0, -1.0, -1.0};  // theta they belong to
  // K-apply workspace (mode space), sized for cmax columns
  int cmax = 0;
  double* d_ws = nullptr;       // 3 * n * cmax
  int* d_flags = nullptr;       // device status flags
  double* d_ident = nullptr;    // stacked identities n x nl (tree order), for the leaf pass
  double* d_red = nullptr;      // per-leaf partials of tree_reduce
  size_t red_doubles = 0;
  // precision policy of the panel products (tree_reduce / tree_expand):
  // mixed = 1 allows FP32 MFMA in the phases that open a PrecScope (2: BF16 in the trace
  // phases as well); panel_prec is
  // the precision in effect (0 FP64, 1 FP32 operands with FP32 accumulation).
  int mixed = 0;
  int panel_prec = 0;
  // kernel variants of the panel products, chosen per model by hm_model_autotune
  // (defaults: one row block of 16 on each of four wavefronts in the expand;
  // four-wavefront row split in the reduce below 1024 workgroups)
  int tune_expand_rb = 0;        // expand variant: 0 = default (variant 1), else 1, 2 or 3
  long tune_reduce_nw4 = 1024;   // reduce launches with fewer workgroups split rows over 4 wavefronts
  int prof_family = PF_NONE;
  std::vector<ProfRec> prof;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
};
// Marks a phase whose panel products may run in reduced precision: FP32 when a mixed
// policy is on (mixed = 1 or 2); in the trace phases (trace = true) BF16 under policy 2.
struct PrecScope {
  Model* m;
  int saved;
  explicit PrecScope(Model* mm, bool trace = false) : m(mm), saved(mm->panel_prec) {
    m->panel_prec = (m->mixed == 2 && trace) ? 2 : (m->mixed ? 1 : 0);
  }
  ~PrecScope() { m->panel_prec = saved; }
};
// profiling helpers (no-ops unless the family is enabled)
bool prof_on(Model* m, int family);
void prof_begin(Model* m, int family);
// a record whose two events the caller hands to hipExtLaunchKernel (null when off)
void prof_begin_launch(Model* m, int family, hipEvent_t& a, hipEvent_t& b);
void prof_end(Model* m, int family, double flops, double bytes);
// grow the tree_reduce partial buffer (setup calls only; never inside an iteration)
hm_status ensure_reduce_ws(Model* m, size_t doubles);

struct Sketch {
  Model* m = nullptr;
  int rank = 0, oversample = 0, ell = 0;
  double rank_tol = 1e-10;    // kept singular values of a block's sample exceed rank_tol * sigma_1
  int kc = 0;                 // column width of every panel block (max kept rank)
  std::vector<int> kblk;      // kept rank per block (heap index of the parent), size 2^levels - 1
  double* d_XR = nullptr;     // n x (levels*kc): level-l test matrix Omega V (right-children rows)
  int* d_k = nullptr;         // device copy of kblk
};


// ---------------------------------------------------------------------------
// kernels / host helpers shared across translation units
// ---------------------------------------------------------------------------
inline int ceil_div(long a, long b) { return (int)((a + b - 1) / b); }

// K-apply: outputs (any may be null) = {K, dK/dkappa, dK/dalpha} X, tree order in and out.
// X: n x c (ld ldx); outputs n x c (ld ldo). c <= m->cmax.
hm_status kapply(Model* m, const double* theta, const double* X, int ldx, int c, double* outK,
                 double* outKap, double* outAlp, int ldo);

// The same K-apply (every row in and out) with its transform scratch supplied by the
// caller: ws holds 5 * n * cblk doubles, and the columns are processed cblk at a time.
hm_status kapply_ws(Model* m, double* ws, int cblk, const double* theta, const double* X, int ldx, int c,
                    double* outK, double* outKap, double* outAlp, int ldo);

// Generic FP64 GEMM, column-major: C = alpha*op(A)*op(B) + beta*C, batched by strides.
hm_status gemm(hipStream_t st, bool ta, bool tb, int M, int Nc, int K, double alpha, const double* A,
               int lda, long sA, const double* B, int ldb, long sB, double beta, double* C, int ldc,
               long sC, int batch);

// Column ranges that depend on the tree depth d of the node being processed:
//   cols(d) = [base + (d-1)*stride, base + (d-1)*stride + w0 + (d-1)*grow)
struct ColSpec {
  int base, stride, w0, grow;
  __host__ __device__ int c0(int d) const { return base + (d - 1) * stride; }
  __host__ __device__ int w(int d) const { return w0 + (d - 1) * grow; }
};
inline ColSpec cs_fixed(int base, int w) { return ColSpec{base, 0, w, 0}; }
inline ColSpec cs_block(int bw) { return ColSpec{0, bw, bw, 0}; }           // block d of width bw
inline ColSpec cs_block_at(int base, int bw) { return ColSpec{base, bw, bw, 0}; }
inline ColSpec cs_prefix(int bw) { return ColSpec{0, 0, 0, bw}; }          // blocks 1..d-1
inline ColSpec cs_prefix_incl(int bw) { return ColSpec{0, 0, bw, bw}; }    // blocks 1..d

// Leaf selection: rows of leaves whose ancestor at depth sel_depth is a left (1) or
// right (2) child; 0 selects every leaf.
struct LeafSel { int mode, depth; };
inline LeafSel sel_all() { return LeafSel{0, 1}; }

// K-apply for an input that vanishes outside the rows of in_sel, whose output is
// needed only on the rows of out_sel (one side of a split, or all rows); output
// rows outside out_sel are left unwritten.  Same result on the needed rows.
hm_status kapply_sel(Model* m, const double* theta, const double* X, int ldx, int c, double* outK,
                     double* outKap, double* outAlp, int ldo, LeafSel in_sel, LeafSel out_sel);
// The same with per-output column counts: outK gets the first cK columns of K X, outKap /
// outAlp the first cKap / cAlp columns of the tangents (one pass of forward transforms).
hm_status kapply_multi(Model* m, const double* theta, const double* X, int ldx, int c, double* outK, int cK,
                       double* outKap, int cKap, double* outAlp, int cAlp, int ldo, LeafSel in_sel,
                       LeafSel out_sel);

// For every node c at depth d in [d0,d1]:  out_c = A[c rows, ac(d)]^T X[c rows, xc(d)]
// (wa x wx(d) column-major, ld wa, stored at out + heap(c)*out_stride).  Rows of
// unselected leaves count as zero.
struct ReduceJob {
  const double* A; int lda; ColSpec ac;
  const double* X; int ldx; ColSpec xc;
  int d0, d1;
  double* out; long out_stride;
  LeafSel sel;
  // true: nodes without selected rows are left unwritten (their sum is zero); false:
  // every node of the depths is written
  bool only_selected = false;
};
hm_status tree_reduce(Model* m, const ReduceJob& j);
// Up to three independent jobs with the same row operand layout (A's lda and columns),
// depths and selection in one launch of the products and one of the tree sums; other
// job lists run one job after another.  Same results as separate calls.
hm_status tree_reduce_multi(Model* m, const ReduceJob* js, int nj);

// For every row i of a selected leaf L:
//   Y[i, yc(d)] = beta*Y + alpha * sum_{d in [d0,d1]} A[i, ac(d)] * T_{s(c_d)}[r0 + 0:wk, 0:wy(d)]
// where c_d is L's ancestor at depth d, s(c) = c (tmode 0), its sibling (1) or its
// parent (2); r0 = half_off if tmode==2 and c is a right child, else 0.  wk = ac.w0.
// T blocks: T + heap(s(c))*t_stride, ld ldt.  beta is applied once per element of
// the union of yc(d) over the segments.
// Optional second source: A2 with blocks T2 (same layout as A, T) adds alpha2 * A2 T2
// to the same sum, so Y = beta Y + alpha sum A T + alpha2 sum A2 T2 in one launch.
struct ExpandJob {
  const double* A; int lda; ColSpec ac;
  double* Y; int ldy; ColSpec yc;
  const double* T; long t_stride; int ldt; int tmode; int half_off;
  int d0, d1;
  double alpha, beta;
  LeafSel sel;
  const double* A2 = nullptr;
  const double* T2 = nullptr;
  double alpha2 = 0.0;
};
hm_status tree_expand(Model* m, const ExpandJob& j);
// Up to three independent jobs (their own A, Y, output columns, T and second source;
// everything else shared) in one launch; other job lists run one after another.
hm_status tree_expand_multi(Model* m, const ExpandJob* js, int nj);

// out[L rows, 0:w] (+)= Dm_L * X[L rows, 0:w], Dm leaf-major
hm_status leaf_gemm(Model* m, const double* Dm, const double* X, int ldx, double* Y, int ldy, int w,
                    double alpha, double beta, int leaf_lo, int leaf_hi);

// per-node small dense kernels (small.hip); nodes heap0 + i*hstep, i < cnt
hm_status chol_inv_nodes(Model* m, const double* G, long gstride, double* R, double* Rinv, long rstride,
                         int k, const int* d_kblk, int heap0, int hstep, int cnt, int shift, long mrows);
hm_status alg2_fold_nodes(Model* m, const double* W, double* M, long stride, int k, int heap0, int cnt,
                          bool trans = false);
hm_status node_lu(Model* m, const double* S, long sstride, double* Nout, long nstride, double* logdet, int k,
                  int heap0, int cnt);
hm_status model_tables(Model* m);
// theta_full[4] checks shared by the entry points (finite; tau2, sigma2 > 0; for the
// stencil model kappa > 0, alpha >= 0)
hm_status check_theta(const Model* m, const double* t);
// an operator model (the points' KD-tree, padded leaves) with op applying K_op
// nv rows per point (co-located variables, natural index v * n + point), the tree over the points
hm_status model_create_op(Ctx* cx, int dim, const double* coords, int n, int leaf, hm_op_fn op, void* uctx,
                          bool builtin, hm_model** out, int nv = 1);
// the bivariate co-kriging model (bivariate.hip)
hm_status model_create_bivariate(Ctx* cx, int dim, int N, double h, int leaf, hm_model** out);
// entries of theta_full: 5 for the bivariate model (second nugget last), else 4
inline int nparams(const Model* m) { return m->nvars == 2 ? 5 : 4; }
// the stencil model on a full grid (side N, spacing h)
hm_status model_create(Ctx* ctx, int device, void* stream, int dim, int N, double h, int leaf, hm_model** out);
// an observed subset of the stencil model's grid points (select.hip)
hm_status model_create_selection(Ctx* cx, int dim, int N, double h, const int* obs, long nobs, int leaf,
                                 hm_model** out);
// length of the per-mode weight buffer of the reverse sweep
inline long wmode_doubles(const Model* m) { return std::max(3L * m->n + 8, m->op_wmode); }
constexpr int OPWS_DOUBLES = 1024 * 16 + 16;   // d_opws: dot partials + 4 results
// time the panel-kernel variants on this model's shapes (panel width kc) and keep the fastest
hm_status autotune(Model* m, int kc, double* report);

}  // namespace hm

// the public context and model handles (opaque in hmle.h)
struct hm_ctx {
  hm::Ctx c;
};
struct hm_model {
  hm::Model m;
};
