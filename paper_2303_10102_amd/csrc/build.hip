// Randomized peeling construction of K~ and of its derivatives (Sec. 3.2-3.3).
//
// Level l (blocks = sibling pairs (a, b) at depth l, parent P at depth l-1):
//   Y   = K X_R - sum_{d<l} H_d X_R              on left-children rows  (eqs. "lvl1 sample1", "lvl2 sample1")
//   Q R = Y[a]   (thin QR, diag R > 0)                                  (Alg. 1 step 3)
//   C   = (K X_S - sum_{d<l} H_d X_S)[b],  X_S = [Q on a rows]          (eqs. "lvl1 sample2", "lvl2 sample2")
//   block (a,b) of K~ = Q C^T                                           (eqs. "lowrnkB11", "lowrnkB212")
// Tangent for theta_j (X_R, X_S held fixed):
//   dY = K_j X_R - sum_d dH_d X_R;  dQ by Alg. 2;
//   dC = (K_j X_S + K [dQ] - sum_d (dH_d X_S + H_d [dQ]))[b]             (eqs. "prod-rule-2", "lvl2 sample2 diff", "tmp2")
//   block (a,b) of K~_j = dQ C^T + Q dC^T                               (eqs. "diff low-rank", "lvl2 block1 diff")
// Leaves: D = sym(((K - sum_d H_d) [I; I; ...])[L, L]), dD likewise        (eqs. "leaf sample", "diag diff")
// H_d X is applied from the stored panels: t_c = F_c^T X[c] for every node c
// at depth d, then Y[c] -= F_c t_sib(c) (tree_reduce / tree_expand).
// QR: shifted Cholesky-QR3 (Fukaya et al. 2020), which returns the unique thin
// QR with positive diag(R) for condition numbers up to ~1/u with GEMM-shaped work.
#include <algorithm>

#include "hm_internal.h"
#include "hm_build.h"

namespace hm {

hm_status sketch_compress(Model* m, const double* Y, int ldy, int ell, int l, int rank, double tol, double* S,
                          double* R, double* V, int kc, int* d_k, double* d_sig);
size_t qr_stack_doubles(int n, int nint, int ell);
hm_status leaf_sym(Model* m, const double* Z, int ldz, double* D);

__global__ void k_fill(double* p, long cnt, double v) {
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < cnt) p[e] = v;
}
hm_status fill(Model* m, double* p, long cnt, double v) {
  if (cnt <= 0) return HM_OK;
  hipLaunchKernelGGL(k_fill, dim3(ceil_div(cnt, 256)), dim3(256), 0, m->stream, p, cnt, v);
  HM_LAUNCH_CHECK();
  return HM_OK;
}

__device__ __forceinline__ bool row_is_left(long i, int l, int levels, int nl) {
  int L = (int)(i / nl);
  return ((L >> (levels - l)) & 1) == 0;
}

// X[i, j] = omega_l[i, j] on right-children rows at depth l, else 0 (n x ell, ld n)
__global__ void k_pattern_omega(const double* om, double* X, int n, int ell, int l, int levels, int nl) {
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)n * ell) return;
  long i = e % n;
  X[e] = row_is_left(i, l, levels, nl) ? 0.0 : om[e];
}

// Zero columns >= k_P of Y on the rows of block P's child on side `side`
// (1 = left, 2 = right) at depth l.  kblk indexed by the parent's heap index.
// columns c of Y (n x wtot, ld ldy) repeat with period w: block column c % w is masked
__global__ void k_mask_cols(double* Y, int ldy, int n, int wtot, int w, int l, int levels, int nl,
                            const int* kblk, int side) {
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)n * wtot) return;
  long i = e % n;
  int cc = (int)(e / n);
  int c = cc % w;
  bool left = row_is_left(i, l, levels, nl);
  if ((side == 1) != left) return;
  int L = (int)(i / nl);
  int idx = L >> (levels - l);            // node index at depth l
  int parent = ((1 << l) - 1 + idx - 1) >> 1;
  if (c >= kblk[parent]) Y[i + (long)cc * ldy] = 0.0;
}

// out_q[i,c] = left(i) ? A_q[i,c] : (B_q[i,c] + (B2_q ? B2_q[i,c] : 0)), masked to k_P columns,
// for the jobs q = blockIdx.y (up to three).
struct MergeJobs {
  const double* A[3]; const double* B[3]; const double* B2[3]; double* out[3];
};
__global__ void k_merge_lr(MergeJobs jb, int ldo, int n, int w, int l, int levels, int nl, const int* kblk) {
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)n * w) return;
  const int q = blockIdx.y;
  const double* A = q == 0 ? jb.A[0] : (q == 1 ? jb.A[1] : jb.A[2]);
  const double* B = q == 0 ? jb.B[0] : (q == 1 ? jb.B[1] : jb.B[2]);
  const double* B2 = q == 0 ? jb.B2[0] : (q == 1 ? jb.B2[1] : jb.B2[2]);
  double* out = q == 0 ? jb.out[0] : (q == 1 ? jb.out[1] : jb.out[2]);
  long i = e % n;
  int c = (int)(e / n);
  int L = (int)(i / nl);
  int idx = L >> (levels - l);
  int parent = ((1 << l) - 1 + idx - 1) >> 1;
  double v = 0.0;
  if (c < kblk[parent]) {
    if ((idx & 1) == 0) v = A[e];
    else v = B[e] + (B2 ? B2[e] : 0.0);
  }
  out[i + (long)c * ldo] = v;
}

// stacked identities: S[i, j] = 1 where row i is local row j of its leaf (not padding)
__global__ void k_ident(double* S, int n, int nl, const int* perm) {
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)n * nl) return;
  long i = e % n;
  int j = (int)(e / n);
  S[e] = ((int)(i % nl) == j && perm[i] >= 0) ? 1.0 : 0.0;
}

hm_status make_identity_stack(Model* m) {
  hipLaunchKernelGGL(k_ident, dim3(ceil_div((long)m->n * m->nl, 256)), dim3(256), 0, m->stream, m->d_ident, m->n,
                     m->nl, m->d_perm);
  HM_LAUNCH_CHECK();
  return HM_OK;
}

// Leaf blocks (leaf-major) on the padding rows and columns: zero, with diag on the diagonal
// (1 for K~: an identity block, inert in the Cholesky, log-determinant and solves;
// 0 for the derivative matrices).
__global__ void k_leaf_pad(double* D, const int* perm, int nl, long cnt, double diag) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= cnt) return;
  const long ls = (long)nl * nl;
  const long L = e / ls;
  const int le = (int)(e % ls), i = le % nl, j = le / nl;
  if (perm[L * nl + i] < 0 || perm[L * nl + j] < 0) D[e] = (i == j) ? diag : 0.0;
}
hm_status leaf_pad(Model* m, double* D, double diag) {
  if (m->uniform) return HM_OK;
  const long cnt = (long)m->nleaves * m->nl * m->nl;
  hipLaunchKernelGGL(k_leaf_pad, dim3(ceil_div(cnt, 256)), dim3(256), 0, m->stream, D, m->d_perm, m->nl, cnt, diag);
  HM_LAUNCH_CHECK();
  return HM_OK;
}

static hm_status mask_cols(Model* m, double* Y, int wtot, int w, int l, const int* kblk, int side) {
  hipLaunchKernelGGL(k_mask_cols, dim3(ceil_div((long)m->n * wtot, 256)), dim3(256), 0, m->stream, Y, m->n, m->n,
                     wtot, w, l, m->levels, m->nl, kblk, side);
  HM_LAUNCH_CHECK();
  return HM_OK;
}

// ---------------------------------------------------------------------------
// Y[ysel rows] -= sum_{d=1}^{l-1} H_d X ;  dY_j -= sum_d dH_{j,d} X  (if dY)
// ---------------------------------------------------------------------------
hm_status subtract_coarser(Model* m, const PanelSet& ps, int l, const double* X, int w, LeafSel xsel,
                           LeafSel ysel, double* Y, double* const* dY, int nr, const NodeBufs& nb, int wt) {
  if (l <= 1) return HM_OK;
  if (wt < 0) wt = w;   // the tangents take the first wt columns of X
  PrecScope prec(m);   // coarser-level subtraction: FP32 under the mixed policy
  const int bw = ps.bw;
  const long ts = (long)bw * w;   // t_c: bw x w per node; its first wt columns serve the tangents
  // the value and tangent parts are independent: one launch of reduces (t_c = F_c^T X,
  // dt_c = dF_c^T X), then one of expands (Y -= F t; dY_j -= dF_j t + F dt_j)
  const int nj = dY ? 1 + nr : 1;
  ReduceJob rj[3];
  ExpandJob ej[3];
  rj[0] = ReduceJob{ps.F, m->n, cs_block(bw), X, m->n, cs_fixed(0, w), 1, l - 1, nb.t, ts, xsel};
  ej[0] = ExpandJob{ps.F, m->n, cs_block(bw), Y, m->n, cs_fixed(0, w), nb.t, ts, bw, 1, 0, 1, l - 1, -1.0, 1.0, ysel};
  for (int j = 0; j + 1 < nj; ++j) {
    // dt_c: bw x wt, stored with t's node stride so that one expand reads both
    rj[1 + j] = ReduceJob{ps.dF[j], m->n, cs_block(bw), X, m->n, cs_fixed(0, wt), 1, l - 1, nb.dt[j], ts, xsel};
    ExpandJob e{ps.dF[j], m->n, cs_block(bw), dY[j], m->n, cs_fixed(0, wt), nb.t, ts, bw, 1, 0, 1, l - 1, -1.0,
                1.0, ysel};
    e.A2 = ps.F;
    e.T2 = nb.dt[j];
    e.alpha2 = -1.0;
    ej[1 + j] = e;
  }
  HM_CHECK(tree_reduce_multi(m, rj, nj));
  HM_CHECK(tree_expand_multi(m, ej, nj));
  return HM_OK;
}

// Shifted Cholesky-QR3 of Y[a] (w columns) for every left child a at depth l.
// Q -> Qout (left rows; right rows untouched), R^{-1} per left child -> nb.rinv.
static hm_status cholqr3(Model* m, const double* Y, int w, int l, const int* kblk, double* Qout, double* tmp,
                         const NodeBufs& nb) {
  const LeafSel left{1, l};
  const long s2 = (long)w * w;
  const int heap0 = (1 << l) - 1;
  const int cnt = 1 << (l - 1);
  const long mrows = m->n >> l;
  const double* src = Y;
  double* dsts[3] = {Qout, tmp, Qout};
  double* rinv[3] = {nb.r1i, nb.r2i, nb.r3i};
  double* rr[3] = {nb.r1, nb.r2, nb.r3};
  for (int pass = 0; pass < 3; ++pass) {
    ReduceJob g{src, m->n, cs_fixed(0, w), src, m->n, cs_fixed(0, w), l, l, nb.g, s2, left};
    HM_CHECK(tree_reduce(m, g));
    HM_CHECK(chol_inv_nodes(m, nb.g, s2, rr[pass], rinv[pass], s2, w, kblk, heap0, 2, cnt, pass == 0 ? 1 : 0,
                            mrows));
    ExpandJob e{src, m->n, cs_fixed(0, w), dsts[pass], m->n, cs_fixed(0, w), rinv[pass], s2, w, 0, 0, l, l, 1.0,
                0.0, left};
    HM_CHECK(tree_expand(m, e));
    src = dsts[pass];
  }
  // R^{-1} = R1^{-1} R2^{-1} R3^{-1}  (left children only: stride 2 nodes)
  HM_CHECK(gemm(m->stream, false, false, w, w, w, 1.0, nb.r2i + heap0 * s2, w, 2 * s2, nb.r3i + heap0 * s2, w,
                2 * s2, 0.0, nb.w + heap0 * s2, w, 2 * s2, cnt));
  HM_CHECK(gemm(m->stream, false, false, w, w, w, 1.0, nb.r1i + heap0 * s2, w, 2 * s2, nb.w + heap0 * s2, w,
                2 * s2, 0.0, nb.rinv + heap0 * s2, w, 2 * s2, cnt));
  return HM_OK;
}

// Alg. 2 for every left child at depth l and every tangent j < nr (at most two):
// dQ_j = dY_j R^{-1} - Q M_j,  M_j = triu(W_j) + strict_tril(W_j)^T,  W_j = Q^T dY_j R^{-1}.
// dQ_j -> out[j] (left rows).  The tangents share each launch: per left child a, tangent
// j's node blocks sit in heap slot a + j (slot a + 1, the right sibling, is free at this
// depth), G_j^T = dY_j^T Q is reduced directly, so that W_a^T and W_{a+1}^T are one
// product R^{-T} [G_0^T G_1^T] of adjacent blocks.
static hm_status qr_tangents(Model* m, const double* Q, double* const* dY, int nr, int w, int l,
                             double* const* out, const NodeBufs& nb) {
  if (nr <= 0) return HM_OK;
  if (nr > 2 || nb.mfold == nb.w) {   // the fold reads W^T while it writes M
    set_error("qr_tangents: at most two tangents, with separate W and M node buffers");
    return HM_E_INVAL;
  }
  const LeafSel left{1, l};
  const long s2 = (long)w * w;
  const int heap0 = (1 << l) - 1;
  const int cnt = 1 << (l - 1);
  ReduceJob rj[2];
  ExpandJob ej[2];
  for (int j = 0; j < nr; ++j) {
    // right children are left unwritten: their slots hold the other tangent's blocks
    rj[j] = ReduceJob{dY[j], m->n, cs_fixed(0, w), Q, m->n, cs_fixed(0, w), l, l, nb.g + j * s2, s2, left, true};
    // out = dY R^{-1} - Q M in one launch per tangent (both tangents in one launch)
    ExpandJob e{dY[j], m->n, cs_fixed(0, w), out[j], m->n, cs_fixed(0, w), nb.rinv, s2, w, 0, 0, l, l, 1.0, 0.0,
                left};
    e.A2 = Q;
    e.T2 = nb.mfold + j * s2;
    e.alpha2 = -1.0;
    ej[j] = e;
  }
  HM_CHECK(tree_reduce_multi(m, rj, nr));
  // [W_0^T W_1^T] = R^{-T} [G_0^T G_1^T] per left child (node stride two slots)
  HM_CHECK(gemm(m->stream, true, false, w, nr * w, w, 1.0, nb.rinv + heap0 * s2, w, 2 * s2, nb.g + heap0 * s2, w,
                2 * s2, 0.0, nb.w + heap0 * s2, w, 2 * s2, cnt));
  HM_CHECK(alg2_fold_nodes(m, nb.w, nb.mfold, s2, w, heap0, 2 * cnt, true));
  HM_CHECK(tree_expand_multi(m, ej, nr));
  return HM_OK;
}

// One level of the construction.  XR: n x w test matrix (right-children rows).
// Writes panel block l of ps (and of its tangents when nr > 0).
hm_status level_step(Model* m, const double* theta, const PanelSet& ps, int l, const double* XR, int w,
                     const int* kblk, int nr, const int* realidx, const LevelBufs& b, const NodeBufs& nb,
                     const int* kblk_host) {
  const int n = m->n;
  const LeafSel left{1, l}, right{2, l};
  double* dY[2] = {b.dY[0], b.dY[1]};
  auto tangent_outputs = [&](double* const* bufs, double** kap, double** alp) {
    *kap = nullptr;
    *alp = nullptr;
    for (int j = 0; j < nr; ++j) {
      if (realidx[j] == 0) *kap = bufs[j];
      if (realidx[j] == 1) *alp = bufs[j];
    }
  };
  double *kap, *alp;
  // ---- pass 1: sample the column space of each block
  tangent_outputs(dY, &kap, &alp);
  HM_CHECK(kapply_sel(m, theta, XR, n, w, b.Y, kap, alp, n, right, left));
  HM_CHECK(subtract_coarser(m, ps, l, XR, w, right, left, b.Y, nr ? dY : nullptr, nr, nb));
  // Y | dY[j] and XS | XdS[j] adjacent: one mask and one clear for all of them
  bool ycat = true, xcat = true;
  for (int j = 0; j < nr; ++j) {
    ycat = ycat && dY[j] == b.Y + (long)(j + 1) * n * w;
    xcat = xcat && b.XdS[j] == b.XS + (long)(j + 1) * n * w;
  }
  // the mask zeroes columns past each block's kept rank; with the ranks known on the host
  // and every block of this level at full width it has nothing to do
  bool full = kblk_host != nullptr;
  for (int P = (1 << (l - 1)) - 1; full && P < (1 << l) - 1; ++P) full = kblk_host[P] >= w;
  if (full) {
  } else if (ycat) {
    HM_CHECK(mask_cols(m, b.Y, (1 + nr) * w, w, l, kblk, 1));
  } else {
    HM_CHECK(mask_cols(m, b.Y, w, w, l, kblk, 1));
    for (int j = 0; j < nr; ++j) HM_CHECK(mask_cols(m, dY[j], w, w, l, kblk, 1));
  }
  if (xcat) {
    HM_CHECK(fill(m, b.XS, (long)(1 + nr) * n * w, 0.0));
  } else {
    HM_CHECK(fill(m, b.XS, (long)n * w, 0.0));
    for (int j = 0; j < nr; ++j) HM_CHECK(fill(m, b.XdS[j], (long)n * w, 0.0));
  }
  HM_CHECK(cholqr3(m, b.Y, w, l, kblk, b.XS, b.Qt, nb));
  HM_CHECK(qr_tangents(m, b.XS, dY, nr, w, l, b.XdS, nb));
  // ---- pass 2: C = B^T Q on the right-children rows
  double* dZ[2] = {b.dZ[0], b.dZ[1]};
  tangent_outputs(dZ, &kap, &alp);
  bool adjacent = nr > 0;   // XS | XdS[j] and Z | Zq[j] laid out one after another
  for (int j = 0; j < nr; ++j)
    adjacent = adjacent && b.XdS[j] == b.XS + (long)(j + 1) * n * w && b.Zq[j] == b.Z + (long)(j + 1) * n * w;
  if (adjacent) {
    // one K-apply: K on all (1 + nr) w columns, the tangents on the first w; one
    // coarser-level subtraction: the value part on all columns, the tangent part on XS
    HM_CHECK(kapply_multi(m, theta, b.XS, n, (1 + nr) * w, b.Z, (1 + nr) * w, kap, w, alp, w, n, left, right));
    HM_CHECK(subtract_coarser(m, ps, l, b.XS, (1 + nr) * w, left, right, b.Z, nr ? dZ : nullptr, nr, nb, w));
  } else {
    HM_CHECK(kapply_sel(m, theta, b.XS, n, w, b.Z, kap, alp, n, left, right));
    for (int j = 0; j < nr; ++j)
      HM_CHECK(kapply_sel(m, theta, b.XdS[j], n, w, b.Zq[j], nullptr, nullptr, n, left, right));
    HM_CHECK(subtract_coarser(m, ps, l, b.XS, w, left, right, b.Z, nr ? dZ : nullptr, nr, nb));
    for (int j = 0; j < nr; ++j)
      HM_CHECK(subtract_coarser(m, ps, l, b.XdS[j], w, left, right, b.Zq[j], nullptr, 0, nb));
  }
  // ---- store panels: Q on left rows, C on right rows (masked to k_P columns), one launch
  const long off = (long)(l - 1) * ps.bw * n;
  MergeJobs jb{};
  jb.A[0] = b.XS;
  jb.B[0] = b.Z;
  jb.out[0] = ps.F + off;
  for (int j = 0; j < nr; ++j) {
    jb.A[1 + j] = b.XdS[j];
    jb.B[1 + j] = dZ[j];
    jb.B2[1 + j] = b.Zq[j];
    jb.out[1 + j] = ps.dF[j] + off;
  }
  hipLaunchKernelGGL(k_merge_lr, dim3(ceil_div((long)n * w, 256), 1 + nr), dim3(256), 0, m->stream, jb, n, n, w, l,
                     m->levels, m->nl, kblk);
  HM_LAUNCH_CHECK();
  return HM_OK;
}

// Leaf pass: D = sym((K - sum H) S), dD_j likewise (S = stacked identities).
hm_status leaf_pass(Model* m, const double* theta, const PanelSet& ps, int nr, const int* realidx,
                    const LevelBufs& b, const NodeBufs& nb, double* D, double* const* dD) {
  const int n = m->n, nl = m->nl;
  double* dZ[2] = {b.dZl[0], b.dZl[1]};
  double *kap = nullptr, *alp = nullptr;
  for (int j = 0; j < nr; ++j) {
    if (realidx[j] == 0) kap = dZ[j];
    if (realidx[j] == 1) alp = dZ[j];
  }
  HM_CHECK(kapply(m, theta, m->d_ident, n, nl, b.Zl, kap, alp, n));
  HM_CHECK(subtract_coarser(m, ps, m->levels + 1, m->d_ident, nl, sel_all(), sel_all(), b.Zl,
                            nr ? dZ : nullptr, nr, nb));
  HM_CHECK(leaf_sym(m, b.Zl, n, D));
  HM_CHECK(leaf_pad(m, D, 1.0));
  for (int j = 0; j < nr; ++j) {
    HM_CHECK(leaf_sym(m, dZ[j], n, dD[j]));
    HM_CHECK(leaf_pad(m, dD[j], 0.0));
  }
  return HM_OK;
}

// out[p + c n] = in[pad2tree[p] + c n_in] (0 on padding rows), cnt = n x columns
__global__ void k_pad_rows(const double* in, int n_in, double* out, int n, const int* pad2tree, long cnt) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= cnt) return;
  const long c = e / n;
  const int p = (int)(e % n), r = pad2tree[p];
  out[e] = r >= 0 ? in[r + c * n_in] : 0.0;
}

// ---------------------------------------------------------------------------
// sketch creation: per level, ell-wide sample -> compression V -> level step
// with the compressed test matrix (value only), into a temporary panel set.
// ---------------------------------------------------------------------------
hm_status sketch_build(Sketch* s, const double* omega, const double* theta0) {
  Model* m = s->m;
  const int n = m->n, levels = m->levels, ell = s->ell, r = s->rank;
  const int nodes = (1 << (levels + 1)) - 1;
  const int nint = (1 << levels) - 1;
  // temporary allocations (setup only)
  std::vector<void*> allocs;
  bool alloc_failed = false;
  auto alloc = [&](size_t doubles) -> double* {
    void* p = dev_alloc(m->ctx, std::max<size_t>(doubles, 1) * sizeof(double));
    if (!p) {
      alloc_failed = true;
      return nullptr;
    }
    allocs.push_back(p);
    return (double*)p;
  };
  auto cleanup = [&]() {
    for (void* p : allocs) dev_free(m->ctx, p);
  };
  PanelSet ps{};
  ps.bw = r;
  ps.F = alloc((size_t)n * levels * r);
  // draws by tree row of the real points; a non-uniform tree stores them in the padded layout
  double* omega_pad = nullptr;
  if (!m->uniform) omega_pad = alloc((size_t)levels * ell * n);
  double* Xl = alloc((size_t)n * ell);
  double* Yl = alloc((size_t)n * ell);
  double* Xr = alloc((size_t)n * r);
  double* Sqr = alloc(2 * qr_stack_doubles(n, nint, ell));   // stacked R factors of the chunked QR
  double* Rq = alloc((size_t)(nint) * ell * ell);
  double* Vb = alloc((size_t)nint * ell * r);   // V per parent heap index, ell x r
  double* sig = alloc((size_t)nint * ell);
  LevelBufs b{};
  b.Y = alloc((size_t)n * r);
  b.XS = alloc((size_t)n * r);
  b.Z = alloc((size_t)n * r);
  b.Qt = alloc((size_t)n * r);
  NodeBufs nb{};
  const int tw = std::max(ell, r);
  nb.t = alloc((size_t)nodes * r * tw);
  double* nbs[9];
  for (int q = 0; q < 9; ++q) nbs[q] = alloc((size_t)nodes * r * r);
  nb.g = nbs[0]; nb.r1 = nbs[1]; nb.r1i = nbs[2]; nb.r2 = nbs[3]; nb.r2i = nbs[4];
  nb.r3 = nbs[5]; nb.r3i = nbs[6]; nb.rinv = nbs[7]; nb.w = nbs[8];
  nb.mfold = nb.w;
  if (alloc_failed) {
    cleanup();
    set_error("sketch creation: device allocation failed");
    return HM_E_NOMEM;
  }
  hm_status st = HM_OK;
  size_t need = (size_t)m->nleaves * levels * r * tw;
  need = std::max(need, (size_t)m->nleaves * r * r);
  st = ensure_reduce_ws(m, need);
  if (st == HM_OK && omega_pad) {
    const long cnt = (long)levels * ell * n;
    hipLaunchKernelGGL(k_pad_rows, dim3(ceil_div(cnt, 256)), dim3(256), 0, m->stream, omega, m->n_real, omega_pad, n,
                       m->d_pad2tree, cnt);
    st = (hipGetLastError() == hipSuccess) ? HM_OK : HM_E_DEVICE;
    omega = omega_pad;
  }
  if (st == HM_OK) st = fill(m, ps.F, (long)n * levels * r, 0.0);
  for (int l = 1; l <= levels && st == HM_OK; ++l) {
    const double* om = omega + (size_t)(l - 1) * ell * n;
    hipLaunchKernelGGL(k_pattern_omega, dim3(ceil_div((long)n * ell, 256)), dim3(256), 0, m->stream, om, Xl, n,
                       ell, l, levels, m->nl);
    if ((st = (hipGetLastError() == hipSuccess) ? HM_OK : HM_E_DEVICE) != HM_OK) break;
    if ((st = kapply(m, theta0, Xl, n, ell, Yl, nullptr, nullptr, n)) != HM_OK) break;
    if ((st = subtract_coarser(m, ps, l, Xl, ell, LeafSel{2, l}, LeafSel{1, l}, Yl, nullptr, 0, nb)) != HM_OK)
      break;
    const int heap0 = (1 << (l - 1)) - 1;
    if ((st = sketch_compress(m, Yl, n, ell, l, r, s->rank_tol, Sqr, Rq, Vb + (size_t)heap0 * ell * r, r,
                              s->d_k + heap0,
                              sig + (size_t)heap0 * ell)) != HM_OK)
      break;
    // compressed test matrix: X[b rows] = Omega_b V_P
    if ((st = fill(m, Xr, (long)n * r, 0.0)) != HM_OK) break;
    ExpandJob e{om, n, cs_fixed(0, ell), Xr, n, cs_fixed(0, r), Vb, (long)ell * r, ell, 2, 0, l, l, 1.0, 0.0,
                LeafSel{2, l}};
    if ((st = tree_expand(m, e)) != HM_OK) break;
    st = level_step(m, theta0, ps, l, Xr, r, s->d_k, 0, nullptr, b, nb);
  }
  if (st == HM_OK) {
    if (hipStreamSynchronize(m->stream) != hipSuccess) st = HM_E_DEVICE;
  }
  if (st == HM_OK) {
    s->kblk.assign(nint, 0);
    if (hipMemcpy(s->kblk.data(), s->d_k, nint * sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) st = HM_E_DEVICE;
  }
  if (st == HM_OK) {
    int kc = 0;
    for (int l = 1; l <= levels; ++l) {
      int lvl_max = 0;
      for (int i = (1 << (l - 1)) - 1; i < (1 << l) - 1; ++i) lvl_max = std::max(lvl_max, s->kblk[i]);
      if (lvl_max == 0) {
        set_error("sketch creation: every block of level " + std::to_string(l) + " has rank 0");
        st = HM_E_RANK;
      }
      kc = std::max(kc, lvl_max);
    }
    s->kc = kc;
  }
  if (st == HM_OK) {
    s->d_XR = (double*)dev_alloc(m->ctx, (size_t)n * levels * s->kc * sizeof(double));
    if (!s->d_XR) {
      set_error("sketch creation: device allocation failed");
      st = HM_E_NOMEM;
    }
  }
  if (st == HM_OK) st = fill(m, s->d_XR, (long)n * levels * s->kc, 0.0);
  for (int l = 1; l <= levels && st == HM_OK; ++l) {
    const double* om = omega + (size_t)(l - 1) * ell * n;
    ExpandJob e{om, n, cs_fixed(0, ell), s->d_XR + (size_t)(l - 1) * s->kc * n, n, cs_fixed(0, s->kc), Vb,
                (long)ell * r, ell, 2, 0, l, l, 1.0, 0.0, LeafSel{2, l}};
    st = tree_expand(m, e);
  }
  if (st == HM_OK && hipStreamSynchronize(m->stream) != hipSuccess) st = HM_E_DEVICE;
  if (st == HM_OK) {
    int flags = 0;
    if (hipMemcpy(&flags, m->d_flags, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) st = HM_E_DEVICE;
    if (st == HM_OK && (flags & (DF_QR_FAIL | DF_JACOBI))) {
      set_error("sketch creation: QR/SVD of a sketch failed (flags " + std::to_string(flags) + ")");
      st = HM_E_RANK;
    }
  }
  cleanup();
  return st;
}

}  // namespace hm
