// Reverse-mode (adjoint) gradient of the log-likelihood through the factorisation
// and the randomized peeling construction, with the sketches held fixed (Sec. 3.3:
// sampling matrices fixed across iterations, so K~(theta) is a smooth function and
// its gradient is the forward-mode one of Sec. 4.3, eq. "score approximated").
//
// -L~ = n/2 log 2pi + 1/2 log|K~| + 1/2 y^T K~^{-1} y, so dL/dK~ = Kbar = 1/2 (K~^{-1} - z z^T),
// z = K~^{-1} y.  K~ is a function of the stored panels F (Q on left rows, C on
// right rows; block (a,b) = F_a F_b^T) and leaves D, so
//   F_bar_a = 2 Kbar[a,b] F_b = K~^{-1}[a,b] F_b - z_a (z_b^T F_b),   D_bar_L = Kbar[L,L].
// With the Woodbury factors unrolled, K~^{-1} = blockdiag(D_L^{-1}) - sum_P Gp N_P Gp^T
// (Gp = diag(G_a, G_b), G_c = K~_c^{-1} F_c, N_P = (J + S_P)^{-1}; Sec. 3.1, App. C),
//   K~^{-1}[a,b] F_b = -G_a N_P[a,b] S_b - sum_{ancestors} G_c[a] N[c,c] (G_c[b]^T F_b),
//   K~^{-1}[L,L]     = D_L^{-1} - sum_{ancestors c of L} G_c[L] N[c,c] G_c[L]^T.
// The construction is then run backwards (deepest level first; a level's panels
// receive adjoints only from the likelihood, the leaf pass and finer levels):
//   leaf pass   D = sym((K - sum H) S)            -> K-apply VJP, panel adjoints
//   pass 2      C = ((K - sum H) X_S)[b]           -> K-apply VJP, panel adjoints,
//                                                   Q_bar += ((K - sum H) C_bar)[a]
//   QR          Q R = Y                            -> Y_bar = (Q_bar - Q sym(Q^T Q_bar)) R^{-T}
//                                                   (the transpose of Alg. 2)
//   pass 1      Y = ((K - sum H) X_R)[a]           -> K-apply VJP, panel adjoints
// where a subtraction Y -= F_c F_s^T X_s contributes
//   F_bar_c -= Y_bar_c (X_s^T F_s) + X_c (Y_bar_s^T F_s).
// Every K-apply VJP adds its per-mode weights sum_c (S X)(S Y_bar) to one n-vector w;
// the parameter adjoints are sum_m de_m/dtheta_j w_m, so the cost is independent of
// the number of parameters.  Test matrices are recomputed from the stored panels and
// the fixed sketch, never stored per level.
#include "gemm_core.h"
#include "hm_adjoint.h"
#include "hm_internal.h"

namespace hm {

__device__ __forceinline__ bool adj_row_left(long i, int l, int levels, int nl) {
  int L = (int)(i / nl);
  return ((L >> (levels - l)) & 1) == 0;
}

// out = (A + B) on the rows of side `side` (1 left, 2 right children at depth l),
// masked to the block's kept rank; 0 elsewhere.  B may be null.
__global__ void k_side_select(const double* A, const double* B, double* out, int n, int w, int l, int levels,
                              int nl, const int* kblk, int side) {
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)n * w) return;
  long i = e % n;
  int c = (int)(e / n);
  int L = (int)(i / nl);
  int idx = L >> (levels - l);
  int parent = ((1 << l) - 1 + idx - 1) >> 1;
  bool left = adj_row_left(i, l, levels, nl);
  double v = 0.0;
  if (((side == 1) == left) && c < kblk[parent]) v = A[e] + (B ? B[e] : 0.0);
  out[e] = v;
}

// M = B with its upper triangle mirrored: M_ij = B_{min(i,j), max(i,j)}
__global__ void k_sym_up(const double* B, double* M, long stride, int k, int heap0, int hstep) {
  const int node = heap0 + blockIdx.x * hstep;
  const double* b = B + node * stride;
  double* mm = M + node * stride;
  for (int e = threadIdx.x; e < k * k; e += blockDim.x) {
    int i = e % k, j = e / k;
    mm[e] = (i <= j) ? b[i + j * k] : b[j + i * k];
  }
}

__global__ void k_transpose_nodes(const double* R, double* RT, long stride, int k, int heap0, int hstep) {
  const int node = heap0 + blockIdx.x * hstep;
  const double* r = R + node * stride;
  double* t = RT + node * stride;
  for (int e = threadIdx.x; e < k * k; e += blockDim.x) {
    int i = e % k, j = e / k;
    t[e] = r[j + i * k];
  }
}

// Leaf-pass adjoint, one nl x nl block per leaf L (stacked into Zb, n x nl):
//   Zb[L rows, :] = 1/2 (D_L^{-1} - Gs[L rows, :] G[L rows, :]^T - z_L z_L^T)
struct OutLA {
  const double* p; int ld, m0, nl;
  static constexpr bool kfast = false;
  static constexpr int NR = 1;
  __device__ bool load(int i, int k, double (&r)[1]) const {
    const int row = m0 + i;
    const bool ok = row < nl;
    r[0] = p[(ok ? row : 0) + (long)k * ld];
    return ok;
  }
  __device__ double fin(const double (&r)[1]) const { return r[0]; }
};
struct OutLB {
  const double* p; int ld, n0, nl;
  static constexpr bool kfast = false;
  static constexpr int NR = 1;
  __device__ bool load(int k, int j, double (&r)[1]) const {
    const int c = n0 + j;
    const bool ok = c < nl;
    r[0] = p[(ok ? c : 0) + (long)k * ld];
    return ok;
  }
  __device__ double fin(const double (&r)[1]) const { return r[0]; }
};
struct LeafAdjSt {
  double* Zb; const double* Dinv; const double* z; int ldz, nl, m0, n0; long r0;
  static constexpr int NP = 3;
  __device__ void pre(int i, int j, double (&o)[3]) const {
    const int r = m0 + i, c = n0 + j;
    const bool ok = r < nl && c < nl;
    const int rr = ok ? r : 0, cc = ok ? c : 0;
    o[0] = Dinv[rr + (long)cc * nl];
    o[1] = z[r0 + rr];
    o[2] = z[r0 + cc];
  }
  __device__ void put(int i, int j, double v, const double (&o)[3]) const {
    const int r = m0 + i, c = n0 + j;
    if (r >= nl || c >= nl) return;
    Zb[r0 + r + (long)c * ldz] = 0.5 * (o[0] - v - o[1] * o[2]);
  }
};
__global__ void __launch_bounds__(256) k_leaf_adjoint(const double* Gs, const double* G, int ldg, int K,
                                                      const double* Dinv, const double* z, double* Zb, int nl) {
  __shared__ double smem[GSMEM];
  const TileIdx tb = tile_block();
  const int L = tb.z;
  const int m0 = tb.x * GBM, n0 = tb.y * GBN;
  const long r0 = (long)L * nl;
  OutLA la{Gs + r0, ldg, m0, nl};
  OutLB lb{G + r0, ldg, n0, nl};
  TileAcc acc;
  tile_zero(acc);
  tile_gemm(la, lb, 0, K, acc, smem);
  tile_store_pre(LeafAdjSt{Zb, Dinv + (long)L * nl * nl, z, ldg, nl, m0, n0, r0}, acc);
}

static hm_status side_select(Model* m, const double* A, const double* B, double* out, int w, int l, const int* kblk,
                             int side) {
  hipLaunchKernelGGL(k_side_select, dim3(ceil_div((long)m->n * w, 256)), dim3(256), 0, m->stream, A, B, out, m->n,
                     w, l, m->levels, m->nl, kblk, side);
  HM_LAUNCH_CHECK();
  return HM_OK;
}

// Adjoint of Y[ysel] -= sum_{d<l} H_d X[xsel] with respect to the panels:
//   F_bar_c += sign * (Y_bar_c (X_s^T F_s) + X_c (Y_bar_s^T F_s)),  s = sibling of c.
static hm_status subtract_adjoint(Model* m, const double* F, int bw, int l, const double* X, int w, LeafSel xsel,
                                  const double* Yb, LeafSel ysel, double* Fb, double sign, double* tT, double* uT) {
  if (l <= 1) return HM_OK;
  const int n = m->n;
  const long ts = (long)w * bw;
  ReduceJob r1{X, n, cs_fixed(0, w), F, n, cs_block(bw), 1, l - 1, tT, ts, xsel};
  HM_CHECK(tree_reduce(m, r1));
  ReduceJob r2{Yb, n, cs_fixed(0, w), F, n, cs_block(bw), 1, l - 1, uT, ts, ysel};
  HM_CHECK(tree_reduce(m, r2));
  ExpandJob e1{Yb, n, cs_fixed(0, w), Fb, n, cs_block(bw), tT, ts, w, 1, 0, 1, l - 1, sign, 1.0, ysel};
  HM_CHECK(tree_expand(m, e1));
  ExpandJob e2{X, n, cs_fixed(0, w), Fb, n, cs_block(bw), uT, ts, w, 1, 0, 1, l - 1, sign, 1.0, xsel};
  HM_CHECK(tree_expand(m, e2));
  return HM_OK;
}

hm_status adjoint_init(FactorCtx& f, const double* z, AdjBufs& a) {
  Model* m = f.m;
  const int n = m->n, kc = f.kc, levels = m->levels, nl = m->nl;
  const long s2 = (long)kc * kc;
  // Gs_c = G_c N_P[c,c]
  ExpandJob eg{f.G, n, cs_block(kc), a.Gs, n, cs_block(kc), f.Ncc, s2, kc, 0, 0, 1, levels, 1.0, 0.0, sel_all()};
  HM_CHECK(tree_expand(m, eg));
  // leaf blocks of Kbar
  dim3 gl(ceil_div(nl, GBM), ceil_div(nl, GBN), m->nleaves);
  hipLaunchKernelGGL(k_leaf_adjoint, gl, dim3(GCfg::NT), 0, m->stream, a.Gs, f.G, n, levels * kc, f.Dinv, z, a.Zb,
                     nl);
  HM_LAUNCH_CHECK();
  // panel adjoints, level by level
  for (int l = 1; l <= levels; ++l) {
    const ColSpec blk = cs_fixed((l - 1) * kc, kc);
    ExpandJob e0{f.G, n, blk, a.Fb, n, blk, f.Nx, s2, kc, 0, 0, l, l, -1.0, 0.0, sel_all()};
    HM_CHECK(tree_expand(m, e0));
    if (l >= 2) {
      const int wv = (l - 1) * kc;
      ReduceJob rv{f.G, n, cs_fixed(0, wv), f.F, n, blk, l, l, f.nT, (long)wv * kc, sel_all()};
      HM_CHECK(tree_reduce(m, rv));
      ExpandJob ev{a.Gs, n, cs_fixed(0, wv), a.Fb, n, blk, f.nT, (long)wv * kc, wv, 1, 0, l, l, -1.0, 1.0,
                   sel_all()};
      HM_CHECK(tree_expand(m, ev));
    }
  }
  // - z_a (z_b^T F_b) on every level
  ReduceJob rz{z, n, cs_fixed(0, 1), f.F, n, cs_block(kc), 1, levels, a.uT, kc, sel_all()};
  HM_CHECK(tree_reduce(m, rz));
  ExpandJob ez{z, n, cs_fixed(0, 1), a.Fb, n, cs_block(kc), a.uT, kc, 1, 1, 0, 1, levels, -1.0, 1.0, sel_all()};
  HM_CHECK(tree_expand(m, ez));
  return HM_OK;
}

hm_status adjoint_sweep(Model* m, const double* theta, const Sketch* s, const PanelSet& ps, const LevelBufs& lb,
                        const NodeBufs& nb, AdjBufs& a) {
  const int n = m->n, nl = m->nl, levels = m->levels, kc = ps.bw;
  const long s2 = (long)kc * kc;
  HM_CHECK(fill(m, a.wmode, wmode_doubles(m), 0.0));
  // leaf pass
  HM_CHECK(kvjp(m, theta, m->d_ident, n, a.Zb, n, nl, a.wmode));
  HM_CHECK(subtract_adjoint(m, ps.F, kc, levels + 1, m->d_ident, nl, sel_all(), a.Zb, sel_all(), a.Fb, -1.0, nb.t,
                            a.uT));
  double* XS = lb.XS;
  double* Zb = lb.Z;
  double* Qb = lb.Qt;
  double* Yb = lb.Y;
  for (int l = levels; l >= 1; --l) {
    const LeafSel left{1, l}, right{2, l};
    const double* Fl = ps.F + (long)(l - 1) * kc * n;
    const double* Fbl = a.Fb + (long)(l - 1) * kc * n;
    HM_CHECK(side_select(m, Fl, nullptr, XS, kc, l, s->d_k, 1));
    HM_CHECK(side_select(m, Fbl, nullptr, Zb, kc, l, s->d_k, 2));
    // ---- pass 2: C = ((K - sum H) X_S)[right rows]
    HM_CHECK(kvjp(m, theta, XS, n, Zb, n, kc, a.wmode));
    HM_CHECK(subtract_adjoint(m, ps.F, kc, l, XS, kc, left, Zb, right, a.Fb, -1.0, nb.t, a.uT));
    HM_CHECK(kapply_sel(m, theta, Zb, n, kc, a.tmpK, nullptr, nullptr, n, right, left));
    HM_CHECK(subtract_coarser(m, ps, l, Zb, kc, right, left, a.tmpK, nullptr, 0, nb));
    HM_CHECK(side_select(m, Fbl, a.tmpK, Qb, kc, l, s->d_k, 1));
    // ---- QR: Y_bar = (Q_bar - Q sym(Q^T Q_bar)) R^{-T} on every left child at depth l
    const int heap0 = (1 << l) - 1, cnt = 1 << (l - 1);
    ReduceJob rb{XS, n, cs_fixed(0, kc), Qb, n, cs_fixed(0, kc), l, l, nb.g, s2, left};
    HM_CHECK(tree_reduce(m, rb));
    hipLaunchKernelGGL(k_sym_up, dim3(cnt), dim3(256), 0, m->stream, nb.g, nb.w, s2, kc, heap0, 2);
    HM_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_transpose_nodes, dim3(cnt), dim3(256), 0, m->stream, nb.rinv, nb.mfold, s2, kc, heap0, 2);
    HM_LAUNCH_CHECK();
    HM_CHECK(gemm(m->stream, false, true, kc, kc, kc, 1.0, nb.w + heap0 * s2, kc, 2 * s2, nb.rinv + heap0 * s2, kc,
                  2 * s2, 0.0, nb.r1 + heap0 * s2, kc, 2 * s2, cnt));
    HM_CHECK(fill(m, Yb, (long)n * kc, 0.0));
    ExpandJob ey1{Qb, n, cs_fixed(0, kc), Yb, n, cs_fixed(0, kc), nb.mfold, s2, kc, 0, 0, l, l, 1.0, 0.0, left};
    HM_CHECK(tree_expand(m, ey1));
    ExpandJob ey2{XS, n, cs_fixed(0, kc), Yb, n, cs_fixed(0, kc), nb.r1, s2, kc, 0, 0, l, l, -1.0, 1.0, left};
    HM_CHECK(tree_expand(m, ey2));
    // ---- pass 1: Y = ((K - sum H) X_R)[left rows]
    const double* XR = s->d_XR + (long)(l - 1) * kc * n;
    HM_CHECK(kvjp(m, theta, XR, n, Yb, n, kc, a.wmode));
    HM_CHECK(subtract_adjoint(m, ps.F, kc, l, XR, kc, right, Yb, left, a.Fb, -1.0, nb.t, a.uT));
  }
  return HM_OK;
}

}  // namespace hm
