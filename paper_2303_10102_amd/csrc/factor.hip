// Factorisation of K~, log-determinant, solve and H-matvec.
//
// K~ = Dbar (I + U^(tau) V^(tau)T) ... (I + U^(1) V^(1)T)  (Sec. 3.1, eq. "one way factor"; App. C).
// For a node P with children a, b and panels F_a (= Q), F_b (= C) of its
// off-diagonal block K~[a,b] = F_a F_b^T:
//   K~_P = diag(K~_a, K~_b) (I + U_P V_P^T),  U_P = diag(G_a, G_b), G_c = K~_c^{-1} F_c,
//   V_P = [[0, F_a], [F_b, 0]],  I + V_P^T U_P = I + J S_P,  S_P = diag(F_a^T G_a, F_b^T G_b)
// (App. C, eqs. "lvl1 - block1", "factor out lvl2", with the reading U = diag(A1^-1 W, A2^-1 X)).
// Sylvester: log|K~| = sum_L log|D_L| + sum_P log det(I + J S_P)            (Sec. 3.1)
// Woodbury:  (I + U V^T)^{-1} = I - U (I + V^T U)^{-1} V^T = I - U N_P J V^T,
//            N_P = (J + S_P)^{-1}                                           (Sec. 3.1)
// The G_c are formed bottom-up: G = Dbar^{-1} F on every panel, then each node
// P (deepest first) applies its Woodbury factor to the panels of all its
// ancestors restricted to P's rows (the basic factorisation of App. C).
#include <algorithm>
#include <cmath>

#include "hm_build.h"
#include "hm_factor.h"
#include "hm_internal.h"
#include "gemm_core.h"

namespace hm {

// U_P = N_P [T_a; T_b] for every internal node P at depths d0..d1 (T_c: bw x w(d), per
// node stride ts; N_P: 2bw x 2bw; U_P: 2bw x w(d), per node stride us, ld 2bw), with
// w(d) = wa + wb d.  One launch: a 1D grid over the 64 x 64 tiles of every node of
// every depth, each tile one K = 2bw product whose B rows come from T_a (k < bw) and
// T_b (k >= bw).
struct NodeApplyArgs {
  const double* Nn; const double* T; long ts; double* U; long us;
  int bw, wa, wb, d0, d1;
  int tstart[32];   // first tile of depth d0 + i (tstart[d1 - d0 + 1] = total)
};
struct NaA {   // N_P, column-major 2bw x 2bw
  const double* p; int ld, m0, M;
  static constexpr bool kfast = false;
  static constexpr int NR = 1;
  __device__ bool load(int i, int k, double (&v)[1]) const {
    const int r0 = m0 + i;
    const bool ok = r0 < M;
    v[0] = p[(ok ? r0 : 0) + (long)k * ld];
    return ok;
  }
  __device__ double fin(const double (&v)[1]) const { return v[0]; }
};
struct NaB {   // [T_a; T_b], each bw x Nc column-major (ld bw)
  const double* pa; const double* pb; int bw, n0, Nc;
  static constexpr bool kfast = true;
  static constexpr int NR = 1;
  __device__ bool load(int k, int j, double (&v)[1]) const {
    const int c0 = n0 + j;
    const bool ok = c0 < Nc;
    const int c = ok ? c0 : 0;
    v[0] = (k < bw) ? pa[k + (long)c * bw] : pb[(k - bw) + (long)c * bw];
    return ok;
  }
  __device__ double fin(const double (&v)[1]) const { return v[0]; }
};
struct NaC {   // plain store with bounds
  double* p; int ld, m0, n0, M, Nc;
  __device__ void operator()(int i, int j, double v) const {
    const int r = m0 + i, c = n0 + j;
    if (r < M && c < Nc) p[r + (long)c * ld] = v;
  }
};
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) k_node_apply(NodeApplyArgs a) {
  __shared__ double smem[GSMEM];
  const int t = tile_block().x;
  int i = 0;
  while (i < a.d1 - a.d0 && t >= a.tstart[i + 1]) ++i;
  const int d = a.d0 + i;
  const int w = a.wa + a.wb * d, m2 = 2 * a.bw;
  const int mt = (m2 + GBM - 1) / GBM, nt = (w + GBN - 1) / GBN;
  const int r = t - a.tstart[i];
  const int node = r / (mt * nt), rt = r % (mt * nt);
  const int P = (1 << d) - 1 + node;
  const int m0 = (rt % mt) * GBM, n0 = (rt / mt) * GBN;
  NaA la{a.Nn + P * 4L * a.bw * a.bw, m2, m0, m2};
  NaB lb{a.T + (2L * P + 1) * a.ts, a.T + (2L * P + 2) * a.ts, a.bw, n0, w};
  TileAcc acc;
  tile_zero(acc);
  tile_gemm(la, lb, 0, m2, acc, smem);
  tile_store(NaC{a.U + P * a.us, m2, m0, n0, m2, w}, acc);
}

hm_status node_apply_range(Model* m, const double* Nn, const double* T, long ts, double* U, long us, int bw, int wa,
                           int wb, int d0, int d1) {
  if (d1 < d0) return HM_OK;
  if (d1 - d0 + 1 >= 32) {
    set_error("node_apply: too many depths");
    return HM_E_INVAL;
  }
  NodeApplyArgs a{Nn, T, ts, U, us, bw, wa, wb, d0, d1, {}};
  const int mt = ceil_div(2 * bw, GBM);
  long tot = 0;
  for (int d = d0; d <= d1; ++d) {
    a.tstart[d - d0] = (int)tot;
    const int w = wa + wb * d;
    if (w > 0) tot += (long)(1 << d) * mt * ceil_div(w, GBN);
  }
  a.tstart[d1 - d0 + 1] = (int)tot;
  if (tot <= 0) return HM_OK;
  hipLaunchKernelGGL(k_node_apply, dim3((unsigned)tot), dim3(GCfg::NT), 0, m->stream, a);
  HM_LAUNCH_CHECK();
  return HM_OK;
}

// U_P = N_P [T_a; T_b] for all internal nodes P at depth d (w columns)
hm_status node_apply_N(Model* m, const double* Nn, const double* T, long ts, double* U, long us, int bw, int w,
                       int d) {
  if (w <= 0) return HM_OK;
  return node_apply_range(m, Nn, T, ts, U, us, bw, w, 0, d, d);
}

hm_status factorize(FactorCtx& f) {
  Model* m = f.m;
  const int n = m->n, kc = f.kc, levels = m->levels;
  const long s2 = (long)kc * kc;
  HM_CHECK(leaf_factor(m, f.D, f.Dinv, f.logdet_leaf, f.work_leaf));
  // G = Dbar^{-1} F
  HM_CHECK(leaf_gemm(m, f.Dinv, f.F, n, f.G, n, levels * kc, 1.0, 0.0, 0, m->nleaves));
  const long ts = (long)kc * (levels - 1) * kc;  // T_c: kc x (d kc), d <= levels-1
  const long us = 2L * kc * (levels - 1) * kc;
  for (int d = levels - 1; d >= 0; --d) {
    // S_c = F_c^T G_c (node blocks) and, for the Woodbury update of the ancestors'
    // panels, T_c = F_c^T G_c[prefix]: independent products of one launch (S in FP64:
    // it feeds the node factor)
    ReduceJob rs{f.F, n, cs_block(kc), f.G, n, cs_block(kc), d + 1, d + 1, f.Sn, s2, sel_all()};
    ReduceJob rt{f.F, n, cs_block(kc), f.G, n, cs_prefix(kc), d + 1, d + 1, f.nT, ts, sel_all()};
    if (d >= 1 && m->mixed == 0) {   // under the mixed policies T_c is an FP32 product
      const ReduceJob rj[2] = {rs, rt};
      HM_CHECK(tree_reduce_multi(m, rj, 2));
    } else {
      HM_CHECK(tree_reduce(m, rs));
    }
    HM_CHECK(node_lu(m, f.Sn, s2, f.Nn, 4 * s2, f.logdet_node, kc, (1 << d) - 1, 1 << d));
    if (d >= 1) {
      PrecScope prec(m);   // Woodbury panel updates: FP32 under the mixed policy
      if (m->mixed != 0) HM_CHECK(tree_reduce(m, rt));
      HM_CHECK(node_apply_N(m, f.Nn, f.nT, ts, f.nU, us, kc, d * kc, d));
      ExpandJob e{f.G, n, cs_block(kc), f.G, n, cs_prefix(kc), f.nU, us, 2 * kc, 2, kc, d + 1, d + 1, -1.0, 1.0,
                  sel_all()};
      HM_CHECK(tree_expand(m, e));
    }
  }
  return HM_OK;
}

// z = K~^{-1} x (tree order, w columns of ld n; w <= solve_max_cols) by the Woodbury sweep.
hm_status hsolve(FactorCtx& f, const double* x, double* z, int w) {
  Model* m = f.m;
  const int n = m->n, kc = f.kc, levels = m->levels;
  if (w < 1 || w > solve_max_cols(f)) {
    set_error("hsolve: column count out of range");
    return HM_E_INVAL;
  }
  HM_CHECK(leaf_gemm(m, f.Dinv, x, n, z, n, w, 1.0, 0.0, 0, m->nleaves));
  PrecScope prec(m);   // solve sweep: FP32 panels under the mixed policy (refined in FP64 by the caller)
  const long ts = (long)kc * w, us = 2L * kc * w;
  for (int d = levels - 1; d >= 0; --d) {
    ReduceJob r{f.F, n, cs_block(kc), z, n, cs_fixed(0, w), d + 1, d + 1, f.nT, ts, sel_all()};
    HM_CHECK(tree_reduce(m, r));
    HM_CHECK(node_apply_N(m, f.Nn, f.nT, ts, f.nU, us, kc, w, d));
    ExpandJob e{f.G, n, cs_block(kc), z, n, cs_fixed(0, w), f.nU, us, 2 * kc, 2, kc, d + 1, d + 1, -1.0, 1.0,
                sel_all()};
    HM_CHECK(tree_expand(m, e));
  }
  return HM_OK;
}

// the per-node buffers nT, nU hold kc x (levels - 1) kc blocks, i.e. that many columns
int solve_max_cols(const FactorCtx& f) { return f.kc * std::max(1, f.m->levels - 1); }

// y = alpha * B x + beta * y for a symmetric HODLR B with leaf blocks Dl and
// off-diagonal blocks B[a,b] = P1_a P2_b^T + P2_a P1_b^T ... given as the two
// panel sets (Fp, dFp): B[a,b] = dFp_a Fp_b^T + Fp_a dFp_b^T.  If dFp is null,
// B[a,b] = Fp_a Fp_b^T (the K~ case).  x, y: n x w (ld n).
hm_status hmatvec(FactorCtx& f, const double* Dl, const double* Fp, const double* dFp, const double* x, int w,
                  double* y, double alpha, double beta) {
  Model* m = f.m;
  const int n = m->n, kc = f.kc, levels = m->levels;
  HM_CHECK(leaf_gemm(m, Dl, x, n, y, n, w, alpha, beta, 0, m->nleaves));
  const long ts = (long)kc * w;
  ReduceJob r{Fp, n, cs_block(kc), x, n, cs_fixed(0, w), 1, levels, f.nT, ts, sel_all()};
  if (!dFp) {
    HM_CHECK(tree_reduce(m, r));
    ExpandJob e{Fp, n, cs_block(kc), y, n, cs_fixed(0, w), f.nT, ts, kc, 1, 0, 1, levels, alpha, 1.0, sel_all()};
    HM_CHECK(tree_expand(m, e));
    return HM_OK;
  }
  ReduceJob rd{dFp, n, cs_block(kc), x, n, cs_fixed(0, w), 1, levels, f.nU, ts, sel_all()};
  const ReduceJob rj[2] = {r, rd};   // independent: one launch
  HM_CHECK(tree_reduce_multi(m, rj, 2));
  ExpandJob e{dFp, n, cs_block(kc), y, n, cs_fixed(0, w), f.nT, ts, kc, 1, 0, 1, levels, alpha, 1.0, sel_all()};
  e.A2 = Fp;
  e.T2 = f.nU;
  e.alpha2 = alpha;
  HM_CHECK(tree_expand(m, e));
  return HM_OK;
}

}  // namespace hm
