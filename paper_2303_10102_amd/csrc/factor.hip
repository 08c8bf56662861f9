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

namespace hm {

// U_P = N_P [T_a; T_b] for all internal nodes P at depth d (T_c: bw x w, per node
// stride ts; N_P: 2bw x 2bw; U_P: 2bw x w, per node stride us, ld 2bw).
hm_status node_apply_N(Model* m, const double* Nn, const double* T, long ts, double* U, long us, int bw, int w,
                       int d) {
  if (w <= 0) return HM_OK;
  const int P0 = (1 << d) - 1, cnt = 1 << d;
  const long ns = 4L * bw * bw;
  const int m2 = 2 * bw;
  // U = N[:, 0:bw] T_a + N[:, bw:2bw] T_b
  HM_CHECK(gemm(m->stream, false, false, m2, w, bw, 1.0, Nn + P0 * ns, m2, ns, T + (2L * P0 + 1) * ts, bw, 2 * ts,
                0.0, U + P0 * us, m2, us, cnt));
  HM_CHECK(gemm(m->stream, false, false, m2, w, bw, 1.0, Nn + P0 * ns + (long)bw * m2, m2, ns,
                T + (2L * P0 + 2) * ts, bw, 2 * ts, 1.0, U + P0 * us, m2, us, cnt));
  return HM_OK;
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
    ReduceJob rs{f.F, n, cs_block(kc), f.G, n, cs_block(kc), d + 1, d + 1, f.Sn, s2, sel_all()};
    HM_CHECK(tree_reduce(m, rs));
    HM_CHECK(node_lu(m, f.Sn, s2, f.Nn, 4 * s2, f.logdet_node, kc, (1 << d) - 1, 1 << d));
    if (d >= 1) {
      PrecScope prec(m);   // Woodbury panel updates: FP32 under the mixed policy
      ReduceJob rt{f.F, n, cs_block(kc), f.G, n, cs_prefix(kc), d + 1, d + 1, f.nT, ts, sel_all()};
      HM_CHECK(tree_reduce(m, rt));
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
  HM_CHECK(tree_reduce(m, r));
  if (!dFp) {
    ExpandJob e{Fp, n, cs_block(kc), y, n, cs_fixed(0, w), f.nT, ts, kc, 1, 0, 1, levels, alpha, 1.0, sel_all()};
    HM_CHECK(tree_expand(m, e));
    return HM_OK;
  }
  ReduceJob rd{dFp, n, cs_block(kc), x, n, cs_fixed(0, w), 1, levels, f.nU, ts, sel_all()};
  HM_CHECK(tree_reduce(m, rd));
  ExpandJob e{dFp, n, cs_block(kc), y, n, cs_fixed(0, w), f.nT, ts, kc, 1, 0, 1, levels, alpha, 1.0, sel_all()};
  e.A2 = Fp;
  e.T2 = f.nU;
  e.alpha2 = alpha;
  HM_CHECK(tree_expand(m, e));
  return HM_OK;
}

}  // namespace hm
