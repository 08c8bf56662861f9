// Reverse-mode gradient of the log-likelihood (adjoint.hip).
#pragma once
#include "hm_build.h"
#include "hm_factor.h"

namespace hm {

// Device buffers of the reverse sweep (owned by the hm_H that holds them).
struct AdjBufs {
  double* Fb = nullptr;     // adjoint of the panel set (panel set)
  double* Gs = nullptr;     // G_c N_P[c,c] for every node c (panel set)
  double* Zb = nullptr;     // adjoint of the leaf-pass sample, n x nl (stacked leaf blocks)
  double* wmode = nullptr;  // per-mode weights of the K-apply products (n)
  double* tmpK = nullptr;   // n x kc
  double* uT = nullptr;     // per node max(kc, nl) x kc
};

// F_bar, Z_bar of -L~ from the factorisation: with Kbar = 1/2 (K~^{-1} - z z^T),
//   F_bar_a = 2 Kbar[a,b] F_b,  leaf blocks Z_bar_L = Kbar[L,L].
hm_status adjoint_init(FactorCtx& f, const double* z, AdjBufs& a);
// Reverse sweep through the leaf pass and the levels (deepest first); accumulates
// the mode weights from which the parameter adjoints follow.
hm_status adjoint_sweep(Model* m, const double* theta, const Sketch* s, const PanelSet& ps, const LevelBufs& lb,
                        const NodeBufs& nb, AdjBufs& a);
// <Ybar, dK/dtheta_j X> for all j through the per-mode weights (kapply.hip).
hm_status kvjp(Model* m, const double* theta, const double* X, int ldx, const double* Yb, int ldb, int c,
               double* wmode);

}  // namespace hm
