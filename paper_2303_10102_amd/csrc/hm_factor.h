// Factorisation / trace context: views into one hm_H's device memory.
#pragma once
#include "hm_internal.h"

namespace hm {

struct ParamBufs {
  int kind = 0;            // 0 kappa, 1 alpha, 2 tau2, 3 sigma2
  double* dF = nullptr;    // panel tangent (panel set)
  double* dD = nullptr;    // leaf tangent (leaf-major)
  double* Xi = nullptr;    // Xi_c = B_cc G_c (panel set)
  double* dG = nullptr;    // dG_c = K~_c^{-1} (dF_c - Xi_c) (panel set)
  double* Gh = nullptr;    // dG_c N_P[c,c] (panel set)
  double* Hh = nullptr;    // dG_c N_P[c,sib] S_sib (panel set)
  double* Y = nullptr;     // Dinv_L dD_L (leaf-major)
  double* E = nullptr;     // dF_c^T G_c per non-root node (kc^2)
  double* Psi = nullptr;   // G_c^T Xi_c per non-root node (kc^2)
  double* W = nullptr;     // dG_c^T F_c per non-root node (kc^2)
  double* Vt = nullptr;    // (N_P[c,sib] W_sib)^T per non-root node (kc^2)
  double* PsiP = nullptr;  // assembled G_P^T B G_P per internal node ((2kc)^2)
  double* Lam = nullptr;   // N_P dS_P N_P per internal node ((2kc)^2)
};

struct FactorCtx {
  Model* m = nullptr;
  int kc = 0;
  double* F = nullptr;      // panel set of K~
  double* D = nullptr;      // leaves of K~
  double* G = nullptr;      // G_c = K~_c^{-1} F_c
  double* Dinv = nullptr;
  double* Nn = nullptr;     // per internal node (2kc)^2
  double* Sn = nullptr;     // per node kc^2: F_c^T G_c
  double* logdet_leaf = nullptr;
  double* logdet_node = nullptr;
  double* work_leaf = nullptr;   // nleaves * nl^2
  double* nT = nullptr;     // per node kc x (levels-1) kc
  double* nU = nullptr;     // per node 2kc x (levels-1) kc
  double* Ncc = nullptr;    // per node kc^2: N_P[c,c]
  double* Nx = nullptr;     // per node kc^2: N_P[c,sib] S_sib
  double* tmp_panel = nullptr;  // one panel set of scratch
};

hm_status factorize(FactorCtx& f);
hm_status hsolve(FactorCtx& f, const double* x, double* z, int w);
int solve_max_cols(const FactorCtx& f);
hm_status hmatvec(FactorCtx& f, const double* Dl, const double* Fp, const double* dFp, const double* x, int w,
                  double* y, double alpha, double beta);
hm_status node_apply_N(Model* m, const double* Nn, const double* T, long ts, double* U, long us, int bw, int w,
                       int d);
// the same for every depth d0..d1 in one launch, with w(d) = wa + wb d columns at depth d
hm_status node_apply_range(Model* m, const double* Nn, const double* T, long ts, double* U, long us, int bw, int wa,
                           int wb, int d0, int d1);

}  // namespace hm
