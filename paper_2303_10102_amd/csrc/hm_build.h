// Buffers shared by the construction routines (build.hip) and their callers.
#pragma once
#include "hm_internal.h"

namespace hm {

// A panel set (see hm_internal.h) and the panel tangents of the real parameters.
struct PanelSet {
  double* F = nullptr;
  double* dF[2] = {nullptr, nullptr};
  int bw = 0;  // block width (columns per depth)
};

// n x w work matrices of one level step; the leaf pass uses the n x nl ones.
struct LevelBufs {
  double* Y = nullptr;
  double* dY[2] = {nullptr, nullptr};
  double* XS = nullptr;
  double* XdS[2] = {nullptr, nullptr};
  double* Z = nullptr;
  double* dZ[2] = {nullptr, nullptr};
  double* Zq[2] = {nullptr, nullptr};
  double* Qt = nullptr;
  double* Zl = nullptr;
  double* dZl[2] = {nullptr, nullptr};
};

// Per-node small matrices (heap index).  t/dt: bw x max(w) each; others bw x bw.
struct NodeBufs {
  double* t = nullptr;
  double* dt[2] = {nullptr, nullptr};
  double *g = nullptr, *r1 = nullptr, *r1i = nullptr, *r2 = nullptr, *r2i = nullptr, *r3 = nullptr,
         *r3i = nullptr, *rinv = nullptr, *w = nullptr, *mfold = nullptr;
};

hm_status fill(Model* m, double* p, long cnt, double v);
hm_status make_identity_stack(Model* m);
// wt: columns of X that also get the tangent subtraction (default: all w)
hm_status subtract_coarser(Model* m, const PanelSet& ps, int l, const double* X, int w, LeafSel xsel,
                           LeafSel ysel, double* Y, double* const* dY, int nr, const NodeBufs& nb, int wt = -1);
hm_status level_step(Model* m, const double* theta, const PanelSet& ps, int l, const double* XR, int w,
                     const int* kblk, int nr, const int* realidx, const LevelBufs& b, const NodeBufs& nb,
                     const int* kblk_host = nullptr);
hm_status leaf_pass(Model* m, const double* theta, const PanelSet& ps, int nr, const int* realidx,
                    const LevelBufs& b, const NodeBufs& nb, double* D, double* const* dD);
hm_status sketch_build(Sketch* s, const double* omega, const double* theta0);
// padding rows and columns of leaf blocks: zero off the diagonal, diag on it (no-op for uniform trees)
hm_status leaf_pad(Model* m, double* D, double diag);
hm_status leaf_factor(Model* m, const double* D, double* Dinv, double* logdet_leaf, double* work);

}  // namespace hm
