// Kernel-variant autotuner for the panel products.
//
// The reduce and expand kernels have variants whose speed depends on the model's
// shapes (leaf size, panel width, tree depth): the expand can give each wavefront
// one or two 16-row blocks and run four or eight wavefronts per workgroup, and the
// reduce splits a leaf's rows over two or four wavefronts.  autotune() times each
// variant on launches of the shapes the iteration issues (a coarser-level subtraction
// over all depths, the leaf pass's wide subtraction, the per-node products of one
// depth, the Cholesky-QR products over one side of every node), with HIP events on the
// model's stream, and keeps the fastest.  Setup-time only: it allocates and frees its own scratch.
#include <algorithm>
#include <vector>

#include "hm_build.h"
#include "hm_internal.h"

namespace hm {

hm_status autotune(Model* m, int kc, double* report) {
  if (kc < 1 || kc > 64 || kc > m->nl) {
    set_error("autotune: panel width must be in 1..min(64, leaf size)");
    return HM_E_INVAL;
  }
  const int n = m->n, levels = m->levels;
  if (levels < 2) {   // no coarser-level or Woodbury panel products to time
    if (report)
      for (int q = 0; q < 8; ++q) report[q] = 0.0;
    return HM_OK;
  }
  const long nodes = (2L << levels) - 1;
  const long s2 = (long)kc * kc;
  const long ts = s2 * (levels - 1);   // T_c: kc x (d kc), d <= levels-1
  std::vector<void*> allocs;
  bool ok = true;
  auto alloc = [&](size_t doubles) -> double* {
    void* p = dev_alloc(m->ctx, doubles * sizeof(double));
    if (!p) {
      ok = false;
      return nullptr;
    }
    allocs.push_back(p);
    return (double*)p;
  };
  const int nl = m->nl;
  const size_t cnts[7] = {(size_t)n * levels * kc, (size_t)n * levels * kc, (size_t)n * kc, (size_t)nodes * ts,
                          (size_t)nodes * 2 * ts,   (size_t)n * nl,           (size_t)nodes * kc * nl};
  double* bufs[7];
  for (int q = 0; q < 7; ++q) bufs[q] = alloc(cnts[q]);
  double *F = bufs[0], *G = bufs[1], *X = bufs[2], *T = bufs[3], *U = bufs[4], *Yw = bufs[5], *Tw = bufs[6];
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (ok) ok = hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
  auto cleanup = [&]() {
    for (void* p : allocs) dev_free(m->ctx, p);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  };
  if (!ok) {
    cleanup();
    set_error("autotune: device allocation failed");
    return HM_E_NOMEM;
  }
  hm_status st = ensure_reduce_ws(m, (size_t)m->nleaves * (levels - 1) * s2);
  for (int q = 0; q < 7 && st == HM_OK; ++q) st = fill(m, bufs[q], (long)cnts[q], 1.0 / (1 + q));
  // launches of the iteration's shapes: the coarser-level subtraction over depths
  // 1..levels-1 (one column block of width kc), the leaf pass's subtraction over all
  // depths (leaf-size width), per depth the Woodbury products (kc x kc node blocks,
  // prefix panels of width (d-1) kc), and per depth the three Cholesky-QR products
  // Q = Y R^{-1} over the left children's rows (half the leaves)
  auto run_expand = [&]() -> hm_status {
    ExpandJob sub{F, n, cs_block(kc), X, n, cs_fixed(0, kc), T, s2, kc, 1, 0, 1, levels - 1, -1.0, 1.0,
                  sel_all()};
    HM_CHECK(tree_expand(m, sub));
    ExpandJob wide{F, n, cs_block(kc), Yw, n, cs_fixed(0, nl), Tw, (long)kc * nl, kc, 1, 0, 1, levels, -1.0, 1.0,
                   sel_all()};
    HM_CHECK(tree_expand(m, wide));
    for (int d = 2; d <= levels; ++d) {
      ExpandJob e{F, n, cs_block(kc), G, n, cs_prefix(kc), U, 2 * ts, 2 * kc, 2, kc, d, d, -1.0, 1.0, sel_all()};
      HM_CHECK(tree_expand(m, e));
    }
    for (int l = 1; l < levels; ++l)
      for (int pass = 0; pass < 3; ++pass) {
        ExpandJob q{F, n, cs_fixed(0, kc), G, n, cs_fixed(0, kc), T, s2, kc, 0, 0, l, l, 1.0, 0.0, LeafSel{1, l}};
        HM_CHECK(tree_expand(m, q));
      }
    return HM_OK;
  };
  auto run_reduce = [&]() -> hm_status {
    ReduceJob sub{F, n, cs_block(kc), X, n, cs_fixed(0, kc), 1, levels - 1, T, s2, sel_all()};
    HM_CHECK(tree_reduce(m, sub));
    for (int d = 1; d <= levels; ++d) {
      ReduceJob rs{F, n, cs_block(kc), G, n, cs_block(kc), d, d, T, s2, sel_all()};
      HM_CHECK(tree_reduce(m, rs));
      if (d >= 2) {
        ReduceJob rt{F, n, cs_block(kc), G, n, cs_prefix(kc), d, d, T, ts, sel_all()};
        HM_CHECK(tree_reduce(m, rt));
      }
    }
    return HM_OK;
  };
  auto time_ms = [&](auto&& fn) -> double {
    if (fn() != HM_OK) return -1.0;   // warm-up
    if (hipEventRecord(e0, m->stream) != hipSuccess) return -1.0;
    for (int r = 0; r < 3; ++r)
      if (fn() != HM_OK) return -1.0;
    if (hipEventRecord(e1, m->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return -1.0;
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return -1.0;
    return ms / 3.0;
  };
  const int saved_rb = m->tune_expand_rb;
  const long saved_nw4 = m->tune_reduce_nw4;
  const int saved_prec = m->panel_prec;
  m->panel_prec = 0;
  double t_rb[3] = {-1.0, -1.0, -1.0}, t_nw[3] = {-1.0, -1.0, -1.0};
  const long thr[3] = {0L, 1024L, 1L << 40};
  if (st == HM_OK) {
    for (int v = 0; v < 3; ++v) {
      m->tune_expand_rb = v + 1;
      t_rb[v] = time_ms(run_expand);
    }
    m->tune_expand_rb = saved_rb;
    for (int v = 0; v < 3; ++v) {
      m->tune_reduce_nw4 = thr[v];
      t_nw[v] = time_ms(run_reduce);
    }
    m->tune_reduce_nw4 = saved_nw4;
  }
  m->panel_prec = saved_prec;
  if (hipStreamSynchronize(m->stream) != hipSuccess && st == HM_OK) {
    set_error("autotune: device error");
    st = HM_E_DEVICE;
  }
  cleanup();
  if (st != HM_OK) return st;
  for (double t : t_rb)
    if (t < 0) { set_error("autotune: a timed launch failed"); return HM_E_DEVICE; }
  for (double t : t_nw)
    if (t < 0) { set_error("autotune: a timed launch failed"); return HM_E_DEVICE; }
  int bestv = 0;
  for (int v = 1; v < 3; ++v)
    if (t_rb[v] < t_rb[bestv]) bestv = v;
  m->tune_expand_rb = bestv + 1;
  int best = 0;
  for (int v = 1; v < 3; ++v)
    if (t_nw[v] < t_nw[best]) best = v;
  m->tune_reduce_nw4 = thr[best];
  if (report) {
    report[0] = t_rb[0];
    report[1] = t_rb[1];
    report[2] = t_rb[2];
    report[3] = t_nw[0];
    report[4] = t_nw[1];
    report[5] = t_nw[2];
    report[6] = m->tune_expand_rb;
    report[7] = (double)m->tune_reduce_nw4;
  }
  return HM_OK;
}

}  // namespace hm
