// Tree-structured panel products on the HODLR row partition.
//
// Every product the method needs between tall panels (n rows, tree order) and
// per-node small matrices reduces to two shapes over the binary tree:
//   reduce:  out_c = A[c rows, .]^T X[c rows, .]      for all nodes c of some depths
//   expand:  Y[i, .] += sum_d A[i, .] T_{node(i,d)}    for every row i
// Both are computed leaf by leaf (one GEMM tile per leaf and column tile, the
// leaf is the natural row block: all nodes are unions of leaves), so a launch
// always has (#leaves x #column tiles) independent workgroups; reduce then sums
// the per-leaf partials up the tree.  Plus a batched GEMM with the leaf blocks,
// and a plain strided batched GEMM.
#include <hip/hip_ext.h>

#include "hm_internal.h"
#include "gemm_core.h"

namespace hm {

bool prof_on(Model* m, int family) { return m->prof_family == family; }
static hipEvent_t prof_event(Model* m) {
  if (m->ev_used == m->ev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    m->ev_pool.push_back(e);
  }
  return m->ev_pool[m->ev_used++];
}
void prof_begin(Model* m, int family) {
  if (!prof_on(m, family)) return;
  ProfRec r{prof_event(m), prof_event(m), 0.0, 0.0, false};
  if (r.a) (void)hipEventRecord(r.a, m->stream);
  m->prof.push_back(r);
}
void prof_begin_launch(Model* m, int family, hipEvent_t& a, hipEvent_t& b) {
  a = b = nullptr;
  if (!prof_on(m, family)) return;
  ProfRec r{prof_event(m), prof_event(m), 0.0, 0.0, true};
  if (!r.a || !r.b) r.a = r.b = nullptr;   // no events: the launch is not timed
  a = r.a;
  b = r.b;
  m->prof.push_back(r);
}
void prof_end(Model* m, int family, double flops, double bytes) {
  if (!prof_on(m, family) || m->prof.empty()) return;
  ProfRec& r = m->prof.back();
  if (r.b && !r.by_launch) (void)hipEventRecord(r.b, m->stream);
  r.flops = flops;
  r.bytes = bytes;
}

static int count_selected(int nleaves, int levels, LeafSel sel) {
  if (sel.mode == 0) return nleaves;
  return nleaves / 2;  // one side of every node at the selection depth
}

__device__ __forceinline__ bool leaf_selected(int L, int levels, int mode, int depth) {
  if (mode == 0) return true;
  int anc = L >> (levels - depth);
  bool left = (anc & 1) == 0;
  return mode == 1 ? left : !left;
}
// The i-th selected leaf in increasing order, i < count_selected(): the selected
// leaves are every other run of 2^(levels - depth) leaves, starting with the first
// run (left children, mode 1) or the second (right children, mode 2).
__device__ __forceinline__ int selected_leaf(int i, int levels, int mode, int depth) {
  if (mode == 0) return i;
  const int sh = levels - depth;
  return ((2 * (i >> sh) + (mode == 2 ? 1 : 0)) << sh) + (i & ((1 << sh) - 1));
}
static bool sel_valid(const Model* m, LeafSel sel) {
  return sel.mode == 0 || ((sel.mode == 1 || sel.mode == 2) && sel.depth >= 1 && sel.depth <= m->levels);
}

// ----------------------------------------------------------------------------
// generic strided batched GEMM (column-major)
// ----------------------------------------------------------------------------
template <bool TA>
struct LdA {
  const double* p; int ld, m0, M;
  static constexpr bool kfast = TA;
  static constexpr int NR = 1;
  __device__ bool load(int i, int k, double (&v)[1]) const {
    const int r0 = m0 + i;
    const bool ok = r0 < M;
    const int r = ok ? r0 : 0;
    v[0] = TA ? p[k + (long)r * ld] : p[r + (long)k * ld];
    return ok;
  }
  __device__ double fin(const double (&v)[1]) const { return v[0]; }
};
template <bool TB>
struct LdB {
  const double* p; int ld, n0, Nc;
  static constexpr bool kfast = !TB;
  static constexpr int NR = 1;
  __device__ bool load(int k, int j, double (&v)[1]) const {
    const int c0 = n0 + j;
    const bool ok = c0 < Nc;
    const int c = ok ? c0 : 0;
    v[0] = TB ? p[c + (long)k * ld] : p[k + (long)c * ld];
    return ok;
  }
  __device__ double fin(const double (&v)[1]) const { return v[0]; }
};
struct StC {  // C = alpha v + beta C (C not read when beta == 0)
  double* p; int ld, m0, n0, M, Nc; double alpha, beta;
  static constexpr int NP = 1;
  __device__ void pre(int i, int j, double (&o)[1]) const {
    if (beta == 0.0) return;
    const int r = m0 + i, c = n0 + j;
    const bool ok = r < M && c < Nc;
    o[0] = p[(ok ? r : m0) + (long)(ok ? c : n0) * ld];
  }
  __device__ void put(int i, int j, double v, const double (&o)[1]) const {
    const int r = m0 + i, c = n0 + j;
    if (r >= M || c >= Nc) return;
    p[r + (long)c * ld] = (beta == 0.0) ? alpha * v : alpha * v + beta * o[0];
  }
};

template <bool TA, bool TB>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
k_gemm(int M, int Nc, int K, double alpha, const double* A, int lda,
       long sA, const double* B, int ldb, long sB, double beta,
       double* C, int ldc, long sC) {
  __shared__ double smem[GSMEM];
  const TileIdx tb = tile_block();
  int b = tb.z;
  int m0 = tb.x * GBM, n0 = tb.y * GBN;
  LdA<TA> la{A + b * sA, lda, m0, M};
  LdB<TB> lb{B + b * sB, ldb, n0, Nc};
  TileAcc acc;
  tile_zero(acc);
  tile_gemm(la, lb, 0, K, acc, smem);
  tile_store_pre(StC{C + b * sC, ldc, m0, n0, M, Nc, alpha, beta}, acc);
}

hm_status gemm(hipStream_t st, bool ta, bool tb, int M, int Nc, int K, double alpha, const double* A,
               int lda, long sA, const double* B, int ldb, long sB, double beta, double* C, int ldc,
               long sC, int batch) {
  if (M <= 0 || Nc <= 0 || batch <= 0) return HM_OK;
  dim3 grid(ceil_div(M, GBM), ceil_div(Nc, GBN), batch);
  if (!ta && !tb)
    hipLaunchKernelGGL((k_gemm<false, false>), grid, dim3(GCfg::NT), 0, st, M, Nc, K, alpha, A, lda, sA, B,
                       ldb, sB, beta, C, ldc, sC);
  else if (ta && !tb)
    hipLaunchKernelGGL((k_gemm<true, false>), grid, dim3(GCfg::NT), 0, st, M, Nc, K, alpha, A, lda, sA, B,
                       ldb, sB, beta, C, ldc, sC);
  else if (!ta && tb)
    hipLaunchKernelGGL((k_gemm<false, true>), grid, dim3(GCfg::NT), 0, st, M, Nc, K, alpha, A, lda, sA, B,
                       ldb, sB, beta, C, ldc, sC);
  else
    hipLaunchKernelGGL((k_gemm<true, true>), grid, dim3(GCfg::NT), 0, st, M, Nc, K, alpha, A, lda, sA, B,
                       ldb, sB, beta, C, ldc, sC);
  HM_LAUNCH_CHECK();
  return HM_OK;
}

// ----------------------------------------------------------------------------
// reduce: per-leaf partial products, then sums over the leaves of each node
// ----------------------------------------------------------------------------
struct RedArgs {
  const double* A; int lda; ColSpec ac;
  const double* X; int ldx; ColSpec xc;
  int d0, d1, levels, nl;
  double* out; long out_stride;
  double* partial; long pstride;  // per (leaf, depth) stride = wa * max wx
  int sel_mode, sel_depth;
  int only_sel = 0;   // the tree sums skip nodes without selected leaves
  // partials per leaf group: at depth d one partial per min(grp, leaves of a node)
  // consecutive leaves, stored at the group's first leaf (grp 1: per leaf; every
  // selection) -- the stacked-identity path writes groups, the product path leaves
  int grp = 1;
  int wide = 0;   // tree sums: 256 elements per block, one thread per element (else 64, four waves per node's leaves)
  // Up to two further independent jobs in the same launch (grid.z = nj x the products'
  // (leaf, depth) count, job fastest so that every XCD's share of the tiles mixes the
  // jobs; grid.z = jobs of the tree sums): each has its own operands, output, X columns
  // and partial area; everything else is shared.
  int nj = 1;
  const double* jA[2] = {nullptr, nullptr};
  const double* jX[2] = {nullptr, nullptr};
  double* jout[2] = {nullptr, nullptr};
  long jost[2] = {0, 0};
  ColSpec jxc[2] = {};
  double* jpart[2] = {nullptr, nullptr};
  long jpst[2] = {0, 0};
};
// the arguments of job q (0: the launch's own)
__device__ __forceinline__ RedArgs red_job(const RedArgs& a0, int q) {
  RedArgs a = a0;
  if (q > 0) {
    const bool s = q > 1;
    a.A = s ? a0.jA[1] : a0.jA[0];
    a.X = s ? a0.jX[1] : a0.jX[0];
    a.out = s ? a0.jout[1] : a0.jout[0];
    a.out_stride = s ? a0.jost[1] : a0.jost[0];
    a.xc = s ? a0.jxc[1] : a0.jxc[0];
    a.partial = s ? a0.jpart[1] : a0.jpart[0];
    a.pstride = s ? a0.jpst[1] : a0.jpst[0];
  }
  return a;
}

// Reduce with both tall operands fed straight into the matrix cores (P = 0 FP64,
// P = 1 FP32 operands and accumulation for the mixed-precision policy, P = 2 BF16
// operands with FP32 accumulation for its trace panels).  For
// out = A^T X the MFMA's k index runs over rows; lane l of k-group l/16 takes the
// four consecutive rows 4 (l/16) .. 4 (l/16) + 3 of a 16-row group, one per
// MFMA step, so each lane reads 32 contiguous bytes of one column and a 16-lane
// column group covers 128 contiguous bytes.  The output tile is MB x NB blocks of
// 16 x 16 (sized to the real widths, not padded to 64).  NW wavefronts (two, or four
// for launches of few workgroups) split the leaf's rows and combine through LDS; two
// wavefronts per SIMD leave room for two row groups of operands in flight.
template <int P, int MB, int NB, int NW>
__global__ void __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(2, MB * NB > 4 ? 2 : 4)))
k_reduce_direct(RedArgs a0) {
  using MP = MfmaPrec<P>;
  using T = typename MP::T;
  __shared__ double red[(NW - 1) * MB * NB * 4 * 64];
  // grid.z enumerates (selected leaf, depth, job), job fastest, then depth
  const TileIdx tb = tile_block();
  const int zz = tb.z / a0.nj, q = tb.z - zz * a0.nj;
  const RedArgs a = red_job(a0, q);
  const int ndep = a.d1 - a.d0 + 1;
  const int L = selected_leaf(zz / ndep, a.levels, a.sel_mode, a.sel_depth);
  const int d = a.d0 + zz % ndep;
  const int wa = a.ac.w0, wx = a.xc.w(d);
  const int m0 = tb.x * (16 * MB), n0 = tb.y * (16 * NB);
  if (m0 >= wa || n0 >= wx) return;
  const long r0 = (long)L * a.nl;
  const double* Ab = a.A + r0 + (long)(a.ac.c0(d) + m0) * a.lda;
  const double* Xb = a.X + r0 + (long)(a.xc.c0(d) + n0) * a.ldx;
  // the wavefront index is uniform, so the row loop runs on scalar registers
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  const int hrows = ((a.nl + 16 * NW - 1) / (16 * NW)) * 16;   // rows per wavefront, a multiple of 16
  const int rbeg = wave * hrows, rend = min(a.nl, rbeg + hrows);
  typename MP::V acc[MB][NB];
#pragma unroll
  for (int i = 0; i < MB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[i][j] = MP::zero();
  // Lane (li, lk) reads rows g + 4 lk .. g + 4 lk + 3 of its columns: 32 contiguous
  // bytes.  The loads are branch-free (a column past the operand reads the tile's first
  // column, a row group past the range reads rows 0..3) and zeroed where they are used,
  // so each chunk's loads go out as wide loads together.
  const double* Ac[MB];
  const double* Xc[NB];
  bool aok[MB], xok[NB];
#pragma unroll
  for (int i = 0; i < MB; ++i) {
    aok[i] = m0 + 16 * i + li < wa;
    Ac[i] = Ab + (long)(aok[i] ? 16 * i + li : 0) * a.lda;
  }
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    xok[j] = n0 + 16 * j + li < wx;
    Xc[j] = Xb + (long)(xok[j] ? 16 * j + li : 0) * a.ldx;
  }
  // Two register sets alternate (the row-group loop is unrolled by two): the loads of
  // the next group are issued before the current one is multiplied, so each wavefront
  // keeps one group in flight while the matrix cores work.  An odd group count runs
  // one empty group (every row out of range, operands zero); the loop's last loads
  // re-read the final group and are not used.
  struct Grp {
    double ar[MB][4], xr[NB][4];
  };
  const int ngrp = (rend - rbeg + 15) >> 4;
  auto load_grp = [&](int t, Grp& u) {
    const int rr = rbeg + 16 * min(t, ngrp - 1) + 4 * lk;
    // a group of 4 rows inside the leaf (the layout keeps nl a multiple of 4, so a
    // group never straddles the leaf's end; past the range it reads rows 0..3)
    const long rl = (rr + 3 < a.nl) ? rr : 0;
#pragma unroll
    for (int i = 0; i < MB; ++i) {
      const double* pa = Ac[i] + rl;
#pragma unroll
      for (int q = 0; q < 4; ++q) u.ar[i][q] = pa[q];
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const double* px = Xc[j] + rl;
#pragma unroll
      for (int q = 0; q < 4; ++q) u.xr[j][q] = px[q];
    }
  };
  auto mma_grp = [&](int t, const Grp& u) {
    const int rr = rbeg + 16 * t + 4 * lk;
    if constexpr (P == 2) {
      // the lane's four rows are the four k of one BF16 instruction
      auto pick = [&](bool ok, const double (&v)[4], int q) { return (ok && rr + q < rend) ? (float)v[q] : 0.0f; };
      hm_v4bf av[MB], xv[NB];
#pragma unroll
      for (int i = 0; i < MB; ++i)
        av[i] = bf16x4(pick(aok[i], u.ar[i], 0), pick(aok[i], u.ar[i], 1), pick(aok[i], u.ar[i], 2),
                       pick(aok[i], u.ar[i], 3));
#pragma unroll
      for (int j = 0; j < NB; ++j)
        xv[j] = bf16x4(pick(xok[j], u.xr[j], 0), pick(xok[j], u.xr[j], 1), pick(xok[j], u.xr[j], 2),
                       pick(xok[j], u.xr[j], 3));
#pragma unroll
      for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) acc[i][j] = MP::mfma16(av[i], xv[j], acc[i][j]);
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const bool rok = rr + q < rend;
        T av[MB], xv[NB];
#pragma unroll
        for (int i = 0; i < MB; ++i) av[i] = (aok[i] && rok) ? (T)u.ar[i][q] : (T)0;
#pragma unroll
        for (int j = 0; j < NB; ++j) xv[j] = (xok[j] && rok) ? (T)u.xr[j][q] : (T)0;
#pragma unroll
        for (int i = 0; i < MB; ++i)
#pragma unroll
          for (int j = 0; j < NB; ++j) acc[i][j] = MP::mfma(av[i], xv[j], acc[i][j]);
      }
    }
  };
  if (ngrp > 0) {
    Grp U0, U1;
    load_grp(0, U0);
    for (int t = 0; t < ngrp; t += 2) {
      load_grp(t + 1, U1);
      mma_grp(t, U0);
      load_grp(t + 2, U0);
      mma_grp(t + 1, U1);
    }
  }
  if (wave > 0) {
    double* slot = red + (wave - 1) * (MB * NB * 4 * 64);
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
      for (int j = 0; j < NB; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) slot[((i * NB + j) * 4 + v) * 64 + lane] = acc[i][j][v];
  }
  __syncthreads();
  if (wave != 0) return;
  double* dst;
  if (d == a.levels) {
    dst = a.out + ((1 << d) - 1 + L) * a.out_stride;
  } else {
    dst = a.partial + ((long)L * ndep + (d - a.d0)) * a.pstride;
  }
#pragma unroll
  for (int i = 0; i < MB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int mm = m0 + 16 * i + MP::row(v, lk), nn = n0 + 16 * j + li;
        double t = acc[i][j][v];
#pragma unroll
        for (int w = 1; w < NW; ++w) t += red[(w - 1) * (MB * NB * 4 * 64) + ((i * NB + j) * 4 + v) * 64 + lane];
        if (mm < wa && nn < wx) dst[mm + (long)nn * wa] = t;
      }
}

template <int P, int MB, int NW>
static void launch_reduce_direct(Model* m, int nb, dim3 grid, const RedArgs& a) {
  if (nb == 1) hipLaunchKernelGGL((k_reduce_direct<P, MB, 1, NW>), grid, dim3(64 * NW), 0, m->stream, a);
  else if (nb == 2) hipLaunchKernelGGL((k_reduce_direct<P, MB, 2, NW>), grid, dim3(64 * NW), 0, m->stream, a);
  else hipLaunchKernelGGL((k_reduce_direct<P, MB, 3, NW>), grid, dim3(64 * NW), 0, m->stream, a);
}
template <int P>
static void launch_reduce_prec(Model* m, int mb, int nb, bool four, dim3 grid, const RedArgs& a) {
  if (four) {
    if (mb == 1) launch_reduce_direct<P, 1, 4>(m, nb, grid, a);
    else if (mb == 2) launch_reduce_direct<P, 2, 4>(m, nb, grid, a);
    else launch_reduce_direct<P, 3, 4>(m, nb, grid, a);
  } else {
    if (mb == 1) launch_reduce_direct<P, 1, 2>(m, nb, grid, a);
    else if (mb == 2) launch_reduce_direct<P, 2, 2>(m, nb, grid, a);
    else launch_reduce_direct<P, 3, 2>(m, nb, grid, a);
  }
}

// Sum the per-leaf partials into every node of depths d0..min(d1, levels-1):
// grid.y enumerates those nodes (depth-major), grid.x element chunks of 64.  The
// four wavefronts of a block split the node's leaves (each issuing eight
// independent loads per step), then combine through LDS; partials of unselected
// leaves are never read.
__global__ void __launch_bounds__(256) k_reduce_tree(RedArgs a0, int dlast) {
  __shared__ double red[4][64];
  const RedArgs a = red_job(a0, (int)blockIdx.z);   // grid.z enumerates the jobs
  const int ndep = a.d1 - a.d0 + 1;
  // node enumeration: depth d contributes 2^d nodes, starting at depth d0
  int t = blockIdx.y;
  int d = a.d0;
  while (d < dlast && t >= (1 << d)) {
    t -= (1 << d);
    ++d;
  }
  const int idx = t;
  if (a.only_sel && a.sel_mode != 0 && d >= a.sel_depth) {
    // below the selection depth a node's leaves are all selected or all not
    const bool left = ((idx >> (d - a.sel_depth)) & 1) == 0;
    if (left != (a.sel_mode == 1)) return;
  }
  const int wa = a.ac.w0, wx = a.xc.w(d);
  const int ne = wa * wx;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int span = 1 << (a.levels - d);
  const int L0 = idx * span;
  const int G = a.grp < span ? a.grp : span;   // partials at every G-th leaf of the node
  const int nk = span / G;
  const long stride = (long)ndep * a.pstride;
  if (a.wide) {
    // 256 elements per block, each thread sums its element over the node's groups alone
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= ne) return;
    const double* base = a.partial + (long)(d - a.d0) * a.pstride + e;
    double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int k = 0;
    for (; k + 7 < nk; k += 8) {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int Lq = L0 + (k + q) * G;
        if (leaf_selected(Lq, a.levels, a.sel_mode, a.sel_depth)) acc[q] += base[(long)Lq * stride];
      }
    }
    for (; k < nk; ++k) {
      const int L = L0 + k * G;
      if (leaf_selected(L, a.levels, a.sel_mode, a.sel_depth)) acc[0] += base[(long)L * stride];
    }
    const int heap = (1 << d) - 1 + idx;
    a.out[heap * a.out_stride + e] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
    return;
  }
  const int e = blockIdx.x * 64 + lane;
  if (blockIdx.x * 64 >= ne) return;
  const double* base = a.partial + (long)(d - a.d0) * a.pstride + e;
  double s = 0.0;
  if (e < ne) {
    // wave wv takes groups wv, wv + 4, ... of the node (first leaf L0 + k G)
    double acc[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] = 0.0;
    int k = wv;
    for (; k + 28 < nk; k += 32) {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int Lq = L0 + (k + 4 * q) * G;
        if (leaf_selected(Lq, a.levels, a.sel_mode, a.sel_depth)) acc[q] += base[(long)Lq * stride];
      }
    }
    for (; k < nk; k += 4) {
      const int L = L0 + k * G;
      if (leaf_selected(L, a.levels, a.sel_mode, a.sel_depth)) acc[0] += base[(long)L * stride];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) s += acc[q];
  }
  red[wv][lane] = s;
  __syncthreads();
  if (wv == 0 && e < ne) {
    const int heap = (1 << d) - 1 + idx;
    a.out[heap * a.out_stride + e] = red[0][lane] + red[1][lane] + red[2][lane] + red[3][lane];
  }
}

// Reduce against the stacked identity S (the leaf pass): A[c]^T S[c] is the sum over
// the leaves of c of A's leaf blocks (transposed), no product needed.  A workgroup sums
// the blocks of a group of G(d) = min(grp, 2^(levels-d)) consecutive leaves (one node's
// at the deep depths) and writes the sum, through an LDS transpose when `trans`, into
// the partial layout of the product path at the group's first leaf (element (i, j) at
// i + j * rows_out), or at the leaf depth straight into the leaf's output;
// k_reduce_tree then sums the groups of each node.  grid.z enumerates (depth, group),
// depth-major, nleaves / G(d) groups per depth.
__global__ void __launch_bounds__(256) k_leaf_blocks(const double* P, int ldp, ColSpec pc, int d0, int d1,
                                                     int levels, int nl, int nleaves, int w, int trans, int grp,
                                                     double* out, long out_stride, double* partial, long pstride) {
  __shared__ double tile[64][65];
  const int ndep = d1 - d0 + 1;
  int d = d0, zr = blockIdx.z;
  for (;;) {
    const int span = 1 << (levels - d);
    const int ng = nleaves / (grp < span ? grp : span);
    if (zr < ng || d >= d1) break;
    zr -= ng;
    ++d;
  }
  const int span = 1 << (levels - d);
  const int G = grp < span ? grp : span;
  const int L0 = zr * G;
  const int j0 = blockIdx.x * 64, m0 = blockIdx.y * 64;
  double acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = 0.0;
  for (int t = 0; t < G; ++t) {
    const double* src = P + (long)(L0 + t) * nl + (long)pc.c0(d) * ldp;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int e = threadIdx.x + 256 * q;
      const int jj = e % 64, cc = e / 64;
      const int j = j0 + jj, mm = m0 + cc;
      if (j < nl && mm < w) acc[q] += src[j + (long)mm * ldp];
    }
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = threadIdx.x + 256 * q;
    tile[e / 64][e % 64] = acc[q];
  }
  __syncthreads();
  const int L = L0;
  // the leaf depth (groups of one) goes straight to the output; every other depth through
  // the partials, which k_reduce_tree sums (one group per node when G covers it)
  double* dst = (d == levels) ? out + ((1 << d) - 1 + L) * out_stride
                              : partial + ((long)L * ndep + (d - d0)) * pstride;
  for (int q = 0; q < 16; ++q) {
    const int e = threadIdx.x + 256 * q;
    if (trans) {   // out block w x nl: element (mm, j) at mm + j w
      const int cc = e % 64, jj = e / 64;
      const int j = j0 + jj, mm = m0 + cc;
      if (j < nl && mm < w) dst[mm + (long)j * w] = tile[cc][jj];
    } else {       // out block nl x w: element (j, mm) at j + mm nl
      const int jj = e % 64, cc = e / 64;
      const int j = j0 + jj, mm = m0 + cc;
      if (j < nl && mm < w) dst[j + (long)mm * nl] = tile[cc][jj];
    }
  }
}

hm_status ensure_reduce_ws(Model* m, size_t doubles) {
  if (doubles <= m->red_doubles) return HM_OK;
  // setup calls only; the old buffer may still be read by queued work
  if (m->d_red) {
    HM_HIP(hipStreamSynchronize(m->stream));
    dev_free(m->ctx, m->d_red);
  }
  m->d_red = nullptr;
  m->red_doubles = 0;
  m->d_red = (double*)dev_alloc(m->ctx, doubles * sizeof(double));
  if (!m->d_red) {
    set_error("tree_reduce workspace allocation failed");
    return HM_E_NOMEM;
  }
  m->red_doubles = doubles;
  return HM_OK;
}

// Jobs that can share one launch: same row operand layout, depths and selection,
// products only (no identity operand), at most three.
static bool reduce_jobs_compatible(Model* m, const ReduceJob* js, int nj) {
  if (nj < 2 || nj > 3) return false;
  auto is_ident = [&](const double* p) { return p == m->d_ident; };
  for (int q = 0; q < nj; ++q) {
    const ReduceJob& a = js[q];
    const ReduceJob& b = js[0];
    if (is_ident(a.A) || is_ident(a.X)) return false;
    if (a.lda != b.lda || a.ldx != b.ldx || a.d0 != b.d0 || a.d1 != b.d1 || a.sel.mode != b.sel.mode ||
        a.sel.depth != b.sel.depth || a.ac.base != b.ac.base || a.ac.stride != b.ac.stride ||
        a.ac.w0 != b.ac.w0 || a.ac.grow != b.ac.grow || a.only_selected != b.only_selected)
      return false;
  }
  return true;
}

hm_status tree_reduce(Model* m, const ReduceJob& j) { return tree_reduce_multi(m, &j, 1); }

hm_status tree_reduce_multi(Model* m, const ReduceJob* js, int nj) {
  if (nj <= 0) return HM_OK;
  if (nj > 3) {
    for (int q = 0; q < nj; ++q) HM_CHECK(tree_reduce_multi(m, js + q, 1));
    return HM_OK;
  }
  const ReduceJob& j = js[0];
  for (int q = 0; q < nj; ++q) {
    if (js[q].d0 < 1 || js[q].d1 > m->levels || js[q].d0 > js[q].d1) {
      set_error("tree_reduce: bad depth range");
      return HM_E_INVAL;
    }
    if (!sel_valid(m, js[q].sel)) {
      set_error("tree_reduce: bad leaf selection");
      return HM_E_INVAL;
    }
  }
  const int ndep = j.d1 - j.d0 + 1;
  const int wa = j.ac.w0;
  // per-job widest X block and partial area (leaves x depths x wa x wx)
  int wxq[3] = {0, 0, 0};
  size_t offq[3] = {0, 0, 0};
  size_t need = 0;
  for (int q = 0; q < nj; ++q) {
    for (int d = js[q].d0; d <= js[q].d1; ++d) wxq[q] = std::max(wxq[q], js[q].xc.w(d));
    offq[q] = need;
    need += (size_t)m->nleaves * ndep * wa * wxq[q];
  }
  if (nj > 1 && (!reduce_jobs_compatible(m, js, nj) || need > m->red_doubles)) {
    for (int q = 0; q < nj; ++q) HM_CHECK(tree_reduce_multi(m, js + q, 1));
    return HM_OK;
  }
  int wxmax = 0;
  for (int q = 0; q < nj; ++q) wxmax = std::max(wxmax, wxq[q]);
  if (wa <= 0 || wxmax <= 0) return HM_OK;
  RedArgs a{j.A, j.lda, j.ac, j.X, j.ldx, j.xc, j.d0, j.d1, m->levels, m->nl, j.out, j.out_stride,
            m->d_red, (long)wa * wxq[0], j.sel.mode, j.sel.depth};
  a.only_sel = j.only_selected ? 1 : 0;
  for (int q = 1; q < nj; ++q) {
    a.jA[q - 1] = js[q].A;
    a.jX[q - 1] = js[q].X;
    a.jout[q - 1] = js[q].out;
    a.jost[q - 1] = js[q].out_stride;
    a.jxc[q - 1] = js[q].xc;
    a.jpart[q - 1] = m->d_red + offq[q];
    a.jpst[q - 1] = (long)wa * wxq[q];
  }
  if (need > m->red_doubles) {
    set_error("tree_reduce: partial workspace too small (" + std::to_string(need) + " > " +
              std::to_string(m->red_doubles) + ")");
    return HM_E_INVAL;
  }
  const bool pf = prof_on(m, PF_REDUCE);
  if (pf) prof_begin(m, PF_REDUCE);
  auto is_ident = [&](const double* p, const ColSpec& c) {
    return p == m->d_ident && c.base == 0 && c.stride == 0 && c.w0 == m->nl && c.grow == 0;
  };
  const bool xid = nj == 1 && is_ident(j.X, j.xc) && j.sel.mode == 0;
  const bool aid = nj == 1 && is_ident(j.A, j.ac) && j.sel.mode == 0 && j.xc.grow == 0;
  const int nsel = count_selected(m->nleaves, m->levels, j.sel);
  a.nj = nj;
  if (xid || aid) {
    // sums of leaf blocks (no product): A[c]^T S[c] (xid) or S[c]^T X[c] (aid)
    const double* P = xid ? j.A : j.X;
    const int ldp = xid ? j.lda : j.ldx;
    const ColSpec pc = xid ? j.ac : j.xc;
    const int w = xid ? wa : j.xc.w0;
    // leaf groups of up to 8: a copy per leaf is cheap, the partials it saves are not
    a.grp = 8;
    long zc = 0;
    for (int d = j.d0; d <= j.d1; ++d) zc += m->nleaves / std::min(a.grp, 1 << (m->levels - d));
    dim3 g(ceil_div(m->nl, 64), ceil_div(w, 64), (unsigned)zc);
    hipLaunchKernelGGL(k_leaf_blocks, g, dim3(256), 0, m->stream, P, ldp, pc, j.d0, j.d1, m->levels, m->nl,
                       m->nleaves, w, xid ? 1 : 0, a.grp, j.out, j.out_stride, m->d_red, (long)wa * wxmax);
  } else {
    // output tile sized to the widths: MB x NB blocks of 16
    auto blocks = [](int w) {   // up to 3 x 3 blocks per tile keeps two wavefronts per SIMD
      const int nbk = ceil_div(w, 16);
      if (nbk <= 3) return nbk;
      return (nbk % 3 == 0) ? 3 : (nbk % 2 == 0 ? 2 : 3);
    };
    const int mb = blocks(wa), nb = blocks(wxmax);
    dim3 grid(ceil_div(wa, 16 * mb), ceil_div(wxmax, 16 * nb), nsel * ndep * nj);
    // few workgroups (e.g. one depth of per-leaf products): split each leaf's rows
    // over four wavefronts instead of two
    const long wgs = (long)grid.x * grid.y * grid.z;
    const bool four = wgs < m->tune_reduce_nw4;
    if (m->panel_prec == 2) launch_reduce_prec<2>(m, mb, nb, four, grid, a);
    else if (m->panel_prec == 1) launch_reduce_prec<1>(m, mb, nb, four, grid, a);
    else launch_reduce_prec<0>(m, mb, nb, four, grid, a);
  }
  HM_LAUNCH_CHECK();
  if (pf) {
    const double rows = (double)nsel * m->nl;
    double fl = 0.0, by = 0.0;
    for (int q = 0; q < nj; ++q)
      for (int d = j.d0; d <= j.d1; ++d) {
        const int wx = js[q].xc.w(d);
        if (xid || aid) {   // a copy of the non-identity operand's leaf blocks
          by += 16.0 * rows * (xid ? wa : wx);
          continue;
        }
        fl += 2.0 * rows * wa * wx;
        by += 8.0 * (rows * wa + rows * wx + (rows / m->nl) * wa * wx);
      }
    prof_end(m, PF_REDUCE, fl, by);
  }
  const int dlast = std::min(j.d1, m->levels - 1);
  if (dlast >= j.d0) {
    int nodes = 0, nemax = 0;
    for (int d = j.d0; d <= dlast; ++d) {
      nodes += 1 << d;
      for (int q = 0; q < nj; ++q) nemax = std::max(nemax, wa * js[q].xc.w(d));
    }
    if (nemax > 0) {
      // one thread per element pays off for the grouped partials (few per node); with a
      // partial per leaf the shallow nodes' sums need the four waves (measured slower
      // otherwise: tree sums 1.29 -> 1.74 ms per iteration)
      a.wide = a.grp > 1 ? 1 : 0;
      dim3 g2(ceil_div(nemax, a.wide ? 256 : 64), nodes, nj);
      hipLaunchKernelGGL(k_reduce_tree, g2, dim3(256), 0, m->stream, a, dlast);
      HM_LAUNCH_CHECK();
    }
  }
  return HM_OK;
}

// ----------------------------------------------------------------------------
// expand: Y[i, yc(d)] = beta Y + alpha sum_d A[i, ac(d)] T_{s(c_d)}
// ----------------------------------------------------------------------------
struct ExpArgs {
  const double* A; int lda; ColSpec ac;
  double* Y; int ldy; ColSpec yc;
  const double* T; long t_stride; int ldt; int tmode; int half_off;
  int d0, d1, levels, nl;
  double alpha, beta;
  int ylo, yhi;  // union of the output columns
  int sel_mode, sel_depth;
  const double* A2; const double* T2; double t2_scale;   // second source (A2 null: none)
  // Up to two further independent jobs in the same launch (grid.z = nj x the selected
  // leaves, job fastest so that every XCD's share of the tiles mixes the jobs): their
  // own A, Y, output columns, T and second source; everything else is shared.
  int nj = 1;
  const double* jA[2] = {nullptr, nullptr};
  double* jY[2] = {nullptr, nullptr};
  ColSpec jyc[2] = {};
  int jyhi[2] = {0, 0};
  const double* jT[2] = {nullptr, nullptr};
  const double* jA2[2] = {nullptr, nullptr};
  const double* jT2[2] = {nullptr, nullptr};
  double jt2s[2] = {0.0, 0.0};
};
// the arguments of job q (0: the launch's own)
__device__ __forceinline__ ExpArgs exp_job(const ExpArgs& a0, int q) {
  ExpArgs a = a0;
  if (q > 0) {
    const bool s = q > 1;
    a.A = s ? a0.jA[1] : a0.jA[0];
    a.Y = s ? a0.jY[1] : a0.jY[0];
    a.yc = s ? a0.jyc[1] : a0.jyc[0];
    a.yhi = s ? a0.jyhi[1] : a0.jyhi[0];
    a.T = s ? a0.jT[1] : a0.jT[0];
    a.A2 = s ? a0.jA2[1] : a0.jA2[0];
    a.T2 = s ? a0.jT2[1] : a0.jT2[0];
    a.t2_scale = s ? a0.jt2s[1] : a0.jt2s[0];
  }
  return a;
}

// Expand with the tall operand fed straight into the matrix cores (P = 0 FP64,
// P = 1 FP32 operands and accumulation for the mixed-precision policy, P = 2 BF16
// operands with FP32 accumulation for its trace panels).  The
// product is formed transposed, D = T^T A^T (16 output columns x 16 rows per
// MFMA block), so that
//   * the B operand of v_mfma_f64_16x16x4 (lane l: row l%16, k l/16) is read from
//     the column-major panel without LDS: each group of 16 lanes reads 128
//     contiguous bytes of one column;
//   * the small per-node block T goes through LDS, once per workgroup and unit;
//   * the accumulator (lane l, element v: output column 4v + l/16, row l%16) is
//     stored as 128-byte runs of one output column.
// Work is a sequence of units (segment d, 32-deep k chunk).  The panel and T
// loads of the next unit are issued before the current unit is computed, and the
// workgroup barriers wait on LDS traffic only, so those loads stay in flight.
// Workgroup: NWV wavefronts x RB blocks of 16 rows of one leaf, up to 64 output
// columns (16 NB); the T block of a unit is staged once for all of them.
constexpr int EXK = 32;   // k chunk of one unit

__device__ __forceinline__ void lds_barrier() {
  // LDS stores of this wavefront complete, then the workgroup barrier; global loads
  // in flight are not waited for
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

__device__ __forceinline__ bool exp_seg_active(const ExpArgs& a, int d, int j0, int tw) {
  const int yc0 = a.yc.c0(d), wy = a.yc.w(d);
  return wy > 0 && j0 < yc0 + wy && j0 + tw > yc0;
}
// next unit after (src, d, k0); d < d0 means "before the first" of that source.  The
// units of the second source (if any) follow those of the first.
__device__ __forceinline__ bool exp_next_unit(const ExpArgs& a, int j0, int tw, int& src, int& d, int& k0) {
  if (d >= a.d0) {
    k0 += EXK;
    if (k0 < a.ac.w0) return true;
  }
  for (;;) {
    for (++d; d <= a.d1; ++d)
      if (exp_seg_active(a, d, j0, tw)) {
        k0 = 0;
        return true;
      }
    if (src != 0 || !a.A2) return false;
    src = 1;
    d = a.d0 - 1;
  }
}
__device__ __forceinline__ const double* exp_T(const ExpArgs& a, int src, int L, int d) {
  const int c = L >> (a.levels - d);
  const int heap = (1 << d) - 1 + c;
  int sel = heap, roff = 0;
  if (a.tmode == 1) sel = (heap & 1) ? heap + 1 : heap - 1;
  else if (a.tmode == 2) { sel = (heap - 1) >> 1; roff = (c & 1) ? a.half_off : 0; }
  return (src ? a.T2 : a.T) + sel * a.t_stride + roff;
}

template <int P, int NB, int RB, int NWV>
__global__ void __launch_bounds__(64 * NWV) k_expand_direct(ExpArgs a0) {
  constexpr int NT = 64 * NWV;
  constexpr int EXT = EXK * 64 / NT;
  constexpr int CS = NT / EXK;   // T columns staged per pass of the workgroup
  using MP = MfmaPrec<P>;
  using T = typename MP::T;
  __shared__ T Ts[2][EXK * 65];
  // grid.z enumerates (selected leaf, job), job fastest
  const TileIdx tb = tile_block();
  const int zl = tb.z / a0.nj, q = tb.z - zl * a0.nj;
  const ExpArgs a = exp_job(a0, q);
  const int L = selected_leaf(zl, a.levels, a.sel_mode, a.sel_depth);
  constexpr int TW = 16 * NB;   // tile width in output columns
  const int m0 = tb.x * (16 * RB * NWV);
  const int j0 = a.ylo + tb.y * TW;
  if (j0 >= a.yhi) return;   // a job narrower than the launch's widest
  const long r0 = (long)L * a.nl;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int li = lane & 15, lk = lane >> 4;
  // RB row blocks of 16 per wavefront: every T value read from LDS feeds RB MFMAs.
  // Rows past the leaf read row 0 (a valid address) and are never stored.
  int row[RB], rowc[RB];
  bool rok[RB];
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    row[r] = m0 + wave * (16 * RB) + 16 * r + li;
    rok[r] = row[r] < a.nl;
    rowc[r] = rok[r] ? row[r] : 0;
  }
  const int wk = a.ac.w0;
  const int ldt = a.ldt;
  typename MP::V acc[RB][NB];
#pragma unroll
  for (int r = 0; r < RB; ++r)
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[r][b] = MP::zero();

  // Raw loads of one unit (segment d, k chunk k0), free of branches: an element
  // outside the operand reads a valid address and is zeroed where it is used, so
  // every load of the unit is in flight at once and the waits count exactly.
  struct Unit {
    double av[RB][EXK / 4];
    double tv[EXT];
  };
  const int kk_t = tid % EXK, cc_t = tid / EXK;   // this thread's T elements: (kk_t, cc_t + CS q)
  auto load_unit = [&](int src, int d, int k0, Unit& u) {
    const double* Ab = (src ? a.A2 : a.A) + r0 + (long)a.ac.c0(d) * a.lda;
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
      for (int s = 0; s < EXK / 4; ++s) {
        // FP64 / FP32: k = 4 s + lk (one k per instruction); BF16: the four consecutive k
        // 16 (s / 4) + 4 lk + s % 4 of one 16-deep instruction
        const int k = k0 + (P == 2 ? 16 * (s >> 2) + 4 * lk + (s & 3) : 4 * s + lk);
        u.av[r][s] = Ab[rowc[r] + (long)(k < wk ? k : 0) * a.lda];
      }
    const double* Tb = exp_T(a, src, L, d);
    const int cbase = j0 - a.yc.c0(d), wy = a.yc.w(d);
    const int k = k0 + kk_t;
#pragma unroll
    for (int q = 0; q < EXT; ++q) {
      const int col = cbase + cc_t + CS * q;
      const bool ok = k < wk && col >= 0 && col < wy;
      u.tv[q] = Tb[(ok ? k : 0) + (long)(ok ? col : 0) * ldt];
    }
  };
  auto stash_T = [&](const Unit& u, int src, int d, int k0, T* buf) {
    const int cbase = j0 - a.yc.c0(d), wy = a.yc.w(d);
    const bool kok = k0 + kk_t < wk;
    const double sc = src ? a.t2_scale : 1.0;
#pragma unroll
    for (int q = 0; q < EXT; ++q) {
      const int cc = cc_t + CS * q;
      const int col = cbase + cc;
      const bool ok = kok && cc < TW && col >= 0 && col < wy;
      buf[kk_t * 65 + cc] = ok ? (T)(sc * u.tv[q]) : (T)0;
    }
  };
  auto mfma_unit = [&](const Unit& u, int k0, const T* buf) {
    const int kn = min(EXK, wk - k0);
    if constexpr (P == 2) {
#pragma unroll
      for (int c = 0; c < EXK / 16; ++c) {
        if (16 * c < kn) {
          const int kb = 16 * c + 4 * lk;   // this lane's first k of the instruction
          hm_v4bf av[RB];
#pragma unroll
          for (int r = 0; r < RB; ++r) {
            float x[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) x[q] = (kb + q < kn) ? (float)u.av[r][4 * c + q] : 0.0f;
            av[r] = bf16x4(x[0], x[1], x[2], x[3]);
          }
#pragma unroll
          for (int b = 0; b < NB; ++b) {
            const T* tp = buf + kb * 65 + b * 16 + li;   // k >= kn is staged as zero
            const hm_v4bf tv = bf16x4(tp[0], tp[65], tp[130], tp[195]);
#pragma unroll
            for (int r = 0; r < RB; ++r) acc[r][b] = MP::mfma16(tv, av[r], acc[r][b]);
          }
        }
      }
    } else {
#pragma unroll
      for (int s = 0; s < EXK / 4; ++s) {
        if (4 * s < kn) {
          const int kk = 4 * s + lk;
          const bool kok = kk < kn;
          T av[RB];
#pragma unroll
          for (int r = 0; r < RB; ++r) av[r] = kok ? (T)u.av[r][s] : (T)0;
#pragma unroll
          for (int b = 0; b < NB; ++b) {
            const T tv = buf[kk * 65 + b * 16 + li];
#pragma unroll
            for (int r = 0; r < RB; ++r) acc[r][b] = MP::mfma(tv, av[r], acc[r][b]);
          }
        }
      }
    }
  };

  // Two register sets alternate (the loop is unrolled by two) and T is staged in a
  // double-buffered LDS block: while unit u is computed, unit u + 1 is loading, and
  // one barrier per unit suffices (a wavefront passing the barrier of unit u has
  // finished computing unit u - 1, whose buffer unit u + 1 overwrites).
  int src = 0, d = a.d0 - 1, k0 = 0;
  if (exp_next_unit(a, j0, TW, src, d, k0)) {
    Unit U0, U1;
    load_unit(src, d, k0, U0);
    while (true) {
      int sn = src, dn = d, kn0 = k0;
      const bool more = exp_next_unit(a, j0, TW, sn, dn, kn0);
      if (!more) { sn = src; dn = d; kn0 = k0; }   // the last step re-reads its own unit
      load_unit(sn, dn, kn0, U1);
      stash_T(U0, src, d, k0, Ts[0]);
      lds_barrier();
      mfma_unit(U0, k0, Ts[0]);
      if (!more) break;
      src = sn;
      d = dn;
      k0 = kn0;
      const bool more2 = exp_next_unit(a, j0, TW, sn, dn, kn0);
      if (!more2) { sn = src; dn = d; kn0 = k0; }
      load_unit(sn, dn, kn0, U0);
      stash_T(U1, src, d, k0, Ts[1]);
      lds_barrier();
      mfma_unit(U1, k0, Ts[1]);
      if (!more2) break;
      src = sn;
      d = dn;
      k0 = kn0;
    }
  }
  // Y = alpha * acc + beta * Y: every old value is loaded before the first store
  double old[RB][NB][4];
  const bool rmw = a.beta != 0.0;
  if (rmw) {
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int col = j0 + b * 16 + MP::row(v, lk);
          old[r][b][v] = a.Y[r0 + rowc[r] + (long)(col < a.yhi ? col : j0) * a.ldy];
        }
  }
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    if (!rok[r]) continue;
    double* Yr = a.Y + r0 + row[r];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int col = j0 + b * 16 + MP::row(v, lk);
        if (col < a.yhi) {
          const double x = a.alpha * (double)acc[r][b][v];
          Yr[(long)col * a.ldy] = rmw ? x + a.beta * old[r][b][v] : x;
        }
      }
  }
}

// ea, eb (may be null): events set to the kernel's start and end
template <int P, int RB, int NWV>
static void launch_expand_direct(Model* m, int nb, dim3 grid, const ExpArgs& a, hipEvent_t ea, hipEvent_t eb) {
  const dim3 blk(64 * NWV);
  if (nb == 1) hipExtLaunchKernelGGL((k_expand_direct<P, 1, RB, NWV>), grid, blk, 0, m->stream, ea, eb, 0, a);
  else if (nb == 2) hipExtLaunchKernelGGL((k_expand_direct<P, 2, RB, NWV>), grid, blk, 0, m->stream, ea, eb, 0, a);
  else if (nb == 3) hipExtLaunchKernelGGL((k_expand_direct<P, 3, RB, NWV>), grid, blk, 0, m->stream, ea, eb, 0, a);
  else hipExtLaunchKernelGGL((k_expand_direct<P, 4, RB, NWV>), grid, blk, 0, m->stream, ea, eb, 0, a);
}

// Jobs that can share one launch: same A layout, T layout, depths, scaling and
// selection, and the same first output column; at most three.
static bool expand_jobs_compatible(const ExpandJob* js, int nj, const int* ylo) {
  if (nj < 2 || nj > 3) return false;
  const ExpandJob& b = js[0];
  for (int q = 1; q < nj; ++q) {
    const ExpandJob& a = js[q];
    if (a.lda != b.lda || a.ldy != b.ldy || a.t_stride != b.t_stride || a.ldt != b.ldt || a.tmode != b.tmode ||
        a.half_off != b.half_off || a.d0 != b.d0 || a.d1 != b.d1 || a.alpha != b.alpha || a.beta != b.beta ||
        a.sel.mode != b.sel.mode || a.sel.depth != b.sel.depth || a.ac.base != b.ac.base ||
        a.ac.stride != b.ac.stride || a.ac.w0 != b.ac.w0 || a.ac.grow != b.ac.grow || ylo[q] != ylo[0])
      return false;
  }
  return true;
}

hm_status tree_expand(Model* m, const ExpandJob& j) { return tree_expand_multi(m, &j, 1); }

hm_status tree_expand_multi(Model* m, const ExpandJob* js, int nj) {
  if (nj <= 0) return HM_OK;
  if (nj > 3) {
    for (int q = 0; q < nj; ++q) HM_CHECK(tree_expand_multi(m, js + q, 1));
    return HM_OK;
  }
  int ylo[3], yhi[3];
  for (int q = 0; q < nj; ++q) {
    const ExpandJob& j = js[q];
    if (j.d0 < 1 || j.d1 > m->levels || j.d0 > j.d1) {
      set_error("tree_expand: bad depth range");
      return HM_E_INVAL;
    }
    if (!sel_valid(m, j.sel)) {
      set_error("tree_expand: bad leaf selection");
      return HM_E_INVAL;
    }
    if (j.A2 && (!j.T2 || j.alpha == 0.0)) {
      set_error("tree_expand: a second source needs its T blocks and a nonzero alpha");
      return HM_E_INVAL;
    }
    ylo[q] = 1 << 30;
    yhi[q] = -1;
    for (int d = j.d0; d <= j.d1; ++d) {
      if (j.yc.w(d) <= 0) continue;
      ylo[q] = std::min(ylo[q], j.yc.c0(d));
      yhi[q] = std::max(yhi[q], j.yc.c0(d) + j.yc.w(d));
    }
  }
  if (nj > 1) {
    bool empty = false;
    for (int q = 0; q < nj; ++q) empty = empty || yhi[q] <= ylo[q];
    if (empty || !expand_jobs_compatible(js, nj, ylo)) {
      for (int q = 0; q < nj; ++q) HM_CHECK(tree_expand_multi(m, js + q, 1));
      return HM_OK;
    }
  }
  const ExpandJob& j = js[0];
  if (yhi[0] <= ylo[0]) return HM_OK;
  int wmax = 0;
  bool fixed = true;   // every job's output columns are one range shared by all depths
  for (int q = 0; q < nj; ++q) {
    wmax = std::max(wmax, yhi[q] - ylo[0]);
    fixed = fixed && js[q].yc.stride == 0 && js[q].yc.grow == 0;
  }
  ExpArgs a{j.A, j.lda, j.ac, j.Y, j.ldy, j.yc, j.T, j.t_stride, j.ldt, j.tmode, j.half_off,
            j.d0, j.d1, m->levels, m->nl, j.alpha, j.beta, ylo[0], yhi[0], j.sel.mode, j.sel.depth,
            j.A2, j.T2, j.A2 ? j.alpha2 / j.alpha : 0.0};
  for (int q = 1; q < nj; ++q) {
    a.jA[q - 1] = js[q].A;
    a.jY[q - 1] = js[q].Y;
    a.jyc[q - 1] = js[q].yc;
    a.jyhi[q - 1] = yhi[q];
    a.jT[q - 1] = js[q].T;
    a.jA2[q - 1] = js[q].A2;
    a.jT2[q - 1] = js[q].T2;
    a.jt2s[q - 1] = js[q].A2 ? js[q].alpha2 / js[q].alpha : 0.0;
  }
  const bool pf = prof_on(m, PF_EXPAND);
  hipEvent_t ea = nullptr, eb = nullptr;
  if (pf) prof_begin_launch(m, PF_EXPAND, ea, eb);
  // output blocks of 16 columns per tile: a launch narrower than 64 columns runs
  // fewer MFMA blocks; a wide output made of panel blocks (cs_block / cs_prefix of a
  // width that is a multiple of 16) is tiled at that width, so no tile straddles two
  // blocks with different segment sets; a wide output of one column range for all
  // depths takes 48 or 64 columns, whichever pads the jobs' widths less
  int nb;
  if (wmax <= 64) {
    nb = ceil_div(wmax, 16);
  } else if (fixed) {
    long pad3 = 0, pad4 = 0;
    for (int q = 0; q < nj; ++q) {
      const int w = yhi[q] - ylo[0];
      pad3 += 48L * ceil_div(w, 48) - w;
      pad4 += 64L * ceil_div(w, 64) - w;
    }
    nb = pad3 < pad4 ? 3 : 4;
  } else {
    const int bw = (j.yc.stride > 0 && j.yc.stride == j.yc.w0 && j.yc.grow == 0) ? j.yc.w0
                   : (j.yc.w0 == 0 && j.yc.stride == 0 && j.yc.grow > 0 ? j.yc.grow : 0);
    nb = (bw > 0 && bw % 16 == 0 && bw <= 64 && j.yc.base % bw == 0) ? bw / 16 : 4;
  }
  // variant: 1 = one row block of 16 per wavefront, 4 wavefronts (64 rows per
  // workgroup; the default); 2 = two row blocks (128 rows: each T value feeds two MFMAs);
  // 3 = one row block, 8 wavefronts (128 rows sharing one staged T block)
  const int var = m->tune_expand_rb ? m->tune_expand_rb : 1;
  const int rb = (var == 2) ? 2 : 1, nwv = (var == 3) ? 8 : 4;
  const int nsel = count_selected(m->nleaves, m->levels, j.sel);
  a.nj = nj;
  dim3 grid(ceil_div(m->nl, 16 * rb * nwv), ceil_div(wmax, 16 * nb), nsel * nj);
  if (m->panel_prec == 2) {
    if (var == 2) launch_expand_direct<2, 2, 4>(m, nb, grid, a, ea, eb);
    else if (var == 3) launch_expand_direct<2, 1, 8>(m, nb, grid, a, ea, eb);
    else launch_expand_direct<2, 1, 4>(m, nb, grid, a, ea, eb);
  } else if (m->panel_prec == 1) {
    if (var == 2) launch_expand_direct<1, 2, 4>(m, nb, grid, a, ea, eb);
    else if (var == 3) launch_expand_direct<1, 1, 8>(m, nb, grid, a, ea, eb);
    else launch_expand_direct<1, 1, 4>(m, nb, grid, a, ea, eb);
  } else {
    if (var == 2) launch_expand_direct<0, 2, 4>(m, nb, grid, a, ea, eb);
    else if (var == 3) launch_expand_direct<0, 1, 8>(m, nb, grid, a, ea, eb);
    else launch_expand_direct<0, 1, 4>(m, nb, grid, a, ea, eb);
  }
  HM_LAUNCH_CHECK();
  if (pf) {
    const int wk = j.ac.w0;
    const double rows = (double)nsel * m->nl;
    double fl = 0.0, by = 0.0;
    for (int q = 0; q < nj; ++q) {
      const double nsrc = js[q].A2 ? 2.0 : 1.0;   // a second source doubles the products
      for (int d = j.d0; d <= j.d1; ++d) {
        const int wy = js[q].yc.w(d);
        if (wy <= 0) continue;
        fl += nsrc * 2.0 * rows * wk * wy;
        by += nsrc * 8.0 * (rows * wk + std::min((double)nsel, (double)(1 << d)) * wk * wy);
      }
      by += 8.0 * rows * (yhi[q] - ylo[q]) * (j.beta == 0.0 ? 1.0 : 2.0);
    }
    prof_end(m, PF_EXPAND, fl, by);
  }
  return HM_OK;
}

// ----------------------------------------------------------------------------
// leaf-block GEMM: Y[L rows, 0:w] = beta Y + alpha Dm_L X[L rows, 0:w]
// ----------------------------------------------------------------------------
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
k_leaf_gemm(const double* Dm, const double* X, int ldx, double* Y,
            int ldy, int w, int nl, double alpha, double beta,
            int leaf_lo) {
  __shared__ double smem[GSMEM];
  const TileIdx tb = tile_block();
  const int L = leaf_lo + tb.z;
  const int m0 = tb.x * GBM, n0 = tb.y * GBN;
  const long r0 = (long)L * nl;
  LdA<false> la{Dm + (long)L * nl * nl, nl, m0, nl};
  LdB<false> lb{X + r0, ldx, n0, w};
  TileAcc acc;
  tile_zero(acc);
  tile_gemm(la, lb, 0, nl, acc, smem);
  tile_store_pre(StC{Y + r0, ldy, m0, n0, nl, w, alpha, beta}, acc);
}

hm_status leaf_gemm(Model* m, const double* Dm, const double* X, int ldx, double* Y, int ldy, int w,
                    double alpha, double beta, int leaf_lo, int leaf_hi) {
  if (w <= 0 || leaf_hi <= leaf_lo) return HM_OK;
  dim3 grid(ceil_div(m->nl, GBM), ceil_div(w, GBN), leaf_hi - leaf_lo);
  const bool pf = prof_on(m, PF_LEAFGEMM);
  if (pf) prof_begin(m, PF_LEAFGEMM);
  hipLaunchKernelGGL(k_leaf_gemm, grid, dim3(GCfg::NT), 0, m->stream, Dm, X, ldx, Y, ldy, w, m->nl, alpha,
                     beta, leaf_lo);
  HM_LAUNCH_CHECK();
  if (pf) {
    const double L = leaf_hi - leaf_lo, nl = m->nl;
    prof_end(m, PF_LEAFGEMM, 2.0 * L * nl * nl * w,
             8.0 * (L * nl * nl + L * nl * w * (beta == 0.0 ? 2.0 : 3.0)));
  }
  return HM_OK;
}

}  // namespace hm
