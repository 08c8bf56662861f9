// FP64 tile-GEMM core shared by all panel/leaf/transform kernels.
//
// A workgroup of NT = (BM/TM)*(BN/TN) threads computes a BM x BN tile of
// C = sum_k A(i,k) B(k,j).  Operands are fetched through loader functors so the
// same core serves plain column-major GEMMs, per-leaf panel products with tree
// addressing, and the sine transform with the tree<->grid gather fused into the
// load.  Tiles are staged through LDS; each thread keeps a TM x TN register
// tile whose rows/columns are strided by BM/TM and BN/TN (conflict-free LDS
// reads for 8-byte elements).
#pragma once
#include <hip/hip_runtime.h>

namespace hm {

template <int BM, int BN, int BK, int TM, int TN>
struct TileCfg {
  static constexpr int NT = (BM / TM) * (BN / TN);
  static constexpr int RS = BM / TM;   // row stride of a thread's register tile
  static constexpr int CS = BN / TN;   // column stride
  static constexpr int LDS_A = BK * (BM + 1);
  static constexpr int LDS_B = BK * (BN + 1);
  static constexpr int LDS_DOUBLES = LDS_A + LDS_B;
};

// LA: double operator()(int i, int k) const  -- i in [0,BM) tile row, k global
//     static constexpr bool kfast            -- consecutive k adjacent in memory
// LB: double operator()(int k, int j) const  -- j in [0,BN) tile column
template <int BM, int BN, int BK, int TM, int TN, class LA, class LB>
__device__ __forceinline__ void tile_gemm_acc(const LA& la, const LB& lb, int k0, int k1,
                                              double (&acc)[TM][TN], double* smem) {
  using C = TileCfg<BM, BN, BK, TM, TN>;
  double* As = smem;             // [BK][BM+1]
  double* Bs = smem + C::LDS_A;  // [BK][BN+1]
  const int tid = threadIdx.x;
  const int tr = tid / C::CS;
  const int tc = tid % C::CS;
  for (int kb = k0; kb < k1; kb += BK) {
    // ---- stage A tile
#pragma unroll
    for (int e0 = 0; e0 < BM * BK; e0 += C::NT) {
      int e = e0 + tid;
      int i, kk;
      if (LA::kfast) { kk = e % BK; i = e / BK; } else { i = e % BM; kk = e / BM; }
      int k = kb + kk;
      As[kk * (BM + 1) + i] = (k < k1) ? la(i, k) : 0.0;
    }
    // ---- stage B tile
#pragma unroll
    for (int e0 = 0; e0 < BN * BK; e0 += C::NT) {
      int e = e0 + tid;
      int j, kk;
      if (LB::kfast) { kk = e % BK; j = e / BK; } else { j = e % BN; kk = e / BN; }
      int k = kb + kk;
      Bs[kk * (BN + 1) + j] = (k < k1) ? lb(k, j) : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; ++kk) {
      double a[TM], b[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) a[i] = As[kk * (BM + 1) + tr + i * C::RS];
#pragma unroll
      for (int j = 0; j < TN; ++j) b[j] = Bs[kk * (BN + 1) + tc + j * C::CS];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
}

template <int BM, int BN, int TM, int TN>
__device__ __forceinline__ void tile_zero(double (&acc)[TM][TN]) {
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = 0.0;
}

// ST: void operator()(int i, int j, double v) const  (tile-relative; does its own bounds)
template <int BM, int BN, int BK, int TM, int TN, class ST>
__device__ __forceinline__ void tile_store(const ST& st, const double (&acc)[TM][TN]) {
  using C = TileCfg<BM, BN, BK, TM, TN>;
  const int tid = threadIdx.x;
  const int tr = tid / C::CS;
  const int tc = tid % C::CS;
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) st(tr + i * C::RS, tc + j * C::CS, acc[i][j]);
}

// Standard configuration used by the panel kernels: 64 x 64 tiles, 256 threads.
constexpr int GBM = 64, GBN = 64, GBK = 16, GTM = 4, GTN = 4;
using GCfg = TileCfg<GBM, GBN, GBK, GTM, GTN>;
// LDS doubles a kernel must reserve for tile_gemm (two slabs)
constexpr int GSMEM = 2 * GCfg::LDS_DOUBLES;

// ---------------------------------------------------------------------------
// Matrix-core path (CDNA3/CDNA4 v_mfma_f64_16x16x4_f64).  The 64 x 64 tile is
// split over the 4 wavefronts of the workgroup, each owning a 32 x 32 quadrant
// made of 2 x 2 blocks of 16 x 16.  Operand lane layout of the instruction:
// lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]; accumulator element
// v of lane l is D[4 v + l / 16][l % 16].  Same LDS staging as the FMA path.
// ---------------------------------------------------------------------------
#ifndef HM_MFMA
#define HM_MFMA 1
#endif
typedef double hm_v4d __attribute__((ext_vector_type(4)));

#if HM_MFMA
struct TileAcc {
  hm_v4d c[2][2];
};
__device__ __forceinline__ void tile_zero(TileAcc& acc) {
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc.c[a][b] = hm_v4d{0.0, 0.0, 0.0, 0.0};
}
// Pipelined: two K-slabs ahead are in flight in registers while the current one is
// consumed from LDS (double-buffered), so one barrier per slab and two global
// round trips overlap each slab's matrix-core work.  The slab loop is unrolled by
// two so that the two register sets alternate statically (a register copy would
// wait for its loads).  smem must hold 2 * GCfg::LDS_DOUBLES.
template <class LA, class LB>
__device__ __forceinline__ void tile_gemm(const LA& la, const LB& lb, int k0, int k1, TileAcc& acc, double* smem) {
  constexpr int BM = GBM, BN = GBN, BK = GBK, NT = GCfg::NT;
  constexpr int NA = BM * BK / NT, NB = BN * BK / NT;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
  struct Regs {
    double a[NA], b[NB];
  };
  auto fetch = [&](int kb, Regs& r) {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      int e = q * NT + tid;
      int i, kk;
      if (LA::kfast) { kk = e % BK; i = e / BK; } else { i = e % BM; kk = e / BM; }
      int k = kb + kk;
      r.a[q] = (k < k1) ? la(i, k) : 0.0;
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      int e = q * NT + tid;
      int j, kk;
      if (LB::kfast) { kk = e % BK; j = e / BK; } else { j = e % BN; kk = e / BN; }
      int k = kb + kk;
      r.b[q] = (k < k1) ? lb(k, j) : 0.0;
    }
  };
  auto stash = [&](const Regs& r, double* buf) {
    double* As = buf;
    double* Bs = buf + GCfg::LDS_A;
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      int e = q * NT + tid;
      int i, kk;
      if (LA::kfast) { kk = e % BK; i = e / BK; } else { i = e % BM; kk = e / BM; }
      As[kk * (BM + 1) + i] = r.a[q];
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      int e = q * NT + tid;
      int j, kk;
      if (LB::kfast) { kk = e % BK; j = e / BK; } else { j = e % BN; kk = e / BN; }
      Bs[kk * (BN + 1) + j] = r.b[q];
    }
  };
  auto compute = [&](const double* buf) {
    const double* As = buf;
    const double* Bs = buf + GCfg::LDS_A;
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int kr = kk + lk;
      const double a0 = As[kr * (BM + 1) + wr + li];
      const double a1 = As[kr * (BM + 1) + wr + 16 + li];
      const double b0 = Bs[kr * (BN + 1) + wc + li];
      const double b1 = Bs[kr * (BN + 1) + wc + 16 + li];
      // operands swapped: each block accumulates the transpose (see tile_store)
      acc.c[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(b0, a0, acc.c[0][0], 0, 0, 0);
      acc.c[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(b1, a0, acc.c[0][1], 0, 0, 0);
      acc.c[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(b0, a1, acc.c[1][0], 0, 0, 0);
      acc.c[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(b1, a1, acc.c[1][1], 0, 0, 0);
    }
  };
  if (k0 >= k1) return;
  double* buf0 = smem;
  double* buf1 = smem + GCfg::LDS_DOUBLES;
  Regs r1, r2;
  fetch(k0, r1);
  stash(r1, buf0);
  if (k0 + BK < k1) fetch(k0 + BK, r1);
  __syncthreads();
  // invariant at the top of a step for slab kb: slab kb in LDS, slab kb + BK in flight
  for (int kb = k0; kb < k1; kb += 2 * BK) {
    // slab kb from buf0; slab kb + BK (r1) to buf1; slab kb + 2 BK fetched into r2
    if (kb + 2 * BK < k1) fetch(kb + 2 * BK, r2);
    compute(buf0);
    if (kb + BK >= k1) break;
    stash(r1, buf1);
    __syncthreads();
    // slab kb + BK from buf1; slab kb + 2 BK (r2) to buf0; slab kb + 3 BK fetched into r1
    if (kb + 3 * BK < k1) fetch(kb + 3 * BK, r1);
    compute(buf1);
    if (kb + 2 * BK >= k1) break;
    stash(r2, buf0);
    __syncthreads();
  }
  // the last slab's LDS reads are done before a caller reuses smem
  __syncthreads();
}
template <class ST>
__device__ __forceinline__ void tile_store(const ST& st, const TileAcc& acc) {
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
  // block (a, b) holds its transpose: element v of lane l is C[row l % 16][col 4 v + l / 16],
  // so the 16 lanes of a group write 16 consecutive rows (one column-major run)
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) st(wr + a * 16 + li, wc + b * 16 + 4 * v + lk, acc.c[a][b][v]);
}
// Store of two accumulators of the same tile: st(i, j, e, o)
template <class ST>
__device__ __forceinline__ void tile_store2(const ST& st, const TileAcc& e, const TileAcc& o) {
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        st(wr + a * 16 + li, wc + b * 16 + 4 * v + lk, e.c[a][b][v], o.c[a][b][v]);
}
// ---------------------------------------------------------------------------
// Precision trait of the panel kernels that feed MFMA operands directly:
// P = 0 FP64 (v_mfma_f64_16x16x4_f64), P = 1 FP32 operands with FP32 accumulation
// (v_mfma_f32_16x16x4_f32) for the mixed-precision policy.  Both take lane l's
// operands as A[l % 16][l / 16] and B[l / 16][l % 16]; their accumulators differ:
// element v of lane l is D[4 v + l / 16][l % 16] (FP64) and D[4 (l / 16) + v][l % 16] (FP32).
// ---------------------------------------------------------------------------
typedef float hm_v4f __attribute__((ext_vector_type(4)));
template <int P>
struct MfmaPrec;
template <>
struct MfmaPrec<0> {
  using T = double;
  using V = hm_v4d;
  static __device__ __forceinline__ V zero() { return V{0.0, 0.0, 0.0, 0.0}; }
  static __device__ __forceinline__ V mfma(T a, T b, V c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  // row of the 16 x 16 block held by accumulator element v of a lane in k-group lk
  static __device__ __forceinline__ int row(int v, int lk) { return 4 * v + lk; }
};
template <>
struct MfmaPrec<1> {
  using T = float;
  using V = hm_v4f;
  static __device__ __forceinline__ V zero() { return V{0.0f, 0.0f, 0.0f, 0.0f}; }
  static __device__ __forceinline__ V mfma(T a, T b, V c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  static __device__ __forceinline__ int row(int v, int lk) { return 4 * lk + v; }
};
#else
struct TileAcc {
  double c[GTM][GTN];
};
__device__ __forceinline__ void tile_zero(TileAcc& acc) { tile_zero<GBM, GBN, GTM, GTN>(acc.c); }
constexpr int GSMEM_FMA = GCfg::LDS_DOUBLES;
template <class LA, class LB>
__device__ __forceinline__ void tile_gemm(const LA& la, const LB& lb, int k0, int k1, TileAcc& acc, double* smem) {
  tile_gemm_acc<GBM, GBN, GBK, GTM, GTN>(la, lb, k0, k1, acc.c, smem);
}
template <class ST>
__device__ __forceinline__ void tile_store(const ST& st, const TileAcc& acc) {
  tile_store<GBM, GBN, GBK, GTM, GTN>(st, acc.c);
}
template <class ST>
__device__ __forceinline__ void tile_store2(const ST& st, const TileAcc& e, const TileAcc& o) {
  const int tr = threadIdx.x / GCfg::CS, tc = threadIdx.x % GCfg::CS;
#pragma unroll
  for (int i = 0; i < GTM; ++i)
#pragma unroll
    for (int j = 0; j < GTN; ++j) st(tr + i * GCfg::RS, tc + j * GCfg::CS, e.c[i][j], o.c[i][j]);
}
#endif

}  // namespace hm
