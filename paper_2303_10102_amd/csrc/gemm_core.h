// FP64 tile-GEMM core shared by the transform, leaf and generic GEMM kernels.
//
// A workgroup of 256 threads (4 wavefronts) computes a 64 x 64 tile of
// C = sum_k A(i,k) B(k,j) on the matrix cores.  Operands are fetched through
// loader functors, so the same core serves plain column-major GEMMs, per-leaf
// products and the sine transforms with the tree<->grid reordering computed in
// the load.  K-slabs of 16 are staged through double-buffered LDS.
//
// Loader protocol (A indexed (i, k), B indexed (k, j)):
//   static constexpr bool kfast;   consecutive k adjacent in memory
//   static constexpr int NR;       raw values loaded per element
//   bool load(int, int, double (&raw)[NR]) const;
//       issues the loads only, always at a valid address (an element outside the
//       operand reads a dummy one) and returns whether the element is inside;
//   double fin(const double (&raw)[NR]) const;
//       the element from its raw values (products, sums), evaluated when the
//       slab is written to LDS.
// Keeping the arithmetic out of the load phase and the loads free of branches
// lets every load of a slab be in flight at once.
#pragma once
#include <hip/hip_runtime.h>

namespace hm {

constexpr int GBM = 64, GBN = 64, GBK = 16;
struct GCfg {
  static constexpr int NT = 256;
  static constexpr int LDS_A = GBK * (GBM + 1);
  static constexpr int LDS_B = GBK * (GBN + 1);
  static constexpr int LDS_DOUBLES = LDS_A + LDS_B;
};
// LDS doubles a kernel must reserve for tile_gemm (two slabs)
constexpr int GSMEM = 2 * GCfg::LDS_DOUBLES;

// ---------------------------------------------------------------------------
// Matrix-core path (v_mfma_f64_16x16x4_f64).  The 64 x 64 tile is split over the
// 4 wavefronts, each owning a 32 x 32 quadrant made of 2 x 2 blocks of 16 x 16.
// Operand lane layout of the instruction: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; accumulator element v of lane l is D[4 v + l / 16][l % 16].
// ---------------------------------------------------------------------------
typedef double hm_v4d __attribute__((ext_vector_type(4)));

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
// wait for its loads).  smem must hold GSMEM doubles.
template <class LA, class LB>
__device__ __forceinline__ void tile_gemm(const LA& la, const LB& lb, int k0, int k1, TileAcc& acc, double* smem) {
  constexpr int BM = GBM, BN = GBN, BK = GBK, NT = GCfg::NT;
  constexpr int NA = BM * BK / NT, NB = BN * BK / NT;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
  struct Regs {
    double a[NA][LA::NR], b[NB][LB::NR];
    bool va[NA], vb[NB];
  };
  auto a_index = [&](int q, int& i, int& kk) {
    const int e = q * NT + tid;
    if (LA::kfast) { kk = e % BK; i = e / BK; } else { i = e % BM; kk = e / BM; }
  };
  auto b_index = [&](int q, int& j, int& kk) {
    const int e = q * NT + tid;
    if (LB::kfast) { kk = e % BK; j = e / BK; } else { j = e % BN; kk = e / BN; }
  };
  auto fetch = [&](int kb, Regs& r) {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      int i, kk;
      a_index(q, i, kk);
      const int k = kb + kk;
      const bool kin = k < k1;
      r.va[q] = la.load(i, kin ? k : k0, r.a[q]) && kin;
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      int j, kk;
      b_index(q, j, kk);
      const int k = kb + kk;
      const bool kin = k < k1;
      r.vb[q] = lb.load(kin ? k : k0, j, r.b[q]) && kin;
    }
  };
  auto stash = [&](const Regs& r, double* buf) {
    double* As = buf;
    double* Bs = buf + GCfg::LDS_A;
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      int i, kk;
      a_index(q, i, kk);
      As[kk * (BM + 1) + i] = r.va[q] ? la.fin(r.a[q]) : 0.0;
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      int j, kk;
      b_index(q, j, kk);
      Bs[kk * (BN + 1) + j] = r.vb[q] ? lb.fin(r.b[q]) : 0.0;
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
// ST: void operator()(int i, int j, double v) const  (tile-relative; does its own bounds)
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
// Store that reads before it writes (C = alpha AB + beta C and the like):
//   static constexpr int NP;  bool pre(int i, int j, double (&o)[NP]) const  -- issue the
//   loads the element needs (valid addresses only); void put(int i, int j, double v,
//   const double (&o)[NP]) const -- combine and store (does its own bounds).
// All loads of the tile are issued before the first store, so they are in flight together.
template <class ST>
__device__ __forceinline__ void tile_store_pre(const ST& st, const TileAcc& acc) {
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
  double o[2][2][4][ST::NP];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) st.pre(wr + a * 16 + li, wc + b * 16 + 4 * v + lk, o[a][b][v]);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) st.put(wr + a * 16 + li, wc + b * 16 + 4 * v + lk, acc.c[a][b][v], o[a][b][v]);
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
// (v_mfma_f32_16x16x4_f32) for the mixed-precision policy, P = 2 BF16 operands (below).  Both take lane l's
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
// P = 2: BF16 operands with FP32 accumulation (v_mfma_f32_16x16x16_bf16): lane l supplies
// four consecutive k, A[l % 16][4 (l / 16) + q] and B[4 (l / 16) + q][l % 16], q = 0..3, so
// one instruction covers 16 k; the accumulator is laid out as for FP32.  Operands are
// rounded to nearest even from FP32.
typedef short hm_v4bf __attribute__((ext_vector_type(4)));
__device__ __forceinline__ short bf16_rne(float f) {
  unsigned u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (short)0x7fc0;   // NaN stays NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}
__device__ __forceinline__ hm_v4bf bf16x4(float a, float b, float c, float d) {
  return hm_v4bf{bf16_rne(a), bf16_rne(b), bf16_rne(c), bf16_rne(d)};
}
template <>
struct MfmaPrec<2> {
  using T = float;   // staging type (LDS); operands are packed to BF16 per instruction
  using V = hm_v4f;
  static __device__ __forceinline__ V zero() { return V{0.0f, 0.0f, 0.0f, 0.0f}; }
  static __device__ __forceinline__ V mfma16(hm_v4bf a, hm_v4bf b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int v, int lk) { return 4 * lk + v; }
};

}  // namespace hm
