// Batched GEMM on MFMA (FP64 v_mfma_f64_16x16x4f64; FP32 and BF16 inputs
// with FP32 accumulation for the mixed-precision solve), the small dense
// factorisations of the truncation (pivoted Cholesky, one-sided Jacobi)
// and a batched cyclic Jacobi eigensolver.
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "linalg.h"
#include "prof.h"

namespace lrfg {

namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int BM = 64, BN = 64;  // tile of the mixed-precision kernel

// Block of 4 waves (256 threads) in a WM x WN x WK layout (WM WN WK = 4):
// the block tile is (32 WM) x (32 WN); each wave computes a 32 x 32 sub-tile
// as 2 x 2 MFMA 16 x 16 blocks and, with WK > 1, the WK waves that share a
// sub-tile take disjoint 16-wide quarters of each K slab (TK = 16 WK) and
// add their sums through LDS at the end in a fixed order.  MFMA blocks that
// lie wholly outside the m x n output are skipped (a wave-uniform test), so
// a small output does not pay for the padded tile.  MFMA f64 16x16x4 lane
// layout: A operand lane l -> A[l % 16][l / 16]; B operand lane l ->
// B[l / 16][l % 16]; result lane l holds D[l / 16 + 4 i][l % 16], i < 4.
// With `part` != null the raw product of this K split is stored to
// part[(bz * m + row) * n + col] for a later reduction.
template <bool TA, bool TB, int WM, int WN>
__global__ __launch_bounds__(256) void k_gemm(int m, int n, int k, const double* __restrict__ A,
                                              long long lda, long long sA, const double* __restrict__ B,
                                              long long ldb, long long sB, double* __restrict__ C,
                                              long long ldc, long long sC, double alpha, double beta,
                                              int ksplit, int kchunk, double* __restrict__ part, BatchMap bm) {
  constexpr int WK = 4 / (WM * WN);
  constexpr int TM = 32 * WM, TN = 32 * WN, TK = 16 * WK;
  constexpr int RA = (TM * TK) / 256, RB = (TK * TN) / 256;
  __shared__ double As[TK][TM + 1];
  __shared__ double Bs[TK][TN + 1];
  __shared__ double red[WK > 1 ? (WK - 1) * (WM * WN) * 16 * 64 : 1];
  const int bz = blockIdx.z;
  const int bt = bz / ksplit;
  const int ks = bz - bt * ksplit;
  const long long tg = bm.tbase + bt;
  A += bm.a_off(tg, sA);
  B += bm.b_off(tg, sB);
  const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
  const int kb = ks * kchunk;
  const int ke = min(k, kb + kchunk);
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wk = wave / (WM * WN), wr = wave - wk * (WM * WN);
  const int wm = wr / WN, wn = wr - (wr / WN) * WN;
  // which of the wave's 2 x 2 MFMA blocks touch the output (wave-uniform)
  const bool r0 = m0 + wm * 32 < m, r1 = m0 + wm * 32 + 16 < m;
  const bool c0 = n0 + wn * 32 < n, c1 = n0 + wn * 32 + 16 < n;
  dbl4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
  // register prefetch of the next K slab while the current one is multiplied
  double pa[RA], pb[RB];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int r = 0; r < RA; ++r) {
      const int e = threadIdx.x + r * 256;
      int i, kk;
      if (!TA) { i = e / TK; kk = e % TK; } else { kk = e / TM; i = e % TM; }
      const int gi = m0 + i, gk = k0 + kk;
      pa[r] = (gi < m && gk < ke) ? (TA ? A[(long long)gk * lda + gi] : A[(long long)gi * lda + gk]) : 0.0;
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const int e = threadIdx.x + r * 256;
      int kk, j;
      if (!TB) { kk = e / TN; j = e % TN; } else { j = e / TK; kk = e % TK; }
      const int gk = k0 + kk, gj = n0 + j;
      pb[r] = (gj < n && gk < ke) ? (TB ? B[(long long)gj * ldb + gk] : B[(long long)gk * ldb + bm.bcol(gj)]) : 0.0;
    }
  };
  // The K loop with the wave's live MFMA blocks (NR x NC of its 2 x 2,
  // wave-uniform) fixed at compile time: no branch between the MFMAs.
  auto kloop = [&](auto nr_c, auto nc_c) {
    constexpr int NR = decltype(nr_c)::value, NC = decltype(nc_c)::value;
    if (kb < ke) fetch(kb);
    for (int k0 = kb; k0 < ke; k0 += TK) {
#pragma unroll
      for (int r = 0; r < RA; ++r) {
        const int e = threadIdx.x + r * 256;
        int i, kk;
        if (!TA) { i = e / TK; kk = e % TK; } else { kk = e / TM; i = e % TM; }
        As[kk][i] = pa[r];
      }
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        const int e = threadIdx.x + r * 256;
        int kk, j;
        if (!TB) { kk = e / TN; j = e % TN; } else { j = e / TK; kk = e % TK; }
        Bs[kk][j] = pb[r];
      }
      __syncthreads();
      if (k0 + TK < ke) fetch(k0 + TK);
      if constexpr (NR > 0 && NC > 0) {
#pragma unroll
        for (int kq = 0; kq < 16; kq += 4) {
          const int kk = wk * 16 + kq;
          double a[2], b[2];
#pragma unroll
          for (int bi = 0; bi < NR; ++bi) a[bi] = As[kk + (lane >> 4)][wm * 32 + bi * 16 + (lane & 15)];
#pragma unroll
          for (int bj = 0; bj < NC; ++bj) b[bj] = Bs[kk + (lane >> 4)][wn * 32 + bj * 16 + (lane & 15)];
#pragma unroll
          for (int bi = 0; bi < NR; ++bi)
#pragma unroll
            for (int bj = 0; bj < NC; ++bj)
              acc[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[bi], b[bj], acc[bi][bj], 0, 0, 0);
        }
      }
      __syncthreads();
    }
  };
  using I0 = std::integral_constant<int, 0>;
  using I1 = std::integral_constant<int, 1>;
  using I2 = std::integral_constant<int, 2>;
  if (r1 && c1) kloop(I2{}, I2{});
  else if (r1 && c0) kloop(I2{}, I1{});
  else if (r0 && c1) kloop(I1{}, I2{});
  else if (r0 && c0) kloop(I1{}, I1{});
  else kloop(I0{}, I0{});
  if (WK > 1) {
    // waves wk > 0 hand their sums to the wave wk = 0 of their sub-tile
    // through LDS
    if (wk > 0) {
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            red[((((wk - 1) * (WM * WN) + wr) * 16) + (bi * 2 + bj) * 4 + r) * 64 + lane] = acc[bi][bj][r];
    }
    __syncthreads();
    if (wk == 0) {
#pragma unroll
      for (int q = 0; q < WK - 1; ++q)
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
          for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[bi][bj][r] += red[(((q * (WM * WN) + wr) * 16) + (bi * 2 + bj) * 4 + r) * 64 + lane];
    }
  }
  if (wk != 0) return;
  double* const Cb = C + bm.c_off(tg, sC);
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * 32 + bi * 16 + (lane >> 4) + 4 * r;
        const int col = n0 + wn * 32 + bj * 16 + (lane & 15);
        if (row < m && col < n) {
          const double v = acc[bi][bj][r];
          if (part != nullptr) {
            part[((long long)bz * m + row) * n + col] = v;
          } else {
            double* c = Cb + (long long)row * ldc + bm.ccol(col);
            *c = (beta == 0.0) ? alpha * v : alpha * v + beta * (*c);
          }
        }
      }
}

// The block tile of the large-tile kernels: WM x WN waves, each computing
// BI x BJ MFMA 16 x 16 blocks, so the tile is (16 BI WM) x (16 BJ WN) and a
// K slab of 16 staged in LDS feeds 4 BI BJ MFMAs per wave.  Two slab
// buffers: the next slab is written while the current one feeds the MFMAs,
// one barrier per slab.  Every MFMA runs (the staging writes zeros outside
// the output, and the epilogue drops those entries).  Same operand layouts,
// batch and column maps and split-K partials as k_gemm.
template <bool TA, bool TB, int WM, int WN, int BI, int BJ>
__device__ __forceinline__ void gemm_tile(int m, int n, int k, const double* __restrict__ A, long long lda,
                                          long long sA, const double* __restrict__ B, long long ldb, long long sB,
                                          double* __restrict__ C, long long ldc, long long sC, double alpha,
                                          double beta, int ksplit, int kchunk, double* __restrict__ part,
                                          const BatchMap& bm) {
  static_assert(WM * WN == 4, "four waves");
  constexpr int TM = 16 * BI * WM, TN = 16 * BJ * WN, TK = 16;
  constexpr int RA = (TM * TK) / 256, RB = (TK * TN) / 256;
  static_assert(RA * 256 == TM * TK && RB * 256 == TK * TN, "staging split");
  __shared__ double As[2][TK][TM + 1];
  __shared__ double Bs[2][TK][TN + 1];
  const int bz = blockIdx.z;
  const int bt = bz / ksplit;
  const int ks = bz - bt * ksplit;
  const long long tg = bm.tbase + bt;
  A += bm.a_off(tg, sA);
  B += bm.b_off(tg, sB);
  const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
  const int kb = ks * kchunk;
  const int ke = min(k, kb + kchunk);
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wm = wave / WN, wn = wave - (wave / WN) * WN;
  dbl4 acc[BI][BJ];
#pragma unroll
  for (int i = 0; i < BI; ++i)
#pragma unroll
    for (int j = 0; j < BJ; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
  double pa[RA], pb[RB];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int r = 0; r < RA; ++r) {
      const int e = threadIdx.x + r * 256;
      int i, kk;
      if (!TA) { i = e / TK; kk = e % TK; } else { kk = e / TM; i = e % TM; }
      const int gi = m0 + i, gk = k0 + kk;
      pa[r] = (gi < m && gk < ke) ? (TA ? A[(long long)gk * lda + gi] : A[(long long)gi * lda + gk]) : 0.0;
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const int e = threadIdx.x + r * 256;
      int kk, j;
      if (!TB) { kk = e / TN; j = e % TN; } else { j = e / TK; kk = e % TK; }
      const int gk = k0 + kk, gj = n0 + j;
      pb[r] = (gj < n && gk < ke) ? (TB ? B[(long long)gj * ldb + gk] : B[(long long)gk * ldb + bm.bcol(gj)]) : 0.0;
    }
  };
  auto stage = [&](int buf) {
#pragma unroll
    for (int r = 0; r < RA; ++r) {
      const int e = threadIdx.x + r * 256;
      int i, kk;
      if (!TA) { i = e / TK; kk = e % TK; } else { kk = e / TM; i = e % TM; }
      As[buf][kk][i] = pa[r];
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const int e = threadIdx.x + r * 256;
      int kk, j;
      if (!TB) { kk = e / TN; j = e % TN; } else { j = e / TK; kk = e % TK; }
      Bs[buf][kk][j] = pb[r];
    }
  };
  if (kb < ke) {
    fetch(kb);
    stage(0);
  }
  __syncthreads();
  int buf = 0;
  for (int k0 = kb; k0 < ke; k0 += TK) {
    const bool more = k0 + TK < ke;
    if (more) fetch(k0 + TK);
#pragma unroll
    for (int kq = 0; kq < TK; kq += 4) {
      const int kk = kq + (lane >> 4);
      double a[BI], b[BJ];
#pragma unroll
      for (int i = 0; i < BI; ++i) a[i] = As[buf][kk][wm * 16 * BI + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < BJ; ++j) b[j] = Bs[buf][kk][wn * 16 * BJ + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < BI; ++i)
#pragma unroll
        for (int j = 0; j < BJ; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    // the other buffer was last read before the previous barrier
    if (more) stage(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  double* const Cb = C + bm.c_off(tg, sC);
#pragma unroll
  for (int i = 0; i < BI; ++i)
#pragma unroll
    for (int j = 0; j < BJ; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * 16 * BI + i * 16 + (lane >> 4) + 4 * r;
        const int col = n0 + wn * 16 * BJ + j * 16 + (lane & 15);
        if (row < m && col < n) {
          const double v = acc[i][j][r];
          if (part != nullptr) {
            part[((long long)bz * m + row) * n + col] = v;
          } else {
            double* c = Cb + (long long)row * ldc + bm.ccol(col);
            *c = (beta == 0.0) ? alpha * v : alpha * v + beta * (*c);
          }
        }
      }
}

#define LRFG_GEMM_TILE_KERNEL(NAME, BOUNDS, WM, WN, BI, BJ)                                                    \
  template <bool TA, bool TB>                                                                                 \
  __global__ BOUNDS void NAME(int m, int n, int k, const double* __restrict__ A, long long lda, long long sA,  \
                              const double* __restrict__ B, long long ldb, long long sB, double* __restrict__ C, \
                              long long ldc, long long sC, double alpha, double beta, int ksplit, int kchunk,   \
                              double* __restrict__ part, BatchMap bm) {                                        \
    gemm_tile<TA, TB, WM, WN, BI, BJ>(m, n, k, A, lda, sA, B, ldb, sB, C, ldc, sC, alpha, beta, ksplit, kchunk,  \
                                      part, bm);                                                               \
  }
// 128 x 128 tiles, 2 x 2 waves of 64 x 64: twice the flops per staged byte
// of the 64 x 64 tile of k_gemm
LRFG_GEMM_TILE_KERNEL(k_gemm128, __launch_bounds__(256, 2), 2, 2, 4, 4)
// 96 x 96 tiles, 2 x 2 waves of 48 x 48, for outputs with a side of 65..96:
// such a side fits one tile, so each operand is read once per tile row or
// column instead of three times with 32-wide tiles
LRFG_GEMM_TILE_KERNEL(k_gemm96, __launch_bounds__(256), 2, 2, 3, 3)
// 80 x 128 tiles, 1 x 4 waves of 80 x 32, for m of 65..80 against n of at
// least 128 (the products over the coefficient's ranks): 9 % padding on m
// where the 96 x 96 tile has 42 %
LRFG_GEMM_TILE_KERNEL(k_gemm80, __launch_bounds__(256), 1, 4, 5, 2)
#undef LRFG_GEMM_TILE_KERNEL

// Reduced-precision variant for the mixed-precision solve: FP64 operands
// in memory, rounded to FP32 (BF = false) or BF16 (BF = true) when staged,
// products accumulated in FP32 on MFMA, the sum stored as FP64.  Tile
// 64 x 64 x 32 per 256-thread block, waves as in k_gemm.  Lane layouts
// (checked on gfx950): v_mfma_f32_16x16x4f32 takes A[l % 16][l / 16] and
// B[l / 16][l % 16]; v_mfma_f32_16x16x32_bf16 takes A[l % 16][8 (l / 16) + j]
// and B[8 (l / 16) + j][l % 16], j < 8; both return D[4 (l / 16) + i][l % 16].
typedef float flt4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
constexpr int LK = 32;

template <bool TA, bool TB, bool BF>
__global__ __launch_bounds__(256) void k_gemm_lp(int m, int n, int k, const double* __restrict__ A, long long lda,
                                                 long long sA, const double* __restrict__ B, long long ldb,
                                                 long long sB, double* __restrict__ C, long long ldc, long long sC,
                                                 double alpha, double beta, int ksplit, int kchunk,
                                                 double* __restrict__ part, BatchMap bm) {
  __shared__ float As[LK][BM + 1];
  __shared__ float Bs[LK][BN + 1];
  const int bz = blockIdx.z;
  const int bt = bz / ksplit;
  const int ks = bz - bt * ksplit;
  const long long tg = bm.tbase + bt;
  A += bm.a_off(tg, sA);
  B += bm.b_off(tg, sB);
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int kb = ks * kchunk;
  const int ke = min(k, kb + kchunk);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  constexpr int RA = (BM * LK) / 256, RB = (LK * BN) / 256;
  flt4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = flt4{0.f, 0.f, 0.f, 0.f};
  float pa[RA], pb[RB];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int r = 0; r < RA; ++r) {
      const int e = threadIdx.x + r * 256;
      int i, kk;
      if (!TA) { i = e / LK; kk = e % LK; } else { kk = e / BM; i = e % BM; }
      const int gi = m0 + i, gk = k0 + kk;
      pa[r] = (gi < m && gk < ke) ? (float)(TA ? A[(long long)gk * lda + gi] : A[(long long)gi * lda + gk]) : 0.f;
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const int e = threadIdx.x + r * 256;
      int kk, j;
      if (!TB) { kk = e / BN; j = e % BN; } else { j = e / LK; kk = e % LK; }
      const int gk = k0 + kk, gj = n0 + j;
      pb[r] = (gj < n && gk < ke) ? (float)(TB ? B[(long long)gj * ldb + gk] : B[(long long)gk * ldb + gj]) : 0.f;
    }
  };
  if (kb < ke) fetch(kb);
  for (int k0 = kb; k0 < ke; k0 += LK) {
#pragma unroll
    for (int r = 0; r < RA; ++r) {
      const int e = threadIdx.x + r * 256;
      int i, kk;
      if (!TA) { i = e / LK; kk = e % LK; } else { kk = e / BM; i = e % BM; }
      As[kk][i] = pa[r];
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const int e = threadIdx.x + r * 256;
      int kk, j;
      if (!TB) { kk = e / BN; j = e % BN; } else { j = e / LK; kk = e % LK; }
      Bs[kk][j] = pb[r];
    }
    __syncthreads();
    if (k0 + LK < ke) fetch(k0 + LK);
    if (BF) {
      // two-term split of each FP32 operand: x = hi + lo (both BF16, lo =
      // BF16(x - hi)); the product takes hi*hi + hi*lo + lo*hi (lo*lo, of
      // relative size 2^-16, dropped), about 16 significant bits
      bf16x8 a[2], b[2], al[2], bl[2];
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const float x = As[8 * (lane >> 4) + j][wm * 32 + bi * 16 + (lane & 15)];
          a[bi][j] = (__bf16)x;
          al[bi][j] = (__bf16)(x - (float)a[bi][j]);
        }
#pragma unroll
      for (int bj = 0; bj < 2; ++bj)
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const float x = Bs[8 * (lane >> 4) + j][wn * 32 + bj * 16 + (lane & 15)];
          b[bj][j] = (__bf16)x;
          bl[bj][j] = (__bf16)(x - (float)b[bj][j]);
        }
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) {
          acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[bi], b[bj], acc[bi][bj], 0, 0, 0);
          acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[bi], bl[bj], acc[bi][bj], 0, 0, 0);
          acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[bi], b[bj], acc[bi][bj], 0, 0, 0);
        }
    } else {
#pragma unroll
      for (int kk = 0; kk < LK; kk += 4) {
        float a[2], b[2];
#pragma unroll
        for (int bi = 0; bi < 2; ++bi) a[bi] = As[kk + (lane >> 4)][wm * 32 + bi * 16 + (lane & 15)];
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) b[bj] = Bs[kk + (lane >> 4)][wn * 32 + bj * 16 + (lane & 15)];
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
          for (int bj = 0; bj < 2; ++bj)
            acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[bi], b[bj], acc[bi][bj], 0, 0, 0);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * 32 + bi * 16 + 4 * (lane >> 4) + r;
        const int col = n0 + wn * 32 + bj * 16 + (lane & 15);
        if (row < m && col < n) {
          const double v = (double)acc[bi][bj][r];
          if (part != nullptr) {
            part[((long long)bz * m + row) * n + col] = v;
          } else {
            double* c = C + bm.c_off(tg, sC) + (long long)row * ldc + col;
            *c = (beta == 0.0) ? alpha * v : alpha * v + beta * (*c);
          }
        }
      }
}

// C = alpha * sum_ks part[ks] + beta * C.  The partials were just written
// from every XCD, so they come from HBM / the Infinity Cache: a block
// spreads the splits of 32 outputs over 8 thread groups, each with eight
// loads in flight, and adds the 8 group sums in a fixed order.
__global__ __launch_bounds__(256) void k_splitk_reduce(int m, int n, int ksplit, int batch,
                                                       const double* __restrict__ part, double* __restrict__ C,
                                                       long long ldc, long long sC, double alpha, double beta,
                                                       BatchMap bm) {
  __shared__ double red[8][33];
  const long long mn = (long long)m * n;
  const long long tot = (long long)batch * mn;
  const int o = threadIdx.x & 31, g = threadIdx.x >> 5;
  const long long e = (long long)blockIdx.x * 32 + o;
  double v = 0.0;
  if (e < tot) {
    const long long bt = e / mn, idx = e - bt * mn;
    const double* p = part + bt * ksplit * mn + idx;
    double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int k = g;
    for (; k + 56 < ksplit; k += 64) {
#pragma unroll
      for (int u = 0; u < 8; ++u) a[u] += p[(long long)(k + 8 * u) * mn];
    }
    for (; k < ksplit; k += 8) a[0] += p[(long long)k * mn];
    v = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  }
  red[g][o] = v;
  __syncthreads();
  if (g == 0 && e < tot) {
    const double sum = ((red[0][o] + red[1][o]) + (red[2][o] + red[3][o])) +
                       ((red[4][o] + red[5][o]) + (red[6][o] + red[7][o]));
    const long long bt = e / mn, idx = e - bt * mn;
    const int row = (int)(idx / n), col = (int)(idx - (idx / n) * n);
    double* c = C + bm.c_off(bm.tbase + bt, sC) + (long long)row * ldc + bm.ccol(col);
    *c = (beta == 0.0) ? alpha * sum : alpha * sum + beta * (*c);
  }
}

// Wave layout of k_gemm for one matrix's shape: outputs of at most 32 x 32
// split K four ways inside the block, narrow outputs stack the waves along
// the long side, the rest use the 2 x 2 layout of 64 x 64 tiles.
// {4, 4} stands for k_gemm128 (128 x 128 tiles, 64 x 64 per wave), {3, 3}
// for k_gemm96 (96 x 96 tiles, 48 x 48 per wave) and {5, 2} for k_gemm80
// (80 x 128 tiles, 80 x 32 per wave).
struct GemmLayout {
  int wm, wn;
  bool large() const { return wm * wn == 16 || wm * wn == 9 || wm == 5; }
  int tm() const { return wm == 5 ? 80 : 32 * wm; }
  int tn() const { return wm == 5 ? 128 : 32 * wn; }
  int tk() const { return large() ? 16 : 16 * (4 / (wm * wn)); }
};
GemmLayout gemm_layout(const Gemm& g) {
  if (g.m >= 128 && g.n >= 128) return {4, 4};
  // m of 65..80 against n of at least 128: 80 x 128 tiles ({5, 2}, k_gemm80)
  if (g.m > 64 && g.m <= 80 && g.n >= 128) return {5, 2};
  // a side of 65..96 and the other of 65..96 or above 128: 96 x 96 tiles
  // ({3, 3}, k_gemm96), one tile across that side
  const int lo = g.m < g.n ? g.m : g.n, hi = g.m < g.n ? g.n : g.m;
  if (lo > 64 && lo <= 96 && (hi <= 96 || hi > 128)) return {3, 3};
  // a side of 65..96 fills three 32-wide tiles (76-100 %) rather than two
  // 64-wide ones (51-75 %)
  if (g.m > 64 && g.m <= 96 && g.n >= 128) return {1, 4};
  if (g.n > 64 && g.n <= 96 && g.m >= 128) return {4, 1};
  if (g.m <= 32 && g.n <= 32) return {1, 1};
  if (g.n <= 32) return g.m <= 64 ? GemmLayout{2, 1} : GemmLayout{4, 1};
  if (g.m <= 32) return g.n <= 64 ? GemmLayout{1, 2} : GemmLayout{1, 4};
  return {2, 2};
}

// K splits from the shape of one matrix only, so a matrix gets the same
// summation order whatever the batch it travels in (batched solves
// reproduce single solves bit for bit).
int choose_ksplit(const Gemm& g) {
  if (g.nosplit) return 1;
  const bool lp = g.prec != 0;
  const GemmLayout L = lp ? GemmLayout{2, 2} : gemm_layout(g);
  const long long tiles = (long long)ceil_div(g.m, L.tm()) * ceil_div(g.n, L.tn());
  if (tiles >= 128 || g.k < 256) return 1;
  long long ks = 512 / tiles;
  const long long kmax = g.k / 64;  // at least 64 of K per split
  if (ks > kmax) ks = kmax;
  if (ks > 128) ks = 128;
  return ks < 1 ? 1 : (int)ks;
}

// ---------------------------------------------------------------- Jacobi
// One 256-thread block per matrix; A and V in LDS (stride n).  Cyclic
// round-robin ordering: m = n rounded up to even, position 0 fixed, the
// others rotate by one per step; pair k of a step joins positions k and
// m-1-k, so the pairs of a step are disjoint.  Rotation of the symmetric
// Schur step (Golub and Van Loan): tau = (a_qq - a_pp)/(2 a_pq),
// t = sign(tau)/(|tau| + sqrt(1 + tau^2)), c = 1/sqrt(1 + t^2), s = t c,
// J = [[c, s], [-s, c]] on (p, q).  A <- J^T A J is applied as independent
// 2 x 2 blocks (pair k rows, pair l columns), V <- V J row by row.  A
// rotation is skipped when |a_pq| is below 1e-18 of the largest initial
// diagonal entry; the iteration ends after the first sweep that applies no
// rotation.
__device__ inline int fdivi(int x, int d, float rd) {
  int q = (int)((float)x * rd);
  if (q * d > x) --q;
  else if ((q + 1) * d <= x) ++q;
  return q;
}

__global__ __launch_bounds__(256) void k_syevj(int n, const double* __restrict__ Ag, long long lda, long long sA,
                                               double* __restrict__ Wg, long long sW, double* __restrict__ Vg,
                                               long long sV, int max_sweeps) {
  extern __shared__ double sm[];
  double* a = sm;
  double* v = sm + n * n;
  __shared__ double cs[2 * 32];
  __shared__ int pq[2 * 32];
  __shared__ int rot_any;
  __shared__ double dmax_s;
  const int b = blockIdx.x;
  const double* A = Ag + b * sA;
  const int tid = threadIdx.x, nt = blockDim.x;
  const float rn = 1.0f / (float)n;
  for (int e = tid; e < n * n; e += nt) {
    const int i = fdivi(e, n, rn), j = e - fdivi(e, n, rn) * n;
    a[e] = 0.5 * (A[(long long)i * lda + j] + A[(long long)j * lda + i]);
    v[e] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  if (tid == 0) {
    double dm = 0.0;
    for (int i = 0; i < n; ++i) dm = fmax(dm, fabs(a[i * n + i]));
    dmax_s = dm;
  }
  const int m = n + (n & 1);
  const int np = m / 2;
  const float rnp = 1.0f / (float)np;
  const int nblk = np * np;
  __syncthreads();
  const double abs_floor = 1e-18 * dmax_s;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    if (tid == 0) rot_any = 0;
    __syncthreads();
    for (int step = 0; step < m - 1; ++step) {
      if (tid < np) {
        const int k = tid;
        int t0 = 0;
        if (k != 0) {
          const int u = k - 1 + step;
          t0 = 1 + (u >= m - 1 ? u - (m - 1) : u);
        }
        const int u1 = (m - 1 - k) - 1 + step;
        const int t1 = 1 + (u1 >= m - 1 ? u1 - (m - 1) : u1);
        int p = t0 < t1 ? t0 : t1;
        int q = t0 < t1 ? t1 : t0;
        double c = 1.0, s = 0.0;
        if (q < n) {
          const double apq = a[p * n + q];
          const double app = a[p * n + p], aqq = a[q * n + q];
          if (fabs(apq) > abs_floor) {
            const double tau = (aqq - app) / (2.0 * apq);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
            rot_any = 1;
          }  // else: both rows stay, identity rotation (c = 1, s = 0)
        } else {
          q = p;  // dummy partner: identity
        }
        cs[2 * k] = c;
        cs[2 * k + 1] = s;
        pq[2 * k] = p;
        pq[2 * k + 1] = q;
      }
      __syncthreads();
      // 2 x 2 blocks (rows of pair k, columns of pair l): B' = J_k^T B J_l
      for (int w = tid; w < nblk; w += nt) {
        const int k = fdivi(w, np, rnp), l = w - fdivi(w, np, rnp) * np;
        const int p = pq[2 * k], q = pq[2 * k + 1];
        const int r = pq[2 * l], t = pq[2 * l + 1];
        if (p == q && r == t) continue;
        const double ck = cs[2 * k], sk = cs[2 * k + 1];
        const double cl = cs[2 * l], sl = cs[2 * l + 1];
        if (p == q) {  // single row p, columns (r, t)
          const double x0 = a[p * n + r], x1 = a[p * n + t];
          a[p * n + r] = cl * x0 - sl * x1;
          a[p * n + t] = sl * x0 + cl * x1;
        } else if (r == t) {  // rows (p, q), single column r
          const double x0 = a[p * n + r], x1 = a[q * n + r];
          a[p * n + r] = ck * x0 - sk * x1;
          a[q * n + r] = sk * x0 + ck * x1;
        } else {
          const double b00 = a[p * n + r], b01 = a[p * n + t];
          const double b10 = a[q * n + r], b11 = a[q * n + t];
          const double u00 = ck * b00 - sk * b10, u01 = ck * b01 - sk * b11;
          const double u10 = sk * b00 + ck * b10, u11 = sk * b01 + ck * b11;
          a[p * n + r] = cl * u00 - sl * u01;
          a[p * n + t] = sl * u00 + cl * u01;
          a[q * n + r] = cl * u10 - sl * u11;
          a[q * n + t] = sl * u10 + cl * u11;
        }
      }
      // V <- V J: row i, pair l
      for (int w = tid; w < n * np; w += nt) {
        const int i = fdivi(w, np, rnp), l = w - fdivi(w, np, rnp) * np;
        const int r = pq[2 * l], t = pq[2 * l + 1];
        if (r == t || cs[2 * l + 1] == 0.0) continue;
        const double cl = cs[2 * l], sl = cs[2 * l + 1];
        const double x0 = v[i * n + r], x1 = v[i * n + t];
        v[i * n + r] = cl * x0 - sl * x1;
        v[i * n + t] = sl * x0 + cl * x1;
      }
      __syncthreads();
    }
    if (!rot_any) break;
  }
  // sort descending: rank of eigenvalue j = #{i : w_i > w_j or (w_i == w_j and i < j)}
  double* W = Wg + b * sW;
  double* V = Vg + b * sV;
  for (int j = tid; j < n; j += nt) {
    const double wj = a[j * n + j];
    int rank = 0;
    for (int i = 0; i < n; ++i) {
      const double wi = a[i * n + i];
      rank += (wi > wj) || (wi == wj && i < j);
    }
    W[rank] = wj;
    for (int i = 0; i < n; ++i) V[(long long)i * n + rank] = v[i * n + j];
  }
}

// DPP lane moves within a row of 16 lanes (quad_perm swaps, half-row and
// row mirrors) on 64-bit values.
template <int CTRL>
__device__ inline unsigned long long dpp_move_u64(unsigned long long v) {
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(v & 0xffffffffull), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(v >> 32), CTRL, 0xF, 0xF, false);
  return ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
}
template <int CTRL>
__device__ inline double dpp_move(double v) {
  // every lane of these patterns reads a lane of its own row, so no lane
  // keeps an old value and none needs initialising
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}
constexpr int kDppSwap1 = 0xB1;      // quad_perm [1,0,3,2]
constexpr int kDppSwap2 = 0x4E;      // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141; // lane i <-> 7 - i within 8
constexpr int kDppMirror = 0x140;     // lane i <-> 15 - i within 16

// Maximum of a 64-bit key over the 64-lane wave (every lane gets it).
__device__ inline unsigned long long wave_max_u64(unsigned long long k) {
  unsigned long long o;
  o = dpp_move_u64<kDppSwap1>(k);
  k = o > k ? o : k;
  o = dpp_move_u64<kDppSwap2>(k);
  k = o > k ? o : k;
  o = dpp_move_u64<kDppHalfMirror>(k);
  k = o > k ? o : k;
  o = dpp_move_u64<kDppMirror>(k);
  k = o > k ? o : k;
  o = __shfl_xor(k, 16, 64);
  k = o > k ? o : k;
  o = __shfl_xor(k, 32, 64);
  k = o > k ? o : k;
  return k;
}

// 1 / sqrt(x) from the hardware estimate plus two Newton steps
__device__ inline double rsq_nr2(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double h = 0.5 * x * y;
  y = fma(y, fma(-h, y, 0.5), y);
  h = 0.5 * x * y;
  return fma(y, fma(-h, y, 0.5), y);
}

// Maximum of a 32-bit key over the 64-lane wave, returned uniform: DPP
// maxima within each row of 16 lanes, then the four row results read out.
__device__ inline unsigned wave_max_u32(unsigned v) {
  unsigned t;
  t = (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, kDppSwap1, 0xF, 0xF, false);
  v = t > v ? t : v;
  t = (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, kDppSwap2, 0xF, 0xF, false);
  v = t > v ? t : v;
  t = (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, kDppHalfMirror, 0xF, 0xF, false);
  v = t > v ? t : v;
  t = (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, kDppMirror, 0xF, 0xF, false);
  v = t > v ? t : v;
  const unsigned a = __builtin_amdgcn_readlane(v, 0), b = __builtin_amdgcn_readlane(v, 16);
  const unsigned c = __builtin_amdgcn_readlane(v, 32), d = __builtin_amdgcn_readlane(v, 48);
  const unsigned ab = a > b ? a : b, cd = c > d ? c : d;
  return ab > cd ? ab : cd;
}

// Rank-revealing Cholesky with diagonal pivoting of the symmetric positive
// semidefinite n x n matrix G in g (LDS, read only), n <= NMAX <= 64, by
// one wave (lane j owns index j).  Step k takes the largest remaining
// diagonal entry p = perm[k] as pivot (entries within 2^-17 relative of
// each other, compared in FP32 as fractions of the largest initial diagonal
// entry, go to the lower index) and stores the pivot
// column of the factor, in the original index order, as row k of L (LDS,
// n x n, zero on entry): G = sum_{k<r} L[k]^T L[k].  It stops when the
// largest remaining diagonal entry is at most tau times the largest initial
// one and returns r (uniform).  With WITHZ it also builds Z (LDS, n x n,
// zero on entry; row k = z_k, original coordinates), z_k = (e_p - sum_{j<k}
// L[j][p] z_j) / L[k][p], the columns of P R^-1 (Gram-Schmidt in the G
// inner product), so that Y z_k are orthonormal when G = Y^T Y.
// Left-looking: the pivot row of the Schur complement is formed as
// G[p][.] - sum_{m<k} L[m][p] L[m][.] from the rows of L written so far
// (rows not yet written are zero, so chunks of 8 rows are skipped whole
// once past k); the diagonal is kept in registers and updated with the
// new row.  One wave needs no barrier: LDS operations of a wave complete
// in order.
template <int NMAX, bool WITHZ>
__device__ int pchol_wave(int n, const double* __restrict__ g, double* __restrict__ L, double* __restrict__ Z,
                          int* __restrict__ perm, double tau) {
  constexpr int CH = 8;
  static_assert(NMAX % CH == 0, "NMAX is a multiple of the row chunk");
  const int lane = threadIdx.x & 63;
  const int jc = lane < n ? lane : n - 1;  // loads of lanes >= n stay in range
  double dg = lane < n ? g[lane * n + lane] : 0.0;
  const double d0 =
      __longlong_as_double((long long)wave_max_u64((unsigned long long)__double_as_longlong(fmax(dg, 0.0))));
  // keys are taken relative to the largest diagonal entry, so that the FP32
  // comparison neither overflows nor flushes for any scale of G
  const double rel = d0 > 0.0 ? 1.0 / d0 : 0.0;
  bool chosen = lane >= n;
  int r = n;
  for (int k = 0; k < n; ++k) {
    // key: FP32 value bits of the (non-negative) diagonal relative to d0,
    // low 6 bits = 63 - lane
    const float fv = (float)(fmax(dg, 0.0) * rel);
    const unsigned key = wave_max_u32(chosen ? 0u : ((__float_as_uint(fv) & ~63u) | (unsigned)(63 - lane)));
    const int p = 63 - (int)(key & 63u);
    const double best = key == 0u ? 0.0
                                  : __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(dg), p),
                                                     __builtin_amdgcn_readlane(__double2loint(dg), p));
    if (!(best > tau * d0) || !(best > 0.0)) {
      r = k;
      break;
    }
    const double inv = rsq_nr2(best);
    double s0 = g[p * n + jc], s1 = 0.0, a0 = 0.0, a1 = 0.0;
#pragma unroll
    for (int c = 0; c < NMAX / CH; ++c) {
      if (c * CH < k) {
        double lp[CH], lj[CH], zj[CH];
#pragma unroll
        for (int i = 0; i < CH; ++i) {
          const int m = c * CH + i;
          const int mc = m < n ? m : n - 1;
          lp[i] = L[mc * n + p];
          lj[i] = L[mc * n + jc];
          if (WITHZ) zj[i] = Z[mc * n + jc];
        }
#pragma unroll
        for (int i = 0; i < CH; i += 2) {
          s0 = fma(-lp[i], lj[i], s0);
          s1 = fma(-lp[i + 1], lj[i + 1], s1);
          if (WITHZ) {
            a0 = fma(lp[i], zj[i], a0);
            a1 = fma(lp[i + 1], zj[i + 1], a1);
          }
        }
      }
    }
    const double lrow = chosen ? 0.0 : (s0 + s1) * inv;
    if (lane < n) {
      L[k * n + lane] = lrow;
      if (WITHZ) Z[k * n + lane] = (((lane == p) ? 1.0 : 0.0) - (a0 + a1)) * inv;
    }
    dg = fma(-lrow, lrow, dg);
    if (lane == p) chosen = true;
    if (lane == 0) perm[k] = p;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  return r;
}

// S = P R^-1 (n x n) for the pivoted Cholesky factor of G (see
// pchol_wave): Q = Y S has orthonormal columns spanning the numerical
// range of Y when G = Y^T Y; columns r.. of S are zero.
template <int NMAX>
__global__ __launch_bounds__(256) void k_pchol_s(int n, const double* __restrict__ Gg, long long sG, double tau,
                                                 double* __restrict__ Sg, long long sS, int* __restrict__ rank_out) {
  extern __shared__ double sm[];
  double* g = sm;
  double* L = sm + n * n;
  double* Z = sm + 2 * n * n;
  __shared__ int perm[64];
  __shared__ int rank_s;
  const int b = blockIdx.x, tid = threadIdx.x;
  const double* G = Gg + b * sG;
  for (int e = tid; e < n * n; e += 256) {
    g[e] = G[e];
    L[e] = 0.0;
    Z[e] = 0.0;
  }
  __syncthreads();
  if (tid < 64) {
    const int rr = pchol_wave<NMAX, true>(n, g, L, Z, perm, tau);
    if (tid == 0) rank_s = rr;
  }
  __syncthreads();
  const int r = rank_s;
  double* S = Sg + b * sS;
  const int ri = tid >> 2, rj = tid & 3;  // S[o][k] = z_k[o]
  if (ri < n)
    for (int k = rj; k < n; k += 4) S[ri * n + k] = (k < r) ? Z[k * n + ri] : 0.0;
  if (tid == 0 && rank_out != nullptr) rank_out[b] = r;
}

// Truncation basis of a PSD Gram matrix G (n x n, n <= 64) in one block:
// pivoted Cholesky G = L^T L (numerical rank r at tau), then one-sided
// Jacobi on the r columns of W = L^T until every pair is orthogonal to
// eps relative; the columns w_j then give the eigenpairs of G as
// lambda_j = |w_j|^2, v_j = w_j / |w_j|.  Kept: at most c, positive and
// above floor_rel * lambda_max, and (tol2 > 0) the fewest whose dropped
// tail (with the mass below the Cholesky threshold) stays within tol2 *
// trace(G).  S (n x c, row-major) = kept eigenvectors by decreasing
// eigenvalue, zero columns beyond.  Groups of 8 lanes rotate one column
// pair each (round-robin ordering, up to 32 pairs per round).
constexpr int kCutSweeps = 30;
// Sums over each aligned group of 8 (LPG = 16: 16) lanes of three values,
// the same sums in all lanes of the group; the three reductions advance a
// stage at a time so that their DPP moves and adds overlap.
template <int CTRL>
__device__ inline void dpp_add3(double& a, double& b, double& c) {
  const double ta = dpp_move<CTRL>(a), tb = dpp_move<CTRL>(b), tc = dpp_move<CTRL>(c);
  a += ta;
  b += tb;
  c += tc;
}
template <int LPG>
__device__ inline void sum_lanes3(double& a, double& b, double& c) {
  dpp_add3<kDppSwap1>(a, b, c);
  dpp_add3<kDppSwap2>(a, b, c);
  dpp_add3<kDppHalfMirror>(a, b, c);
  if (LPG == 16) dpp_add3<kDppMirror>(a, b, c);
}
// 1 / x and 1 / sqrt(x) from the hardware estimates plus one Newton step
__device__ inline double rcp_nr(double x) {
  const double y = __builtin_amdgcn_rcp(x);
  return fma(y, fma(-x, y, 1.0), y);
}
__device__ inline double rsq_nr(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x * y;
  return fma(y, fma(-h, y, 0.5), y);
}
// NT threads = 8 lanes x NT / 8 column pairs (2 NT / 8 >= n); NE = 8 * NE >= n.
template <int NT, int NE, int LPG = 8>
__global__ __launch_bounds__(NT) void k_cut_psd(int n, int c, const double* __restrict__ Gg, long long sG,
                                                 double tau, double eps, double tol2, double floor_rel,
                                                 double* __restrict__ Sg, long long sS, int* __restrict__ kept_out,
                                                 int* __restrict__ sweeps_out) {
  static_assert(LPG == 8 || LPG == 16, "column pairs are rotated by 8 or 16 lanes");
  constexpr int NP = LPG * NE;  // padded column length
  extern __shared__ double sm[];
  double* g = sm;
  double* L = sm + n * n;          // rows of the pivoted Cholesky factor
  double* W = sm + 2 * n * n;      // column j of W = row j of L, zero-padded to NP
  __shared__ int perm[64];
  __shared__ int order[64];
  __shared__ double lam[64];
  __shared__ int flags[kCutSweeps];
  __shared__ int rank_s;
  __shared__ double trace_s;
  __shared__ int kept_s;
  __shared__ int scale_s;
  const int b = blockIdx.x, tid = threadIdx.x;
  const double* G = Gg + b * sG;
  for (int e = tid; e < n * n; e += NT) {
    g[e] = G[e];
    L[e] = 0.0;
  }
  if (tid < kCutSweeps) flags[tid] = 0;
  __syncthreads();
  // G is used divided by a power of two near its largest diagonal entry
  // (exact): the squared column norms of the Jacobi are then at most
  // trace <= n and the smallest the Cholesky threshold lets through near
  // tau, so the pair tests and angles stay in range whatever the scale of
  // G, and G and 2^k G (neither with subnormal entries) give the same
  // basis bit for bit
  if (tid < 64) {
    double dm = (tid < n) ? fmax(g[tid * n + tid], 0.0) : 0.0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) dm = fmax(dm, __shfl_xor(dm, o, 64));
    if (tid == 0) scale_s = dm > 0.0 ? __builtin_amdgcn_frexp_exp(dm) : 0;
  }
  __syncthreads();
  {
    const int sx = scale_s;
    for (int e = tid; e < n * n; e += NT) g[e] = __builtin_amdgcn_ldexp(g[e], -sx);
  }
  __syncthreads();
  if (tid < 64) {
    double t = (tid < n) ? fmax(g[tid * n + tid], 0.0) : 0.0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
    if (tid == 0) trace_s = t;
  }
  if (tid < 64) {
    const int rr = pchol_wave<NP, false>(n, g, L, nullptr, perm, tau);
    if (tid == 0) rank_s = rr;
  }
  __syncthreads();
  const int r = rank_s;
  for (int e = tid; e < r * NP; e += NT) {
    const int j = e / NP, i = e - (e / NP) * NP;
    W[e] = (i < n) ? L[j * n + i] : 0.0;
  }
  __syncthreads();
  // one-sided Jacobi on columns 0..r-1 of W (the zero padding rotates into
  // zeros, so the lanes need no bounds tests)
  const int sub = tid % LPG, grp = tid / LPG;
  const int m = r + (r & 1), np = m / 2;
  const double eps2 = (eps * n) * (eps * n);
  // a sweep whose rotations all had |cos angle between the columns| below
  // sqrt(eps n) leaves pairs at O(eps n) (quadratic convergence): stop there
  // instead of spending a further sweep to observe it
  const double big2 = eps * n;
  int sweeps = 0;
  for (int sweep = 0; sweep < kCutSweeps && r > 1; ++sweep) {
    sweeps = sweep + 1;
    // the group's two positions, less one, advance by one per step modulo
    // m - 1 (group 0 keeps position 0)
    int u0 = grp - 1, u1 = m - 2 - grp;
    for (int step = 0; step < m - 1; ++step) {
      const int t0 = grp == 0 ? 0 : 1 + u0, t1 = 1 + u1;
      u0 = u0 + 1 == m - 1 ? 0 : u0 + 1;
      u1 = u1 + 1 == m - 1 ? 0 : u1 + 1;
      if (grp < np) {
        const int p = t0 < t1 ? t0 : t1, q = t0 < t1 ? t1 : t0;
        if (q < r) {
          double wp[NE], wq[NE];
          double a = 0.0, bb = 0.0, gg = 0.0;
#pragma unroll
          for (int t = 0; t < NE; ++t) {
            const int i = sub + LPG * t;
            wp[t] = W[p * NP + i];
            wq[t] = W[q * NP + i];
            a += wp[t] * wp[t];
            bb += wq[t] * wq[t];
            gg += wp[t] * wq[t];
          }
          sum_lanes3<LPG>(a, bb, gg);
          if (gg * gg > eps2 * a * bb) {
            // the rotation angle comes from the hardware estimates alone:
            // any angle gives an orthogonal rotation, and an angle off by
            // the estimates' relative error leaves the pair's inner product
            // at that fraction of its old value for the next sweep; c is
            // refined so that c^2 (1 + t^2) = 1 to rounding.  t is the
            // smaller root of t^2 + 2 z t - 1 = 0 with z = (b - a) / (2 g),
            // written as sign(b - a) 2 g / (|b - a| + hypot(b - a, 2 g)) so
            // that no quotient can overflow when g is tiny against b - a
            // (a, b <= trace(G) <= n after the scaling, so the squares stay
            // in range)
            const double tau = bb - a, rho = 2.0 * gg;
            const double w = fma(tau, tau, rho * rho);
            const double h = w * __builtin_amdgcn_rsq(w);
            const double t = (tau >= 0.0 ? rho : -rho) * __builtin_amdgcn_rcp(fabs(tau) + h);
            const double cs = rsq_nr(1.0 + t * t), sn = t * cs;
#pragma unroll
            for (int tt = 0; tt < NE; ++tt) {
              const int i = sub + LPG * tt;
              W[p * NP + i] = cs * wp[tt] - sn * wq[tt];
              W[q * NP + i] = sn * wp[tt] + cs * wq[tt];
            }
            if (sub == 0 && gg * gg > big2 * a * bb) flags[sweep] = 1;
          }
        }
      }
      __syncthreads();
    }
    if (!flags[sweep]) break;
  }
  // eigenvalues, order by decreasing value (ties: lower index first)
  if (tid < r) {
    double v = 0.0;
    for (int i = 0; i < n; ++i) v += W[tid * NP + i] * W[tid * NP + i];
    lam[tid] = v;
  }
  __syncthreads();
  if (tid < r) {
    const double v = lam[tid];
    int rank = 0;
    for (int i = 0; i < r; ++i) rank += (lam[i] > v) || (lam[i] == v && i < tid);
    order[rank] = tid;
  }
  __syncthreads();
  if (tid == 0) {
    double sum = 0.0;
    for (int j = 0; j < r; ++j) sum += lam[j];
    int kept = c < r ? c : r;
    const double l0 = r > 0 ? lam[order[0]] : 0.0;
    while (kept > 0 && !(lam[order[kept - 1]] > floor_rel * l0 && lam[order[kept - 1]] > 0.0)) --kept;
    if (tol2 > 0.0) {
      const double total = trace_s;
      double tail = fmax(total - sum, 0.0);
      for (int j = r - 1; j >= kept; --j) tail += lam[order[j]];
      while (kept > 1) {
        const double t2 = tail + lam[order[kept - 1]];
        if (t2 <= tol2 * total) {
          tail = t2;
          --kept;
        } else {
          break;
        }
      }
    }
    kept_s = kept;
    if (kept_out != nullptr) kept_out[b] = kept;
    if (sweeps_out != nullptr) sweeps_out[b] = sweeps;
  }
  __syncthreads();
  const int kept = kept_s;
  double* S = Sg + b * sS;
  for (int e = tid; e < n * c; e += NT) {
    const int i = e / c, j = e - (e / c) * c;
    double v = 0.0;
    if (j < kept) {
      const int col = order[j];
      v = W[col * NP + i] / sqrt(lam[col]);
    }
    S[e] = v;
  }
}

// ---------------------------------------------------------------- n <= 128
// The factorisations above keep G, the factor and Z (or the Jacobi columns)
// as separate n x n arrays in LDS, which caps n at 64.  Sketch sizes up to
// 128 (rank caps up to about 118) use the forms below, which hold the
// Schur complement in registers spread over the whole block.

constexpr int kBigN = 128;

// Maximum of a 32-bit key with ties impossible: the low 7 bits carry
// 127 - index.
__device__ inline int pivot_of(unsigned key) { return 127 - (int)(key & 127u); }

// Rank-revealing pivoted Cholesky of a PSD n x n matrix, n <= NP <= 128,
// right-looking over a block of NT = (NP / BR) (NP / BC) threads: thread
// (ti, tj) holds in a[][] the BR x BC block of the Schur complement at rows
// BR ti.., columns BC tj.. (zero beyond n), and with WITHZ the same block of
// bz[q][j] = sum_{m<k} L[m][q] z_m[j] (zero on entry).  Step k takes the
// largest remaining diagonal entry p as pivot (the key rule of pchol_wave:
// FP32 value bits relative to the largest initial diagonal entry d0, ties
// to the lower index), publishes row p of both through LDS, and stops when
// that entry is at most tau d0.  The factor row is L[k][j] = a[p][j] /
// sqrt(a[p][p]) at the indices not chosen before (zero at the others); z_k
// (column k of P R^-1, so that Y z_k are orthonormal when G = Y^T Y) is
// 1 / L[k][p] at p, -bz[p][j] / L[k][p] at the indices chosen before and
// zero elsewhere.  Every entry is updated by fma(-L[k][i], L[k][j], a)
// (and bz by fma(L[k][q], z_k[j], bz)) in step order, which are the fma
// chains of the left-looking formation.  out(k, j, L[k][j], z_k[j]) is
// called once per step and index j < NP by the threads of block row 0.
// Returns the rank r (uniform).  LDS: rowbuf (2 NP doubles), keys (2),
// dmax (1).  Every thread of the block must call it.
template <int NT, int NP, int BR, int BC, bool WITHZ, class Out>
__device__ int pchol_block(int n, double (&a)[BR][BC], double (&bz)[BR][BC], double tau, double* rowbuf,
                           unsigned* keys, unsigned long long* dmax, Out out) {
  constexpr int TC = NP / BC;
  static_assert((NP / BR) * TC == NT && NP % BR == 0 && NP % BC == 0 && NP <= kBigN, "block grid");
  const int tid = threadIdx.x, ti = tid / TC, tj = tid - (tid / TC) * TC;
  const int i0 = BR * ti, j0 = BC * tj;
  // chosen (or absent) row and column indices of this thread's block
  unsigned rch = 0u, cch = 0u;
#pragma unroll
  for (int u = 0; u < BR; ++u) rch |= (i0 + u >= n) ? (1u << u) : 0u;
#pragma unroll
  for (int v = 0; v < BC; ++v) cch |= (j0 + v >= n) ? (1u << v) : 0u;
  // largest key over this thread's diagonal entries (0: none left)
  auto diag_key = [&](double rel) -> unsigned {
    unsigned best = 0u;
#pragma unroll
    for (int u = 0; u < BR; ++u)
#pragma unroll
      for (int v = 0; v < BC; ++v)
        if (i0 + u == j0 + v && !((rch >> u) & 1u)) {
          const float fv = (float)(fmax(a[u][v], 0.0) * rel);
          const unsigned q = (__float_as_uint(fv) & ~127u) | (unsigned)(127 - (i0 + u));
          best = q > best ? q : best;
        }
    return best;
  };
  if (tid == 0) {
    keys[0] = 0u;
    keys[1] = 0u;
    *dmax = 0ull;
  }
  __syncthreads();
  {
    unsigned long long dm = 0ull;
#pragma unroll
    for (int u = 0; u < BR; ++u)
#pragma unroll
      for (int v = 0; v < BC; ++v)
        if (i0 + u == j0 + v && i0 + u < n) {
          const unsigned long long q = (unsigned long long)__double_as_longlong(fmax(a[u][v], 0.0));
          dm = q > dm ? q : dm;
        }
    if (dm != 0ull) atomicMax(dmax, dm);
  }
  __syncthreads();
  const double d0 = __longlong_as_double((long long)*dmax);
  const double rel = d0 > 0.0 ? 1.0 / d0 : 0.0;
  {
    const unsigned q = diag_key(rel);
    if (q != 0u) atomicMax(&keys[0], q);
  }
  __syncthreads();
  int r = n;
  for (int k = 0; k < n; ++k) {
    const unsigned key = keys[k & 1];
    const int p = pivot_of(key);
    if (tid == 0) keys[(k + 1) & 1] = 0u;
    // publish row p (its owners: block row p / BR)
    if (ti == p / BR) {
      const int up = p - i0;
#pragma unroll
      for (int u = 0; u < BR; ++u)
        if (u == up) {
#pragma unroll
          for (int v = 0; v < BC; ++v) {
            rowbuf[j0 + v] = a[u][v];
            if (WITHZ) rowbuf[NP + j0 + v] = bz[u][v];
          }
        }
    }
    __syncthreads();
    const double best = key == 0u ? 0.0 : rowbuf[p];
    if (!(best > tau * d0) || !(best > 0.0)) {
      r = k;
      break;
    }
    const double inv = rsq_nr2(best);
    double li[BR], lj[BC], zj[BC];
#pragma unroll
    for (int u = 0; u < BR; ++u) li[u] = ((rch >> u) & 1u) ? 0.0 : rowbuf[i0 + u] * inv;
#pragma unroll
    for (int v = 0; v < BC; ++v) {
      const bool chv = (cch >> v) & 1u;
      lj[v] = chv ? 0.0 : rowbuf[j0 + v] * inv;
      if (WITHZ) zj[v] = (j0 + v == p) ? inv : (chv ? -rowbuf[NP + j0 + v] * inv : 0.0);
    }
    if (ti == 0)
#pragma unroll
      for (int v = 0; v < BC; ++v) out(k, j0 + v, lj[v], WITHZ ? zj[v] : 0.0);
#pragma unroll
    for (int u = 0; u < BR; ++u)
#pragma unroll
      for (int v = 0; v < BC; ++v) {
        a[u][v] = fma(-li[u], lj[v], a[u][v]);
        if (WITHZ) bz[u][v] = fma(li[u], zj[v], bz[u][v]);
      }
    if (p >= i0 && p < i0 + BR) rch |= 1u << (p - i0);
    if (p >= j0 && p < j0 + BC) cch |= 1u << (p - j0);
    {
      const unsigned q = diag_key(rel);
      if (q != 0u) atomicMax(&keys[(k + 1) & 1], q);
    }
    __syncthreads();
  }
  return r;
}

// S = P R^-1 (n x n, 64 < n <= 128) of the pivoted Cholesky factor of G
// (pchol_block, 512 threads holding 8 x 4 blocks); see k_pchol_s.
__global__ __launch_bounds__(512) void k_pchol_s_big(int n, const double* __restrict__ Gg, long long sG, double tau,
                                                     double* __restrict__ Sg, long long sS,
                                                     int* __restrict__ rank_out) {
  constexpr int NT = 512, NP = kBigN, BR = 8, BC = 4, TC = NP / BC;
  __shared__ double rowbuf[2 * NP];
  __shared__ unsigned keys[2];
  __shared__ unsigned long long dmax;
  const int b = blockIdx.x, tid = threadIdx.x;
  const int i0 = BR * (tid / TC), j0 = BC * (tid - (tid / TC) * TC);
  const double* G = Gg + b * sG;
  double* S = Sg + b * sS;
  double a[BR][BC], bz[BR][BC];
#pragma unroll
  for (int u = 0; u < BR; ++u)
#pragma unroll
    for (int v = 0; v < BC; ++v) {
      const int i = i0 + u, j = j0 + v;
      a[u][v] = (i < n && j < n) ? G[(long long)i * n + j] : 0.0;
      bz[u][v] = 0.0;
    }
  // S[o][k] = z_k[o]
  const int r = pchol_block<NT, NP, BR, BC, true>(n, a, bz, tau, rowbuf, keys, &dmax,
                                                  [&](int k, int j, double, double z) {
                                                    if (j < n) S[(long long)j * n + k] = z;
                                                  });
  for (int e = tid; e < n * n; e += NT) {
    const int k = e - (e / n) * n;
    if (k >= r) S[e] = 0.0;
  }
  if (tid == 0 && rank_out != nullptr) rank_out[b] = r;
}

// Truncation basis of a PSD Gram matrix G (n x n, 64 < n <= 128): the
// steps of k_cut_psd (scaling, pivoted Cholesky, one-sided Jacobi on the
// factor's rows, selection), the factor formed by pchol_block (the whole
// block, 4 x 4 or 3 x 4 register blocks) and written in pivot order.
// NT = 16 lanes x NT / 16 column pairs (2 NT / 16 >= n), rows padded to
// NP = 16 NE >= n.
template <int NT, int NE>
__global__ __launch_bounds__(NT) void k_cut_psd_big(int n, int c, const double* __restrict__ Gg, long long sG,
                                                     double tau, double eps, double tol2, double floor_rel,
                                                     double* __restrict__ Sg, long long sS,
                                                     int* __restrict__ kept_out, int* __restrict__ sweeps_out) {
  constexpr int LPG = 16;
  constexpr int NP = LPG * NE;
  constexpr int BR = NP / 32, BC = 4, TC = NP / BC;  // pchol_block grid: 32 x TC threads
  extern __shared__ double sm[];
  double* W = sm;  // n rows of stride NP
  __shared__ int order[kBigN];
  __shared__ double lam[kBigN];
  __shared__ int flags[kCutSweeps];
  __shared__ double trace_s;
  __shared__ int kept_s;
  __shared__ unsigned long long dm_s;
  __shared__ double rowbuf[NP];
  __shared__ unsigned keys[2];
  __shared__ unsigned long long dmax;
  const int b = blockIdx.x, tid = threadIdx.x;
  const int i0 = BR * (tid / TC), j0 = BC * (tid - (tid / TC) * TC);
  const double* G = Gg + b * sG;
  for (int e = tid; e < n * NP; e += NT) W[e] = 0.0;
  if (tid < kCutSweeps) flags[tid] = 0;
  if (tid == 0) dm_s = 0ull;
  double a[BR][BC], bz[BR][BC];
#pragma unroll
  for (int u = 0; u < BR; ++u)
#pragma unroll
    for (int v = 0; v < BC; ++v) {
      const int i = i0 + u, j = j0 + v;
      a[u][v] = (i < n && j < n) ? G[(long long)i * n + j] : 0.0;
      bz[u][v] = 0.0;
    }
  __syncthreads();
  // scale by a power of two near the largest diagonal entry (see k_cut_psd)
  {
    unsigned long long dm = 0ull;
#pragma unroll
    for (int u = 0; u < BR; ++u)
#pragma unroll
      for (int v = 0; v < BC; ++v)
        if (i0 + u == j0 + v && i0 + u < n) {
          const unsigned long long q = (unsigned long long)__double_as_longlong(fmax(a[u][v], 0.0));
          dm = q > dm ? q : dm;
        }
    if (dm != 0ull) atomicMax(&dm_s, dm);
  }
  __syncthreads();
  const double dmx = __longlong_as_double((long long)dm_s);
  const int sx = dmx > 0.0 ? __builtin_amdgcn_frexp_exp(dmx) : 0;
#pragma unroll
  for (int u = 0; u < BR; ++u)
#pragma unroll
    for (int v = 0; v < BC; ++v) a[u][v] = __builtin_amdgcn_ldexp(a[u][v], -sx);
  if (tid < 64) {
    double t = 0.0;
    for (int i = tid; i < n; i += 64) t += fmax(__builtin_amdgcn_ldexp(G[(long long)i * n + i], -sx), 0.0);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
    if (tid == 0) trace_s = t;
  }
  // factor row k -> row k of W (rows r.. stay zero)
  const int r = pchol_block<NT, NP, BR, BC, false>(n, a, bz, tau, rowbuf, keys, &dmax,
                                                   [&](int k, int j, double l, double) { W[k * NP + j] = l; });
  __syncthreads();
  // one-sided Jacobi on rows 0..r-1 of W, as in k_cut_psd
  const int sub = tid % LPG, grp = tid / LPG;
  const int m = r + (r & 1), np = m / 2;
  const double eps2 = (eps * n) * (eps * n);
  const double big2 = eps * n;
  int sweeps = 0;
  for (int sweep = 0; sweep < kCutSweeps && r > 1; ++sweep) {
    sweeps = sweep + 1;
    int u0 = grp - 1, u1 = m - 2 - grp;
    for (int step = 0; step < m - 1; ++step) {
      const int t0 = grp == 0 ? 0 : 1 + u0, t1 = 1 + u1;
      u0 = u0 + 1 == m - 1 ? 0 : u0 + 1;
      u1 = u1 + 1 == m - 1 ? 0 : u1 + 1;
      if (grp < np) {
        const int p = t0 < t1 ? t0 : t1, q = t0 < t1 ? t1 : t0;
        if (q < r) {
          double wp[NE], wq[NE];
          double a = 0.0, bb = 0.0, gg = 0.0;
#pragma unroll
          for (int t = 0; t < NE; ++t) {
            const int i = sub + LPG * t;
            wp[t] = W[p * NP + i];
            wq[t] = W[q * NP + i];
            a += wp[t] * wp[t];
            bb += wq[t] * wq[t];
            gg += wp[t] * wq[t];
          }
          sum_lanes3<LPG>(a, bb, gg);
          if (gg * gg > eps2 * a * bb) {
            const double tau_ = bb - a, rho = 2.0 * gg;
            const double w = fma(tau_, tau_, rho * rho);
            const double h = w * __builtin_amdgcn_rsq(w);
            const double t = (tau_ >= 0.0 ? rho : -rho) * __builtin_amdgcn_rcp(fabs(tau_) + h);
            const double cs = rsq_nr(1.0 + t * t), sn = t * cs;
#pragma unroll
            for (int tt = 0; tt < NE; ++tt) {
              const int i = sub + LPG * tt;
              W[p * NP + i] = cs * wp[tt] - sn * wq[tt];
              W[q * NP + i] = sn * wp[tt] + cs * wq[tt];
            }
            if (sub == 0 && gg * gg > big2 * a * bb) flags[sweep] = 1;
          }
        }
      }
      __syncthreads();
    }
    if (!flags[sweep]) break;
  }
  for (int j = tid; j < r; j += NT) {
    double v = 0.0;
    for (int i = 0; i < n; ++i) v += W[j * NP + i] * W[j * NP + i];
    lam[j] = v;
  }
  __syncthreads();
  for (int j = tid; j < r; j += NT) {
    const double v = lam[j];
    int rank = 0;
    for (int i = 0; i < r; ++i) rank += (lam[i] > v) || (lam[i] == v && i < j);
    order[rank] = j;
  }
  __syncthreads();
  if (tid == 0) {
    double sum = 0.0;
    for (int j = 0; j < r; ++j) sum += lam[j];
    int kept = c < r ? c : r;
    const double l0 = r > 0 ? lam[order[0]] : 0.0;
    while (kept > 0 && !(lam[order[kept - 1]] > floor_rel * l0 && lam[order[kept - 1]] > 0.0)) --kept;
    if (tol2 > 0.0) {
      const double total = trace_s;
      double tail = fmax(total - sum, 0.0);
      for (int j = r - 1; j >= kept; --j) tail += lam[order[j]];
      while (kept > 1) {
        const double t2 = tail + lam[order[kept - 1]];
        if (t2 <= tol2 * total) {
          tail = t2;
          --kept;
        } else {
          break;
        }
      }
    }
    kept_s = kept;
    if (kept_out != nullptr) kept_out[b] = kept;
    if (sweeps_out != nullptr) sweeps_out[b] = sweeps;
  }
  __syncthreads();
  const int kept = kept_s;
  double* S = Sg + b * sS;
  for (int e = tid; e < n * c; e += NT) {
    const int i = e / c, j = e - (e / c) * c;
    double v = 0.0;
    if (j < kept) {
      const int col = order[j];
      v = W[col * NP + i] / sqrt(lam[col]);
    }
    S[e] = v;
  }
}

}  // namespace

size_t gemm_scratch_doubles(const Gemm& g) {
  const int ks = choose_ksplit(g);
  if (ks <= 1) return 0;
  return (size_t)g.batch * ks * g.m * g.n;
}

int gemm(const Gemm& g, double* scratch, size_t scratch_doubles, hipStream_t s) {
  if (g.m <= 0 || g.n <= 0 || g.batch <= 0) return LRFG_OK;
  if ((g.bcw > 0 && (g.tb || g.prec != 0)) || (g.ccw > 0 && g.prec != 0)) {
    set_error("gemm: column maps need FP64 and an untransposed B");
    return LRFG_EUNSUPPORTED;
  }
  int ks = choose_ksplit(g);
  if (ks > 1) {
    // as many splits as the scratch holds for one matrix
    const size_t per1 = (size_t)g.m * g.n;
    const size_t fit = scratch == nullptr ? 0 : scratch_doubles / per1;
    if ((size_t)ks > fit) ks = (int)fit;
    if (ks < 2) ks = 1;
  }
  const GemmLayout lay = g.prec != 0 ? GemmLayout{2, 2} : gemm_layout(g);
  const int KQ = g.prec != 0 ? LK : lay.tk();  // K slab of the kernel used
  const int kchunk = ks > 1 ? ((g.k + ks - 1) / ks + KQ - 1) / KQ * KQ : (g.k > 0 ? g.k : 1);
  if (ks > 1) ks = (g.k + kchunk - 1) / kchunk;
  // matrices per launch: all of them, or as many as the split partials fit,
  // within the grid's z limit
  int chunk = g.batch;
  if (ks > 1) {
    const size_t per = (size_t)ks * g.m * g.n;
    chunk = (int)std::min<size_t>((size_t)g.batch, scratch_doubles / per);
  }
  chunk = std::min(chunk, 65535 / ks);
  double* part = ks > 1 ? scratch : nullptr;
  for (int b0 = 0; b0 < g.batch; b0 += chunk) {
    Gemm c = g;
    c.batch = std::min(chunk, g.batch - b0);
    const BatchMap bm{b0, g.adiv, g.amod, g.bdiv, g.bmod, g.sA2, g.sB2, g.cdiv, g.cmod, g.sC2,
                      g.bcw, g.ccw, g.bchi, g.cchi};
    const int gtm = c.prec != 0 ? BM : lay.tm(), gtn = c.prec != 0 ? BN : lay.tn();
    dim3 grid(ceil_div(c.n, gtn), ceil_div(c.m, gtm), c.batch * ks);
#define LRFG_GEMM_F64(TA, TB, WM, WN)                                                                         \
  LRFG_LAUNCH_TIMED("gemm", 2.0 * c.m * c.n * (double)c.k * c.batch, (k_gemm<TA, TB, WM, WN>), grid, dim3(256), \
                    0, s, c.m, c.n, c.k, c.A, c.lda, c.sA, c.B, c.ldb, c.sB, c.C, c.ldc, c.sC, c.alpha, c.beta, ks, \
                    kchunk, part, bm)
#define LRFG_GEMM_LAUNCH(TA, TB)                                                                              \
  do {                                                                                                       \
    if (c.prec == LRFG_PREC_MIXED_FP32)                                                                      \
      LRFG_LAUNCH_TIMED("gemm", 2.0 * c.m * c.n * (double)c.k * c.batch, (k_gemm_lp<TA, TB, false>), grid,   \
                        dim3(256), 0, s, c.m, c.n, c.k, c.A, c.lda, c.sA, c.B, c.ldb, c.sB, c.C, c.ldc, c.sC,   \
                        c.alpha, c.beta, ks, kchunk, part, bm);                                              \
    else if (c.prec == LRFG_PREC_MIXED_BF16)                                                                 \
      LRFG_LAUNCH_TIMED("gemm", 2.0 * c.m * c.n * (double)c.k * c.batch, (k_gemm_lp<TA, TB, true>), grid,    \
                        dim3(256), 0, s, c.m, c.n, c.k, c.A, c.lda, c.sA, c.B, c.ldb, c.sB, c.C, c.ldc, c.sC,   \
                        c.alpha, c.beta, ks, kchunk, part, bm);                                              \
    else if (lay.wm == 1 && lay.wn == 1) LRFG_GEMM_F64(TA, TB, 1, 1);                                         \
    else if (lay.wm == 2 && lay.wn == 1) LRFG_GEMM_F64(TA, TB, 2, 1);                                         \
    else if (lay.wm == 4 && lay.wn == 1) LRFG_GEMM_F64(TA, TB, 4, 1);                                         \
    else if (lay.wm == 1 && lay.wn == 2) LRFG_GEMM_F64(TA, TB, 1, 2);                                         \
    else if (lay.wm == 1 && lay.wn == 4) LRFG_GEMM_F64(TA, TB, 1, 4);                                         \
    else if (lay.wm == 4 && lay.wn == 4)                                                                      \
      LRFG_LAUNCH_TIMED("gemm", 2.0 * c.m * c.n * (double)c.k * c.batch, (k_gemm128<TA, TB>), grid, dim3(256),   \
                        0, s, c.m, c.n, c.k, c.A, c.lda, c.sA, c.B, c.ldb, c.sB, c.C, c.ldc, c.sC, c.alpha, c.beta, \
                        ks, kchunk, part, bm);                                                               \
    else if (lay.wm == 3 && lay.wn == 3)                                                                      \
      LRFG_LAUNCH_TIMED("gemm", 2.0 * c.m * c.n * (double)c.k * c.batch, (k_gemm96<TA, TB>), grid, dim3(256),    \
                        0, s, c.m, c.n, c.k, c.A, c.lda, c.sA, c.B, c.ldb, c.sB, c.C, c.ldc, c.sC, c.alpha, c.beta, \
                        ks, kchunk, part, bm);                                                               \
    else if (lay.wm == 5)                                                                                     \
      LRFG_LAUNCH_TIMED("gemm", 2.0 * c.m * c.n * (double)c.k * c.batch, (k_gemm80<TA, TB>), grid, dim3(256),    \
                        0, s, c.m, c.n, c.k, c.A, c.lda, c.sA, c.B, c.ldb, c.sB, c.C, c.ldc, c.sC, c.alpha, c.beta, \
                        ks, kchunk, part, bm);                                                               \
    else LRFG_GEMM_F64(TA, TB, 2, 2);                                                                         \
  } while (0)
    if (!c.ta && !c.tb) LRFG_GEMM_LAUNCH(false, false);
    else if (c.ta && !c.tb) LRFG_GEMM_LAUNCH(true, false);
    else if (!c.ta && c.tb) LRFG_GEMM_LAUNCH(false, true);
    else LRFG_GEMM_LAUNCH(true, true);
#undef LRFG_GEMM_LAUNCH
#undef LRFG_GEMM_F64
    LRFG_LAUNCHED();
    if (ks > 1) {
      const long long tot = (long long)c.batch * c.m * c.n;
      const int gr = (int)((tot + 31) / 32);
      hipLaunchKernelGGL(k_splitk_reduce, dim3(gr), dim3(256), 0, s, c.m, c.n, ks, c.batch, (const double*)part,
                         c.C, c.ldc, c.sC, c.alpha, c.beta, bm);
      LRFG_LAUNCHED();
    }
  }
  return LRFG_OK;
}

namespace {
constexpr int kDotChunk = 16384;  // elements per block of dot_rows
__global__ __launch_bounds__(256) void k_dot_partial(long long n, const double* __restrict__ x, long long sx,
                                                     int xdiv, const double* __restrict__ y, long long sy,
                                                     int nblk, double* __restrict__ part) {
  __shared__ double red[4];
  const int t = blockIdx.y, blk = blockIdx.x;
  const double* xp = x + (long long)(t / xdiv) * sx;
  const double* yp = y + (long long)t * sy;
  const long long i0 = (long long)blk * kDotChunk, i1 = min(n, i0 + kDotChunk);
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  long long i = i0 + threadIdx.x;
  for (; i + 768 < i1; i += 1024) {
    a0 += xp[i] * yp[i];
    a1 += xp[i + 256] * yp[i + 256];
    a2 += xp[i + 512] * yp[i + 512];
    a3 += xp[i + 768] * yp[i + 768];
  }
  for (; i < i1; i += 256) a0 += xp[i] * yp[i];
  double v = (a0 + a1) + (a2 + a3);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) part[(long long)t * nblk + blk] = (red[0] + red[1]) + (red[2] + red[3]);
}
}  // namespace

size_t dot_rows_scratch(long long n, int batch) {
  const long long nblk = (n + kDotChunk - 1) / kDotChunk;
  return (size_t)(nblk < 1 ? 1 : nblk) * batch;
}

int dot_rows(long long n, const double* x, long long sx, int xdiv, const double* y, long long sy, double* out,
             int batch, double* scratch, size_t scratch_doubles, hipStream_t s) {
  if (batch <= 0) return LRFG_OK;
  const int nblk = (int)std::max<long long>(1, (n + kDotChunk - 1) / kDotChunk);
  if (scratch == nullptr || scratch_doubles < (size_t)nblk * batch) {
    set_error("dot_rows: scratch too small");
    return LRFG_EWORKSPACE;
  }
  hipLaunchKernelGGL(k_dot_partial, dim3(nblk, batch), dim3(256), 0, s, n, x, sx, xdiv < 1 ? 1 : xdiv, y, sy, nblk,
                     scratch);
  LRFG_LAUNCHED();
  const int gr = (batch + 31) / 32;
  const BatchMap bm{0, 1, 0, 1, 0, 0, 0, 1, 0, 0};
  hipLaunchKernelGGL(k_splitk_reduce, dim3(gr), dim3(256), 0, s, 1, 1, nblk, batch, (const double*)scratch, out,
                     (long long)1, (long long)1, 1.0, 0.0, bm);
  LRFG_LAUNCHED();
  return LRFG_OK;
}

int syevj(int n, const double* A, long long lda, long long sA, double* W, long long sW, double* V, long long sV,
          int batch, hipStream_t s) {
  if (n < 1 || n > kMaxSyevj) {
    set_error("syevj: n = %d outside [1, %d]", n, kMaxSyevj);
    return LRFG_EINVAL;
  }
  if (batch <= 0) return LRFG_OK;
  const size_t shm = sizeof(double) * 2 * n * n;
  static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_syevj),
                                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                                     (int)(sizeof(double) * 2 * kMaxSyevj * kMaxSyevj));
  (void)attr;
  ProfScope ps_("syevj", s);
  hipLaunchKernelGGL(k_syevj, dim3(batch), dim3(256), shm, s, n, A, lda, sA, W, sW, V, sV, 20);
  LRFG_LAUNCHED();
  return LRFG_OK;
}

int pchol_s(int n, const double* G, long long sG, double tau, double* S, long long sS, int* rank, int batch,
            hipStream_t s) {
  if (n < 1 || n > kMaxEig) {
    set_error("pchol: n = %d outside [1, %d]", n, kMaxEig);
    return LRFG_EINVAL;
  }
  if (batch <= 0) return LRFG_OK;
  ProfScope ps_("pchol", s);
  if (n > 64) {
    hipLaunchKernelGGL(k_pchol_s_big, dim3(batch), dim3(512), 0, s, n, G, sG, tau, S, sS, rank);
    LRFG_LAUNCHED();
    return LRFG_OK;
  }
  const size_t shm = sizeof(double) * 3 * n * n;
  static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_pchol_s<64>),
                                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                                     (int)(sizeof(double) * 3 * 64 * 64));
  (void)attr;
  if (n <= 32)
    hipLaunchKernelGGL(k_pchol_s<32>, dim3(batch), dim3(256), shm, s, n, G, sG, tau, S, sS, rank);
  else
    hipLaunchKernelGGL(k_pchol_s<64>, dim3(batch), dim3(256), shm, s, n, G, sG, tau, S, sS, rank);
  LRFG_LAUNCHED();
  return LRFG_OK;
}

int cut_psd(int n, int c, const double* G, long long sG, double tol2, double* S, long long sS, int* kept, int batch,
            hipStream_t s, int* sweeps) {
  if (n < 1 || n > kMaxEig || c < 1) {
    set_error("cut: n = %d outside [1, %d] or c = %d < 1", n, kMaxEig, c);
    return LRFG_EINVAL;
  }
  if (batch <= 0) return LRFG_OK;
  if (n > 64) {
    ProfScope ps_("cut", s);
#define LRFG_CUT_BIG(NT, NE)                                                                                 \
  do {                                                                                                       \
    static const hipError_t attr = hipFuncSetAttribute(                                                      \
        reinterpret_cast<const void*>(&k_cut_psd_big<NT, NE>), hipFuncAttributeMaxDynamicSharedMemorySize,   \
        (int)(sizeof(double) * kMaxEig * 16 * NE));                                                          \
    (void)attr;                                                                                              \
    hipLaunchKernelGGL((k_cut_psd_big<NT, NE>), dim3(batch), dim3(NT), sizeof(double) * n * 16 * NE, s, n, c, \
                       G, sG, kCutTau, kCutEps, tol2, kCutFloor, S, sS, kept, sweeps);                       \
  } while (0)
    // 16 lanes per column pair; rows padded to 96 or 128
    if (n <= 96)
      LRFG_CUT_BIG(768, 6);
    else
      LRFG_CUT_BIG(1024, 8);
#undef LRFG_CUT_BIG
    LRFG_LAUNCHED();
    return LRFG_OK;
  }
  const int np_ = n <= 16 ? 16 : (n <= 32 ? 32 : 64);  // padded column length of the launched variant
  const size_t shm = sizeof(double) * (2 * n * n + (size_t)n * np_);
  ProfScope ps_("cut", s);
#define LRFG_CUT_LAUNCH(NT, NE, LPG)                                                                          \
  do {                                                                                                       \
    static const hipError_t attr = hipFuncSetAttribute(                                                      \
        reinterpret_cast<const void*>(&k_cut_psd<NT, NE, LPG>), hipFuncAttributeMaxDynamicSharedMemorySize,  \
        (int)(sizeof(double) * 3 * 64 * 64));                                                                \
    (void)attr;                                                                                              \
    hipLaunchKernelGGL((k_cut_psd<NT, NE, LPG>), dim3(batch), dim3(NT), shm, s, n, c, G, sG, kCutTau, kCutEps, \
                       tol2, kCutFloor, S, sS, kept, sweeps);                                                \
  } while (0)
  // lanes per column pair: 8 in one wave up to n = 16; 16 in four waves up
  // to n = 32 (a shorter dependent chain per rotation step, measured 7 %
  // faster than 8 lanes in two waves at n = 26); 8 in four waves beyond
  if (n <= 16)
    LRFG_CUT_LAUNCH(64, 2, 8);
  else if (n <= 32)
    LRFG_CUT_LAUNCH(256, 2, 16);
  else
    LRFG_CUT_LAUNCH(256, 8, 8);
#undef LRFG_CUT_LAUNCH
  LRFG_LAUNCHED();
  return LRFG_OK;
}

}  // namespace lrfg
