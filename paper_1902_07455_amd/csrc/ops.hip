// Operation-level C-ABI entry points of the low-rank path: batched GEMM,
// batched symmetric eigensolver and TT rounding, each callable on its own.
#include <algorithm>

#include "common.h"
#include "linalg.h"
#include "tt.h"
#include "tucker.h"

using namespace lrfg;

namespace {

int tt_round_sizes(int d, const int N[3], const int rin[4], int cap, int oversample, int c[4], Rounder& R,
                   int nE) {
  if (d != 2 && d != 3) {
    set_error("d must be 2 or 3");
    return LRFG_EINVAL;
  }
  for (int j = 0; j < d; ++j)
    if (N[j] < 1) {
      set_error("N must be positive");
      return LRFG_EINVAL;
    }
  if (rin[0] != 1 || rin[d] != 1) {
    set_error("r_0 = r_d = 1 required");
    return LRFG_EINVAL;
  }
  if (cap < 1 || oversample < 0 || nE < 1) {
    set_error("cap >= 1, oversample >= 0, nE >= 1");
    return LRFG_EINVAL;
  }
  c[0] = 1;
  c[d] = 1;
  if (d == 3) {
    c[1] = std::min(cap, std::min(N[0], N[1] * N[2]));
    c[2] = std::min(cap, std::min(N[2], N[0] * N[1]));
  } else {
    c[1] = std::min(cap, std::min(N[0], N[1]));
  }
  R.d = d;
  R.nE = nE;
  for (int j = 0; j < 3; ++j) R.N[j] = j < d ? N[j] : 1;
  R.oversample = oversample;
  for (int j = 1; j < d; ++j) {
    if (rin[j] < 1) {
      set_error("ranks must be >= 1");
      return LRFG_EINVAL;
    }
    R.Rmax[j - 1] = rin[j];
    R.Lmax[j - 1] = c[j] + oversample;
    if (std::min(R.Lmax[j - 1], rin[j]) > kMaxEig) {
      set_error("sketch size %d exceeds %d", R.Lmax[j - 1], kMaxEig);
      return LRFG_EUNSUPPORTED;
    }
  }
  return LRFG_OK;
}

}  // namespace

extern "C" {

size_t lrfg_gemm_workspace_bytes(int m, int n, int k, int batch) {
  Gemm g;
  g.m = m;
  g.n = n;
  g.k = k;
  g.batch = batch;
  return sizeof(double) * gemm_scratch_doubles(g) + 256;
}

int lrfg_gemm(int ta, int tb, int m, int n, int k, double alpha, const double* A, long long lda, long long sA,
              const double* B, long long ldb, long long sB, double beta, double* C, long long ldc, long long sC,
              int batch, void* d_ws, size_t ws_bytes, void* stream) {
  clear_error();
  if (m < 0 || n < 0 || k < 0 || batch < 0 || (m * n > 0 && (A == nullptr || B == nullptr || C == nullptr))) {
    set_error("bad arguments");
    return LRFG_EINVAL;
  }
  Gemm g;
  g.m = m;
  g.n = n;
  g.k = k;
  g.A = A;
  g.lda = lda;
  g.sA = sA;
  g.ta = ta != 0;
  g.B = B;
  g.ldb = ldb;
  g.sB = sB;
  g.tb = tb != 0;
  g.C = C;
  g.ldc = ldc;
  g.sC = sC;
  g.alpha = alpha;
  g.beta = beta;
  g.batch = batch;
  return gemm(g, static_cast<double*>(d_ws), ws_bytes / sizeof(double), static_cast<hipStream_t>(stream));
}

int lrfg_gemm_mixed(int precision, int ta, int tb, int m, int n, int k, double alpha, const double* A, long long lda,
                    long long sA, const double* B, long long ldb, long long sB, double beta, double* C,
                    long long ldc, long long sC, int batch, void* d_ws, size_t ws_bytes, void* stream) {
  clear_error();
  if (precision != LRFG_PREC_FP64 && precision != LRFG_PREC_MIXED_FP32 && precision != LRFG_PREC_MIXED_BF16) {
    set_error("unknown precision %d", precision);
    return LRFG_EINVAL;
  }
  if (m < 0 || n < 0 || k < 0 || batch < 0 || (m * n > 0 && (A == nullptr || B == nullptr || C == nullptr))) {
    set_error("bad arguments");
    return LRFG_EINVAL;
  }
  Gemm g;
  g.m = m;
  g.n = n;
  g.k = k;
  g.A = A;
  g.lda = lda;
  g.sA = sA;
  g.ta = ta != 0;
  g.B = B;
  g.ldb = ldb;
  g.sB = sB;
  g.tb = tb != 0;
  g.C = C;
  g.ldc = ldc;
  g.sC = sC;
  g.alpha = alpha;
  g.beta = beta;
  g.batch = batch;
  g.prec = precision;
  return gemm(g, static_cast<double*>(d_ws), ws_bytes / sizeof(double), static_cast<hipStream_t>(stream));
}

int lrfg_syevj(int n, const double* A, int batch, double* W, double* V, void* stream) {
  clear_error();
  if (A == nullptr || W == nullptr || V == nullptr || batch < 0) {
    set_error("bad arguments");
    return LRFG_EINVAL;
  }
  return syevj(n, A, n, (long long)n * n, W, n, V, (long long)n * n, batch, static_cast<hipStream_t>(stream));
}

int lrfg_gram_cut(int n, int c, const double* G, int batch, double tol, double* S, int* kept, int* sweeps,
                  void* stream) {
  clear_error();
  if (G == nullptr || S == nullptr || batch < 0 || !(tol >= 0.0)) {
    set_error("bad arguments");
    return LRFG_EINVAL;
  }
  return cut_psd(n, c, G, (long long)n * n, tol * tol, S, (long long)n * c, kept, batch,
                 static_cast<hipStream_t>(stream), sweeps);
}

size_t lrfg_tt_round_workspace_bytes(int d, const int N[3], const int rin[4], int cap, int oversample, int nE) {
  Rounder R;
  int c[4];
  if (tt_round_sizes(d, N, rin, cap, oversample, c, R, nE) != LRFG_OK) return 0;
  Arena ar;
  R.carve(ar);
  return ar.used + 256;
}

}  // extern "C"

namespace lrfg {
namespace {

// n x n identity (row-major)
__global__ void k_identity(double* __restrict__ p, int n) {
  const long long tot = (long long)n * n;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < tot; i += (long long)gridDim.x * blockDim.x)
    p[i] = (i / n == i % n) ? 1.0 : 0.0;
}

// A full field as an exact train: identity carriage, the field, identity
// carriage (d = 3: ranks 1, N1, N3, 1; d = 2: 1, N1, 1).
void full_as_tt_ranks(int d, const int N[3], int rin[4]) {
  rin[0] = 1;
  rin[1] = N[0];
  rin[2] = d == 3 ? N[2] : 1;
  rin[3] = 1;
  if (d == 2) rin[2] = 1;
}

}  // namespace
}  // namespace lrfg

extern "C" {

}  // extern "C"

namespace {

int tucker_round_sizes(const int N[3], const int rin[3], int cap, int oversample, int nE, int c[3], TkRounder& R) {
  if (N == nullptr || rin == nullptr || cap < 1 || oversample < 0 || nE < 1) {
    set_error("bad arguments");
    return LRFG_EINVAL;
  }
  int cmax = 1;
  for (int j = 0; j < 3; ++j) {
    if (N[j] < 1 || rin[j] < 1) {
      set_error("N and ranks must be positive");
      return LRFG_EINVAL;
    }
    c[j] = std::min(cap, N[j]);
    cmax = std::max(cmax, c[j]);
  }
  if (cmax > kMaxEig) {
    set_error("rank cap %d exceeds %d", cmax, kMaxEig);
    return LRFG_EUNSUPPORTED;
  }
  R.nE = nE;
  for (int j = 0; j < 3; ++j) {
    R.N[j] = N[j];
    R.Rmax[j] = rin[j];
  }
  R.oversample = oversample;
  R.Lmax = std::min(cmax + oversample, kMaxEig);
  return LRFG_OK;
}

}  // namespace

extern "C" {

size_t lrfg_tucker_round_workspace_bytes(const int N[3], const int rin[3], int cap, int oversample, int nE) {
  TkRounder R;
  int c[3];
  if (tucker_round_sizes(N, rin, cap, oversample, nE, c, R) != LRFG_OK) return 0;
  Arena ar;
  R.carve(ar);
  return ar.used + 256;
}

int lrfg_tucker_round(const int N[3], const int rin[3], double* const* in_frames, const double* in_core, int cap,
                      double tol, int oversample, uint64_t seed, double* const* out_frames, double* out_core,
                      int* out_ranks, int* kept, int nE, void* d_ws, size_t ws_bytes, void* stream) {
  clear_error();
  if (in_frames == nullptr || in_core == nullptr || out_frames == nullptr || out_core == nullptr || !(tol >= 0.0)) {
    set_error("bad arguments");
    return LRFG_EINVAL;
  }
  TkRounder R;
  int c[3];
  LRFG_TRY(tucker_round_sizes(N, rin, cap, oversample, nE, c, R));
  R.seed = seed;
  Arena ar;
  ar.base = static_cast<char*>(d_ws);
  ar.cap = ws_bytes;
  R.carve(ar);
  if (ar.overflow || d_ws == nullptr) {
    set_error("workspace too small");
    return LRFG_EWORKSPACE;
  }
  TKB in, out;
  for (int j = 0; j < 3; ++j) {
    in.N[j] = out.N[j] = N[j];
    in.r[j] = rin[j];
    out.r[j] = c[j];
    in.U[j] = in_frames[j];
    in.sU[j] = in.usize(j);
    out.U[j] = out_frames[j];
    out.sU[j] = out.usize(j);
  }
  in.G = const_cast<double*>(in_core);
  in.sG = in.gsize();
  out.G = out_core;
  out.sG = out.gsize();
  hipStream_t s = static_cast<hipStream_t>(stream);
  LRFG_TRY(R.round(in, out, tol, s));
  if (out_ranks)
    for (int j = 0; j < 3; ++j) out_ranks[j] = c[j];
  if (kept) {
    LRFG_HIP(hipMemcpyAsync(kept, R.kept, sizeof(int) * 3 * nE, hipMemcpyDeviceToHost, s));
    LRFG_HIP(hipStreamSynchronize(s));
  }
  return LRFG_OK;
}

size_t lrfg_compress_tucker_workspace_bytes(const int N[3], int cap, int oversample) {
  if (N == nullptr) return 0;
  TkRounder R;
  int c[3];
  if (tucker_round_sizes(N, N, cap, oversample, 1, c, R) != LRFG_OK) return 0;
  Arena ar;
  R.carve(ar);
  for (int j = 0; j < 3; ++j) ar.take<double>((size_t)N[j] * N[j]);
  return ar.used + 256;
}

int lrfg_compress_tucker(const int N[3], const double* a, int cap, double tol, int oversample, uint64_t seed,
                         double* const* out_frames, double* out_core, int* out_ranks, int* kept, void* d_ws,
                         size_t ws_bytes, void* stream) {
  clear_error();
  if (N == nullptr || a == nullptr || out_frames == nullptr || out_core == nullptr || !(tol >= 0.0)) {
    set_error("bad arguments");
    return LRFG_EINVAL;
  }
  TkRounder R;
  int c[3];
  LRFG_TRY(tucker_round_sizes(N, N, cap, oversample, 1, c, R));
  R.seed = seed;
  Arena ar;
  ar.base = static_cast<char*>(d_ws);
  ar.cap = ws_bytes;
  R.carve(ar);
  double* id[3];
  for (int j = 0; j < 3; ++j) id[j] = ar.take<double>((size_t)N[j] * N[j]);
  if (ar.overflow || d_ws == nullptr) {
    set_error("workspace too small");
    return LRFG_EWORKSPACE;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  for (int j = 0; j < 3; ++j)
    hipLaunchKernelGGL(lrfg::k_identity, dim3(std::min(4096, (N[j] * N[j] + 255) / 256)), dim3(256), 0, s, id[j],
                       N[j]);
  LRFG_LAUNCHED();
  // the exact Tucker form of the field: identity frames, the field as core
  TKB in, out;
  for (int j = 0; j < 3; ++j) {
    in.N[j] = out.N[j] = N[j];
    in.r[j] = N[j];
    out.r[j] = c[j];
    in.U[j] = id[j];
    in.sU[j] = in.usize(j);
    out.U[j] = out_frames[j];
    out.sU[j] = out.usize(j);
  }
  in.G = const_cast<double*>(a);
  in.sG = in.gsize();
  out.G = out_core;
  out.sG = out.gsize();
  LRFG_TRY(R.round(in, out, tol, s));
  if (out_ranks)
    for (int j = 0; j < 3; ++j) out_ranks[j] = c[j];
  if (kept) {
    LRFG_HIP(hipMemcpyAsync(kept, R.kept, sizeof(int) * 3, hipMemcpyDeviceToHost, s));
    LRFG_HIP(hipStreamSynchronize(s));
  }
  return LRFG_OK;
}

size_t lrfg_compress_workspace_bytes(int d, const int N[3], int cap, int oversample) {
  using namespace lrfg;
  if (N == nullptr || (d != 2 && d != 3)) return 0;
  int rin[4];
  full_as_tt_ranks(d, N, rin);
  Rounder R;
  int c[4];
  if (tt_round_sizes(d, N, rin, cap, oversample, c, R, 1) != LRFG_OK) return 0;
  Arena ar;
  R.carve(ar);
  ar.take<double>((size_t)N[0] * N[0]);
  if (d == 3) ar.take<double>((size_t)N[2] * N[2]);
  return ar.used + 256;
}

int lrfg_compress_tt(int d, const int N[3], const double* a, int cap, double tol, int oversample, uint64_t seed,
                     double* const* out_cores, int* out_ranks, int* kept, void* d_ws, size_t ws_bytes,
                     void* stream) {
  using namespace lrfg;
  clear_error();
  if (N == nullptr || a == nullptr || out_cores == nullptr || !(tol >= 0.0) || (d != 2 && d != 3)) {
    set_error("bad arguments");
    return LRFG_EINVAL;
  }
  int rin[4];
  full_as_tt_ranks(d, N, rin);
  Rounder R;
  int c[4];
  LRFG_TRY(tt_round_sizes(d, N, rin, cap, oversample, c, R, 1));
  R.seed = seed;
  Arena ar;
  ar.base = static_cast<char*>(d_ws);
  ar.cap = ws_bytes;
  R.carve(ar);
  double* id0 = ar.take<double>((size_t)N[0] * N[0]);
  double* id2 = d == 3 ? ar.take<double>((size_t)N[2] * N[2]) : nullptr;
  if (ar.overflow || d_ws == nullptr) {
    set_error("workspace too small");
    return LRFG_EWORKSPACE;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_identity, dim3(std::min(4096, (N[0] * N[0] + 255) / 256)), dim3(256), 0, s, id0, N[0]);
  if (d == 3)
    hipLaunchKernelGGL(k_identity, dim3(std::min(4096, (N[2] * N[2] + 255) / 256)), dim3(256), 0, s, id2, N[2]);
  LRFG_LAUNCHED();
  TTB in, out;
  in.d = out.d = d;
  for (int j = 0; j < 3; ++j) in.N[j] = out.N[j] = j < d ? N[j] : 1;
  for (int j = 0; j <= d; ++j) {
    in.r[j] = rin[j];
    out.r[j] = c[j];
  }
  in.c[0] = id0;
  in.c[1] = const_cast<double*>(a);
  if (d == 3) in.c[2] = id2;
  for (int j = 0; j < d; ++j) {
    in.s[j] = in.size(j);
    out.c[j] = out_cores[j];
    out.s[j] = out.size(j);
  }
  LRFG_TRY(R.round(in, out, tol, s));
  if (out_ranks)
    for (int j = 0; j <= d; ++j) out_ranks[j] = c[j];
  if (kept) {
    LRFG_HIP(hipMemcpyAsync(kept, R.kept, sizeof(int), hipMemcpyDeviceToHost, s));
    if (d == 3) LRFG_HIP(hipMemcpyAsync(kept + 1, R.kept + R.nE, sizeof(int), hipMemcpyDeviceToHost, s));
    LRFG_HIP(hipStreamSynchronize(s));
  }
  return LRFG_OK;
}

int lrfg_tt_round(int d, const int N[3], const int rin[4], double* const* in_cores, int cap, double tol,
                  int oversample, uint64_t seed, double* const* out_cores, int* out_ranks, int* kept, int nE,
                  void* d_ws, size_t ws_bytes, void* stream) {
  clear_error();
  if (N == nullptr || rin == nullptr || in_cores == nullptr || out_cores == nullptr || !(tol >= 0.0)) {
    set_error("bad arguments");
    return LRFG_EINVAL;
  }
  Rounder R;
  int c[4];
  LRFG_TRY(tt_round_sizes(d, N, rin, cap, oversample, c, R, nE));
  R.seed = seed;
  Arena ar;
  ar.base = static_cast<char*>(d_ws);
  ar.cap = ws_bytes;
  R.carve(ar);
  if (ar.overflow || d_ws == nullptr) {
    set_error("workspace too small");
    return LRFG_EWORKSPACE;
  }
  TTB in, out;
  in.d = out.d = d;
  for (int j = 0; j < 3; ++j) in.N[j] = out.N[j] = j < d ? N[j] : 1;
  for (int j = 0; j <= d; ++j) {
    in.r[j] = rin[j];
    out.r[j] = c[j];
  }
  for (int j = 0; j < d; ++j) {
    in.c[j] = in_cores[j];
    in.s[j] = in.size(j);
    out.c[j] = out_cores[j];
    out.s[j] = out.size(j);
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  LRFG_TRY(R.round(in, out, tol, s));
  if (out_ranks)
    for (int j = 0; j <= d; ++j) out_ranks[j] = c[j];
  if (kept) {
    LRFG_HIP(hipMemcpyAsync(kept, R.kept, sizeof(int) * 2 * nE, hipMemcpyDeviceToHost, s));
    LRFG_HIP(hipStreamSynchronize(s));
  }
  return LRFG_OK;
}

}  // extern "C"
