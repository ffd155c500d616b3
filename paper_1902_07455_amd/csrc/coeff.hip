// Coefficient staging: a coefficient given in CP form (sum of separable
// terms, the form of the paper's eq. cano) or TT form (eq. TT) expanded to
// its nodal values on the device.
#include <cstring>
#include <vector>

#include "common.h"
#include "linalg.h"
#include "lowrank.h"

namespace lrfg {

namespace {

// a[j1][j2][j3] = sum_t w[t] f1[t][j1] f2[t][j2] f3[t][j3]; d = 2 uses
// (j2, j3) with f1 = 1.
__global__ void k_cp_expand(const double* __restrict__ w, const double* __restrict__ f1,
                            const double* __restrict__ f2, const double* __restrict__ f3, int R, int N1,
                            int N2, int N3, double* __restrict__ out) {
  const long long n = (long long)N1 * N2 * N3;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const int j3 = (int)(i % N3);
    const long long r = i / N3;
    const int j2 = (int)(r % N2);
    const int j1 = (int)(r / N2);
    double acc = 0.0;
    for (int t = 0; t < R; ++t) {
      double v = w[t] * f2[(long long)t * N2 + j2] * f3[(long long)t * N3 + j3];
      if (f1 != nullptr) v *= f1[(long long)t * N1 + j1];
      acc += v;
    }
    out[i] = acc;
  }
}

// TT, d = 2: a[j1][j2] = G1[0][j1][:] G2[:][j2][0].
// Order-preserving 64-bit key of a double (the unsigned order of the keys
// is the order of the values), for an atomic minimum.
__device__ inline unsigned long long order_key(double v) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

// Rows of a d = 3 low-rank expansion, one block per row (j1, j2) =
// (blockIdx.y, blockIdx.x): P[c] = sum_{b < K} x[b] M[b][c] (c < Rn; with
// x = NULL, P[c] = M[0][c]) in LDS, then a[j1][j2][j3] = sum_c P[c]
// Y[c ysc + j3 ysj], j3 < Nrow.  x and M are offset per row by
// j1 sx1 + j2 sx2 and j1 sM1 + j2 sM2; M's rows are ldM apart.  A TT gives
// x = G1[j1][:], M = G2[:][j2][:], Y = G3; a Tucker tensor x = U2[j2][:],
// M = (U1 x_1 core)[j1], Y = U3.  out (if not NULL) receives the values;
// minkey and nonfin (if not NULL) the smallest value's key and the number
// of non-finite values (atomics).
__global__ __launch_bounds__(256) void k_lr_rows(const double* __restrict__ x, long long sx1, long long sx2,
                                                 const double* __restrict__ M, long long sM1, long long sM2,
                                                 long long ldM, int K, int Rn, const double* __restrict__ Y,
                                                 long long ysc, long long ysj, int N2, int Nrow,
                                                 double* __restrict__ out, unsigned long long* minkey,
                                                 int* nonfin) {
  __shared__ double P[kMaxCoeffRank];
  __shared__ double redm[4];
  __shared__ int redn[4];
  const int j2 = blockIdx.x, j1 = blockIdx.y, tid = threadIdx.x;
  const double* xr = x != nullptr ? x + j1 * sx1 + j2 * sx2 : nullptr;
  const double* Mr = M + j1 * sM1 + j2 * sM2;
  for (int c = tid; c < Rn; c += blockDim.x) {
    double v;
    if (xr == nullptr) {
      v = Mr[c];
    } else {
      v = 0.0;
      for (int b = 0; b < K; ++b) v = fma(xr[b], Mr[b * ldM + c], v);
    }
    P[c] = v;
  }
  __syncthreads();
  double mn = INFINITY;
  int bad = 0;
  double* orow = out != nullptr ? out + ((long long)j1 * N2 + j2) * Nrow : nullptr;
  for (int j3 = tid; j3 < Nrow; j3 += blockDim.x) {
    double v = 0.0;
    for (int c = 0; c < Rn; ++c) v = fma(P[c], Y[c * ysc + j3 * ysj], v);
    if (orow != nullptr) orow[j3] = v;
    if (isfinite(v)) mn = fmin(mn, v); else ++bad;
  }
  if (minkey == nullptr) return;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    mn = fmin(mn, __shfl_xor(mn, o, 64));
    bad += __shfl_xor(bad, o, 64);
  }
  if ((tid & 63) == 0) {
    redm[tid >> 6] = mn;
    redn[tid >> 6] = bad;
  }
  __syncthreads();
  if (tid == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int w = 1; w < nw; ++w) {
      mn = fmin(mn, redm[w]);
      bad += redn[w];
    }
    atomicMin(minkey, order_key(mn));
    if (bad) atomicAdd(nonfin, bad);
  }
}

__global__ void k_minkey_init(unsigned long long* minkey, int* nonfin) {
  *minkey = ~0ull;
  *nonfin = 0;
}

__global__ void k_tt_expand2(const double* __restrict__ G1, const double* __restrict__ G2, int r1, int N1,
                             int N2, double* __restrict__ out) {
  const long long n = (long long)N1 * N2;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const int j2 = (int)(i % N2);
    const int j1 = (int)(i / N2);
    double acc = 0.0;
    for (int a = 0; a < r1; ++a) acc += G1[(long long)j1 * r1 + a] * G2[(long long)a * N2 + j2];
    out[i] = acc;
  }
}

}  // namespace

size_t coeff_staging_bytes(const lrfg_problem& p) {
  long long R = 1;
  long long sumN = 0;
  for (int i = 0; i < p.d; ++i) {
    R *= p.N[i];
    sumN += p.N[i];
  }
  const long long K = kMaxCoeffRank;
  // full field + the larger of the CP and TT staging
  long long cp = K + K * sumN;
  long long tt = 0;
  for (int i = 0; i < p.d; ++i) tt += K * K * p.N[i];
  return sizeof(double) * (size_t)(R + (cp > tt ? cp : tt)) + 4 * 256;
}

int expand_coeff(const lrfg_problem& p, const lrfg_coeff& a, double* dst, size_t bytes, hipStream_t s) {
  long long R = 1;
  for (int i = 0; i < p.d; ++i) R *= p.N[i];
  Arena ar;
  ar.base = reinterpret_cast<char*>(dst);
  ar.cap = bytes;
  double* full = ar.take<double>(R);
  const int grid = (int)std::min<long long>(4096, (R + 255) / 256);
  if (a.weights != nullptr) {
    const int Rk = a.rank;
    if (Rk < 1 || Rk > kMaxCoeffRank) {
      set_error("CP coefficient rank %d outside [1, %d]", Rk, kMaxCoeffRank);
      return LRFG_EINVAL;
    }
    for (int i = 0; i < p.d; ++i) {
      if (a.factors[i] == nullptr) {
        set_error("CP coefficient: factor %d is NULL", i);
        return LRFG_EINVAL;
      }
    }
    const double* w = a.weights;
    const double* f[3] = {a.factors[0], a.factors[1], p.d == 3 ? a.factors[2] : nullptr};
    if (!a.on_device) {
      double* dw = ar.take<double>(Rk);
      double* df[3] = {nullptr, nullptr, nullptr};
      for (int i = 0; i < p.d; ++i) df[i] = ar.take<double>((size_t)Rk * p.N[i]);
      if (ar.overflow) {
        set_error("coefficient staging overflow");
        return LRFG_EWORKSPACE;
      }
      LRFG_HIP(hipMemcpyAsync(dw, w, sizeof(double) * Rk, hipMemcpyHostToDevice, s));
      for (int i = 0; i < p.d; ++i)
        LRFG_HIP(hipMemcpyAsync(df[i], f[i], sizeof(double) * Rk * p.N[i], hipMemcpyHostToDevice, s));
      w = dw;
      for (int i = 0; i < p.d; ++i) f[i] = df[i];
    }
    if (p.d == 3) {
      hipLaunchKernelGGL(k_cp_expand, dim3(grid), dim3(256), 0, s, w, f[0], f[1], f[2], Rk, p.N[0], p.N[1],
                         p.N[2], full);
    } else {
      hipLaunchKernelGGL(k_cp_expand, dim3(grid), dim3(256), 0, s, w, (const double*)nullptr, f[0], f[1], Rk, 1,
                         p.N[0], p.N[1], full);
    }
    LRFG_LAUNCHED();
    return LRFG_OK;
  }
  // TT form
  const int* rk = a.tt_ranks;
  if (rk[0] != 1 || rk[p.d] != 1) {
    set_error("TT coefficient: r_0 = r_d = 1 required");
    return LRFG_EINVAL;
  }
  for (int i = 1; i < p.d; ++i) {
    if (rk[i] < 1 || rk[i] > kMaxCoeffRank) {
      set_error("TT coefficient rank %d outside [1, %d]", rk[i], kMaxCoeffRank);
      return LRFG_EINVAL;
    }
  }
  const double* G[3] = {a.tt_cores[0], a.tt_cores[1], p.d == 3 ? a.tt_cores[2] : nullptr};
  for (int i = 0; i < p.d; ++i) {
    if (G[i] == nullptr) {
      set_error("TT coefficient: core %d is NULL", i);
      return LRFG_EINVAL;
    }
  }
  if (!a.on_device) {
    for (int i = 0; i < p.d; ++i) {
      const size_t n = (size_t)rk[i] * p.N[i] * rk[i + 1];
      double* dg = ar.take<double>(n);
      if (ar.overflow) {
        set_error("coefficient staging overflow");
        return LRFG_EWORKSPACE;
      }
      LRFG_HIP(hipMemcpyAsync(dg, G[i], sizeof(double) * n, hipMemcpyHostToDevice, s));
      G[i] = dg;
    }
  }
  if (p.d == 3) {
    hipLaunchKernelGGL(k_lr_rows, dim3(p.N[1], p.N[0]), dim3(256), 0, s, G[0], (long long)rk[1], 0LL, G[1], 0LL,
                       (long long)rk[2], (long long)p.N[1] * rk[2], rk[1], rk[2], G[2], (long long)p.N[2], 1LL,
                       p.N[1], p.N[2], full, (unsigned long long*)nullptr, (int*)nullptr);
  } else {
    hipLaunchKernelGGL(k_tt_expand2, dim3(grid), dim3(256), 0, s, G[0], G[1], rk[1], p.N[0], p.N[1], full);
  }
  LRFG_LAUNCHED();
  return LRFG_OK;
}

namespace {
int finish_check(unsigned long long* keys, hipStream_t s, double* min_out, long long* nonfinite_out) {
  unsigned long long h[2] = {0, 0};
  LRFG_HIP(hipMemcpyAsync(h, keys, sizeof(unsigned long long) + sizeof(int), hipMemcpyDeviceToHost, s));
  LRFG_HIP(hipStreamSynchronize(s));
  const unsigned long long k = h[0];
  const unsigned long long u = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
  double v;
  memcpy(&v, &u, sizeof(v));
  *min_out = v;
  *nonfinite_out = (long long)(int)(h[1] & 0xffffffffull);
  return LRFG_OK;
}
}  // namespace

int tt_coeff_check(int d, const int N[3], const int rk[4], const double* const* cores, void* scratch,
                   hipStream_t s, double* min_out, long long* nonfinite_out) {
  for (int j = 1; j < d; ++j)
    if (rk[j] < 1 || rk[j] > kMaxCoeffRank) {
      set_error("coefficient rank %d outside [1, %d]", rk[j], kMaxCoeffRank);
      return LRFG_EINVAL;
    }
  auto* keys = static_cast<unsigned long long*>(scratch);
  int* bad = reinterpret_cast<int*>(keys + 1);
  hipLaunchKernelGGL(k_minkey_init, dim3(1), dim3(1), 0, s, keys, bad);
  if (d == 3)
    hipLaunchKernelGGL(k_lr_rows, dim3(N[1], N[0]), dim3(256), 0, s, cores[0], (long long)rk[1], 0LL, cores[1], 0LL,
                       (long long)rk[2], (long long)N[1] * rk[2], rk[1], rk[2], cores[2], (long long)N[2], 1LL, N[1],
                       N[2], (double*)nullptr, keys, bad);
  else
    hipLaunchKernelGGL(k_lr_rows, dim3(1, N[0]), dim3(256), 0, s, (const double*)nullptr, 0LL, 0LL, cores[0],
                       (long long)rk[1], 0LL, 0LL, 1, rk[1], cores[1], (long long)N[1], 1LL, 1, N[1], (double*)nullptr,
                       keys, bad);
  LRFG_LAUNCHED();
  return finish_check(keys, s, min_out, nonfinite_out);
}

int tucker_coeff_check(const int N[3], const int r[3], const double* core, const double* const* U, double* W,
                       void* scratch, hipStream_t s, double* min_out, long long* nonfinite_out) {
  for (int j = 0; j < 3; ++j)
    if (r[j] < 1 || r[j] > kMaxCoeffRank) {
      set_error("coefficient rank %d outside [1, %d]", r[j], kMaxCoeffRank);
      return LRFG_EINVAL;
    }
  auto* keys = static_cast<unsigned long long*>(scratch);
  int* bad = reinterpret_cast<int*>(keys + 1);
  hipLaunchKernelGGL(k_minkey_init, dim3(1), dim3(1), 0, s, keys, bad);
  // W[j1][b][c] = sum_a U1[j1][a] core[a][b][c]: rows j1 of (U1 x_1 core)
  {
    Gemm g;
    g.m = N[0];
    g.n = r[1] * r[2];
    g.k = r[0];
    g.A = U[0];
    g.lda = r[0];
    g.B = core;
    g.ldb = (long long)r[1] * r[2];
    g.C = W;
    g.ldc = (long long)r[1] * r[2];
    LRFG_TRY(gemm(g, nullptr, 0, s));
  }
  hipLaunchKernelGGL(k_lr_rows, dim3(N[1], N[0]), dim3(256), 0, s, U[1], 0LL, (long long)r[1], (const double*)W,
                     (long long)r[1] * r[2], 0LL, (long long)r[2], r[1], r[2], U[2], 1LL, (long long)r[2], N[1], N[2],
                     (double*)nullptr, keys, bad);
  LRFG_LAUNCHED();
  return finish_check(keys, s, min_out, nonfinite_out);
}

}  // namespace lrfg
