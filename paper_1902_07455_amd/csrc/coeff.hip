// Coefficient staging: a coefficient given in CP form (sum of separable
// terms, the form of the paper's eq. cano) or TT form (eq. TT) expanded to
// its nodal values on the device.
#include <vector>

#include "common.h"
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

// TT: a[j1][j2][j3] = G1[0][j1][:] G2[:][j2][:] G3[:][j3][0]; d = 2 uses G1, G2.
__global__ void k_tt_expand3(const double* __restrict__ G1, const double* __restrict__ G2,
                             const double* __restrict__ G3, int r1, int r2, int N1, int N2, int N3,
                             double* __restrict__ out) {
  const long long n = (long long)N1 * N2 * N3;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const int j3 = (int)(i % N3);
    const long long r = i / N3;
    const int j2 = (int)(r % N2);
    const int j1 = (int)(r / N2);
    double acc = 0.0;
    for (int a = 0; a < r1; ++a) {
      const double g1 = G1[(long long)j1 * r1 + a];
      double inner = 0.0;
      for (int b = 0; b < r2; ++b)
        inner += G2[((long long)a * N2 + j2) * r2 + b] * G3[(long long)b * N3 + j3];
      acc += g1 * inner;
    }
    out[i] = acc;
  }
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
    hipLaunchKernelGGL(k_tt_expand3, dim3(grid), dim3(256), 0, s, G[0], G[1], G[2], rk[1], rk[2], p.N[0], p.N[1],
                       p.N[2], full);
  } else {
    hipLaunchKernelGGL(k_tt_expand2, dim3(grid), dim3(256), 0, s, G[0], G[1], rk[1], p.N[0], p.N[1], full);
  }
  LRFG_LAUNCHED();
  return LRFG_OK;
}

}  // namespace lrfg
