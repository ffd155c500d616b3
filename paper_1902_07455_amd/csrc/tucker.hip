// Tucker-format operations on the device (paper Sec. 3.1.2 and Appendix
// A.2), d = 3: per-mode DFT operators on the frames, the element-wise
// product (Khatri-Rao frames and Kronecker core), sums (frames side by side,
// block-diagonal core), inner products, and truncation.
//
// Truncation reaches the paper's HOSVD cut through a randomised range
// finder (Halko, Martinsson and Tropp) with Khatri-Rao structured sketches,
// so that no frame QR or core unfolding larger than the sketch is ever
// factorised:
//   1. Z_j = U_j^T Om_j for Gaussian Om_j (N_j x l), and the sketch of the
//      mode-j unfolding Y_j = X_(j) (Om_k (.) Om_m) = U_j G_(j) (Z_k (.) Z_m),
//      formed from the core without expanding anything (the structured
//      sketch of Sun, Guo, Luo, Tropp and Udell, SIMAX 2020);
//   2. Q_j = orth(Y_j) (Gram matrix and pivoted Cholesky, twice);
//   3. the core of the projected tensor C = G x_j (Q_j^T U_j) (l x l x l);
//   4. the paper's cut: the HOSVD of C from its three l x l mode Gram
//      matrices, at most c_j per mode and the fewest whose dropped
//      eigenvalues stay within tol^2 ||X||^2 / 3 per mode, so the total
//      error is within tol ||X|| (Appendix A.2 bound).
// Output ranks are fixed (c_1, c_2, c_3); directions beyond the kept rank
// are zero columns.
#include <algorithm>
#include <cmath>

#include "prof.h"
#include "tucker.h"

namespace lrfg {

int launch_mode_op_oop(const double* xin, double* x, long long outer, int N, long long inner, int op, double t,
                       double mult, const FftDev& f, hipStream_t s, long long fib_per_group);
int launch_randn(double* out, long long n, uint64_t key, hipStream_t s);

namespace {

constexpr int kB = 256;

inline int grid_for(long long n) {
  long long g = (n + kB - 1) / kB;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  return (int)g;
}

#define GRID_STRIDE(i, n) \
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (long long)gridDim.x * blockDim.x)

// out[e][n][i s + k] = a[e][n][i] x[e][n][k]   (frames [N][r])
__global__ void k_frame_kr(const double* __restrict__ a, long long sa, int ra, const double* __restrict__ x,
                           long long sx, int rx, int N, double* __restrict__ out, long long so, int nE) {
  const long long R = (long long)ra * rx, per = N * R;
  GRID_STRIDE(idx, per * nE) {
    const long long e = idx / per;
    const long long rem = idx - e * per;
    const long long n = rem / R, c = rem - n * R;
    const long long i = c / rx, k = c - i * rx;
    out[e * so + rem] = a[e * sa + n * ra + i] * x[e * sx + n * rx + k];
  }
}

// out[e][I1][I2][I3] = a[e][p1][p2][p3] x[e][q1][q2][q3], I_j = p_j rx_j + q_j
__global__ void k_core_kron(const double* __restrict__ a, long long sa, int a1, int a2, int a3,
                            const double* __restrict__ x, long long sx, int x1, int x2, int x3,
                            double* __restrict__ out, long long so, int nE) {
  const long long R2 = (long long)a2 * x2, R3 = (long long)a3 * x3;
  const long long per = (long long)a1 * x1 * R2 * R3;
  GRID_STRIDE(idx, per * nE) {
    const long long e = idx / per;
    long long rem = idx - e * per;
    const long long I3 = rem % R3;
    rem /= R3;
    const long long I2 = rem % R2, I1 = rem / R2;
    const long long p1 = I1 / x1, q1 = I1 - p1 * x1;
    const long long p2 = I2 / x2, q2 = I2 - p2 * x2;
    const long long p3 = I3 / x3, q3 = I3 - p3 * x3;
    out[e * so + (idx - e * per)] =
        a[e * sa + (p1 * a2 + p2) * a3 + p3] * x[e * sx + (q1 * x2 + q2) * x3 + q3];
  }
}

// Block sum of up to kTkSumTerms Tucker tensors in two launches: the frames
// of mode blockIdx.z side by side (term t's columns at offset o[t][j]), and
// the block-diagonal core (term t's block at (o[t][0], o[t][1], o[t][2]),
// times mult_t coef_t[e], zeros elsewhere).  Per-system indices in 32 bits.
constexpr int kTkSumTerms = 4;
struct TkSumArgs {
  const double* U[kTkSumTerms][3];
  long long sU[kTkSumTerms][3];
  const double* G[kTkSumTerms];
  long long sG[kTkSumTerms];
  int r[kTkSumTerms][3], o[kTkSumTerms][3];
  const double* coef[kTkSumTerms];
  double mult[kTkSumTerms];
  int nt;
};
__global__ __launch_bounds__(256) void k_tk_sum_frames(TkSumArgs T, int N0, int N1, int N2, double* __restrict__ u0,
                                                       double* __restrict__ u1, double* __restrict__ u2,
                                                       long long so0, long long so1, long long so2, int R0, int R1,
                                                       int R2) {
  const int j = blockIdx.z, e = blockIdx.y;
  const int N = j == 0 ? N0 : (j == 1 ? N1 : N2);
  const int R = j == 0 ? R0 : (j == 1 ? R1 : R2);
  double* out = (j == 0 ? u0 : (j == 1 ? u1 : u2)) + e * (j == 0 ? so0 : (j == 1 ? so1 : so2));
  const int per = N * R;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < per; idx += gridDim.x * blockDim.x) {
    const int n = idx / R, K = idx - (idx / R) * R;
    double v = 0.0;
    for (int t = 0; t < T.nt; ++t) {
      const int k = K - T.o[t][j];
      if (k >= 0 && k < T.r[t][j]) v = T.U[t][j][e * T.sU[t][j] + (long long)n * T.r[t][j] + k];
    }
    out[idx] = v;
  }
}
__global__ __launch_bounds__(256) void k_tk_sum_core(TkSumArgs T, int R0, int R1, int R2, double* __restrict__ out,
                                                     long long so) {
  const int e = blockIdx.y;
  const int per = R0 * R1 * R2;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < per; idx += gridDim.x * blockDim.x) {
    const int K = idx % R2, r = idx / R2;
    const int J = r % R1, I = r / R1;
    double v = 0.0;
    for (int t = 0; t < T.nt; ++t) {
      const int i = I - T.o[t][0], jj = J - T.o[t][1], k = K - T.o[t][2];
      if (i >= 0 && i < T.r[t][0] && jj >= 0 && jj < T.r[t][1] && k >= 0 && k < T.r[t][2]) {
        const double c = T.mult[t] * (T.coef[t] != nullptr ? T.coef[t][e] : 1.0);
        v = c * T.G[t][e * T.sG[t] + ((long long)i * T.r[t][1] + jj) * T.r[t][2] + k];
      }
    }
    out[e * so + idx] = v;
  }
}

// out[e][o1 + i][o2 + j][o3 + k] = c_e x[e][i][j][k]
__global__ void k_core_place(const double* __restrict__ x, long long sx, int r1, int r2, int r3,
                             const double* __restrict__ coef, double mult, double* __restrict__ out, long long so,
                             int R2, int R3, int o1, int o2, int o3, int nE) {
  const long long per = (long long)r1 * r2 * r3;
  GRID_STRIDE(idx, per * nE) {
    const long long e = idx / per;
    long long rem = idx - e * per;
    const long long k = rem % r3;
    rem /= r3;
    const long long j = rem % r2, i = rem / r2;
    const double c = mult * (coef != nullptr ? coef[e] : 1.0);
    out[e * so + ((o1 + i) * R2 + o2 + j) * R3 + o3 + k] = c * x[e * sx + (idx - e * per)];
  }
}

// Mode-2 product: out[e][a][b][c] = sum_q W'[b][q] in[e][a][q][c] with
// W' = W[e] (Bo x Bi) or, transposed, W[e]^T (W[e] is Bi x Bo).
__global__ void k_mode2(const double* __restrict__ in, long long sin, int A, int Bi, int Cd,
                        const double* __restrict__ W, long long sW, int Bo, int wt, double* __restrict__ out,
                        long long sout, int nE) {
  const long long per = (long long)A * Bo * Cd;
  GRID_STRIDE(idx, per * nE) {
    const long long e = idx / per;
    long long rem = idx - e * per;
    const long long c = rem % Cd;
    rem /= Cd;
    const long long b = rem % Bo, a = rem / Bo;
    const double* w = W + e * sW;
    const double* x = in + e * sin + a * Bi * Cd + c;
    double acc = 0.0;
    if (wt) {
      for (int q = 0; q < Bi; ++q) acc += w[(long long)q * Bo + b] * x[(long long)q * Cd];
    } else {
      for (int q = 0; q < Bi; ++q) acc += w[b * Bi + q] * x[(long long)q * Cd];
    }
    out[e * sout + (idx - e * per)] = acc;
  }
}

// Y cores of modes 1 and 2 from H = G x_3 Z_3^T (R1 x R2 x l):
// y1[i1][t] = sum_i2 H[i1][i2][t] Z2[i2][t], y2[i2][t] = sum_i1 H[i1][i2][t] Z1[i1][t].
// One block per (output row, system): thread (p, t) of the 256 sums the
// terms p, p + P, ... of column t (P = 256 / l partitions, each stream of
// loads coalesced along t), then the P partial sums of each column are
// added in partition order.
__global__ __launch_bounds__(256) void k_tcontract(const double* __restrict__ H, long long sH,
                                                   const double* __restrict__ Z1, long long sZ1,
                                                   const double* __restrict__ Z2, long long sZ2, int R1, int R2,
                                                   int l, double* __restrict__ y1, long long sy1,
                                                   double* __restrict__ y2, long long sy2) {
  __shared__ double part[256];
  const int e = blockIdx.y, row = blockIdx.x;
  const int P = 256 / l;
  const int p = threadIdx.x / l, t = threadIdx.x - (threadIdx.x / l) * l;
  double a = 0.0;
  if (p < P) {
    if (row < R1) {
      const double* hr = H + e * sH + (long long)row * R2 * l + t;
      const double* z = Z2 + e * sZ2 + t;
#pragma unroll 4
      for (int i2 = p; i2 < R2; i2 += P) a = fma(hr[(long long)i2 * l], z[(long long)i2 * l], a);
    } else {
      const double* hc = H + e * sH + (long long)(row - R1) * l + t;
      const double* z = Z1 + e * sZ1 + t;
      const long long st = (long long)R2 * l;
#pragma unroll 4
      for (int i1 = p; i1 < R1; i1 += P) a = fma(hc[i1 * st], z[(long long)i1 * l], a);
    }
  }
  part[threadIdx.x] = a;
  __syncthreads();
  if (threadIdx.x < l) {
    double v = 0.0;
    for (int q = 0; q < P; ++q) v += part[q * l + threadIdx.x];
    if (row < R1)
      y1[e * sy1 + (long long)row * l + threadIdx.x] = v;
    else
      y2[e * sy2 + (long long)(row - R1) * l + threadIdx.x] = v;
  }
}

// KR[e][i1 R2 + i2][t] = Z1[e][i1][t] Z2[e][i2][t]
__global__ void k_kr_rows(const double* __restrict__ Z1, long long s1, int R1, const double* __restrict__ Z2,
                          long long s2, int R2, int l, double* __restrict__ KR, long long sk, int nE) {
  const long long per = (long long)R1 * R2 * l;
  GRID_STRIDE(idx, per * nE) {
    const long long e = idx / per;
    const long long rem = idx - e * per;
    const long long t = rem % l, row = rem / l;
    const long long i1 = row / R2, i2 = row - i1 * R2;
    KR[e * sk + rem] = Z1[e * s1 + i1 * l + t] * Z2[e * s2 + i2 * l + t];
  }
}

// out[o][b][a][q] = in[o][a][b][q] (o < outer, a < A, b < B, q < inner)
__global__ void k_swap_mid(const double* __restrict__ in, double* __restrict__ out, long long outer, int A, int B,
                           long long inner) {
  const long long per = (long long)A * B * inner;
  GRID_STRIDE(idx, per * outer) {
    const long long o = idx / per;
    long long rem = idx - o * per;
    const long long q = rem % inner;
    rem /= inner;
    const long long b = rem % B, a = rem / B;
    out[o * per + (b * A + a) * inner + q] = in[idx];
  }
}

// Kronecker-core unfolding: in[(i1, i2)][t][k1][q] (q < inner = rx2 l) ->
// out[t][i1][k1][i2][q], the core-sketch layout [(i1, k1)][(i2, k2)][c].
__global__ void k_kron_unfold(const double* __restrict__ in, double* __restrict__ out, int ra1, int ra2, int nb,
                              int rx1, long long inner) {
  const long long tot = (long long)ra1 * ra2 * nb * rx1 * inner;
  GRID_STRIDE(idx, tot) {
    long long rem = idx;
    const long long q = rem % inner;
    rem /= inner;
    const long long k1 = rem % rx1;
    rem /= rx1;
    const long long t = rem % nb;
    rem /= nb;
    const long long i2 = rem % ra2, i1 = rem / ra2;
    out[(((t * ra1 + i1) * rx1 + k1) * ra2 + i2) * inner + q] = in[idx];
  }
}

// Khatri-Rao rows in Kronecker order: W[t][k1][k2][i1][i2][c] =
// Z1[t][i1 rx1 + k1][c] Z2[t][i2 rx2 + k2][c]
__global__ void k_kr_kron(const double* __restrict__ Z1, long long s1, const double* __restrict__ Z2, long long s2,
                          int ra1, int rx1, int ra2, int rx2, int l, double* __restrict__ W, int nb) {
  const long long per = (long long)rx1 * rx2 * ra1 * ra2 * l;
  GRID_STRIDE(idx, per * nb) {
    const long long t = idx / per;
    long long rem = idx - t * per;
    const long long c = rem % l;
    rem /= l;
    const long long i2 = rem % ra2;
    rem /= ra2;
    const long long i1 = rem % ra1;
    rem /= ra1;
    const long long k2 = rem % rx2, k1 = rem / rx2;
    W[idx] = Z1[t * s1 + (i1 * rx1 + k1) * l + c] * Z2[t * s2 + (i2 * rx2 + k2) * l + c];
  }
}

// P[e][b][a][c] = C[e][a][b][c] (l x l x l), so that the mode-2 Gram matrix
// is the GEMM P P^T over (a, c)
__global__ void k_swap01(const double* __restrict__ Cc, long long sc, int l, double* __restrict__ P, int nE) {
  const long long per = (long long)l * l * l;
  GRID_STRIDE(idx, per * nE) {
    const long long e = idx / per;
    const long long rem = idx - e * per;
    const long long c = rem % l, ab = rem / l;
    const long long b = ab % l, a = ab / l;
    P[e * per + (b * l + a) * l + c] = Cc[e * sc + rem];
  }
}

struct GB {
  Gemm g;
  GB(int m, int n, int k, int batch) {
    g.m = m;
    g.n = n;
    g.k = k;
    g.batch = batch;
  }
  GB& a(const double* p, long long ld, long long st, bool t = false) {
    g.A = p;
    g.lda = ld;
    g.sA = st;
    g.ta = t;
    return *this;
  }
  GB& b(const double* p, long long ld, long long st, bool t = false) {
    g.B = p;
    g.ldb = ld;
    g.sB = st;
    g.tb = t;
    return *this;
  }
  GB& c(double* p, long long ld, long long st) {
    g.C = p;
    g.ldc = ld;
    g.sC = st;
    return *this;
  }
};

// The truncation's contractions in a given precision (FP64, or FP32 / BF16
// inputs with FP32 accumulation).
inline Gemm& with_prec(Gemm& g, int prec) {
  g.prec = prec;
  return g;
}

// Mode-2 product out[e][a][b][c] = sum_q W'[e][b][q] in[e][a][q][c] (W' = W[e]
// or, with wt, W[e]^T) as one batched GEMM over (e, a) when in and out are
// compact per system, else by k_mode2.
int mode2(const double* in, long long sin, int A, int Bi, int Cd, const double* W, long long sW, int Bo, int wt,
          double* out, long long sout, int nE, double* gscr, size_t gscr_n, hipStream_t s, int prec = 0) {
  if (sin == (long long)A * Bi * Cd && sout == (long long)A * Bo * Cd) {
    GB g(Bo, Cd, Bi, A * nE);
    g.a(W, wt ? Bo : Bi, sW, wt != 0);
    g.g.adiv = A;
    g.b(in, Cd, (long long)Bi * Cd).c(out, Cd, (long long)Bo * Cd);
    g.g.prec = prec;
    return gemm(g.g, gscr, gscr_n, s);
  }
  hipLaunchKernelGGL(k_mode2, dim3(grid_for((long long)A * Bo * Cd * nE)), dim3(kB), 0, s, in, sin, A, Bi, Cd, W, sW,
                     Bo, wt, out, sout, nE);
  LRFG_LAUNCHED();
  return LRFG_OK;
}


constexpr size_t kTkDotSplitK = (size_t)2 * 1024 * 1024;

}  // namespace

// ====================================================================== basics
TKB tk_alloc(Arena& ar, const int N[3], const int r[3], int nE) {
  TKB t;
  for (int j = 0; j < 3; ++j) {
    t.N[j] = N[j];
    t.r[j] = r[j];
    t.sU[j] = t.usize(j);
    t.U[j] = ar.take<double>((size_t)t.sU[j] * nE);
  }
  t.sG = t.gsize();
  t.G = ar.take<double>((size_t)t.sG * nE);
  return t;
}

int tk_zero(TKB& x, int nE, hipStream_t s) {
  for (int j = 0; j < 3; ++j)
    if (x.U[j]) LRFG_HIP(hipMemsetAsync(x.U[j], 0, sizeof(double) * x.usize(j) * (x.sU[j] ? nE : 1), s));
  LRFG_HIP(hipMemsetAsync(x.G, 0, sizeof(double) * x.gsize() * (x.sG ? nE : 1), s));
  return LRFG_OK;
}

static int copy_block(double* dst, long long sd, const double* src, long long ss, long long n, int nE,
                      hipStream_t s) {
  if (sd == n && ss == n) {
    LRFG_HIP(hipMemcpyAsync(dst, src, sizeof(double) * n * nE, hipMemcpyDeviceToDevice, s));
    return LRFG_OK;
  }
  for (int e = 0; e < nE; ++e)
    LRFG_HIP(hipMemcpyAsync(dst + e * sd, src + e * ss, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  return LRFG_OK;
}

int tk_copy(const TKB& x, TKB& y, int nE, hipStream_t s) {
  for (int j = 0; j < 3; ++j) {
    if (x.r[j] != y.r[j]) {
      set_error("tk_copy: rank mismatch");
      return LRFG_EINVAL;
    }
    LRFG_TRY(copy_block(y.U[j], y.sU[j], x.U[j], x.sU[j], x.usize(j), nE, s));
  }
  return copy_block(y.G, y.sG, x.G, x.sG, x.gsize(), nE, s);
}

int tk_copy_system(const TKB& x, TKB& y, int e, hipStream_t s) {
  for (int j = 0; j < 3; ++j)
    LRFG_HIP(hipMemcpyAsync(y.U[j] + e * y.sU[j], x.U[j] + e * x.sU[j], sizeof(double) * x.usize(j),
                            hipMemcpyDeviceToDevice, s));
  LRFG_HIP(hipMemcpyAsync(y.G + e * y.sG, x.G + e * x.sG, sizeof(double) * x.gsize(), hipMemcpyDeviceToDevice, s));
  return LRFG_OK;
}

int tk_mode_apply(const TKB& x, TKB& y, int j, int op, double t, double mult, const FftDev& f, int nE,
                  hipStream_t s) {
  double* uj = y.U[j];
  y = x;
  y.U[j] = uj;
  y.sU[j] = x.sU[j] == 0 ? 0 : x.usize(j);
  const int reps = x.sU[j] == 0 ? 1 : nE;
  return launch_mode_op_oop(x.U[j], uj, reps, x.N[j], x.r[j], op, t, mult, f, s, x.r[j]);
}

int tk_hadamard(const TKB& a, const TKB& x, TKB& out, int nE, hipStream_t s) {
  ProfScope ps_("tk_hadamard", s);
  for (int j = 0; j < 3; ++j) {
    out.r[j] = a.r[j] * x.r[j];
    out.sU[j] = out.usize(j);
  }
  out.sG = out.gsize();
  for (int j = 0; j < 3; ++j) {
    const long long tot = out.usize(j) * nE;
    hipLaunchKernelGGL(k_frame_kr, dim3(grid_for(tot)), dim3(kB), 0, s, (const double*)a.U[j], a.sU[j], a.r[j],
                       (const double*)x.U[j], x.sU[j], x.r[j], x.N[j], out.U[j], out.sU[j], nE);
  }
  hipLaunchKernelGGL(k_core_kron, dim3(grid_for(out.gsize() * nE)), dim3(kB), 0, s, (const double*)a.G, a.sG, a.r[0],
                     a.r[1], a.r[2], (const double*)x.G, x.sG, x.r[0], x.r[1], x.r[2], out.G, out.sG, nE);
  LRFG_LAUNCHED();
  return LRFG_OK;
}

int tk_hadamard_frames(const TKB& a, const TKB& x, TKB& out, int nE, hipStream_t s) {
  for (int j = 0; j < 3; ++j) {
    out.r[j] = a.r[j] * x.r[j];
    out.sU[j] = out.usize(j);
    const long long tot = out.usize(j) * nE;
    hipLaunchKernelGGL(k_frame_kr, dim3(grid_for(tot)), dim3(kB), 0, s, (const double*)a.U[j], a.sU[j], a.r[j],
                       (const double*)x.U[j], x.sU[j], x.r[j], x.N[j], out.U[j], out.sU[j], nE);
  }
  LRFG_LAUNCHED();
  return LRFG_OK;
}

int tk_place_core(const TKB& x, const double* coef, double mult, TKB& out, const int o[3], int nE, hipStream_t s) {
  hipLaunchKernelGGL(k_core_place, dim3(grid_for(x.gsize() * nE)), dim3(kB), 0, s, (const double*)x.G, x.sG, x.r[0],
                     x.r[1], x.r[2], coef, mult, out.G, out.sG, out.r[1], out.r[2], o[0], o[1], o[2], nE);
  LRFG_LAUNCHED();
  return LRFG_OK;
}

int tk_sum(const TKTerm* terms, int nt, TKB& out, int nE, hipStream_t s) {
  int R[3] = {0, 0, 0};
  for (int t = 0; t < nt; ++t)
    for (int j = 0; j < 3; ++j) R[j] += terms[t].x->r[j];
  for (int j = 0; j < 3; ++j) {
    if (R[j] != out.r[j]) {
      set_error("tk_sum: output ranks do not match the terms");
      return LRFG_EINVAL;
    }
  }
  long long biggest = out.gsize();
  for (int j = 0; j < 3; ++j) biggest = std::max(biggest, out.usize(j));
  if (nt > kTkSumTerms || nE > 65535 || biggest > 0x7fffffffLL) {
    set_error("tk_sum: %d terms (at most %d) or sizes beyond the kernels'", nt, kTkSumTerms);
    return LRFG_EINVAL;
  }
  TkSumArgs T;
  T.nt = nt;
  int o[3] = {0, 0, 0};
  for (int t = 0; t < nt; ++t) {
    const TKB& x = *terms[t].x;
    for (int j = 0; j < 3; ++j) {
      T.U[t][j] = x.U[j];
      T.sU[t][j] = x.sU[j];
      T.r[t][j] = x.r[j];
      T.o[t][j] = o[j];
      o[j] += x.r[j];
    }
    T.G[t] = x.G;
    T.sG[t] = x.sG;
    T.coef[t] = terms[t].coef;
    T.mult[t] = terms[t].mult;
  }
  long long fmax = 0;
  for (int j = 0; j < 3; ++j) fmax = std::max(fmax, out.usize(j));
  const int gf = (int)std::min<long long>(1024, (fmax + kB - 1) / kB);
  hipLaunchKernelGGL(k_tk_sum_frames, dim3(gf > 0 ? gf : 1, nE, 3), dim3(kB), 0, s, T, out.N[0], out.N[1], out.N[2],
                     out.U[0], out.U[1], out.U[2], out.sU[0], out.sU[1], out.sU[2], out.r[0], out.r[1], out.r[2]);
  const int gc = (int)std::min<long long>(1024, (out.gsize() + kB - 1) / kB);
  hipLaunchKernelGGL(k_tk_sum_core, dim3(gc > 0 ? gc : 1, nE), dim3(kB), 0, s, T, out.r[0], out.r[1], out.r[2], out.G,
                     out.sG);
  LRFG_LAUNCHED();
  return LRFG_OK;
}

size_t tk_dot_scratch(const TKB& x, const TKB& y, int nE) {
  size_t n = 0;
  for (int j = 0; j < 3; ++j) n += (size_t)x.r[j] * y.r[j];
  n += (size_t)y.r[0] * y.r[1] * x.r[2];   // T1
  n += (size_t)x.r[0] * y.r[1] * x.r[2];   // T2
  n += (size_t)x.gsize();                  // T3
  return n * nE + 4096 + kTkDotSplitK;
}

int tk_dot(const TKB& x, const TKB& y, double* dots, double* scratch, int nE, hipStream_t s, int pairs) {
  // With pairs = P the batch runs over t = e P + j: x system e with y system
  // (e / P) P + j (every pair within each group of P systems).
  const int P = pairs > 0 ? pairs : 1;
  const int T = pairs > 0 ? nE * P : nE;
  auto map_y_b = [&](GB& g, const double* p, long long ld, long long sy, bool t) {
    g.b(p, ld, pairs > 0 ? sy * P : sy, t);
    if (pairs > 0) {
      g.g.bdiv = P * P;
      g.g.bmod = P;
      g.g.sB2 = sy;
    }
  };
  double* p = scratch;
  double* W[3];
  double* gs = scratch + tk_dot_scratch(x, y, T) - kTkDotSplitK;
  for (int j = 0; j < 3; ++j) {
    W[j] = p;
    p += (size_t)x.r[j] * y.r[j] * T;
    // W_j = U_xj^T U_yj (rx_j x ry_j)
    GB g(x.r[j], y.r[j], x.N[j], T);
    g.a(x.U[j], x.r[j], x.sU[j], true);
    g.g.adiv = P;
    map_y_b(g, y.U[j], y.r[j], y.sU[j], false);
    g.c(W[j], y.r[j], (long long)x.r[j] * y.r[j]);
    LRFG_TRY(gemm(g.g, gs, kTkDotSplitK, s));
  }
  const int rx1 = x.r[0], rx2 = x.r[1], rx3 = x.r[2], ry1 = y.r[0], ry2 = y.r[1], ry3 = y.r[2];
  double* T1 = p;
  p += (size_t)ry1 * ry2 * rx3 * T;
  double* T2 = p;
  p += (size_t)rx1 * ry2 * rx3 * T;
  double* T3 = p;
  // T1 = G_y (ry1 ry2 x ry3) W3^T
  { GB g(ry1 * ry2, rx3, ry3, T);
    g.a(y.G, ry3, pairs > 0 ? y.sG * P : y.sG);
    if (pairs > 0) {
      g.g.adiv = P * P;
      g.g.amod = P;
      g.g.sA2 = y.sG;
    }
    g.b(W[2], ry3, (long long)rx3 * ry3, true).c(T1, rx3, (long long)ry1 * ry2 * rx3);
    LRFG_TRY(gemm(g.g, gs, kTkDotSplitK, s)); }
  // T2 = W1 (rx1 x ry1) T1 (ry1 x ry2 rx3)
  { GB g(rx1, ry2 * rx3, ry1, T); g.a(W[0], ry1, (long long)rx1 * ry1).b(T1, (long long)ry2 * rx3, (long long)ry1 * ry2 * rx3)
        .c(T2, (long long)ry2 * rx3, (long long)rx1 * ry2 * rx3);
    LRFG_TRY(gemm(g.g, gs, kTkDotSplitK, s)); }
  // T3 = T2 x_2 W2 (rx2 x ry2)
  const long long n3 = (long long)rx1 * rx2 * rx3;
  LRFG_TRY(mode2(T2, (long long)rx1 * ry2 * rx3, rx1, ry2, rx3, W[1], (long long)rx2 * ry2, rx2, 0, T3, n3, T, gs,
                kTkDotSplitK, s));
  // dots[t] = <G_x, T3_t>
  return dot_rows(n3, x.G, x.sG, P, T3, n3, dots, T, gs, kTkDotSplitK, s);
}

// ====================================================================== rounding
void TkRounder::carve(Arena& ar) {
  const int L = Lmax;
  auto T = [&](long long n) { return ar.take<double>((size_t)n * nE); };
  const long long R1 = Rmax[0], R2 = Rmax[1], R3 = Rmax[2];
  long long Nm = 1;
  for (int j = 0; j < 3; ++j) Nm = std::max<long long>(Nm, N[j]);
  // Y, Q and S of the three modes live in one buffer each, so that the
  // orthonormalisation and the cut of all modes can run as one batch
  Yall = T(3 * Nm * L);
  Qall = T(3 * Nm * L);
  Sall = T(3LL * L * L);
  for (int j = 0; j < 3; ++j) {
    om[j] = ar.take<double>((size_t)N[j] * L);
    Z[j] = T(Rmax[j] * L);
    Yc[j] = T(Rmax[j] * L);
    M[j] = T(Rmax[j] * L);
  }
  H = T(R1 * R2 * L);  // H, then the Khatri-Rao rows, then T1 (R1 R2 x l)
  T2 = T((long long)L * R2 * L);
  Cc = T((long long)L * L * L);
  T3 = T((long long)L * L * L);
  T4 = T((long long)L * L * L);
  Gr = T(3LL * L * L);
  Gs = T(3LL * L * L);
  Ss = T(3LL * L * L);
  Ytmp = T(3 * Nm * L);
  if (kron) {
    Kp = T(R1 * R2 * L);
    Kh = T(R1 * R2 * L);
    Kw = T(R1 * R2 * L);
    KY = T(R3 * L);
    KM = T(R3 * L);
  }
  kept = ar.take<int>((size_t)3 * nE);
  gscr_n = (size_t)4 * 1024 * 1024;
  gscr = ar.take<double>(gscr_n);
  KR = H;
  T1 = H;
}

namespace {

// Q (m x l) = orth(Y) by Gram matrix + pivoted Cholesky, twice.
int tk_orth(TkRounder& R, const double* Y, double* Q, int m, int l, int batch, hipStream_t s) {
  const double tau = 1e-14;
  const double* src = Y;
  double* dsts[2] = {R.Ytmp, Q};
  for (int pass = 0; pass < 2; ++pass) {
    GB gg(l, l, m, batch);
    gg.a(src, l, (long long)m * l, true).b(src, l, (long long)m * l).c(R.Gs, l, (long long)l * l);
    LRFG_TRY(gemm(gg.g, R.gscr, R.gscr_n, s));
    LRFG_TRY(pchol_s(l, R.Gs, (long long)l * l, tau, R.Ss, (long long)l * l, nullptr, batch, s));
    GB gq(m, l, l, batch);
    gq.a(src, l, (long long)m * l).b(R.Ss, l, (long long)l * l).c(dsts[pass], l, (long long)m * l);
    LRFG_TRY(gemm(gq.g, R.gscr, R.gscr_n, s));
    src = dsts[pass];
  }
  return LRFG_OK;
}

}  // namespace

// (G_a (x) G_x) x_3 B for B = (R3 x l) per system (Z3, or M3 transposed),
// written to `dst` in the core-sketch layout [(i1, k1)][(i2, k2)][c]: a GEMM
// over i3 with G_a, a GEMM over k3 with G_x (batch ordered (i1, i2) major),
// and one reordering pass.
int TkRounder::kron_mode3(const KronCore& kc, const double* B, long long sB, int l, int nb, double* dst,
                          hipStream_t s, int gp) {
  const int ra1 = kc.ra[0], ra2 = kc.ra[1], ra3 = kc.ra[2], rx1 = kc.rx[0], rx2 = kc.rx[1], rx3 = kc.rx[2];
  // P[t][(i1, i2)][(k3, c)] = sum_{i3} Ga[(i1, i2)][i3] B[t][i3][(k3, c)]
  {
    GB g(ra1 * ra2, rx3 * l, ra3, nb);
    g.a(kc.Ga, ra3, kc.sGa).b(B, (long long)rx3 * l, sB).c(Kp, (long long)rx3 * l, (long long)ra1 * ra2 * rx3 * l);
    LRFG_TRY(gemm(with_prec(g.g, gp), gscr, gscr_n, s));
  }
  // H'[(i1, i2)][t][(k1, k2)][c] = sum_{k3} Gx[t][(k1, k2)][k3] P[t][(i1, i2)][k3][c]
  {
    GB g(rx1 * rx2, l, rx3, ra1 * ra2 * nb);
    g.a(kc.Gx, rx3, 0);
    g.g.amod = kc.xmod;
    g.g.sA2 = kc.sGx;
    g.b(Kp, l, (long long)rx3 * l);
    g.g.bdiv = nb;
    g.g.bmod = nb;
    g.g.sB2 = (long long)ra1 * ra2 * rx3 * l;
    g.c(Kh, l, (long long)rx1 * rx2 * l);
    LRFG_TRY(gemm(with_prec(g.g, gp), gscr, gscr_n, s));
  }
  const long long tot = (long long)ra1 * ra2 * nb * rx1 * rx2 * l;
  hipLaunchKernelGGL(k_kron_unfold, dim3(grid_for(tot)), dim3(kB), 0, s, (const double*)Kh, dst, ra1, ra2, nb, rx1,
                     (long long)rx2 * l);
  LRFG_LAUNCHED();
  return LRFG_OK;
}

int TkRounder::round(const TKB& in, TKB& out, double tol, hipStream_t s, int batch, const KronCore* kc) {
  ProfScope ps_("tk_round", s);
  if (batch < 0) batch = nE;
  if (batch > nE) {
    set_error("tk_round: batch %d exceeds the plan's %d", batch, nE);
    return LRFG_EINVAL;
  }
  const int nb = batch;
  const int R1 = in.r[0], R2 = in.r[1], R3 = in.r[2];
  const int Rj[3] = {R1, R2, R3};
  int cmax = 1;
  for (int j = 0; j < 3; ++j) cmax = std::max(cmax, out.r[j]);
  const int l = std::min(cmax + oversample, kMaxEig);
  for (int j = 0; j < 3; ++j) {
    if (Rj[j] > Rmax[j] || out.r[j] > l) {
      set_error("tk_round: sizes exceed the plan");
      return LRFG_EINVAL;
    }
  }
  if (l > Lmax) {
    set_error("tk_round: sketch %d exceeds the plan's %d", l, Lmax);
    return LRFG_EINVAL;
  }
  if (kc != nullptr) {
    if (!kron) {
      set_error("tk_round: the plan holds no Kronecker buffers");
      return LRFG_EINVAL;
    }
    for (int j = 0; j < 3; ++j) {
      if (kc->ra[j] * kc->rx[j] != Rj[j]) {
        set_error("tk_round: Kronecker ranks do not match the frames");
        return LRFG_EINVAL;
      }
    }
    if ((long long)kc->ra[0] * kc->ra[1] * kc->rx[2] > (long long)Rmax[0] * Rmax[1] ||
        (long long)kc->ra[2] * kc->rx[2] > Rmax[2] || kc->xmod < 1 || nb % kc->xmod != 0) {
      set_error("tk_round: Kronecker shapes exceed the plan");
      return LRFG_EINVAL;
    }
  }
  // sketch contractions in the rounder's precision, projections onto the
  // orthonormal bases at least FP32, Gram matrices and factorisations FP64
  const int pj = prec == LRFG_PREC_MIXED_BF16 ? LRFG_PREC_MIXED_FP32 : prec;
  const double tol2 = tol * tol / 3.0;
  const uint64_t key = (seed * 0x9E3779B97F4A7C15ull) ^ (0xD1B54A32D192ED03ull * (++counter));
  const long long sZ[3] = {(long long)R1 * l, (long long)R2 * l, (long long)R3 * l};
  // 1. Z_j = U_j^T Om_j
  for (int j = 0; j < 3; ++j) {
    LRFG_TRY(launch_randn(om[j], (long long)N[j] * l, key ^ (0xA5A5A5A5A5A5A5A5ull * (uint64_t)(j + 1)), s));
    GB g(Rj[j], l, N[j], nb);
    g.a(in.U[j], Rj[j], in.sU[j], true).b(om[j], l, 0).c(Z[j], l, sZ[j]);
    LRFG_TRY(gemm(with_prec(g.g, prec), gscr, gscr_n, s));
  }
  // 2. sketch cores: H = G x_3 Z3^T, Y cores of modes 1 and 2 from H; mode 3
  //    from the Khatri-Rao rows of Z1, Z2
  const long long sH = (long long)R1 * R2 * l;
  if (kc == nullptr) {
    GB g(R1 * R2, l, R3, nb);
    g.a(in.G, R3, in.sG).b(Z[2], l, sZ[2]).c(H, l, sH);
    LRFG_TRY(gemm(with_prec(g.g, prec), gscr, gscr_n, s));
  } else {
    LRFG_TRY(kron_mode3(*kc, Z[2], sZ[2], l, nb, H, s, prec));
  }
  hipLaunchKernelGGL(k_tcontract, dim3(R1 + R2, nb), dim3(256), 0, s, (const double*)H, sH, (const double*)Z[0], sZ[0],
                     (const double*)Z[1], sZ[1], R1, R2, l, Yc[0], sZ[0], Yc[1], sZ[1]);
  LRFG_LAUNCHED();
  if (kc == nullptr) {
    hipLaunchKernelGGL(k_kr_rows, dim3(grid_for(sH * nb)), dim3(kB), 0, s, (const double*)Z[0], sZ[0], R1,
                       (const double*)Z[1], sZ[1], R2, l, KR, sH, nb);
    LRFG_LAUNCHED();
    GB g(R3, l, R1 * R2, nb);
    g.a(in.G, R3, in.sG, true).b(KR, l, sH).c(Yc[2], l, sZ[2]);
    LRFG_TRY(gemm(with_prec(g.g, prec), gscr, gscr_n, s));
  } else {
    // Yc3[(i3, k3)][c] = sum Ga[i1, i2, i3] Gx[k1, k2, k3] Z1[(i1, k1)][c] Z2[(i2, k2)][c]
    const int ra1 = kc->ra[0], ra2 = kc->ra[1], ra3 = kc->ra[2], rx1 = kc->rx[0], rx2 = kc->rx[1],
              rx3 = kc->rx[2];
    const long long sW = (long long)rx1 * rx2 * ra1 * ra2 * l;
    hipLaunchKernelGGL(k_kr_kron, dim3(grid_for(sW * nb)), dim3(kB), 0, s, (const double*)Z[0], sZ[0],
                       (const double*)Z[1], sZ[1], ra1, rx1, ra2, rx2, l, Kw, nb);
    LRFG_LAUNCHED();
    {
      // V[t][k3][(i1, i2, c)] = sum_{(k1, k2)} Gx[t][(k1, k2)][k3] W[t][(k1, k2)][(i1, i2, c)]
      GB g(rx3, ra1 * ra2 * l, rx1 * rx2, nb);
      g.a(kc->Gx, rx3, 0, true);
      g.g.amod = kc->xmod;
      g.g.sA2 = kc->sGx;
      g.b(Kw, (long long)ra1 * ra2 * l, sW).c(Kp, (long long)ra1 * ra2 * l, (long long)rx3 * ra1 * ra2 * l);
      LRFG_TRY(gemm(with_prec(g.g, prec), gscr, gscr_n, s));
    }
    {
      // Y'[t][k3][i3][c] = sum_{(i1, i2)} Ga[(i1, i2)][i3] V[t][k3][(i1, i2)][c]
      GB g(ra3, l, ra1 * ra2, nb * rx3);
      g.a(kc->Ga, ra3, kc->sGa, true);
      g.g.adiv = rx3;
      g.b(Kp, l, (long long)ra1 * ra2 * l).c(KY, l, (long long)ra3 * l);
      LRFG_TRY(gemm(with_prec(g.g, prec), gscr, gscr_n, s));
    }
    hipLaunchKernelGGL(k_swap_mid, dim3(grid_for((long long)R3 * l * nb)), dim3(kB), 0, s, (const double*)KY, Yc[2],
                       (long long)nb, rx3, ra3, (long long)l);
    LRFG_LAUNCHED();
  }
  // 3. Y_j = U_j Yc_j, Q_j = orth(Y_j), M_j = Q_j^T U_j; with equal N_j the
  //    three modes sit back to back and are orthonormalised in one batch
  const bool same_n = N[0] == N[1] && N[1] == N[2];
  for (int j = 0; j < 3; ++j) {
    Y[j] = Yall + (long long)j * nb * N[0] * l;
    Q[j] = Qall + (long long)j * nb * N[0] * l;
    if (!same_n) {
      long long off = 0;
      for (int q = 0; q < j; ++q) off += (long long)nb * N[q] * l;
      Y[j] = Yall + off;
      Q[j] = Qall + off;
    }
    const long long sY = (long long)N[j] * l;
    GB g(N[j], l, Rj[j], nb);
    g.a(in.U[j], Rj[j], in.sU[j]).b(Yc[j], l, sZ[j]).c(Y[j], l, sY);
    LRFG_TRY(gemm(with_prec(g.g, prec), gscr, gscr_n, s));
  }
  if (same_n) {
    LRFG_TRY(tk_orth(*this, Yall, Qall, N[0], l, 3 * nb, s));
  } else {
    for (int j = 0; j < 3; ++j) LRFG_TRY(tk_orth(*this, Y[j], Q[j], N[j], l, nb, s));
  }
  for (int j = 0; j < 3; ++j) {
    const long long sY = (long long)N[j] * l;
    GB g(l, Rj[j], N[j], nb);
    g.a(Q[j], l, sY, true).b(in.U[j], Rj[j], in.sU[j]).c(M[j], Rj[j], sZ[j]);
    LRFG_TRY(gemm(with_prec(g.g, pj), gscr, gscr_n, s));
  }
  // 4. C = G x_3 M3 x_1 M1 x_2 M2 (l x l x l)
  const long long l3 = (long long)l * l * l;
  if (kc == nullptr) {
    GB g(R1 * R2, l, R3, nb);
    g.a(in.G, R3, in.sG).b(M[2], R3, sZ[2], true).c(T1, l, sH);
    LRFG_TRY(gemm(with_prec(g.g, pj), gscr, gscr_n, s));
  } else {
    // M3^T (R3 x l per system), then the structured mode-3 product
    hipLaunchKernelGGL(k_swap_mid, dim3(grid_for((long long)R3 * l * nb)), dim3(kB), 0, s, (const double*)M[2], KM,
                       (long long)nb, l, R3, (long long)1);
    LRFG_LAUNCHED();
    LRFG_TRY(kron_mode3(*kc, KM, sZ[2], l, nb, T1, s, pj));
  }
  const long long sT2 = (long long)l * R2 * l;
  { GB g(l, R2 * l, R1, nb); g.a(M[0], R1, sZ[0]).b(T1, (long long)R2 * l, sH).c(T2, (long long)R2 * l, sT2);
    LRFG_TRY(gemm(with_prec(g.g, pj), gscr, gscr_n, s)); }
  LRFG_TRY(mode2(T2, sT2, l, R2, l, M[1], sZ[1], l, 0, Cc, l3, nb, gscr, gscr_n, s, pj));
  // 5. the cut: mode Gram matrices of C (mode j's nb matrices at
  //    Gr + j nb l^2), kept eigenvectors S_j (l x c_j); kept ranks of mode j
  //    at kept + j nb; with equal c_j one cut launch for all three modes
  const long long sG2 = (long long)l * l;
  double* Grj[3] = {Gr, Gr + sG2 * nb, Gr + 2 * sG2 * nb};
  {
    GB g(l, l, l * l, nb);
    g.a(Cc, (long long)l * l, l3).b(Cc, (long long)l * l, l3, true).c(Grj[0], l, sG2);
    LRFG_TRY(gemm(g.g, gscr, gscr_n, s));
  }
  hipLaunchKernelGGL(k_swap01, dim3(grid_for(l3 * nb)), dim3(kB), 0, s, (const double*)Cc, l3, l, T3, nb);
  LRFG_LAUNCHED();
  {
    GB g(l, l, l * l, nb);
    g.a(T3, (long long)l * l, l3).b(T3, (long long)l * l, l3, true).c(Grj[1], l, sG2);
    LRFG_TRY(gemm(g.g, gscr, gscr_n, s));
  }
  {
    GB g(l, l, l * l, nb);
    g.a(Cc, l, l3, true).b(Cc, l, l3).c(Grj[2], l, sG2);
    LRFG_TRY(gemm(g.g, gscr, gscr_n, s));
  }
  kept_batch = nb;
  const bool same_c = out.r[0] == out.r[1] && out.r[1] == out.r[2];
  for (int j = 0; j < 3; ++j) S[j] = Sall + (long long)j * nb * l * (same_c ? out.r[0] : l);
  if (same_c) {
    LRFG_TRY(cut_psd(l, out.r[0], Gr, sG2, tol2, Sall, (long long)l * out.r[0], kept, 3 * nb, s));
  } else {
    for (int j = 0; j < 3; ++j)
      LRFG_TRY(cut_psd(l, out.r[j], Grj[j], sG2, tol2, S[j], (long long)l * out.r[j], kept + j * nb, nb, s));
  }
  // 6. frames Q_j S_j and core C x_j S_j^T
  for (int j = 0; j < 3; ++j) {
    GB g(N[j], out.r[j], l, nb);
    g.a(Q[j], l, (long long)N[j] * l).b(S[j], out.r[j], (long long)l * out.r[j]).c(out.U[j], out.r[j], out.sU[j]);
    LRFG_TRY(gemm(with_prec(g.g, pj), gscr, gscr_n, s));
  }
  const int c1 = out.r[0], c2 = out.r[1], c3 = out.r[2];
  { GB g(l * l, c3, l, nb); g.a(Cc, l, l3).b(S[2], c3, (long long)l * c3).c(T3, c3, (long long)l * l * c3);
    LRFG_TRY(gemm(with_prec(g.g, pj), gscr, gscr_n, s)); }
  { GB g(c1, l * c3, l, nb); g.a(S[0], c1, (long long)l * c1, true).b(T3, (long long)l * c3, (long long)l * l * c3)
        .c(T4, (long long)l * c3, (long long)c1 * l * c3);
    LRFG_TRY(gemm(with_prec(g.g, pj), gscr, gscr_n, s)); }
  const long long nout = (long long)c1 * c2 * c3;
  (void)nout;
  return mode2(T4, (long long)c1 * l * c3, c1, l, c3, S[1], (long long)l * c2, c2, 1, out.G, out.sG, nb, gscr, gscr_n,
               s, pj);
}

}  // namespace lrfg
