// Tensor-train operations on the device (paper Sec. 3.1.3 and Appendix
// A.3): carriage-wise Hadamard products, block sums, per-mode 1-D DFT
// operators, inner products, and rank truncation.
//
// Truncation T reaches the rounded train through a randomised sketch of the
// input, then an SVD cut:
//   1. right partial contractions of the input with a Gaussian TT sketch of
//      ranks (l1, l2) = (c1 + p, c2 + p) (capped by the input ranks);
//   2. left-to-right: Y_j = (left part) x (right sketch), Q_j = orth(Y_j),
//      project the carriage onto Q_j and carry the rest to the right.  This
//      is the "randomise-then-orthogonalise" TT rounding of Al Daas, Ballard
//      et al. (SIAM J. Sci. Comput. 2023); it never forms the SVDs of the
//      large unfoldings the paper's rounding uses (Appendix A.3);
//   3. the left-orthogonal train of ranks (l1, l2) is then cut exactly as
//      the paper's rounding does: the singular values of each unfolding
//      (from l x l Gram matrices) decide the kept rank, at most the nominal
//      rank c_j and at least what the tolerance needs,
//      ||dropped||^2 <= tol^2 ||X||^2 / (d - 1).
// Output ranks are fixed (c1, c2); directions beyond the kept rank are zero
// columns, so every launch shape is known on the host.
// orth(Y): Gram Y^T Y, rank-revealing pivoted Cholesky Y^T Y = R^T R,
// Q = Y P R^-1 on the numerical rank, done twice (the second pass restores
// orthogonality to rounding level).  The cut's eigenvectors come from the
// same pivoted Cholesky followed by one-sided Jacobi on the factor
// (cut_psd), which needs a handful of sweeps on the graded factor.
// A Hadamard product a (.) g can enter with its middle carriage unformed
// (KrMid): the two contractions that read that carriage (the sketch T2 and
// the projection X2') then run over g's and a's carriages in turn.
#include <algorithm>
#include <cmath>
#include <cstdio>

#include "prof.h"
#include "tt.h"

namespace lrfg {

int launch_mode_op_oop(const double* xin, double* x, long long outer, int N, long long inner, int op, double t,
                       double mult, const FftDev& f, hipStream_t s, long long fib_per_group);

constexpr size_t kDotSplitK = (size_t)2 * 1024 * 1024;  // doubles of split-K partials in tt_dot

namespace {

constexpr int kB = 256;

inline int grid_for(long long n) {
  long long g = (n + kB - 1) / kB;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  return (int)g;
}

__global__ void k_fill(double* __restrict__ p, long long n, double v) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}

// batch identity matrices n x n (row-major, stride n * n)
__global__ void k_eye(double* __restrict__ p, int n, int batch) {
  const long long tot = (long long)n * n * batch;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < tot; i += (long long)gridDim.x * blockDim.x) {
    const long long k = i % ((long long)n * n);
    p[i] = (k / n == k % n) ? 1.0 : 0.0;
  }
}

__device__ inline uint64_t smix(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

// Standard normal numbers from a counter-based hash (splitmix64) and the
// Box-Muller transform.
__global__ void k_randn(double* __restrict__ out, long long n, uint64_t key) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const uint64_t a = smix(key ^ (2ull * (uint64_t)i));
    const uint64_t b = smix(key ^ (2ull * (uint64_t)i + 1ull) ^ 0x5851F42D4C957F2Dull);
    const double u1 = ((double)(a >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    const double u2 = ((double)(b >> 11)) * (1.0 / 9007199254740992.0);
    out[i] = sqrt(-2.0 * log(u1)) * cos(2.0 * kPi * u2);
  }
}

// Two independent streams of the same numbers in one launch: element i of
// o1 is k_randn's element i under k1, element i of o2 its element i under k2.
__global__ void k_randn2(double* __restrict__ o1, long long n1, uint64_t k1, double* __restrict__ o2, long long n2,
                         uint64_t k2) {
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n1 + n2;
       t += (long long)gridDim.x * blockDim.x) {
    const bool first = t < n1;
    const long long i = first ? t : t - n1;
    const uint64_t key = first ? k1 : k2;
    const uint64_t a = smix(key ^ (2ull * (uint64_t)i));
    const uint64_t b = smix(key ^ (2ull * (uint64_t)i + 1ull) ^ 0x5851F42D4C957F2Dull);
    const double u1 = ((double)(a >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    const double u2 = ((double)(b >> 11)) * (1.0 / 9007199254740992.0);
    (first ? o1 : o2)[i] = sqrt(-2.0 * log(u1)) * cos(2.0 * kPi * u2);
  }
}

// The same product for wide carriages (ra1 rx1 >= 64): rows (I, n) of the
// output, kKrRows per block, one thread per output column J, so the row
// indices are block-uniform and a thread splits its own J once; the rows'
// loads are independent and issue together.
constexpr int kKrRows = 8;
__global__ __launch_bounds__(256) void k_khatri_rao_rows(const double* __restrict__ a, long long sa, int ra0,
                                                         int ra1, const double* __restrict__ x, long long sx,
                                                         int rx0, int rx1, int N, double* __restrict__ out,
                                                         long long so) {
  constexpr int RB = kKrRows;
  const int R1 = ra1 * rx1;
  const int J = blockIdx.x * blockDim.x + threadIdx.x;
  if (J >= R1) return;
  const int j = J / rx1, m = J - (J / rx1) * rx1;
  const int e = blockIdx.z;
  const double* ae = a + e * sa;
  const double* xe = x + e * sx;
  double* oe = out + e * so;
  const int nrows = ra0 * rx0 * N;
  const int row0 = blockIdx.y * RB;
  double av[RB], xv[RB];
#pragma unroll
  for (int t = 0; t < RB; ++t) {
    const int row = row0 + t < nrows ? row0 + t : nrows - 1;
    const int I = row / N, n = row - (row / N) * N;
    const int i = I / rx0, k = I - (I / rx0) * rx0;
    av[t] = ae[((long long)i * N + n) * ra1 + j];
    xv[t] = xe[((long long)k * N + n) * rx1 + m];
  }
#pragma unroll
  for (int t = 0; t < RB; ++t)
    if (row0 + t < nrows) oe[(long long)(row0 + t) * R1 + J] = av[t] * xv[t];
}

// out[e][(i rx0 + k)][n][(j rx1 + m)] = a[i][n][j] x[e][k][n][m]
__global__ void k_khatri_rao(const double* __restrict__ a, long long sa, int ra0, int ra1,
                             const double* __restrict__ x, long long sx, int rx0, int rx1, int N,
                             double* __restrict__ out, long long so, int nE) {
  const long long R0 = (long long)ra0 * rx0, R1 = (long long)ra1 * rx1;
  const long long per = R0 * N * R1;
  const long long tot = per * nE;
  for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < tot;
       idx += (long long)gridDim.x * blockDim.x) {
    const int e = (int)(idx / per);
    long long r = idx - e * per;
    const long long J = r % R1;
    r /= R1;
    const int n = (int)(r % N);
    const long long I = r / N;
    const int i = (int)(I / rx0), k = (int)(I % rx0);
    const int j = (int)(J / rx1), m = (int)(J % rx1);
    out[e * so + (I * N + n) * R1 + J] =
        a[e * sa + ((long long)i * N + n) * ra1 + j] * x[e * sx + ((long long)k * N + n) * rx1 + m];
  }
}

// Second steps of the structured middle carriage X2 = a (.) g (system s
// reads coefficient train s % amod):
//   T2[s][i rg0 + k][n][l] = sum_j a[i][n][j] Z[s][j][k][n][l]
//   X2'[s][p][n][j rg1 + m] = sum_i a[i][n][j] U[s][p][i][n][m]
// For coefficient ranks up to RA: one block per (mode index n, train) and
// every coefficient-rank term of one thread's column held in registers: the
// slice a[:][n][:] is the same for the whole block, so it is read through
// the scalar cache once per block rather than by every thread, and a thread
// reads its Z (or U) column once and writes all ra0 (or ra1) outputs of it,
// each sum over the coefficient rank in order.  Wider coefficients take
// both steps as batched GEMMs (Rounder::round).
template <int RA>
__global__ __launch_bounds__(256) void k_kr_t2_reg(const double* __restrict__ a, long long sa, int amod, int ra0,
                                                   int ra1, int N, const double* __restrict__ Z, long long sz,
                                                   int rg0, int l2, double* __restrict__ T2, long long st) {
  const int n = blockIdx.x, s = blockIdx.y;
  const double* an = a + (long long)(s % amod) * sa + (long long)n * ra1;  // a[i][n][j] = an[i N ra1 + j]
  const double* zs = Z + (long long)s * sz;
  double* ts = T2 + (long long)s * st;
  const long long Q = (long long)rg0 * N * l2;
  const int E = rg0 * l2;  // (k, l) at this n
  for (int e = threadIdx.x; e < E; e += blockDim.x) {
    const int k = e / l2, l = e - (e / l2) * l2;
    const long long q = ((long long)k * N + n) * l2 + l;
    double z[RA];
#pragma unroll
    for (int j = 0; j < RA; ++j) z[j] = j < ra1 ? zs[(long long)j * Q + q] : 0.0;
    for (int i = 0; i < ra0; ++i) {
      const double* ar = an + (long long)i * N * ra1;
      double v = 0.0;
#pragma unroll
      for (int j = 0; j < RA; ++j)
        if (j < ra1) v = fma(ar[j], z[j], v);
      ts[(long long)i * Q + q] = v;
    }
  }
}
template <int RA>
__global__ __launch_bounds__(256) void k_kr_x2_reg(const double* __restrict__ a, long long sa, int amod, int ra0,
                                                   int ra1, int N, const double* __restrict__ U, long long su,
                                                   int rg1, int l1, double* __restrict__ X, long long sx) {
  const int n = blockIdx.x, s = blockIdx.y;
  const double* an = a + (long long)(s % amod) * sa + (long long)n * ra1;  // a[i][n][j] = an[i N ra1 + j]
  const double* us = U + (long long)s * su;
  double* xs = X + (long long)s * sx;
  const int E = l1 * rg1;  // (p, m) at this n
  for (int e = threadIdx.x; e < E; e += blockDim.x) {
    const int p = e / rg1, m = e - (e / rg1) * rg1;
    const double* up = us + ((long long)p * ra0 * N + n) * rg1 + m;
    double u[RA];
#pragma unroll
    for (int i = 0; i < RA; ++i) u[i] = i < ra0 ? up[(long long)i * N * rg1] : 0.0;
    double* xo = xs + (((long long)p * N + n) * ra1) * rg1 + m;
    for (int j = 0; j < ra1; ++j) {
      double v = 0.0;
#pragma unroll
      for (int i = 0; i < RA; ++i)
        if (i < ra0) v = fma(an[(long long)i * N * ra1 + j], u[i], v);
      xo[(long long)j * rg1] = v;
    }
  }
}
constexpr int kKrRegRank = 16;

// Copy of the carriages of the systems whose bit is set (one launch for
// every carriage and system; system e = blockIdx.y).
struct CopySel {
  const double* x[3];
  double* y[3];
  long long sx[3], sy[3], n[3];
  int d;
  unsigned long long mask[4];
};
__global__ __launch_bounds__(256) void k_tt_copy_sel(CopySel A) {
  const int e = blockIdx.y;
  if (!((A.mask[e >> 6] >> (e & 63)) & 1ull)) return;
  for (int j = 0; j < A.d; ++j)
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < A.n[j];
         i += (long long)gridDim.x * blockDim.x)
      A.y[j][e * A.sy[j] + i] = A.x[j][e * A.sx[j] + i];
}

// Carriage of a block sum of up to kSumTerms trains, every output element
// written once: term t's carriage sits at row offset o0[t], column offset
// o1[t] (times c_t = mult_t coef_t[e] on the first carriage), zeros
// elsewhere.  Indices are per system (blockIdx.y), in 32 bits.
constexpr int kSumTerms = 12;
struct SumCarriage {
  const double* x[kSumTerms];
  long long sx[kSumTerms];
  int r0[kSumTerms], r1[kSumTerms], o0[kSumTerms], o1[kSumTerms];
  const double* coef[kSumTerms];
  double mult[kSumTerms];
  int nt;
};
__global__ __launch_bounds__(256) void k_sum_carriage(SumCarriage T, int R0, int N, int R1,
                                                      double* __restrict__ out, long long so) {
  const int e = blockIdx.y;
  const int per = R0 * N * R1;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < per; idx += gridDim.x * blockDim.x) {
    const int J = idx % R1;
    const int r = idx / R1;
    const int n = r % N, I = r / N;
    double v = 0.0;
    for (int t = 0; t < T.nt; ++t) {
      const int i = I - T.o0[t], j = J - T.o1[t];
      if (i >= 0 && i < T.r0[t] && j >= 0 && j < T.r1[t]) {
        const double c = T.mult[t] * (T.coef[t] != nullptr ? T.coef[t][e] : 1.0);
        v = c * T.x[t][e * T.sx[t] + ((long long)i * N + n) * T.r1[t] + j];
      }
    }
    out[e * so + idx] = v;
  }
}

}  // namespace

int launch_randn(double* out, long long n, uint64_t key, hipStream_t s) {
  if (n <= 0) return LRFG_OK;
  hipLaunchKernelGGL(k_randn, dim3(grid_for(n)), dim3(kB), 0, s, out, n, key);
  LRFG_LAUNCHED();
  return LRFG_OK;
}

// ====================================================================== host helpers
TTB tt_alloc(Arena& ar, int d, const int N[3], const int r[4], int nE) {
  TTB t;
  t.d = d;
  for (int j = 0; j < 3; ++j) t.N[j] = (j < d) ? N[j] : 1;
  for (int j = 0; j < 4; ++j) t.r[j] = (j <= d) ? r[j] : 1;
  t.r[0] = 1;
  t.r[d] = 1;
  for (int j = 0; j < d; ++j) {
    t.s[j] = t.size(j);
    t.c[j] = ar.take<double>((size_t)t.s[j] * nE);
  }
  return t;
}

int tt_fill(double* p, long long n, double v, hipStream_t s) {
  if (n <= 0) return LRFG_OK;
  hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(kB), 0, s, p, n, v);
  LRFG_LAUNCHED();
  return LRFG_OK;
}

int tt_zero(TTB& x, int nE, hipStream_t s) {
  for (int j = 0; j < x.d; ++j) LRFG_TRY(tt_fill(x.c[j], x.size(j) * (x.s[j] ? nE : 1), 0.0, s));
  return LRFG_OK;
}

int tt_copy_systems(const TTB& x, TTB& y, int nE, const unsigned long long* mask, hipStream_t s) {
  if (nE <= 0) return LRFG_OK;
  if (nE > 256) {
    set_error("tt_copy: %d systems (at most 256)", nE);
    return LRFG_EINVAL;
  }
  CopySel A;
  A.d = x.d;
  long long nmax = 0;
  for (int j = 0; j < x.d; ++j) {
    if (x.size(j) != y.size(j)) {
      set_error("tt_copy: rank mismatch");
      return LRFG_EINVAL;
    }
    A.x[j] = x.c[j];
    A.y[j] = y.c[j];
    A.sx[j] = x.s[j];
    A.sy[j] = y.s[j];
    A.n[j] = x.size(j);
    nmax = std::max(nmax, A.n[j]);
  }
  bool any = false;
  for (int k = 0; k < 4; ++k) {
    A.mask[k] = mask != nullptr ? mask[k] : ~0ull;
    any = any || A.mask[k] != 0ull;
  }
  if (!any) return LRFG_OK;
  const int gx = (int)std::min<long long>(1024, std::max<long long>(1, (nmax + kB - 1) / kB));
  hipLaunchKernelGGL(k_tt_copy_sel, dim3(gx, nE), dim3(kB), 0, s, A);
  LRFG_LAUNCHED();
  return LRFG_OK;
}

int tt_copy(const TTB& x, TTB& y, int nE, hipStream_t s) { return tt_copy_systems(x, y, nE, nullptr, s); }

int tt_mode_apply(const TTB& x, TTB& y, int j, int op, double t, double mult, const FftDev& f, int nE,
                  hipStream_t s) {
  // y shares every carriage of x except j, which is y.c[j] (caller's buffer)
  if (x.s[j] != 0 && x.s[j] != x.size(j)) {
    set_error("tt_mode_apply: carriage %d is not compact", j);
    return LRFG_EINVAL;
  }
  double* cj = y.c[j];
  y = x;
  y.c[j] = cj;
  y.s[j] = x.size(j);
  if (x.s[j] == 0) y.s[j] = 0;
  const int reps = (x.s[j] == 0) ? 1 : nE;
  return launch_mode_op_oop(x.c[j], y.c[j], (long long)reps * x.r[j], x.N[j], x.r[j + 1], op, t, mult, f, s,
                            (long long)x.r[j] * x.r[j + 1]);
}

int tt_hadamard(const TTB& a, const TTB& x, TTB& out, int nE, hipStream_t s, int skip) {
  for (int j = 0; j < x.d; ++j) {
    if (out.r[j] != a.r[j] * x.r[j] || out.r[j + 1] != a.r[j + 1] * x.r[j + 1]) {
      set_error("tt_hadamard: output ranks");
      return LRFG_EINVAL;
    }
    if (j == skip) continue;
    const long long tot = out.size(j) * nE;
    ProfScope ps_("khatri_rao", s);
    const int R1 = out.r[j + 1];
    const long long nrows = (long long)out.r[j] * x.N[j];
    const long long rblocks = (nrows + kKrRows - 1) / kKrRows;
    if (R1 >= 64 && rblocks <= 65535 && nE <= 65535) {
      const int bt = R1 >= 256 ? 256 : (R1 + 63) / 64 * 64;
      const dim3 grid((unsigned)((R1 + bt - 1) / bt), (unsigned)rblocks, (unsigned)nE);
      hipLaunchKernelGGL(k_khatri_rao_rows, grid, dim3(bt), 0, s, (const double*)a.c[j], a.s[j], a.r[j], a.r[j + 1],
                         (const double*)x.c[j], x.s[j], x.r[j], x.r[j + 1], x.N[j], out.c[j], out.s[j]);
    } else {
      hipLaunchKernelGGL(k_khatri_rao, dim3(grid_for(tot)), dim3(kB), 0, s, (const double*)a.c[j], a.s[j], a.r[j],
                         a.r[j + 1], (const double*)x.c[j], x.s[j], x.r[j], x.r[j + 1], x.N[j], out.c[j], out.s[j],
                         nE);
    }
    LRFG_LAUNCHED();
  }
  return LRFG_OK;
}

int tt_sum(const TTTerm* terms, int nt, TTB& out, int nE, hipStream_t s) {
  const int d = out.d;
  int o[4] = {0, 0, 0, 0};  // running offsets per bond
  for (int j = 1; j < d; ++j) {
    int sum = 0;
    for (int t = 0; t < nt; ++t) sum += terms[t].x->r[j];
    if (sum != out.r[j]) {
      set_error("tt_sum: output rank %d != %d at bond %d", out.r[j], sum, j);
      return LRFG_EINVAL;
    }
  }
  long long biggest = 0;
  for (int j = 0; j < d; ++j) biggest = std::max(biggest, out.size(j));
  if (nt > kSumTerms || nE > 65535 || biggest > 0x7fffffffLL) {
    set_error("tt_sum: %d terms (at most %d) or sizes beyond the kernel's", nt, kSumTerms);
    return LRFG_EINVAL;
  }
  // one launch per carriage writes every block and the zeros between them
  // (the middle carriages are block diagonal)
  SumCarriage T[3];
  for (int j = 0; j < d; ++j) T[j].nt = nt;
  for (int t = 0; t < nt; ++t) {
    const TTB& x = *terms[t].x;
    for (int j = 0; j < d; ++j) {
      T[j].x[t] = x.c[j];
      T[j].sx[t] = x.s[j];
      T[j].r0[t] = x.r[j];
      T[j].r1[t] = x.r[j + 1];
      T[j].o0[t] = o[j];
      T[j].o1[t] = o[j + 1];
      T[j].coef[t] = j == 0 ? terms[t].coef : nullptr;
      T[j].mult[t] = j == 0 ? terms[t].mult : 1.0;
    }
    for (int j = 1; j < d; ++j) o[j] += x.r[j];
  }
  for (int j = 0; j < d; ++j) {
    const long long per = out.size(j);
    const int gx = (int)std::min<long long>(1024, (per + kB - 1) / kB);
    hipLaunchKernelGGL(k_sum_carriage, dim3(gx > 0 ? gx : 1, nE), dim3(kB), 0, s, T[j], out.r[j], out.N[j],
                       out.r[j + 1], out.c[j], out.s[j]);
    LRFG_LAUNCHED();
  }
  return LRFG_OK;
}

int tt_blocks(const TTBlock* const blocks[3], const int nb[3], TTB& out, int nE, hipStream_t s) {
  const int d = out.d;
  if (nE > 65535) {
    set_error("tt_blocks: %d systems", nE);
    return LRFG_EINVAL;
  }
  for (int j = 0; j < d; ++j) {
    if (nb[j] < 1 || nb[j] > kSumTerms || out.size(j) > 0x7fffffffLL) {
      set_error("tt_blocks: %d blocks in carriage %d (1..%d) or sizes beyond the kernel's", nb[j], j, kSumTerms);
      return LRFG_EINVAL;
    }
    SumCarriage T;
    T.nt = nb[j];
    for (int t = 0; t < nb[j]; ++t) {
      const TTBlock& b = blocks[j][t];
      if (b.o0 < 0 || b.o1 < 0 || b.o0 + b.r0 > out.r[j] || b.o1 + b.r1 > out.r[j + 1]) {
        set_error("tt_blocks: block %d of carriage %d outside the %d x %d carriage", t, j, out.r[j], out.r[j + 1]);
        return LRFG_EINVAL;
      }
      T.x[t] = b.x;
      T.sx[t] = b.sx;
      T.r0[t] = b.r0;
      T.r1[t] = b.r1;
      T.o0[t] = b.o0;
      T.o1[t] = b.o1;
      T.coef[t] = b.coef;
      T.mult[t] = b.mult;
    }
    const long long per = out.size(j);
    const int gx = (int)std::min<long long>(1024, (per + kB - 1) / kB);
    hipLaunchKernelGGL(k_sum_carriage, dim3(gx > 0 ? gx : 1, nE), dim3(kB), 0, s, T, out.r[j], out.N[j],
                       out.r[j + 1], out.c[j], out.s[j]);
    LRFG_LAUNCHED();
  }
  return LRFG_OK;
}

size_t tt_dot_scratch(const TTB& x, const TTB& y, int nE) {
  size_t n = 0;
  for (int j = 0; j < x.d; ++j) {
    n += (size_t)x.r[j + 1] * y.r[j + 1];          // M_j
    n += (size_t)x.r[j] * y.N[j] * y.r[j + 1];     // U_j
  }
  return n * nE + 4096 + kDotSplitK;               // + split-K space
}

int tt_dot(const TTB& x, const TTB& y, double* dots, double* scratch, int nE, hipStream_t s, int pairs) {
  const int d = x.d;
  // M_0 = 1; U_j = M_{j-1} Y_j  (x.r[j] x N y.r[j+1]); M_j = X_j^T U_j
  // (contraction over (r_{j-1}, n)); the last step contracts everything.
  // With pairs = P the batch runs over t = e P + j: x system e with y system
  // (e / P) P + j, so every pair within each group of P systems in one pass.
  const int P = pairs > 0 ? pairs : 1;
  const int T = pairs > 0 ? nE * P : nE;
  double* M = nullptr;  // previous M, (x.r[j] x y.r[j]) per system
  long long sM = 0;
  double* p = scratch;
  double* gs = scratch + tt_dot_scratch(x, y, T) - kDotSplitK;
  const size_t gsn = kDotSplitK;
  // y system of pair t as a batch map on the B operand
  auto map_y = [&](Gemm& g, long long sy) {
    if (pairs > 0) {
      g.bdiv = P * P;
      g.sB = sy * P;
      g.bmod = P;
      g.sB2 = sy;
    } else {
      g.sB = sy;
    }
  };
  for (int j = 0; j < d; ++j) {
    const int a0 = x.r[j], a1 = x.r[j + 1], b0 = y.r[j], b1 = y.r[j + 1], N = y.N[j];
    // U = M Y_j : (a0 x b0)(b0 x N b1); j = 0 -> U = Y_0 (a0 = b0 = 1)
    const double* U = y.c[j];
    long long sU = y.s[j];
    bool u_is_y = true;
    if (j > 0) {
      double* Ub = p;
      p += (size_t)a0 * N * b1 * T;
      Gemm g;
      g.m = a0;
      g.n = N * b1;
      g.k = b0;
      g.A = M;
      g.lda = b0;
      g.sA = sM;
      g.B = y.c[j];
      g.ldb = (long long)N * b1;
      map_y(g, y.s[j]);
      g.C = Ub;
      g.ldc = (long long)N * b1;
      g.sC = (long long)a0 * N * b1;
      g.batch = T;
      LRFG_TRY(gemm(g, gs, gsn, s));
      U = Ub;
      sU = g.sC;
      u_is_y = false;
    }
    // M_j = X_j^T U : (a1 x a0 N)(a0 N x b1); the last one (1 x 1) is a
    // plain dot product
    if (j == d - 1 && a1 == 1 && b1 == 1 && !u_is_y)
      return dot_rows((long long)a0 * N, x.c[j], x.s[j], P, U, sU, dots, T, gs, gsn, s);
    double* Mn = (j == d - 1) ? dots : p;
    if (j < d - 1) p += (size_t)a1 * b1 * T;
    Gemm g;
    g.m = a1;
    g.n = b1;
    g.k = a0 * N;
    g.A = x.c[j];
    g.lda = a1;
    g.sA = x.s[j];
    g.adiv = P;
    g.ta = true;
    g.B = U;
    g.ldb = b1;
    if (u_is_y) map_y(g, sU); else g.sB = sU;
    g.C = Mn;
    g.ldc = b1;
    g.sC = (j == d - 1) ? 1 : (long long)a1 * b1;
    g.batch = T;
    LRFG_TRY(gemm(g, gs, gsn, s));
    M = Mn;
    sM = g.sC;
  }
  return LRFG_OK;
}

// ====================================================================== rounding
void Rounder::carve(Arena& ar) {
  const int L1 = Lmax[0], L2 = Lmax[1];
  const int R1 = Rmax[0], R2 = Rmax[1];
  const int N1 = N[0], N2 = N[1], N3 = N[2];
  const int L = L1 > L2 ? L1 : L2;
  auto T = [&](long long n) { return ar.take<double>((size_t)n * nE); };
  if (d == 3) {
    om[1] = ar.take<double>((size_t)L1 * N2 * L2);
    om[2] = ar.take<double>((size_t)L2 * N3);
    W3 = T((long long)R2 * L2);
    T2 = T((long long)R1 * N2 * L2);
    W2 = T((long long)R1 * L1);
    Y1 = T((long long)N1 * L1);
    Q1 = T((long long)N1 * L1);
    M1 = T((long long)L1 * R1);
    X2p = T((long long)L1 * N2 * R2);
    Y2 = T((long long)L1 * N2 * L2);
    Q2 = T((long long)L1 * N2 * L2);
    M2 = T((long long)L2 * R2);
    X3p = T((long long)L2 * N3);
    Ytmp = T((long long)(N1 * L1 > L1 * N2 * L2 ? N1 * L1 : L1 * N2 * L2));
    Q2s = T((long long)L1 * N2 * L2);
    U = T((long long)L1 * N2 * L2);
  } else {
    om[2] = ar.take<double>((size_t)L1 * N2);
    W2 = T((long long)R1 * L1);
    Y1 = T((long long)N1 * L1);
    Q1 = T((long long)N1 * L1);
    M1 = T((long long)L1 * R1);
    X3p = T((long long)L1 * N2);
    Ytmp = T((long long)N1 * L1);
    W3 = T2 = X2p = Y2 = Q2 = M2 = Q2s = U = nullptr;
  }
  G = T((long long)L * L);
  S = T((long long)L * L);
  S3 = T((long long)L * L);
  S1 = T((long long)L * L);
  P = T((long long)L * L);
  kept = ar.take<int>((size_t)2 * nE);
  if (d == 3 && kr_ra > 0) {
    // Z = g x W3 (kr_ra kr_rg N2 L2) or U = M1 x g (L1 kr_ra N2 kr_rg) per system
    const long long z = (long long)kr_ra * kr_rg * N2 * L2, u = (long long)L1 * kr_ra * N2 * kr_rg;
    kz = T(z > u ? z : u);
  }
  // split-K partials: at least 4 Mi doubles, and for d = 3 enough for the
  // two long contractions (W2 and M2) of all nE trains in one launch, which
  // then fill the device, up to 96 Mi doubles
  gscr_n = (size_t)4 * 1024 * 1024;
  if (d == 3) {
    Gemm w2, m2;
    w2.m = R1; w2.n = L1; w2.k = N2 * L2; w2.batch = nE; w2.tb = true;
    m2.m = L2; m2.n = R2; m2.k = L1 * N2; m2.batch = nE; m2.ta = true;
    const size_t need = std::max(gemm_scratch_doubles(w2), gemm_scratch_doubles(m2));
    gscr_n = std::min<size_t>(std::max(gscr_n, need), (size_t)96 * 1024 * 1024);
  }
  gscr = ar.take<double>(gscr_n);
}

namespace {

// The truncation's contractions run in the Rounder's precision.
inline Gemm& prec_of(Gemm& g, int prec) {
  g.prec = prec;
  return g;
}

struct GemmB {
  Gemm g;
  GemmB(int m, int n, int k, int batch) {
    g.m = m;
    g.n = n;
    g.k = k;
    g.batch = batch;
  }
  GemmB& a(const double* p, long long ld, long long st, bool t = false) {
    g.A = p;
    g.lda = ld;
    g.sA = st;
    g.ta = t;
    return *this;
  }
  GemmB& b(const double* p, long long ld, long long st, bool t = false) {
    g.B = p;
    g.ldb = ld;
    g.sB = st;
    g.tb = t;
    return *this;
  }
  GemmB& c(double* p, long long ld, long long st) {
    g.C = p;
    g.ldc = ld;
    g.sC = st;
    return *this;
  }
};

}  // namespace

// Q (m x l per system, stride m*l) = orth(Y): Gram Y^T Y, rank-revealing
// pivoted Cholesky, Q = Y P R^-1 (zero columns beyond the numerical rank);
// a second pass on Q restores orthogonality to rounding level.  Ytmp holds
// the first pass.
static int orth(Rounder& R, const double* Y, double* Q, int m, int l, int batch, hipStream_t s) {
  const double tau = 1e-14;
  const double* src = Y;
  double* dsts[2] = {R.Ytmp, Q};
  for (int pass = 0; pass < 2; ++pass) {
    GemmB gg(l, l, m, batch);
    gg.a(src, l, (long long)m * l, true).b(src, l, (long long)m * l).c(R.G, l, (long long)l * l);
    LRFG_TRY(gemm(prec_of(gg.g, LRFG_PREC_FP64), R.gscr, R.gscr_n, s));
    LRFG_TRY(pchol_s(l, R.G, (long long)l * l, tau, R.S, (long long)l * l, nullptr, batch, s));
    GemmB gq(m, l, l, batch);
    gq.a(src, l, (long long)m * l).b(R.S, l, (long long)l * l).c(dsts[pass], l, (long long)m * l);
    LRFG_TRY(gemm(prec_of(gq.g, LRFG_PREC_FP64), R.gscr, R.gscr_n, s));
    src = dsts[pass];
  }
  return LRFG_OK;
}

// T2 = X2 W3 ((R1 N2) x l2 per system, R1 = ra0 rg0, R2 = ra1 rg1) for the
// middle carriage X2 = a (.) g given by its factors, ns systems; W3 is
// R2 x l2 per system (compact), kz scratch.  First the sum over g's rank:
// Z = g x W3 (GEMM over m), then the sum over a's rank:
// T2[i rg0 + k][n][l] = sum_j a[i][n][j] Z[j][k][n][l].
static int kr_t2(const KrMid& mid, int N2, int l2, const double* W3, double* T2, double* kz, int nE, int prec,
                 double* gscr, size_t gscr_n, hipStream_t s) {
  const int ra0 = mid.ra0, ra1 = mid.ra1, rg0 = mid.rg0, rg1 = mid.rg1;
  const int R1 = ra0 * rg0;
  const long long zs = (long long)ra1 * rg0 * N2 * l2;  // Z per system
  const long long st = (long long)R1 * N2 * l2;         // T2 per system
  if (ra1 <= kKrRegRank) {
    // Z[j][k][n][l] (GEMM, batch t = s ra1 + j), then the sum over j in
    // registers (k_kr_t2_reg, FP64)
    { GemmB g(rg0 * N2, l2, rg1, nE * ra1);
      g.a(mid.g, rg1, mid.sg).b(W3, l2, (long long)rg1 * l2).c(kz, l2, (long long)rg0 * N2 * l2);
      g.g.adiv = ra1;
      LRFG_TRY(gemm(prec_of(g.g, prec), gscr, gscr_n, s)); }
    const dim3 grid((unsigned)N2, (unsigned)nE);
    hipLaunchKernelGGL(k_kr_t2_reg<kKrRegRank>, grid, dim3(kB), 0, s, mid.a, mid.sa, mid.amod, ra0, ra1, N2,
                       (const double*)kz, zs, rg0, l2, T2, st);
    LRFG_LAUNCHED();
    return LRFG_OK;
  }
  // wide coefficient ranks: both steps on MFMA, Z stored as Z[k][n][j][l]
  // so that the sum over j is one small GEMM per (k, n):
  // Z[(k,n)][j][l] = sum_m g[k][n][m] W3[j rg1 + m][l]   (batch s ra1 + j)
  { GemmB g(rg0 * N2, l2, rg1, nE * ra1);
    g.a(mid.g, rg1, mid.sg).b(W3, l2, (long long)rg1 * l2).c(kz, (long long)ra1 * l2, zs);
    g.g.adiv = ra1;
    g.g.cdiv = ra1;
    g.g.cmod = ra1;
    g.g.sC2 = l2;
    LRFG_TRY(gemm(prec_of(g.g, prec), gscr, gscr_n, s)); }
  // T2[i rg0 + k][n][l] = sum_j a[i][n][j] Z[(k,n)][j][l]   (batch (s, k, n)),
  // in groups of amod systems (system s reads coefficient s % amod)
  const int amod = mid.amod > 0 ? mid.amod : nE;
  for (int s0 = 0; s0 < nE; s0 += amod) {
    const int ns = std::min(amod, nE - s0);
    GemmB g(ra0, l2, ra1, ns * rg0 * N2);
    g.a(mid.a, (long long)N2 * ra1, mid.sa).b(kz + s0 * zs, l2, (long long)ra1 * l2)
        .c(T2 + s0 * st, (long long)rg0 * N2 * l2, st);
    g.g.adiv = rg0 * N2;
    g.g.amod = N2;
    g.g.sA2 = ra1;
    g.g.cdiv = rg0 * N2;
    g.g.cmod = rg0 * N2;
    g.g.sC2 = l2;
    LRFG_TRY(gemm(prec_of(g.g, prec), gscr, gscr_n, s));
  }
  return LRFG_OK;
}

int Rounder::kr_dot(const TTB& kr, const KrMid& mid, const TTB& y, double* dots, double* dscr, size_t dscr_n,
                    int ns, hipStream_t s) {
  ProfScope ps_("kr_dot", s);
  const int N1 = N[0], N2 = N[1], N3 = N[2];
  const int R1 = kr.r[1], R2 = kr.r[2], ry1 = y.r[1], ry2 = y.r[2];
  if (d != 3 || ns > nE || kz == nullptr || mid.ra0 * mid.rg0 != R1 || mid.ra1 * mid.rg1 != R2 ||
      mid.ra0 > kr_ra || mid.ra1 > kr_ra || mid.rg0 > kr_rg || mid.rg1 > kr_rg || R1 > Rmax[0] || R2 > Rmax[1] ||
      ry1 > Lmax[0] || ry2 > Lmax[1] || (long long)R1 * ry2 > (long long)Lmax[0] * Rmax[1]) {
    set_error("kr_dot: sizes (R %d %d, y ranks %d %d, %d systems) exceed the plan", R1, R2, ry1, ry2, ns);
    return LRFG_EINVAL;
  }
  // Lf = X1^T y1 (R1 x ry1) and Rt = X3 y3^T (R2 x ry2)
  { GemmB g(R1, ry1, N1, ns); g.a(kr.c[0], R1, kr.s[0], true).b(y.c[0], ry1, y.s[0]).c(W2, ry1, (long long)R1 * ry1);
    LRFG_TRY(gemm(g.g, gscr, gscr_n, s)); }
  { GemmB g(R2, ry2, N3, ns); g.a(kr.c[2], N3, kr.s[2]).b(y.c[2], N3, y.s[2], true).c(W3, ry2, (long long)R2 * ry2);
    LRFG_TRY(gemm(g.g, gscr, gscr_n, s)); }
  const long long nv = (long long)R1 * N2 * ry2;
  const int ra0 = mid.ra0, ra1 = mid.ra1, rg0 = mid.rg0, rg1 = mid.rg1;
  // (H fits T2's space and the dot scratch when ra0 ra1 <= Rmax[0] Lmax[1]
  // and ra1 <= rg0 ry2)
  if (ra1 > kKrRegRank && (long long)ra0 * ra1 <= (long long)Rmax[0] * Lmax[1] &&
      (long long)ra1 <= (long long)rg0 * ry2) {
    // <a (.) g, y> = sum_n sum_{i,j} a[i][n][j] H[i][n][j] with
    // H_n = V_n Z_n^T over (k, l) (K = rg0 ry2, one product per grid index):
    // V[n][i][k][l] = sum_j' Lf[i rg0 + k][j'] y2[j'][n][l] and
    // Z[n][j][k][l] = sum_m g[k][n][m] Rt[j rg1 + m][l]; the same sums as
    // <X2 Rt, Lf y2> regrouped, with the long contraction on MFMA
    const long long zn = (long long)ra1 * rg0 * ry2, sh = (long long)ra0 * N2 * ra1;
    { GemmB g(rg0, ra1 * ry2, rg1, ns * N2);
      g.a(mid.g, (long long)N2 * rg1, mid.sg).b(W3, ry2, (long long)R2 * ry2).c(kz, ry2, zn);
      g.g.adiv = N2; g.g.amod = N2; g.g.sA2 = rg1;
      g.g.bdiv = N2;
      g.g.bcw = ry2; g.g.bchi = (long long)rg1 * ry2;
      g.g.ccw = ry2; g.g.cchi = (long long)rg0 * ry2;
      LRFG_TRY(gemm(g.g, gscr, gscr_n, s)); }
    { GemmB g(R1, N2 * ry2, ry1, ns);
      g.a(W2, ry1, (long long)R1 * ry1).b(y.c[1], (long long)N2 * ry2, y.s[1]).c(X2p, ry2, nv);
      g.g.ccw = ry2; g.g.cchi = (long long)R1 * ry2;
      LRFG_TRY(gemm(g.g, gscr, gscr_n, s)); }
    { GemmB g(ra0, ra1, rg0 * ry2, ns * N2);
      g.a(X2p, (long long)rg0 * ry2, nv).b(kz, (long long)rg0 * ry2, zn, true).c(T2, (long long)N2 * ra1, sh);
      g.g.adiv = N2; g.g.amod = N2; g.g.sA2 = (long long)R1 * ry2;
      g.g.cdiv = N2; g.g.cmod = N2; g.g.sC2 = ra1;
      g.g.nosplit = true;
      LRFG_TRY(gemm(g.g, gscr, gscr_n, s)); }
    // system e reads coefficient e % amod
    const int amod = mid.amod > 0 ? mid.amod : ns;
    if (amod == 1) return dot_rows(sh, mid.a, 0, 1, T2, sh, dots, ns, dscr, dscr_n, s);
    for (int s0 = 0; s0 < ns; s0 += amod)
      LRFG_TRY(dot_rows(sh, mid.a, mid.sa, 1, T2 + s0 * sh, sh, dots + s0, std::min(amod, ns - s0), dscr, dscr_n, s));
    return LRFG_OK;
  }
  // T2' = X2 Rt over the unformed middle carriage, V = Lf y2; the product is <T2', V>
  LRFG_TRY(kr_t2(mid, N2, ry2, W3, T2, kz, ns, LRFG_PREC_FP64, gscr, gscr_n, s));
  { GemmB g(R1, N2 * ry2, ry1, ns); g.a(W2, ry1, (long long)R1 * ry1).b(y.c[1], (long long)N2 * ry2, y.s[1])
        .c(X2p, (long long)N2 * ry2, nv);
    LRFG_TRY(gemm(g.g, gscr, gscr_n, s)); }
  return dot_rows(nv, T2, nv, 1, X2p, nv, dots, ns, dscr, dscr_n, s);
}

static int trunc_mask(Rounder& R, const double* Gm, int l, int c, double tol2, double* S, int* kept,
                      int nE, hipStream_t s) {
  (void)R;
  return cut_psd(l, c, Gm, (long long)l * l, tol2, S, (long long)l * c, kept, nE, s);
}

int Rounder::round(const TTB& in, TTB& out, double tol, hipStream_t s, int batch, const KrMid* mid, int nblk) {
  ProfScope ps_("tt_round", s);
  if (batch < 0) batch = nE;
  if (batch > nE) {
    set_error("tt_round: batch %d exceeds the plan's %d", batch, nE);
    return LRFG_EINVAL;
  }
  const int nE = batch;
  // sketch contractions (against the Gaussian carriages) run in the
  // Rounder's precision; projections onto the orthonormal bases need more
  // than BF16's 8-bit significands and run in FP32 at the BF16 setting
  const int pj = prec == LRFG_PREC_MIXED_BF16 ? LRFG_PREC_MIXED_FP32 : prec;
  const double tol2 = tol * tol / (double)(d - 1);
  const uint64_t key = (seed * 0x9E3779B97F4A7C15ull) ^ (0xD1B54A32D192ED03ull * (++counter));
  if (d == 3) {
    const int N1 = N[0], N2 = N[1], N3 = N[2];
    const int R1 = in.r[1], R2 = in.r[2];
    const int c1 = out.r[1], c2 = out.r[2];
    int l1 = c1 + oversample, l2 = c2 + oversample;
    if (l1 > R1) l1 = R1;
    if (l2 > R2) l2 = R2;
    if (l1 > N1) l1 = N1;
    if (l2 > N3) l2 = N3;
    if (l1 > Lmax[0] || l2 > Lmax[1] || R1 > Rmax[0] || R2 > Rmax[1] || l1 > kMaxEig || l2 > kMaxEig) {
      set_error("tt_round: sizes (R %d %d, l %d %d) exceed the plan", R1, R2, l1, l2);
      return LRFG_EINVAL;
    }
    // Gaussian sketch carriages.  A sketch as wide as the whole space it
    // samples needs no randomness: bond 2's (l2 = N3) is the identity, so
    // Y2 is the unfolding itself, and bond 1's basis (l1 = N1) is the
    // identity (below).  A square Gaussian factor would only worsen the
    // conditioning, and the Gram-based orthonormalisation then loses the
    // directions it shrinks below its threshold.
    { const long long n1 = (long long)l1 * N2 * l2, n2 = (long long)l2 * N3;
      hipLaunchKernelGGL(k_randn2, dim3(grid_for(n1 + n2)), dim3(kB), 0, s, om[1], n1, key, om[2], n2,
                         key ^ 0xA5A5A5A5A5A5A5A5ull); }
    LRFG_LAUNCHED();
    if (l2 == N3) {
      hipLaunchKernelGGL(k_eye, dim3(grid_for((long long)N3 * N3)), dim3(kB), 0, s, om[2], N3, 1);
      LRFG_LAUNCHED();
    }
    // W3 = X3 Om3^T (R2 x l2)
    { GemmB g(R2, l2, N3, nE); g.a(in.c[2], N3, in.s[2]).b(om[2], N3, 0, true).c(W3, l2, (long long)R2 * l2);
      LRFG_TRY(gemm(prec_of(g.g, prec), gscr, gscr_n, s)); }
    if (mid != nullptr && (d != 3 || kz == nullptr || mid->ra0 * mid->rg0 != R1 || mid->ra1 * mid->rg1 != R2 ||
                           mid->ra0 > kr_ra || mid->ra1 > kr_ra || mid->rg0 > kr_rg || mid->rg1 > kr_rg)) {
      set_error("tt_round: structured middle carriage does not fit (R %d %d)", R1, R2);
      return LRFG_EINVAL;
    }
    if (nblk != 1 && (nblk < 1 || mid != nullptr || prec != LRFG_PREC_FP64 || R1 % nblk != 0 || R2 % nblk != 0)) {
      set_error("tt_round: %d diagonal blocks do not fit (R %d %d)", nblk, R1, R2);
      return LRFG_EINVAL;
    }
    // block m of a block-diagonal middle carriage: rows (i, n), i in
    // [m rb0, (m + 1) rb0), columns [m rb1, (m + 1) rb1); its first entry
    // lies m (rb0 N2 R2 + rb1) past the carriage's
    const int rb0 = R1 / nblk, rb1 = R2 / nblk;
    const long long sblk = (long long)rb0 * N2 * R2 + rb1;
    // T2 = X2 W3 ((R1 N2) x l2)
    if (nblk > 1) {
      // rows of block m times rows [m rb1, (m + 1) rb1) of W3
      GemmB g(rb0 * N2, l2, rb1, nE * nblk);
      g.a(in.c[1], R2, in.s[1]).b(W3, l2, (long long)R2 * l2).c(T2, l2, (long long)R1 * N2 * l2);
      g.g.adiv = nblk; g.g.amod = nblk; g.g.sA2 = sblk;
      g.g.bdiv = nblk; g.g.bmod = nblk; g.g.sB2 = (long long)rb1 * l2;
      g.g.cdiv = nblk; g.g.cmod = nblk; g.g.sC2 = (long long)rb0 * N2 * l2;
      LRFG_TRY(gemm(g.g, gscr, gscr_n, s));
    } else if (mid == nullptr) {
      GemmB g(R1 * N2, l2, R2, nE); g.a(in.c[1], R2, in.s[1]).b(W3, l2, (long long)R2 * l2).c(T2, l2, (long long)R1 * N2 * l2);
      LRFG_TRY(gemm(prec_of(g.g, prec), gscr, gscr_n, s));
    } else {
      LRFG_TRY(kr_t2(*mid, N2, l2, W3, T2, kz, nE, prec, gscr, gscr_n, s));
    }
    // W2 = T2 Om2^T (R1 x l1), contraction over (n, l2)
    { GemmB g(R1, l1, N2 * l2, nE); g.a(T2, (long long)N2 * l2, (long long)R1 * N2 * l2).b(om[1], (long long)N2 * l2, 0, true)
          .c(W2, l1, (long long)R1 * l1);
      LRFG_TRY(gemm(prec_of(g.g, prec), gscr, gscr_n, s)); }
    // Y1 = X1 W2 (N1 x l1) ; Q1 = orth(Y1)
    { GemmB g(N1, l1, R1, nE); g.a(in.c[0], R1, in.s[0]).b(W2, l1, (long long)R1 * l1).c(Y1, l1, (long long)N1 * l1);
      LRFG_TRY(gemm(prec_of(g.g, prec), gscr, gscr_n, s)); }
    if (l1 == N1) {
      hipLaunchKernelGGL(k_eye, dim3(grid_for((long long)N1 * N1 * nE)), dim3(kB), 0, s, Q1, N1, nE);
      LRFG_LAUNCHED();
    } else {
      LRFG_TRY(orth(*this, Y1, Q1, N1, l1, nE, s));
    }
    // M1 = Q1^T X1 (l1 x R1) ; X2' = M1 X2 (l1 x N2 R2)
    { GemmB g(l1, R1, N1, nE); g.a(Q1, l1, (long long)N1 * l1, true).b(in.c[0], R1, in.s[0]).c(M1, R1, (long long)l1 * R1);
      LRFG_TRY(gemm(prec_of(g.g, pj), gscr, gscr_n, s)); }
    if (nblk > 1) {
      // columns (n, [m rb1, (m + 1) rb1)) of X2' = M1[:, m rb0 .. (m + 1) rb0)
      // times block m, both sides' columns mapped to (n, k) -> n R2 + k
      GemmB g(l1, N2 * rb1, rb0, nE * nblk);
      g.a(M1, R1, (long long)l1 * R1).b(in.c[1], (long long)N2 * R2, in.s[1])
          .c(X2p, (long long)N2 * R2, (long long)l1 * N2 * R2);
      g.g.adiv = nblk; g.g.amod = nblk; g.g.sA2 = rb0;
      g.g.bdiv = nblk; g.g.bmod = nblk; g.g.sB2 = sblk;
      g.g.cdiv = nblk; g.g.cmod = nblk; g.g.sC2 = rb1;
      g.g.bcw = rb1; g.g.bchi = R2;
      g.g.ccw = rb1; g.g.cchi = R2;
      LRFG_TRY(gemm(g.g, gscr, gscr_n, s));
    } else if (mid == nullptr) {
      GemmB g(l1, N2 * R2, R1, nE); g.a(M1, R1, (long long)l1 * R1).b(in.c[1], (long long)N2 * R2, in.s[1])
          .c(X2p, (long long)N2 * R2, (long long)l1 * N2 * R2);
      LRFG_TRY(gemm(prec_of(g.g, pj), gscr, gscr_n, s));
    } else {
      // U[l1][i][n][m] = sum_k M1[l1][i rg0 + k] g[k][n][m] (GEMM), then
      // X2'[l1][n][j rg1 + m] = sum_i a[i][n][j] U[l1][i][n][m] (k_kr_x2, FP64)
      const int ra0 = mid->ra0, ra1 = mid->ra1, rg0 = mid->rg0, rg1 = mid->rg1;
      { GemmB g(l1 * ra0, N2 * rg1, rg0, nE);
        g.a(M1, rg0, (long long)l1 * R1).b(mid->g, (long long)N2 * rg1, mid->sg)
            .c(kz, (long long)N2 * rg1, (long long)l1 * ra0 * N2 * rg1);
        LRFG_TRY(gemm(prec_of(g.g, pj), gscr, gscr_n, s)); }
      const long long su = (long long)l1 * ra0 * N2 * rg1, sx = (long long)l1 * N2 * R2;
      if (ra0 <= kKrRegRank) {
        const dim3 grid((unsigned)N2, (unsigned)nE);
        hipLaunchKernelGGL(k_kr_x2_reg<kKrRegRank>, grid, dim3(kB), 0, s, mid->a, mid->sa, mid->amod, ra0, ra1,
                           N2, (const double*)kz, su, rg1, l1, X2p, sx);
        LRFG_LAUNCHED();
      } else {
        // X2'[p][n][j rg1 + m] = sum_i a[i][n][j] U[p][i][n][m], in groups
        // of amod systems.  FP64: one product a_n^T (ra1 x ra0) times
        // U_n (ra0 x l1 rg1) per (system, n), its columns (p, m) mapped onto
        // U's and X2''s layouts; otherwise one small product per (system,
        // p, n)
        const int amod = mid->amod > 0 ? mid->amod : nE;
        for (int s0 = 0; s0 < nE; s0 += amod) {
          const int ns = std::min(amod, nE - s0);
          if (pj == LRFG_PREC_FP64) {
            GemmB g(ra1, l1 * rg1, ra0, ns * N2);
            g.a(mid->a, (long long)N2 * ra1, mid->sa, true).b(kz + s0 * su, (long long)N2 * rg1, su)
                .c(X2p + s0 * sx, rg1, sx);
            g.g.adiv = N2; g.g.amod = N2; g.g.sA2 = ra1;
            g.g.bdiv = N2; g.g.bmod = N2; g.g.sB2 = rg1;
            g.g.cdiv = N2; g.g.cmod = N2; g.g.sC2 = R2;
            g.g.bcw = rg1; g.g.bchi = (long long)ra0 * N2 * rg1;
            g.g.ccw = rg1; g.g.cchi = (long long)N2 * R2;
            LRFG_TRY(gemm(g.g, gscr, gscr_n, s));
          } else {
            GemmB g(ra1, rg1, ra0, ns * l1 * N2);
            g.a(mid->a, (long long)N2 * ra1, mid->sa, true).b(kz + s0 * su, (long long)N2 * rg1, (long long)ra0 * N2 * rg1)
                .c(X2p + s0 * sx, rg1, (long long)ra1 * rg1);
            g.g.adiv = l1 * N2;
            g.g.amod = N2;
            g.g.sA2 = ra1;
            g.g.bdiv = N2;
            g.g.bmod = N2;
            g.g.sB2 = rg1;
            LRFG_TRY(gemm(prec_of(g.g, pj), gscr, gscr_n, s));
          }
        }
      }
    }
    // Y2 = X2' W3 ((l1 N2) x l2) ; Q2 = orth(Y2)
    { GemmB g(l1 * N2, l2, R2, nE); g.a(X2p, R2, (long long)l1 * N2 * R2).b(W3, l2, (long long)R2 * l2)
          .c(Y2, l2, (long long)l1 * N2 * l2);
      LRFG_TRY(gemm(prec_of(g.g, prec), gscr, gscr_n, s)); }
    LRFG_TRY(orth(*this, Y2, Q2, l1 * N2, l2, nE, s));
    // M2 = Q2^T X2' (l2 x R2) ; X3' = M2 X3 (l2 x N3)
    { GemmB g(l2, R2, l1 * N2, nE); g.a(Q2, l2, (long long)l1 * N2 * l2, true).b(X2p, R2, (long long)l1 * N2 * R2)
          .c(M2, R2, (long long)l2 * R2);
      LRFG_TRY(gemm(prec_of(g.g, pj), gscr, gscr_n, s)); }
    { GemmB g(l2, N3, R2, nE); g.a(M2, R2, (long long)l2 * R2).b(in.c[2], N3, in.s[2]).c(X3p, N3, (long long)l2 * N3);
      LRFG_TRY(gemm(prec_of(g.g, pj), gscr, gscr_n, s)); }
    // ---- cut at bond 2: G = X3' X3'^T, S3 = kept eigenvectors (l2 x c2)
    { GemmB g(l2, l2, N3, nE); g.a(X3p, N3, (long long)l2 * N3).b(X3p, N3, (long long)l2 * N3, true).c(G, l2, (long long)l2 * l2);
      LRFG_TRY(gemm(prec_of(g.g, LRFG_PREC_FP64), gscr, gscr_n, s)); }
    LRFG_TRY(trunc_mask(*this, G, l2, c2, tol2, S3, kept + this->nE, nE, s));
    { GemmB g(c2, N3, l2, nE); g.a(S3, c2, (long long)l2 * c2, true).b(X3p, N3, (long long)l2 * N3).c(out.c[2], N3, out.s[2]);
      LRFG_TRY(gemm(prec_of(g.g, pj), gscr, gscr_n, s)); }
    // Q2s = Q2 S3 ((l1 N2) x c2); P = X3 X3^T (c2 x c2); U = Q2s P
    { GemmB g(l1 * N2, c2, l2, nE); g.a(Q2, l2, (long long)l1 * N2 * l2).b(S3, c2, (long long)l2 * c2)
          .c(Q2s, c2, (long long)l1 * N2 * c2);
      LRFG_TRY(gemm(prec_of(g.g, pj), gscr, gscr_n, s)); }
    { GemmB g(c2, c2, N3, nE); g.a(out.c[2], N3, out.s[2]).b(out.c[2], N3, out.s[2], true).c(P, c2, (long long)c2 * c2);
      LRFG_TRY(gemm(prec_of(g.g, LRFG_PREC_FP64), gscr, gscr_n, s)); }
    { GemmB g(l1 * N2, c2, c2, nE); g.a(Q2s, c2, (long long)l1 * N2 * c2).b(P, c2, (long long)c2 * c2)
          .c(U, c2, (long long)l1 * N2 * c2);
      LRFG_TRY(gemm(prec_of(g.g, pj), gscr, gscr_n, s)); }
    // ---- cut at bond 1: G1 = U Q2s^T over (n, b) (l1 x l1)
    { GemmB g(l1, l1, N2 * c2, nE); g.a(U, (long long)N2 * c2, (long long)l1 * N2 * c2)
          .b(Q2s, (long long)N2 * c2, (long long)l1 * N2 * c2, true).c(G, l1, (long long)l1 * l1);
      LRFG_TRY(gemm(prec_of(g.g, LRFG_PREC_FP64), gscr, gscr_n, s)); }
    LRFG_TRY(trunc_mask(*this, G, l1, c1, tol2, S1, kept, nE, s));
    { GemmB g(N1, c1, l1, nE); g.a(Q1, l1, (long long)N1 * l1).b(S1, c1, (long long)l1 * c1).c(out.c[0], c1, out.s[0]);
      LRFG_TRY(gemm(prec_of(g.g, pj), gscr, gscr_n, s)); }
    { GemmB g(c1, N2 * c2, l1, nE); g.a(S1, c1, (long long)l1 * c1, true).b(Q2s, (long long)N2 * c2, (long long)l1 * N2 * c2)
          .c(out.c[1], (long long)N2 * c2, out.s[1]);
      LRFG_TRY(gemm(prec_of(g.g, pj), gscr, gscr_n, s)); }
    return LRFG_OK;
  }
  // d = 2
  const int N1 = N[0], N2 = N[1];
  const int R1 = in.r[1];
  const int c1 = out.r[1];
  int l = c1 + oversample;
  if (l > R1) l = R1;
  if (l > N1) l = N1;
  if (l > N2) l = N2;
  if (l > Lmax[0] || R1 > Rmax[0] || l > kMaxEig) {
    set_error("tt_round: sizes exceed the plan");
    return LRFG_EINVAL;
  }
  // a sketch as wide as the space it samples is the identity (see d = 3)
  if (l == N2) {
    hipLaunchKernelGGL(k_eye, dim3(grid_for((long long)N2 * N2)), dim3(kB), 0, s, om[2], N2, 1);
  } else {
    hipLaunchKernelGGL(k_randn, dim3(grid_for((long long)l * N2)), dim3(kB), 0, s, om[2], (long long)l * N2, key);
  }
  LRFG_LAUNCHED();
  { GemmB g(R1, l, N2, nE); g.a(in.c[1], N2, in.s[1]).b(om[2], N2, 0, true).c(W2, l, (long long)R1 * l);
    LRFG_TRY(gemm(prec_of(g.g, prec), gscr, gscr_n, s)); }
  { GemmB g(N1, l, R1, nE); g.a(in.c[0], R1, in.s[0]).b(W2, l, (long long)R1 * l).c(Y1, l, (long long)N1 * l);
    LRFG_TRY(gemm(prec_of(g.g, prec), gscr, gscr_n, s)); }
  if (l == N1) {
    hipLaunchKernelGGL(k_eye, dim3(grid_for((long long)N1 * N1 * nE)), dim3(kB), 0, s, Q1, N1, nE);
    LRFG_LAUNCHED();
  } else {
    LRFG_TRY(orth(*this, Y1, Q1, N1, l, nE, s));
  }
  { GemmB g(l, R1, N1, nE); g.a(Q1, l, (long long)N1 * l, true).b(in.c[0], R1, in.s[0]).c(M1, R1, (long long)l * R1);
    LRFG_TRY(gemm(prec_of(g.g, pj), gscr, gscr_n, s)); }
  { GemmB g(l, N2, R1, nE); g.a(M1, R1, (long long)l * R1).b(in.c[1], N2, in.s[1]).c(X3p, N2, (long long)l * N2);
    LRFG_TRY(gemm(prec_of(g.g, pj), gscr, gscr_n, s)); }
  { GemmB g(l, l, N2, nE); g.a(X3p, N2, (long long)l * N2).b(X3p, N2, (long long)l * N2, true).c(G, l, (long long)l * l);
    LRFG_TRY(gemm(prec_of(g.g, LRFG_PREC_FP64), gscr, gscr_n, s)); }
  LRFG_TRY(trunc_mask(*this, G, l, c1, tol * tol, S1, kept, nE, s));
  { GemmB g(c1, N2, l, nE); g.a(S1, c1, (long long)l * c1, true).b(X3p, N2, (long long)l * N2).c(out.c[1], N2, out.s[1]);
    LRFG_TRY(gemm(prec_of(g.g, pj), gscr, gscr_n, s)); }
  { GemmB g(N1, c1, l, nE); g.a(Q1, l, (long long)N1 * l).b(S1, c1, (long long)l * c1).c(out.c[0], c1, out.s[0]);
    LRFG_TRY(gemm(prec_of(g.g, pj), gscr, gscr_n, s)); }
  return LRFG_OK;
}

}  // namespace lrfg
