// Full-grid GaNi solve: preconditioned CG on the Fourier-space system
//   K u^ = b^,  K = grad*^ F a F^-1 grad^,  b^ = -grad*^ F (a E)
// (paper Sec. 2.2.2, eq. ls_GaNi_fourier), preconditioner P^-1 = the
// pseudo-inverse of the Fourier Laplacian 4 pi^2 k.k (Sec. 2.3,
// eq. Pls_GaNi_fourier), A_H from the energy form of eq. (homog).
//
// Storage: real fields [N1][N2][N3] (FP64), Fourier fields as the half
// spectrum [N1][N2][H] (H = (N3+1)/2 complex; odd N3 has no Nyquist plane),
// the other half given by Hermitian symmetry.  A d = 2 problem is stored as
// N1 = 1.
//
// One matvec q = K p for all right-hand sides is five LDS-FFT passes:
//   P1 axis 1, inverse, prologue x 2 pi i k_alpha (one output per alpha)
//   P2 axis 2, inverse, in place
//   P3 axis 3: C2R, x a, R2C in one pass (two real lines per complex FFT)
//   P4 axis 2, forward, in place
//   P5 axis 1, forward, sum_alpha -2 pi i k_alpha (.), 1/|N| scale, and the
//      partial sums of (p, q) for the CG step length
// followed by two CG vector kernels.  All CG scalars stay on the device;
// converged systems are skipped by a device flag.
#include <cmath>
#include <cstdio>
#include <vector>

#include "fft.h"
#include "fft2.h"
#include "full.h"
#include "prof.h"

namespace lrfg {

int launch_pinv(const double2* u, double2* o, int N1, int N2, int N3, hipStream_t s);

namespace {

constexpr int kBlock = 256;

struct G3 {
  int N1, N2, N3, H;
  long long S;  // complex entries of a half spectrum
  long long R;  // real entries
};

// Entry and line ids of a grid stay below 2^32 (full_solve and full_op
// refuse larger grids), so their splits take 32-bit divisions.
__device__ inline long long addr3(long long l, int n, int N, long long inner) {
  const unsigned lu = (unsigned)l, iu = (unsigned)inner;
  const unsigned o = lu / iu;
  const unsigned i = lu - o * iu;
  return ((long long)o * N + n) * inner + i;
}
constexpr long long kMaxGridEntries = (1ll << 32) - 1;

// Frequencies of half-spectrum entry (n1, n2, h).
__device__ inline void kvec(const G3& g, int n1, int n2, int h, double k[3]) {
  k[0] = (double)freq_of(n1, g.N1);
  k[1] = (double)freq_of(n2, g.N2);
  k[2] = (double)h;
}

__device__ inline double pinv_of(const double k[3]) {
  const double kk = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
  return kk > 0.0 ? 1.0 / (4.0 * kPi * kPi * kk) : 0.0;
}

// Constant anisotropic part B of the coefficient A~ = a I + B (Sec. 4.4),
// embedded in the internal 3-D axes.  Its share of the operator,
// grad*^ B grad^ = 4 pi^2 k.Bk, is diagonal in Fourier space, so it is added
// to the divergence pass's output from the input p it reads anyway; its
// share of A_H, mean_x B grad u_i . grad u_j, is the Fourier sum of
// 4 pi^2 k.Bk Re(u^_i conj u^_j).
struct Aniso3 {
  double b00, b11, b22, b01, b02, b12;  // scaled by 4 pi^2
  int on;
};
// Ga (exact integration, Sec. 2.2.3): trial and test functions in T_N, kept
// on the double grid M >= 2N - 1 as spectra whose frequencies beyond
// |k_i| <= kmax_i are zero (the injection I and its adjoint I*).  on = 0:
// GaNi, no mask.
struct Mask3 {
  int k0, k1, k2;
  int on;
};
__device__ inline bool masked_out(const Mask3& m, int f0, int f1, int h) {
  return m.on && (abs(f0) > m.k0 || abs(f1) > m.k1 || h > m.k2);
}

__device__ inline double aniso_symbol(const Aniso3& B, double k0, double k1, double k2) {
  return B.b00 * k0 * k0 + B.b11 * k1 * k1 + B.b22 * k2 * k2 +
         2.0 * (B.b01 * k0 * k1 + B.b02 * k0 * k2 + B.b12 * k1 * k2);
}

// ---------------------------------------------------------------- P1
// dst[e][a] = F^-1_axis1 ( 2 pi i k_alpha src[e] ),  alpha = alpha0 + a.
// grid.x = tiles * nalpha (alpha fastest, so the tiles of one src share L2),
// grid.y = e.
template <bool GEN>
__global__ __launch_bounds__(kFftBlock) void k_grad_axis1(const double2* __restrict__ src, double2* __restrict__ dst,
                                                           G3 g, int alpha0, int nalpha, long long dst_stride_e,
                                                           long long dst_stride_a, int T, FftDev f,
                                                           const int* __restrict__ done) {
  extern __shared__ double2 sm[];
  const int e = blockIdx.y;
  if (done != nullptr && done[e]) return;
  const int a = blockIdx.x % nalpha;
  const int tile = blockIdx.x / nalpha;
  const int alpha = alpha0 + a;
  const int N = g.N1;
  const long long inner = (long long)g.N2 * g.H;
  const long long l0 = (long long)tile * T;
  const int tcount = (int)min((long long)T, inner - l0);
  const double2* s = src + (long long)e * g.S;
  double2* d = dst + e * dst_stride_e + a * dst_stride_a;
  const int total = T * N;
  const float rT = 1.0f / (float)T, rN = 1.0f / (float)N;
  double2* tw = sm + total;
  stage_twiddles(tw, f);
  double2 v[kFftMaxE];
#pragma unroll
  for (int i = 0; i < kFftMaxE; ++i) {
    const int idx = threadIdx.x + i * kFftBlock;
    const int n = fdiv(idx, T, rT), t = idx - n * T;
    v[i] = (idx < total && t < tcount) ? s[(long long)n * inner + l0 + t] : make_double2(0.0, 0.0);
  }
#pragma unroll
  for (int i = 0; i < kFftMaxE; ++i) {
    const int idx = threadIdx.x + i * kFftBlock;
    const int n = fdiv(idx, T, rT), t = idx - n * T;
    if (idx < total) {
      const long long ii = l0 + t;
      double kk;
      if (alpha == 0) kk = (double)freq_of(n, g.N1);
      else if (alpha == 1) kk = (double)freq_of((int)((unsigned)ii / (unsigned)g.H), g.N2);
      else kk = (double)((unsigned)ii % (unsigned)g.H);
      sm[t * N + n] = cmul_i(v[i], 2.0 * kPi * kk);
    }
  }
  __syncthreads();
  lds_fft1<1, GEN>(sm, T, f, tw);
#pragma unroll
  for (int i = 0; i < kFftMaxE; ++i) {
    const int idx = threadIdx.x + i * kFftBlock;
    const int n = fdiv(idx, T, rT), t = idx - n * T;
    if (idx < total && t < tcount) d[(long long)n * inner + l0 + t] = sm[t * N + n];
  }
}

// ---------------------------------------------------------------- P5
// q[e] = (1/|N|) sum_alpha -2 pi i k_alpha F_axis1(t[e][alpha]); also the
// partial sums of (p[e], q[e]) (Hermitian weights: 1 on h = 0, else 2).
template <bool GEN>
__global__ __launch_bounds__(kFftBlock) void k_div_axis1(const double2* __restrict__ t, double2* __restrict__ q,
                                                          const double2* __restrict__ p, G3 g, int alpha0, int nalpha,
                                                          double inv_vol, int T, FftDev f,
                                                          const int* __restrict__ done, double* __restrict__ part_pq,
                                                          Aniso3 an, Mask3 mk) {
  extern __shared__ double2 sm[];
  __shared__ double red[kBlock / 64];
  const int e = blockIdx.y;
  if (done[e]) return;
  const int N = g.N1;
  const long long inner = (long long)g.N2 * g.H;
  const long long l0 = (long long)blockIdx.x * T;
  const int tcount = (int)min((long long)T, inner - l0);
  const int total = T * N;
  const float rT = 1.0f / (float)T, rN = 1.0f / (float)N;
  double2* tw = sm + total;
  stage_twiddles(tw, f);
  double2 acc[kFftMaxE];
#pragma unroll
  for (int j = 0; j < kFftMaxE; ++j) acc[j] = make_double2(0.0, 0.0);
  for (int a = 0; a < nalpha; ++a) {
    const int alpha = alpha0 + a;
    const double2* s = t + ((long long)e * nalpha + a) * g.S;
    double2 v[kFftMaxE];
#pragma unroll
    for (int i = 0; i < kFftMaxE; ++i) {
      const int idx = threadIdx.x + i * kFftBlock;
      const int n = fdiv(idx, T, rT), tt = idx - n * T;
      v[i] = (idx < total && tt < tcount) ? s[(long long)n * inner + l0 + tt] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int i = 0; i < kFftMaxE; ++i) {
      const int idx = threadIdx.x + i * kFftBlock;
      const int n = fdiv(idx, T, rT), tt = idx - n * T;
      if (idx < total) sm[tt * N + n] = v[i];
    }
    __syncthreads();
    lds_fft1<-1, GEN>(sm, T, f, tw);
#pragma unroll
    for (int j = 0; j < kFftMaxE; ++j) {
      const int idx = threadIdx.x + j * kFftBlock;
      if (idx < total) {
        const int n = fdiv(idx, T, rT), tt = idx - n * T;
        const long long i = l0 + tt;
        double kk;
        if (alpha == 0) kk = (double)freq_of(n, g.N1);
        else if (alpha == 1) kk = (double)freq_of((int)(i / g.H), g.N2);
        else kk = (double)(i % g.H);
        const double2 w = sm[tt * N + n];
        const double c = -2.0 * kPi * kk * inv_vol;
        acc[j].x += -w.y * c;
        acc[j].y += w.x * c;
      }
    }
    __syncthreads();
  }
  double pq = 0.0;
  const double2* pe = p + (long long)e * g.S;
  double2* qe = q + (long long)e * g.S;
#pragma unroll
  for (int j = 0; j < kFftMaxE; ++j) {
    const int idx = threadIdx.x + j * kFftBlock;
    const int n = fdiv(idx, T, rT), tt = idx - n * T;
    if (idx < total && tt < tcount) {
      const long long i = l0 + tt;
      const long long ad = (long long)n * inner + i;
      const double2 pv = pe[ad];
      if (an.on) {
        const double c = aniso_symbol(an, (double)freq_of(n, g.N1), (double)freq_of((int)(i / g.H), g.N2),
                                      (double)(i % g.H));
        acc[j].x += c * pv.x;
        acc[j].y += c * pv.y;
      }
      if (masked_out(mk, freq_of(n, g.N1), freq_of((int)(i / g.H), g.N2), (int)(i % g.H)))
        acc[j] = make_double2(0.0, 0.0);
      qe[ad] = acc[j];
      const double w = (i % g.H) == 0 ? 1.0 : 2.0;
      pq += w * (pv.x * acc[j].x + pv.y * acc[j].y);
    }
  }
  const double s = block_sum(pq, red);
  if (threadIdx.x == 0) part_pq[(long long)e * gridDim.x + blockIdx.x] = s;
}

// ---------------------------------------------------------------- P3 / axis 3
// MODE 0: in place  X <- R2C( a . C2R(X) )        (material law)
// MODE 1: real src -> half spectrum dst (R2C, scale)
// MODE 2: half spectrum src -> real dst (C2R)
// Two real lines (l0, l0+1) share one complex FFT.  grid.x = pair tiles,
// grid.y = array index b (array b at src + b*src_stride, dst likewise),
// done index = b / done_div.
template <int MODE, bool GEN>
__global__ __launch_bounds__(kFftBlock) void k_axis3(const void* __restrict__ src_, void* __restrict__ dst_,
                                                      const double* __restrict__ acoef, G3 g, long long src_stride,
                                                      long long dst_stride, int T, FftDev f, double scale,
                                                      const int* __restrict__ done, int done_div) {
  extern __shared__ double2 sm[];
  const int b = blockIdx.y;
  if (done != nullptr && done[b / done_div]) return;
  const int N = g.N3, H = g.H;
  const long long nl = (long long)g.N1 * g.N2;
  const long long p0 = (long long)blockIdx.x * T;      // first pair
  const int total = T * N;
  const float rT = 1.0f / (float)T, rN = 1.0f / (float)N;
  double2* tw = sm + total;
  stage_twiddles(tw, f);
  // load (two real lines per complex line)
  {
    double2 v[kFftMaxE];
#pragma unroll
    for (int i = 0; i < kFftMaxE; ++i) {
      const int idx = threadIdx.x + i * kFftBlock;
      const int t = fdiv(idx, N, rN), n = idx - t * N;
      const long long la = 2 * (p0 + t), lb = la + 1;
      double2 z = make_double2(0.0, 0.0);
      if (idx < total) {
        if (MODE == 1) {
          const double* s = static_cast<const double*>(src_) + b * src_stride;
          const double xa = la < nl ? s[la * N + n] : 0.0;
          const double xb = lb < nl ? s[lb * N + n] : 0.0;
          z = make_double2(xa, xb);
        } else {
          const double2* s = static_cast<const double2*>(src_) + b * src_stride;
          const int m = n < H ? n : N - n;
          const bool cj = n >= H;
          double2 xa = make_double2(0.0, 0.0), xb = make_double2(0.0, 0.0);
          if (la < nl) xa = s[la * H + m];
          if (lb < nl) xb = s[lb * H + m];
          if (cj) {
            xa.y = -xa.y;
            xb.y = -xb.y;
          }
          z = make_double2(xa.x - xb.y, xa.y + xb.x);  // Xa + i Xb
        }
      }
      v[i] = z;
    }
#pragma unroll
    for (int i = 0; i < kFftMaxE; ++i) {
      const int idx = threadIdx.x + i * kFftBlock;
      if (idx < total) sm[idx] = v[i];
    }
  }
  __syncthreads();
  if (MODE != 1) {
    lds_fft1<1, GEN>(sm, T, f, tw);
    if (MODE == 2) {
      double* d = static_cast<double*>(dst_) + b * dst_stride;
#pragma unroll
      for (int i = 0; i < kFftMaxE; ++i) {
        const int idx = threadIdx.x + i * kFftBlock;
        const int t = fdiv(idx, N, rN), n = idx - t * N;
        const long long la = 2 * (p0 + t), lb = la + 1;
        if (idx < total) {
          const double2 w = sm[idx];
          if (la < nl) d[la * N + n] = w.x * scale;
          if (lb < nl) d[lb * N + n] = w.y * scale;
        }
      }
      return;
    }
    // multiply the two real parts by their coefficient lines
#pragma unroll
    for (int i = 0; i < kFftMaxE; ++i) {
      const int idx = threadIdx.x + i * kFftBlock;
      const int t = fdiv(idx, N, rN), n = idx - t * N;
      const long long la = 2 * (p0 + t), lb = la + 1;
      if (idx < total) {
        const double aa = la < nl ? acoef[la * N + n] : 0.0;
        const double ab = lb < nl ? acoef[lb * N + n] : 0.0;
        const double2 w = sm[idx];
        sm[idx] = make_double2(w.x * aa, w.y * ab);
      }
    }
    __syncthreads();
  }
  lds_fft1<-1, GEN>(sm, T, f, tw);
  // separate the two Hermitian spectra and store h in [0, H)
  double2* d = static_cast<double2*>(MODE == 0 ? const_cast<void*>(src_) : dst_) +
               b * (MODE == 0 ? src_stride : dst_stride);
  const int htot = T * H;
  for (int idx = threadIdx.x; idx < htot; idx += blockDim.x) {
    const int h = idx % H, t = idx / H;
    const long long la = 2 * (p0 + t), lb = la + 1;
    const double2 W1 = sm[t * N + h];
    const double2 W2 = sm[t * N + (h == 0 ? 0 : N - h)];
    // Xa = (W1 + conj W2)/2, Xb = (W1 - conj W2)/(2i)
    const double2 xa = make_double2(0.5 * (W1.x + W2.x), 0.5 * (W1.y - W2.y));
    const double2 dd = make_double2(W1.x - W2.x, W1.y + W2.y);
    const double2 xb = make_double2(0.5 * dd.y, -0.5 * dd.x);
    if (la < nl) d[la * H + h] = cscale(xa, scale);
    if (lb < nl) d[lb * H + h] = cscale(xb, scale);
  }
}

// ---------------------------------------------------------------- register passes
// The hot passes in the register form of fft2.h, for N along the pass in
// split_of's table.  A tile holds T lines (axis 1) or T pairs of real lines
// (axis 3).  Loads and stores address the arrays by 32-bit byte offsets
// from wave-uniform bases (the launchers check that the arrays fit).

// P1: dst[e][alpha - alpha0] = F^-1_axis1(2 pi i k_alpha src[e]) for the
// nalpha directions from alpha0.  k_1 and k_2 are constant along an axis-1
// line, so those outputs are one inverse transform of src scaled per line;
// k_0 varies along the line and takes a transform of its own.
template <int A, int B, int C>
__global__ __launch_bounds__(kFftBlock) void k3_grad_axis1(const double2* __restrict__ src, double2* __restrict__ dst,
                                                            G3 g, int alpha0, int nalpha, long long dst_stride_e,
                                                            long long dst_stride_a, FftDev f,
                                                            const int* __restrict__ done) {
  constexpr int N = A * B * C;
  constexpr int T = split_lines(N);
  using F = Fft3<A, B, C, 1, T, false, kFftBlock>;
  __shared__ double2 S[T * N];
  __shared__ double2 tw[N];
  const int e = blockIdx.y;
  if (done != nullptr && done[e]) return;
  const unsigned inner = (unsigned)g.N2 * (unsigned)g.H;
  const unsigned l0 = xcd_tile(blockIdx.x, gridDim.x) * (unsigned)T;
  const int tcount = (int)min(T, (int)(inner - l0));
  const double2* s = src + (long long)e * g.S;
  double2* d = dst + e * dst_stride_e;
  for (int i = threadIdx.x; i < N; i += kFftBlock) tw[i] = f.tw[i];
  const int a_end = alpha0 + nalpha;
  for (int pass = 0; pass < 2; ++pass) {
    // pass 0: the directions 1 and 2 (one transform); pass 1: direction 0
    const bool weighted = pass == 1;
    if (weighted ? alpha0 > 0 : a_end <= 1) continue;
    __syncthreads();  // tw staged / S free again
    for (int it = threadIdx.x; it < F::I1; it += kFftBlock) {
      int t, j;
      F::item1(it, t, j);
      const bool ok = t < tcount;
      const unsigned l = l0 + (unsigned)t;
      double2 v[A];
#pragma unroll
      for (int a = 0; a < A; ++a) {
        const int n = j + F::M * a;
        const double2 x = ok ? ld32(s, ((unsigned)n * inner + l) * 16u) : make_double2(0.0, 0.0);
        v[a] = weighted ? cmul_i(x, 2.0 * kPi * (double)freq_of(n, N)) : x;
      }
      F::stage1(v, t, j, S, tw);
    }
    __syncthreads();
    F::stage2(S, tw);
    __syncthreads();
    for (int it = threadIdx.x; it < F::IL; it += kFftBlock) {
      int t, k1, k2;
      F::itemL(it, t, k1, k2);
      double2 z[F::R];
      F::last(z, t, k1, k2, S);
      if (t < tcount) {
        const unsigned l = l0 + (unsigned)t;
        if (weighted) {
#pragma unroll
          for (int r = 0; r < F::R; ++r) st32(d, ((unsigned)F::out_n(k1, k2, r) * inner + l) * 16u, z[r]);
        } else {
          for (int al = alpha0 > 1 ? alpha0 : 1; al < a_end; ++al) {
            const double kk = al == 1 ? (double)freq_of((int)(l / (unsigned)g.H), g.N2) : (double)(l % (unsigned)g.H);
            double2* da = d + (long long)(al - alpha0) * dst_stride_a;
#pragma unroll
            for (int r = 0; r < F::R; ++r)
              st32(da, ((unsigned)F::out_n(k1, k2, r) * inner + l) * 16u, cmul_i(z[r], 2.0 * kPi * kk));
          }
        }
      }
    }
  }
}

// P5: q[e] = (1/|N|) sum_alpha -2 pi i k_alpha F_axis1(t[e][alpha]) and the
// partial sums of (p[e], q[e]).  The directions 1 and 2 (constant k along
// the line) are combined before one forward transform; direction 0 is
// transformed alone and weighted after it.
template <int A, int B, int C>
__global__ __launch_bounds__(kFftBlock) void k3_div_axis1(const double2* __restrict__ t, double2* __restrict__ q,
                                                           const double2* __restrict__ p, G3 g, int alpha0,
                                                           int nalpha, double inv_vol, FftDev f,
                                                           const int* __restrict__ done, double* __restrict__ part_pq,
                                                           Aniso3 an, Mask3 mk) {
  constexpr int N = A * B * C;
  constexpr int T = split_lines(N);
  using F = Fft3<A, B, C, -1, T, false, kFftBlock>;
  __shared__ double2 S[T * N];
  __shared__ double2 tw[N];
  __shared__ double red[kFftBlock / 64];
  const int e = blockIdx.y;
  if (done[e]) return;
  const unsigned inner = (unsigned)g.N2 * (unsigned)g.H;
  const unsigned l0 = xcd_tile(blockIdx.x, gridDim.x) * (unsigned)T;
  const int tcount = (int)min(T, (int)(inner - l0));
  for (int i = threadIdx.x; i < N; i += kFftBlock) tw[i] = f.tw[i];
  const int a_end = alpha0 + nalpha;
  double2 acc[F::PL][F::R];
#pragma unroll
  for (int pi = 0; pi < F::PL; ++pi)
#pragma unroll
    for (int r = 0; r < F::R; ++r) acc[pi][r] = make_double2(0.0, 0.0);
  for (int pass = 0; pass < 2; ++pass) {
    // pass 0: direction 0 (weighted after the transform); pass 1: 1 and 2
    const bool along = pass == 0;
    if (along ? alpha0 > 0 : a_end <= 1) continue;
    __syncthreads();
    for (int it = threadIdx.x; it < F::I1; it += kFftBlock) {
      int tt, j;
      F::item1(it, tt, j);
      const bool ok = tt < tcount;
      const unsigned l = l0 + (unsigned)tt;
      double2 v[A];
      if (along) {
        const double2* s = t + ((long long)e * nalpha + (0 - alpha0)) * g.S;
#pragma unroll
        for (int a = 0; a < A; ++a)
          v[a] = ok ? ld32(s, ((unsigned)(j + F::M * a) * inner + l) * 16u) : make_double2(0.0, 0.0);
      } else {
#pragma unroll
        for (int a = 0; a < A; ++a) v[a] = make_double2(0.0, 0.0);
        for (int al = alpha0 > 1 ? alpha0 : 1; al < a_end; ++al) {
          const double kk = al == 1 ? (double)freq_of((int)(l / (unsigned)g.H), g.N2) : (double)(l % (unsigned)g.H);
          const double c = -2.0 * kPi * kk * inv_vol;
          const double2* s = t + ((long long)e * nalpha + (al - alpha0)) * g.S;
#pragma unroll
          for (int a = 0; a < A; ++a) {
            const double2 x = ok ? ld32(s, ((unsigned)(j + F::M * a) * inner + l) * 16u) : make_double2(0.0, 0.0);
            v[a] = cadd(v[a], cmul_i(x, c));
          }
        }
      }
      F::stage1(v, tt, j, S, tw);
    }
    __syncthreads();
    F::stage2(S, tw);
    __syncthreads();
#pragma unroll
    for (int pi = 0; pi < F::PL; ++pi) {
      const int it = threadIdx.x + pi * kFftBlock;
      if (it < F::IL) {
        int tt, k1, k2;
        F::itemL(it, tt, k1, k2);
        double2 z[F::R];
        F::last(z, tt, k1, k2, S);
#pragma unroll
        for (int r = 0; r < F::R; ++r) {
          if (along) {
            const double c = -2.0 * kPi * (double)freq_of(F::out_n(k1, k2, r), N) * inv_vol;
            acc[pi][r] = cmul_i(z[r], c);
          } else {
            acc[pi][r] = cadd(acc[pi][r], z[r]);
          }
        }
      }
    }
  }
  double pq = 0.0;
  const double2* pe = p + (long long)e * g.S;
  double2* qe = q + (long long)e * g.S;
#pragma unroll
  for (int pi = 0; pi < F::PL; ++pi) {
    const int it = threadIdx.x + pi * kFftBlock;
    if (it < F::IL) {
      int tt, k1, k2;
      F::itemL(it, tt, k1, k2);
      if (tt < tcount) {
        const unsigned l = l0 + (unsigned)tt;
        const double w = (l % (unsigned)g.H) == 0 ? 1.0 : 2.0;
#pragma unroll
        for (int r = 0; r < F::R; ++r) {
          const int n1 = F::out_n(k1, k2, r);
          const unsigned off = ((unsigned)n1 * inner + l) * 16u;
          const double2 pv = ld32(pe, off);
          if (an.on) {
            const double c = aniso_symbol(an, (double)freq_of(n1, N), (double)freq_of((int)(l / (unsigned)g.H), g.N2),
                                          (double)(l % (unsigned)g.H));
            acc[pi][r].x += c * pv.x;
            acc[pi][r].y += c * pv.y;
          }
          if (masked_out(mk, freq_of(n1, N), freq_of((int)(l / (unsigned)g.H), g.N2), (int)(l % (unsigned)g.H)))
            acc[pi][r] = make_double2(0.0, 0.0);
          st32(qe, off, acc[pi][r]);
          pq += w * (pv.x * acc[pi][r].x + pv.y * acc[pi][r].y);
        }
      }
    }
  }
  const double sum = block_sum(pq, red);
  if (threadIdx.x == 0) part_pq[(long long)e * gridDim.x + blockIdx.x] = sum;
}

// P3: X <- R2C(a . C2R(X)) along axis 3 for the array blockIdx.y (two real
// lines per complex line).  The inverse's last stage leaves the values at
// n = j + A B r (j = k1 + A k2) in registers, the input order of the
// mirrored forward split's stage 1: coefficient and forward stage 1 run on
// the same registers.  A last exchange pairs the entries h and N - h that
// separate the two Hermitian spectra.
template <int A, int B, int C>
__global__ __launch_bounds__(kFftBlock) void k3_axis3(double2* __restrict__ X, const double* __restrict__ acoef, G3 g,
                                                       long long stride, FftDev f, const int* __restrict__ done,
                                                       int done_div) {
  constexpr int N = A * B * C;
  constexpr int T = split_lines(N), H = (N + 1) / 2;
  using FI = Fft3<A, B, C, 1, T, true, kFftBlock>;
  using FF = typename MirrorOf<FI>::type;
  static_assert(FF::A == FI::R && FF::M == A * FI::KL, "mirrored split");
  __shared__ double2 S[T * N];
  __shared__ double2 tw[N];
  const int bi = blockIdx.y;
  if (done != nullptr && done[bi / done_div]) return;
  const unsigned nl = (unsigned)g.N1 * (unsigned)g.N2;
  const unsigned p0 = xcd_tile(blockIdx.x, gridDim.x) * (unsigned)T;
  double2* x = X + bi * stride;
  for (int i = threadIdx.x; i < N; i += kFftBlock) tw[i] = f.tw[i];
  __syncthreads();
  // inverse stage 1: items (pair, j), j fastest
  for (int it = threadIdx.x; it < FI::I1; it += kFftBlock) {
    int tp, j;
    FI::item1(it, tp, j);
    const unsigned la = 2 * (p0 + (unsigned)tp), lb = la + 1;
    double2 v[A];
#pragma unroll
    for (int a = 0; a < A; ++a) {
      const int n = j + FI::M * a;
      const bool cj = n >= H;
      const unsigned m = (unsigned)(cj ? N - n : n);
      double2 xa = la < nl ? ld32(x, (la * (unsigned)H + m) * 16u) : make_double2(0.0, 0.0);
      double2 xb = lb < nl ? ld32(x, (lb * (unsigned)H + m) * 16u) : make_double2(0.0, 0.0);
      if (cj) {
        xa.y = -xa.y;
        xb.y = -xb.y;
      }
      v[a] = make_double2(xa.x - xb.y, xa.y + xb.x);  // Xa + i Xb
    }
    FI::stage1(v, tp, j, S, tw);
  }
  __syncthreads();
  FI::stage2(S, tw);
  __syncthreads();
  // inverse last stage, coefficient, forward stage 1 (held across the barrier)
  double2 hold[FI::PL][FI::R];
#pragma unroll
  for (int pi = 0; pi < FI::PL; ++pi) {
    const int it = threadIdx.x + pi * kFftBlock;
    if (it < FI::IL) {
      int tp, k1, k2;
      FI::itemL(it, tp, k1, k2);
      FI::last(hold[pi], tp, k1, k2, S);
      const unsigned la = 2 * (p0 + (unsigned)tp), lb = la + 1;
#pragma unroll
      for (int r = 0; r < FI::R; ++r) {
        const unsigned n = (unsigned)FI::out_n(k1, k2, r);
        const double aa = la < nl ? ld32(acoef, (la * (unsigned)N + n) * 8u) : 0.0;
        const double ab = lb < nl ? ld32(acoef, (lb * (unsigned)N + n) * 8u) : 0.0;
        hold[pi][r] = make_double2(hold[pi][r].x * aa, hold[pi][r].y * ab);
      }
      FF::stage1_regs(hold[pi], k1 + A * k2, tw);
    }
  }
  __syncthreads();
#pragma unroll
  for (int pi = 0; pi < FI::PL; ++pi) {
    const int it = threadIdx.x + pi * kFftBlock;
    if (it < FI::IL) {
      int tp, k1, k2;
      FI::itemL(it, tp, k1, k2);
      FF::stage1_write(hold[pi], tp, k1 + A * k2, S);
    }
  }
  __syncthreads();
  FF::stage2(S, tw);
  __syncthreads();
  // forward last stage, then natural order in LDS for the separation
  double2 fw[FF::PL][FF::R];
#pragma unroll
  for (int pi = 0; pi < FF::PL; ++pi) {
    const int it = threadIdx.x + pi * kFftBlock;
    if (it < FF::IL) {
      int tp, k1, k2;
      FF::itemL(it, tp, k1, k2);
      FF::last(fw[pi], tp, k1, k2, S);
    }
  }
  __syncthreads();
#pragma unroll
  for (int pi = 0; pi < FF::PL; ++pi) {
    const int it = threadIdx.x + pi * kFftBlock;
    if (it < FF::IL) {
      int tp, k1, k2;
      FF::itemL(it, tp, k1, k2);
#pragma unroll
      for (int r = 0; r < FF::R; ++r) S[tp * N + FF::out_n(k1, k2, r)] = fw[pi][r];
    }
  }
  __syncthreads();
  // separate the two Hermitian spectra and store h in [0, H)
  for (int it = threadIdx.x; it < T * H; it += kFftBlock) {
    const int tp = it / H, h = it - tp * H;
    const unsigned la = 2 * (p0 + (unsigned)tp), lb = la + 1;
    const double2 W1 = S[tp * N + h];
    const double2 W2 = S[tp * N + (h == 0 ? 0 : N - h)];
    const double2 xa = make_double2(0.5 * (W1.x + W2.x), 0.5 * (W1.y - W2.y));
    const double2 dd = make_double2(W1.x - W2.x, W1.y + W2.y);
    const double2 xb = make_double2(0.5 * dd.y, -0.5 * dd.x);
    if (la < nl) st32(x, (la * (unsigned)H + (unsigned)h) * 16u, xa);
    if (lb < nl) st32(x, (lb * (unsigned)H + (unsigned)h) * 16u, xb);
  }
}

// Launchers of the register passes for the lengths of split_of's table
// whose arrays fit 32-bit byte offsets (LRFG_EUNSUPPORTED otherwise).
#define LRFG_SPLIT_CASES(X) X(45) X(75) X(81) X(135) X(225) X(243) X(405) X(625) X(675) X(729)

bool pass_register(int N, const G3& g) {
  return split_of(N).A > 0 && fft_two_level() && g.S * 16 < (1ll << 32) && g.R * 8 < (1ll << 32);
}
int pass_tiles1(const G3& g) { return ceil_div((long long)g.N2 * g.H, split_lines(g.N1)); }
int pass_tiles3(const G3& g) { return ceil_div(((long long)g.N1 * g.N2 + 1) / 2, split_lines(g.N3)); }

int launch3_grad(const double2* src, double2* dst, const G3& g, int alpha0, int nalpha, long long dse,
                 long long dsa, const FftDev& f, const int* done, int nsys, hipStream_t s) {
  const dim3 grid(pass_tiles1(g), nsys);
#define LRFG_G3(NN)                                                                                          \
  case NN:                                                                                                   \
    hipLaunchKernelGGL((k3_grad_axis1<split_of(NN).A, split_of(NN).B, split_of(NN).C>), grid, dim3(kFftBlock), 0, \
                       s, src, dst, g, alpha0, nalpha, dse, dsa, f, done);                                   \
    break;
  switch (g.N1) {
    LRFG_SPLIT_CASES(LRFG_G3)
    default: return LRFG_EUNSUPPORTED;
  }
#undef LRFG_G3
  LRFG_LAUNCHED();
  return LRFG_OK;
}

int launch3_div(const double2* t, double2* q, const double2* p, const G3& g, int alpha0, int nalpha, double inv_vol,
                const FftDev& f, const int* done, double* part, int nsys, hipStream_t s, const Aniso3& an,
                const Mask3& mk) {
  const dim3 grid(pass_tiles1(g), nsys);
#define LRFG_D3(NN)                                                                                          \
  case NN:                                                                                                   \
    hipLaunchKernelGGL((k3_div_axis1<split_of(NN).A, split_of(NN).B, split_of(NN).C>), grid, dim3(kFftBlock), 0, \
                       s, t, q, p, g, alpha0, nalpha, inv_vol, f, done, part, an, mk);                       \
    break;
  switch (g.N1) {
    LRFG_SPLIT_CASES(LRFG_D3)
    default: return LRFG_EUNSUPPORTED;
  }
#undef LRFG_D3
  LRFG_LAUNCHED();
  return LRFG_OK;
}

int launch3_axis3(double2* x, const double* a, const G3& g, long long stride, const FftDev& f, const int* done,
                  int done_div, int narrays, hipStream_t s) {
  const dim3 grid(pass_tiles3(g), narrays);
#define LRFG_A3(NN)                                                                                            \
  case NN:                                                                                                     \
    hipLaunchKernelGGL((k3_axis3<split_of(NN).A, split_of(NN).B, split_of(NN).C>), grid, dim3(kFftBlock), 0, s, x, \
                       a, g, stride, f, done, done_div);                                                       \
    break;
  switch (g.N3) {
    LRFG_SPLIT_CASES(LRFG_A3)
    default: return LRFG_EUNSUPPORTED;
  }
#undef LRFG_A3
  LRFG_LAUNCHED();
  return LRFG_OK;
}

// ---------------------------------------------------------------- CG kernels
struct CgState {
  double rho[2];
  double z0;
  double floor_abs;
  double pq;
  double alpha;
  double res;
  int done;     // 0 running, 1 converged/zero rhs, 2 breakdown
  int iters;
};

__device__ inline void decode(const G3& g, long long s, int& n1, int& n2, int& h) {
  const unsigned su = (unsigned)s, Hu = (unsigned)g.H, N2u = (unsigned)g.N2;
  const unsigned r = su / Hu;
  h = (int)(su - r * Hu);
  const unsigned q = r / N2u;
  n2 = (int)(r - q * N2u);
  n1 = (int)q;
}

// Sum of part[0..n) by one block, same order in every block; result broadcast.
__device__ inline double block_reduce_array(const double* __restrict__ part, int n, double* red,
                                            double* bcast) {
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) v += part[i];
  const double s = block_sum(v, red);
  if (threadIdx.x == 0) *bcast = s;
  __syncthreads();
  return *bcast;
}

// r = b^ = 2 pi i (k.E_e) a^ ; x = 0 ; z = P^-1 r ; p = z ; partial (r,z), (z,z)
__global__ void k_cg_init(const double2* __restrict__ ahat, const double* __restrict__ E3, G3 g,
                          double2* __restrict__ x, double2* __restrict__ r, double2* __restrict__ p,
                          double* __restrict__ part_rz, double* __restrict__ part_zz, Mask3 mk) {
  __shared__ double red[kBlock / 64];
  const int e = blockIdx.y;
  const double* E = E3 + 3 * e;
  double rz = 0.0, zz = 0.0;
  const long long off = (long long)e * g.S;
  for (long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x; s < g.S;
       s += (long long)gridDim.x * blockDim.x) {
    int n1, n2, h;
    decode(g, s, n1, n2, h);
    double k[3];
    kvec(g, n1, n2, h, k);
    const double ke = k[0] * E[0] + k[1] * E[1] + k[2] * E[2];
    const double2 rv = masked_out(mk, (int)k[0], (int)k[1], h) ? make_double2(0.0, 0.0) : cmul_i(ahat[s], 2.0 * kPi * ke);
    const double pi = pinv_of(k);
    const double2 zv = cscale(rv, pi);
    x[off + s] = make_double2(0.0, 0.0);
    r[off + s] = rv;
    p[off + s] = zv;
    const double w = h == 0 ? 1.0 : 2.0;
    rz += w * (rv.x * zv.x + rv.y * zv.y);
    zz += w * (zv.x * zv.x + zv.y * zv.y);
  }
  const double a = block_sum(rz, red);
  const double b = block_sum(zz, red);
  if (threadIdx.x == 0) {
    part_rz[(long long)e * gridDim.x + blockIdx.x] = a;
    part_zz[(long long)e * gridDim.x + blockIdx.x] = b;
  }
}

__global__ void k_cg_init2(CgState* st, int* done, const double* __restrict__ part_rz,
                           const double* __restrict__ part_zz, int nparts,
                           const double* __restrict__ floor_abs) {
  __shared__ double red[kBlock / 64];
  __shared__ double bc;
  const int e = blockIdx.x;
  const double rz = block_reduce_array(part_rz + (long long)e * nparts, nparts, red, &bc);
  const double zz = block_reduce_array(part_zz + (long long)e * nparts, nparts, red, &bc);
  if (threadIdx.x == 0) {
    CgState s;
    s.rho[0] = rz;
    s.rho[1] = 0.0;
    s.z0 = sqrt(zz);
    s.floor_abs = floor_abs[e];
    s.pq = 0.0;
    s.alpha = 0.0;
    s.res = 1.0;
    s.iters = 0;
    s.done = (s.z0 <= s.floor_abs) ? 1 : 0;
    st[e] = s;
    done[e] = s.done;
  }
}

// x += alpha p ; r -= alpha q ; partial (r, P^-1 r), (P^-1 r, P^-1 r)
__global__ void k_cg_update1(CgState* st, int* done, G3 g, int it, const double* __restrict__ part_pq,
                             int npq, double2* __restrict__ x, double2* __restrict__ r,
                             const double2* __restrict__ p, const double2* __restrict__ q,
                             double* __restrict__ part_rz, double* __restrict__ part_zz) {
  __shared__ double red[kBlock / 64];
  __shared__ double bc;
  const int e = blockIdx.y;
  if (done[e]) return;
  const double pq = block_reduce_array(part_pq + (long long)e * npq, npq, red, &bc);
  const double rho = st[e].rho[it & 1];
  const double alpha = rho / pq;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st[e].pq = pq;
    st[e].alpha = alpha;
  }
  const long long off = (long long)e * g.S;
  double rz = 0.0, zz = 0.0;
  for (long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x; s < g.S;
       s += (long long)gridDim.x * blockDim.x) {
    int n1, n2, h;
    decode(g, s, n1, n2, h);
    double k[3];
    kvec(g, n1, n2, h, k);
    const double2 pv = p[off + s], qv = q[off + s];
    double2 xv = x[off + s], rv = r[off + s];
    xv.x += alpha * pv.x;
    xv.y += alpha * pv.y;
    rv.x -= alpha * qv.x;
    rv.y -= alpha * qv.y;
    x[off + s] = xv;
    r[off + s] = rv;
    const double2 zv = cscale(rv, pinv_of(k));
    const double w = h == 0 ? 1.0 : 2.0;
    rz += w * (rv.x * zv.x + rv.y * zv.y);
    zz += w * (zv.x * zv.x + zv.y * zv.y);
  }
  const double a = block_sum(rz, red);
  const double b = block_sum(zz, red);
  if (threadIdx.x == 0) {
    part_rz[(long long)e * gridDim.x + blockIdx.x] = a;
    part_zz[(long long)e * gridDim.x + blockIdx.x] = b;
  }
}

// p = P^-1 r + beta p ; convergence test ; residual history
__global__ void k_cg_update2(CgState* st, int* done, G3 g, int it, const double* __restrict__ part_rz,
                             const double* __restrict__ part_zz, int nparts, const double2* __restrict__ r,
                             double2* __restrict__ p, double tol, double* __restrict__ hist,
                             int max_iter) {
  __shared__ double red[kBlock / 64];
  __shared__ double bc;
  const int e = blockIdx.y;
  if (done[e]) return;
  const double rz = block_reduce_array(part_rz + (long long)e * nparts, nparts, red, &bc);
  const double zz = block_reduce_array(part_zz + (long long)e * nparts, nparts, red, &bc);
  const double rho = st[e].rho[it & 1];
  const double beta = rz / rho;
  const long long off = (long long)e * g.S;
  for (long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x; s < g.S;
       s += (long long)gridDim.x * blockDim.x) {
    int n1, n2, h;
    decode(g, s, n1, n2, h);
    double k[3];
    kvec(g, n1, n2, h, k);
    const double2 zv = cscale(r[off + s], pinv_of(k));
    double2 pv = p[off + s];
    pv.x = zv.x + beta * pv.x;
    pv.y = zv.y + beta * pv.y;
    p[off + s] = pv;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const double zn = sqrt(zz);
    const double res = zn / st[e].z0;
    st[e].rho[(it + 1) & 1] = rz;
    st[e].res = res;
    st[e].iters = it + 1;
    if (hist != nullptr && it < max_iter) hist[(long long)e * max_iter + it] = res;
    if (!(st[e].pq > 0.0)) done[e] = 2;
    else if (res <= tol || zn <= st[e].floor_abs) done[e] = 1;
  }
}

// Partial sums of a and a^2 over the real grid.
__global__ void k_coef_stats(const double* __restrict__ a, long long n, double* __restrict__ part,
                             int* __restrict__ bad) {
  __shared__ double red[kBlock / 64];
  double s1 = 0.0, s2 = 0.0;
  int nb = 0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const double v = a[i];
    if (!(v > 0.0) || !isfinite(v)) nb = 1;
    s1 += v;
    s2 += v * v;
  }
  if (nb) atomicOr(bad, 1);
  const double x = block_sum(s1, red);
  const double y = block_sum(s2, red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = x;
    part[2 * blockIdx.x + 1] = y;
  }
}

// Per-block partial sums for A_H at one alpha: sum a g_e (nE values) and
// sum a g_i g_j (i <= j), real fields g_e at g + e*gstride.
__global__ void k_ah_reduce(const double* __restrict__ a, const double* __restrict__ gf,
                            long long gstride, int nE, long long n, double* __restrict__ part) {
  __shared__ double red[kBlock / 64];
  const int nv = nE + nE * (nE + 1) / 2;
  double acc[3 + 6];
  for (int v = 0; v < nv; ++v) acc[v] = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const double av = a[i];
    double gv[3];
    for (int e = 0; e < nE; ++e) gv[e] = gf[e * gstride + i];
    int v = 0;
    for (int e = 0; e < nE; ++e) acc[v++] += av * gv[e];
    for (int ii = 0; ii < nE; ++ii)
      for (int jj = ii; jj < nE; ++jj) acc[v++] += av * gv[ii] * gv[jj];
  }
  for (int v = 0; v < nv; ++v) {
    const double s = block_sum(acc[v], red);
    if (threadIdx.x == 0) part[(long long)blockIdx.x * nv + v] = s;
  }
}

// Ga's coefficient on the double grid (Sec. 2.2.3): the half spectrum
// C(m) = A^(m) prod_i exp(-pi i m_i (M_i - 1)/M_i), A^(m) the exact Fourier
// integral of the inclusion coefficient (value vin inside, vout outside):
// square/cube |x_i| < size: (vin - vout) prod_i s(m_i) + vout delta_m0 with
// s(0) = 2 size, s(m) = sin(2 pi m size)/(pi m); ball |x| < size:
// (vin - vout)(sin z - z cos z)/(2 pi^2 rho^3) + vout delta_m0, z = 2 pi size rho
// (4 pi size^3 / 3 at rho = 0).  The phase places the unnormalised inverse DFT
// at the points x_j = -1/2 + (j + 1/2)/M.  d = 2 uses axes 1 and 2.
__global__ void k_incl_spectrum(double2* __restrict__ out, G3 g, int d, int shape, double size, double vin,
                                double vout, Mask3 trunc) {
  for (long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x; s < g.S;
       s += (long long)gridDim.x * blockDim.x) {
    int n1, n2, h;
    decode(g, s, n1, n2, h);
    double k[3];
    kvec(g, n1, n2, h, k);
    const int Ms[3] = {g.N1, g.N2, g.N3};
    double chi;
    if (shape == 1) {
      chi = 1.0;
      for (int a = 3 - d; a < 3; ++a)
        chi *= k[a] == 0.0 ? 2.0 * size : sin(2.0 * kPi * k[a] * size) / (kPi * k[a]);
    } else {
      const double rho = sqrt(k[0] * k[0] + k[1] * k[1] + k[2] * k[2]);
      if (rho == 0.0) {
        chi = 4.0 * kPi * size * size * size / 3.0;
      } else {
        const double z = 2.0 * kPi * size * rho;
        chi = (sin(z) - z * cos(z)) / (2.0 * kPi * kPi * rho * rho * rho);
      }
    }
    double v = (vin - vout) * chi;
    if (k[0] == 0.0 && k[1] == 0.0 && k[2] == 0.0) v += vout;
    // the series stops at |m_i| <= N_i - 1 (a double grid above 2N - 1 holds more)
    if (fabs(k[0]) > trunc.k0 || fabs(k[1]) > trunc.k1 || fabs(k[2]) > trunc.k2) v = 0.0;
    double ph = 0.0;
    for (int a = 0; a < 3; ++a) ph -= kPi * k[a] * (double)(Ms[a] - 1) / (double)Ms[a];
    out[s] = make_double2(v * cos(ph), v * sin(ph));
  }
}

// Per-block partial sums of sum_k w 4 pi^2 k.Bk Re(x^_i conj x^_j), i <= j,
// over the half spectrum (w = 1 on h = 0, else 2): the B share of A_H
// (the Fourier coefficients carry the grid mean's normalisation).
__global__ void k_aniso_energy(const double2* __restrict__ x, G3 g, int nE, Aniso3 an,
                               double* __restrict__ part) {
  __shared__ double red[kBlock / 64];
  const int nv = nE * (nE + 1) / 2;
  double acc[6];
  for (int v = 0; v < nv; ++v) acc[v] = 0.0;
  for (long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x; s < g.S;
       s += (long long)gridDim.x * blockDim.x) {
    int n1, n2, h;
    decode(g, s, n1, n2, h);
    const double c = (h == 0 ? 1.0 : 2.0) *
                     aniso_symbol(an, (double)freq_of(n1, g.N1), (double)freq_of(n2, g.N2), (double)h);
    double2 xv[3];
    for (int e = 0; e < nE; ++e) xv[e] = x[(long long)e * g.S + s];
    int v = 0;
    for (int i = 0; i < nE; ++i)
      for (int j = i; j < nE; ++j) acc[v++] += c * (xv[i].x * xv[j].x + xv[i].y * xv[j].y);
  }
  for (int v = 0; v < nv; ++v) {
    const double t = block_sum(acc[v], red);
    if (threadIdx.x == 0) part[(long long)blockIdx.x * nv + v] = t;
  }
}

}  // namespace

// ====================================================================== host
struct FullLayout {
  G3 g;
  int nE;
  double2 *tw1, *tw2, *tw3;
  double* a;       // real coefficient
  double2 *x, *r, *p, *q, *t;
  double* part_pq;
  double* part_rz;
  double* part_zz;
  double* part_misc;
  double* floor_abs;
  double* E3;
  CgState* st;
  int* done;
  int* bad;
  double* hist;
  int grid_vec;   // blocks of the vector kernels
  int tiles1;     // axis-1 tiles of the Stockham kernels
  int tdiv;       // blocks of the divergence pass in use (partial sums of (p, q))
  int T1, T3;
  int nstat;      // blocks of coef stats / ah reduce
};

static int tile1_lines(int N1) { return lines_per_tile1(N1); }

static G3 make_g3(const int N[3]) {
  G3 g;
  g.N1 = N[0];
  g.N2 = N[1];
  g.N3 = N[2];
  g.H = (N[2] + 1) / 2;
  g.S = (long long)g.N1 * g.N2 * g.H;
  g.R = (long long)g.N1 * g.N2 * g.N3;
  return g;
}

static void carve(Arena& ar, FullLayout& L, const int N3d[3], int nE, int d, int max_iter) {
  L.g = make_g3(N3d);
  L.nE = nE;
  const G3& g = L.g;
  L.T1 = tile1_lines(g.N1);
  L.T3 = lines_per_tile1(g.N3);
  L.tiles1 = ceil_div((long long)g.N2 * g.H, L.T1);
  L.tdiv = pass_register(g.N1, g) ? pass_tiles1(g) : L.tiles1;
  long long gv = ceil_div(g.S, kBlock * 4);
  if (gv > 1024) gv = 1024;
  if (gv < 1) gv = 1;
  L.grid_vec = (int)gv;
  long long gs = ceil_div(g.R, kBlock * 8);
  if (gs > 1024) gs = 1024;
  if (gs < 1) gs = 1;
  L.nstat = (int)gs;
  L.tw1 = ar.take<double2>(g.N1);
  L.tw2 = ar.take<double2>(g.N2);
  L.tw3 = ar.take<double2>(g.N3);
  L.a = ar.take<double>(g.R);
  L.x = ar.take<double2>(g.S * nE);
  L.r = ar.take<double2>(g.S * nE);
  L.p = ar.take<double2>(g.S * nE);
  L.q = ar.take<double2>(g.S * nE);
  L.t = ar.take<double2>(g.S * nE * d);
  L.part_pq = ar.take<double>((size_t)std::max(L.tiles1, L.tdiv) * nE);
  L.part_rz = ar.take<double>((size_t)L.grid_vec * nE);
  L.part_zz = ar.take<double>((size_t)L.grid_vec * nE);
  L.part_misc = ar.take<double>((size_t)L.nstat * 9 + 16);
  L.floor_abs = ar.take<double>(nE);
  L.E3 = ar.take<double>(3 * nE);
  L.st = ar.take<CgState>(nE);
  L.done = ar.take<int>(nE);
  L.bad = ar.take<int>(4);
  L.hist = ar.take<double>((size_t)nE * max_iter);
}

size_t full_workspace_bytes(const int N3d[3], int nE, int d, int max_iter) {
  Arena ar;
  FullLayout L;
  carve(ar, L, N3d, nE, d, max_iter);
  return ar.used + 256;
}

int full_solve(const FullSolveArgs& A, FullSolveOut* out) {
  hipStream_t s = static_cast<hipStream_t>(A.stream);
  const int d = A.d;
  const int nE = A.nE;
  // internal 3-D geometry: d = 2 is stored with a unit first axis
  int N3d[3];
  if (d == 3) {
    N3d[0] = A.N[0];
    N3d[1] = A.N[1];
    N3d[2] = A.N[2];
  } else {
    N3d[0] = 1;
    N3d[1] = A.N[0];
    N3d[2] = A.N[1];
  }
  const int alpha0 = 3 - d;
  if ((long long)N3d[0] * N3d[1] * N3d[2] > kMaxGridEntries) {
    set_error("full-grid solve: %d x %d x %d grid above 2^32 - 1 entries", N3d[0], N3d[1], N3d[2]);
    return LRFG_EUNSUPPORTED;
  }
  // B embedded in the internal axes (d = 2: axes 1 and 2), times 4 pi^2
  Aniso3 an{};
  {
    double B3[3][3] = {};
    for (int i = 0; i < d; ++i)
      for (int j = 0; j < d; ++j) {
        B3[alpha0 + i][alpha0 + j] = A.B[i * d + j];
        if (A.B[i * d + j] != 0.0) an.on = 1;
      }
    const double f = 4.0 * kPi * kPi;
    an.b00 = f * B3[0][0];
    an.b11 = f * B3[1][1];
    an.b22 = f * B3[2][2];
    an.b01 = f * 0.5 * (B3[0][1] + B3[1][0]);
    an.b02 = f * 0.5 * (B3[0][2] + B3[2][0]);
    an.b12 = f * 0.5 * (B3[1][2] + B3[2][1]);
  }
  // Ga: the N-frequencies in the internal axes (d = 2: axes 1 and 2)
  const bool ga = A.ga_N[0] > 0;
  Mask3 mk{0, 0, 0, 0};
  if (ga) {
    int lim[3] = {0, 0, 0};
    for (int i = 0; i < d; ++i) lim[alpha0 + i] = (A.ga_N[i] - 1) / 2;
    mk = Mask3{lim[0], lim[1], lim[2], 1};
  }
  Arena ar;
  ar.base = static_cast<char*>(A.ws);
  ar.cap = A.ws_bytes;
  FullLayout L;
  carve(ar, L, N3d, nE, d, A.max_iter);
  if (ar.overflow) {
    set_error("workspace too small: need %zu bytes, have %zu", ar.used, A.ws_bytes);
    return LRFG_EWORKSPACE;
  }
  const G3 g = L.g;
  ScopedEvents<3> evs3;
  LRFG_TRY(evs3.create());
  hipEvent_t &ev0 = evs3[0], &ev1 = evs3[1], &ev2 = evs3[2];
  LRFG_HIP(hipEventRecord(ev0, s));

  FftDev f1, f2, f3;
  LRFG_TRY(fft_dev_upload(*A.plan1, L.tw1, s, &f1));
  LRFG_TRY(fft_dev_upload(*A.plan2, L.tw2, s, &f2));
  LRFG_TRY(fft_dev_upload(*A.plan3, L.tw3, s, &f3));
  const bool G1 = plan_generic(f1), G3 = plan_generic(f3);
  const bool two1 = pass_register(g.N1, g), two3 = pass_register(g.N3, g);

  // coefficient
  if (ga) {
    // the inclusion's Fourier integrals on the double grid, then the
    // unnormalised inverse transform (axes 1 and 2, C2R along axis 3) to its
    // nodal values; q[0] is free until the first matvec
    int lim[3] = {0, 0, 0};
    for (int i = 0; i < d; ++i) lim[alpha0 + i] = A.ga_N[i] - 1;
    hipLaunchKernelGGL(k_incl_spectrum, dim3(L.grid_vec), dim3(kBlock), 0, s, L.q, g, d, A.incl, A.incl_size,
                       A.incl_in, A.incl_out, Mask3{lim[0], lim[1], lim[2], 1});
    LRFG_LAUNCHED();
    LRFG_TRY(launch_fft_lines(L.q, 1, g.N1, (long long)g.N2 * g.H, 1, f1, 1.0, s));
    LRFG_TRY(launch_fft_lines(L.q, g.N1, g.N2, g.H, 1, f2, 1.0, s));
    {
      const size_t shm3c = size_t(L.T3 + 1) * g.N3 * sizeof(double2);
      const int tiles3c = ceil_div(((long long)g.N1 * g.N2 + 1) / 2, L.T3);
      hipLaunchKernelGGL((G3 ? k_axis3<2, true> : k_axis3<2, false>), dim3(tiles3c, 1), dim3(kBlock), shm3c, s,
                         (const void*)L.q, (void*)L.a, (const double*)nullptr, g, g.S, 0LL, L.T3, f3, 1.0,
                         (const int*)nullptr, 1);
      LRFG_LAUNCHED();
    }
  } else if (A.a_on_device) {
    LRFG_HIP(hipMemcpyAsync(L.a, A.a, sizeof(double) * g.R, hipMemcpyDeviceToDevice, s));
  } else {
    LRFG_HIP(hipMemcpyAsync(L.a, A.a, sizeof(double) * g.R, hipMemcpyHostToDevice, s));
  }
  // E embedded in 3-D
  std::vector<double> E3(3 * nE, 0.0);
  for (int e = 0; e < nE; ++e)
    for (int al = 0; al < d; ++al) E3[3 * e + alpha0 + al] = A.E[e * d + al];
  LRFG_HIP(hipMemcpyAsync(L.E3, E3.data(), sizeof(double) * 3 * nE, hipMemcpyHostToDevice, s));
  LRFG_HIP(hipMemsetAsync(L.bad, 0, sizeof(int) * 4, s));
  LRFG_HIP(hipMemsetAsync(L.done, 0, sizeof(int) * nE, s));
  if (A.max_iter > 0)
    LRFG_HIP(hipMemsetAsync(L.hist, 0, sizeof(double) * nE * A.max_iter, s));

  hipLaunchKernelGGL(k_coef_stats, dim3(L.nstat), dim3(kBlock), 0, s, L.a, g.R, L.part_misc, L.bad);
  LRFG_LAUNCHED();
  std::vector<double> stat(2 * L.nstat);
  int bad = 0;
  LRFG_HIP(hipMemcpyAsync(stat.data(), L.part_misc, sizeof(double) * 2 * L.nstat, hipMemcpyDeviceToHost, s));
  LRFG_HIP(hipMemcpyAsync(&bad, L.bad, sizeof(int), hipMemcpyDeviceToHost, s));
  LRFG_HIP(hipStreamSynchronize(s));
  // Ga's double-grid coefficient is a truncated Fourier series: it may dip
  // below zero near the inclusion's boundary while the bilinear form (the
  // integral of the true coefficient) stays positive
  if (bad && !ga) {
    set_error("coefficient must be finite and positive");
    return LRFG_ECOEFF;
  }
  double sum_a = 0.0, sum_a2 = 0.0;
  for (int i = 0; i < L.nstat; ++i) {
    sum_a += stat[2 * i];
    sum_a2 += stat[2 * i + 1];
  }
  const double mean_a = sum_a / (double)g.R;
  const double rms_a = std::sqrt(sum_a2 / (double)g.R);
  std::vector<double> floors(nE);
  for (int e = 0; e < nE; ++e) {
    double en = 0.0;
    for (int al = 0; al < d; ++al) en += A.E[e * d + al] * A.E[e * d + al];
    floors[e] = 1e-14 * rms_a * std::sqrt(en);
  }
  LRFG_HIP(hipMemcpyAsync(L.floor_abs, floors.data(), sizeof(double) * nE, hipMemcpyHostToDevice, s));

  const size_t shm1 = size_t(L.T1 + 1) * g.N1 * sizeof(double2);
  const size_t shm3 = size_t(L.T3 + 1) * g.N3 * sizeof(double2);
  const long long pairs = ((long long)g.N1 * g.N2 + 1) / 2;
  const int tiles3 = ceil_div(pairs, L.T3);
  const double inv_vol = 1.0 / (double)g.R;

  // a^ = F(a): R2C along axis 3, then axes 2 and 1 (scale 1/|N| at the end).
  double2* ahat = L.q;  // q[0] is free until the first matvec
  hipLaunchKernelGGL((G3 ? k_axis3<1, true> : k_axis3<1, false>), dim3(tiles3, 1), dim3(kBlock), shm3, s, (const void*)L.a, (void*)ahat,
                     (const double*)nullptr, g, 0LL, 0LL, L.T3, f3, 1.0, (const int*)nullptr, 1);
  LRFG_LAUNCHED();
  LRFG_TRY(launch_fft_lines(ahat, g.N1, g.N2, g.H, -1, f2, 1.0, s));
  LRFG_TRY(launch_fft_lines(ahat, 1, g.N1, (long long)g.N2 * g.H, -1, f1, inv_vol, s));

  hipLaunchKernelGGL(k_cg_init, dim3(L.grid_vec, nE), dim3(kBlock), 0, s, (const double2*)ahat,
                     (const double*)L.E3, g, L.x, L.r, L.p, L.part_rz, L.part_zz, mk);
  LRFG_LAUNCHED();
  hipLaunchKernelGGL(k_cg_init2, dim3(nE), dim3(kBlock), 0, s, L.st, L.done, (const double*)L.part_rz,
                     (const double*)L.part_zz, L.grid_vec, (const double*)L.floor_abs);
  LRFG_LAUNCHED();
  LRFG_HIP(hipEventRecord(ev1, s));

  // ------------------------------------------------------------ PCG loop
  const int ring = 4;
  int* pinned = A.pinned_flags;  // ring * nE ints, pinned host memory from the plan
  ScopedEvents<4> evs;
  LRFG_TRY(evs.create(hipEventDisableTiming));
  int it = 0;
  bool all_done = false;
  int checked = -1;
  for (it = 0; it < A.max_iter; ++it) {
    if (it > 0 && it % 4 == 0) gate_point();  // between blocks of 4 iterations (the flag ring's depth)
    // P1
    {
      ProfScope ps_("grad_axis1", s);
      if (two1) {
        LRFG_TRY(launch3_grad((const double2*)L.p, L.t, g, alpha0, d, (long long)d * g.S, g.S, f1,
                              (const int*)L.done, nE, s));
      } else {
        hipLaunchKernelGGL((G1 ? k_grad_axis1<true> : k_grad_axis1<false>), dim3(L.tiles1 * d, nE), dim3(kBlock), shm1,
                           s, (const double2*)L.p, L.t, g, alpha0, d, (long long)d * g.S, g.S, L.T1, f1,
                           (const int*)L.done);
        LRFG_LAUNCHED();
      }
    }
    // P2
    LRFG_TRY(launch_fft_lines(L.t, (long long)nE * d * g.N1, g.N2, g.H, 1, f2, 1.0, s, "fft_axis2",
                              L.done, (long long)d * g.N1 * g.H));
    // P3
    {
      ProfScope ps_("axis3", s);
      if (two3) {
        LRFG_TRY(launch3_axis3(L.t, (const double*)L.a, g, g.S, f3, (const int*)L.done, d, nE * d, s));
      } else {
        hipLaunchKernelGGL((G3 ? k_axis3<0, true> : k_axis3<0, false>), dim3(tiles3, nE * d), dim3(kBlock), shm3, s,
                           (const void*)L.t, (void*)nullptr, (const double*)L.a, g, g.S, 0LL, L.T3, f3, 1.0,
                           (const int*)L.done, d);
        LRFG_LAUNCHED();
      }
    }
    // P4
    LRFG_TRY(launch_fft_lines(L.t, (long long)nE * d * g.N1, g.N2, g.H, -1, f2, 1.0, s, "fft_axis2",
                              L.done, (long long)d * g.N1 * g.H));
    // P5
    {
      ProfScope ps_("div_axis1", s);
      if (two1) {
        LRFG_TRY(launch3_div((const double2*)L.t, L.q, (const double2*)L.p, g, alpha0, d, inv_vol, f1,
                             (const int*)L.done, L.part_pq, nE, s, an, mk));
      } else {
        hipLaunchKernelGGL((G1 ? k_div_axis1<true> : k_div_axis1<false>), dim3(L.tiles1, nE), dim3(kBlock), shm1, s,
                           (const double2*)L.t, L.q, (const double2*)L.p, g, alpha0, d, inv_vol, L.T1, f1,
                           (const int*)L.done, L.part_pq, an, mk);
        LRFG_LAUNCHED();
      }
    }
    {
      ProfScope ps_("cg_update1", s);
      hipLaunchKernelGGL(k_cg_update1, dim3(L.grid_vec, nE), dim3(kBlock), 0, s, L.st, L.done, g, it,
                         (const double*)L.part_pq, L.tdiv, L.x, L.r, (const double2*)L.p,
                         (const double2*)L.q, L.part_rz, L.part_zz);
    }
    LRFG_LAUNCHED();
    {
      ProfScope ps_("cg_update2", s);
      hipLaunchKernelGGL(k_cg_update2, dim3(L.grid_vec, nE), dim3(kBlock), 0, s, L.st, L.done, g, it,
                         (const double*)L.part_rz, (const double*)L.part_zz, L.grid_vec,
                         (const double2*)L.r, L.p, A.tol, L.hist, A.max_iter);
    }
    LRFG_LAUNCHED();
    LRFG_HIP(hipMemcpyAsync(pinned + (it % ring) * nE, L.done, sizeof(int) * nE, hipMemcpyDeviceToHost, s));
    LRFG_HIP(hipEventRecord(evs[it % ring], s));
    // look at the flags of an earlier iteration while this one runs
    const int look = it - (ring - 1);
    if (look >= 0) {
      LRFG_HIP(hipEventSynchronize(evs[look % ring]));
      checked = look;
      bool ad = true;
      for (int e = 0; e < nE; ++e) ad = ad && (pinned[(look % ring) * nE + e] != 0);
      if (ad) {
        all_done = true;
        ++it;
        break;
      }
    }
  }
  (void)checked;
  (void)all_done;
  LRFG_HIP(hipStreamSynchronize(s));

  // ------------------------------------------------------------ A_H
  // For each alpha: g_{e,alpha} = F^-1(2 pi i k_alpha x_e) into the q buffers
  // (real layout), then partial sums of a g and a g g.
  const int nv = nE + nE * (nE + 1) / 2;
  std::vector<double> m1(nE * d, 0.0), m2((size_t)nE * nE * d, 0.0);
  std::vector<double> part((size_t)L.nstat * nv);
  for (int al = 0; al < d; ++al) {
    hipLaunchKernelGGL((G1 ? k_grad_axis1<true> : k_grad_axis1<false>), dim3(L.tiles1, nE), dim3(kBlock), shm1, s, (const double2*)L.x, L.t, g,
                       alpha0 + al, 1, g.S, 0LL, L.T1, f1, (const int*)nullptr);
    LRFG_LAUNCHED();
    LRFG_TRY(launch_fft_lines(L.t, (long long)nE * g.N1, g.N2, g.H, 1, f2, 1.0, s));
    hipLaunchKernelGGL((G3 ? k_axis3<2, true> : k_axis3<2, false>), dim3(tiles3, nE), dim3(kBlock), shm3, s, (const void*)L.t, (void*)L.q,
                       (const double*)nullptr, g, g.S, 2 * g.S, L.T3, f3, 1.0, (const int*)nullptr, 1);
    LRFG_LAUNCHED();
    hipLaunchKernelGGL(k_ah_reduce, dim3(L.nstat), dim3(kBlock), 0, s, (const double*)L.a,
                       (const double*)L.q, 2 * g.S, nE, g.R, L.part_misc);
    LRFG_LAUNCHED();
    LRFG_HIP(hipMemcpyAsync(part.data(), L.part_misc, sizeof(double) * L.nstat * nv, hipMemcpyDeviceToHost, s));
    LRFG_HIP(hipStreamSynchronize(s));
    std::vector<double> acc(nv, 0.0);
    for (int b = 0; b < L.nstat; ++b)
      for (int v = 0; v < nv; ++v) acc[v] += part[(size_t)b * nv + v];
    int v = 0;
    for (int e = 0; e < nE; ++e) m1[e * d + al] = acc[v++] / (double)g.R;
    for (int i = 0; i < nE; ++i)
      for (int j = i; j < nE; ++j) {
        const double val = acc[v++] / (double)g.R;
        m2[((size_t)i * nE + j) * d + al] = val;
        m2[((size_t)j * nE + i) * d + al] = val;
      }
  }
  // B share of A_H: E_i.B E_j + mean_x B grad u_i . grad u_j
  std::vector<double> mb((size_t)nE * nE, 0.0);
  if (an.on) {
    const int nb = nE * (nE + 1) / 2;
    hipLaunchKernelGGL(k_aniso_energy, dim3(L.nstat), dim3(kBlock), 0, s, (const double2*)L.x, g, nE, an,
                       L.part_misc);
    LRFG_LAUNCHED();
    std::vector<double> pb((size_t)L.nstat * nb);
    LRFG_HIP(hipMemcpyAsync(pb.data(), L.part_misc, sizeof(double) * L.nstat * nb, hipMemcpyDeviceToHost, s));
    LRFG_HIP(hipStreamSynchronize(s));
    std::vector<double> acc(nb, 0.0);
    for (int b = 0; b < L.nstat; ++b)
      for (int v = 0; v < nb; ++v) acc[v] += pb[(size_t)b * nb + v];
    int v = 0;
    for (int i = 0; i < nE; ++i)
      for (int j = i; j < nE; ++j) {
        double eb = 0.0;
        for (int al = 0; al < d; ++al)
          for (int be = 0; be < d; ++be) eb += A.E[i * d + al] * A.B[al * d + be] * A.E[j * d + be];
        mb[(size_t)i * nE + j] = mb[(size_t)j * nE + i] = eb + acc[v++];
      }
  }
  LRFG_HIP(hipEventRecord(ev2, s));
  std::vector<CgState> st(nE);
  LRFG_HIP(hipMemcpyAsync(st.data(), L.st, sizeof(CgState) * nE, hipMemcpyDeviceToHost, s));
  std::vector<double> hist((size_t)nE * A.max_iter);
  if (A.max_iter > 0)
    LRFG_HIP(hipMemcpyAsync(hist.data(), L.hist, sizeof(double) * nE * A.max_iter, hipMemcpyDeviceToHost, s));
  std::vector<int> dn(nE);
  LRFG_HIP(hipMemcpyAsync(dn.data(), L.done, sizeof(int) * nE, hipMemcpyDeviceToHost, s));
  LRFG_HIP(hipStreamSynchronize(s));
  float ms_setup = 0.f, ms_solve = 0.f;
  LRFG_HIP(hipEventElapsedTime(&ms_setup, ev0, ev1));
  LRFG_HIP(hipEventElapsedTime(&ms_solve, ev1, ev2));

  // A_H[i][j] = mean(a) E_i.E_j + sum_alpha (E_i,alpha m1[j] + E_j,alpha m1[i] + m2[i][j])
  int rc = LRFG_OK;
  for (int i = 0; i < nE; ++i) {
    for (int j = 0; j < nE; ++j) {
      double v = mb[(size_t)i * nE + j];
      for (int al = 0; al < d; ++al) {
        const double ei = A.E[i * d + al], ej = A.E[j * d + al];
        v += mean_a * ei * ej + ei * m1[j * d + al] + ej * m1[i * d + al] + m2[((size_t)i * nE + j) * d + al];
      }
      if (out->A_H) out->A_H[i * nE + j] = v;
    }
    const int its = dn[i] == 0 ? A.max_iter : st[i].iters;
    if (out->iters) out->iters[i] = its;
    int stc = LRFG_OK;
    if (dn[i] == 0) stc = LRFG_NOT_CONVERGED;
    if (dn[i] == 2) stc = LRFG_NOT_CONVERGED;
    if (out->status) out->status[i] = stc;
    if (stc != LRFG_OK) rc = LRFG_NOT_CONVERGED;
    if (out->res_hist)
      for (int k = 0; k < A.max_iter; ++k) out->res_hist[(size_t)i * A.max_iter + k] = hist[(size_t)i * A.max_iter + k];
  }
  out->setup_ms = ms_setup;
  out->solve_ms = ms_solve;
  return rc;
}

// ------------------------------------------------------------ op-level entry
size_t full_op_workspace_bytes(const int N[3]) {
  Arena ar;
  G3 g = make_g3(N);
  ar.take<double2>(g.N1);
  ar.take<double2>(g.N2);
  ar.take<double2>(g.N3);
  ar.take<double2>(g.S * 3);
  ar.take<double>(ceil_div((long long)g.N2 * g.H, 1) + 16);
  ar.take<int>(4);
  return ar.used + 256;
}

int full_op(int which, const int N[3], const FftPlan* p1, const FftPlan* p2, const FftPlan* p3,
            const double* a, const double* u, double* outp, void* ws, size_t ws_bytes, hipStream_t s) {
  G3 g = make_g3(N);
  if (g.R > kMaxGridEntries) {
    set_error("full-grid operator: grid above 2^32 - 1 entries");
    return LRFG_EUNSUPPORTED;
  }
  Arena ar;
  ar.base = static_cast<char*>(ws);
  ar.cap = ws_bytes;
  double2* tw1 = ar.take<double2>(g.N1);
  double2* tw2 = ar.take<double2>(g.N2);
  double2* tw3 = ar.take<double2>(g.N3);
  double2* t = ar.take<double2>(g.S * 3);
  double* part = ar.take<double>(ceil_div((long long)g.N2 * g.H, 1) + 16);
  int* done = ar.take<int>(4);
  if (ar.overflow) {
    set_error("workspace too small");
    return LRFG_EWORKSPACE;
  }
  const double2* uh = reinterpret_cast<const double2*>(u);
  double2* oh = reinterpret_cast<double2*>(outp);
  if (which == 1) return launch_pinv(uh, oh, g.N1, g.N2, g.N3, s);
  FftDev f1, f2, f3;
  LRFG_TRY(fft_dev_upload(*p1, tw1, s, &f1));
  LRFG_TRY(fft_dev_upload(*p2, tw2, s, &f2));
  LRFG_TRY(fft_dev_upload(*p3, tw3, s, &f3));
  const bool G1 = plan_generic(f1), G3 = plan_generic(f3);
  LRFG_HIP(hipMemsetAsync(done, 0, sizeof(int) * 4, s));
  const int T1 = tile1_lines(g.N1);
  const int T3 = lines_per_tile1(g.N3);
  const int tiles1 = ceil_div((long long)g.N2 * g.H, T1);
  const size_t shm1 = size_t(T1 + 1) * g.N1 * sizeof(double2);
  const size_t shm3 = size_t(T3 + 1) * g.N3 * sizeof(double2);
  const long long pairs = ((long long)g.N1 * g.N2 + 1) / 2;
  const int tiles3 = ceil_div(pairs, T3);
  const bool two1 = pass_register(g.N1, g), two3 = pass_register(g.N3, g);
  if (two1) {
    LRFG_TRY(launch3_grad(uh, t, g, 0, 3, 3 * g.S, g.S, f1, (const int*)done, 1, s));
  } else {
    hipLaunchKernelGGL((G1 ? k_grad_axis1<true> : k_grad_axis1<false>), dim3(tiles1 * 3, 1), dim3(kBlock), shm1, s, uh,
                       t, g, 0, 3, 3 * g.S, g.S, T1, f1, (const int*)done);
    LRFG_LAUNCHED();
  }
  LRFG_TRY(launch_fft_lines(t, 3LL * g.N1, g.N2, g.H, 1, f2, 1.0, s));
  if (two3) {
    LRFG_TRY(launch3_axis3(t, a, g, g.S, f3, (const int*)done, 3, 3, s));
  } else {
    hipLaunchKernelGGL((G3 ? k_axis3<0, true> : k_axis3<0, false>), dim3(tiles3, 3), dim3(kBlock), shm3, s,
                       (const void*)t, (void*)nullptr, a, g, g.S, 0LL, T3, f3, 1.0, (const int*)done, 3);
    LRFG_LAUNCHED();
  }
  LRFG_TRY(launch_fft_lines(t, 3LL * g.N1, g.N2, g.H, -1, f2, 1.0, s));
  if (two1) {
    LRFG_TRY(launch3_div((const double2*)t, oh, uh, g, 0, 3, 1.0 / (double)g.R, f1, (const int*)done, part, 1, s,
                         Aniso3{}, Mask3{}));
  } else {
    hipLaunchKernelGGL((G1 ? k_div_axis1<true> : k_div_axis1<false>), dim3(tiles1, 1), dim3(kBlock), shm1, s,
                       (const double2*)t, oh, uh, g, 0, 3, 1.0 / (double)g.R, T1, f1, (const int*)done, part,
                       Aniso3{}, Mask3{});
    LRFG_LAUNCHED();
  }
  return LRFG_OK;
}

namespace {
__global__ void k_pinv(const double2* __restrict__ u, double2* __restrict__ o, G3 g) {
  for (long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x; s < g.S;
       s += (long long)gridDim.x * blockDim.x) {
    int n1, n2, h;
    decode(g, s, n1, n2, h);
    double k[3];
    kvec(g, n1, n2, h, k);
    o[s] = cscale(u[s], pinv_of(k));
  }
}
}  // namespace

int launch_pinv(const double2* u, double2* o, int N1, int N2, int N3, hipStream_t s) {
  const int N[3] = {N1, N2, N3};
  G3 g = make_g3(N);
  if (g.R > kMaxGridEntries) {
    set_error("inverse Laplacian: grid above 2^32 - 1 entries");
    return LRFG_EUNSUPPORTED;
  }
  long long gv = ceil_div(g.S, kBlock * 4);
  if (gv > 4096) gv = 4096;
  hipLaunchKernelGGL(k_pinv, dim3((int)gv), dim3(kBlock), 0, s, u, o, g);
  LRFG_LAUNCHED();
  return LRFG_OK;
}

}  // namespace lrfg
