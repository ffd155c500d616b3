// Batched odd-length 1-D DFTs staged in LDS (gfx950).
//
// The DFT matrices are those of the paper's Sec. 2.2.1: forward
// F_N[m,k] = exp(-2 pi i m k / N) / N, inverse exp(+2 pi i m k / N)
// (the 1/N factor is applied by the callers' epilogues).  Odd N only, so the
// factorisation uses odd primes: 3 and 5 have closed-form butterflies, any
// other prime p is a direct length-p DFT (O(N p) per line), which also
// covers prime N.
//
// Algorithm: Stockham autosort, decimation in time.  Stage s combines p
// transforms of length L into transforms of length L' = p L.  With the data
// of a line held as X[j][k] (index j*L + k, j in [0, N/L), k in [0, L)):
//   X'[j'][k + c L] = sum_q w_p^{q c} ( w_N^{q k N/L'} X[j' + q N/L'][k] )
// for j' in [0, N/L'), k in [0, L), c in [0, p).  Ping-pong LDS buffers.
#pragma once

#include <vector>

#include "common.h"

namespace lrfg {

constexpr int kMaxStages = 24;
constexpr int kMaxTerms = 32;   // exponential-sum terms handled per launch

// Device view of one length's plan, passed by value to kernels.
struct FftDev {
  int N;
  int nstage;
  int radix[kMaxStages];
  const double2* tw;  // tw[i] = exp(-2 pi i i / N), i in [0, N)
};

// Host plan: factorisation and twiddle table (uploaded into the workspace).
struct FftPlan {
  int N = 0;
  int nstage = 0;
  int radix[kMaxStages] = {};
  std::vector<double2> table;
};

int fft_plan_make(int N, FftPlan* out);
// Process-lifetime plan for length N (its host table outlives async uploads).
const FftPlan* fft_plan_cached(int N);
int fft_dev_upload(const FftPlan& p, double2* d_table, hipStream_t s, FftDev* out);
// Whether the full-grid passes and strided line transforms use the
// register kernels (fft2.h) for the lengths they cover; set
// LRFG_FFT_TWO_LEVEL=0 in the environment for the Stockham LDS kernels
// everywhere (read once per process).
bool fft_two_level();
// In-place batched DFT of the lines of x[outer][N][inner] (complex),
// dir -1 forward / +1 inverse, result multiplied by `scale`.
// With `done`, a tile whose lines all belong to systems flagged done
// (flag index = line / lines_per_flag) is skipped.
int launch_fft_lines(double2* x, long long outer, int N, long long inner, int dir, const FftDev& f,
                     double scale, hipStream_t s, const char* tag = "fft_lines",
                     const int* done = nullptr, long long lines_per_flag = 1);
// In-place real circulant F^-1 diag(s(k)) F along the middle index of the
// real array x[outer][N][inner]; op 0: s = 2 pi i k, op 1: s = exp(-t k^2).
int launch_mode_op(double* x, long long outer, int N, long long inner, int op, double t,
                   const FftDev& f, hipStream_t s);
// All M heat-kernel terms of one carriage in one launch, written into the
// block carriage of their sum (see fft.hip).
int launch_mode_op_blocks(const double* xin, long long sx, int r0, int r1, int nE, double* out, long long so,
                          int R1, bool bl0, bool bl1, int M, const double* t, const double* sc, const FftDev& f,
                          hipStream_t s);

// ---------------------------------------------------------------- device
template <int DIR>
__device__ inline double2 tw_at(const double2* tw, int e) {
  double2 w = tw[e];
  if (DIR > 0) w.y = -w.y;
  return w;
}

// One Stockham stage on T lines; `in` and `out` are LDS line arrays of
// stride N.  DIR = -1 forward exponent sign, +1 inverse.
template <int DIR>
__device__ inline void fft_stage(const double2* in, double2* out,
                                 int T, int N, int p, int L, const double2* __restrict__ tw) {
  const int Lp = L * p;
  const int m = N / Lp;
  if (p == 3) {
    const int nb = N / 3;
    const int total = T * nb;
    const double s3 = 0.86602540378443864676372317075294;  // sin(pi/3)
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
      const int t = idx / nb;
      const int b = idx - t * nb;
      const int jp = b / L, k = b - jp * L;
      const double2* li = in + t * N;
      double2* lo = out + t * N;
      double2 x0 = li[jp * L + k];
      double2 x1 = li[(jp + m) * L + k];
      double2 x2 = li[(jp + 2 * m) * L + k];
      if (k != 0) {
        x1 = cmul(x1, tw_at<DIR>(tw, k * m));
        x2 = cmul(x2, tw_at<DIR>(tw, 2 * k * m));
      }
      const double2 s = cadd(x1, x2);
      const double2 dd = csub(x1, x2);
      const double2 tt = make_double2(x0.x - 0.5 * s.x, x0.y - 0.5 * s.y);
      // forward: y1 = tt - i s3 dd ; inverse: y1 = tt + i s3 dd
      const double sg = (DIR < 0) ? -s3 : s3;
      const double2 u = make_double2(-dd.y * sg, dd.x * sg);
      const int o = jp * Lp + k;
      lo[o] = cadd(x0, s);
      lo[o + L] = cadd(tt, u);
      lo[o + 2 * L] = csub(tt, u);
    }
  } else if (p == 5) {
    const int nb = N / 5;
    const int total = T * nb;
    const double c1 = 0.30901699437494742410229341718282;   // cos(2pi/5)
    const double c2 = -0.80901699437494742410229341718282;  // cos(4pi/5)
    const double s1 = 0.95105651629515357211643933337938;   // sin(2pi/5)
    const double s2 = 0.58778525229247312916870595463907;   // sin(4pi/5)
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
      const int t = idx / nb;
      const int b = idx - t * nb;
      const int jp = b / L, k = b - jp * L;
      const double2* li = in + t * N;
      double2* lo = out + t * N;
      double2 x0 = li[jp * L + k];
      double2 x1 = li[(jp + m) * L + k];
      double2 x2 = li[(jp + 2 * m) * L + k];
      double2 x3 = li[(jp + 3 * m) * L + k];
      double2 x4 = li[(jp + 4 * m) * L + k];
      if (k != 0) {
        const int e = k * m;
        x1 = cmul(x1, tw_at<DIR>(tw, e));
        x2 = cmul(x2, tw_at<DIR>(tw, 2 * e));
        x3 = cmul(x3, tw_at<DIR>(tw, 3 * e));
        x4 = cmul(x4, tw_at<DIR>(tw, 4 * e));
      }
      const double2 a1 = cadd(x1, x4), b1 = csub(x1, x4);
      const double2 a2 = cadd(x2, x3), b2 = csub(x2, x3);
      const double2 r1 = make_double2(x0.x + c1 * a1.x + c2 * a2.x, x0.y + c1 * a1.y + c2 * a2.y);
      const double2 r2 = make_double2(x0.x + c2 * a1.x + c1 * a2.x, x0.y + c2 * a1.y + c1 * a2.y);
      // i-terms: forward y1 = r1 - i (s1 b1 + s2 b2), y2 = r2 - i (s2 b1 - s1 b2)
      const double sg = (DIR < 0) ? -1.0 : 1.0;
      const double2 v1 = make_double2(s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y);
      const double2 v2 = make_double2(s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y);
      const double2 iv1 = make_double2(-v1.y * sg, v1.x * sg);
      const double2 iv2 = make_double2(-v2.y * sg, v2.x * sg);
      const int o = jp * Lp + k;
      lo[o] = make_double2(x0.x + a1.x + a2.x, x0.y + a1.y + a2.y);
      lo[o + L] = cadd(r1, iv1);
      lo[o + 4 * L] = csub(r1, iv1);
      lo[o + 2 * L] = cadd(r2, iv2);
      lo[o + 3 * L] = csub(r2, iv2);
    }
  } else {
    // Generic prime radix: (a) twiddle the inputs in place (each input
    // element belongs to exactly one butterfly), (b) one output per work
    // item, a direct length-p DFT.
    double2* ino = const_cast<double2*>(in);
    const int total = T * N;
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
      const int t = idx / N;
      const int e = idx - t * N;       // e = (jp + q m) L + k
      const int k = e % L;
      const int r = e / L;
      const int q = r / m;
      if (q != 0 && k != 0) ino[idx] = cmul(ino[idx], tw_at<DIR>(tw, q * k * m));
    }
    __syncthreads();
    const int step = N / p;          // w_p^x = tw[x * N/p]
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
      const int t = idx / N;
      const int o = idx - t * N;       // o = jp Lp + k + c L
      const int jp = o / Lp;
      const int rem = o - jp * Lp;
      const int c = rem / L;
      const int k = rem - c * L;
      const double2* li = in + t * N;
      double2 acc = li[jp * L + k];
      int ex = 0;
      for (int q = 1; q < p; ++q) {
        ex += c;
        if (ex >= p) ex -= p;
        const double2 w = tw_at<DIR>(tw, ex * step);
        const double2 v = li[(jp + q * m) * L + k];
        acc.x += w.x * v.x - w.y * v.y;
        acc.y += w.x * v.y + w.y * v.x;
      }
      out[idx] = acc;
    }
  }
}

// Full transform of T lines (stride N) in LDS.  Returns the buffer holding
// the result (a or b).  Must be called by every thread of the block.
template <int DIR>
__device__ inline double2* lds_fft(double2* a, double2* b, int T, const FftDev& f) {
  int L = 1;
  for (int s = 0; s < f.nstage; ++s) {
    const int p = f.radix[s];
    fft_stage<DIR>(a, b, T, f.N, p, L, f.tw);
    __syncthreads();
    double2* tmp = a;
    a = b;
    b = tmp;
    L *= p;
  }
  return a;
}

// ---------------------------------------------------------------- single buffer
// In-place variant: each thread keeps the butterflies it owns in registers
// between a read phase and a write phase, so one LDS buffer of T*N values
// suffices.  Requires T*N <= kFftMaxE * kFftBlock.  The twiddle table is
// read from LDS (`tw`, N values staged by the caller).  GENERIC = false
// compiles only the radix-3 and radix-5 butterflies (plans whose lengths
// are 3^a 5^b); GENERIC = true adds the direct length-p DFT for other
// primes.
constexpr int kFftBlock = 256;
constexpr int kFftMaxE = 8;   // elements per thread: T*N <= 2048

// x / d for 0 <= x < 2^21, d >= 1, from a float reciprocal with a one-step fix.
__device__ inline int fdiv(int x, int d, float rd) {
  int q = (int)((float)x * rd);
  if (q * d > x) --q;
  else if ((q + 1) * d <= x) ++q;
  return q;
}

template <int DIR>
__device__ inline double2 twl(const double2* tw, int e) {
  double2 w = tw[e];
  if (DIR > 0) w.y = -w.y;
  return w;
}

// Copy the length-N twiddle table into LDS (call before lds_fft1; the
// first barrier of the caller's load phase publishes it).
__device__ inline void stage_twiddles(double2* tw_lds, const FftDev& f) {
  for (int i = threadIdx.x; i < f.N; i += blockDim.x) tw_lds[i] = f.tw[i];
}

template <int DIR, bool GENERIC>
__device__ inline void lds_fft1(double2* buf, int T, const FftDev& f, const double2* tw) {
  const int N = f.N;
  const int tid = threadIdx.x;
  int L = 1;
  for (int st = 0; st < f.nstage; ++st) {
    const int p = f.radix[st];
    const int Lp = L * p;
    const int m = N / Lp;
    const float rL = 1.0f / (float)L;
    if (p == 3) {
      constexpr int MB = (kFftMaxE + 2) / 3;
      const int nb = N / 3;
      const float rnb = 1.0f / (float)nb;
      const int tot = T * nb;
      const double s3 = 0.86602540378443864676372317075294;
      const double sg = (DIR < 0) ? -s3 : s3;
      double2 y0[MB], y1[MB], y2[MB];
      int ob[MB];
#pragma unroll
      for (int i = 0; i < MB; ++i) {
        const int idx = tid + i * kFftBlock;
        ob[i] = -1;
        if (idx < tot) {
          const int t = fdiv(idx, nb, rnb);
          const int b = idx - t * nb;
          const int jp = fdiv(b, L, rL), k = b - jp * L;
          const double2* li = buf + t * N;
          double2 x0 = li[jp * L + k];
          double2 x1 = li[(jp + m) * L + k];
          double2 x2 = li[(jp + 2 * m) * L + k];
          if (k != 0) {
            x1 = cmul(x1, twl<DIR>(tw, k * m));
            x2 = cmul(x2, twl<DIR>(tw, 2 * k * m));
          }
          const double2 s = cadd(x1, x2);
          const double2 dd = csub(x1, x2);
          const double2 tt = make_double2(x0.x - 0.5 * s.x, x0.y - 0.5 * s.y);
          const double2 u = make_double2(-dd.y * sg, dd.x * sg);
          y0[i] = cadd(x0, s);
          y1[i] = cadd(tt, u);
          y2[i] = csub(tt, u);
          ob[i] = t * N + jp * Lp + k;
        }
      }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < MB; ++i) {
        if (ob[i] >= 0) {
          buf[ob[i]] = y0[i];
          buf[ob[i] + L] = y1[i];
          buf[ob[i] + 2 * L] = y2[i];
        }
      }
      __syncthreads();
    } else if (p == 5) {
      constexpr int MB = (kFftMaxE + 4) / 5;
      const int nb = N / 5;
      const float rnb = 1.0f / (float)nb;
      const int tot = T * nb;
      const double c1 = 0.30901699437494742410229341718282;
      const double c2 = -0.80901699437494742410229341718282;
      const double s1 = 0.95105651629515357211643933337938;
      const double s2 = 0.58778525229247312916870595463907;
      const double sg = (DIR < 0) ? -1.0 : 1.0;
      double2 y[MB][5];
      int ob[MB];
#pragma unroll
      for (int i = 0; i < MB; ++i) {
        const int idx = tid + i * kFftBlock;
        ob[i] = -1;
        if (idx < tot) {
          const int t = fdiv(idx, nb, rnb);
          const int b = idx - t * nb;
          const int jp = fdiv(b, L, rL), k = b - jp * L;
          const double2* li = buf + t * N;
          double2 x0 = li[jp * L + k];
          double2 x1 = li[(jp + m) * L + k];
          double2 x2 = li[(jp + 2 * m) * L + k];
          double2 x3 = li[(jp + 3 * m) * L + k];
          double2 x4 = li[(jp + 4 * m) * L + k];
          if (k != 0) {
            const int e = k * m;
            x1 = cmul(x1, twl<DIR>(tw, e));
            x2 = cmul(x2, twl<DIR>(tw, 2 * e));
            x3 = cmul(x3, twl<DIR>(tw, 3 * e));
            x4 = cmul(x4, twl<DIR>(tw, 4 * e));
          }
          const double2 a1 = cadd(x1, x4), b1 = csub(x1, x4);
          const double2 a2 = cadd(x2, x3), b2 = csub(x2, x3);
          const double2 r1 = make_double2(x0.x + c1 * a1.x + c2 * a2.x, x0.y + c1 * a1.y + c2 * a2.y);
          const double2 r2 = make_double2(x0.x + c2 * a1.x + c1 * a2.x, x0.y + c2 * a1.y + c1 * a2.y);
          const double2 v1 = make_double2(s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y);
          const double2 v2 = make_double2(s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y);
          const double2 iv1 = make_double2(-v1.y * sg, v1.x * sg);
          const double2 iv2 = make_double2(-v2.y * sg, v2.x * sg);
          y[i][0] = make_double2(x0.x + a1.x + a2.x, x0.y + a1.y + a2.y);
          y[i][1] = cadd(r1, iv1);
          y[i][4] = csub(r1, iv1);
          y[i][2] = cadd(r2, iv2);
          y[i][3] = csub(r2, iv2);
          ob[i] = t * N + jp * Lp + k;
        }
      }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < MB; ++i) {
        if (ob[i] >= 0) {
#pragma unroll
          for (int c = 0; c < 5; ++c) buf[ob[i] + c * L] = y[i][c];
        }
      }
      __syncthreads();
    } else if (GENERIC) {
      // generic prime radix: twiddle in place, then one output per work
      // item (a direct length-p DFT) staged in registers
      const int total = T * N;
      const float rN = 1.0f / (float)N, rm = 1.0f / (float)m, rLp = 1.0f / (float)Lp;
      for (int idx = tid; idx < total; idx += kFftBlock) {
        const int t = fdiv(idx, N, rN);
        const int e = idx - t * N;
        const int r = fdiv(e, L, rL);
        const int k = e - r * L;
        const int q = fdiv(r, m, rm);
        if (q != 0 && k != 0) buf[idx] = cmul(buf[idx], twl<DIR>(tw, q * k * m));
      }
      __syncthreads();
      const int step = N / p;
      double2 y[kFftMaxE];
#pragma unroll
      for (int i = 0; i < kFftMaxE; ++i) {
        const int idx = tid + i * kFftBlock;
        if (idx < total) {
          const int t = fdiv(idx, N, rN);
          const int o = idx - t * N;
          const int jp = fdiv(o, Lp, rLp);
          const int rem = o - jp * Lp;
          const int c = fdiv(rem, L, rL);
          const int k = rem - c * L;
          const double2* li = buf + t * N;
          double2 acc = li[jp * L + k];
          int ex = 0;
          for (int q = 1; q < p; ++q) {
            ex += c;
            if (ex >= p) ex -= p;
            const double2 w = twl<DIR>(tw, ex * step);
            const double2 v = li[(jp + q * m) * L + k];
            acc.x += w.x * v.x - w.y * v.y;
            acc.y += w.x * v.y + w.y * v.x;
          }
          y[i] = acc;
        }
      }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < kFftMaxE; ++i) {
        const int idx = tid + i * kFftBlock;
        if (idx < total) buf[idx] = y[i];
      }
      __syncthreads();
    }
    L = Lp;
  }
}

inline bool plan_generic(const FftDev& f) {
  for (int s = 0; s < f.nstage; ++s)
    if (f.radix[s] != 3 && f.radix[s] != 5) return true;
  return false;
}

// Lines per tile for the single-buffer kernels: T*N <= kFftMaxE*kFftBlock.
inline int lines_per_tile1(int N, int tmax = 64) {
  int T = (kFftMaxE * kFftBlock) / N;
  if (T > tmax) T = tmax;
  if (T < 1) T = 1;
  return T;
}

}  // namespace lrfg
