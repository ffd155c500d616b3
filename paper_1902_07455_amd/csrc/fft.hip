// Host-side FFT plans and the generic batched line kernels
// (lrfg_fft_lines, lrfg_mode_op).
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>

#include "fft.h"
#include "fft2.h"
#include "prof.h"

namespace lrfg {

int fft_plan_make(int N, FftPlan* out) {
  if (N < 1 || (N % 2) == 0) {
    set_error("FFT length %d: odd lengths only", N);
    return LRFG_EINVAL;
  }
  FftPlan p;
  p.N = N;
  int n = N;
  // radix order: 5s, then 3s, then the remaining odd primes ascending
  const int pref[2] = {5, 3};
  for (int r : pref) {
    while (n % r == 0) {
      p.radix[p.nstage++] = r;
      n /= r;
    }
  }
  for (int f = 7; n > 1; f += 2) {
    while (n % f == 0) {
      if (p.nstage >= kMaxStages) {
        set_error("FFT length %d: too many factors", N);
        return LRFG_EINVAL;
      }
      p.radix[p.nstage++] = f;
      n /= f;
    }
    if ((long long)f * f > n && n > 1) {
      p.radix[p.nstage++] = n;  // remaining prime
      n = 1;
    }
  }
  p.table.resize(N);
  for (int i = 0; i < N; ++i) {
    // exp(-2 pi i i/N) in extended precision, rounded once to double
    const long double ang = -2.0L * 3.141592653589793238462643383279502884L * (long double)i / (long double)N;
    p.table[i] = make_double2((double)cosl(ang), (double)sinl(ang));
  }
  *out = std::move(p);
  return LRFG_OK;
}

bool fft_two_level() {
  static const bool on = [] {
    const char* v = std::getenv("LRFG_FFT_TWO_LEVEL");
    return v == nullptr || std::strcmp(v, "0") != 0;
  }();
  return on;
}

const FftPlan* fft_plan_cached(int N) {
  static std::mutex mu;
  static std::map<int, std::unique_ptr<FftPlan>> cache;
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find(N);
  if (it != cache.end()) return it->second.get();
  std::unique_ptr<FftPlan> p(new FftPlan());
  if (fft_plan_make(N, p.get()) != LRFG_OK) return nullptr;
  const FftPlan* raw = p.get();
  cache[N] = std::move(p);
  return raw;
}

// ---------------------------------------------------------------- kernels
// Tile = T consecutive line ids of the view x[outer][N][inner]; line id
// l = o*inner + i.  Elements of a tile are loaded so that consecutive
// threads touch consecutive addresses.
// Line ids and inner strides stay below 2^32 (the launchers check), so the
// split of a line id takes a 32-bit division rather than a 64-bit one.
__device__ inline long long line_addr(long long l, int n, int N, int inner) {
  const unsigned lu = (unsigned)l, iu = (unsigned)inner;
  const unsigned o = lu / iu;
  const unsigned i = lu - o * iu;
  return ((long long)o * N + n) * (long long)inner + i;
}
// The (line, index) of element idx < T N of a tile: line-fast when the
// lines are adjacent in memory (inner > 1), index-fast otherwise.
__device__ inline int2 tile_pos(int idx, bool line_fast, int T, float rT, int N, float rN) {
  if (line_fast) {
    const int n = fdiv(idx, T, rT);
    return make_int2(idx - n * T, n);
  }
  const int t = fdiv(idx, N, rN);
  return make_int2(t, idx - t * N);
}

template <int DIR, bool GEN>
__global__ __launch_bounds__(kFftBlock) void k_fft_lines(double2* __restrict__ x, long long nlines, int inner,
                                                          int T, FftDev f, double scale, const int* __restrict__ done,
                                                          long long lines_per_flag) {
  extern __shared__ double2 sm[];
  const int N = f.N;
  const long long l0 = (long long)blockIdx.x * T;
  const int tcount = (int)min((long long)T, nlines - l0);
  // A tile is skipped when every system its lines belong to (system =
  // line / lines_per_flag) is flagged done.  Lines of a finished system
  // inside a running tile are transformed too: that system's arrays are
  // scratch no later kernel reads.
  if (done != nullptr) {
    bool all_done = true;
    for (long long e = l0 / lines_per_flag; e <= (l0 + tcount - 1) / lines_per_flag; ++e)
      all_done = all_done && (done[e] != 0);
    if (all_done) return;
  }
  const int total = T * N;
  const float rT = 1.0f / (float)T, rN = 1.0f / (float)N;
  double2* tw = sm + total;
  stage_twiddles(tw, f);
  double2 v[kFftMaxE];
#pragma unroll
  for (int i = 0; i < kFftMaxE; ++i) {
    const int idx = threadIdx.x + i * kFftBlock;
    int t, n;
    const int2 tn = tile_pos(idx, inner > 1, T, rT, N, rN);
    t = tn.x;
    n = tn.y;
    v[i] = (idx < total && t < tcount) ? x[line_addr(l0 + t, n, N, inner)] : make_double2(0.0, 0.0);
  }
#pragma unroll
  for (int i = 0; i < kFftMaxE; ++i) {
    const int idx = threadIdx.x + i * kFftBlock;
    int t, n;
    const int2 tn = tile_pos(idx, inner > 1, T, rT, N, rN);
    t = tn.x;
    n = tn.y;
    if (idx < total) sm[t * N + n] = v[i];
  }
  __syncthreads();
  lds_fft1<DIR, GEN>(sm, T, f, tw);
#pragma unroll
  for (int i = 0; i < kFftMaxE; ++i) {
    const int idx = threadIdx.x + i * kFftBlock;
    int t, n;
    const int2 tn = tile_pos(idx, inner > 1, T, rT, N, rN);
    t = tn.x;
    n = tn.y;
    if (idx < total && t < tcount) x[line_addr(l0 + t, n, N, inner)] = cscale(sm[t * N + n], scale);
  }
}

// Register form of k_fft_lines (fft2.h) for strided lines (inner > 1) of
// the lengths split_of covers.  Tile = T consecutive line ids; work items
// are line-fast, so each load and store of a wave covers T adjacent
// complex values per mode index.  Addresses are 32-bit byte offsets from
// the tile's first outer block (the launcher checks they fit).  In place:
// every element of the tile is read in stage 1, before the first barrier,
// and written in the last stage.
template <int A, int B, int C, int DIR>
__global__ __launch_bounds__(kFftBlock) void k3_fft_lines(double2* __restrict__ x, long long nlines, int inner,
                                                           FftDev f, double scale, const int* __restrict__ done,
                                                           long long lines_per_flag) {
  constexpr int N = A * B * C;
  constexpr int T = split_lines(N);
  using F = Fft3<A, B, C, DIR, T, false, kFftBlock>;
  __shared__ double2 S[T * N];
  __shared__ double2 tw[N];
  const long long l0 = (long long)xcd_tile(blockIdx.x, gridDim.x) * T;
  const int tcount = (int)min((long long)T, nlines - l0);
  if (done != nullptr) {
    bool all_done = true;
    for (long long e = l0 / lines_per_flag; e <= (l0 + tcount - 1) / lines_per_flag; ++e)
      all_done = all_done && (done[e] != 0);
    if (all_done) return;
  }
  const unsigned in = (unsigned)inner;
  const unsigned o0 = (unsigned)l0 / in;
  double2* base = x + (long long)o0 * N * inner;
  for (int i = threadIdx.x; i < N; i += kFftBlock) tw[i] = f.tw[i];
  __syncthreads();
  for (int it = threadIdx.x; it < F::I1; it += kFftBlock) {
    int t, j;
    F::item1(it, t, j);
    const bool ok = t < tcount;
    const unsigned l = (unsigned)l0 + (unsigned)t, o = l / in;
    const unsigned lo = (o - o0) * (unsigned)N * in + (l - o * in);
    double2 v[A];
#pragma unroll
    for (int a = 0; a < A; ++a)
      v[a] = ok ? ld32(base, (lo + (unsigned)(j + F::M * a) * in) * 16u) : make_double2(0.0, 0.0);
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
      const unsigned l = (unsigned)l0 + (unsigned)t, o = l / in;
      const unsigned lo = (o - o0) * (unsigned)N * in + (l - o * in);
#pragma unroll
      for (int r = 0; r < F::R; ++r)
        st32(base, (lo + (unsigned)F::out_n(k1, k2, r) * in) * 16u, cscale(z[r], scale));
    }
  }
}

template <int A, int B, int C>
int launch3_fft_lines(double2* x, long long nlines, int inner, int dir, const FftDev& f, double scale,
                      hipStream_t s, const char* tag, const int* done, long long lines_per_flag) {
  constexpr int N = A * B * C;
  constexpr int T = split_lines(N);
  const int grid = ceil_div(nlines, T);
  const double bytes = 2.0 * 16.0 * (double)nlines * N;
  if (dir < 0)
    LRFG_LAUNCH_TIMED(tag, bytes, (k3_fft_lines<A, B, C, -1>), dim3(grid), dim3(kFftBlock), 0, s, x, nlines, inner,
                      f, scale, done, lines_per_flag);
  else
    LRFG_LAUNCH_TIMED(tag, bytes, (k3_fft_lines<A, B, C, 1>), dim3(grid), dim3(kFftBlock), 0, s, x, nlines, inner,
                      f, scale, done, lines_per_flag);
  LRFG_LAUNCHED();
  return LRFG_OK;
}

// The register kernels for N in split_of's table (LRFG_EUNSUPPORTED
// otherwise, or when a tile's byte offsets would not fit 32 bits).
int launch3_fft_lines_any(double2* x, long long nlines, int N, int inner, int dir, const FftDev& f, double scale,
                          hipStream_t s, const char* tag, const int* done, long long lines_per_flag) {
  if ((long long)(split_lines(N) + 1) * N * inner * 16 >= (1ll << 32)) return LRFG_EUNSUPPORTED;
#define LRFG_S3(NN)                                                                                         \
  case NN:                                                                                                  \
    return launch3_fft_lines<split_of(NN).A, split_of(NN).B, split_of(NN).C>(x, nlines, inner, dir, f, scale, s, \
                                                                              tag, done, lines_per_flag);
  switch (N) {
    LRFG_S3(45) LRFG_S3(75) LRFG_S3(81) LRFG_S3(135) LRFG_S3(225) LRFG_S3(243) LRFG_S3(405) LRFG_S3(625)
    LRFG_S3(675) LRFG_S3(729)
    default: return LRFG_EUNSUPPORTED;
  }
#undef LRFG_S3
}

// Fibre pairs: the F fibres of each system are paired among themselves
// (2q, 2q+1; the last one alone when F is odd), so a fibre's rounding never
// depends on a neighbouring system and a batch reproduces its systems'
// single results bit for bit.  Pair p of P = ceil(F/2) per system.
__device__ inline long long pair_first(long long p, long long F, long long P, bool* has_second) {
  const unsigned pu = (unsigned)p, Pu = (unsigned)P;
  const unsigned e = pu / Pu, q = pu - e * Pu;
  *has_second = 2 * (long long)q + 1 < F;
  return (long long)e * F + 2 * (long long)q;
}

// Real circulant along the mode index: two real fibres packed into one
// complex line (the operator is real, so it acts on real and imaginary
// parts separately).  op 0: 2 pi i k; op 1: exp(-t k^2); op 2: 1 for |k| <= t,
// else 0 (the projection onto the trigonometric polynomials of degree t);
// result times mult.
// Reads xin, writes x (the same array for in-place use).  Fibres are paired
// within groups of F (one system).
template <bool GEN>
__global__ __launch_bounds__(kFftBlock) void k_mode_op(const double* xin, double* x, long long nfib, long long F,
                                                        int inner, int T, FftDev f, int op, double tparam,
                                                        double mult) {
  extern __shared__ double2 sm[];
  const int N = f.N;
  const long long P = (F + 1) / 2;
  const long long npair = (nfib / F) * P;
  const long long p0 = (long long)blockIdx.x * T;
  const int total = T * N;
  const float rT = 1.0f / (float)T, rN = 1.0f / (float)N;
  double2* tw = sm + total;
  stage_twiddles(tw, f);
  double2 v[kFftMaxE];
#pragma unroll
  for (int i = 0; i < kFftMaxE; ++i) {
    const int idx = threadIdx.x + i * kFftBlock;
    int t, n;
    const int2 tn = tile_pos(idx, inner > 1, T, rT, N, rN);
    t = tn.x;
    n = tn.y;
    bool hb = false;
    const bool ok = idx < total && p0 + t < npair;
    const long long fa = ok ? pair_first(p0 + t, F, P, &hb) : 0;
    const double re = ok ? xin[line_addr(fa, n, N, inner)] : 0.0;
    const double im = (ok && hb) ? xin[line_addr(fa + 1, n, N, inner)] : 0.0;
    v[i] = make_double2(re, im);
  }
#pragma unroll
  for (int i = 0; i < kFftMaxE; ++i) {
    const int idx = threadIdx.x + i * kFftBlock;
    int t, n;
    const int2 tn = tile_pos(idx, inner > 1, T, rT, N, rN);
    t = tn.x;
    n = tn.y;
    if (idx < total) sm[t * N + n] = v[i];
  }
  __syncthreads();
  lds_fft1<-1, GEN>(sm, T, f, tw);
  __syncthreads();
  // one factor per mode index, applied down the T lines of the tile
  for (int n = threadIdx.x; n < N; n += blockDim.x) {
    const int k = freq_of(n, N);
    const double fk = op == 0   ? mult * 2.0 * kPi * (double)k / (double)N
                      : op == 1 ? mult * exp(-tparam * (double)k * (double)k) / (double)N
                                : ((double)abs(k) <= tparam ? mult / (double)N : 0.0);
    for (int t = 0; t < T; ++t) {
      const double2 w = sm[t * N + n];
      sm[t * N + n] = op == 0 ? cmul_i(w, fk) : cscale(w, fk);
    }
  }
  __syncthreads();
  lds_fft1<1, GEN>(sm, T, f, tw);
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kFftMaxE; ++i) {
    const int idx = threadIdx.x + i * kFftBlock;
    int t, n;
    const int2 tn = tile_pos(idx, inner > 1, T, rT, N, rN);
    t = tn.x;
    n = tn.y;
    if (idx < total && p0 + t < npair) {
      bool hb = false;
      const long long fa = pair_first(p0 + t, F, P, &hb);
      const double2 w = sm[t * N + n];
      x[line_addr(fa, n, N, inner)] = w.x;
      if (hb) x[line_addr(fa + 1, n, N, inner)] = w.y;
    }
  }
}

// Heat-kernel terms of a separable exponential sum written straight into
// the block carriage of their sum: for term m (blockIdx.y), the fibres of
// the input carriage x[e][a][:][b] (r0 x N x r1 per system, stride sx) go
// through F^-1 diag(exp(-t_m k^2)) F, are scaled by sc_m, and land at
// out[e][o0 + a][:][o1 + b] of the R0 x N x R1 output (stride so) with
// o0 = m r0 when bl0, o1 = m r1 when bl1.
struct TermParams {
  double t[kMaxTerms];
  double sc[kMaxTerms];
};

template <bool GEN>
__global__ __launch_bounds__(kFftBlock) void k_mode_op_blocks(const double* __restrict__ xin, long long sx, int r0,
                                                               int r1, int nE, double* __restrict__ out,
                                                               long long so, int R1, int bl0, int bl1, int T,
                                                               FftDev f, TermParams tp) {
  extern __shared__ double2 sm[];
  const int N = f.N;
  const int m = blockIdx.y;
  const long long F = (long long)r0 * r1;
  const long long P = (F + 1) / 2;
  const long long npair = (long long)nE * P;
  const long long p0 = (long long)blockIdx.x * T;
  const int total = T * N;
  const float rT = 1.0f / (float)T, rN = 1.0f / (float)N;
  double2* tw = sm + total;
  stage_twiddles(tw, f);
  const int o0 = bl0 ? m * r0 : 0, o1 = bl1 ? m * r1 : 0;
  // fibre ids l < nE r0 r1 < 2^32 (the launcher checks): 32-bit splits
  const unsigned Fu = (unsigned)F, r1u = (unsigned)r1;
  auto in_addr = [&](long long l, int n) -> long long {
    const unsigned lu = (unsigned)l, e = lu / Fu, rem = lu - e * Fu, a = rem / r1u, b = rem - a * r1u;
    return (long long)e * sx + ((long long)a * N + n) * r1 + b;
  };
  auto out_addr = [&](long long l, int n) -> long long {
    const unsigned lu = (unsigned)l, e = lu / Fu, rem = lu - e * Fu, a = rem / r1u, b = rem - a * r1u;
    return (long long)e * so + ((long long)(o0 + (int)a) * N + n) * R1 + o1 + b;
  };
  const bool fibre_fast = r1 > 1;  // consecutive fibres are adjacent in memory
  double2 v[kFftMaxE];
#pragma unroll
  for (int i = 0; i < kFftMaxE; ++i) {
    const int idx = threadIdx.x + i * kFftBlock;
    int t, n;
    const int2 tn = tile_pos(idx, fibre_fast, T, rT, N, rN);
    t = tn.x;
    n = tn.y;
    bool hb = false;
    const bool ok = idx < total && p0 + t < npair;
    const long long fa = ok ? pair_first(p0 + t, F, P, &hb) : 0;
    const double re = ok ? xin[in_addr(fa, n)] : 0.0;
    const double im = (ok && hb) ? xin[in_addr(fa + 1, n)] : 0.0;
    v[i] = make_double2(re, im);
  }
#pragma unroll
  for (int i = 0; i < kFftMaxE; ++i) {
    const int idx = threadIdx.x + i * kFftBlock;
    int t, n;
    const int2 tn = tile_pos(idx, fibre_fast, T, rT, N, rN);
    t = tn.x;
    n = tn.y;
    if (idx < total) sm[t * N + n] = v[i];
  }
  __syncthreads();
  lds_fft1<-1, GEN>(sm, T, f, tw);
  __syncthreads();
  const double tm = tp.t[m], scm = tp.sc[m];
  for (int n = threadIdx.x; n < N; n += blockDim.x) {
    const int k = freq_of(n, N);
    const double fk = scm * exp(-tm * (double)k * (double)k) / (double)N;
    for (int t = 0; t < T; ++t) sm[t * N + n] = cscale(sm[t * N + n], fk);
  }
  __syncthreads();
  lds_fft1<1, GEN>(sm, T, f, tw);
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kFftMaxE; ++i) {
    const int idx = threadIdx.x + i * kFftBlock;
    int t, n;
    const int2 tn = tile_pos(idx, fibre_fast, T, rT, N, rN);
    t = tn.x;
    n = tn.y;
    if (idx < total && p0 + t < npair) {
      bool hb = false;
      const long long fa = pair_first(p0 + t, F, P, &hb);
      const double2 w = sm[t * N + n];
      out[out_addr(fa, n)] = w.x;
      if (hb) out[out_addr(fa + 1, n)] = w.y;
    }
  }
}

int launch_mode_op_blocks(const double* xin, long long sx, int r0, int r1, int nE, double* out, long long so,
                          int R1, bool bl0, bool bl1, int M, const double* t, const double* sc, const FftDev& f,
                          hipStream_t s) {
  if (M < 1 || M > kMaxTerms) {
    set_error("exponential sum with %d terms (1..%d)", M, kMaxTerms);
    return LRFG_EUNSUPPORTED;
  }
  const int N = f.N;
  if (N > kFftMaxE * kFftBlock) {
    set_error("FFT length %d above %d", N, kFftMaxE * kFftBlock);
    return LRFG_EUNSUPPORTED;
  }
  const long long nfib = (long long)nE * r0 * r1;
  if (nfib == 0) return LRFG_OK;
  if (nfib >= (1ll << 32)) {
    set_error("mode op: %lld fibres (at most 2^32 - 1)", nfib);
    return LRFG_EUNSUPPORTED;
  }
  TermParams tp;
  for (int i = 0; i < kMaxTerms; ++i) {
    tp.t[i] = i < M ? t[i] : 0.0;
    tp.sc[i] = i < M ? sc[i] : 0.0;
  }
  const long long npair = (long long)nE * ((r0 * r1 + 1) / 2);
  const int T = lines_per_tile1(N, (int)std::min<long long>(64, std::max<long long>(1, (npair * M + 511) / 512)));
  const size_t shm = size_t(T + 1) * N * sizeof(double2);
  dim3 grid(ceil_div(npair, T), M);
  ProfScope ps_("mode_op_blocks", s);
  if (plan_generic(f))
    hipLaunchKernelGGL(k_mode_op_blocks<true>, grid, dim3(kFftBlock), shm, s, xin, sx, r0, r1, nE, out, so, R1,
                       (int)bl0, (int)bl1, T, f, tp);
  else
    hipLaunchKernelGGL(k_mode_op_blocks<false>, grid, dim3(kFftBlock), shm, s, xin, sx, r0, r1, nE, out, so, R1,
                       (int)bl0, (int)bl1, T, f, tp);
  LRFG_LAUNCHED();
  return LRFG_OK;
}

int fft_dev_upload(const FftPlan& p, double2* d_table, hipStream_t s, FftDev* out) {
  LRFG_HIP(hipMemcpyAsync(d_table, p.table.data(), sizeof(double2) * p.N, hipMemcpyHostToDevice, s));
  FftDev f;
  f.N = p.N;
  f.nstage = p.nstage;
  for (int i = 0; i < kMaxStages; ++i) f.radix[i] = p.radix[i];
  f.tw = d_table;
  *out = f;
  return LRFG_OK;
}

int launch_fft_lines(double2* x, long long outer, int N, long long inner, int dir, const FftDev& f,
                     double scale, hipStream_t s, const char* tag, const int* done,
                     long long lines_per_flag) {
  const long long nlines = outer * inner;
  if (nlines == 0) return LRFG_OK;
  if (nlines >= (1ll << 32) || inner >= (1ll << 31)) {
    set_error("FFT lines: %lld lines of stride %lld (at most 2^32 - 1 and 2^31 - 1)", nlines, inner);
    return LRFG_EUNSUPPORTED;
  }
  if (N > kFftMaxE * kFftBlock) {
    set_error("FFT length %d above %d", N, kFftMaxE * kFftBlock);
    return LRFG_EUNSUPPORTED;
  }
  if (inner > 1 && split_of(N).A > 0 && fft_two_level() &&
      (long long)(split_lines(N) + 1) * N * inner * 16 < (1ll << 32))
    return launch3_fft_lines_any(x, nlines, N, (int)inner, dir, f, scale, s, tag, done, lines_per_flag);
  const int T = lines_per_tile1(N);
  const size_t shm = size_t(T + 1) * N * sizeof(double2);
  const int grid = ceil_div(nlines, T);
  const double bytes = 2.0 * 16.0 * (double)nlines * N;  // nominal: every line read and written once
  const bool gen = plan_generic(f);
#define LRFG_FL(D, G)                                                                                      \
  LRFG_LAUNCH_TIMED(tag, bytes, (k_fft_lines<D, G>), dim3(grid), dim3(kFftBlock), shm, s, x, nlines, (int)inner, \
                    T, f, scale, done, lines_per_flag)
  if (dir < 0) {
    if (gen) LRFG_FL(-1, true); else LRFG_FL(-1, false);
  } else {
    if (gen) LRFG_FL(1, true); else LRFG_FL(1, false);
  }
#undef LRFG_FL
  LRFG_LAUNCHED();
  return LRFG_OK;
}

int launch_mode_op_oop(const double* xin, double* x, long long outer, int N, long long inner, int op, double t,
                       double mult, const FftDev& f, hipStream_t s, long long fib_per_group) {
  const long long nfib = outer * inner;
  if (nfib == 0) return LRFG_OK;
  const long long F = fib_per_group > 0 ? fib_per_group : nfib;
  if (nfib % F != 0) {
    set_error("mode op: %lld fibres are not whole groups of %lld", nfib, F);
    return LRFG_EINVAL;
  }
  const long long npair = (nfib / F) * ((F + 1) / 2);
  if (nfib >= (1ll << 32) || inner >= (1ll << 31)) {
    set_error("mode op: %lld fibres of stride %lld (at most 2^32 - 1 and 2^31 - 1)", nfib, inner);
    return LRFG_EUNSUPPORTED;
  }
  if (N > kFftMaxE * kFftBlock) {
    set_error("FFT length %d above %d", N, kFftMaxE * kFftBlock);
    return LRFG_EUNSUPPORTED;
  }
  // few lines: fewer per block, so that they spread over the CUs (a line's
  // transform is the same whatever the tile it sits in)
  const int T = lines_per_tile1(N, (int)std::min<long long>(64, std::max<long long>(1, (npair + 511) / 512)));
  const size_t shm = size_t(T + 1) * N * sizeof(double2);
  const int grid = ceil_div(npair, T);
  ProfScope ps_("mode_op", s);
  if (plan_generic(f))
    hipLaunchKernelGGL(k_mode_op<true>, dim3(grid), dim3(kFftBlock), shm, s, xin, x, nfib, F, (int)inner, T, f, op,
                       t, mult);
  else
    hipLaunchKernelGGL(k_mode_op<false>, dim3(grid), dim3(kFftBlock), shm, s, xin, x, nfib, F, (int)inner, T, f, op,
                       t, mult);
  LRFG_LAUNCHED();
  return LRFG_OK;
}

int launch_mode_op(double* x, long long outer, int N, long long inner, int op, double t, const FftDev& f,
                   hipStream_t s) {
  return launch_mode_op_oop(x, x, outer, N, inner, op, t, 1.0, f, s, 0);
}

}  // namespace lrfg
