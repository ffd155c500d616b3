// Register-resident two-level DFT of lengths N = A B (A, B products of 3s
// and 5s), for the full-grid passes and the batched line transform.
//
// The DFT of Sec. 2.2.1 along a line, X[k] = sum_n x[n] w^(n k) with
// w = exp(DIR 2 pi i / N), is split once (Cooley-Tukey with n = b + B a,
// k = k1 + A k2):
//   X[k1 + A k2] = sum_b w_B^(b k2) [ w_N^(b k1) sum_a x[b + B a] w_A^(a k1) ]
// Phase 1: one work item per (line, b) holds the A values x[b + B a] in
// registers, transforms them (length A), multiplies by w_N^(b k1) and
// writes them to LDS.  Phase 2: one item per (line, k1) reads the B values
// of its k1, transforms them (length B) and holds X[k1 + A k2], k2 < B.
// One LDS exchange per transform, against one read and one write of the
// whole tile per radix stage in the Stockham form of fft.h.  The output
// order of phase 2 (item k1 holds k1 + A k2) is the input order of the
// <B, A> split, so an inverse and a forward transform chain without an
// exchange between them.
//
// Inside an item the length-A (or B) DFT is an unrolled mixed-radix
// recursion L = p q (p = 3 or 5) over a register array whose twiddles are
// compile-time constants (a table evaluated by the compiler).
#pragma once

#include "common.h"

namespace lrfg {

// ------------------------------------------------------------ constants
struct CosSin {
  double c, s;
};

// cos and sin of |x| <= pi/4 by their Taylor series (twelve terms each
// leave a remainder below 1e-20 there).
constexpr CosSin cs_small(double x) {
  const double x2 = x * x;
  double t = x, s = x;
  for (int k = 1; k < 12; ++k) {
    t *= -x2 / ((2.0 * k) * (2.0 * k + 1.0));
    s += t;
  }
  double u = 1.0, c = 1.0;
  for (int k = 1; k < 12; ++k) {
    u *= -x2 / ((2.0 * k - 1.0) * (2.0 * k));
    c += u;
  }
  return CosSin{c, s};
}

// cos and sin of 2 pi e / L, e in [0, L): the angle is q pi/2 + d with
// |d| <= pi/4 (eighths of the circle, exact in integers), the quarter
// turns applied exactly.
constexpr CosSin unit_root(int e, int L) {
  const double quarter_pi = 0.78539816339744830961566084581988;
  const int o = (8 * e) / L;
  const int rem = 8 * e - o * L;
  int q = 0;
  double d = 0.0;
  if (o % 2 == 0) {
    q = o / 2;
    d = quarter_pi * ((double)rem / (double)L);
  } else {
    q = (o + 1) / 2;
    d = -quarter_pi * ((double)(L - rem) / (double)L);
  }
  const CosSin w = cs_small(d);
  switch (q & 3) {
    case 0: return CosSin{w.c, w.s};
    case 1: return CosSin{-w.s, w.c};
    case 2: return CosSin{-w.c, -w.s};
    default: return CosSin{w.s, -w.c};
  }
}

template <int L>
struct RootTable {
  double c[L], s[L];
  constexpr RootTable() : c(), s() {
    for (int e = 0; e < L; ++e) {
      const CosSin w = unit_root(e, L);
      c[e] = w.c;
      s[e] = w.s;
    }
  }
};
template <int L>
inline constexpr RootTable<L> kRoots{};

// exp(DIR 2 pi i e / L); e is a constant after unrolling, so the table
// entry folds into immediates.
template <int DIR, int L>
__host__ __device__ __forceinline__ double2 root(int e) {
  return make_double2(kRoots<L>.c[e], DIR > 0 ? kRoots<L>.s[e] : -kRoots<L>.s[e]);
}

// ------------------------------------------------------------ butterflies
template <int DIR>
__host__ __device__ __forceinline__ void bfly3(double2 (&v)[3]) {
  const double h = 0.86602540378443864676372317075294;  // sin(pi/3)
  const double sg = DIR > 0 ? h : -h;
  const double2 t = cadd(v[1], v[2]);
  const double2 u = csub(v[1], v[2]);
  const double2 m = make_double2(v[0].x - 0.5 * t.x, v[0].y - 0.5 * t.y);
  const double2 iu = make_double2(-u.y * sg, u.x * sg);  // i sg u
  v[0] = cadd(v[0], t);
  v[1] = cadd(m, iu);
  v[2] = csub(m, iu);
}

template <int DIR>
__host__ __device__ __forceinline__ void bfly5(double2 (&v)[5]) {
  const double c1 = 0.30901699437494742410229341718282;   // cos(2 pi/5)
  const double c2 = -0.80901699437494742410229341718282;  // cos(4 pi/5)
  const double s1 = 0.95105651629515357211643933337938;   // sin(2 pi/5)
  const double s2 = 0.58778525229247312916870595463907;   // sin(4 pi/5)
  const double sg = DIR > 0 ? 1.0 : -1.0;
  const double2 a1 = cadd(v[1], v[4]), b1 = csub(v[1], v[4]);
  const double2 a2 = cadd(v[2], v[3]), b2 = csub(v[2], v[3]);
  const double2 r1 = make_double2(v[0].x + c1 * a1.x + c2 * a2.x, v[0].y + c1 * a1.y + c2 * a2.y);
  const double2 r2 = make_double2(v[0].x + c2 * a1.x + c1 * a2.x, v[0].y + c2 * a1.y + c1 * a2.y);
  const double2 g1 = make_double2(s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y);
  const double2 g2 = make_double2(s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y);
  const double2 i1 = make_double2(-g1.y * sg, g1.x * sg);
  const double2 i2 = make_double2(-g2.y * sg, g2.x * sg);
  v[0] = make_double2(v[0].x + a1.x + a2.x, v[0].y + a1.y + a2.y);
  v[1] = cadd(r1, i1);
  v[4] = csub(r1, i1);
  v[2] = cadd(r2, i2);
  v[3] = csub(r2, i2);
}

template <int L>
struct SmallestFactor {
  static constexpr int value = (L % 3 == 0) ? 3 : ((L % 5 == 0) ? 5 : L);
};

// In-register DFT of length L = 3^a 5^b, natural order in and out:
// L = p q, n = q n1 + n2, k = k1 + p k2.
template <int DIR, int L>
__host__ __device__ __forceinline__ void rdft(double2 (&x)[L]) {
  if constexpr (L > 1) {
    constexpr int p = SmallestFactor<L>::value;
    static_assert(p == 3 || p == 5, "register DFT lengths are products of 3s and 5s");
    constexpr int q = L / p;
    double2 y[p][q];
#pragma unroll
    for (int n2 = 0; n2 < q; ++n2) {
      double2 v[p];
#pragma unroll
      for (int n1 = 0; n1 < p; ++n1) v[n1] = x[q * n1 + n2];
      if constexpr (p == 3) bfly3<DIR>(v);
      else bfly5<DIR>(v);
#pragma unroll
      for (int k1 = 0; k1 < p; ++k1) y[k1][n2] = (n2 == 0 || k1 == 0) ? v[k1] : cmul(v[k1], root<DIR, L>(n2 * k1));
    }
#pragma unroll
    for (int k1 = 0; k1 < p; ++k1) rdft<DIR, q>(y[k1]);
#pragma unroll
    for (int k1 = 0; k1 < p; ++k1)
#pragma unroll
      for (int k2 = 0; k2 < q; ++k2) x[k1 + p * k2] = y[k1][k2];
  }
}

// ------------------------------------------------------------ two levels
// The splits built as register kernels: N -> (A, B).  Other lengths take
// the Stockham LDS path of fft.h.
struct Split2 {
  int A, B;
};
constexpr Split2 split2_of(int N) {
  switch (N) {
    case 45: return Split2{9, 5};
    case 75: return Split2{15, 5};
    case 81: return Split2{9, 9};
    case 135: return Split2{15, 9};
    case 225: return Split2{15, 15};
    case 243: return Split2{27, 9};
    case 405: return Split2{27, 15};
    case 675: return Split2{27, 25};
    case 729: return Split2{27, 27};
    default: return Split2{0, 0};
  }
}

// Lines per tile and threads per block of the two-level kernels: the
// tile's LDS exchange (T N complex values) stays near 32 KB, so that five
// tiles share a CU.
constexpr int split2_lines(int N) { return N <= 150 ? 16 : (N <= 300 ? 8 : 4); }

// XCD-aware order of tiles: the dispatcher hands consecutive workgroups
// to the eight XCDs in turn; this maps them so that each XCD takes one
// contiguous run of tiles, and neighbouring tiles (which share cache
// lines at their edges) meet in the same L2.
__device__ __forceinline__ unsigned xcd_tile(unsigned b, unsigned G) {
  const unsigned q = G >> 3, r = G & 7u;
  const unsigned x = b & 7u, j = b >> 3;
  return x * q + (x < r ? x : r) + j;
}

// Phase 1 of one item: x[a] = x[b + B a] on entry; leaves
// w_N^(b k1) sum_a x[b + B a] w_A^(a k1) in x[k1].  tw: the length-N
// table exp(-2 pi i e / N) in LDS.
template <int DIR, int A, int B>
__device__ __forceinline__ void split2_phase1(double2 (&x)[A], int b, const double2* __restrict__ tw) {
  rdft<DIR, A>(x);
#pragma unroll
  for (int k1 = 1; k1 < A; ++k1) {
    if (b != 0) {
      double2 w = tw[b * k1];
      if (DIR > 0) w.y = -w.y;
      x[k1] = cmul(x[k1], w);
    }
  }
}

}  // namespace lrfg
