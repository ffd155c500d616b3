// Register-resident DFTs of lengths N = A B C (factors products of 3s and
// 5s, at most 15), for the full-grid passes and strided line transforms.
//
// The DFT of Sec. 2.2.1 along a line, X[k] = sum_n x[n] w^(n k) with
// w = exp(DIR 2 pi i / N), is split by Cooley-Tukey twice.  With M = B C,
// n = j + M a and k = k1 + A k':
//   X[k1 + A k'] = sum_j w_M^(j k') [ w_N^(j k1) sum_a x[j + M a] w_A^(a k1) ]
// and the inner length-M transform over j = c + C b again as
//   sum_c w_C^(c k3) [ w_M^(c k2) sum_b y[c + C b] w_B^(b k2) ],  k' = k2 + B k3.
// Stage 1: one work item per (line, j) holds the A values x[j + M a] in
// registers, transforms them, multiplies by w_N^(j k1) and writes them to
// LDS.  Stage 2: one item per (line, k1, c) transforms its B values in
// place (length B, twiddle w_M^(c k2)).  Last stage: one item per (line,
// k1, k2) transforms its C values and holds X[k1 + A k2 + A B k3], k3 < C.
// With C = 1 stage 2 is the last (items (line, k1), X[k1 + A k2]).  Two LDS
// exchanges per transform at most, against one read and one write of the
// whole tile per radix stage in the Stockham form of fft.h, and no item
// holds more than 15 complex values.  The last stage's output order is the
// input order of stage 1 of the mirrored split, so an inverse and a
// forward transform chain without an exchange between them.
//
// Inside an item a DFT is an unrolled mixed-radix recursion L = p q
// (p = 3 or 5) over a register array whose twiddles are compile-time
// constants (a table evaluated by the compiler).
#pragma once

#include <type_traits>

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

// ------------------------------------------------------------ splits
// The lengths built as register kernels: N -> (A, B, C).  Other lengths
// take the Stockham LDS path of fft.h.
struct Split3 {
  int A, B, C;
};
constexpr Split3 split_of(int N) {
  switch (N) {
    case 45: return Split3{9, 5, 1};
    case 75: return Split3{15, 5, 1};
    case 81: return Split3{9, 9, 1};
    case 135: return Split3{15, 9, 1};
    case 225: return Split3{15, 15, 1};
    case 243: return Split3{9, 9, 3};
    case 405: return Split3{9, 9, 5};
    case 625: return Split3{5, 25, 5};
    case 675: return Split3{9, 15, 5};
    case 729: return Split3{9, 9, 9};
    default: return Split3{0, 0, 0};
  }
}

// Lines per tile: the tile's LDS buffer (T N complex values) stays near
// 32 KB, so that four or five tiles share a CU.
constexpr int split_lines(int N) { return N <= 150 ? 16 : (N <= 300 ? 8 : (N <= 450 ? 5 : 3)); }

// XCD-aware order of tiles: the dispatcher hands consecutive workgroups
// to the eight XCDs in turn; this maps them so that each XCD takes one
// contiguous run of tiles, and neighbouring tiles (which share cache
// lines at their edges) meet in the same L2.
__device__ __forceinline__ unsigned xcd_tile(unsigned b, unsigned G) {
  const unsigned q = G >> 3, r = G & 7u;
  const unsigned x = b & 7u, j = b >> 3;
  return x * q + (x < r ? x : r) + j;
}

// Element at a 32-bit byte offset from a wave-uniform base: one VGPR per
// address (the callers' launchers check that the arrays stay below 4 GB).
template <typename V>
__device__ __forceinline__ V ld32(const V* base, unsigned byte_off) {
  return *reinterpret_cast<const V*>(reinterpret_cast<const char*>(base) + byte_off);
}
template <typename V>
__device__ __forceinline__ void st32(V* base, unsigned byte_off, V v) {
  *reinterpret_cast<V*>(reinterpret_cast<char*>(base) + byte_off) = v;
}

// One split of a tile of T lines held in LDS, block of NT threads.  LF:
// the lines are contiguous in memory (work items index-fast, LDS line by
// line); otherwise the lines are adjacent entries of strided arrays (items
// line-fast, LDS line-fast).  tw: exp(-2 pi i e / N), e < N, in LDS.
template <int A_, int B_, int C_, int DIR, int T, bool LF, int NT>
struct Fft3 {
  static constexpr int A = A_, B = B_, C = C_;
  static constexpr int M = B * C, N = A * M;
  static constexpr int KL = C > 1 ? B : 1;   // k2 range of the last stage
  static constexpr int R = C > 1 ? C : B;    // outputs per last-stage item
  static constexpr int I1 = T * M, I2 = T * A * C, IL = T * A * KL;
  static constexpr int P1 = (I1 + NT - 1) / NT, PL = (IL + NT - 1) / NT;  // items per thread

  __host__ __device__ static int sidx(int t, int k1, int j) { return LF ? (t * A + k1) * M + j : (k1 * M + j) * T + t; }
  __host__ __device__ static void item1(int i, int& t, int& j) {
    if (LF) { j = i % M; t = i / M; } else { t = i % T; j = i / T; }
  }
  __host__ __device__ static void item2(int i, int& t, int& k1, int& c) {
    if (LF) { c = i % C; const int r = i / C; k1 = r % A; t = r / A; }
    else { t = i % T; const int r = i / T; c = r % C; k1 = r / C; }
  }
  __host__ __device__ static void itemL(int i, int& t, int& k1, int& k2) {
    if (LF) { k1 = i % A; const int r = i / A; k2 = r % KL; t = r / KL; }
    else { t = i % T; const int r = i / T; k1 = r % A; k2 = r / A; }
  }
  // output index of last-stage value r of item (k1, k2)
  __host__ __device__ static constexpr int out_n(int k1, int k2, int r) { return k1 + A * k2 + A * KL * r; }

  __host__ __device__ static double2 twid(const double2* tw, int e) {
    double2 w = tw[e];
    if (DIR > 0) w.y = -w.y;
    return w;
  }
  // stage 1 of item (t, j): v[a] = x[j + M a] on entry; the register part,
  // then the LDS write
  __host__ __device__ static void stage1_regs(double2 (&v)[A], int j, const double2* tw) {
    rdft<DIR, A>(v);
    if (j != 0) {
#pragma unroll
      for (int k1 = 1; k1 < A; ++k1) v[k1] = cmul(v[k1], twid(tw, j * k1));
    }
  }
  __host__ __device__ static void stage1_write(const double2 (&v)[A], int t, int j, double2* S) {
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) S[sidx(t, k1, j)] = v[k1];
  }
  __host__ __device__ static void stage1(double2 (&v)[A], int t, int j, double2* S, const double2* tw) {
    stage1_regs(v, j, tw);
    stage1_write(v, t, j, S);
  }
  // stage 2 of item i (C > 1); in place: an item reads and writes the
  // same LDS entries
  __host__ __device__ static void stage2_item(double2* S, const double2* tw, int i) {
    int t, k1, c;
    item2(i, t, k1, c);
    double2 y[B];
#pragma unroll
    for (int b = 0; b < B; ++b) y[b] = S[sidx(t, k1, c + C * b)];
    rdft<DIR, B>(y);
    if (c != 0) {
#pragma unroll
      for (int k2 = 1; k2 < B; ++k2) y[k2] = cmul(y[k2], twid(tw, A * c * k2));
    }
#pragma unroll
    for (int k2 = 0; k2 < B; ++k2) S[sidx(t, k1, c + C * k2)] = y[k2];
  }
  __device__ static void stage2(double2* S, const double2* tw) {
    if constexpr (C > 1) {
      for (int i = threadIdx.x; i < I2; i += NT) stage2_item(S, tw, i);
    }
  }
  // last stage of item (t, k1, k2): z[r] = X[out_n(k1, k2, r)]
  __host__ __device__ static void last(double2 (&z)[R], int t, int k1, int k2, const double2* S) {
#pragma unroll
    for (int q = 0; q < R; ++q) z[q] = S[sidx(t, k1, k2 * R + q)];
    rdft<DIR, R>(z);
  }
};

// The split of the forward transform that takes the inverse's last-stage
// output order as its stage-1 input order.
template <class F>
struct MirrorOf;
template <int A, int B, int C, int DIR, int T, bool LF, int NT>
struct MirrorOf<Fft3<A, B, C, DIR, T, LF, NT>> {
  using type = std::conditional_t<(C > 1), Fft3<C, B, A, -DIR, T, LF, NT>, Fft3<B, A, 1, -DIR, T, LF, NT>>;
};

}  // namespace lrfg
