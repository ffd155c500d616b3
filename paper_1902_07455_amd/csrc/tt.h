// Tensor-train tensors on the device and their operations (internal).
//
// A batched TT holds nE independent tensors (one per corrector) with the
// same ranks; core j of system e is [r_{j-1}][N_j][r_j] (the carriages of the
// paper's eq. TT) at c[j] + e * s[j].  A stride of 0 shares the core across
// systems (the coefficient).  d = 2 uses cores 0 and 1.
#pragma once

#include "common.h"
#include "fft.h"
#include "linalg.h"

namespace lrfg {

struct TTB {
  int d = 3;
  int N[3] = {1, 1, 1};
  int r[4] = {1, 1, 1, 1};
  double* c[3] = {nullptr, nullptr, nullptr};
  long long s[3] = {0, 0, 0};
  long long size(int j) const { return (long long)r[j] * N[j] * r[j + 1]; }
};

// Carve a batched TT with ranks r (capacity = these ranks) from an arena.
TTB tt_alloc(Arena& ar, int d, const int N[3], const int r[4], int nE);

// One term of a block sum: coef_e = mult * (coef ? coef[e] : 1).
struct TTTerm {
  const TTB* x;
  const double* coef;
  double mult;
};

// Middle carriage (d = 3) of a Hadamard product a (.) g given by its
// factors instead of formed: X[i rg0 + k][n][j rg1 + m] = a[i][n][j]
// g[k][n][m].  Input system s takes coefficient train s % amod (stride sa;
// 0 = shared) and g train s (stride sg).
struct KrMid {
  const double* a = nullptr;
  long long sa = 0;
  int ra0 = 1, ra1 = 1, amod = 1;
  const double* g = nullptr;
  long long sg = 0;
  int rg0 = 1, rg1 = 1;
};

// Randomised TT rounding (sketch, Gram-based orthonormalisation, SVD cut)
// with fixed output ranks; see tt.hip.
struct Rounder {
  int d = 3, nE = 1;
  int N[3] = {1, 1, 1};
  int Rmax[2] = {1, 1};     // largest input ranks at bonds 1, 2
  int Lmax[2] = {1, 1};     // largest sketch sizes
  int oversample = 10;
  int prec = 0;             // lrfg_precision of the sketch and projection
                            // contractions; the orthonormalisation, the
                            // Gram matrices of the cut and the small
                            // factorisations are always FP64
  uint64_t seed = 0;
  uint64_t counter = 0;
  double* om[3] = {};       // sketch cores
  double *W3, *T2, *W2, *Y1, *Q1, *M1, *X2p, *Y2, *Q2, *M2, *X3p;
  double *G, *S, *Ytmp, *S3, *Q2s, *P, *U, *S1;
  double* gscr = nullptr;   // GEMM split-K scratch
  size_t gscr_n = 0;
  int* kept = nullptr;      // kept ranks per bond per system (diagnostics)
  // with kr_ra > 0: scratch for a structured middle carriage of coefficient
  // ranks up to kr_ra and factor ranks up to kr_rg
  int kr_ra = 0, kr_rg = 0;
  double* kz = nullptr;
  void carve(Arena& ar);
  // out (ranks preset to the nominal output ranks) <- T(in) for `batch`
  // systems (default: nE, the capacity it was carved for); with mid, the
  // middle carriage of `in` is mid's Hadamard product (in.c[1] unused);
  // with nblk > 1 (d = 3, FP64, no mid) it is block diagonal, nblk blocks
  // of (R1 / nblk) x N2 x (R2 / nblk) in the dense layout, and the entries
  // off those blocks are never read (they need not be zero)
  int round(const TTB& in, TTB& out, double tol, hipStream_t s, int batch = -1, const KrMid* mid = nullptr,
            int nblk = 1);
  // dots[e] = <a (.) x_e, y_e> for ns systems (d = 3, FP64) with the middle
  // carriage of a (.) x unformed: kr holds the product's first and last
  // carriages (tt_hadamard with skip = 1), mid its middle as factors (x's
  // middle carriage as g); y may have stride 0 (one train for every
  // system).  Uses the rounding buffers; dscr: dot_rows scratch.
  int kr_dot(const TTB& kr, const KrMid& mid, const TTB& y, double* dots, double* dscr, size_t dscr_n, int ns,
             hipStream_t s);
};

int tt_fill(double* p, long long n, double v, hipStream_t s);
int tt_zero(TTB& x, int nE, hipStream_t s);
int tt_copy(const TTB& x, TTB& y, int nE, hipStream_t s);
// tt_copy of the systems e < nE (<= 256) whose bit e of mask[4] is set
// (one launch; no launch when none is).
int tt_copy_systems(const TTB& x, TTB& y, int nE, const unsigned long long* mask, hipStream_t s);
// y = x with core j replaced by the real circulant op (0: derivative,
// 1: heat kernel exp(-t k^2)) along its mode index, times mult.
int tt_mode_apply(const TTB& x, TTB& y, int j, int op, double t, double mult, const FftDev& f, int nE,
                  hipStream_t s);
// out = a (.) x, slice-wise Kronecker of the carriages (ranks multiply);
// carriage `skip` (if >= 0) is left unformed.
int tt_hadamard(const TTB& a, const TTB& x, TTB& out, int nE, hipStream_t s, int skip = -1);
// out = sum of terms as one TT with block carriages (ranks add); out's
// ranks must equal the sums of the terms' ranks.
int tt_sum(const TTTerm* terms, int nt, TTB& out, int nE, hipStream_t s);
// One block of an assembled carriage: rows [o0, o0 + r0) and columns
// [o1, o1 + r1) take coef_e * mult * x (x: [r0][N][r1] per system at
// x + e * sx; coef may be NULL).
struct TTBlock {
  const double* x;
  long long sx;
  int r0, r1, o0, o1;
  const double* coef;
  double mult;
};
// out's carriage j (j < d) assembled from blocks[j][0..nb[j]) (at most 12,
// not overlapping), zeros elsewhere: block-structured trains such as a
// train multiplied by a low-rank TT operator.
int tt_blocks(const TTBlock* const blocks[3], const int nb[3], TTB& out, int nE, hipStream_t s);
// dots[e] = <x_e, y_e>; scratch of tt_dot_scratch(x, y, nE) doubles.  With
// pairs = P > 0 (nE a multiple of P): dots[e P + j] = <x_e, y_{(e/P) P + j}>,
// every pair within each group of P systems, scratch of
// tt_dot_scratch(x, y, nE P) doubles.
size_t tt_dot_scratch(const TTB& x, const TTB& y, int nE);
int tt_dot(const TTB& x, const TTB& y, double* dots, double* scratch, int nE, hipStream_t s, int pairs = 0);

}  // namespace lrfg
