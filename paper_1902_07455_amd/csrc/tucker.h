// Tucker tensors on the device and their operations (internal), d = 3.
//
// A batched Tucker tensor holds nE independent tensors with the same mode
// ranks: x = G x_1 U_1 x_2 U_2 x_3 U_3 (the paper's eq. tucker), frame j of
// system e is [N_j][r_j] (row-major: the columns are the mode fibres) at
// U[j] + e * sU[j], the core [r_1][r_2][r_3] at G + e * sG.  A stride of 0
// shares a frame or the core across systems.
#pragma once

#include "common.h"
#include "fft.h"
#include "linalg.h"

namespace lrfg {

struct TKB {
  int N[3] = {1, 1, 1};
  int r[3] = {1, 1, 1};
  double* U[3] = {nullptr, nullptr, nullptr};
  long long sU[3] = {0, 0, 0};
  double* G = nullptr;
  long long sG = 0;
  long long usize(int j) const { return (long long)N[j] * r[j]; }
  long long gsize() const { return (long long)r[0] * r[1] * r[2]; }
};

// Carve a batched Tucker tensor with capacity ranks r.
TKB tk_alloc(Arena& ar, const int N[3], const int r[3], int nE);
int tk_zero(TKB& x, int nE, hipStream_t s);
int tk_copy(const TKB& x, TKB& y, int nE, hipStream_t s);
int tk_copy_system(const TKB& x, TKB& y, int e, hipStream_t s);
// y = x with frame j replaced by the real circulant op (0: derivative,
// 1: heat kernel) of its columns, times mult; y.U[j] is the caller's buffer.
int tk_mode_apply(const TKB& x, TKB& y, int j, int op, double t, double mult, const FftDev& f, int nE,
                  hipStream_t s);
// out = a (.) x: Khatri-Rao frames (column i s_j + k) and Kronecker core.
int tk_hadamard(const TKB& a, const TKB& x, TKB& out, int nE, hipStream_t s);
// out = sum of terms: frames side by side, block-diagonal core; the term's
// coefficient (coef[e] * mult) scales its core block.
struct TKTerm {
  const TKB* x;
  const double* coef;
  double mult;
};
int tk_sum(const TKTerm* terms, int nt, TKB& out, int nE, hipStream_t s);
// Core block of a term written at offsets (o1, o2, o3) of out's core
// (out's core must be cleared first); used for sums whose frames are
// written by other kernels.
int tk_place_core(const TKB& x, const double* coef, double mult, TKB& out, const int o[3], int nE, hipStream_t s);
// dots[e] = <x_e, y_e>, scratch of tk_dot_scratch(x, y, nE) doubles.  With
// pairs = P > 0 (nE a multiple of P): dots[e P + j] = <x_e, y_{(e/P) P + j}>,
// scratch of tk_dot_scratch(x, y, nE P) doubles.
size_t tk_dot_scratch(const TKB& x, const TKB& y, int nE);
int tk_dot(const TKB& x, const TKB& y, double* dots, double* scratch, int nE, hipStream_t s, int pairs = 0);

// out = a (.) x without the core: Khatri-Rao frames only (column i s_j + k).
int tk_hadamard_frames(const TKB& a, const TKB& x, TKB& out, int nE, hipStream_t s);

// The core of a Khatri-Rao product a (.) x given by its two factors
// (G_a (x) G_x, index (i r_x + k) per mode), never formed: system t of a
// truncation batch takes G_a at t sGa (sGa = 0: shared) and G_x at
// (t % xmod) sGx.
struct KronCore {
  const double* Ga;
  long long sGa;
  int ra[3];
  const double* Gx;
  long long sGx;
  int xmod;
  int rx[3];
};

// Truncation of batched Tucker tensors to fixed mode ranks (randomised
// HOSVD with Khatri-Rao sketches; see tucker.hip).
struct TkRounder {
  int nE = 1;
  int N[3] = {1, 1, 1};
  int Rmax[3] = {1, 1, 1};   // largest input mode ranks
  int Lmax = 1;              // largest sketch size
  int oversample = 10;
  uint64_t seed = 0;
  uint64_t counter = 0;
  double* om[3] = {};
  double *Z[3], *H, *KR, *Yc[3], *Y[3], *Q[3], *M[3], *T1, *T2, *Cc, *Gr, *S[3], *T3, *T4, *Gs, *Ss, *Ytmp;
  double *Yall, *Qall, *Sall;
  bool kron = false;         // carve the buffers of Kronecker-core inputs
  double *Kp = nullptr, *Kh = nullptr, *Kw = nullptr, *KY = nullptr, *KM = nullptr;
  double* gscr = nullptr;
  size_t gscr_n = 0;
  int* kept = nullptr;       // kept ranks of the last call: mode j of system e at kept[j kept_batch + e]
  int kept_batch = 0;
  int prec = 0;              // lrfg_precision of the sketch contractions
  void carve(Arena& ar);
  // in's core is ignored when kc is given (the input is a Khatri-Rao
  // product whose frames are in.U and whose core is described by kc)
  int round(const TKB& in, TKB& out, double tol, hipStream_t s, int batch = -1, const KronCore* kc = nullptr);
  int kron_mode3(const KronCore& kc, const double* B, long long sB, int l, int nb, double* dst, hipStream_t s,
                 int gp);
};

}  // namespace lrfg
