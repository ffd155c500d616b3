// Low-rank solve path: the corrector is a tensor train (paper Sec. 3.1.3;
// the CP format for d = 2 is the same train, Sec. 3.1.3 notes TT = CP in 2D)
// and the preconditioned operator is applied with a truncation after every
// rank-raising step (Sec. 3.2, eq. Pls_lowrank):
//
//   C v ~ T P^-1 T div grad-type sum T (a (.) grad v)
//
// in a real-space reading of the paper's Fourier-space scheme: a train of
// nodal values v, the derivative D_alpha = F^-1 diag(2 pi i k) F applied to
// carriage alpha by per-mode 1-D DFTs (Appendix A.3: DFTs act on the
// carriages along their mode index), D_alpha^T = -D_alpha, the material law
// as a carriage-wise Kronecker (Khatri-Rao) product with the coefficient
// train (Appendix A.3, element-wise multiplication), and the Laplacian
// pseudo-inverse as a positive exponential sum of per-mode heat kernels
// (1/(4 pi^2 |k|^2) ~ (1/4 pi^2) sum_m w_m prod_alpha exp(-t_m k_alpha^2)),
// a rank-M element-wise factor in Fourier space (Table 1: preconditioning
// raises the rank).  Because the SVD truncation is invariant under the
// unitary per-mode DFTs, T(F v) = F T(v), so this is the paper's iteration
// up to rounding.
//
// Solvers (Sec. 3.3): truncated preconditioned CG, and the truncated
// minimal-residual iteration u <- T[u + omega r], omega = (Cr, r)/||Cr||^2,
// stopped when the residual fails to decrease (Sec. 4.3); both keep the best
// iterate.  A_H from the energy form of eq. (homog) with the exact operator
// applied to the final train (Sec. 4.3: the error in A_H is the squared
// energy norm of the corrector error).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "lowrank.h"
#include "prof.h"
#include "tt.h"
#include "tucker.h"

namespace lrfg {

struct LowRankPlan {
  lrfg_problem p;
  int d = 3;
  int N[3] = {1, 1, 1};
  FftPlan mode[3];
  int c[4] = {1, 1, 1, 1};   // nominal corrector ranks
  int ra = 16;               // coefficient rank bound
  int M = 2;                 // exponential-sum terms
  std::vector<double> t, w;  // exponents and weights
  int over = 10;
  bool aniso = false;        // constant anisotropic part B present (Sec. 4.4)
  double B[3][3] = {};
  // Ga (exact integration, Sec. 2.2.3): N above is the double grid 2 ga_N - 1
  // and every corrector-side train is kept on the frequencies of ga_N
  // (0: GaNi)
  int ga_N[3] = {0, 0, 0};
};

namespace {

// Positive exponential sum for 1/y on [1, R] from the trapezoidal rule of
// 1/y = int exp(s - e^s y) ds: s_m = s_lo + m h, t_m = e^{s_m},
// w_m = h e^{s_m}, s_lo = ln(eps/R), s_hi = ln(ln(1/eps)), eps = 1e-2,
// h = (s_hi - s_lo)/(M - 1); default M makes h <= 2.
void expsum(double R, int M_req, int* M, std::vector<double>* t, std::vector<double>* w) {
  const double eps = 1e-2;
  const double slo = std::log(eps / R), shi = std::log(std::log(1.0 / eps));
  int m = M_req;
  if (m == 0) m = (int)std::ceil((shi - slo) / 2.0) + 1;
  if (m < 2) m = 2;
  const double h = (shi - slo) / (m - 1);
  t->resize(m);
  w->resize(m);
  for (int i = 0; i < m; ++i) {
    const double s = slo + h * i;
    (*t)[i] = std::exp(s);
    (*w)[i] = h * std::exp(s);
  }
  *M = m;
}

__global__ void k_cp_to_tt(const double* __restrict__ w, const double* __restrict__ f0,
                           const double* __restrict__ f1, const double* __restrict__ f2, int R, int d, int N0, int N1,
                           int N2, double* __restrict__ c0, double* __restrict__ c1, double* __restrict__ c2) {
  // c0[0][n][t] = w_t f0[t][n]; d = 3: c1[t][n][t'] = delta f1[t][n], c2[t][n][0] = f2[t][n];
  // d = 2: c1[t][n][0] = f1[t][n].
  const long long n0 = (long long)N0 * R;
  const long long n1 = (d == 3) ? (long long)R * N1 * R : (long long)R * N1;
  const long long n2 = (d == 3) ? (long long)R * N2 : 0;
  const long long tot = n0 + n1 + n2;
  for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < tot;
       idx += (long long)gridDim.x * blockDim.x) {
    if (idx < n0) {
      const int n = (int)(idx / R), t = (int)(idx % R);
      c0[idx] = w[t] * f0[(long long)t * N0 + n];
    } else if (idx < n0 + n1) {
      const long long i = idx - n0;
      if (d == 3) {
        const int tp = (int)(i % R);
        const long long r = i / R;
        const int n = (int)(r % N1);
        const int t = (int)(r / N1);
        c1[i] = (t == tp) ? f1[(long long)t * N1 + n] : 0.0;
      } else {
        const int n = (int)(i % N1), t = (int)(i / N1);
        c1[i] = f1[(long long)t * N1 + n];
      }
    } else {
      const long long i = idx - n0 - n1;
      const int n = (int)(i % N2), t = (int)(i / N2);
      c2[i] = f2[(long long)t * N2 + n];
    }
  }
}

// alpha_e = done ? 0 : num_e / den_e
__global__ void k_ratio(const double* __restrict__ num, const double* __restrict__ den, const int* __restrict__ done,
                        double* __restrict__ out, int nE) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nE) out[e] = (done[e] || !(den[e] != 0.0)) ? 0.0 : num[e] / den[e];
}

// coef2 = [c; -c]
__global__ void k_pm(const double* __restrict__ c, double* __restrict__ coef2, int nE) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nE) {
    coef2[e] = c[e];
    coef2[nE + e] = -c[e];
  }
}

// beta_e = rz_e / rho_e (0 when done); rho_e <- rz_e
__global__ void k_beta(const double* __restrict__ rz, double* __restrict__ rho, const int* __restrict__ done,
                       double* __restrict__ beta, int nE) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nE) {
    beta[e] = (done[e] || !(rho[e] != 0.0)) ? 0.0 : rz[e] / rho[e];
    if (!done[e]) rho[e] = rz[e];
  }
}

// Restarts of a truncated PCG system from its best iterate before it is
// declared stagnant.
constexpr int kMaxRestarts = 3;
// Sketch counters of the restart steps (the iterations' counters stay far below).
constexpr uint64_t kRestartKeys = 1ull << 62;

// dst_e = src_e for the systems e whose bit is set in mask
struct SysMask {
  unsigned long long m[4];
};
// v[a] <-> v[b] (one thread)
__global__ void k_swap2(double* __restrict__ v, int a, int b) {
  const double t = v[a];
  v[a] = v[b];
  v[b] = t;
}

__global__ void k_pick(double* __restrict__ dst, const double* __restrict__ src, SysMask mask, int nE) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nE && ((mask.m[e >> 6] >> (e & 63)) & 1ull)) dst[e] = src[e];
}
__device__ __host__ inline bool sys_bit(const SysMask& m, int e) { return (m.m[e >> 6] >> (e & 63)) & 1ull; }

struct Ctx {
  LowRankPlan* pl;
  int d, nE;
  int na;                   // coefficient trains held: 1 (shared) or nE (one per system)
  hipStream_t s;
  FftDev f[3];
  Rounder rd;
  TTB a;                    // coefficient: shared (stride 0) or one train per system
  TTB xr;                   // [x; r]: 2 nE trains updated by one truncation
  TTB pq;                   // [p; q]
  TTB x, r, p, q;           // views of the halves
  TTB z, xb, b;             // correctors (ranks c)
  TTB kr;                   // Hadamard products a (.) D_alpha v, d nE trains (ranks ra c)
  TTB comb;                 // block sums (capacity ranks, 2 nE trains)
  TTB h;                    // rounded material terms, d nE trains
  double* gcore;            // carriage buffer for D_alpha v
  double* gmid;             // middle carriages of the d gradients (d = 3), d nE compact
  double* hcore[3];         // carriage buffers for D_alpha^T h_alpha
  double* pcore;            // M * d carriage buffers for the preconditioner terms
  long long pcore_stride;
  double* acore[3];         // carriage buffers of D_alpha a (right-hand side)
  double* bcore;            // anisotropic part: D_j v_j and D_j^2 v_j, 2 d carriage buffers
  long long bstride;
  TTB tmp;                  // extra corrector-size train
  TTB x0;                   // starting corrector of a rank-adaptive stage
  TTB b0, xa, xbest;        // mixed precision: right-hand side, corrector, best corrector
  double *dots, *rho, *pqd, *alpha, *beta, *zz, *Ecoef, *coef2, *dscr;
  double *ones, *mones;     // per-system +1 / -1 coefficients
  int* done;
  size_t dscr_n;
  int comb_cap[4];
};

// na = 1: one coefficient shared by the nE systems; na = nE: one each.
int carve_ctx(Arena& ar, LowRankPlan* pl, int nE, int na, Ctx& C) {
  const int d = pl->d;
  C.pl = pl;
  C.d = d;
  C.nE = nE;
  C.na = na;
  int rc[4] = {1, 1, 1, 1};
  for (int j = 0; j <= d; ++j) rc[j] = pl->c[j];
  int ra[4] = {1, pl->ra, d == 3 ? pl->ra : 1, 1};
  ra[d] = 1;
  // twiddles
  for (int j = 0; j < d; ++j) C.f[j].tw = ar.take<double2>(pl->N[j]);
  C.a = tt_alloc(ar, d, pl->N, ra, na);
  if (na == 1)
    for (int j = 0; j < d; ++j) C.a.s[j] = 0;
  C.xr = tt_alloc(ar, d, pl->N, rc, 2 * nE);
  C.pq = tt_alloc(ar, d, pl->N, rc, 2 * nE);
  C.x = C.xr;
  C.r = C.xr;
  C.p = C.pq;
  C.q = C.pq;
  for (int j = 0; j < d; ++j) {
    C.r.c[j] = C.xr.c[j] + (long long)nE * C.xr.s[j];
    C.q.c[j] = C.pq.c[j] + (long long)nE * C.pq.s[j];
  }
  C.z = tt_alloc(ar, d, pl->N, rc, nE);
  C.xb = tt_alloc(ar, d, pl->N, rc, nE);
  C.b = tt_alloc(ar, d, pl->N, rc, nE);
  C.tmp = tt_alloc(ar, d, pl->N, rc, nE);
  C.x0 = tt_alloc(ar, d, pl->N, rc, nE);
  if (pl->p.precision != LRFG_PREC_FP64) {
    C.b0 = tt_alloc(ar, d, pl->N, rc, nE);
    C.xa = tt_alloc(ar, d, pl->N, rc, nE);
    C.xbest = tt_alloc(ar, d, pl->N, rc, nE);
  }
  // material truncation ranks: the corrector's, except under Ga, where the
  // product a (.) D v on the double grid leaves T_N and its projection back
  // is taken after the truncation, so the truncation keeps the product's
  // full rank r_a c (bounded by the unfoldings) and loses nothing
  int rh[4] = {1, 1, 1, 1};
  for (int j = 1; j < d; ++j) rh[j] = rc[j];
  if (pl->ga_N[0] > 0) {
    if (d == 3) {
      rh[1] = std::min(ra[1] * rc[1], std::min(pl->N[0], pl->N[1] * pl->N[2]));
      rh[2] = std::min(ra[2] * rc[2], std::min(pl->N[2], pl->N[0] * pl->N[1]));
    } else {
      rh[1] = std::min(ra[1] * rc[1], std::min(pl->N[0], pl->N[1]));
    }
  }
  C.h = tt_alloc(ar, d, pl->N, rh, d * nE);
  int rkr[4] = {1, 1, 1, 1};
  for (int j = 1; j < d; ++j) rkr[j] = ra[j] * rc[j];
  if (d == 3) {
    // the middle carriage of a (.) D_alpha v is never formed (the material
    // truncation, the energy form and A_H contract a's and D_alpha v's
    // middle carriages in turn), so only the first and last are held
    C.kr.d = 3;
    for (int j = 0; j < 3; ++j) C.kr.N[j] = pl->N[j];
    for (int j = 0; j < 4; ++j) C.kr.r[j] = rkr[j];
    for (int j = 0; j < 3; ++j) {
      C.kr.s[j] = C.kr.size(j);
      C.kr.c[j] = j == 1 ? nullptr : ar.take<double>((size_t)C.kr.s[j] * d * nE);
    }
  } else {
    C.kr = tt_alloc(ar, d, pl->N, rkr, d * nE);
  }
  // block sums: d material terms, M preconditioner terms, 2 update terms, d coefficient terms
  int cap[4] = {1, 1, 1, 1};
  for (int j = 1; j < d; ++j) {
    int m = d * rh[j];
    if (pl->M * rc[j] > m) m = pl->M * rc[j];
    if (2 * rc[j] > m) m = 2 * rc[j];
    if (d * ra[j] > m) m = d * ra[j];
    if (pl->aniso && d * rh[j] + 3 * rc[j] > m) m = d * rh[j] + 3 * rc[j];  // material terms + K_B v
    cap[j] = m;
  }
  for (int j = 0; j < 4; ++j) C.comb_cap[j] = cap[j];
  C.comb = tt_alloc(ar, d, pl->N, cap, 2 * nE);
  long long maxcore = 0;
  for (int j = 0; j < d; ++j) maxcore = std::max(maxcore, (long long)rc[j] * pl->N[j] * rc[j + 1]);
  C.gcore = ar.take<double>((size_t)maxcore * nE);
  C.gmid = d == 3 ? ar.take<double>((size_t)maxcore * d * nE) : nullptr;
  long long maxh = 0;
  for (int j = 0; j < d; ++j) maxh = std::max(maxh, (long long)rh[j] * pl->N[j] * rh[j + 1]);
  for (int al = 0; al < d; ++al) C.hcore[al] = ar.take<double>((size_t)maxh * nE);
  C.pcore_stride = maxcore * nE;
  C.pcore = ar.take<double>((size_t)C.pcore_stride * pl->M * d);
  long long acmax = 0;
  for (int j = 0; j < d; ++j) acmax = std::max(acmax, (long long)ra[j] * pl->N[j] * ra[j + 1]);
  for (int al = 0; al < d; ++al) C.acore[al] = ar.take<double>((size_t)acmax * na);
  C.bstride = maxcore * nE;
  C.bcore = pl->aniso ? ar.take<double>((size_t)C.bstride * 2 * d) : nullptr;
  // rounding workspace
  Rounder& R = C.rd;
  R.d = d;
  R.nE = std::max(d, 2) * nE;
  for (int j = 0; j < 3; ++j) R.N[j] = (j < d) ? pl->N[j] : 1;
  R.oversample = pl->over;
  R.seed = pl->p.seed;
  for (int j = 1; j < d; ++j) {
    R.Rmax[j - 1] = std::max(cap[j], rkr[j]);
    R.Lmax[j - 1] = std::max(rc[j], rh[j]) + pl->over;
  }
  if (d == 3) {
    // the material truncation takes the middle carriage as a (.) D v
    R.kr_ra = pl->ra;
    R.kr_rg = std::max(rc[1], rc[2]);
  }
  R.carve(ar);
  // per-system scalars (dots also holds the 2 d nE energy-form products)
  C.dots = ar.take<double>((size_t)7 * nE + 64);
  C.rho = ar.take<double>(nE);
  C.pqd = ar.take<double>(nE);
  C.alpha = ar.take<double>(nE);
  C.beta = ar.take<double>(nE);
  C.zz = ar.take<double>(nE);
  C.Ecoef = ar.take<double>((size_t)3 * nE);
  C.coef2 = ar.take<double>((size_t)2 * nE);
  C.done = ar.take<int>(nE);
  C.ones = ar.take<double>(nE);
  C.mones = ar.take<double>(nE);
  // dot scratch: largest pair (kr, c) or (a, a); the A_H cross terms take
  // up to 3 pairs per system
  size_t dn = tt_dot_scratch(C.z, C.z, 3 * nE);
  dn = std::max(dn, tt_dot_scratch(C.a, C.z, nE));
  dn = std::max(dn, tt_dot_scratch(C.a, C.a, nE));
  if (d == 3)
    dn = std::max(dn, dot_rows_scratch((long long)rkr[1] * pl->N[1] * rc[2], nE));  // kr_dot
  else
    dn = std::max(dn, tt_dot_scratch(C.kr, C.z, 3 * nE));
  if (pl->aniso) {
    // <x, K_B x> with K_B x of ranks 3 c
    TTB w = C.z;
    for (int j = 1; j < d; ++j) w.r[j] = 3 * rc[j];
    dn = std::max(dn, tt_dot_scratch(C.z, w, nE));
  }
  C.dscr_n = dn;
  C.dscr = ar.take<double>(dn);
  return LRFG_OK;
}

// ------------------------------------------------------------------ anisotropic part
// K_B v = sum_{alpha beta} B_{alpha beta} D_alpha^T D_beta v for the constant
// matrix B of Sec. 4.4 (D_alpha^T = -D_alpha).  Its symbol 4 pi^2 k.Bk is a
// quadratic form in separate variables, so K_B is a TT operator of ranks 3
// whose carriages hold I, D and D^2 of one mode:
//   first   [ -B00 D^2 | D | I ]
//   middle  [ I 0 0 ; -2 B01 D | -2 B02 I | 0 ; -B11 D^2 | -2 B12 D | I ]
//   last    [ I ; D ; -B22 D^2 ]           (d = 3)
//   last    [ I ; -2 B01 D ; -B11 D^2 ]    (d = 2)
// and K_B v is a train of ranks 3 r whose carriage blocks are those
// operators applied to v's carriages.  Appends these blocks, placed at the
// bond offsets o[0..d] (o[0] = o[d] = 0), to blk/nb; D v_j and D^2 v_j go to
// C.bcore.
constexpr int kMaxBlk = 12;
int aniso_blocks(Ctx& C, const TTB& v, int n, const int o[4], TTBlock blk[3][kMaxBlk], int nb[3]) {
  const int d = C.d;
  const double(*B)[3] = C.pl->B;
  TTB dv[3], d2v[3];
  for (int j = 0; j < d; ++j) {
    dv[j] = v;
    dv[j].c[j] = C.bcore + (long long)(2 * j) * C.bstride;
    LRFG_TRY(tt_mode_apply(v, dv[j], j, 0, 0.0, 1.0, C.f[j], n, C.s));
    d2v[j] = dv[j];
    d2v[j].c[j] = C.bcore + (long long)(2 * j + 1) * C.bstride;
    LRFG_TRY(tt_mode_apply(dv[j], d2v[j], j, 0, 0.0, 1.0, C.f[j], n, C.s));
  }
  auto add = [&](int j, const TTB& src, int a, int b, double mult) {
    TTBlock t;
    t.x = src.c[j];
    t.sx = src.s[j];
    t.r0 = v.r[j];
    t.r1 = v.r[j + 1];
    t.o0 = o[j] + a * v.r[j];
    t.o1 = o[j + 1] + b * v.r[j + 1];
    t.coef = nullptr;
    t.mult = mult;
    blk[j][nb[j]++] = t;
  };
  add(0, d2v[0], 0, 0, -B[0][0]);
  add(0, dv[0], 0, 1, 1.0);
  add(0, v, 0, 2, 1.0);
  if (d == 3) {
    add(1, v, 0, 0, 1.0);
    add(1, dv[1], 1, 0, -2.0 * B[0][1]);
    add(1, v, 1, 1, -2.0 * B[0][2]);
    add(1, d2v[1], 2, 0, -B[1][1]);
    add(1, dv[1], 2, 1, -2.0 * B[1][2]);
    add(1, v, 2, 2, 1.0);
    add(2, v, 0, 0, 1.0);
    add(2, dv[2], 1, 0, 1.0);
    add(2, d2v[2], 2, 0, -B[2][2]);
  } else {
    add(1, v, 0, 0, 1.0);
    add(1, dv[1], 1, 0, -2.0 * B[0][1]);
    add(1, d2v[1], 2, 0, -B[1][1]);
  }
  return LRFG_OK;
}

// Ga: the trains' mode fibres projected onto the trigonometric polynomials
// of the corrector's grid (|k_j| <= (N_j - 1)/2 on the double grid), in place
int ga_project(Ctx& C, TTB& x, int n) {
  for (int j = 0; j < C.d; ++j) {
    TTB y = x;
    LRFG_TRY(tt_mode_apply(x, y, j, 2, (double)((C.pl->ga_N[j] - 1) / 2), 1.0, C.f[j], n, C.s));
  }
  return LRFG_OK;
}

// T(in) into out; under Ga the result is projected onto T_N's frequencies
// again: the Gram-based orthonormalisation works to about sqrt(eps), and the
// components it leaves outside T_N are invisible to the projected operator
// but not to the double-grid energy form, so they must not accumulate
int round_s(Ctx& C, const TTB& in, TTB& out, double tol, int batch, const KrMid* mid = nullptr, int nblk = 1) {
  LRFG_TRY(C.rd.round(in, out, tol, C.s, batch, mid, nblk));
  if (C.pl->ga_N[0] > 0) LRFG_TRY(ga_project(C, out, batch));
  return LRFG_OK;
}

// W = K_B v for n trains, into C.comb (ranks 3 r)
int aniso_train(Ctx& C, const TTB& v, int n, TTB& W) {
  TTBlock blk[3][kMaxBlk];
  int nb[3] = {0, 0, 0};
  const int o[4] = {0, 0, 0, 0};
  LRFG_TRY(aniso_blocks(C, v, n, o, blk, nb));
  W = C.comb;
  for (int j = 1; j < C.d; ++j) W.r[j] = 3 * v.r[j];
  for (int j = 0; j < C.d; ++j) W.s[j] = W.size(j);
  const TTBlock* bp[3] = {blk[0], blk[1], blk[2]};
  return tt_blocks(bp, nb, W, n, C.s);
}

// ------------------------------------------------------------------ operators
// out = T(sum_alpha D_alpha^T T(a (.) D_alpha v)); the d material
// truncations run as one batched truncation of d nE trains.  For d = 3 the
// middle carriage of a (.) D_alpha v, (r_a c)^2 N per train, is never formed:
// the truncation contracts a's and D_alpha v's carriages in turn.
int apply_K(Ctx& C, const TTB& v, TTB& out) {
  const int d = C.d, nE = C.nE;
  const bool mid = d == 3;
  const long long gs = v.size(1);
  for (int al = 0; al < d; ++al) {
    TTB g = v;
    g.c[al] = C.gcore;
    LRFG_TRY(tt_mode_apply(v, g, al, 0, 0.0, 1.0, C.f[al], nE, C.s));
    TTB kra = C.kr;
    for (int j = 0; j < d; ++j)
      if (!(mid && j == 1)) kra.c[j] = C.kr.c[j] + (long long)al * nE * C.kr.s[j];
    LRFG_TRY(tt_hadamard(C.a, g, kra, nE, C.s, mid ? 1 : -1));
    if (mid) {
      double* dst = C.gmid + (long long)al * nE * gs;
      if (g.s[1] == gs) {
        LRFG_HIP(hipMemcpyAsync(dst, g.c[1], sizeof(double) * gs * nE, hipMemcpyDeviceToDevice, C.s));
      } else {
        for (int e = 0; e < nE; ++e)
          LRFG_HIP(hipMemcpyAsync(dst + e * gs, g.c[1] + e * g.s[1], sizeof(double) * gs, hipMemcpyDeviceToDevice,
                                  C.s));
      }
    }
  }
  KrMid km;
  km.a = C.a.c[1];
  km.sa = C.a.s[1];
  km.ra0 = C.a.r[1];
  km.ra1 = C.a.r[2];
  km.amod = nE;
  km.g = C.gmid;
  km.sg = gs;
  km.rg0 = v.r[1];
  km.rg1 = v.r[2];
  LRFG_TRY(C.rd.round(C.kr, C.h, 0.0, C.s, d * nE, mid ? &km : nullptr));
  TTB ha[3], hd[3];
  TTTerm terms[3];
  for (int al = 0; al < d; ++al) {
    ha[al] = C.h;
    for (int j = 0; j < d; ++j) ha[al].c[j] = C.h.c[j] + (long long)al * nE * C.h.s[j];
    hd[al] = ha[al];
    hd[al].c[al] = C.hcore[al];
    LRFG_TRY(tt_mode_apply(ha[al], hd[al], al, 0, 0.0, -1.0, C.f[al], nE, C.s));
    // Ga: the test functions are T_N's, so the material terms are projected
    // back onto its frequencies before the sum's truncation (I* of eq.
    // ls_Ga_fourier)
    if (C.pl->ga_N[0] > 0) LRFG_TRY(ga_project(C, hd[al], nE));
    terms[al] = TTTerm{&hd[al], nullptr, 1.0};
  }
  TTB comb = C.comb;
  if (!C.pl->aniso) {
    for (int j = 1; j < d; ++j) comb.r[j] = d * C.h.r[j];
    for (int j = 0; j < d; ++j) comb.s[j] = comb.size(j);
    LRFG_TRY(tt_sum(terms, d, comb, nE, C.s));
    return round_s(C, comb, out, C.pl->p.trunc_tol, nE);
  }
  // with the anisotropic part: the d material terms (block diagonal) and
  // K_B v (ranks 3 r, exact) in one sum before the truncation
  TTBlock blk[3][kMaxBlk];
  int nb[3] = {0, 0, 0};
  const TTB& h = C.h;
  for (int j = 0; j < d; ++j)
    for (int al = 0; al < d; ++al) {
      TTBlock t;
      t.x = hd[al].c[j];
      t.sx = hd[al].s[j];
      t.r0 = h.r[j];
      t.r1 = h.r[j + 1];
      t.o0 = al * (j == 0 ? 0 : h.r[j]);
      t.o1 = al * (j == d - 1 ? 0 : h.r[j + 1]);
      t.coef = nullptr;
      t.mult = 1.0;
      blk[j][nb[j]++] = t;
    }
  int o[4] = {0, 0, 0, 0};
  for (int j = 1; j < d; ++j) o[j] = d * h.r[j];
  LRFG_TRY(aniso_blocks(C, v, nE, o, blk, nb));
  for (int j = 1; j < d; ++j) comb.r[j] = d * h.r[j] + 3 * v.r[j];
  for (int j = 0; j < d; ++j) comb.s[j] = comb.size(j);
  const TTBlock* bp[3] = {blk[0], blk[1], blk[2]};
  LRFG_TRY(tt_blocks(bp, nb, comb, nE, C.s));
  return round_s(C, comb, out, C.pl->p.trunc_tol, nE);
}

// out = T(P~^-1 v), P~^-1 = (1/4 pi^2) sum_m w_m prod_alpha H_{m,alpha}:
// the M terms are written straight into the block carriages of their sum
// (one launch per carriage), then truncated.  The middle carriage of the
// sum is block diagonal; an FP64 truncation (d = 3) contracts its M
// diagonal blocks alone, so the zeros off them are neither written nor
// read.
int apply_P(Ctx& C, const TTB& v, TTB& out) {
  const int d = C.d, nE = C.nE;
  const int M = C.pl->M;
  const bool blocks = d == 3 && C.rd.prec == LRFG_PREC_FP64;
  TTB comb = C.comb;
  for (int j = 1; j < d; ++j) comb.r[j] = M * v.r[j];
  for (int j = 0; j < d; ++j) comb.s[j] = comb.size(j);
  if (!blocks)
    for (int j = 1; j < d - 1; ++j) LRFG_TRY(tt_fill(comb.c[j], comb.size(j) * nE, 0.0, C.s));
  std::vector<double> sc(M), one(M, 1.0);
  for (int m = 0; m < M; ++m) sc[m] = C.pl->w[m] / (4.0 * kPi * kPi);
  for (int j = 0; j < d; ++j) {
    LRFG_TRY(launch_mode_op_blocks(v.c[j], v.s[j], v.r[j], v.r[j + 1], nE, comb.c[j], comb.s[j], comb.r[j + 1],
                                   j > 0, j < d - 1, M, C.pl->t.data(), j == 0 ? sc.data() : one.data(), C.f[j],
                                   C.s));
  }
  return round_s(C, comb, out, C.pl->p.trunc_tol, nE, nullptr, blocks ? M : 1);
}

// [x; r] <- T([x; r] + coef2 [p; q]) as one truncation of 2 nE trains
int update_xr(Ctx& C) {
  TTTerm t[2] = {TTTerm{&C.xr, nullptr, 1.0}, TTTerm{&C.pq, C.coef2, 1.0}};
  TTB comb = C.comb;
  for (int j = 1; j < C.d; ++j) comb.r[j] = 2 * C.xr.r[j];
  for (int j = 0; j < C.d; ++j) comb.s[j] = comb.size(j);
  LRFG_TRY(tt_sum(t, 2, comb, 2 * C.nE, C.s));
  return round_s(C, comb, C.xr, C.pl->p.trunc_tol, 2 * C.nE);
}

// out = T(x + cb y) for nE trains
int axpby(Ctx& C, const TTB& x, const TTB& y, const double* cb, TTB& out) {
  TTTerm t[2] = {TTTerm{&x, nullptr, 1.0}, TTTerm{&y, cb, 1.0}};
  TTB comb = C.comb;
  for (int j = 1; j < C.d; ++j) comb.r[j] = x.r[j] + y.r[j];
  for (int j = 0; j < C.d; ++j) comb.s[j] = comb.size(j);
  LRFG_TRY(tt_sum(t, 2, comb, C.nE, C.s));
  return round_s(C, comb, out, C.pl->p.trunc_tol, C.nE);
}

int dot(Ctx& C, const TTB& x, const TTB& y, double* out) { return tt_dot(x, y, out, C.dscr, C.nE, C.s); }

// The middle carriage of a (.) g (d = 3) as its factors: system e reads
// coefficient train e % nE (one train shared, or one per system) and g's
// middle carriage e.
KrMid kr_mid(const Ctx& C, const TTB& g) {
  KrMid km;
  km.a = C.a.c[1];
  km.sa = C.a.s[1];
  km.ra0 = C.a.r[1];
  km.ra1 = C.a.r[2];
  km.amod = C.nE;
  km.g = g.c[1];
  km.sg = g.s[1];
  km.rg0 = g.r[1];
  km.rg1 = g.r[2];
  return km;
}

int read_dev(Ctx& C, const double* dptr, double* host, int n) {
  LRFG_HIP(hipMemcpyAsync(host, dptr, sizeof(double) * n, hipMemcpyDeviceToHost, C.s));
  LRFG_HIP(hipStreamSynchronize(C.s));
  return LRFG_OK;
}

}  // namespace

// ====================================================================== plan
// nominal corrector ranks: the rank cap, limited by the unfoldings' sizes
static void plan_ranks(LowRankPlan& pl) {
  const lrfg_problem& p = pl.p;
  if (p.d == 3) {
    pl.c[1] = std::min(p.rank_cap, std::min(p.N[0], p.N[1] * p.N[2]));
    pl.c[2] = std::min(p.rank_cap, std::min(p.N[2], p.N[0] * p.N[1]));
  } else {
    pl.c[1] = std::min(p.rank_cap, std::min(p.N[0], p.N[1]));
  }
}

int lowrank_plan_create(const lrfg_problem& p, const FftPlan* mode, LowRankPlan** out, const int* ga_N) {
  LowRankPlan* pl = new LowRankPlan();
  pl->p = p;
  if (ga_N != nullptr)
    for (int j = 0; j < p.d; ++j) pl->ga_N[j] = ga_N[j];
  pl->d = p.d;
  for (int j = 0; j < p.d; ++j) {
    pl->N[j] = p.N[j];
    pl->mode[j] = mode[j];
  }
  for (int i = 0; i < p.d; ++i)
    for (int j = 0; j < p.d; ++j) {
      pl->B[i][j] = p.aniso[i * p.d + j];
      if (pl->B[i][j] != 0.0) pl->aniso = true;
    }
  pl->ra = p.coeff_rank > 0 ? p.coeff_rank : 16;
  if (pl->ga_N[0] > 0) pl->ra = 2;  // Ga's square/cube coefficient: CP rank 2 on the double grid
  pl->over = p.oversample > 0 ? p.oversample : 10;
  if (pl->ra > kMaxCoeffRank) {
    set_error("coeff_rank %d exceeds the supported %d", pl->ra, kMaxCoeffRank);
    delete pl;
    return LRFG_EUNSUPPORTED;
  }
  plan_ranks(*pl);
  for (int j = 1; j < p.d; ++j) {
    // under Ga the material truncation keeps ranks up to r_a c (see carve_ctx)
    const int cj = pl->ga_N[0] > 0 ? std::min(pl->ra * pl->c[j], j == 1 ? p.N[0] : p.N[p.d - 1]) : pl->c[j];
    if (cj + pl->over > kMaxEig) {
      // the sketch size bounds the small eigenproblems
      int o = kMaxEig - cj;
      if (o < 0) {
        set_error("rank_cap %d exceeds the supported %d", p.rank_cap, kMaxEig);
        delete pl;
        return LRFG_EUNSUPPORTED;
      }
      pl->over = std::min(pl->over, o);
    }
  }
  if (p.format == LRFG_FORMAT_TUCKER) {
    if (p.d != 3) {
      set_error("the Tucker format is built for d = 3");
      delete pl;
      return LRFG_EUNSUPPORTED;
    }
    for (int j = 0; j < 3; ++j) pl->c[j + 1] = std::min(p.rank_cap, p.N[j]);  // mode ranks c[1..3]
    if (std::max(pl->c[1], std::max(pl->c[2], pl->c[3])) + 1 > kMaxEig) {
      set_error("rank_cap %d exceeds the supported %d", p.rank_cap, kMaxEig - 1);
      delete pl;
      return LRFG_EUNSUPPORTED;
    }
  }
  // the preconditioner's range: the corrector's frequencies (Ga: those of ga_N)
  double R = 0.0;
  for (int j = 0; j < p.d; ++j) {
    const int n = ga_N != nullptr ? ga_N[j] : p.N[j];
    R += (double)((n - 1) / 2) * ((n - 1) / 2);
  }
  expsum(R, p.precond_terms, &pl->M, &pl->t, &pl->w);
  *out = pl;
  return LRFG_OK;
}

void lowrank_plan_destroy(LowRankPlan* lr) { delete lr; }

size_t tucker_workspace_bytes(const LowRankPlan* lr, int max_nE);
int tucker_solve(LowRankPlan* pl, const lrfg_coeff& ac, const double* E, int nE, void* ws, size_t ws_bytes,
                 hipStream_t s, lrfg_result* out);

size_t lowrank_workspace_bytes(const LowRankPlan* lr, int max_nE) {
  if (lr->p.format == LRFG_FORMAT_TUCKER) return tucker_workspace_bytes(lr, std::min(max_nE, 3));
  // room for one coefficient train per system (the batched form)
  Arena ar;
  Ctx C;
  carve_ctx(ar, const_cast<LowRankPlan*>(lr), max_nE, max_nE, C);
  return ar.used + 1024;
}

// ====================================================================== solve
namespace {

// Coefficient b as a TT into system slot `e` of C.a (CP factors -> TT
// carriages, or TT cores copied); checks its ranks against `rk`.
int load_coeff(Ctx& C, const lrfg_coeff& ac, int e, int* rk) {
  LowRankPlan* pl = C.pl;
  const int d = C.d;
  hipStream_t s = C.s;
  double* dst[3];
  for (int j = 0; j < d; ++j) dst[j] = C.a.c[j] + (long long)e * C.a.s[j];
  if (ac.full != nullptr) {
    set_error("the low-rank path takes the coefficient in CP or TT form");
    return LRFG_EUNSUPPORTED;
  }
  if (ac.weights != nullptr) {
    const int R = ac.rank;
    if (R < 1 || R > pl->ra) {
      set_error("coefficient rank %d outside [1, coeff_rank = %d]", R, pl->ra);
      return LRFG_EINVAL;
    }
    if (rk[1] != 0 && rk[1] != R) {
      set_error("all coefficients of one batch need the same rank (%d vs %d)", R, rk[1]);
      return LRFG_EINVAL;
    }
    rk[0] = 1;
    rk[d] = 1;
    for (int j = 1; j < d; ++j) rk[j] = R;
    const double* w = ac.weights;
    const double* f[3] = {ac.factors[0], ac.factors[1], d == 3 ? ac.factors[2] : ac.factors[1]};
    if (!ac.on_device) {
      // stage host factors through the product buffer (not yet in use)
      size_t n = R;
      for (int j = 0; j < d; ++j) n += (size_t)R * pl->N[j];
      if (n > (size_t)C.comb.size(0) * 2 * C.nE) {
        set_error("coefficient staging too small");
        return LRFG_EWORKSPACE;
      }
      double* dstage = C.comb.c[0];
      LRFG_HIP(hipMemcpyAsync(dstage, w, sizeof(double) * R, hipMemcpyHostToDevice, s));
      size_t off = R;
      const double* df[3];
      for (int j = 0; j < d; ++j) {
        LRFG_HIP(hipMemcpyAsync(dstage + off, ac.factors[j], sizeof(double) * R * pl->N[j], hipMemcpyHostToDevice,
                                s));
        df[j] = dstage + off;
        off += (size_t)R * pl->N[j];
      }
      w = dstage;
      for (int j = 0; j < d; ++j) f[j] = df[j];
      if (d == 2) f[2] = df[1];
    }
    const long long tot = (long long)pl->N[0] * R + (d == 3 ? (long long)R * pl->N[1] * R + (long long)R * pl->N[2]
                                                           : (long long)R * pl->N[1]);
    hipLaunchKernelGGL(k_cp_to_tt, dim3((int)std::min<long long>(4096, (tot + 255) / 256)), dim3(256), 0, s, w, f[0],
                       f[1], f[2], R, d, pl->N[0], pl->N[1], d == 3 ? pl->N[2] : 1, dst[0], dst[1],
                       d == 3 ? dst[2] : nullptr);
    LRFG_LAUNCHED();
    return LRFG_OK;
  }
  const int* r = ac.tt_ranks;
  if (r[0] != 1 || r[d] != 1) {
    set_error("TT coefficient: r_0 = r_d = 1 required");
    return LRFG_EINVAL;
  }
  for (int j = 1; j < d; ++j) {
    if (r[j] < 1 || r[j] > pl->ra) {
      set_error("TT coefficient rank %d outside [1, coeff_rank = %d]", r[j], pl->ra);
      return LRFG_EINVAL;
    }
    if (rk[j] != 0 && rk[j] != r[j]) {
      set_error("all coefficients of one batch need the same TT ranks");
      return LRFG_EINVAL;
    }
  }
  for (int j = 0; j <= d; ++j) rk[j] = r[j];
  for (int j = 0; j < d; ++j) {
    const size_t n = (size_t)r[j] * pl->N[j] * r[j + 1];
    LRFG_HIP(hipMemcpyAsync(dst[j], ac.tt_cores[j], sizeof(double) * n,
                            ac.on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
  }
  return LRFG_OK;
}

}  // namespace

// Ga's coefficient of a square/cube inclusion on the double grid as a CP
// tensor of rank 2: A_M = vout + (vin - vout) prod_j chi_j, chi_j the Fourier
// series of the 1-D indicator of |x| < size truncated to |m| <= N_j - 1
// (coefficients 2 size at m = 0, sin(2 pi m size)/(pi m) otherwise) at the
// double-grid points x_p = -1/2 + (p + 1/2)/M_j.
struct GaCP {
  std::vector<double> w, f[3];
  lrfg_coeff c{};
};
static void ga_cp(const LowRankPlan* pl, const lrfg_coeff& ac, GaCP& g) {
  const int d = pl->d;
  g.w = {ac.incl_outside, ac.incl_inside - ac.incl_outside};
  g.c = lrfg_coeff{};
  g.c.on_device = 0;
  g.c.rank = 2;
  g.c.weights = g.w.data();
  for (int j = 0; j < d; ++j) {
    const int M = pl->N[j], N = pl->ga_N[j];
    g.f[j].assign((size_t)2 * M, 1.0);
    for (int p = 0; p < M; ++p) {
      const double x = -0.5 + (p + 0.5) / M;
      double chi = 2.0 * ac.incl_size;
      for (int m = 1; m <= N - 1; ++m)
        chi += 2.0 * std::sin(2.0 * kPi * m * ac.incl_size) / (kPi * m) * std::cos(2.0 * kPi * m * x);
      g.f[j][(size_t)M + p] = chi;
    }
    g.c.factors[j] = g.f[j].data();
  }
}

// Correctors kept on the host between the stages of a rank-adaptive solve:
// nE trains of ranks r, carriage j of system e at core[j][e * size_j].
struct HostTrains {
  int r[4] = {1, 1, 1, 1};
  std::vector<double> core[3];
};

namespace {

// One solve at the plan's ranks.  With x0 (FP64 PCG): the truncated PCG
// continues from x0 (zero-padded to the plan's ranks) with its true residual
// T(b - K x0), residuals relative to ||P~^-1 b||; a system whose true
// residual already meets solver_tol stops there.  With xout: the returned
// correctors, copied to the host.
int solve_stage(LowRankPlan* pl, const lrfg_coeff* acs, int nB, const double* E, int nEp, void* ws,
                size_t ws_bytes, hipStream_t s, lrfg_result* outs, const HostTrains* x0, HostTrains* xout) {
  const int d = pl->d;
  const lrfg_problem& P = pl->p;
  if (P.format == LRFG_FORMAT_TUCKER) {
    // microstructures one after another in the same workspace
    int rc = LRFG_OK;
    for (int b = 0; b < nB; ++b) {
      const int r = tucker_solve(pl, acs[b], E, nEp, ws, ws_bytes, s, &outs[b]);
      if (r < 0) return r;
      rc = worse_status(rc, r);
    }
    return rc;
  }
  const int nE = nB * nEp;  // system e = b nEp + f: microstructure b, field f
  if (nB < 1 || nEp < 1 || nE > kMaxSystems) {
    set_error("%d microstructures x %d fields outside [1, %d] systems", nB, nEp, kMaxSystems);
    return LRFG_EINVAL;
  }
  Arena ar;
  ar.base = static_cast<char*>(ws);
  ar.cap = ws_bytes;
  Ctx C;
  carve_ctx(ar, pl, nE, nB == 1 ? 1 : nE, C);
  if (ar.overflow) {
    set_error("workspace too small");
    return LRFG_EWORKSPACE;
  }
  C.s = s;
  const int na = C.na;
  ScopedEvents<3> evs3;
  LRFG_TRY(evs3.create());
  hipEvent_t &ev0 = evs3[0], &ev1 = evs3[1], &ev2 = evs3[2];
  LRFG_HIP(hipEventRecord(ev0, s));
  for (int j = 0; j < d; ++j) {
    double2* tw = const_cast<double2*>(C.f[j].tw);
    LRFG_TRY(fft_dev_upload(pl->mode[j], tw, s, &C.f[j]));
  }
  // ---------------------------------------------------------------- coefficient trains
  int rk[4] = {0, 0, 0, 0};
  const bool ga = pl->ga_N[0] > 0;
  std::vector<GaCP> gcp(ga ? nB : 0);
  for (int b = 0; b < nB; ++b) {
    if (ga) {
      ga_cp(pl, acs[b], gcp[b]);
      LRFG_TRY(load_coeff(C, gcp[b].c, na == 1 ? 0 : b * nEp, rk));
    } else {
      LRFG_TRY(load_coeff(C, acs[b], na == 1 ? 0 : b * nEp, rk));
    }
  }
  for (int j = 1; j < d; ++j) C.a.r[j] = rk[j];
  // admissibility (the coefficient must be positive and finite at every
  // grid point, as for the full grid): truncated or user-given factors can
  // undershoot, which would make the operator indefinite
  // (Ga's double-grid coefficient is a truncated Fourier series: it may dip
  // below zero at the interface while the bilinear form stays positive)
  for (int b = 0; b < nB && !ga; ++b) {
    const double* cores[3];
    for (int j = 0; j < d; ++j) cores[j] = C.a.c[j] + (long long)(na == 1 ? 0 : b * nEp) * C.a.s[j];
    double amin = 0.0;
    long long nonfin = 0;
    LRFG_TRY(tt_coeff_check(d, pl->N, rk, cores, C.dots, s, &amin, &nonfin));
    if (nonfin > 0 || !(amin > 0.0)) {
      set_error("coefficient %d is not admissible: minimum %.6g, %lld non-finite values", b, amin, nonfin);
      return LRFG_ECOEFF;
    }
  }
  if (na > 1) {
    // every field of microstructure b reads its own copy of the train
    for (int j = 0; j < d; ++j) C.a.s[j] = C.a.size(j);
    for (int b = 0; b < nB; ++b)
      for (int f = 1; f < nEp; ++f)
        for (int j = 0; j < d; ++j)
          LRFG_HIP(hipMemcpyAsync(C.a.c[j] + (long long)(b * nEp + f) * C.a.s[j],
                                  C.a.c[j] + (long long)(b * nEp) * C.a.s[j], sizeof(double) * C.a.size(j),
                                  hipMemcpyDeviceToDevice, s));
  }
  // Hadamard output ranks follow the actual coefficient ranks
  for (int j = 1; j < d; ++j) C.kr.r[j] = C.a.r[j] * pl->c[j];
  for (int j = 0; j < d; ++j) C.kr.s[j] = C.kr.size(j);

  // ---------------------------------------------------------------- right-hand side
  // b_e = sum_alpha E_e,alpha D_alpha a_e  (real-space form of -div^ F (a E))
  auto Ev = [&](int e, int al) { return E[(e % nEp) * d + al]; };
  std::vector<double> Ecol(3 * nE, 0.0);
  for (int al = 0; al < d; ++al)
    for (int e = 0; e < nE; ++e) Ecol[al * nE + e] = Ev(e, al);
  LRFG_HIP(hipMemcpyAsync(C.Ecoef, Ecol.data(), sizeof(double) * d * nE, hipMemcpyHostToDevice, s));
  {
    TTB da[3];
    TTTerm terms[3];
    for (int al = 0; al < d; ++al) {
      da[al] = C.a;
      da[al].c[al] = C.acore[al];
      LRFG_TRY(tt_mode_apply(C.a, da[al], al, 0, 0.0, 1.0, C.f[al], na, s));
      terms[al] = TTTerm{&da[al], C.Ecoef + al * nE, 1.0};
    }
    TTB comb = C.comb;
    for (int j = 1; j < d; ++j) comb.r[j] = d * C.a.r[j];
    for (int j = 0; j < d; ++j) comb.s[j] = comb.size(j);
    LRFG_TRY(tt_sum(terms, d, comb, nE, s));
    if (ga) {
      // Ga: the right-hand side's test functions are T_N's (I* of eq.
      // ls_Ga_fourier), projected before the truncation
      TTB cb = comb;
      LRFG_TRY(ga_project(C, cb, nE));
    }
    LRFG_TRY(round_s(C, comb, C.b, P.trunc_tol, nE));
  }
  // scale for the zero-right-hand-side floor: rms(a) |E|, per coefficient train
  std::vector<double> a2(na, 0.0);
  {
    LRFG_TRY(tt_dot(C.a, C.a, C.dots, C.dscr, na, s));
    LRFG_TRY(read_dev(C, C.dots, a2.data(), na));
  }
  double Ntot = 1.0;
  for (int j = 0; j < d; ++j) Ntot *= pl->N[j];
  std::vector<double> floor_abs(nE);
  for (int e = 0; e < nE; ++e) {
    const double rms_a = std::sqrt(std::max(a2[na == 1 ? 0 : e], 0.0) / Ntot);
    double en = 0.0;
    for (int al = 0; al < d; ++al) en += Ev(e, al) * Ev(e, al);
    // real-space norms carry sqrt(|N|) relative to Fourier coefficients
    floor_abs[e] = 1e-14 * rms_a * std::sqrt(en) * std::sqrt(Ntot);
  }
  LRFG_HIP(hipEventRecord(ev1, s));

  // mean of each coefficient train (the E.E term of the energy form)
  std::vector<double> mean_a(na, 0.0);
  {
    // <a, 1>: a train of ones
    TTB one = C.tmp;
    int r1[4] = {1, 1, 1, 1};
    for (int j = 0; j <= 3; ++j) one.r[j] = r1[j];
    for (int j = 0; j < d; ++j) {
      one.s[j] = 0;
      LRFG_TRY(tt_fill(one.c[j], pl->N[j], 1.0, s));
    }
    LRFG_TRY(tt_dot(C.a, one, C.dots, C.dscr, na, s));
    LRFG_TRY(read_dev(C, C.dots, mean_a.data(), na));
    for (auto& v : mean_a) v /= Ntot;
  }

  // Energy form of eq. (homog) for system e's own field: A(x_e) =
  // mean(a)|E_e|^2 + 2 E_e.m1 + sum_alpha <a (.) D_alpha x_e, D_alpha x_e>/|N|,
  // exact for the given trains (no truncation); it bounds A_H E_e.E_e from
  // above and decreases as x_e improves (Sec. 4.3).  For the first n trains
  // of X; train k holds system slot[k] (all of them, in order, without slot).
  auto energy_diag = [&](const TTB& X, std::vector<double>& en, int n, const int* slot) -> int {
    for (int k = 0; k < n; ++k) {
      const int e = slot != nullptr ? slot[k] : k;
      double ee = 0.0;
      for (int al = 0; al < d; ++al) ee += Ev(e, al) * Ev(e, al);
      en[k] = mean_a[na == 1 ? 0 : e] * ee;
    }
    // <a, D_alpha x_k> into dots[2 alpha n + k], <a (.) D_alpha x_k, D_alpha x_k>
    // into dots[(2 alpha + 1) n + k]; one read at the end
    for (int al = 0; al < d; ++al) {
      TTB g = X;
      g.c[al] = C.gcore;
      LRFG_TRY(tt_mode_apply(X, g, al, 0, 0.0, 1.0, C.f[al], n, s));
      LRFG_TRY(tt_dot(C.a, g, C.dots + 2 * al * n, C.dscr, n, s));
      if (d == 3) {
        LRFG_TRY(tt_hadamard(C.a, g, C.kr, n, s, 1));
        const KrMid km = kr_mid(C, g);
        LRFG_TRY(C.rd.kr_dot(C.kr, km, g, C.dots + (2 * al + 1) * n, C.dscr, C.dscr_n, n, s));
      } else {
        LRFG_TRY(tt_hadamard(C.a, g, C.kr, n, s));
        LRFG_TRY(tt_dot(C.kr, g, C.dots + (2 * al + 1) * n, C.dscr, n, s));
      }
    }
    // anisotropic part: E.B E + <x_k, K_B x_k>/|N| into dots[2 d n + k]
    const int nv = (pl->aniso ? 2 * d + 1 : 2 * d) * n;
    if (pl->aniso) {
      TTB W;
      LRFG_TRY(aniso_train(C, X, n, W));
      LRFG_TRY(tt_dot(X, W, C.dots + 2 * d * n, C.dscr, n, s));
    }
    std::vector<double> v((size_t)nv);
    LRFG_TRY(read_dev(C, C.dots, v.data(), nv));
    for (int al = 0; al < d; ++al)
      for (int k = 0; k < n; ++k) {
        const int e = slot != nullptr ? slot[k] : k;
        en[k] += (2.0 * Ev(e, al) * v[(size_t)2 * al * n + k] + v[(size_t)(2 * al + 1) * n + k]) / Ntot;
      }
    if (pl->aniso)
      for (int k = 0; k < n; ++k) {
        const int e = slot != nullptr ? slot[k] : k;
        double eb = 0.0;
        for (int al = 0; al < d; ++al)
          for (int be = 0; be < d; ++be) eb += Ev(e, al) * pl->B[al][be] * Ev(e, be);
        en[k] += eb + v[(size_t)2 * d * n + k] / Ntot;
      }
    return LRFG_OK;
  };

  // ---------------------------------------------------------------- solver
  const int maxit = P.max_iter;
  std::vector<double> hist((size_t)nE * maxit, 0.0);
  std::vector<int> iters(nE, 0), status(nE, LRFG_OK);
  const int patience = (P.solver == LRFG_SOLVER_PCG) ? 5 : 1;
  // truncated PCG: restarts from the best iterate with the true residual
  // before a system is declared stagnant
  const int max_restarts = (P.solver == LRFG_SOLVER_PCG) ? kMaxRestarts : 0;
  // kept ranks of the latest x truncation (bond 1 then bond 2, per system),
  // copied with the residual read, and those of each system's kept iterate
  std::vector<int> kx(2 * nE, 0), kbest(2 * nE, 0);
  // kx[k], kx[nE + k]: kept ranks of train k of the latest x truncation, k < n
  auto fetch_kept = [&](int n) -> int {
    LRFG_HIP(hipMemcpyAsync(kx.data(), C.rd.kept, sizeof(int) * n, hipMemcpyDeviceToHost, s));
    LRFG_HIP(hipMemcpyAsync(kx.data() + nE, C.rd.kept + C.rd.nE, sizeof(int) * n, hipMemcpyDeviceToHost, s));
    return LRFG_OK;
  };
  auto upload_done = [&](const std::vector<int>& hd, int n) -> int {
    LRFG_HIP(hipMemcpyAsync(C.done, hd.data(), sizeof(int) * n, hipMemcpyHostToDevice, s));
    return LRFG_OK;
  };
  // One truncated PCG (or MR) solve of K x = C.b, best iterate into C.xb,
  // in the current precision of the truncation.  Systems with skip[e] keep
  // xb = 0.  res0[e] = ||P~^-1 b_e|| (Fourier-coefficient scaling), st[e] its
  // status; with `record` the relative residuals go to hist and the
  // iteration counts to iters, else the counts are added to iters.
  //
  // Host state is kept per system, device state per slot: slot k holds
  // system perm[k].  With one coefficient train for all systems, a system
  // that finishes leaves the batch: its slot takes the state of the last
  // active slot and the batched steps run on the nA active slots only.  A
  // system's arithmetic does not depend on its slot or on the batch it
  // travels in (per-matrix GEMM splits, one sketch per truncation call), so
  // the results are those of the full batch; the slot order is restored
  // at the end.
  //
  // With xstart (PCG): the iteration starts from that corrector instead of
  // zero (r = T(b - K x), p = z = T(P~^-1 r), the start as the first best
  // iterate, skipped systems keep it) and residuals are relative to ref
  // (the norms ||P~^-1 b|| of the unshifted start).
  auto inner = [&](double tol, int max_it, const std::vector<int>& skip, std::vector<double>& res0,
                   std::vector<int>& st, bool record, const TTB* xstart = nullptr,
                   const std::vector<double>* ref = nullptr) -> int {
    const bool compact = na == 1;
    int nA = nE;
    std::vector<int> perm(nE), slot_done(nE);
    for (int k = 0; k < nE; ++k) perm[k] = k;
    std::vector<int> hdone(skip), since_best(nE, 0), its(nE, 0), restarts(nE, 0);
    // whether the latest restart was followed by a new best iterate: a restart
    // that brings none ends the solve (the residual sits at the rank floor)
    std::vector<char> restart_paid(nE, 1);
    std::vector<double> best(nE, INFINITY), zzh(nE), en(nE), best_en(nE, INFINITY);
    // Once a system's residual has failed to decrease, the FP64 PCG keeps
    // the iterate of lowest energy (the energy form of eq. homog, evaluated
    // exactly on the train): energy - A_H E.E is the squared energy norm of
    // the iterate's error (Sec. 4.3), whereas the recursive residual of a
    // truncated iteration carries the truncation noise and can fall while
    // the error grows.  While the residual keeps decreasing it decides, and
    // no energy is evaluated.
    const bool by_energy = record && P.solver == LRFG_SOLVER_PCG && C.rd.prec == LRFG_PREC_FP64;
    std::vector<char> emode(nE, 0);
    auto push_done = [&]() -> int {
      for (int k = 0; k < nA; ++k) slot_done[k] = hdone[perm[k]];
      return upload_done(slot_done, nA);
    };
    // train k of a batch view
    auto one = [&](const TTB& X, int k) {
      TTB v = X;
      for (int j = 0; j < d; ++j) v.c[j] = X.c[j] + (long long)k * X.s[j];
      return v;
    };
    auto swap_trains = [&](const TTB& X, int a, int b) -> int {
      TTB t0 = one(C.tmp, 0), xa = one(X, a), xb = one(X, b);
      LRFG_TRY(tt_copy(xa, t0, 1, s));
      LRFG_TRY(tt_copy(xb, xa, 1, s));
      LRFG_TRY(tt_copy(t0, xb, 1, s));
      return LRFG_OK;
    };
    auto set_views = [&](int n) {
      C.nE = n;
      for (int j = 0; j < d; ++j) {
        C.r.c[j] = C.xr.c[j] + (long long)n * C.xr.s[j];
        C.q.c[j] = C.pq.c[j] + (long long)n * C.pq.s[j];
      }
    };
    // finished systems leave the active prefix
    auto compact_slots = [&]() -> int {
      int n = nA;
      for (int k = nA - 1; k >= 0; --k) {
        if (!hdone[perm[k]]) continue;
        const int last = n - 1;
        if (k != last) {
          LRFG_TRY(swap_trains(C.x, k, last));
          LRFG_TRY(swap_trains(C.r, k, last));
          LRFG_TRY(swap_trains(C.p, k, last));
          LRFG_TRY(swap_trains(C.xb, k, last));
          LRFG_TRY(swap_trains(C.b, k, last));
          hipLaunchKernelGGL(k_swap2, dim3(1), dim3(1), 0, s, C.rho, k, last);
          LRFG_LAUNCHED();
          std::swap(perm[k], perm[last]);
        }
        --n;
      }
      if (n == nA) return LRFG_OK;
      // r of the active systems moves down to follow x: [x; r] stays one
      // batch of 2 n trains (ascending copies never overwrite a pending source)
      for (int k = 0; k < n; ++k) {
        TTB dst = one(C.xr, n + k);
        LRFG_TRY(tt_copy(one(C.xr, nA + k), dst, 1, s));
      }
      nA = n;
      set_views(nA);
      return push_done();
    };
    // the slot order of the outputs back to the system order
    auto restore_order = [&]() -> int {
      bool moved = false;
      for (int k = 0; k < nE; ++k) moved = moved || perm[k] != k;
      if (moved) {
        for (const TTB* X : {&C.xb, &C.b}) {
          for (int k = 0; k < nE; ++k) {
            TTB dst = one(C.z, perm[k]);
            LRFG_TRY(tt_copy(one(*X, k), dst, 1, s));
          }
          TTB dst = *X;
          LRFG_TRY(tt_copy(C.z, dst, nE, s));
        }
      }
      nA = nE;
      set_views(nE);
      return LRFG_OK;
    };
    for (int e = 0; e < nE; ++e) st[e] = LRFG_OK;
    LRFG_TRY(tt_fill(C.mones, nE, -1.0, s));
    LRFG_TRY(tt_zero(C.xr, 2 * nE, s));
    LRFG_TRY(tt_zero(C.xb, nE, s));
    set_views(nE);
    LRFG_TRY(push_done());
    const bool from_x = xstart != nullptr && P.solver == LRFG_SOLVER_PCG;
    if (from_x) {
      LRFG_TRY(tt_copy(*xstart, C.x, nE, s));
      LRFG_TRY(tt_copy(*xstart, C.xb, nE, s));
      LRFG_TRY(apply_K(C, C.x, C.tmp));
      LRFG_TRY(axpby(C, C.b, C.tmp, C.mones, C.r));
      LRFG_TRY(apply_P(C, C.r, C.z));
      LRFG_TRY(tt_copy(C.z, C.p, nE, s));
      LRFG_TRY(dot(C, C.r, C.z, C.rho));
      LRFG_TRY(dot(C, C.z, C.z, C.zz));
    } else if (P.solver == LRFG_SOLVER_PCG) {
      LRFG_TRY(tt_copy(C.b, C.r, nE, s));
      LRFG_TRY(apply_P(C, C.r, C.z));
      LRFG_TRY(tt_copy(C.z, C.p, nE, s));
      LRFG_TRY(dot(C, C.r, C.z, C.rho));
      LRFG_TRY(dot(C, C.z, C.z, C.zz));
    } else {
      // d = T(P~^-1 b) held in b's place via z; r = d
      LRFG_TRY(apply_P(C, C.b, C.z));
      LRFG_TRY(tt_copy(C.z, C.b, nE, s));
      LRFG_TRY(tt_copy(C.b, C.r, nE, s));
      LRFG_TRY(dot(C, C.r, C.r, C.zz));
    }
    LRFG_TRY(read_dev(C, C.zz, zzh.data(), nE));
    for (int e = 0; e < nE; ++e) {
      res0[e] = from_x ? (*ref)[e] : std::sqrt(std::max(zzh[e], 0.0));
      if (res0[e] <= floor_abs[e]) hdone[e] = 1;
      if (from_x && res0[e] > 0.0) {
        // the start is the first best iterate; reaching the tolerance there
        // ends the system at once
        best[e] = std::sqrt(std::max(zzh[e], 0.0)) / res0[e];
        if (best[e] <= tol) hdone[e] = 1;
      }
    }
    LRFG_TRY(push_done());
    if (compact) LRFG_TRY(compact_slots());
    for (int it = 0; it < max_it; ++it) {
      if (it > 0) gate_point();
      bool all = true;
      for (int e = 0; e < nE; ++e) all = all && hdone[e];
      if (all) break;
      if (P.solver == LRFG_SOLVER_PCG) {
        LRFG_TRY(apply_K(C, C.p, C.q));
        LRFG_TRY(dot(C, C.p, C.q, C.pqd));
        hipLaunchKernelGGL(k_ratio, dim3(1), dim3(kMaxSystems), 0, s, (const double*)C.rho, (const double*)C.pqd,
                           (const int*)C.done, C.alpha, nA);
        hipLaunchKernelGGL(k_pm, dim3(1), dim3(kMaxSystems), 0, s, (const double*)C.alpha, C.coef2, nA);
        LRFG_LAUNCHED();
        LRFG_TRY(update_xr(C));   // x += alpha p ; r -= alpha q
        LRFG_TRY(fetch_kept(nA));
        LRFG_TRY(apply_P(C, C.r, C.z));
        LRFG_TRY(dot(C, C.r, C.z, C.dots));
        LRFG_TRY(dot(C, C.z, C.z, C.zz));
        hipLaunchKernelGGL(k_beta, dim3(1), dim3(kMaxSystems), 0, s, (const double*)C.dots, C.rho,
                           (const int*)C.done, C.beta, nA);
        LRFG_LAUNCHED();
        LRFG_TRY(axpby(C, C.z, C.p, C.beta, C.tmp));
        LRFG_TRY(tt_copy(C.tmp, C.p, nA, s));
      } else {
        // Cr = T(P~^-1 T(K r)); omega = (Cr, r)/(Cr, Cr); u += omega r; r -= omega Cr
        LRFG_TRY(apply_K(C, C.r, C.tmp));
        LRFG_TRY(apply_P(C, C.tmp, C.z));
        LRFG_TRY(dot(C, C.z, C.r, C.dots));
        LRFG_TRY(dot(C, C.z, C.z, C.pqd));
        hipLaunchKernelGGL(k_ratio, dim3(1), dim3(kMaxSystems), 0, s, (const double*)C.dots, (const double*)C.pqd,
                           (const int*)C.done, C.alpha, nA);
        hipLaunchKernelGGL(k_pm, dim3(1), dim3(kMaxSystems), 0, s, (const double*)C.alpha, C.coef2, nA);
        LRFG_LAUNCHED();
        // [p; q] = [r; Cr] then [u; r] += [omega; -omega] [r; Cr]
        LRFG_TRY(tt_copy(C.r, C.p, nA, s));
        LRFG_TRY(tt_copy(C.z, C.q, nA, s));
        LRFG_TRY(update_xr(C));
        LRFG_TRY(fetch_kept(nA));
        LRFG_TRY(dot(C, C.r, C.r, C.zz));
      }
      LRFG_TRY(read_dev(C, C.zz, zzh.data(), nA));
      bool need_en = false;
      for (int k = 0; k < nA; ++k) need_en = need_en || (!hdone[perm[k]] && emode[perm[k]]);
      if (need_en) LRFG_TRY(energy_diag(C.x, en, nA, perm.data()));
      bool changed = false, switched = false;
      unsigned long long improved[4] = {0, 0, 0, 0};  // slots whose x becomes the best iterate
      SysMask restart{{0, 0, 0, 0}};                  // slots restarted from their best iterate
      SysMask to_energy{{0, 0, 0, 0}};                // slots switching to the energy rule
      for (int k = 0; k < nA; ++k) {
        const int e = perm[k];
        if (hdone[e]) continue;
        const double res = std::sqrt(std::max(zzh[k], 0.0)) / res0[e];
        if (record) hist[(size_t)e * maxit + it] = res;
        its[e] = it + 1;
        // an energy step counts when it exceeds solver_tol^2 of the energy:
        // below that it is under the accuracy the tolerance asks for
        const bool better =
            emode[e] ? (std::isfinite(best_en[e]) ? en[k] < best_en[e] - tol * tol * std::fabs(best_en[e]) : true)
                     : res < best[e];
        if (res < best[e]) best[e] = res;
        if (!better && by_energy && !emode[e]) {
          emode[e] = 1;
          switched = true;
          to_energy.m[k >> 6] |= 1ull << (k & 63);
        }
        if (better) {
          if (emode[e]) best_en[e] = en[k];
          since_best[e] = 0;
          restart_paid[e] = 1;
          improved[k >> 6] |= 1ull << (k & 63);
          if (record) {
            kbest[e] = kx[k];
            kbest[nE + e] = kx[nE + k];
          }
        } else {
          ++since_best[e];
        }
        if (res <= tol || std::sqrt(std::max(zzh[k], 0.0)) <= floor_abs[e]) {
          hdone[e] = 1;
          changed = true;
        } else if (since_best[e] >= patience && restarts[e] < max_restarts && restart_paid[e]) {
          // the recursive residual has drifted from b - K x under truncation
          // (Sec. 3.3): restart from the best iterate
          ++restarts[e];
          since_best[e] = 0;
          restart_paid[e] = 0;
          restart.m[k >> 6] |= 1ull << (k & 63);
        } else if (since_best[e] >= patience) {
          hdone[e] = 1;  // stagnation: the residual failed to decrease
          changed = true;
          if (best[e] > tol) st[e] = LRFG_RANK_LIMITED;
        }
      }
      LRFG_TRY(tt_copy_systems(C.x, C.xb, nA, improved, s));
      if (changed) LRFG_TRY(push_done());
      if (switched) {
        // the best iterate so far (by residual) enters the energy rule
        std::vector<double> eb(nA);
        LRFG_TRY(energy_diag(C.xb, eb, nA, perm.data()));
        for (int k = 0; k < nA; ++k)
          if (sys_bit(to_energy, k)) best_en[perm[k]] = eb[k];
      }
      if (restart.m[0] | restart.m[1] | restart.m[2] | restart.m[3]) {
        // residual replacement: x = x_best, r = T(b - K x), z = T(P~^-1 r),
        // p = z, rho = (r, z) for the restarted systems (the others keep
        // their state: the batched steps run for every slot and are
        // copied into the restarted ones only)
        // The restart's truncations draw their sketches from a key space of
        // their own and leave the iteration's sequence as it was, so that a
        // system's iterates do not depend on when other systems of a batch
        // restart (batched solves equal single ones)
        const uint64_t saved = C.rd.counter;
        C.rd.counter = kRestartKeys | ((uint64_t)it << 8);
        LRFG_TRY(apply_K(C, C.xb, C.tmp));
        LRFG_TRY(axpby(C, C.b, C.tmp, C.mones, C.z));
        LRFG_TRY(tt_copy_systems(C.z, C.r, nA, restart.m, s));
        LRFG_TRY(tt_copy_systems(C.xb, C.x, nA, restart.m, s));
        LRFG_TRY(apply_P(C, C.r, C.z));
        C.rd.counter = saved;
        LRFG_TRY(tt_copy_systems(C.z, C.p, nA, restart.m, s));
        LRFG_TRY(dot(C, C.r, C.z, C.dots));
        hipLaunchKernelGGL(k_pick, dim3(1), dim3(kMaxSystems), 0, s, C.rho, (const double*)C.dots, restart, nA);
        LRFG_LAUNCHED();
        // the best residual becomes the true one of the best iterate
        LRFG_TRY(dot(C, C.z, C.z, C.zz));
        LRFG_TRY(read_dev(C, C.zz, zzh.data(), nA));
        if (!by_energy)
          for (int k = 0; k < nA; ++k)
            if (sys_bit(restart, k)) best[perm[k]] = std::sqrt(std::max(zzh[k], 0.0)) / res0[perm[k]];
      }
      if (compact && changed) LRFG_TRY(compact_slots());
    }
    LRFG_TRY(restore_order());
    for (int e = 0; e < nE; ++e) {
      if (!hdone[e]) st[e] = LRFG_NOT_CONVERGED;
      if (skip[e] || res0[e] <= floor_abs[e]) st[e] = LRFG_OK;  // zero right-hand side: zero corrector
      iters[e] = record ? its[e] : iters[e] + its[e];
    }
    return LRFG_OK;
  };

  const std::vector<int> none(nE, 0);
  std::vector<double> res0(nE, 0.0);
  if (P.precision == LRFG_PREC_FP64 && x0 != nullptr) {
    // continue from x0: its carriages zero-padded to this stage's ranks
    for (int j = 0; j < d; ++j) {
      const int a0 = x0->r[j], a1 = x0->r[j + 1], b0 = C.x0.r[j], b1 = C.x0.r[j + 1], Nj = pl->N[j];
      if (a0 > b0 || a1 > b1) {
        set_error("rank-adaptive stage: starting ranks above the stage's");
        return LRFG_EINVAL;
      }
      const long long sa = (long long)a0 * Nj * a1, sb = (long long)b0 * Nj * b1;
      std::vector<double> h((size_t)sb * nE, 0.0);
      for (int e = 0; e < nE; ++e)
        for (int i = 0; i < a0; ++i)
          for (int n = 0; n < Nj; ++n)
            for (int k = 0; k < a1; ++k)
              h[(size_t)(e * sb + ((long long)i * Nj + n) * b1 + k)] =
                  x0->core[j][(size_t)(e * sa + ((long long)i * Nj + n) * a1 + k)];
      LRFG_HIP(hipMemcpyAsync(C.x0.c[j], h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice, s));
      LRFG_HIP(hipStreamSynchronize(s));
    }
    // residuals relative to ||P~^-1 b||, as in a solve from zero
    std::vector<double> zzh(nE), ref(nE);
    LRFG_TRY(apply_P(C, C.b, C.z));
    LRFG_TRY(dot(C, C.z, C.z, C.zz));
    LRFG_TRY(read_dev(C, C.zz, zzh.data(), nE));
    for (int e = 0; e < nE; ++e) ref[e] = std::sqrt(std::max(zzh[e], 0.0));
    LRFG_TRY(inner(P.solver_tol, maxit, none, res0, status, true, &C.x0, &ref));
  } else if (P.precision == LRFG_PREC_FP64) {
    LRFG_TRY(inner(P.solver_tol, maxit, none, res0, status, true));
  } else {
    // Mixed precision (iterative refinement): the inner solves run their
    // contractions with FP32 or BF16 inputs (FP32 accumulation) on the
    // current residual; the correction is added, and the residual
    // r = T(b - K x) recomputed, in FP64.  The truncated operator gives that
    // residual a floor set by the rank cap, so progress is judged by the
    // energy form instead (it decreases to A_H as x improves, Sec. 4.3):
    // the refinement stops when the residual reaches solver_tol or the
    // energy has failed twice in a row to decrease by more than
    // solver_tol^2 of itself, and keeps the lowest-energy iterate.  A BF16
    // inner solve can return a correction that makes the iterate worse (its
    // 8-bit significands perturb the truncated operator by more than the
    // inner tolerance for some fields): the first outer step without an
    // energy gain under BF16 moves the remaining inner solves of the call to
    // FP32.  The FP64 residual history (relative to
    // ||P~^-1 b||) is reported; iters counts inner iterations.
    int lowp = P.precision;
    double tol_in = std::max(P.solver_tol, lowp == LRFG_PREC_MIXED_BF16 ? 1e-2 : 1e-4);
    const double tol_en = std::max(P.solver_tol * P.solver_tol, 1e-15);
    LRFG_TRY(tt_fill(C.ones, nE, 1.0, s));
    LRFG_TRY(tt_fill(C.mones, nE, -1.0, s));
    LRFG_TRY(tt_copy(C.b, C.b0, nE, s));
    LRFG_TRY(tt_zero(C.xa, nE, s));
    LRFG_TRY(tt_zero(C.xbest, nE, s));
    C.rd.prec = LRFG_PREC_FP64;
    std::vector<double> rn0(nE, 0.0), zzh(nE), best(nE, INFINITY), en(nE);
    LRFG_TRY(apply_P(C, C.b0, C.z));
    LRFG_TRY(dot(C, C.z, C.z, C.zz));
    LRFG_TRY(read_dev(C, C.zz, zzh.data(), nE));
    std::vector<int> odone(nE, 0), st_in(nE), capped(nE, 1), no_gain(nE, 0);
    for (int e = 0; e < nE; ++e) {
      rn0[e] = std::sqrt(std::max(zzh[e], 0.0));
      if (rn0[e] <= floor_abs[e]) {
        odone[e] = 1;
        capped[e] = 0;
      }
    }
    std::vector<double> r0_in(nE);
    for (int outer = 0; outer < maxit; ++outer) {
      bool all = true;
      for (int e = 0; e < nE; ++e) all = all && odone[e];
      if (all) break;
      C.rd.prec = lowp;
      LRFG_TRY(inner(tol_in, maxit, odone, r0_in, st_in, false));
      C.rd.prec = LRFG_PREC_FP64;
      LRFG_TRY(axpby(C, C.xa, C.xb, C.ones, C.tmp));   // x <- T(x + delta)
      LRFG_TRY(fetch_kept(nE));
      LRFG_TRY(tt_copy(C.tmp, C.xa, nE, s));
      LRFG_TRY(apply_K(C, C.xa, C.tmp));               // r <- T(b - K x)
      LRFG_TRY(axpby(C, C.b0, C.tmp, C.mones, C.b));
      LRFG_TRY(apply_P(C, C.b, C.z));
      LRFG_TRY(dot(C, C.z, C.z, C.zz));
      LRFG_TRY(read_dev(C, C.zz, zzh.data(), nE));
      LRFG_TRY(energy_diag(C.xa, en, nE, nullptr));
      bool escalate = false;
      unsigned long long improved[4] = {0, 0, 0, 0};
      for (int e = 0; e < nE; ++e) {
        if (odone[e]) continue;
        const double rel = std::sqrt(std::max(zzh[e], 0.0)) / rn0[e];
        hist[(size_t)e * maxit + outer] = rel;
        const bool gain = en[e] < best[e] - tol_en * std::fabs(en[e]);
        if (en[e] < best[e]) {
          best[e] = en[e];
          improved[e >> 6] |= 1ull << (e & 63);
          kbest[e] = kx[e];
          kbest[nE + e] = kx[nE + e];
        }
        no_gain[e] = gain ? 0 : no_gain[e] + 1;
        if (!gain && lowp == LRFG_PREC_MIXED_BF16) escalate = true;
        if (rel <= P.solver_tol || no_gain[e] >= 2) {
          odone[e] = 1;
          capped[e] = 0;
        }
      }
      LRFG_TRY(tt_copy_systems(C.xa, C.xbest, nE, improved, s));
      if (escalate) {
        lowp = LRFG_PREC_MIXED_FP32;
        tol_in = std::max(P.solver_tol, 1e-4);
        for (int e = 0; e < nE; ++e) no_gain[e] = 0;
      }
    }
    for (int e = 0; e < nE; ++e) status[e] = capped[e] ? LRFG_NOT_CONVERGED : LRFG_OK;
    LRFG_TRY(tt_copy(C.xbest, C.xb, nE, s));
    res0 = rn0;
  }

  // ---------------------------------------------------------------- A_H (eq. homog)
  // A_H[i][j] = mean(a) E_i.E_j + sum_alpha (E_i,alpha m1[j] + E_j,alpha m1[i] + m2[i][j])
  // m1[e][alpha] = <a, D_alpha x_e>/|N|, m2[i][j][alpha] = <a (.) D_alpha x_i, D_alpha x_j>/|N|,
  // i and j fields of the same microstructure
  std::vector<double> m1((size_t)nE * d), m2((size_t)nE * nEp * d);
  for (int al = 0; al < d; ++al) {
    TTB g = C.xb;
    g.c[al] = C.gcore;
    LRFG_TRY(tt_mode_apply(C.xb, g, al, 0, 0.0, 1.0, C.f[al], nE, s));
    // m1: <a_e, g_e>
    LRFG_TRY(tt_dot(C.a, g, C.dots, C.dscr, nE, s));
    std::vector<double> v(nE);
    LRFG_TRY(read_dev(C, C.dots, v.data(), nE));
    for (int e = 0; e < nE; ++e) m1[(size_t)e * d + al] = v[e] / Ntot;
    // m2: <a (.) g_i, g_j> for every pair within each microstructure
    std::vector<double> w2((size_t)nE * nEp);
    if (d == 3) {
      // per microstructure b and field j: the nEp systems of b against g_j
      LRFG_TRY(tt_hadamard(C.a, g, C.kr, nE, s, 1));
      std::vector<double> wj(nEp);
      for (int b = 0; b < nB; ++b) {
        TTB kb = C.kr, gb = g, gj = g;
        for (int j = 0; j < d; ++j) {
          kb.c[j] = j == 1 ? nullptr : C.kr.c[j] + (long long)b * nEp * C.kr.s[j];
          gb.c[j] = g.c[j] + (long long)b * nEp * g.s[j];
        }
        KrMid km = kr_mid(C, gb);
        km.a = C.a.c[1] + (long long)(na == 1 ? 0 : b * nEp) * C.a.s[1];
        for (int j = 0; j < nEp; ++j) {
          for (int q = 0; q < d; ++q) {
            gj.c[q] = g.c[q] + (long long)(b * nEp + j) * g.s[q];
            gj.s[q] = 0;
          }
          LRFG_TRY(C.rd.kr_dot(kb, km, gj, C.dots, C.dscr, C.dscr_n, nEp, s));
          LRFG_TRY(read_dev(C, C.dots, wj.data(), nEp));
          for (int i = 0; i < nEp; ++i) w2[(size_t)(b * nEp + i) * nEp + j] = wj[i];
        }
      }
    } else {
      LRFG_TRY(tt_hadamard(C.a, g, C.kr, nE, s));
      LRFG_TRY(tt_dot(C.kr, g, C.dots, C.dscr, nE, s, nEp));
      LRFG_TRY(read_dev(C, C.dots, w2.data(), nE * nEp));
    }
    for (size_t k = 0; k < w2.size(); ++k) m2[k * d + al] = w2[k] / Ntot;
  }
  // anisotropic part: mb[i][j] = E_i.B E_j + <x_j, K_B x_i>/|N|, per microstructure
  std::vector<double> mb((size_t)nE * nEp, 0.0);
  if (pl->aniso) {
    TTB W;
    LRFG_TRY(aniso_train(C, C.xb, nE, W));
    std::vector<double> wj(nEp);
    for (int b = 0; b < nB; ++b) {
      TTB xb = C.xb, w1 = W;
      for (int q = 0; q < d; ++q) xb.c[q] = C.xb.c[q] + (long long)b * nEp * C.xb.s[q];
      for (int j = 0; j < nEp; ++j) {
        for (int q = 0; q < d; ++q) {
          w1.c[q] = W.c[q] + (long long)(b * nEp + j) * W.s[q];
          w1.s[q] = 0;
        }
        LRFG_TRY(tt_dot(xb, w1, C.dots, C.dscr, nEp, s));
        LRFG_TRY(read_dev(C, C.dots, wj.data(), nEp));
        for (int i = 0; i < nEp; ++i) {
          double eb = 0.0;
          for (int al = 0; al < d; ++al)
            for (int be = 0; be < d; ++be) eb += E[i * d + al] * pl->B[al][be] * E[j * d + be];
          mb[(size_t)(b * nEp + i) * nEp + j] = eb + wj[i] / Ntot;
        }
      }
    }
  }
  // final ranks: those the truncation kept for each system's returned iterate
  const std::vector<int>& kept = kbest;
  LRFG_HIP(hipEventRecord(ev2, s));
  LRFG_HIP(hipStreamSynchronize(s));
  float ms_setup = 0.f, ms_solve = 0.f;
  LRFG_HIP(hipEventElapsedTime(&ms_setup, ev0, ev1));
  LRFG_HIP(hipEventElapsedTime(&ms_solve, ev1, ev2));
  int rc = LRFG_OK;
  for (int b = 0; b < nB; ++b) {
    lrfg_result* out = &outs[b];
    const double ma = mean_a[na == 1 ? 0 : b * nEp];
    for (int i = 0; i < nEp; ++i) {
      const int ei = b * nEp + i;
      for (int j = 0; j < nEp; ++j) {
        const int ej = b * nEp + j;
        double v = mb[(size_t)ei * nEp + j];
        for (int al = 0; al < d; ++al) {
          const double xi = E[i * d + al], xj = E[j * d + al];
          v += ma * xi * xj + xi * m1[(size_t)ej * d + al] + xj * m1[(size_t)ei * d + al] +
               m2[((size_t)ei * nEp + j) * d + al];
        }
        if (out->A_H) out->A_H[i * nEp + j] = v;
      }
      if (out->iters) out->iters[i] = iters[ei];
      if (out->status) out->status[i] = status[ei];
      rc = worse_status(rc, status[ei]);
      if (out->res_hist)
        for (int k = 0; k < maxit; ++k) out->res_hist[(size_t)i * maxit + k] = hist[(size_t)ei * maxit + k];
      if (out->ranks) {
        out->ranks[i * (d + 1)] = 1;
        out->ranks[i * (d + 1) + d] = 1;
        if (d == 3) {
          out->ranks[i * (d + 1) + 1] = kept[ei];
          out->ranks[i * (d + 1) + 2] = kept[nE + ei];
        } else {
          out->ranks[i * (d + 1) + 1] = kept[ei];
        }
      }
    }
    out->setup_ms = ms_setup;
    out->solve_ms = ms_solve;
  }
  if (xout != nullptr) {
    for (int j = 0; j <= d; ++j) xout->r[j] = C.xb.r[j];
    for (int j = 0; j < d; ++j) {
      xout->core[j].resize((size_t)C.xb.size(j) * nE);
      for (int e = 0; e < nE; ++e)
        LRFG_HIP(hipMemcpyAsync(xout->core[j].data() + (size_t)e * C.xb.size(j), C.xb.c[j] + (long long)e * C.xb.s[j],
                                sizeof(double) * C.xb.size(j), hipMemcpyDeviceToHost, s));
    }
    LRFG_HIP(hipStreamSynchronize(s));
  }
  return rc;
}

}  // namespace

// Rank-adaptive solve (Sec. 4.2: start at a low solution rank and raise it
// during the iterations).  Stages at rank caps c_0 = rank_start,
// c_{k+1} = min(rank_cap, max(c_k + 1, ceil(1.5 c_k))), each a truncated PCG
// at its cap; the first starts from zero, every later one continues from the
// previous stage's corrector (zero-padded to the larger ranks) with its true
// residual, so a system that a stage's recursive residual called converged
// is checked again (and stops at once if it is).  A stage ends for a system
// at solver_tol, stagnant at the rank floor of its cap, or at max_iter (per
// stage).  A_H, the statuses and the ranks are those of the last stage, the
// iteration counts and times add up over the stages, and res_hist holds the
// first stage's history.
int lowrank_solve(LowRankPlan* pl, const lrfg_coeff* acs, int nB, const double* E, int nEp, void* ws,
                  size_t ws_bytes, hipStream_t s, lrfg_result* outs) {
  const lrfg_problem& P = pl->p;
  const bool adaptive = P.rank_start > 0 && P.rank_start < P.rank_cap && P.format != LRFG_FORMAT_TUCKER;
  if (!adaptive) return solve_stage(pl, acs, nB, E, nEp, ws, ws_bytes, s, outs, nullptr, nullptr);
  std::vector<int> caps;
  for (int c = P.rank_start; c < P.rank_cap; c = std::max(c + 1, (int)std::ceil(1.5 * c))) caps.push_back(c);
  caps.push_back(P.rank_cap);
  const int nE = nB * nEp;
  HostTrains xa, xb;
  std::vector<int> its(nE, 0), st_it(nE), st_st(nE);
  std::vector<double> setup(nB, 0.0), solve(nB, 0.0);
  std::vector<lrfg_result> r(nB);
  int rc = LRFG_OK;
  for (size_t k = 0; k < caps.size(); ++k) {
    LowRankPlan stp = *pl;
    stp.p.rank_cap = caps[k];
    stp.p.rank_start = 0;
    plan_ranks(stp);
    const bool last = k + 1 == caps.size();
    for (int b = 0; b < nB; ++b) {
      r[b] = outs[b];
      r[b].iters = st_it.data() + b * nEp;
      r[b].status = st_st.data() + b * nEp;
      if (k > 0) r[b].res_hist = nullptr;  // the first stage's history stays
    }
    rc = solve_stage(&stp, acs, nB, E, nEp, ws, ws_bytes, s, r.data(), k > 0 ? &xa : nullptr, last ? nullptr : &xb);
    if (rc < 0) return rc;
    for (int e = 0; e < nE; ++e) its[e] += st_it[e];
    for (int b = 0; b < nB; ++b) {
      setup[b] += r[b].setup_ms;
      solve[b] += r[b].solve_ms;
    }
    std::swap(xa, xb);
  }
  for (int b = 0; b < nB; ++b) {
    for (int i = 0; i < nEp; ++i) {
      if (outs[b].iters) outs[b].iters[i] = its[b * nEp + i];
      if (outs[b].status) outs[b].status[i] = st_st[b * nEp + i];
    }
    outs[b].setup_ms = setup[b];
    outs[b].solve_ms = solve[b];
  }
  return rc;
}

// ====================================================================== Tucker solve
// The same truncated PCG / MR as the train path with the corrector held in
// Tucker form (Sec. 3.1.2, Appendix A.2), d = 3, one microstructure: the
// derivative acts on frame alpha, the material law is the Khatri-Rao /
// Kronecker product with the coefficient (given in CP form: frames = the
// factors, superdiagonal core of the weights), the preconditioner's M heat-
// kernel terms act on all three frames (block sum of M Tuckers), and every
// rank-raising step is followed by the Tucker truncation.
namespace {

// Coefficient in CP form as a Tucker tensor: frames f_j^T (N_j x R),
// superdiagonal core G[t][t][t] = w[t].
__global__ void k_cp_to_tucker(const double* __restrict__ w, const double* __restrict__ f0,
                               const double* __restrict__ f1, const double* __restrict__ f2, int R, int N0, int N1,
                               int N2, double* __restrict__ u0, double* __restrict__ u1, double* __restrict__ u2,
                               double* __restrict__ G) {
  const long long n0 = (long long)N0 * R, n1 = (long long)N1 * R, n2 = (long long)N2 * R;
  const long long ng = (long long)R * R * R;
  const long long tot = n0 + n1 + n2 + ng;
  for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < tot;
       idx += (long long)gridDim.x * blockDim.x) {
    if (idx < n0) {
      const long long n = idx / R, t = idx % R;
      u0[idx] = f0[t * N0 + n];
    } else if (idx < n0 + n1) {
      const long long i = idx - n0, n = i / R, t = i % R;
      u1[i] = f1[t * N1 + n];
    } else if (idx < n0 + n1 + n2) {
      const long long i = idx - n0 - n1, n = i / R, t = i % R;
      u2[i] = f2[t * N2 + n];
    } else {
      const long long i = idx - n0 - n1 - n2;
      const long long t3 = i % R, t2 = (i / R) % R, t1 = i / ((long long)R * R);
      G[i] = (t1 == t2 && t2 == t3) ? w[t1] : 0.0;
    }
  }
}

struct TkCtx {
  LowRankPlan* pl;
  int nE;
  hipStream_t s;
  FftDev f[3];
  TkRounder rd;
  TKB a;                    // coefficient (shared, stride 0)
  TKB xr, pq, x, r, p, q;   // [x; r], [p; q] and their halves
  TKB z, xb, b, tmp;
  TKB b0, xa, xbest;        // refinement: right-hand side, iterate, best iterate
  TKB kr;                   // a (.) D_alpha v, d nE tensors
  TKB h;                    // truncated material terms, d nE tensors
  TKB comb;                 // block sums, 2 nE tensors (capacity ranks)
  double* gframe;           // frame buffer for D_alpha v
  double* hframe[3];        // frame buffers for D_alpha^T h_alpha
  double* aframe[3];        // frames of D_alpha a (right-hand side)
  double *dots, *rho, *pqd, *alpha, *beta, *zz, *Ecoef, *coef2, *dscr;
  double *ones, *mones;
  double* stage;            // host CP coefficient staged on the device
  double* wchk;             // admissibility check: U1 x_1 core
  int* done;
  int cap[3];
  int ra;
};

int tk_carve(Arena& ar, LowRankPlan* pl, int nE, TkCtx& C) {
  C.pl = pl;
  C.nE = nE;
  const int* N = pl->N;
  int rc[3] = {pl->c[1], pl->c[2], pl->c[3]};
  int ra[3] = {pl->ra, pl->ra, pl->ra};
  C.ra = pl->ra;
  for (int j = 0; j < 3; ++j) C.f[j].tw = ar.take<double2>(N[j]);
  C.a = tk_alloc(ar, N, ra, 1);
  for (int j = 0; j < 3; ++j) C.a.sU[j] = 0;
  C.a.sG = 0;
  C.xr = tk_alloc(ar, N, rc, 2 * nE);
  C.pq = tk_alloc(ar, N, rc, 2 * nE);
  C.x = C.xr;
  C.r = C.xr;
  C.p = C.pq;
  C.q = C.pq;
  for (int j = 0; j < 3; ++j) {
    C.r.U[j] = C.xr.U[j] + (long long)nE * C.xr.sU[j];
    C.q.U[j] = C.pq.U[j] + (long long)nE * C.pq.sU[j];
  }
  C.r.G = C.xr.G + (long long)nE * C.xr.sG;
  C.q.G = C.pq.G + (long long)nE * C.pq.sG;
  C.z = tk_alloc(ar, N, rc, nE);
  C.xb = tk_alloc(ar, N, rc, nE);
  C.b = tk_alloc(ar, N, rc, nE);
  C.tmp = tk_alloc(ar, N, rc, nE);
  if (pl->p.precision != LRFG_PREC_FP64) {
    C.b0 = tk_alloc(ar, N, rc, nE);
    C.xa = tk_alloc(ar, N, rc, nE);
    C.xbest = tk_alloc(ar, N, rc, nE);
  }
  C.h = tk_alloc(ar, N, rc, 3 * nE);
  int rkr[3], cap[3];
  for (int j = 0; j < 3; ++j) {
    rkr[j] = ra[j] * rc[j];
    int m = 3 * rc[j];
    m = std::max(m, pl->M * rc[j]);
    m = std::max(m, 2 * rc[j]);
    m = std::max(m, 3 * ra[j]);
    cap[j] = m;
    C.cap[j] = m;
  }
  // Khatri-Rao frames of the d nE material products; their Kronecker cores
  // are never formed inside the iterations (the truncation contracts the
  // factor cores), only once per direction for A_H (nE cores)
  for (int j = 0; j < 3; ++j) {
    C.kr.N[j] = N[j];
    C.kr.r[j] = rkr[j];
    C.kr.sU[j] = C.kr.usize(j);
    C.kr.U[j] = ar.take<double>((size_t)C.kr.sU[j] * 3 * nE);
  }
  C.kr.sG = C.kr.gsize();
  C.kr.G = ar.take<double>((size_t)C.kr.sG * nE);
  C.comb = tk_alloc(ar, N, cap, 2 * nE);
  long long fmax = 0;
  for (int j = 0; j < 3; ++j) fmax = std::max(fmax, (long long)N[j] * rc[j]);
  C.gframe = ar.take<double>((size_t)fmax * nE);
  for (int al = 0; al < 3; ++al) C.hframe[al] = ar.take<double>((size_t)fmax * nE);
  long long amax = 0;
  for (int j = 0; j < 3; ++j) amax = std::max(amax, (long long)N[j] * ra[j]);
  for (int al = 0; al < 3; ++al) C.aframe[al] = ar.take<double>((size_t)amax);
  TkRounder& R = C.rd;
  R.nE = 3 * nE;
  for (int j = 0; j < 3; ++j) {
    R.N[j] = N[j];
    R.Rmax[j] = std::max(cap[j], rkr[j]);
  }
  R.oversample = pl->over;
  R.seed = pl->p.seed;
  R.Lmax = std::min(std::max(rc[0], std::max(rc[1], rc[2])) + pl->over, kMaxEig);
  R.kron = true;
  R.carve(ar);
  C.dots = ar.take<double>((size_t)3 * nE + 64);
  C.rho = ar.take<double>(nE);
  C.pqd = ar.take<double>(nE);
  C.alpha = ar.take<double>(nE);
  C.beta = ar.take<double>(nE);
  C.zz = ar.take<double>(nE);
  C.Ecoef = ar.take<double>((size_t)3 * nE);
  C.coef2 = ar.take<double>((size_t)2 * nE);
  C.done = ar.take<int>(nE);
  C.ones = ar.take<double>(nE);
  C.mones = ar.take<double>(nE);
  C.stage = ar.take<double>((size_t)pl->ra * (1 + N[0] + N[1] + N[2]));
  C.wchk = ar.take<double>((size_t)N[0] * pl->ra * pl->ra);
  size_t dn = tk_dot_scratch(C.kr, C.z, 3 * nE);  // A_H cross terms: up to 3 pairs per system
  dn = std::max(dn, tk_dot_scratch(C.a, C.a, nE));
  dn = std::max(dn, tk_dot_scratch(C.z, C.z, nE));
  C.dscr = ar.take<double>(dn);
  return LRFG_OK;
}

// TKB view of a sub-batch (systems off.., stride kept)
TKB tk_sub(const TKB& x, long long off) {
  TKB y = x;
  for (int j = 0; j < 3; ++j) y.U[j] = x.U[j] + off * x.sU[j];
  y.G = x.G + off * x.sG;
  return y;
}

// comb view with ranks rr and compact strides
TKB tk_comb(const TkCtx& C, const int rr[3]) {
  TKB c = C.comb;
  for (int j = 0; j < 3; ++j) {
    c.r[j] = rr[j];
    c.sU[j] = c.usize(j);
  }
  c.sG = c.gsize();
  return c;
}

int tk_apply_K(TkCtx& C, const TKB& v, TKB& out) {
  const int nE = C.nE;
  for (int al = 0; al < 3; ++al) {
    TKB g = v;
    g.U[al] = C.gframe;
    LRFG_TRY(tk_mode_apply(v, g, al, 0, 0.0, 1.0, C.f[al], nE, C.s));
    TKB kra = tk_sub(C.kr, (long long)al * nE);
    LRFG_TRY(tk_hadamard_frames(C.a, g, kra, nE, C.s));
  }
  TKB kr = C.kr;
  for (int j = 0; j < 3; ++j) {
    kr.r[j] = C.a.r[j] * v.r[j];
    kr.sU[j] = kr.usize(j);
  }
  // core of system al nE + e: G_a (x) G_v[e] (the derivative acts on frames)
  const KronCore kc{C.a.G, C.a.sG, {C.a.r[0], C.a.r[1], C.a.r[2]}, v.G, v.sG, nE, {v.r[0], v.r[1], v.r[2]}};
  LRFG_TRY(C.rd.round(kr, C.h, 0.0, C.s, 3 * nE, &kc));
  TKB hd[3];
  TKTerm terms[3];
  for (int al = 0; al < 3; ++al) {
    TKB ha = tk_sub(C.h, (long long)al * nE);
    hd[al] = ha;
    hd[al].U[al] = C.hframe[al];
    LRFG_TRY(tk_mode_apply(ha, hd[al], al, 0, 0.0, -1.0, C.f[al], nE, C.s));
    terms[al] = TKTerm{&hd[al], nullptr, 1.0};
  }
  int rr[3];
  for (int j = 0; j < 3; ++j) rr[j] = 3 * v.r[j];
  TKB comb = tk_comb(C, rr);
  LRFG_TRY(tk_sum(terms, 3, comb, nE, C.s));
  return C.rd.round(comb, out, C.pl->p.trunc_tol, C.s, nE);
}

// out = T(P~^-1 v): term m has all three frames through the heat kernel
// exp(-t_m k^2) (frame 0 also scaled by w_m / 4 pi^2), written straight into
// the block frames of the sum; the core blocks are copies of v's core.
int tk_apply_P(TkCtx& C, const TKB& v, TKB& out) {
  const int nE = C.nE;
  const int M = C.pl->M;
  int rr[3];
  for (int j = 0; j < 3; ++j) rr[j] = M * v.r[j];
  TKB comb = tk_comb(C, rr);
  std::vector<double> sc(M), one(M, 1.0);
  for (int m = 0; m < M; ++m) sc[m] = C.pl->w[m] / (4.0 * kPi * kPi);
  for (int j = 0; j < 3; ++j) {
    LRFG_TRY(launch_mode_op_blocks(v.U[j], v.sU[j], 1, v.r[j], nE, comb.U[j], comb.sU[j], comb.r[j], false, true, M,
                                   C.pl->t.data(), j == 0 ? sc.data() : one.data(), C.f[j], C.s));
  }
  LRFG_HIP(hipMemsetAsync(comb.G, 0, sizeof(double) * comb.gsize() * nE, C.s));
  for (int m = 0; m < M; ++m) {
    const int o[3] = {m * v.r[0], m * v.r[1], m * v.r[2]};
    LRFG_TRY(tk_place_core(v, nullptr, 1.0, comb, o, nE, C.s));
  }
  return C.rd.round(comb, out, C.pl->p.trunc_tol, C.s, nE);
}

int tk_update_xr(TkCtx& C) {
  TKTerm t[2] = {TKTerm{&C.xr, nullptr, 1.0}, TKTerm{&C.pq, C.coef2, 1.0}};
  int rr[3];
  for (int j = 0; j < 3; ++j) rr[j] = 2 * C.xr.r[j];
  TKB comb = tk_comb(C, rr);
  LRFG_TRY(tk_sum(t, 2, comb, 2 * C.nE, C.s));
  return C.rd.round(comb, C.xr, C.pl->p.trunc_tol, C.s, 2 * C.nE);
}

int tk_axpby(TkCtx& C, const TKB& x, const TKB& y, const double* cb, TKB& out) {
  TKTerm t[2] = {TKTerm{&x, nullptr, 1.0}, TKTerm{&y, cb, 1.0}};
  int rr[3];
  for (int j = 0; j < 3; ++j) rr[j] = x.r[j] + y.r[j];
  TKB comb = tk_comb(C, rr);
  LRFG_TRY(tk_sum(t, 2, comb, C.nE, C.s));
  return C.rd.round(comb, out, C.pl->p.trunc_tol, C.s, C.nE);
}

int tk_read(TkCtx& C, const double* dptr, double* host, int n) {
  LRFG_HIP(hipMemcpyAsync(host, dptr, sizeof(double) * n, hipMemcpyDeviceToHost, C.s));
  LRFG_HIP(hipStreamSynchronize(C.s));
  return LRFG_OK;
}

}  // namespace

size_t tucker_workspace_bytes(const LowRankPlan* lr, int max_nE) {
  Arena ar;
  TkCtx C;
  tk_carve(ar, const_cast<LowRankPlan*>(lr), max_nE, C);
  return ar.used + 1024;
}

int tucker_solve(LowRankPlan* pl, const lrfg_coeff& ac, const double* E, int nE, void* ws, size_t ws_bytes,
                 hipStream_t s, lrfg_result* out) {
  const lrfg_problem& P = pl->p;
  if (nE < 1 || nE > 3) {
    set_error("Tucker solve: nE in [1, 3]");
    return LRFG_EINVAL;
  }
  Arena ar;
  ar.base = static_cast<char*>(ws);
  ar.cap = ws_bytes;
  TkCtx C;
  tk_carve(ar, pl, nE, C);
  if (ar.overflow) {
    set_error("workspace too small");
    return LRFG_EWORKSPACE;
  }
  C.s = s;
  ScopedEvents<3> evs3;
  LRFG_TRY(evs3.create());
  hipEvent_t &ev0 = evs3[0], &ev1 = evs3[1], &ev2 = evs3[2];
  LRFG_HIP(hipEventRecord(ev0, s));
  for (int j = 0; j < 3; ++j) {
    double2* tw = const_cast<double2*>(C.f[j].tw);
    LRFG_TRY(fft_dev_upload(pl->mode[j], tw, s, &C.f[j]));
  }
  // ---------------------------------------------------------------- coefficient
  // CP form: frames f_j^T and a superdiagonal core of the weights; Tucker
  // form: frames and core as given.
  int ra3[3];
  if (ac.weights != nullptr) {
    const int Ra = ac.rank;
    if (Ra < 1 || Ra > pl->ra) {
      set_error("coefficient rank %d outside [1, coeff_rank = %d]", Ra, pl->ra);
      return LRFG_EINVAL;
    }
    const double* w = ac.weights;
    const double* f[3] = {ac.factors[0], ac.factors[1], ac.factors[2]};
    if (!ac.on_device) {
      double* st = C.stage;
      LRFG_HIP(hipMemcpyAsync(st, w, sizeof(double) * Ra, hipMemcpyHostToDevice, s));
      size_t off = Ra;
      for (int j = 0; j < 3; ++j) {
        LRFG_HIP(hipMemcpyAsync(st + off, ac.factors[j], sizeof(double) * Ra * pl->N[j], hipMemcpyHostToDevice, s));
        f[j] = st + off;
        off += (size_t)Ra * pl->N[j];
      }
      w = st;
    }
    for (int j = 0; j < 3; ++j) ra3[j] = Ra;
    const long long tot = (long long)(pl->N[0] + pl->N[1] + pl->N[2]) * Ra + (long long)Ra * Ra * Ra;
    hipLaunchKernelGGL(k_cp_to_tucker, dim3((int)std::min<long long>(4096, (tot + 255) / 256)), dim3(256), 0, s, w,
                       f[0], f[1], f[2], Ra, pl->N[0], pl->N[1], pl->N[2], C.a.U[0], C.a.U[1], C.a.U[2], C.a.G);
    LRFG_LAUNCHED();
  } else if (ac.tucker_core != nullptr) {
    for (int j = 0; j < 3; ++j) {
      ra3[j] = ac.tucker_ranks[j];
      if (ra3[j] < 1 || ra3[j] > pl->ra) {
        set_error("Tucker coefficient rank %d outside [1, coeff_rank = %d]", ra3[j], pl->ra);
        return LRFG_EINVAL;
      }
    }
    const hipMemcpyKind kind = ac.on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    for (int j = 0; j < 3; ++j)
      LRFG_HIP(hipMemcpyAsync(C.a.U[j], ac.tucker_frames[j], sizeof(double) * pl->N[j] * ra3[j], kind, s));
    LRFG_HIP(hipMemcpyAsync(C.a.G, ac.tucker_core, sizeof(double) * ra3[0] * ra3[1] * ra3[2], kind, s));
  } else {
    set_error("the Tucker path takes the coefficient in CP or Tucker form");
    return LRFG_EUNSUPPORTED;
  }
  for (int j = 0; j < 3; ++j) C.a.r[j] = ra3[j];
  {
    // admissibility: positive and finite at every grid point
    double amin = 0.0;
    long long nonfin = 0;
    const double* U[3] = {C.a.U[0], C.a.U[1], C.a.U[2]};
    LRFG_TRY(tucker_coeff_check(pl->N, ra3, C.a.G, U, C.wchk, C.dots, s, &amin, &nonfin));
    if (nonfin > 0 || !(amin > 0.0)) {
      set_error("coefficient is not admissible: minimum %.6g, %lld non-finite values", amin, nonfin);
      return LRFG_ECOEFF;
    }
  }
  for (int j = 0; j < 3; ++j) {
    C.kr.r[j] = ra3[j] * C.xr.r[j];
    C.kr.sU[j] = C.kr.usize(j);
  }
  C.kr.sG = C.kr.gsize();
  // ---------------------------------------------------------------- right-hand side
  std::vector<double> Ecol(3 * nE, 0.0);
  for (int al = 0; al < 3; ++al)
    for (int e = 0; e < nE; ++e) Ecol[al * nE + e] = E[e * 3 + al];
  LRFG_HIP(hipMemcpyAsync(C.Ecoef, Ecol.data(), sizeof(double) * 3 * nE, hipMemcpyHostToDevice, s));
  {
    TKB da[3];
    TKTerm terms[3];
    for (int al = 0; al < 3; ++al) {
      da[al] = C.a;
      da[al].U[al] = C.aframe[al];
      LRFG_TRY(tk_mode_apply(C.a, da[al], al, 0, 0.0, 1.0, C.f[al], 1, s));
      terms[al] = TKTerm{&da[al], C.Ecoef + al * nE, 1.0};
    }
    int rr[3] = {3 * ra3[0], 3 * ra3[1], 3 * ra3[2]};
    TKB comb = tk_comb(C, rr);
    LRFG_TRY(tk_sum(terms, 3, comb, nE, s));
    LRFG_TRY(C.rd.round(comb, C.b, P.trunc_tol, s, nE));
  }
  double a2 = 0.0;
  LRFG_TRY(tk_dot(C.a, C.a, C.dots, C.dscr, 1, s));
  LRFG_TRY(tk_read(C, C.dots, &a2, 1));
  double Ntot = (double)pl->N[0] * pl->N[1] * pl->N[2];
  const double rms_a = std::sqrt(std::max(a2, 0.0) / Ntot);
  std::vector<double> floor_abs(nE);
  for (int e = 0; e < nE; ++e) {
    double en = 0.0;
    for (int al = 0; al < 3; ++al) en += E[e * 3 + al] * E[e * 3 + al];
    floor_abs[e] = 1e-14 * rms_a * std::sqrt(en) * std::sqrt(Ntot);
  }
  LRFG_HIP(hipEventRecord(ev1, s));
  // mean of the coefficient (the E.E term of the energy form)
  double mean_a = 0.0;
  {
    TKB one = C.tmp;
    for (int j = 0; j < 3; ++j) {
      one.r[j] = 1;
      one.sU[j] = 0;
      LRFG_TRY(tt_fill(one.U[j], pl->N[j], 1.0, s));
    }
    one.sG = 0;
    LRFG_TRY(tt_fill(one.G, 1, 1.0, s));
    LRFG_TRY(tk_dot(C.a, one, C.dots, C.dscr, 1, s));
    LRFG_TRY(tk_read(C, C.dots, &mean_a, 1));
    mean_a /= Ntot;
  }
  // Energy form of eq. (homog) for system e's own field (an upper bound of
  // A_H E_e.E_e that decreases as x_e improves, Sec. 4.3), exact for the
  // given Tucker tensors: the Hadamard core is formed for nE systems here.
  auto energy_diag = [&](const TKB& X, std::vector<double>& en) -> int {
    for (int e = 0; e < nE; ++e) {
      double ee = 0.0;
      for (int al = 0; al < 3; ++al) ee += E[e * 3 + al] * E[e * 3 + al];
      en[e] = mean_a * ee;
    }
    std::vector<double> v(nE);
    for (int al = 0; al < 3; ++al) {
      TKB g = X;
      g.U[al] = C.gframe;
      LRFG_TRY(tk_mode_apply(X, g, al, 0, 0.0, 1.0, C.f[al], nE, s));
      LRFG_TRY(tk_dot(C.a, g, C.dots, C.dscr, nE, s));
      LRFG_TRY(tk_read(C, C.dots, v.data(), nE));
      for (int e = 0; e < nE; ++e) en[e] += 2.0 * E[e * 3 + al] * v[e] / Ntot;
      TKB kr = C.kr;
      LRFG_TRY(tk_hadamard(C.a, g, kr, nE, s));
      LRFG_TRY(tk_dot(kr, g, C.dots, C.dscr, nE, s));
      LRFG_TRY(tk_read(C, C.dots, v.data(), nE));
      for (int e = 0; e < nE; ++e) en[e] += v[e] / Ntot;
    }
    return LRFG_OK;
  };
  // ---------------------------------------------------------------- solver
  const int maxit = P.max_iter;
  std::vector<double> hist((size_t)nE * maxit, 0.0), res0(nE, 0.0);
  std::vector<int> iters(nE, 0), status(nE, LRFG_OK);
  const int patience = (P.solver == LRFG_SOLVER_PCG) ? 5 : 1;
  const int max_restarts = (P.solver == LRFG_SOLVER_PCG) ? kMaxRestarts : 0;
  // kept mode ranks of the latest x truncation (mode j of system e at
  // kx[j nE + e]) and those of each system's kept iterate
  std::vector<int> kx(3 * nE, 0), kbest(3 * nE, 0);
  auto fetch_kept = [&]() -> int {
    for (int j = 0; j < 3; ++j)
      LRFG_HIP(hipMemcpyAsync(kx.data() + j * nE, C.rd.kept + (long long)j * C.rd.kept_batch, sizeof(int) * nE,
                              hipMemcpyDeviceToHost, s));
    return LRFG_OK;
  };
  auto upload_done = [&](const std::vector<int>& hd) -> int {
    LRFG_HIP(hipMemcpyAsync(C.done, hd.data(), sizeof(int) * nE, hipMemcpyHostToDevice, s));
    return LRFG_OK;
  };
  // One truncated PCG (or MR) solve of K x = C.b, best iterate into C.xb, in
  // the rounder's current precision; the same contract as the train path's.
  auto inner = [&](double tol, int max_it, const std::vector<int>& skip, std::vector<double>& r0,
                   std::vector<int>& st, bool record) -> int {
    std::vector<int> hdone(skip), since_best(nE, 0), its(nE, 0), restarts(nE, 0);
    // whether the latest restart was followed by a new best iterate: a restart
    // that brings none ends the solve (the residual sits at the rank floor)
    std::vector<char> restart_paid(nE, 1);
    std::vector<double> best(nE, INFINITY), zzh(nE);
    for (int e = 0; e < nE; ++e) st[e] = LRFG_OK;
    LRFG_TRY(tt_fill(C.mones, nE, -1.0, s));
    LRFG_TRY(tk_zero(C.xr, 2 * nE, s));
    LRFG_TRY(tk_zero(C.xb, nE, s));
    LRFG_TRY(upload_done(hdone));
    if (P.solver == LRFG_SOLVER_PCG) {
      LRFG_TRY(tk_copy(C.b, C.r, nE, s));
      LRFG_TRY(tk_apply_P(C, C.r, C.z));
      LRFG_TRY(tk_copy(C.z, C.p, nE, s));
      LRFG_TRY(tk_dot(C.r, C.z, C.rho, C.dscr, nE, s));
      LRFG_TRY(tk_dot(C.z, C.z, C.zz, C.dscr, nE, s));
    } else {
      LRFG_TRY(tk_apply_P(C, C.b, C.z));
      LRFG_TRY(tk_copy(C.z, C.b, nE, s));
      LRFG_TRY(tk_copy(C.b, C.r, nE, s));
      LRFG_TRY(tk_dot(C.r, C.r, C.zz, C.dscr, nE, s));
    }
    LRFG_TRY(tk_read(C, C.zz, zzh.data(), nE));
    for (int e = 0; e < nE; ++e) {
      r0[e] = std::sqrt(std::max(zzh[e], 0.0));
      if (r0[e] <= floor_abs[e]) hdone[e] = 1;
    }
    LRFG_TRY(upload_done(hdone));
    for (int it = 0; it < max_it; ++it) {
      if (it > 0) gate_point();
      bool all = true;
      for (int e = 0; e < nE; ++e) all = all && hdone[e];
      if (all) break;
      if (P.solver == LRFG_SOLVER_PCG) {
        LRFG_TRY(tk_apply_K(C, C.p, C.q));
        LRFG_TRY(tk_dot(C.p, C.q, C.pqd, C.dscr, nE, s));
        hipLaunchKernelGGL(k_ratio, dim3(1), dim3(kMaxSystems), 0, s, (const double*)C.rho, (const double*)C.pqd,
                           (const int*)C.done, C.alpha, nE);
        hipLaunchKernelGGL(k_pm, dim3(1), dim3(kMaxSystems), 0, s, (const double*)C.alpha, C.coef2, nE);
        LRFG_LAUNCHED();
        LRFG_TRY(tk_update_xr(C));
        LRFG_TRY(fetch_kept());
        LRFG_TRY(tk_apply_P(C, C.r, C.z));
        LRFG_TRY(tk_dot(C.r, C.z, C.dots, C.dscr, nE, s));
        LRFG_TRY(tk_dot(C.z, C.z, C.zz, C.dscr, nE, s));
        hipLaunchKernelGGL(k_beta, dim3(1), dim3(kMaxSystems), 0, s, (const double*)C.dots, C.rho,
                           (const int*)C.done, C.beta, nE);
        LRFG_LAUNCHED();
        LRFG_TRY(tk_axpby(C, C.z, C.p, C.beta, C.tmp));
        LRFG_TRY(tk_copy(C.tmp, C.p, nE, s));
      } else {
        LRFG_TRY(tk_apply_K(C, C.r, C.tmp));
        LRFG_TRY(tk_apply_P(C, C.tmp, C.z));
        LRFG_TRY(tk_dot(C.z, C.r, C.dots, C.dscr, nE, s));
        LRFG_TRY(tk_dot(C.z, C.z, C.pqd, C.dscr, nE, s));
        hipLaunchKernelGGL(k_ratio, dim3(1), dim3(kMaxSystems), 0, s, (const double*)C.dots, (const double*)C.pqd,
                           (const int*)C.done, C.alpha, nE);
        hipLaunchKernelGGL(k_pm, dim3(1), dim3(kMaxSystems), 0, s, (const double*)C.alpha, C.coef2, nE);
        LRFG_LAUNCHED();
        LRFG_TRY(tk_copy(C.r, C.p, nE, s));
        LRFG_TRY(tk_copy(C.z, C.q, nE, s));
        LRFG_TRY(tk_update_xr(C));
        LRFG_TRY(fetch_kept());
        LRFG_TRY(tk_dot(C.r, C.r, C.zz, C.dscr, nE, s));
      }
      LRFG_TRY(tk_read(C, C.zz, zzh.data(), nE));
      bool changed = false;
      SysMask restart{{0, 0, 0, 0}};
      for (int e = 0; e < nE; ++e) {
        if (hdone[e]) continue;
        const double res = std::sqrt(std::max(zzh[e], 0.0)) / r0[e];
        if (record) hist[(size_t)e * maxit + it] = res;
        its[e] = it + 1;
        if (res < best[e]) {
          best[e] = res;
          since_best[e] = 0;
          restart_paid[e] = 1;
          LRFG_TRY(tk_copy_system(C.x, C.xb, e, s));
          if (record)
            for (int j = 0; j < 3; ++j) kbest[j * nE + e] = kx[j * nE + e];
        } else {
          ++since_best[e];
        }
        if (res <= tol || std::sqrt(std::max(zzh[e], 0.0)) <= floor_abs[e]) {
          hdone[e] = 1;
          changed = true;
        } else if (since_best[e] >= patience && restarts[e] < max_restarts && restart_paid[e]) {
          ++restarts[e];  // restart from the best iterate (as in the train path)
          since_best[e] = 0;
          restart_paid[e] = 0;
          restart.m[e >> 6] |= 1ull << (e & 63);
        } else if (since_best[e] >= patience) {
          hdone[e] = 1;
          changed = true;
          if (best[e] > tol) st[e] = LRFG_RANK_LIMITED;
        }
      }
      if (changed) LRFG_TRY(upload_done(hdone));
      if (restart.m[0] | restart.m[1] | restart.m[2] | restart.m[3]) {
        // residual replacement for the restarted systems: x = x_best,
        // r = T(b - K x), z = T(P~^-1 r), p = z, rho = (r, z)
        const uint64_t saved = C.rd.counter;  // sketches of their own (see the train path)
        C.rd.counter = kRestartKeys | ((uint64_t)it << 8);
        LRFG_TRY(tk_apply_K(C, C.xb, C.tmp));
        LRFG_TRY(tk_axpby(C, C.b, C.tmp, C.mones, C.z));
        for (int e = 0; e < nE; ++e)
          if (sys_bit(restart, e)) {
            LRFG_TRY(tk_copy_system(C.z, C.r, e, s));
            LRFG_TRY(tk_copy_system(C.xb, C.x, e, s));
          }
        LRFG_TRY(tk_apply_P(C, C.r, C.z));
        C.rd.counter = saved;
        for (int e = 0; e < nE; ++e)
          if (sys_bit(restart, e)) LRFG_TRY(tk_copy_system(C.z, C.p, e, s));
        LRFG_TRY(tk_dot(C.r, C.z, C.dots, C.dscr, nE, s));
        hipLaunchKernelGGL(k_pick, dim3(1), dim3(kMaxSystems), 0, s, C.rho, (const double*)C.dots, restart, nE);
        LRFG_LAUNCHED();
        LRFG_TRY(tk_dot(C.z, C.z, C.zz, C.dscr, nE, s));
        LRFG_TRY(tk_read(C, C.zz, zzh.data(), nE));
        for (int e = 0; e < nE; ++e)
          if (sys_bit(restart, e)) best[e] = std::sqrt(std::max(zzh[e], 0.0)) / r0[e];
      }
    }
    for (int e = 0; e < nE; ++e) {
      if (!hdone[e]) st[e] = LRFG_NOT_CONVERGED;
      if (skip[e] || r0[e] <= floor_abs[e]) st[e] = LRFG_OK;
      iters[e] = record ? its[e] : iters[e] + its[e];
    }
    return LRFG_OK;
  };

  const std::vector<int> none(nE, 0);
  if (P.precision == LRFG_PREC_FP64) {
    LRFG_TRY(inner(P.solver_tol, maxit, none, res0, status, true));
  } else {
    // Mixed precision: the train path's iterative refinement (inner solves
    // in reduced precision on the residual, correction update, residual and
    // energy in FP64, stop at solver_tol or after two outer steps without an
    // energy gain, the first such step under BF16 moving the inner solves to
    // FP32), with the Tucker operations.
    int lowp = P.precision;
    double tol_in = std::max(P.solver_tol, lowp == LRFG_PREC_MIXED_BF16 ? 1e-2 : 1e-4);
    const double tol_en = std::max(P.solver_tol * P.solver_tol, 1e-15);
    LRFG_TRY(tt_fill(C.ones, nE, 1.0, s));
    LRFG_TRY(tt_fill(C.mones, nE, -1.0, s));
    LRFG_TRY(tk_copy(C.b, C.b0, nE, s));
    LRFG_TRY(tk_zero(C.xa, nE, s));
    LRFG_TRY(tk_zero(C.xbest, nE, s));
    C.rd.prec = LRFG_PREC_FP64;
    std::vector<double> rn0(nE, 0.0), zzh(nE), best(nE, INFINITY), en(nE);
    LRFG_TRY(tk_apply_P(C, C.b0, C.z));
    LRFG_TRY(tk_dot(C.z, C.z, C.zz, C.dscr, nE, s));
    LRFG_TRY(tk_read(C, C.zz, zzh.data(), nE));
    std::vector<int> odone(nE, 0), st_in(nE), capped(nE, 1), no_gain(nE, 0);
    for (int e = 0; e < nE; ++e) {
      rn0[e] = std::sqrt(std::max(zzh[e], 0.0));
      if (rn0[e] <= floor_abs[e]) {
        odone[e] = 1;
        capped[e] = 0;
      }
    }
    std::vector<double> r0_in(nE);
    for (int outer = 0; outer < maxit; ++outer) {
      bool all = true;
      for (int e = 0; e < nE; ++e) all = all && odone[e];
      if (all) break;
      C.rd.prec = lowp;
      LRFG_TRY(inner(tol_in, maxit, odone, r0_in, st_in, false));
      C.rd.prec = LRFG_PREC_FP64;
      LRFG_TRY(tk_axpby(C, C.xa, C.xb, C.ones, C.tmp));   // x <- T(x + delta)
      LRFG_TRY(fetch_kept());
      LRFG_TRY(tk_copy(C.tmp, C.xa, nE, s));
      LRFG_TRY(tk_apply_K(C, C.xa, C.tmp));               // r <- T(b - K x)
      LRFG_TRY(tk_axpby(C, C.b0, C.tmp, C.mones, C.b));
      LRFG_TRY(tk_apply_P(C, C.b, C.z));
      LRFG_TRY(tk_dot(C.z, C.z, C.zz, C.dscr, nE, s));
      LRFG_TRY(tk_read(C, C.zz, zzh.data(), nE));
      LRFG_TRY(energy_diag(C.xa, en));
      bool escalate = false;
      for (int e = 0; e < nE; ++e) {
        if (odone[e]) continue;
        const double rel = std::sqrt(std::max(zzh[e], 0.0)) / rn0[e];
        hist[(size_t)e * maxit + outer] = rel;
        const bool gain = en[e] < best[e] - tol_en * std::fabs(en[e]);
        if (en[e] < best[e]) {
          best[e] = en[e];
          LRFG_TRY(tk_copy_system(C.xa, C.xbest, e, s));
          for (int j = 0; j < 3; ++j) kbest[j * nE + e] = kx[j * nE + e];
        }
        no_gain[e] = gain ? 0 : no_gain[e] + 1;
        if (!gain && lowp == LRFG_PREC_MIXED_BF16) escalate = true;
        if (rel <= P.solver_tol || no_gain[e] >= 2) {
          odone[e] = 1;
          capped[e] = 0;
        }
      }
      if (escalate) {
        lowp = LRFG_PREC_MIXED_FP32;
        tol_in = std::max(P.solver_tol, 1e-4);
        for (int e = 0; e < nE; ++e) no_gain[e] = 0;
      }
    }
    for (int e = 0; e < nE; ++e) status[e] = capped[e] ? LRFG_NOT_CONVERGED : LRFG_OK;
    LRFG_TRY(tk_copy(C.xbest, C.xb, nE, s));
    res0 = rn0;
  }
  // ---------------------------------------------------------------- A_H (eq. homog)
  std::vector<double> m1((size_t)nE * 3), m2((size_t)nE * nE * 3);
  for (int al = 0; al < 3; ++al) {
    TKB g = C.xb;
    g.U[al] = C.gframe;
    LRFG_TRY(tk_mode_apply(C.xb, g, al, 0, 0.0, 1.0, C.f[al], nE, s));
    LRFG_TRY(tk_dot(C.a, g, C.dots, C.dscr, nE, s));
    std::vector<double> v(nE);
    LRFG_TRY(tk_read(C, C.dots, v.data(), nE));
    for (int e = 0; e < nE; ++e) m1[(size_t)e * 3 + al] = v[e] / Ntot;
    TKB kr = C.kr;
    LRFG_TRY(tk_hadamard(C.a, g, kr, nE, s));
    LRFG_TRY(tk_dot(kr, g, C.dots, C.dscr, nE, s, nE));  // every (i, j) pair in one pass
    std::vector<double> w2((size_t)nE * nE);
    LRFG_TRY(tk_read(C, C.dots, w2.data(), nE * nE));
    for (int i = 0; i < nE; ++i)
      for (int j = 0; j < nE; ++j) m2[((size_t)i * nE + j) * 3 + al] = w2[(size_t)i * nE + j] / Ntot;
  }
  LRFG_HIP(hipEventRecord(ev2, s));
  LRFG_HIP(hipStreamSynchronize(s));
  float ms_setup = 0.f, ms_solve = 0.f;
  LRFG_HIP(hipEventElapsedTime(&ms_setup, ev0, ev1));
  LRFG_HIP(hipEventElapsedTime(&ms_solve, ev1, ev2));
  int rc = LRFG_OK;
  for (int i = 0; i < nE; ++i) {
    for (int j = 0; j < nE; ++j) {
      double v = 0.0;
      for (int al = 0; al < 3; ++al) {
        const double ei = E[i * 3 + al], ej = E[j * 3 + al];
        v += mean_a * ei * ej + ei * m1[(size_t)j * 3 + al] + ej * m1[(size_t)i * 3 + al] +
             m2[((size_t)i * nE + j) * 3 + al];
      }
      if (out->A_H) out->A_H[i * nE + j] = v;
    }
    if (out->iters) out->iters[i] = iters[i];
    if (out->status) out->status[i] = status[i];
    rc = worse_status(rc, status[i]);
    if (out->res_hist)
      for (int k = 0; k < maxit; ++k) out->res_hist[(size_t)i * maxit + k] = hist[(size_t)i * maxit + k];
    if (out->ranks) {
      // kept mode ranks (r_1, r_2, r_3) of the returned iterate; the fourth
      // entry of the d + 1 is 0
      for (int j = 0; j < 3; ++j) out->ranks[i * 4 + j] = kbest[j * nE + i];
      out->ranks[i * 4 + 3] = 0;
    }
  }
  out->setup_ms = ms_setup;
  out->solve_ms = ms_solve;
  return rc;
}

}  // namespace lrfg
