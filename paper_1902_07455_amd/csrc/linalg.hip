// FP64 batched GEMM on MFMA (v_mfma_f64_16x16x4f64) and a batched cyclic
// Jacobi eigensolver for small symmetric matrices.
#include <cmath>

#include "linalg.h"
#include "prof.h"

namespace lrfg {

namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int BM = 64, BN = 64, BK = 16;

// Tile 64 x 64 per 256-thread block; wave w = (wm, wn) in 2 x 2 computes a
// 32 x 32 sub-tile as 2 x 2 MFMA 16 x 16 blocks.  MFMA f64 16x16x4 lane
// layout: A operand lane l -> A[l % 16][l / 16]; B operand lane l ->
// B[l / 16][l % 16]; result lane l holds D[l / 16 + 4 i][l % 16], i < 4.
// With `part` != null the raw product of this K split is stored to
// part[(bz * m + row) * n + col] for a later reduction.
template <bool TA, bool TB>
__global__ __launch_bounds__(256) void k_gemm(int m, int n, int k, const double* __restrict__ A,
                                              long long lda, long long sA, const double* __restrict__ B,
                                              long long ldb, long long sB, double* __restrict__ C,
                                              long long ldc, long long sC, double alpha, double beta,
                                              int ksplit, int kchunk, double* __restrict__ part) {
  __shared__ double As[BK][BM + 1];
  __shared__ double Bs[BK][BN + 1];
  const int bz = blockIdx.z;
  const int bt = bz / ksplit;
  const int ks = bz - bt * ksplit;
  A += bt * sA;
  B += bt * sB;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int kb = ks * kchunk;
  const int ke = min(k, kb + kchunk);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  constexpr int RA = (BM * BK) / 256, RB = (BK * BN) / 256;
  dbl4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
  // register prefetch of the next K tile while the current one is multiplied
  double pa[RA], pb[RB];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int r = 0; r < RA; ++r) {
      const int e = threadIdx.x + r * 256;
      int i, kk;
      if (!TA) { i = e / BK; kk = e % BK; } else { kk = e / BM; i = e % BM; }
      const int gi = m0 + i, gk = k0 + kk;
      pa[r] = (gi < m && gk < ke) ? (TA ? A[(long long)gk * lda + gi] : A[(long long)gi * lda + gk]) : 0.0;
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const int e = threadIdx.x + r * 256;
      int kk, j;
      if (!TB) { kk = e / BN; j = e % BN; } else { j = e / BK; kk = e % BK; }
      const int gk = k0 + kk, gj = n0 + j;
      pb[r] = (gj < n && gk < ke) ? (TB ? B[(long long)gj * ldb + gk] : B[(long long)gk * ldb + gj]) : 0.0;
    }
  };
  if (kb < ke) fetch(kb);
  for (int k0 = kb; k0 < ke; k0 += BK) {
#pragma unroll
    for (int r = 0; r < RA; ++r) {
      const int e = threadIdx.x + r * 256;
      int i, kk;
      if (!TA) { i = e / BK; kk = e % BK; } else { kk = e / BM; i = e % BM; }
      As[kk][i] = pa[r];
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const int e = threadIdx.x + r * 256;
      int kk, j;
      if (!TB) { kk = e / BN; j = e % BN; } else { j = e / BK; kk = e % BK; }
      Bs[kk][j] = pb[r];
    }
    __syncthreads();
    if (k0 + BK < ke) fetch(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      double a[2], b[2];
#pragma unroll
      for (int bi = 0; bi < 2; ++bi) a[bi] = As[kk + (lane >> 4)][wm * 32 + bi * 16 + (lane & 15)];
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) b[bj] = Bs[kk + (lane >> 4)][wn * 32 + bj * 16 + (lane & 15)];
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
          acc[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[bi], b[bj], acc[bi][bj], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * 32 + bi * 16 + (lane >> 4) + 4 * r;
        const int col = n0 + wn * 32 + bj * 16 + (lane & 15);
        if (row < m && col < n) {
          const double v = acc[bi][bj][r];
          if (part != nullptr) {
            part[((long long)bz * m + row) * n + col] = v;
          } else {
            double* c = C + bt * sC + (long long)row * ldc + col;
            *c = (beta == 0.0) ? alpha * v : alpha * v + beta * (*c);
          }
        }
      }
}

// Skinny variant: 32 x 32 tile per 64-thread block (one wave computing
// 2 x 2 MFMA 16 x 16 blocks), for shapes whose m or n is at most 32.
constexpr int SM = 32, SK = 16;
template <bool TA, bool TB>
__global__ __launch_bounds__(64) void k_gemm_s(int m, int n, int k, const double* __restrict__ A, long long lda,
                                               long long sA, const double* __restrict__ B, long long ldb,
                                               long long sB, double* __restrict__ C, long long ldc, long long sC,
                                               double alpha, double beta, int ksplit, int kchunk,
                                               double* __restrict__ part) {
  __shared__ double As[SK][SM + 1];
  __shared__ double Bs[SK][SM + 1];
  const int bz = blockIdx.z;
  const int bt = bz / ksplit;
  const int ks = bz - bt * ksplit;
  A += bt * sA;
  B += bt * sB;
  const int m0 = blockIdx.y * SM, n0 = blockIdx.x * SM;
  const int kb = ks * kchunk;
  const int ke = min(k, kb + kchunk);
  const int lane = threadIdx.x;
  dbl4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
  for (int k0 = kb; k0 < ke; k0 += SK) {
#pragma unroll
    for (int r = 0; r < (SM * SK) / 64; ++r) {
      const int e = lane + r * 64;
      int i, kk;
      if (!TA) { i = e / SK; kk = e % SK; } else { kk = e / SM; i = e % SM; }
      const int gi = m0 + i, gk = k0 + kk;
      double v = 0.0;
      if (gi < m && gk < ke) v = TA ? A[(long long)gk * lda + gi] : A[(long long)gi * lda + gk];
      As[kk][i] = v;
    }
#pragma unroll
    for (int r = 0; r < (SK * SM) / 64; ++r) {
      const int e = lane + r * 64;
      int kk, j;
      if (!TB) { kk = e / SM; j = e % SM; } else { j = e / SK; kk = e % SK; }
      const int gk = k0 + kk, gj = n0 + j;
      double v = 0.0;
      if (gj < n && gk < ke) v = TB ? B[(long long)gj * ldb + gk] : B[(long long)gk * ldb + gj];
      Bs[kk][j] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < SK; kk += 4) {
      double a[2], b[2];
#pragma unroll
      for (int bi = 0; bi < 2; ++bi) a[bi] = As[kk + (lane >> 4)][bi * 16 + (lane & 15)];
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) b[bj] = Bs[kk + (lane >> 4)][bj * 16 + (lane & 15)];
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
          acc[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[bi], b[bj], acc[bi][bj], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + bi * 16 + (lane >> 4) + 4 * r;
        const int col = n0 + bj * 16 + (lane & 15);
        if (row < m && col < n) {
          const double v = acc[bi][bj][r];
          if (part != nullptr) {
            part[((long long)bz * m + row) * n + col] = v;
          } else {
            double* c = C + bt * sC + (long long)row * ldc + col;
            *c = (beta == 0.0) ? alpha * v : alpha * v + beta * (*c);
          }
        }
      }
}

__global__ void k_splitk_reduce(int m, int n, int ksplit, int batch, const double* __restrict__ part,
                                double* __restrict__ C, long long ldc, long long sC, double alpha,
                                double beta) {
  const long long tot = (long long)batch * m * n;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (long long)gridDim.x * blockDim.x) {
    const int col = (int)(e % n);
    const long long r = e / n;
    const int row = (int)(r % m);
    const int bt = (int)(r / m);
    double v = 0.0;
    for (int ks = 0; ks < ksplit; ++ks) v += part[(((long long)bt * ksplit + ks) * m + row) * n + col];
    double* c = C + bt * sC + (long long)row * ldc + col;
    *c = (beta == 0.0) ? alpha * v : alpha * v + beta * (*c);
  }
}

// The one-wave 32 x 32 tile measured slower than the 64 x 64 tile on the
// truncation's shapes (more blocks, same K loop), so it is not selected.
bool use_small(const Gemm&) { return false; }

int choose_ksplit(const Gemm& g) {
  const bool sm = use_small(g);
  const int tm = sm ? SM : BM, tn = sm ? SM : BN;
  const long long tiles = (long long)ceil_div(g.m, tm) * ceil_div(g.n, tn) * g.batch;
  if (tiles >= 128 || g.k < 256) return 1;
  long long ks = 512 / tiles;
  const long long kmax = g.k / 64;  // at least 64 of K per split
  if (ks > kmax) ks = kmax;
  if (ks > 128) ks = 128;
  return ks < 1 ? 1 : (int)ks;
}

// ---------------------------------------------------------------- Jacobi
// One 256-thread block per matrix; A and V in LDS (stride n).  Cyclic
// round-robin ordering: m = n rounded up to even, position 0 fixed, the
// others rotate by one per step; pair k of a step joins positions k and
// m-1-k, so the pairs of a step are disjoint.  Rotation of the symmetric
// Schur step (Golub and Van Loan): tau = (a_qq - a_pp)/(2 a_pq),
// t = sign(tau)/(|tau| + sqrt(1 + tau^2)), c = 1/sqrt(1 + t^2), s = t c,
// J = [[c, s], [-s, c]] on (p, q).  A <- J^T A J is applied as independent
// 2 x 2 blocks (pair k rows, pair l columns), V <- V J row by row.  A
// rotation is skipped when |a_pq| is below 1e-18 of the largest initial
// diagonal entry; the iteration ends after the first sweep that applies no
// rotation.
__device__ inline int fdivi(int x, int d, float rd) {
  int q = (int)((float)x * rd);
  if (q * d > x) --q;
  else if ((q + 1) * d <= x) ++q;
  return q;
}

__global__ __launch_bounds__(256) void k_syevj(int n, const double* __restrict__ Ag, long long lda, long long sA,
                                               double* __restrict__ Wg, long long sW, double* __restrict__ Vg,
                                               long long sV, int max_sweeps) {
  extern __shared__ double sm[];
  double* a = sm;
  double* v = sm + n * n;
  __shared__ double cs[2 * 32];
  __shared__ int pq[2 * 32];
  __shared__ int rot_any;
  __shared__ double dmax_s;
  const int b = blockIdx.x;
  const double* A = Ag + b * sA;
  const int tid = threadIdx.x, nt = blockDim.x;
  const float rn = 1.0f / (float)n;
  for (int e = tid; e < n * n; e += nt) {
    const int i = fdivi(e, n, rn), j = e - fdivi(e, n, rn) * n;
    a[e] = 0.5 * (A[(long long)i * lda + j] + A[(long long)j * lda + i]);
    v[e] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  if (tid == 0) {
    double dm = 0.0;
    for (int i = 0; i < n; ++i) dm = fmax(dm, fabs(a[i * n + i]));
    dmax_s = dm;
  }
  const int m = n + (n & 1);
  const int np = m / 2;
  const float rnp = 1.0f / (float)np;
  const int nblk = np * np;
  __syncthreads();
  const double abs_floor = 1e-18 * dmax_s;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    if (tid == 0) rot_any = 0;
    __syncthreads();
    for (int step = 0; step < m - 1; ++step) {
      if (tid < np) {
        const int k = tid;
        int t0 = 0;
        if (k != 0) {
          const int u = k - 1 + step;
          t0 = 1 + (u >= m - 1 ? u - (m - 1) : u);
        }
        const int u1 = (m - 1 - k) - 1 + step;
        const int t1 = 1 + (u1 >= m - 1 ? u1 - (m - 1) : u1);
        int p = t0 < t1 ? t0 : t1;
        int q = t0 < t1 ? t1 : t0;
        double c = 1.0, s = 0.0;
        if (q < n) {
          const double apq = a[p * n + q];
          const double app = a[p * n + p], aqq = a[q * n + q];
          if (fabs(apq) > abs_floor) {
            const double tau = (aqq - app) / (2.0 * apq);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
            rot_any = 1;
          }  // else: both rows stay, identity rotation (c = 1, s = 0)
        } else {
          q = p;  // dummy partner: identity
        }
        cs[2 * k] = c;
        cs[2 * k + 1] = s;
        pq[2 * k] = p;
        pq[2 * k + 1] = q;
      }
      __syncthreads();
      // 2 x 2 blocks (rows of pair k, columns of pair l): B' = J_k^T B J_l
      for (int w = tid; w < nblk; w += nt) {
        const int k = fdivi(w, np, rnp), l = w - fdivi(w, np, rnp) * np;
        const int p = pq[2 * k], q = pq[2 * k + 1];
        const int r = pq[2 * l], t = pq[2 * l + 1];
        if (p == q && r == t) continue;
        const double ck = cs[2 * k], sk = cs[2 * k + 1];
        const double cl = cs[2 * l], sl = cs[2 * l + 1];
        if (p == q) {  // single row p, columns (r, t)
          const double x0 = a[p * n + r], x1 = a[p * n + t];
          a[p * n + r] = cl * x0 - sl * x1;
          a[p * n + t] = sl * x0 + cl * x1;
        } else if (r == t) {  // rows (p, q), single column r
          const double x0 = a[p * n + r], x1 = a[q * n + r];
          a[p * n + r] = ck * x0 - sk * x1;
          a[q * n + r] = sk * x0 + ck * x1;
        } else {
          const double b00 = a[p * n + r], b01 = a[p * n + t];
          const double b10 = a[q * n + r], b11 = a[q * n + t];
          const double u00 = ck * b00 - sk * b10, u01 = ck * b01 - sk * b11;
          const double u10 = sk * b00 + ck * b10, u11 = sk * b01 + ck * b11;
          a[p * n + r] = cl * u00 - sl * u01;
          a[p * n + t] = sl * u00 + cl * u01;
          a[q * n + r] = cl * u10 - sl * u11;
          a[q * n + t] = sl * u10 + cl * u11;
        }
      }
      // V <- V J: row i, pair l
      for (int w = tid; w < n * np; w += nt) {
        const int i = fdivi(w, np, rnp), l = w - fdivi(w, np, rnp) * np;
        const int r = pq[2 * l], t = pq[2 * l + 1];
        if (r == t || cs[2 * l + 1] == 0.0) continue;
        const double cl = cs[2 * l], sl = cs[2 * l + 1];
        const double x0 = v[i * n + r], x1 = v[i * n + t];
        v[i * n + r] = cl * x0 - sl * x1;
        v[i * n + t] = sl * x0 + cl * x1;
      }
      __syncthreads();
    }
    if (!rot_any) break;
  }
  // sort descending: rank of eigenvalue j = #{i : w_i > w_j or (w_i == w_j and i < j)}
  double* W = Wg + b * sW;
  double* V = Vg + b * sV;
  for (int j = tid; j < n; j += nt) {
    const double wj = a[j * n + j];
    int rank = 0;
    for (int i = 0; i < n; ++i) {
      const double wi = a[i * n + i];
      rank += (wi > wj) || (wi == wj && i < j);
    }
    W[rank] = wj;
    for (int i = 0; i < n; ++i) V[(long long)i * n + rank] = v[i * n + j];
  }
}

// Rank-revealing Cholesky with diagonal pivoting of a symmetric positive
// semidefinite G (n x n): G[perm, perm] = L L^T with L n x r lower
// trapezoidal, stopped when the largest remaining diagonal entry is below
// tau times the largest initial one.  Writes S (n x n) = P R^-1 with
// R = L^T (r x r) in the first r columns and zeros elsewhere, so Q = Y S
// has orthonormal columns spanning the numerical range of Y when
// G = Y^T Y.  One 64-lane wave per matrix, lane i owns row i; R^-1 by
// Gauss-Jordan elimination on the triangle (r parallel steps).
__global__ __launch_bounds__(64) void k_pchol_s(int n, const double* __restrict__ Gg, long long sG, double tau,
                                                double* __restrict__ Sg, long long sS, int* __restrict__ rank_out) {
  extern __shared__ double sm[];
  double* g = sm;            // n x n working matrix
  double* ri = sm + n * n;   // n x n: R^-1 (upper)
  __shared__ int perm[64];
  __shared__ double lcol[64];
  const int b = blockIdx.x;
  const int lane = threadIdx.x;
  const double* G = Gg + b * sG;
  for (int e = lane; e < n * n; e += 64) g[e] = G[e];
  if (lane < n) perm[lane] = lane;
  __syncthreads();
  double dmax0 = (lane < n) ? g[lane * n + lane] : 0.0;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) dmax0 = fmax(dmax0, __shfl_xor(dmax0, o, 64));
  int r = n;
  for (int k = 0; k < n; ++k) {
    // argmax of the remaining diagonal over the wave (ties: lowest index)
    double best = (lane >= k && lane < n) ? g[lane * n + lane] : -1.0;
    int p = lane;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double ob = __shfl_xor(best, o, 64);
      const int op = __shfl_xor(p, o, 64);
      if (ob > best || (ob == best && op < p)) {
        best = ob;
        p = op;
      }
    }
    if (!(best > tau * dmax0) || !(best > 0.0)) {
      r = k;
      break;
    }
    if (p != k) {
      // symmetric swap of rows/cols k and p (and the permutation)
      for (int j = lane; j < n; j += 64) {
        const double t = g[k * n + j];
        g[k * n + j] = g[p * n + j];
        g[p * n + j] = t;
      }
      __syncthreads();
      for (int i = lane; i < n; i += 64) {
        const double t = g[i * n + k];
        g[i * n + k] = g[i * n + p];
        g[i * n + p] = t;
      }
      if (lane == 0) {
        const int t = perm[k];
        perm[k] = perm[p];
        perm[p] = t;
      }
      __syncthreads();
    }
    const double lkk = sqrt(g[k * n + k]);
    const double inv = 1.0 / lkk;
    // column k of L (L[i][k] = g[i][k]/lkk) published in lcol, then each
    // lane i > k updates its row: g[i][j] -= L[i][k] L[j][k], j > k
    double lik = 0.0;
    if (lane > k && lane < n) lik = g[lane * n + k] * inv;
    if (lane < n) lcol[lane] = lik;
    __syncthreads();
    if (lane == k) g[k * n + k] = lkk;
    if (lane > k && lane < n) {
      g[lane * n + k] = lik;
      for (int j = k + 1; j < n; ++j) g[lane * n + j] -= lik * lcol[j];
    }
    __syncthreads();
  }
  // R = L^T (r x r upper): R[i][j] = g[j][i] for j >= i.  Gauss-Jordan on
  // [R | I]: for c = r-1 down to 0, scale row c by 1/R[c][c] and eliminate
  // column c from the rows above (lane i owns row i of R^-1).
  for (int e = lane; e < n * n; e += 64) ri[e] = 0.0;
  __syncthreads();
  if (lane < r) ri[lane * n + lane] = 1.0;
  __syncthreads();
  for (int c = r - 1; c >= 0; --c) {
    const double rcc = g[c * n + c];
    if (lane == c)
      for (int j = c; j < r; ++j) ri[c * n + j] /= rcc;
    __syncthreads();
    if (lane < c) {
      const double f = g[c * n + lane];  // R[lane][c]
      for (int j = c; j < r; ++j) ri[lane * n + j] -= f * ri[c * n + j];
    }
    __syncthreads();
  }
  double* S = Sg + b * sS;
  for (int e = lane; e < n * n; e += 64) {
    const int i = e / n, j = e - (e / n) * n;  // S[perm[i]][j] = Rinv[i][j]
    S[perm[i] * n + j] = (i < r && j < r) ? ri[i * n + j] : 0.0;
  }
  if (lane == 0 && rank_out != nullptr) rank_out[b] = r;
}

}  // namespace

size_t gemm_scratch_doubles(const Gemm& g) {
  const int ks = choose_ksplit(g);
  if (ks <= 1) return 0;
  return (size_t)g.batch * ks * g.m * g.n;
}

int gemm(const Gemm& g, double* scratch, size_t scratch_doubles, hipStream_t s) {
  if (g.m <= 0 || g.n <= 0 || g.batch <= 0) return LRFG_OK;
  int ks = choose_ksplit(g);
  if (ks > 1) {
    // as many splits as the scratch holds
    const size_t per = (size_t)g.batch * g.m * g.n;
    const size_t fit = scratch == nullptr ? 0 : scratch_doubles / per;
    if ((size_t)ks > fit) ks = (int)fit;
    if (ks < 2) ks = 1;
  }
  const int kchunk = ks > 1 ? ((g.k + ks - 1) / ks + BK - 1) / BK * BK : (g.k > 0 ? g.k : 1);
  // (BK == SK, so the chunk suits both tile shapes)
  if (ks > 1) ks = (g.k + kchunk - 1) / kchunk;
  const bool sm = use_small(g);
  dim3 grid(ceil_div(g.n, sm ? SM : BN), ceil_div(g.m, sm ? SM : BM), g.batch * ks);
  double* part = ks > 1 ? scratch : nullptr;
  ProfScope ps_("gemm", s);
#define LRFG_GEMM_LAUNCH(TA, TB)                                                                              \
  do {                                                                                                       \
    if (sm)                                                                                                  \
      hipLaunchKernelGGL((k_gemm_s<TA, TB>), grid, dim3(64), 0, s, g.m, g.n, g.k, g.A, g.lda, g.sA, g.B, g.ldb, \
                         g.sB, g.C, g.ldc, g.sC, g.alpha, g.beta, ks, kchunk, part);                            \
    else                                                                                                     \
      hipLaunchKernelGGL((k_gemm<TA, TB>), grid, dim3(256), 0, s, g.m, g.n, g.k, g.A, g.lda, g.sA, g.B, g.ldb,  \
                         g.sB, g.C, g.ldc, g.sC, g.alpha, g.beta, ks, kchunk, part);                            \
  } while (0)
  if (!g.ta && !g.tb) LRFG_GEMM_LAUNCH(false, false);
  else if (g.ta && !g.tb) LRFG_GEMM_LAUNCH(true, false);
  else if (!g.ta && g.tb) LRFG_GEMM_LAUNCH(false, true);
  else LRFG_GEMM_LAUNCH(true, true);
#undef LRFG_GEMM_LAUNCH
  LRFG_LAUNCHED();
  if (ks > 1) {
    const long long tot = (long long)g.batch * g.m * g.n;
    const int gr = (int)std::min<long long>(1024, (tot + 255) / 256);
    hipLaunchKernelGGL(k_splitk_reduce, dim3(gr), dim3(256), 0, s, g.m, g.n, ks, g.batch, (const double*)part, g.C,
                       g.ldc, g.sC, g.alpha, g.beta);
    LRFG_LAUNCHED();
  }
  return LRFG_OK;
}

int syevj(int n, const double* A, long long lda, long long sA, double* W, long long sW, double* V, long long sV,
          int batch, hipStream_t s) {
  if (n < 1 || n > kMaxEig) {
    set_error("syevj: n = %d outside [1, %d]", n, kMaxEig);
    return LRFG_EINVAL;
  }
  if (batch <= 0) return LRFG_OK;
  const size_t shm = sizeof(double) * 2 * n * n;
  static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_syevj),
                                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                                     (int)(sizeof(double) * 2 * kMaxEig * kMaxEig));
  (void)attr;
  ProfScope ps_("syevj", s);
  hipLaunchKernelGGL(k_syevj, dim3(batch), dim3(256), shm, s, n, A, lda, sA, W, sW, V, sV, 20);
  LRFG_LAUNCHED();
  return LRFG_OK;
}

int pchol_s(int n, const double* G, long long sG, double tau, double* S, long long sS, int* rank, int batch,
            hipStream_t s) {
  if (n < 1 || n > kMaxEig) {
    set_error("pchol: n = %d outside [1, %d]", n, kMaxEig);
    return LRFG_EINVAL;
  }
  if (batch <= 0) return LRFG_OK;
  const size_t shm = sizeof(double) * 2 * n * n;
  static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_pchol_s),
                                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                                     (int)(sizeof(double) * 2 * kMaxEig * kMaxEig));
  (void)attr;
  ProfScope ps_("pchol", s);
  hipLaunchKernelGGL(k_pchol_s, dim3(batch), dim3(64), shm, s, n, G, sG, tau, S, sS, rank);
  LRFG_LAUNCHED();
  return LRFG_OK;
}

}  // namespace lrfg
