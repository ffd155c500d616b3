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
  dbl4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
  for (int k0 = kb; k0 < ke; k0 += BK) {
#pragma unroll
    for (int r = 0; r < (BM * BK) / 256; ++r) {
      const int e = threadIdx.x + r * 256;
      int i, kk;
      if (!TA) { i = e / BK; kk = e % BK; } else { kk = e / BM; i = e % BM; }
      const int gi = m0 + i, gk = k0 + kk;
      double v = 0.0;
      if (gi < m && gk < ke) v = TA ? A[(long long)gk * lda + gi] : A[(long long)gi * lda + gk];
      As[kk][i] = v;
    }
#pragma unroll
    for (int r = 0; r < (BK * BN) / 256; ++r) {
      const int e = threadIdx.x + r * 256;
      int kk, j;
      if (!TB) { kk = e / BN; j = e % BN; } else { j = e / BK; kk = e % BK; }
      const int gk = k0 + kk, gj = n0 + j;
      double v = 0.0;
      if (gj < n && gk < ke) v = TB ? B[(long long)gj * ldb + gk] : B[(long long)gk * ldb + gj];
      Bs[kk][j] = v;
    }
    __syncthreads();
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

int choose_ksplit(const Gemm& g) {
  const long long tiles = (long long)ceil_div(g.m, BM) * ceil_div(g.n, BN) * g.batch;
  if (tiles >= 128 || g.k < 512) return 1;
  long long ks = 256 / tiles;
  const long long kmax = g.k / 256;  // at least 256 of K per split
  if (ks > kmax) ks = kmax;
  if (ks > 64) ks = 64;
  return ks < 1 ? 1 : (int)ks;
}

// ---------------------------------------------------------------- Jacobi
// One block per matrix (64 threads for n <= 32, else 256); A and V in LDS
// (stride n).  Cyclic round-robin ordering: m = n rounded up to even,
// position 0 fixed, the others rotate by one per step; pair k of a step
// joins positions k and m-1-k, so the pairs of a step are disjoint.
// Rotation of the symmetric Schur step (Golub and Van Loan):
// tau = (a_qq - a_pp)/(2 a_pq), t = sign(tau)/(|tau| + sqrt(1 + tau^2)),
// c = 1/sqrt(1 + t^2), s = t c, J = [[c, s], [-s, c]] on (p, q).
// A <- J^T A J is applied as independent 2 x 2 blocks (pair k rows,
// pair l columns), V <- V J row by row.
__global__ void k_syevj(int n, const double* __restrict__ Ag, long long lda, long long sA,
                        double* __restrict__ Wg, long long sW, double* __restrict__ Vg, long long sV,
                        int max_sweeps) {
  extern __shared__ double sm[];
  double* a = sm;
  double* v = sm + n * n;
  __shared__ double cs[2 * 32];
  __shared__ int pq[2 * 32];
  __shared__ double red[2 * 4];
  const int b = blockIdx.x;
  const double* A = Ag + b * sA;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int e = tid; e < n * n; e += nt) {
    const int i = e / n, j = e - (e / n) * n;
    a[e] = 0.5 * (A[(long long)i * lda + j] + A[(long long)j * lda + i]);
    v[e] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int m = n + (n & 1);
  const int np = m / 2;
  const int nblk = np * np;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int e = tid; e < n * n; e += nt) {
      const double x = a[e] * a[e];
      tot += x;
      off += (e % (n + 1) != 0) ? x : 0.0;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      off += __shfl_down(off, o, 64);
      tot += __shfl_down(tot, o, 64);
    }
    if ((tid & 63) == 0) {
      red[2 * (tid >> 6)] = off;
      red[2 * (tid >> 6) + 1] = tot;
    }
    __syncthreads();
    double offs = 0.0, tots = 0.0;
    for (int w = 0; w < nt / 64; ++w) {
      offs += red[2 * w];
      tots += red[2 * w + 1];
    }
    __syncthreads();
    if (!(offs > 1e-28 * tots)) break;
    for (int step = 0; step < m - 1; ++step) {
      if (tid < np) {
        const int k = tid;
        int p, q;
        {
          int t0 = (k == 0) ? 0 : 1 + (k - 1 + step) - ((k - 1 + step) >= m - 1 ? m - 1 : 0);
          const int kk = m - 1 - k;
          int t1 = 1 + (kk - 1 + step) - ((kk - 1 + step) >= m - 1 ? m - 1 : 0);
          p = t0 < t1 ? t0 : t1;
          q = t0 < t1 ? t1 : t0;
        }
        double c = 1.0, s = 0.0;
        if (q < n) {
          const double apq = a[p * n + q];
          if (apq != 0.0) {
            const double app = a[p * n + p], aqq = a[q * n + q];
            const double tau = (aqq - app) / (2.0 * apq);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
          }
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
        const int k = w / np, l = w - (w / np) * np;
        const int p = pq[2 * k], q = pq[2 * k + 1];
        const int r = pq[2 * l], t = pq[2 * l + 1];
        const double ck = cs[2 * k], sk = cs[2 * k + 1];
        const double cl = cs[2 * l], sl = cs[2 * l + 1];
        if (p == q && r == t) {
          continue;
        } else if (p == q) {  // single row p, columns (r, t)
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
          // rows: J_k^T
          const double u00 = ck * b00 - sk * b10, u01 = ck * b01 - sk * b11;
          const double u10 = sk * b00 + ck * b10, u11 = sk * b01 + ck * b11;
          // columns: J_l
          a[p * n + r] = cl * u00 - sl * u01;
          a[p * n + t] = sl * u00 + cl * u01;
          a[q * n + r] = cl * u10 - sl * u11;
          a[q * n + t] = sl * u10 + cl * u11;
        }
      }
      // V <- V J: row i, pair l
      for (int w = tid; w < n * np; w += nt) {
        const int i = w / np, l = w - (w / np) * np;
        const int r = pq[2 * l], t = pq[2 * l + 1];
        if (r == t) continue;
        const double cl = cs[2 * l], sl = cs[2 * l + 1];
        const double x0 = v[i * n + r], x1 = v[i * n + t];
        v[i * n + r] = cl * x0 - sl * x1;
        v[i * n + t] = sl * x0 + cl * x1;
      }
      __syncthreads();
    }
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
// G = Y^T Y.  One block of 64 threads per matrix.
__global__ void k_pchol_s(int n, const double* __restrict__ Gg, long long sG, double tau,
                          double* __restrict__ Sg, long long sS, int* __restrict__ rank_out) {
  extern __shared__ double sm[];
  double* g = sm;            // n x n working matrix
  double* ri = sm + n * n;   // n x n: R^-1 (upper)
  __shared__ int perm[64];
  __shared__ int piv_s;
  __shared__ double dmax0_s;
  __shared__ int rank_s;
  const int b = blockIdx.x;
  const int tid = threadIdx.x;
  const double* G = Gg + b * sG;
  for (int e = tid; e < n * n; e += 64) {
    g[e] = G[e];
    ri[e] = 0.0;
  }
  if (tid < n) perm[tid] = tid;
  __syncthreads();
  if (tid == 0) {
    double m0 = 0.0;
    for (int i = 0; i < n; ++i) m0 = fmax(m0, g[i * n + i]);
    dmax0_s = m0;
    rank_s = n;
  }
  __syncthreads();
  const double dmax0 = dmax0_s;
  for (int k = 0; k < n; ++k) {
    if (tid == 0) {
      int p = k;
      double best = g[k * n + k];
      for (int i = k + 1; i < n; ++i)
        if (g[i * n + i] > best) {
          best = g[i * n + i];
          p = i;
        }
      piv_s = p;
      if (!(best > tau * dmax0) || !(best > 0.0)) rank_s = k;
    }
    __syncthreads();
    if (rank_s <= k) break;
    const int p = piv_s;
    if (p != k) {
      // symmetric swap of rows/cols k and p (and the permutation)
      for (int j = tid; j < n; j += 64) {
        const double t = g[k * n + j];
        g[k * n + j] = g[p * n + j];
        g[p * n + j] = t;
      }
      __syncthreads();
      for (int i = tid; i < n; i += 64) {
        const double t = g[i * n + k];
        g[i * n + k] = g[i * n + p];
        g[i * n + p] = t;
      }
      if (tid == 0) {
        const int t = perm[k];
        perm[k] = perm[p];
        perm[p] = t;
      }
      __syncthreads();
    }
    const double lkk = sqrt(g[k * n + k]);
    __syncthreads();
    // column k of L below the diagonal, stored in g[i][k]
    for (int i = k + tid; i < n; i += 64) g[i * n + k] = (i == k) ? lkk : g[i * n + k] / lkk;
    __syncthreads();
    // trailing update g[i][j] -= L[i][k] L[j][k], i, j > k
    for (int e = tid; e < (n - k - 1) * (n - k - 1); e += 64) {
      const int i = k + 1 + e / (n - k - 1), j = k + 1 + e % (n - k - 1);
      g[i * n + j] -= g[i * n + k] * g[j * n + k];
    }
    __syncthreads();
  }
  const int r = rank_s;
  // R = L^T (r x r upper): R[i][j] = L[j][i] = g[j][i] for j >= i.
  // Column j of R^-1 by back substitution (one thread per column).
  for (int j = tid; j < r; j += 64) {
    for (int i = j; i >= 0; --i) {
      double acc = (i == j) ? 1.0 : 0.0;
      for (int t = i + 1; t <= j; ++t) acc -= g[t * n + i] * ri[t * n + j];
      ri[i * n + j] = acc / g[i * n + i];
    }
  }
  __syncthreads();
  double* S = Sg + b * sS;
  for (int e = tid; e < n * n; e += 64) {
    const int i = e / n, j = e % n;  // S[perm[i]][j] = Rinv[i][j]
    S[perm[i] * n + j] = (i < r && j < r) ? ri[i * n + j] : 0.0;
  }
  if (tid == 0 && rank_out != nullptr) rank_out[b] = r;
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
  if (ks > 1) ks = (g.k + kchunk - 1) / kchunk;
  dim3 grid(ceil_div(g.n, BN), ceil_div(g.m, BM), g.batch * ks);
  double* part = ks > 1 ? scratch : nullptr;
  ProfScope ps_("gemm", s);
#define LRFG_GEMM_LAUNCH(TA, TB)                                                                       \
  hipLaunchKernelGGL((k_gemm<TA, TB>), grid, dim3(256), 0, s, g.m, g.n, g.k, g.A, g.lda, g.sA, g.B, g.ldb, \
                     g.sB, g.C, g.ldc, g.sC, g.alpha, g.beta, ks, kchunk, part)
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
  const int nt = n <= 32 ? 64 : 256;
  hipLaunchKernelGGL(k_syevj, dim3(batch), dim3(nt), shm, s, n, A, lda, sA, W, sW, V, sV, 30);
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
