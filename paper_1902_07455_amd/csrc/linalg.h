// Dense linear algebra kernels of the low-rank path (gfx950, FP64):
// batched GEMM on MFMA, batched symmetric Jacobi eigensolver for small
// matrices, and the Gram-based orthonormalisation built on them.
#pragma once

#include "common.h"

namespace lrfg {

// C_b = alpha op(A_b) op(B_b) + beta C_b for b in [0, batch); row-major
// storage with leading dimensions; op = transpose when ta / tb.
struct Gemm {
  int m = 0, n = 0, k = 0;
  const double* A = nullptr;
  long long lda = 0, sA = 0;
  bool ta = false;
  const double* B = nullptr;
  long long ldb = 0, sB = 0;
  bool tb = false;
  double* C = nullptr;
  long long ldc = 0, sC = 0;
  double alpha = 1.0, beta = 0.0;
  int batch = 1;
  int prec = 0;  // lrfg_precision: FP64, or FP32 / BF16 inputs with FP32 accumulation
  // Batch index map: matrix t of the batch reads A at
  // (t / adiv) sA + (t % amod) sA2, B at (t / bdiv) sB + (t % bmod) sB2 and
  // writes C at (t / cdiv) sC + (t % cmod) sC2 (a modulus of 0 drops that
  // term; the defaults give t sA, t sB, t sC).
  int adiv = 1, amod = 0, bdiv = 1, bmod = 0, cdiv = 1, cmod = 0;
  long long sA2 = 0, sB2 = 0, sC2 = 0;
  // Column map (FP64, B not transposed): column c of B lies at
  // (c / bcw) bchi + c % bcw of its row, column c of C at
  // (c / ccw) cchi + c % ccw (a width of 0: at c), so one product can run
  // over columns gathered from several blocks of an array.
  int bcw = 0, ccw = 0;
  long long bchi = 0, cchi = 0;
  // one K range per matrix (no split-K): for batches that fill the device
  // by themselves
  bool nosplit = false;
};

// The batch map as the kernels receive it; t = tbase + the launch's batch index.
struct BatchMap {
  long long tbase;
  int adiv, amod, bdiv, bmod;
  long long sA2, sB2;
  int cdiv, cmod;
  long long sC2;
  int bcw, ccw;
  long long bchi, cchi;
  // batch indices stay below 2^31 (gemm() launches at most 65535 matrices
  // per chunk from a base below the batch count), so the splits are 32-bit
  __host__ __device__ static long long off(long long t, int dv, int md, long long s1, long long s2) {
    const unsigned u = (unsigned)t;
    return (long long)(u / (unsigned)dv) * s1 + (md > 0 ? (long long)(u % (unsigned)md) * s2 : 0);
  }
  __host__ __device__ long long c_off(long long t, long long sC) const { return off(t, cdiv, cmod, sC, sC2); }
  __host__ __device__ long long a_off(long long t, long long sA) const { return off(t, adiv, amod, sA, sA2); }
  __host__ __device__ long long b_off(long long t, long long sB) const { return off(t, bdiv, bmod, sB, sB2); }
  // column maps (columns below 2^31)
  __host__ __device__ long long bcol(int c) const {
    return bcw > 0 ? (long long)((unsigned)c / (unsigned)bcw) * bchi + (long long)((unsigned)c % (unsigned)bcw) : c;
  }
  __host__ __device__ long long ccol(int c) const {
    return ccw > 0 ? (long long)((unsigned)c / (unsigned)ccw) * cchi + (long long)((unsigned)c % (unsigned)ccw) : c;
  }
};

// Scratch doubles gemm() may use for a split-K reduction of this shape.
size_t gemm_scratch_doubles(const Gemm& g);
// `scratch` may be null (no split-K).
int gemm(const Gemm& g, double* scratch, size_t scratch_doubles, hipStream_t s);

// Batched long dot products: out[t] = sum_i x[(t / xdiv) sx + i] y[t sy + i],
// i < n, t < batch; blocks sum fixed chunks, a second pass adds the chunk
// sums in a fixed order (deterministic).  scratch: dot_rows_scratch doubles.
size_t dot_rows_scratch(long long n, int batch);
int dot_rows(long long n, const double* x, long long sx, int xdiv, const double* y, long long sy, double* out,
             int batch, double* scratch, size_t scratch_doubles, hipStream_t s);

// Batched symmetric eigendecomposition, n <= kMaxSyevj: A_b (n x n, row-major,
// leading dimension lda, batch stride sA) -> eigenvalues W_b (descending)
// and eigenvectors V_b (column j = eigenvector j, row-major n x n).
constexpr int kMaxSyevj = 64;
// Largest matrix of the truncation's small factorisations (pchol_s,
// cut_psd): the sketch size, i.e. rank cap plus oversampling.
constexpr int kMaxEig = 128;
int syevj(int n, const double* A, long long lda, long long sA, double* W, long long sW, double* V,
          long long sV, int batch, hipStream_t s);

// Rank-revealing pivoted Cholesky of batched PSD G (n x n, stride sG):
// S (n x n, stride sS) = P R^-1 on the numerical rank (zeros elsewhere),
// so Y S is orthonormal when G = Y^T Y; rank (device, batch ints) or null.
int pchol_s(int n, const double* G, long long sG, double tau, double* S, long long sS, int* rank, int batch,
            hipStream_t s);

// Truncation basis of batched PSD Gram matrices G (n x n, stride sG):
// S (n x c, stride sS) = eigenvectors of the kept eigenvalues, largest
// first (at most c, none below the Cholesky threshold kCutTau or the
// floor kCutFloor relative to the largest, and with tol2 > 0 the fewest
// whose dropped eigenvalue sum is <= tol2 * trace G), zero columns beyond;
// kept and sweeps (device, batch ints: kept rank, Jacobi sweeps) or null.
constexpr double kCutTau = 1e-15;    // pivoted-Cholesky rank threshold (relative diagonal)
constexpr double kCutEps = 2.5e-16;  // one-sided Jacobi: pair orthogonality, relative, per row
constexpr double kCutFloor = 1e-28;  // smallest kept eigenvalue relative to the largest
int cut_psd(int n, int c, const double* G, long long sG, double tol2, double* S, long long sS, int* kept, int batch,
            hipStream_t s, int* sweeps = nullptr);

}  // namespace lrfg
