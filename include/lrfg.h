/*
 * lrfg.h -- C ABI of the MI355X (gfx950) low-rank Fourier-Galerkin
 * homogenisation library (liblrfg.so).
 *
 * The library computes the effective (homogenised) matrix A_H of the scalar
 * periodic cell problem of Vondrejc, Liu, Ladecky and Matthies,
 * "FFT-based homogenisation accelerated by low-rank tensor approximations"
 * (arXiv:1902.07455):
 *
 *   A_H E.E = min over zero-mean periodic v of  mean_Y a(x) |E + grad v|^2
 *   (Sec. 2.1, eq. homog / bilinear),
 *
 * discretised with trigonometric polynomials on an odd grid N^d and the
 * rectangle rule ("GaNi", Sec. 2.2.1-2.2.2, eq. ls_GaNi_fourier),
 * preconditioned by the Fourier Laplacian (Sec. 2.3, eq. Pls_GaNi_fourier).
 * Two solution paths:
 *   FULL    the corrector is a full grid tensor; preconditioned CG with
 *           3-D FFTs (the plain method of Sec. 4);
 *   TT / TUCKER / CP
 *           the corrector is held in a low-rank format (Sec. 3.1) and the
 *           operator is applied with truncation after every rank-raising
 *           step (Sec. 3.2, eq. Pls_lowrank, Table 1); solved by truncated
 *           PCG or the truncated minimal-residual iteration (Sec. 3.3).
 *
 * Conventions shared by every call
 *   - Grid point j in [0, N) of an axis sits at x_j = -1/2 + (j + 1/2)/N
 *     (the regular grid k/N of Sec. 2.2.1 for odd N).  Full fields are
 *     FP64, C order, axis 0 = x_1 slowest.
 *   - Device pointers are HIP device addresses; "stream" is a hipStream_t
 *     passed as void* (NULL = the default stream).  Calls are ordered on
 *     that stream.
 *   - The library never allocates device memory in a solve or an op call:
 *     all device storage is the caller's workspace (d_ws, ws_bytes), whose
 *     required size comes from lrfg_plan_workspace_bytes.  d_ws must be
 *     256-byte aligned.
 *   - Every call returns an lrfg_status; no exception crosses the ABI.
 *     lrfg_last_error() returns a thread-local message for the last failure.
 *   - A plan may be used by one thread at a time.
 */
#ifndef LRFG_H
#define LRFG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LRFG_ABI_VERSION 2

typedef enum {
  LRFG_OK = 0,
  LRFG_NOT_CONVERGED = 1,   /* A_H written; some corrector hit max_iter (or
                               a CG breakdown) above solver_tol            */
  LRFG_RANK_LIMITED = 2,    /* A_H written; a low-rank corrector stopped
                               because its truncated residual stopped
                               decreasing above solver_tol (the floor the
                               rank cap sets, Sec. 4.3); the best iterate is
                               kept.  Worse than OK, better than
                               NOT_CONVERGED when statuses are combined     */
  LRFG_EINVAL = -1,         /* bad argument (d, even or < 3 N, rank_cap < 1,
                               negative or NaN tolerance, CP with d = 3, ...) */
  LRFG_ECOEFF = -2,         /* coefficient not finite and positive           */
  LRFG_EWORKSPACE = -3,     /* workspace too small or misaligned             */
  LRFG_EDEVICE = -4,        /* HIP error or no usable gfx950 device           */
  LRFG_EUNSUPPORTED = -5    /* valid request this build does not implement   */
} lrfg_status;

typedef enum {
  LRFG_FORMAT_FULL = 0,
  LRFG_FORMAT_CP = 1,       /* d = 2 only (Sec. 3.1.1)                       */
  LRFG_FORMAT_TUCKER = 2,   /* Sec. 3.1.2, Appendix A.2                      */
  LRFG_FORMAT_TT = 3        /* Sec. 3.1.3, Appendix A.3                      */
} lrfg_format;

typedef enum {
  LRFG_SOLVER_PCG = 0,      /* preconditioned conjugate gradients            */
  LRFG_SOLVER_MR = 1        /* minimal-residual iteration (Sec. 3.3)         */
} lrfg_solver;

/* Mixed precision (TT, Tucker and CP formats): iterative refinement whose inner
 * truncated solves run the truncation's contractions with FP32 inputs and
 * FP32 accumulation (FP32), or its sketch contractions on BF16 MFMA with
 * each operand split into two BF16 terms (hi + lo, three products, FP32
 * accumulation) and its projections with FP32 inputs (BF16) (inner tolerance
 * max(solver_tol, 1e-4) for FP32, max(solver_tol, 1e-2) for BF16), while the
 * correction update,
 * the residual b - K x, the small factorisations of the truncation, the
 * solver scalars and A_H stay FP64; it stops when the FP64 preconditioned
 * residual reaches solver_tol or when two outer steps in a row fail to
 * lower the energy form of A_H E.E (Sec. 4.3) by solver_tol^2 of itself,
 * and returns the lowest-energy iterate.  Under BF16 the first outer step
 * without an energy gain moves the remaining inner solves to FP32. */
typedef enum {
  LRFG_PREC_FP64 = 0,
  LRFG_PREC_MIXED_FP32 = 1,
  LRFG_PREC_MIXED_BF16 = 2
} lrfg_precision;

/* Discretisation of the bilinear form (Sec. 2.2). */
typedef enum {
  LRFG_DISC_GANI = 0,       /* numerical integration on the grid (Sec. 2.2.2,
                               eq. ls_GaNi_fourier)                          */
  LRFG_DISC_GA = 1          /* exact integration on a double grid of at
                               least 2N - 1 points (lrfg_ga_double_grid;
                               DoGIP, Sec. 2.2.3, eq. ls_Ga_fourier): the
                               coefficient's Fourier integrals up to |m| <= N-1
                               on the double grid, trial and test functions in
                               T_N (every iterate masked to, every low-rank
                               train projected onto, its frequencies); full
                               grid and TT/CP in FP64                        */
} lrfg_discretisation;

/* Inclusion coefficients with closed-form Fourier integrals (Ga only). */
typedef enum {
  LRFG_INCLUSION_NONE = 0,
  LRFG_INCLUSION_SQUARE = 1,  /* centred square (2D) / cube (3D), |x_i| < size */
  LRFG_INCLUSION_BALL = 2     /* centred ball |x| < size (3D)                  */
} lrfg_inclusion;

/* Problem description (the paper's problem statement, Sec. 2.1-2.3, 3.2). */
typedef struct {
  int d;                /* 2 or 3                                            */
  int N[3];             /* odd grid sizes >= 3 (Sec. 2.2.1: odd N only)      */
  int format;           /* lrfg_format of the corrector                      */
  int rank_cap;         /* low-rank formats: maximal rank kept by truncation */
  double trunc_tol;     /* relative truncation tolerance (0: rank cap only)  */
  double solver_tol;    /* stop at ||P^-1 r|| <= solver_tol ||P^-1 b||       */
  int max_iter;         /* iteration limit per corrector (>= 1)              */
  int solver;           /* lrfg_solver                                       */
  int precision;        /* lrfg_precision                                    */
  int precond_terms;    /* low-rank: exponential-sum terms M (0 = automatic) */
  int oversample;       /* low-rank: sketch oversampling p (0 = automatic)   */
  uint64_t seed;        /* low-rank: seed of the sketching generator         */
  int coeff_rank;       /* low-rank: upper bound on the coefficient's rank
                           (CP terms or TT ranks) a solve will receive;
                           sizes the workspace (0 = 16)                      */
  uint32_t flags;       /* reserved, must be 0                               */
  double aniso[9];      /* constant symmetric positive semi-definite matrix B
                           added to the isotropic coefficient, A~(x) =
                           a(x) I + B (the anisotropic materials of Sec.
                           4.4), row-major d x d in the first d*d entries,
                           the rest 0.  All zero: the isotropic problem.
                           Non-symmetric (beyond 1e-12 max|B|), indefinite
                           or non-finite B, or nonzero entries past d*d:
                           LRFG_EINVAL.  Full-grid and TT/CP formats;
                           Tucker with B != 0: LRFG_EUNSUPPORTED           */
  int rank_start;       /* TT/CP, FP64 PCG: rank-adaptive solve (Sec. 4.2: a
                           solver that starts at a low solution rank and
                           raises it during the iterations) when 0 <
                           rank_start < rank_cap: stages at the caps
                           rank_start, then x1.5 (at least +1) up to
                           rank_cap, each started from the previous stage's
                           corrector; a system leaves at the stage that
                           reaches solver_tol.  0 (or >= rank_cap): one
                           solve at rank_cap.  Negative: LRFG_EINVAL; other
                           formats, precisions or solvers with rank_start >
                           0: LRFG_EUNSUPPORTED                            */
  int discretisation;   /* lrfg_discretisation; LRFG_DISC_GA (full grid,
                           TT and CP) takes an inclusion coefficient
                           (lrfg_coeff; the low-rank formats the square/cube
                           only) and runs on the double grid
                           lrfg_ga_double_grid(N)                           */
} lrfg_problem;

/* Coefficient a(x) > 0 (scalar isotropic A = a I).  For FULL, `full` holds
 * a[N1*...*Nd] (C order).  For the low-rank formats the coefficient is given
 * in the CP form a = sum_t w[t] prod_i f_i[t, j_i]: `weights` (R values) and
 * `factors[i]` (R x N_i, row-major) -- every coefficient of the paper's
 * workloads is given this way (Sec. 4.1: rank 2 inclusions, rank-limited
 * smooth fields) -- or in TT form (`tt_cores[i]`, [r_{i-1}][N_i][r_i],
 * tt_ranks[0..d]) -- or, for the Tucker format (d = 3), in Tucker form
 * (Sec. 3.1.2: a = core x_1 U_1 x_2 U_2 x_3 U_3; `tucker_core`
 * [r_1][r_2][r_3], `tucker_frames[i]` N_i x r_i row-major, i.e. the columns
 * are the mode vectors, tucker_ranks[0..2]; lrfg_compress_tucker writes this
 * layout).  Exactly one of full / weights / tt_cores / tucker_core is
 * non-NULL.  The full-grid format takes full, CP or TT coefficients, the TT
 * and CP formats CP or TT, the Tucker format CP or Tucker (anything else:
 * LRFG_EUNSUPPORTED).  Pointers are host addresses unless on_device != 0.
 * Borrowed for the call.
 */
typedef struct {
  int on_device;
  const double* full;
  int rank;                       /* CP form: number of terms R                 */
  const double* weights;          /* CP form: R                                 */
  const double* factors[3];       /* CP form: R x N_i                           */
  int tt_ranks[4];                /* TT form: r_0..r_d (r_0 = r_d = 1)           */
  const double* tt_cores[3];      /* TT form                                    */
  int tucker_ranks[3];            /* Tucker form: r_1..r_3                      */
  const double* tucker_core;      /* Tucker form: [r_1][r_2][r_3]               */
  const double* tucker_frames[3]; /* Tucker form: N_i x r_i                      */
  int inclusion;                  /* lrfg_inclusion (LRFG_DISC_GA only): value
                                     incl_inside in the inclusion of half side /
                                     radius incl_size in (0, 1/2), incl_outside
                                     elsewhere (both > 0)                      */
  double incl_size, incl_inside, incl_outside;
} lrfg_coeff;

/* Results, host memory owned by the caller (any pointer may be NULL). */
typedef struct {
  double* A_H;        /* nE*nE row-major: A_H E_i . E_j (= A_H for E = I)    */
  int* iters;         /* nE: iterations per corrector                        */
  double* res_hist;   /* nE*max_iter: relative preconditioned residual norm,
                         the Euclidean norm of the residual's Fourier
                         coefficients (Sec. 4.2); unused entries set to 0    */
  int* ranks;         /* nE*(d+1): ranks of the returned corrector: TT r_0..r_d;
                         Tucker r_1, r_2, r_3 then 0                        */
  int* status;        /* nE: per-corrector lrfg_status                       */
  double setup_ms;    /* coefficient upload/compression, transforms          */
  double solve_ms;    /* iterations and A_H evaluation                       */
} lrfg_result;

typedef struct lrfg_plan lrfg_plan;

/* Version of this ABI (LRFG_ABI_VERSION). */
int lrfg_abi_version(void);

/* The double grid M that the Ga discretisation (Sec. 2.2.3) uses for N points
 * per axis.  Products of two gradients of T_N carry frequencies |m| <= N - 1,
 * so every odd grid of at least 2N - 1 points integrates the bilinear and
 * energy forms exactly; the paper takes 2N - 1.  Returned: the smallest odd
 * 3^a 5^b >= 2N - 1 (all transforms on the fast passes), or 2N - 1 when that
 * exceeds 2048.  The solution is the same on any such grid, up to rounding.
 * N must be odd and in [1, 1024] (else LRFG_EINVAL).  Host only. */
int lrfg_ga_double_grid(int N);

/* Static description of a status code. */
const char* lrfg_status_string(int status);

/* Thread-local message of the last failing call ("" if none). */
const char* lrfg_last_error(void);

/* LRFG_OK if a HIP device is visible and usable, else LRFG_EDEVICE. */
int lrfg_device_check(void);

/* Validate `p` and build a host-side plan (FFT factorisations, twiddle
 * tables, workspace layout).  No device call.  *out is owned by the caller
 * and released with lrfg_plan_destroy. */
int lrfg_plan_create(const lrfg_problem* p, lrfg_plan** out);

/* Device workspace (bytes) lrfg_solve needs for up to `max_nE` macroscopic
 * fields. */
int lrfg_plan_workspace_bytes(const lrfg_plan* plan, int max_nE, size_t* bytes);

/* Solve the d cell problems for E_1..E_nE and form A_H (eq. homog).
 * E: host array nE x d (row-major) or NULL for the canonical basis (nE = d).
 * Stream-ordered; synchronises `stream` before writing host results.
 * Returns LRFG_NOT_CONVERGED if some corrector stopped at max_iter, else
 * LRFG_RANK_LIMITED if some corrector stopped at its rank floor (per-corrector
 * statuses in out->status). */
int lrfg_solve(lrfg_plan* plan, const lrfg_coeff* a, const double* E, int nE,
               void* d_ws, size_t ws_bytes, void* stream, lrfg_result* out);

/* Allocation-free solve, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): lrfg_solve with the library's own device workspace, one array
 * of LRFG_NOALLOC_BYTES per GPU (held until the process ends) in place of
 * d_ws.  The call allocates no device or pinned host memory (the plan must
 * have been created with a device present; full-grid plans take their
 * pinned flag ring there).  Every call on one GPU uses that GPU's array:
 * calls that overlap on one GPU (other threads or streams) race and must be
 * serialised by the caller.  The array keeps the last call's contents;
 * nothing in a solve depends on them.  Returns LRFG_EWORKSPACE when
 * lrfg_plan_workspace_bytes(plan, nE) exceeds LRFG_NOALLOC_BYTES (checked
 * before any device call), otherwise as lrfg_solve. */
#define LRFG_NOALLOC_BYTES ((size_t)128 << 20)
int lrfg_solve_noalloc(lrfg_plan* plan, const lrfg_coeff* a, const double* E, int nE, void* stream,
                       lrfg_result* out);

/* Batched solve: `count` microstructures a[0..count-1] of the same problem
 * (and, for the low-rank formats, the same coefficient ranks), each with
 * the nE fields E, one result each in results[0..count-1].  The low-rank
 * formats run all count*nE correctors as one batch through every kernel
 * (count*nE <= 256; workspace lrfg_plan_workspace_bytes(plan, count*nE));
 * the full grid runs the microstructures one after another in the
 * workspace of one (lrfg_plan_workspace_bytes(plan, nE)).  Each result
 * equals that of lrfg_solve on the same microstructure up to rounding
 * (the batched kernels split their sums differently).  Errors as
 * lrfg_solve; LRFG_EINVAL also for count < 1 or unequal coefficient
 * ranks. */
int lrfg_solve_batch(lrfg_plan* plan, const lrfg_coeff* a, int count, const double* E, int nE,
                     void* d_ws, size_t ws_bytes, void* stream, lrfg_result* results);

void lrfg_plan_destroy(lrfg_plan* plan);

/* ------------------------------------------------------------------------
 * Operation-level entry points: the kernels of the solve paths, exposed so
 * that each can be checked on its own.  Device pointers, stream-ordered,
 * no allocation, no synchronisation.
 * ---------------------------------------------------------------------- */

/* Batched 1-D DFT of length N along the middle index of a complex array
 * x[outer][N][inner] (interleaved re,im FP64), in place.  direction -1 is
 * the forward transform F_N with its 1/N factor, +1 the unnormalised
 * inverse (Sec. 2.2.1, DFT matrices).  Odd N only.
 * d_ws: lrfg_fft_workspace_bytes(N) bytes (twiddle table). */
size_t lrfg_fft_workspace_bytes(int N);
int lrfg_fft_lines(double* x, int outer, int N, int inner, int direction,
                   void* d_ws, size_t ws_bytes, void* stream);

/* Real circulant operator along the middle index of a real array
 * x[outer][N][inner], in place: x <- F^-1 diag(s(k)) F x per fibre, with
 *   op 0: s(k) = 2 pi i k                (spectral derivative, eq. grad_trig)
 *   op 1: s(k) = exp(-t k^2)             (heat kernel factor of the
 *                                         exponential-sum preconditioner)
 *   op 2: s(k) = 1 for |k| <= t, else 0  (projection onto the trigonometric
 *                                         polynomials of degree t: the
 *                                         low-rank Ga's N-frequencies)
 * k the centred frequency.  This is the per-mode 1-D DFT the low-rank
 * formats apply to their factors (Sec. 3.1, Appendix A). */
int lrfg_mode_op(double* x, int outer, int N, int inner, int op, double t,
                 void* d_ws, size_t ws_bytes, void* stream);

/* Full-grid operator on half-spectrum arrays u[N1][N2][(N3+1)/2] (complex):
 *   which 0: out = K u  = grad*^ F a F^-1 grad^ u    (eq. ls_GaNi_fourier)
 *   which 1: out = P^-1 u = u / (4 pi^2 k.k), 0 at k = 0 (Sec. 2.3)
 * `a` is the real coefficient [N1][N2][N3] on the device. d = 3 only.
 * d_ws: lrfg_full_op_workspace_bytes bytes. */
size_t lrfg_full_op_workspace_bytes(const int N[3]);
int lrfg_full_op(int which, const int N[3], const double* a, const double* u,
                 double* out, void* d_ws, size_t ws_bytes, void* stream);

/* FP64 batched matrix product on the matrix cores (MFMA):
 *   C_b = alpha op(A_b) op(B_b) + beta C_b,  b in [0, batch),
 * row-major with leading dimensions lda/ldb/ldc and batch strides sA/sB/sC
 * (elements); op = transpose when ta / tb != 0; op(A) is m x k, op(B) k x n.
 * beta = 0 does not read C.  d_ws (lrfg_gemm_workspace_bytes) holds split-K
 * partial sums; a smaller workspace only disables the split.  These are the
 * core contractions and Gram products of the truncation (Appendix A.3). */
size_t lrfg_gemm_workspace_bytes(int m, int n, int k, int batch);
int lrfg_gemm(int ta, int tb, int m, int n, int k, double alpha, const double* A, long long lda,
              long long sA, const double* B, long long ldb, long long sB, double beta, double* C,
              long long ldc, long long sC, int batch, void* d_ws, size_t ws_bytes, void* stream);

/* lrfg_gemm with the operands rounded to FP32 (LRFG_PREC_MIXED_FP32) or
 * BF16 (LRFG_PREC_MIXED_BF16) and the products accumulated in FP32 on MFMA
 * (v_mfma_f32_16x16x4f32 / v_mfma_f32_16x16x32_bf16); A, B and C stay FP64
 * in memory, split-K partial sums are added in FP64.  The core
 * contractions of the mixed-precision low-rank solve run here.
 * LRFG_PREC_FP64 is lrfg_gemm.  Workspace as lrfg_gemm_workspace_bytes. */
int lrfg_gemm_mixed(int precision, int ta, int tb, int m, int n, int k, double alpha, const double* A,
                    long long lda, long long sA, const double* B, long long ldb, long long sB,
                    double beta, double* C, long long ldc, long long sC, int batch, void* d_ws,
                    size_t ws_bytes, void* stream);

/* Batched symmetric eigendecomposition (cyclic Jacobi), n <= 64: A is
 * batch x n x n (row-major, symmetrised as (A + A^T)/2), W receives the
 * eigenvalues in descending order (batch x n), V the eigenvectors as
 * columns (batch x n x n).  The small SVDs of the truncation are taken
 * from these Gram eigenpairs (Sec. 3.1.4). */
int lrfg_syevj(int n, const double* A, int batch, double* W, double* V, void* stream);

/* Truncation basis of batched symmetric positive semidefinite Gram
 * matrices (the l x l Gram matrices of the truncation's SVD cut, Sec. 3.1.4
 * and Appendix A.3), n <= 128, all pointers device: G is batch x n x n
 * (row-major); S (batch x n x c) receives the eigenvectors of the kept
 * eigenvalues as columns, largest first, with zero columns beyond the kept
 * count.  Kept: at most c, above the rank threshold of the pivoted
 * Cholesky factorisation G = L^T L (largest remaining diagonal > 1e-15 of
 * the largest initial one), and, when tol > 0, the fewest whose dropped
 * eigenvalue sum (with the mass below that threshold) is at most
 * tol^2 trace(G).  The eigenpairs come from one-sided Jacobi on the columns
 * of L^T.  kept and sweeps (batch ints each: kept count, Jacobi sweeps
 * used) may be NULL.  Stream-ordered; returns LRFG_EINVAL for n outside
 * [1, 128], c < 1, negative or NaN tol or null G/S. */
int lrfg_gram_cut(int n, int c, const double* G, int batch, double tol, double* S, int* kept, int* sweeps,
                  void* stream);

/* TT truncation (rounding, Appendix A.3) of nE trains with input ranks
 * rin[0..d] (rin[0] = rin[d] = 1), carriages in_cores[j] = nE x
 * [r_{j-1}][N_j][r_j] (device).  Output ranks are fixed,
 * c_j = min(cap, N-bounds), written to out_ranks (host, d+1 ints); the
 * directions beyond the kept rank (at most c_j, the fewest whose dropped
 * singular values satisfy ||dropped||^2 <= tol^2 ||X||^2 / (d-1)) are zero.
 * kept (host, 2*nE ints or NULL) receives the kept ranks: bond 1 for every
 * system, then bond 2.  The truncation is randomised (Gaussian TT sketch of
 * ranks c_j + oversample, seeded by seed) and exact whenever the input rank
 * at a bond is at most c_j + oversample.  Synchronises the stream when kept
 * is non-NULL. */
size_t lrfg_tt_round_workspace_bytes(int d, const int N[3], const int rin[4], int cap,
                                     int oversample, int nE);
int lrfg_tt_round(int d, const int N[3], const int rin[4], double* const* in_cores, int cap,
                  double tol, int oversample, uint64_t seed, double* const* out_cores,
                  int* out_ranks, int* kept, int nE, void* d_ws, size_t ws_bytes, void* stream);

/* Tucker truncation (Appendix A.2) of nE tensors of mode ranks rin (d = 3):
 * frames in_frames[j] = nE x [N_j][rin_j] (row-major: columns are the mode
 * fibres), core in_core = nE x [rin_1][rin_2][rin_3] (device).  Output
 * mode ranks are fixed, c_j = min(cap, N_j) (written to out_ranks, host,
 * 3 ints), frames out_frames[j] = nE x [N_j][c_j], core out_core =
 * nE x [c_1][c_2][c_3]; directions beyond the kept rank (at most c_j, the
 * fewest whose dropped singular values of the mode-j unfolding satisfy
 * ||dropped||^2 <= tol^2 ||X||^2 / 3) are zero.  Randomised HOSVD with
 * Khatri-Rao structured sketches of size min(max c_j + oversample, 64),
 * seeded by seed; exact whenever every mode rank is at most that.  kept
 * (host, 3*nE ints, mode-major, or NULL) receives the kept ranks and makes
 * the call synchronise the stream. */
size_t lrfg_tucker_round_workspace_bytes(const int N[3], const int rin[3], int cap, int oversample, int nE);
int lrfg_tucker_round(const int N[3], const int rin[3], double* const* in_frames, const double* in_core,
                      int cap, double tol, int oversample, uint64_t seed, double* const* out_frames,
                      double* out_core, int* out_ranks, int* kept, int nE, void* d_ws, size_t ws_bytes,
                      void* stream);

/* Coefficient compression (setup of the low-rank path, Sec. 3.1.3 and
 * Appendix A.3): the full field a (device, N1 x ... x Nd, C order) as a
 * tensor train with ranks at most cap, the fewest directions whose dropped
 * singular values satisfy ||dropped||^2 <= tol^2 ||a||^2 / (d-1) (tol = 0:
 * cap only).  The field enters as the exact train (I, a, I) of ranks
 * (1, N1, N3, 1) (d = 2: (1, N1, 1)) and goes through the same randomised
 * TT rounding as lrfg_tt_round (sketch ranks cap + oversample <= 64).
 * out_cores[j] (device) receive [c_{j-1}][N_j][c_j] with the nominal ranks
 * c (written to out_ranks, host, d+1 ints; directions beyond the kept rank
 * are zero); kept (host, d-1 ints, or NULL) the kept ranks.  The TT solve
 * takes the cores as its coefficient (tt_ranks = out_ranks); the full-grid
 * solve of the same coefficient takes them too (it expands them), so both
 * solve for the compressed field. */
size_t lrfg_compress_workspace_bytes(int d, const int N[3], int cap, int oversample);
int lrfg_compress_tt(int d, const int N[3], const double* a, int cap, double tol, int oversample,
                     uint64_t seed, double* const* out_cores, int* out_ranks, int* kept, void* d_ws,
                     size_t ws_bytes, void* stream);

/* Coefficient compression to the Tucker form (setup of the Tucker path,
 * Sec. 3.1.2 and Appendix A.2): the full field a (device, N1 x N2 x N3,
 * C order) as a Tucker tensor with mode ranks at most cap, the fewest
 * directions per mode whose dropped singular values of the unfolding
 * satisfy ||dropped||^2 <= tol^2 ||a||^2 / 3 (tol = 0: cap only).  The
 * field enters as the exact Tucker tensor (core a, identity frames) and
 * goes through the randomised HOSVD of lrfg_tucker_round (sketch size
 * min(cap + oversample, 64)).  out_frames[j] (device) receive N_j x c_j,
 * out_core c_1 x c_2 x c_3, c_j = min(cap, N_j) (out_ranks, host, 3 ints;
 * directions beyond the kept rank are zero); kept (host, 3 ints, or NULL)
 * the kept ranks.  The Tucker solve takes them as its coefficient
 * (tucker_frames, tucker_core, tucker_ranks = out_ranks). */
size_t lrfg_compress_tucker_workspace_bytes(const int N[3], int cap, int oversample);
int lrfg_compress_tucker(const int N[3], const double* a, int cap, double tol, int oversample, uint64_t seed,
                         double* const* out_frames, double* out_core, int* out_ranks, int* kept, void* d_ws,
                         size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Serving: a request loop with continuous batching on one device.
 * Requests wait in a queue until the caller's device pool (d_pool,
 * pool_bytes, 256-byte aligned, owned by the caller and untouched outside
 * the requests' workspaces) has room for their workspace: the oldest
 * request that fits is taken with the other queued requests of the same
 * problem, fields and coefficient ranks, up to max_batch of them (a
 * low-rank batch holds at most 256 correctors, so at most 256 / nE
 * requests), and becomes a session solved as one lrfg_solve_batch on a host
 * thread and HIP stream (default priority) of its own.  Sessions share
 * `slots` device permits, granted in arrival order; a session gives its
 * permit back between iterations (every iteration of the low-rank solvers,
 * every four of the full-grid PCG) and queues for it again, so sessions run
 * in turns of iteration blocks and up to `slots` of them have work on the
 * device at once.  Admission happens at once while a permit is free and
 * otherwise at the next such block boundary: a request that arrives while
 * others run joins the rotation there (with the requests queued meanwhile,
 * batched), and a finished session leaves it there, without waiting for
 * other solves to end.  At most 4 slots sessions are admitted at a time.
 * Results equal those of lrfg_solve up to rounding.
 * ---------------------------------------------------------------------- */
typedef struct lrfg_server lrfg_server;

typedef struct {
  uint64_t tag;           /* the submit call's tag                          */
  int status;             /* lrfg_status of the request                     */
  int batch_size;         /* microstructures solved in the same batch       */
  double queue_ms;        /* submit to start of its batch (host clock)      */
  double run_ms;          /* its batch's solve time                         */
  double total_ms;        /* submit to completion                           */
  size_t workspace_bytes; /* pool bytes its batch held                      */
} lrfg_completion;

/* Start the loop on `device` with `slots` device permits (in [1, 16]) and
 * batches of up to max_batch (>= 1) requests.  Returns LRFG_EINVAL for bad
 * arguments, LRFG_EDEVICE for a missing device. */
int lrfg_server_create(int device, int slots, int max_batch, void* d_pool, size_t pool_bytes,
                       lrfg_server** out);

/* Queue one request: problem p (copied), coefficient a and the arrays it
 * points to (read in place when its batch runs: keep them valid and
 * unchanged until the completion is polled), fields E (nE x d, copied;
 * NULL = canonical basis with nE = d), result `out` (the struct and its
 * arrays are written by the worker; read them after the completion).
 * Device coefficients (a->on_device) may still be being written by work
 * queued on `stream` (the caller's stream; NULL = the default stream): an
 * event recorded there at submit orders the worker's reads after that
 * work.  Work the caller queues on other streams must be complete before
 * submit.  Returns the plan-validation codes of lrfg_plan_create,
 * LRFG_EWORKSPACE when the request's workspace exceeds the whole pool,
 * LRFG_EDEVICE when the event cannot be recorded. */
int lrfg_server_submit(lrfg_server* s, const lrfg_problem* p, const lrfg_coeff* a, const double* E,
                       int nE, lrfg_result* out, uint64_t tag, void* stream);

/* Move up to `max` completions into done[0..*n-1]; waits up to timeout_ms
 * for the first (0: no wait, < 0: until one arrives). */
int lrfg_server_poll(lrfg_server* s, lrfg_completion* done, int max, int* n, int timeout_ms);

/* Requests queued or running. */
int lrfg_server_pending(lrfg_server* s);

/* Finish every queued and running request, then stop the workers (the
 * completions not yet polled are dropped). */
void lrfg_server_destroy(lrfg_server* s);

/* ------------------------------------------------------------------------
 * Kernel timing (measurement support).  lrfg_prof_enable(name) makes every
 * later launch of the kernel `name` (one of "fft_lines", "fft_axis2",
 * "mode_op", "mode_op_blocks", "grad_axis1", "axis3", "div_axis1",
 * "cg_update1", "cg_update2", "gemm", "syevj", "pchol", "cut",
 * "khatri_rao", "tt_round"; "fft_axis2" is the axis-2 pass of the
 * full-grid PCG matvec, "gemm" the MFMA GEMM kernel without its split-K
 * reduction) bracketed by HIP events on the stream it runs on; NULL
 * disables and clears.  Every call destroys the events of the previous
 * timing (a recorded event keeps the memory its launch used from returning
 * to the device when it is freed), so read before switching.
 * lrfg_prof_read synchronises those events and
 * returns the number of timed launches and their summed duration in
 * milliseconds; lrfg_prof_work returns the summed algorithmic work of those
 * launches: FLOPs (2 m n k per GEMM) for "gemm", bytes read plus written
 * (16 bytes per complex value, every line once each way) for the FFT line
 * passes, 0 for the others.  Process-wide state.
 * ---------------------------------------------------------------------- */
int lrfg_prof_enable(const char* kernel);
int lrfg_prof_read(int* count, double* total_ms);
int lrfg_prof_work(double* total_work);

#ifdef __cplusplus
}
#endif

#endif /* LRFG_H */
