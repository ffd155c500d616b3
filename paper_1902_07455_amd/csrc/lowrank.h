// Low-rank (CP / Tucker / TT) solve path (internal interface) and the
// coefficient staging shared with the full-grid path.
#pragma once

#include "fft.h"

namespace lrfg {

struct LowRankPlan;

// Coefficient given in CP or TT form, expanded to a full field on the device
// (setup of the full-grid path).  Staging limits: CP rank <= kMaxCoeffRank,
// TT ranks <= kMaxCoeffRank.
constexpr int kMaxCoeffRank = 128;
size_t coeff_staging_bytes(const lrfg_problem& p);
int expand_coeff(const lrfg_problem& p, const lrfg_coeff& a, double* dst, size_t bytes, hipStream_t s);

// Admissibility of a low-rank coefficient (all device pointers): the
// smallest value of its expansion and the number of non-finite values,
// computed row by row without storing the field (synchronises s).
// TT: cores[j] = [rk[j]][N[j]][rk[j+1]], d = 2 or 3.  Tucker (d = 3): core
// [r1][r2][r3], frames U[j] = [N[j]][r[j]], W scratch of N[0] r[1] r[2]
// doubles.  scratch: 16 bytes of device memory.
int tt_coeff_check(int d, const int N[3], const int rk[4], const double* const* cores, void* scratch,
                   hipStream_t s, double* min_out, long long* nonfinite_out);
int tucker_coeff_check(const int N[3], const int r[3], const double* core, const double* const* U, double* W,
                       void* scratch, hipStream_t s, double* min_out, long long* nonfinite_out);

// ga_N: Ga (Sec. 2.2.3) with p.N the double grid 2 ga_N - 1 (NULL: GaNi).
int lowrank_plan_create(const lrfg_problem& p, const FftPlan* mode, LowRankPlan** out,
                        const int* ga_N = nullptr);
void lowrank_plan_destroy(LowRankPlan* lr);
// Systems in one solve (microstructures x fields) are limited to this.
constexpr int kMaxSystems = 256;
size_t lowrank_workspace_bytes(const LowRankPlan* lr, int max_nE);
// nB microstructures (coefficients a[0..nB-1], equal ranks), each with the
// nE fields E (nE x d), solved as one batch of nB nE trains; out[b]
// receives microstructure b's nE x nE A_H and per-field diagnostics.
int lowrank_solve(LowRankPlan* lr, const lrfg_coeff* a, int nB, const double* E, int nE, void* ws,
                  size_t ws_bytes, hipStream_t s, lrfg_result* out);

}  // namespace lrfg
