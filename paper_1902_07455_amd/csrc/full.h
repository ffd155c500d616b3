// Full-grid GaNi PCG solve (internal interface).
#pragma once

#include "fft.h"

namespace lrfg {

struct FullSolveArgs {
  int d;
  int N[3];
  const FftPlan* plan1;   // internal axis lengths (d = 2: 1, N1, N2)
  const FftPlan* plan2;
  const FftPlan* plan3;
  const double* a;        // coefficient nodal values
  int a_on_device;
  const double* E;        // host nE x d
  int nE;
  double tol;
  int max_iter;
  void* ws;
  size_t ws_bytes;
  void* stream;
  int* pinned_flags;      // pinned host ints, 4 * nE
  double B[9] = {};       // constant anisotropic part, d x d row-major (all 0: isotropic)
  // Ga (exact integration, Sec. 2.2.3): N above is the double grid 2 ga_N - 1,
  // a is built from the inclusion's Fourier integrals, and every iterate is
  // kept on the frequencies of ga_N (0: GaNi)
  int ga_N[3] = {0, 0, 0};
  int incl = 0;           // lrfg_inclusion
  double incl_size = 0.0, incl_in = 0.0, incl_out = 0.0;
};

struct FullSolveOut {
  double* A_H;
  int* iters;
  double* res_hist;
  int* status;
  double setup_ms;
  double solve_ms;
};

size_t full_workspace_bytes(const int N3d[3], int nE, int d, int max_iter);
int full_solve(const FullSolveArgs& a, FullSolveOut* out);
size_t full_op_workspace_bytes(const int N[3]);
int full_op(int which, const int N[3], const FftPlan* p1, const FftPlan* p2, const FftPlan* p3,
            const double* a, const double* u, double* out, void* ws, size_t ws_bytes, hipStream_t s);

}  // namespace lrfg
