// C ABI of liblrfg: validation, plans, dispatch to the solve paths and the
// operation-level entry points.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <mutex>
#include <vector>

#include "common.h"
#include "fft.h"
#include "full.h"
#include "lowrank.h"

namespace lrfg {

static thread_local std::string g_last_error;

void set_error(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
}

void clear_error() { g_last_error.clear(); }

}  // namespace lrfg

using namespace lrfg;

struct lrfg_plan {
  lrfg_problem p;
  int N3d[3];            // full grid: internal 3-D geometry (d = 2: 1, N1, N2)
  FftPlan axis[3];       // plans for N3d
  FftPlan mode[3];       // plans for the user's N_i (low-rank mode transforms)
  int* pinned = nullptr; // pinned host flags for the full-grid loop
  int pinned_n = 0;
  LowRankPlan* lr = nullptr;
};

namespace {

bool finite_nonneg(double v) { return std::isfinite(v) && v >= 0.0; }

// Ga's double grid for n points per axis: the products of two gradients of
// T_n have frequencies |m| <= n - 1, so any odd grid of at least 2n - 1
// points integrates the bilinear and energy forms exactly (Sec. 2.2.3 takes
// 2n - 1, the smallest).  The smallest odd 3^a 5^b >= 2n - 1 keeps every
// transform on the register passes; above 2025 (the largest below the grid
// limit 2048) the grid stays at 2n - 1.
int ga_double_grid(int n) {
  const int lo = 2 * n - 1;
  int best = 0;
  for (long long p3 = 1; p3 <= 2048; p3 *= 3)
    for (long long v = p3; v <= 2048; v *= 5)
      if (v >= lo && (best == 0 || v < best)) best = (int)v;
  return best > 0 ? best : lo;
}

int validate(const lrfg_problem* p) {
  if (p == nullptr) {
    set_error("problem is NULL");
    return LRFG_EINVAL;
  }
  if (p->d != 2 && p->d != 3) {
    set_error("d must be 2 or 3 (got %d)", p->d);
    return LRFG_EINVAL;
  }
  for (int i = 0; i < p->d; ++i) {
    if (p->N[i] < 3 || (p->N[i] % 2) == 0) {
      set_error("N[%d] = %d: grid sizes must be odd and >= 3", i, p->N[i]);
      return LRFG_EINVAL;
    }
  }
  for (int i = 0; i < p->d; ++i) {
    if (p->N[i] > 2048) {
      set_error("N[%d] = %d: grid sizes above 2048 are not supported", i, p->N[i]);
      return LRFG_EUNSUPPORTED;
    }
  }
  if (p->format < LRFG_FORMAT_FULL || p->format > LRFG_FORMAT_TT) {
    set_error("unknown format %d", p->format);
    return LRFG_EINVAL;
  }
  if (p->format == LRFG_FORMAT_CP && p->d != 2) {
    set_error("CP format is used for d = 2 only");
    return LRFG_EINVAL;
  }
  if (p->format != LRFG_FORMAT_FULL && p->rank_cap < 1) {
    set_error("rank_cap must be >= 1 (got %d)", p->rank_cap);
    return LRFG_EINVAL;
  }
  if (!finite_nonneg(p->trunc_tol)) {
    set_error("trunc_tol must be finite and >= 0");
    return LRFG_EINVAL;
  }
  if (!(std::isfinite(p->solver_tol) && p->solver_tol > 0.0)) {
    set_error("solver_tol must be finite and > 0");
    return LRFG_EINVAL;
  }
  if (p->max_iter < 1) {
    set_error("max_iter must be >= 1");
    return LRFG_EINVAL;
  }
  if (p->solver != LRFG_SOLVER_PCG && p->solver != LRFG_SOLVER_MR) {
    set_error("unknown solver %d", p->solver);
    return LRFG_EINVAL;
  }
  if (p->precision < LRFG_PREC_FP64 || p->precision > LRFG_PREC_MIXED_BF16) {
    set_error("unknown precision %d", p->precision);
    return LRFG_EINVAL;
  }
  if (p->precond_terms < 0 || p->precond_terms == 1 || p->oversample < 0) {
    set_error("precond_terms must be 0 or >= 2; oversample >= 0");
    return LRFG_EINVAL;
  }
  if (p->flags != 0) {
    set_error("flags must be 0");
    return LRFG_EINVAL;
  }
  {
    // B (Sec. 4.4): finite, symmetric and positive semi-definite (every
    // principal minor >= 0, to a rounding margin), zero past d x d
    const int d = p->d;
    double m = 0.0;
    for (int i = 0; i < 9; ++i) {
      if (!std::isfinite(p->aniso[i])) {
        set_error("aniso[%d] is not finite", i);
        return LRFG_EINVAL;
      }
      if (i >= d * d && p->aniso[i] != 0.0) {
        set_error("aniso[%d] must be 0 for d = %d (B is d x d, row-major)", i, d);
        return LRFG_EINVAL;
      }
      m = std::max(m, std::fabs(p->aniso[i]));
    }
    if (m > 0.0) {
      auto b = [&](int i, int j) { return p->aniso[i * d + j]; };
      const double eps = 1e-12;
      bool ok = true;
      for (int i = 0; i < d; ++i)
        for (int j = i + 1; j < d; ++j) ok = ok && std::fabs(b(i, j) - b(j, i)) <= eps * m;
      if (!ok) {
        set_error("aniso: B must be symmetric");
        return LRFG_EINVAL;
      }
      for (int i = 0; i < d; ++i) ok = ok && b(i, i) >= -eps * m;
      for (int i = 0; i < d; ++i)
        for (int j = i + 1; j < d; ++j) ok = ok && b(i, i) * b(j, j) - b(i, j) * b(j, i) >= -eps * m * m;
      if (d == 3) {
        const double det = b(0, 0) * (b(1, 1) * b(2, 2) - b(1, 2) * b(2, 1)) -
                           b(0, 1) * (b(1, 0) * b(2, 2) - b(1, 2) * b(2, 0)) +
                           b(0, 2) * (b(1, 0) * b(2, 1) - b(1, 1) * b(2, 0));
        ok = ok && det >= -eps * m * m * m;
      }
      if (!ok) {
        set_error("aniso: B must be positive semi-definite");
        return LRFG_EINVAL;
      }
      if (p->format == LRFG_FORMAT_TUCKER) {
        set_error("the anisotropic term is built for the full-grid and TT/CP formats");
        return LRFG_EUNSUPPORTED;
      }
    }
  }
  if (p->discretisation != LRFG_DISC_GANI && p->discretisation != LRFG_DISC_GA) {
    set_error("unknown discretisation %d", p->discretisation);
    return LRFG_EINVAL;
  }
  if (p->discretisation == LRFG_DISC_GA) {
    if (p->format == LRFG_FORMAT_TUCKER || (p->format != LRFG_FORMAT_FULL && p->precision != LRFG_PREC_FP64)) {
      set_error("the Ga discretisation is built for the full grid and the TT/CP formats in FP64");
      return LRFG_EUNSUPPORTED;
    }
    for (int i = 0; i < p->d; ++i)
      if (p->N[i] > 1024) {
        set_error("Ga: N[%d] = %d above 1024 (double grid above 2047)", i, p->N[i]);
        return LRFG_EUNSUPPORTED;
      }
  }
  if (p->rank_start < 0) {
    set_error("rank_start must be >= 0");
    return LRFG_EINVAL;
  }
  if (p->rank_start > 0 && p->rank_start < p->rank_cap &&
      (!(p->format == LRFG_FORMAT_TT || p->format == LRFG_FORMAT_CP) || p->precision != LRFG_PREC_FP64 ||
       p->solver != LRFG_SOLVER_PCG)) {
    set_error("the rank-adaptive solve is built for the TT/CP formats, FP64, PCG");
    return LRFG_EUNSUPPORTED;
  }
  if (p->format == LRFG_FORMAT_FULL && p->precision != LRFG_PREC_FP64) {
    set_error("the full-grid path runs in FP64 only");
    return LRFG_EUNSUPPORTED;
  }
  if (p->format == LRFG_FORMAT_FULL && p->solver != LRFG_SOLVER_PCG) {
    set_error("the full-grid path uses PCG");
    return LRFG_EUNSUPPORTED;
  }
  return LRFG_OK;
}

int device_ok() {
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n < 1) {
    (void)hipGetLastError();
    set_error("no HIP device available");
    return LRFG_EDEVICE;
  }
  return LRFG_OK;
}

}  // namespace

extern "C" {

int lrfg_abi_version(void) { return LRFG_ABI_VERSION; }

int lrfg_ga_double_grid(int N) {
  using namespace lrfg;
  clear_error();
  if (N < 1 || N % 2 == 0 || N > 1024) {
    set_error("Ga grid size N = %d: odd, in [1, 1024]", N);
    return LRFG_EINVAL;
  }
  return ga_double_grid(N);
}

const char* lrfg_status_string(int s) {
  switch (s) {
    case LRFG_OK: return "ok";
    case LRFG_NOT_CONVERGED: return "not converged (A_H written)";
    case LRFG_RANK_LIMITED: return "stopped at the rank cap's residual floor (A_H written)";
    case LRFG_EINVAL: return "invalid argument";
    case LRFG_ECOEFF: return "coefficient not finite and positive";
    case LRFG_EWORKSPACE: return "workspace too small or misaligned";
    case LRFG_EDEVICE: return "HIP device error or no device";
    case LRFG_EUNSUPPORTED: return "unsupported request";
    default: return "unknown status";
  }
}

const char* lrfg_last_error(void) { return g_last_error.c_str(); }

int lrfg_device_check(void) {
  clear_error();
  return device_ok();
}

int lrfg_plan_create(const lrfg_problem* p, lrfg_plan** out) {
  clear_error();
  if (out == nullptr) {
    set_error("out is NULL");
    return LRFG_EINVAL;
  }
  *out = nullptr;
  LRFG_TRY(validate(p));
  lrfg_plan* pl = new lrfg_plan();
  pl->p = *p;
  // full-grid geometry: Ga's double grid (at least 2N - 1)
  const bool ga = p->discretisation == LRFG_DISC_GA;
  auto gridN = [&](int i) { return ga ? ga_double_grid(p->N[i]) : p->N[i]; };
  if (p->d == 3) {
    pl->N3d[0] = gridN(0);
    pl->N3d[1] = gridN(1);
    pl->N3d[2] = gridN(2);
  } else {
    pl->N3d[0] = 1;
    pl->N3d[1] = gridN(0);
    pl->N3d[2] = gridN(1);
  }
  for (int i = 0; i < 3; ++i) {
    int rc = fft_plan_make(pl->N3d[i], &pl->axis[i]);
    if (rc != LRFG_OK) {
      delete pl;
      return rc;
    }
  }
  // low-rank Ga: the carriages live on the double grid
  lrfg_problem pm = *p;
  for (int i = 0; i < p->d; ++i) pm.N[i] = gridN(i);
  for (int i = 0; i < p->d; ++i) {
    int rc = fft_plan_make(pm.N[i], &pl->mode[i]);
    if (rc != LRFG_OK) {
      delete pl;
      return rc;
    }
  }
  if (p->format != LRFG_FORMAT_FULL) {
    int rc = lowrank_plan_create(pm, pl->mode, &pl->lr, p->discretisation == LRFG_DISC_GA ? p->N : nullptr);
    if (rc != LRFG_OK) {
      delete pl;
      return rc;
    }
  } else {
    // the full-grid loop's pinned host flags, taken here when a device is
    // present so that solving allocates nothing (else at the first solve)
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) == hipSuccess && ndev > 0 &&
        hipHostMalloc((void**)&pl->pinned, sizeof(int) * 4 * 3, hipHostMallocDefault) == hipSuccess) {
      pl->pinned_n = 12;
    } else {
      pl->pinned = nullptr;
      (void)hipGetLastError();
    }
  }
  *out = pl;
  return LRFG_OK;
}

int lrfg_plan_workspace_bytes(const lrfg_plan* plan, int max_nE, size_t* bytes) {
  clear_error();
  if (plan == nullptr || bytes == nullptr || max_nE < 1) {
    set_error("bad arguments");
    return LRFG_EINVAL;
  }
  const lrfg_problem& p = plan->p;
  if (p.format == LRFG_FORMAT_FULL) {
    *bytes = full_workspace_bytes(plan->N3d, max_nE, p.d, p.max_iter) + coeff_staging_bytes(p);
  } else {
    *bytes = lowrank_workspace_bytes(plan->lr, max_nE);
  }
  return LRFG_OK;
}

void lrfg_plan_destroy(lrfg_plan* plan) {
  if (plan == nullptr) return;
  if (plan->pinned) (void)hipHostFree(plan->pinned);
  lowrank_plan_destroy(plan->lr);
  delete plan;
}

static int full_one(lrfg_plan* plan, const lrfg_coeff* a, const double* E, int nE, void* d_ws, size_t need,
                    void* stream, lrfg_result* out);

// count microstructures (coefficients a[0..count-1]) with the same fields E.
static int solve_impl(lrfg_plan* plan, const lrfg_coeff* a, int count, const double* E, int nE, void* d_ws,
                      size_t ws_bytes, void* stream, lrfg_result* outs) {
  clear_error();
  if (plan == nullptr || a == nullptr || outs == nullptr) {
    set_error("plan, coefficient and result must be non-NULL");
    return LRFG_EINVAL;
  }
  const lrfg_problem& p = plan->p;
  if (count < 1 || (p.format != LRFG_FORMAT_FULL && count * nE > kMaxSystems)) {
    set_error("count %d outside [1, %d / nE]", count, kMaxSystems);
    return LRFG_EINVAL;
  }
  if (E == nullptr && nE != p.d) {
    set_error("E = NULL means the canonical basis: nE must equal d");
    return LRFG_EINVAL;
  }
  if (nE < 1 || nE > 3) {
    set_error("nE must be in [1, 3]");
    return LRFG_EINVAL;
  }
  if (d_ws == nullptr || (reinterpret_cast<uintptr_t>(d_ws) & 255) != 0) {
    set_error("workspace must be non-NULL and 256-byte aligned");
    return LRFG_EWORKSPACE;
  }
  size_t need = 0;
  LRFG_TRY(lrfg_plan_workspace_bytes(plan, p.format == LRFG_FORMAT_FULL ? nE : count * nE, &need));
  if (ws_bytes < need) {
    set_error("workspace too small: need %zu bytes, have %zu", need, ws_bytes);
    return LRFG_EWORKSPACE;
  }
  for (int b = 0; b < count; ++b) {
    const int nsrc = (a[b].full != nullptr) + (a[b].weights != nullptr) + (a[b].tt_cores[0] != nullptr) +
                     (a[b].tucker_core != nullptr) + (a[b].inclusion != LRFG_INCLUSION_NONE);
    if (nsrc != 1) {
      set_error("coefficient %d: exactly one of full / weights / tt_cores / tucker_core / inclusion must be given",
                b);
      return LRFG_EINVAL;
    }
    if ((a[b].inclusion != LRFG_INCLUSION_NONE) != (p.discretisation == LRFG_DISC_GA)) {
      set_error("coefficient %d: the Ga discretisation takes an inclusion coefficient, and only it does", b);
      return LRFG_EINVAL;
    }
    if (a[b].inclusion != LRFG_INCLUSION_NONE) {
      const lrfg_coeff& c = a[b];
      if (c.inclusion != LRFG_INCLUSION_SQUARE && c.inclusion != LRFG_INCLUSION_BALL) {
        set_error("coefficient %d: unknown inclusion %d", b, c.inclusion);
        return LRFG_EINVAL;
      }
      if (c.inclusion == LRFG_INCLUSION_BALL && p.d != 3) {
        set_error("coefficient %d: the ball inclusion is 3D", b);
        return LRFG_EUNSUPPORTED;
      }
      if (c.inclusion == LRFG_INCLUSION_BALL && p.format != LRFG_FORMAT_FULL) {
        set_error("coefficient %d: the low-rank Ga takes the square/cube (CP rank 2 on the double grid)", b);
        return LRFG_EUNSUPPORTED;
      }
      if (!(std::isfinite(c.incl_size) && c.incl_size > 0.0 && c.incl_size < 0.5)) {
        set_error("coefficient %d: inclusion size must be in (0, 1/2)", b);
        return LRFG_EINVAL;
      }
      if (!(std::isfinite(c.incl_inside) && c.incl_inside > 0.0 && std::isfinite(c.incl_outside) &&
            c.incl_outside > 0.0)) {
        set_error("coefficient %d: inclusion values must be finite and positive", b);
        return LRFG_ECOEFF;
      }
    }
    const bool tucker_in = a[b].tucker_core != nullptr;
    if (tucker_in != (p.format == LRFG_FORMAT_TUCKER && a[b].weights == nullptr)) {
      set_error("coefficient %d: the Tucker format takes CP or Tucker coefficients, and Tucker coefficients only "
                "go with the Tucker format", b);
      return LRFG_EUNSUPPORTED;
    }
    if (tucker_in) {
      for (int j = 0; j < 3; ++j) {
        if (a[b].tucker_frames[j] == nullptr || a[b].tucker_ranks[j] < 1 || a[b].tucker_ranks[j] > p.N[j]) {
          set_error("coefficient %d: Tucker frame %d missing or rank %d outside [1, N]", b, j,
                    a[b].tucker_ranks[j]);
          return LRFG_EINVAL;
        }
      }
    }
  }
  LRFG_TRY(device_ok());
  std::vector<double> Ebuf;
  if (E == nullptr) {
    Ebuf.assign(p.d * p.d, 0.0);
    for (int i = 0; i < p.d; ++i) Ebuf[i * p.d + i] = 1.0;
    E = Ebuf.data();
  }
  for (int i = 0; i < nE * p.d; ++i) {
    if (!std::isfinite(E[i])) {
      set_error("E must be finite");
      return LRFG_EINVAL;
    }
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (p.format != LRFG_FORMAT_FULL) return lowrank_solve(plan->lr, a, count, E, nE, d_ws, ws_bytes, s, outs);
  // full grid: the microstructures run one after another in the same workspace
  int worst = LRFG_OK;
  for (int b = 0; b < count; ++b) {
    const int rc = full_one(plan, &a[b], E, nE, d_ws, need, stream, &outs[b]);
    if (rc < 0) return rc;
    worst = worse_status(worst, rc);
  }
  return worst;
}

int lrfg_solve(lrfg_plan* plan, const lrfg_coeff* a, const double* E, int nE, void* d_ws, size_t ws_bytes,
               void* stream, lrfg_result* out) {
  return solve_impl(plan, a, 1, E, nE, d_ws, ws_bytes, stream, out);
}

int lrfg_solve_batch(lrfg_plan* plan, const lrfg_coeff* a, int count, const double* E, int nE, void* d_ws,
                     size_t ws_bytes, void* stream, lrfg_result* results) {
  return solve_impl(plan, a, count, E, nE, d_ws, ws_bytes, stream, results);
}

// One full-grid solve (validated arguments).
static int full_one(lrfg_plan* plan, const lrfg_coeff* a, const double* E, int nE, void* d_ws, size_t need,
                    void* stream, lrfg_result* out) {
  const lrfg_problem& p = plan->p;
  hipStream_t s = static_cast<hipStream_t>(stream);
  {
    if (plan->pinned == nullptr) {
      LRFG_HIP(hipHostMalloc((void**)&plan->pinned, sizeof(int) * 4 * 3, hipHostMallocDefault));
      plan->pinned_n = 12;
    }
    // Coefficient on the device as a full field (CP / TT forms expanded).
    const double* afull = nullptr;
    int on_dev = a->on_device;
    char* wsc = static_cast<char*>(d_ws);
    const size_t stage = coeff_staging_bytes(p);
    const size_t full_need = need - stage;
    if (a->full != nullptr) {
      afull = a->full;
    } else if (a->inclusion != LRFG_INCLUSION_NONE) {
      afull = nullptr;  // built on the double grid by the solve
    } else {
      double* dst = reinterpret_cast<double*>(wsc + full_need);
      LRFG_TRY(expand_coeff(p, *a, dst, stage, s));
      afull = dst;
      on_dev = 1;
    }
    FullSolveArgs fa;
    fa.d = p.d;
    for (int i = 0; i < 3; ++i) fa.N[i] = p.N[i];
    fa.plan1 = &plan->axis[0];
    fa.plan2 = &plan->axis[1];
    fa.plan3 = &plan->axis[2];
    fa.a = afull;
    fa.a_on_device = on_dev;
    fa.E = E;
    fa.nE = nE;
    fa.tol = p.solver_tol;
    fa.max_iter = p.max_iter;
    fa.ws = d_ws;
    fa.ws_bytes = full_need;
    fa.stream = stream;
    fa.pinned_flags = plan->pinned;
    for (int i = 0; i < p.d * p.d; ++i) fa.B[i] = p.aniso[i];
    if (p.discretisation == LRFG_DISC_GA) {
      // the double grid M >= 2N - 1; trial and test functions on the N-frequencies
      for (int i = 0; i < p.d; ++i) {
        fa.ga_N[i] = p.N[i];
        fa.N[i] = ga_double_grid(p.N[i]);
      }
      fa.incl = a->inclusion;
      fa.incl_size = a->incl_size;
      fa.incl_in = a->incl_inside;
      fa.incl_out = a->incl_outside;
    }
    FullSolveOut fo;
    fo.A_H = out->A_H;
    fo.iters = out->iters;
    fo.res_hist = out->res_hist;
    fo.status = out->status;
    const int rc = full_solve(fa, &fo);
    out->setup_ms = fo.setup_ms;
    out->solve_ms = fo.solve_ms;
    return rc;
  }
}

// ---------------------------------------------------------------- allocation-free solve
}  // extern "C"

namespace {
// The workspace of lrfg_solve_noalloc: one array per GPU, held until the
// process ends and shared by every call on that GPU.  Host code uses the
// device address taken once per device (the array's name is only a host
// stand-in for it).
__device__ __align__(256) char scratch[LRFG_NOALLOC_BYTES];
std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;

int scratch_of_current_device(void** out) {
  int dev = 0;
  LRFG_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    LRFG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (p == nullptr || (reinterpret_cast<uintptr_t>(p) & 255) != 0) {
      set_error("device scratch address unusable");
      return LRFG_EDEVICE;
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return LRFG_OK;
}
}  // namespace

extern "C" {

int lrfg_solve_noalloc(lrfg_plan* plan, const lrfg_coeff* a, const double* E, int nE, void* stream,
                       lrfg_result* out) {
  clear_error();
  if (plan == nullptr || nE < 1) {
    set_error("plan must be non-NULL and nE >= 1");
    return LRFG_EINVAL;
  }
  size_t need = 0;
  LRFG_TRY(lrfg_plan_workspace_bytes(plan, nE, &need));
  if (need > LRFG_NOALLOC_BYTES) {
    set_error("the plan needs %zu bytes of workspace; the allocation-free solve holds %zu", need,
              (size_t)LRFG_NOALLOC_BYTES);
    return LRFG_EWORKSPACE;
  }
  if (plan->p.format == LRFG_FORMAT_FULL && plan->pinned == nullptr) {
    set_error("the plan was created without a device (no pinned flag ring); create it with a device present");
    return LRFG_EUNSUPPORTED;
  }
  LRFG_TRY(device_ok());
  void* ws = nullptr;
  LRFG_TRY(scratch_of_current_device(&ws));
  return solve_impl(plan, a, 1, E, nE, ws, LRFG_NOALLOC_BYTES, stream, out);
}

size_t lrfg_fft_workspace_bytes(int N) { return sizeof(double2) * (size_t)(N > 0 ? N : 1) + 256; }

int lrfg_fft_lines(double* x, int outer, int N, int inner, int direction, void* d_ws, size_t ws_bytes,
                   void* stream) {
  clear_error();
  if (x == nullptr || outer < 0 || inner < 1 || (direction != -1 && direction != 1)) {
    set_error("bad arguments");
    return LRFG_EINVAL;
  }
  if (N < 1 || N % 2 == 0) {
    set_error("odd N only");
    return LRFG_EINVAL;
  }
  if (d_ws == nullptr || ws_bytes < lrfg_fft_workspace_bytes(N)) {
    set_error("workspace too small");
    return LRFG_EWORKSPACE;
  }
  const FftPlan* pl = fft_plan_cached(N);
  if (pl == nullptr) return LRFG_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  FftDev f;
  LRFG_TRY(fft_dev_upload(*pl, static_cast<double2*>(d_ws), s, &f));
  return launch_fft_lines(reinterpret_cast<double2*>(x), outer, N, inner, direction, f,
                          direction < 0 ? 1.0 / N : 1.0, s);
}

int lrfg_mode_op(double* x, int outer, int N, int inner, int op, double t, void* d_ws, size_t ws_bytes,
                 void* stream) {
  clear_error();
  if (x == nullptr || outer < 0 || inner < 1 || (op < 0 || op > 2) || !std::isfinite(t)) {
    set_error("bad arguments");
    return LRFG_EINVAL;
  }
  if (N < 1 || N % 2 == 0) {
    set_error("odd N only");
    return LRFG_EINVAL;
  }
  if (d_ws == nullptr || ws_bytes < lrfg_fft_workspace_bytes(N)) {
    set_error("workspace too small");
    return LRFG_EWORKSPACE;
  }
  const FftPlan* pl = fft_plan_cached(N);
  if (pl == nullptr) return LRFG_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  FftDev f;
  LRFG_TRY(fft_dev_upload(*pl, static_cast<double2*>(d_ws), s, &f));
  return launch_mode_op(x, outer, N, inner, op, t, f, s);
}

size_t lrfg_full_op_workspace_bytes(const int N[3]) { return full_op_workspace_bytes(N); }

int lrfg_full_op(int which, const int N[3], const double* a, const double* u, double* outp, void* d_ws,
                 size_t ws_bytes, void* stream) {
  clear_error();
  if (N == nullptr || u == nullptr || outp == nullptr || (which != 0 && which != 1) ||
      (which == 0 && a == nullptr)) {
    set_error("bad arguments");
    return LRFG_EINVAL;
  }
  for (int i = 0; i < 3; ++i) {
    if (N[i] < 1 || N[i] % 2 == 0) {
      set_error("odd N only");
      return LRFG_EINVAL;
    }
  }
  if (d_ws == nullptr || ws_bytes < full_op_workspace_bytes(N)) {
    set_error("workspace too small");
    return LRFG_EWORKSPACE;
  }
  const FftPlan* p1 = fft_plan_cached(N[0]);
  const FftPlan* p2 = fft_plan_cached(N[1]);
  const FftPlan* p3 = fft_plan_cached(N[2]);
  if (!p1 || !p2 || !p3) return LRFG_EINVAL;
  return full_op(which, N, p1, p2, p3, a, u, outp, d_ws, ws_bytes, static_cast<hipStream_t>(stream));
}

}  // extern "C"
