// Low-rank solve path (placeholder until the TT kernels land).
#include "common.h"
#include "lowrank.h"

namespace lrfg {

struct LowRankPlan {
  lrfg_problem p;
};

int lowrank_plan_create(const lrfg_problem& p, const FftPlan*, LowRankPlan** out) {
  *out = new LowRankPlan{p};
  return LRFG_OK;
}

void lowrank_plan_destroy(LowRankPlan* lr) { delete lr; }

size_t lowrank_workspace_bytes(const LowRankPlan*, int) { return 256; }

int lowrank_solve(LowRankPlan*, const lrfg_coeff&, const double*, int, void*, size_t, hipStream_t,
                  lrfg_result*) {
  set_error("low-rank formats are not built yet");
  return LRFG_EUNSUPPORTED;
}

}  // namespace lrfg
