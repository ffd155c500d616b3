// Optional per-kernel timing: while a kernel name is selected, each of its
// launches is bracketed by HIP events on its stream (no effect otherwise).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

namespace lrfg {

bool prof_active(const char* name);
void prof_begin(const char* name, hipStream_t s);
void prof_end(const char* name, hipStream_t s, double work);

// Kernel-accurate timing of one launch: when `name` is selected, returns a
// start/stop event pair for hipExtLaunchKernelGGL (the events carry the
// dispatch's own begin and end timestamps, with no marker packets around
// it) and adds `work` to the summed work.
bool prof_events(const char* name, hipEvent_t* start, hipEvent_t* stop, double work);

// Launch `kernel` like hipLaunchKernelGGL; timed by its own dispatch
// timestamps while `tag` is selected.
#define LRFG_LAUNCH_TIMED(tag, work, kernel, grid, block, shm, stream, ...)                   \
  do {                                                                                        \
    hipEvent_t lrfg_e0_, lrfg_e1_;                                                            \
    if (::lrfg::prof_events(tag, &lrfg_e0_, &lrfg_e1_, (work)))                               \
      hipExtLaunchKernelGGL(kernel, grid, block, shm, stream, lrfg_e0_, lrfg_e1_, 0, __VA_ARGS__); \
    else                                                                                      \
      hipLaunchKernelGGL(kernel, grid, block, shm, stream, __VA_ARGS__);                      \
  } while (0)

// RAII bracket around one launch; `work` (algorithmic flops or bytes of
// the launch) is summed over the timed launches.
struct ProfScope {
  const char* name;
  hipStream_t s;
  double work;
  bool on;
  ProfScope(const char* n, hipStream_t st, double w = 0.0) : name(n), s(st), work(w), on(prof_active(n)) {
    if (on) prof_begin(name, s);
  }
  ~ProfScope() {
    if (on) prof_end(name, s, work);
  }
};

}  // namespace lrfg
