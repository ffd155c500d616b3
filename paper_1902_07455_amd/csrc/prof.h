// Optional per-kernel timing: while a kernel name is selected, each of its
// launches is bracketed by HIP events on its stream (no effect otherwise).
#pragma once

#include <hip/hip_runtime.h>

namespace lrfg {

bool prof_active(const char* name);
void prof_begin(const char* name, hipStream_t s);
void prof_end(const char* name, hipStream_t s);

// RAII bracket around one launch.
struct ProfScope {
  const char* name;
  hipStream_t s;
  bool on;
  ProfScope(const char* n, hipStream_t st) : name(n), s(st), on(prof_active(n)) {
    if (on) prof_begin(name, s);
  }
  ~ProfScope() {
    if (on) prof_end(name, s);
  }
};

}  // namespace lrfg
