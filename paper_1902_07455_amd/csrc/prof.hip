// Per-kernel event timing used by the benchmark's roofline figure.
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "common.h"
#include "prof.h"

namespace lrfg {

namespace {
std::mutex g_mu;
std::string g_target;
std::vector<hipEvent_t> g_pool;          // recorded pairs: start, end, start, end, ...
size_t g_used = 0;
bool g_open = false;
double g_work = 0.0;
}  // namespace

bool prof_active(const char* name) {
  if (name == nullptr) return false;
  std::lock_guard<std::mutex> lk(g_mu);
  return !g_target.empty() && g_target == name;
}

static hipEvent_t next_event() {
  if (g_used == g_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    g_pool.push_back(e);
  }
  return g_pool[g_used++];
}

void prof_begin(const char*, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_mu);
  hipEvent_t e = next_event();
  if (e) {
    (void)hipEventRecord(e, s);
    g_open = true;
  }
}

void prof_end(const char*, hipStream_t s, double work) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_open) return;
  hipEvent_t e = next_event();
  if (e) {
    (void)hipEventRecord(e, s);
    g_work += work;
  }
  g_open = false;
}

bool prof_events(const char* name, hipEvent_t* start, hipEvent_t* stop, double work) {
  if (name == nullptr) return false;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_target.empty() || g_target != name) return false;
  hipEvent_t a = next_event();
  hipEvent_t b = a ? next_event() : nullptr;
  if (!a || !b) return false;
  *start = a;
  *stop = b;
  g_work += work;
  return true;
}

}  // namespace lrfg

extern "C" {

int lrfg_prof_enable(const char* kernel) {
  using namespace lrfg;
  std::lock_guard<std::mutex> lk(g_mu);
  g_target = kernel ? kernel : "";
  // A recorded event keeps its launch (and with it the memory that launch
  // used) referenced until the event is destroyed, so a freed workspace
  // would not return to the device: the pool is destroyed at every switch.
  for (hipEvent_t e : g_pool) (void)hipEventDestroy(e);
  g_pool.clear();
  g_used = 0;
  g_open = false;
  g_work = 0.0;
  return LRFG_OK;
}

int lrfg_prof_work(double* total_work) {
  using namespace lrfg;
  std::lock_guard<std::mutex> lk(g_mu);
  if (total_work) *total_work = g_work;
  return LRFG_OK;
}

int lrfg_prof_read(int* count, double* total_ms) {
  using namespace lrfg;
  std::lock_guard<std::mutex> lk(g_mu);
  double tot = 0.0;
  int n = 0;
  for (size_t i = 0; i + 1 < g_used; i += 2) {
    if (hipEventSynchronize(g_pool[i + 1]) != hipSuccess) return LRFG_EDEVICE;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, g_pool[i], g_pool[i + 1]) != hipSuccess) return LRFG_EDEVICE;
    tot += ms;
    ++n;
  }
  if (count) *count = n;
  if (total_ms) *total_ms = tot;
  return LRFG_OK;
}

}  // extern "C"
