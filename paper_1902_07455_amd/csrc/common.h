// Internal helpers of liblrfg: status handling, workspace carving, complex
// arithmetic on double2, reductions.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/lrfg.h"

namespace lrfg {

// ---------------------------------------------------------------- errors
void set_error(const char* fmt, ...);
void clear_error();

#define LRFG_HIP(call)                                                        \
  do {                                                                        \
    hipError_t e_ = (call);                                                   \
    if (e_ != hipSuccess) {                                                   \
      ::lrfg::set_error("%s:%d %s -> %s", __FILE__, __LINE__, #call,          \
                        hipGetErrorString(e_));                               \
      return LRFG_EDEVICE;                                                    \
    }                                                                         \
  } while (0)

#define LRFG_TRY(expr)                                                        \
  do {                                                                        \
    int s_ = (expr);                                                          \
    if (s_ < 0) return s_;                                                    \
  } while (0)

// Launch check: hipGetLastError after a kernel launch.
#define LRFG_LAUNCHED()                                                       \
  do {                                                                        \
    hipError_t e_ = hipGetLastError();                                        \
    if (e_ != hipSuccess) {                                                   \
      ::lrfg::set_error("%s:%d launch -> %s", __FILE__, __LINE__,             \
                        hipGetErrorString(e_));                               \
      return LRFG_EDEVICE;                                                    \
    }                                                                         \
  } while (0)

// ---------------------------------------------------------------- iteration gate
// A solve running on a thread with a gate installed (the serving loop's
// session threads) calls pass(ctx) between iterations, at host points where
// none of its device work is being waited for: the scheduler may hand the
// device to other solves there (continuous batching between iteration
// blocks).  No gate is installed outside the serving loop.
struct IterGate {
  void (*pass)(void* ctx) = nullptr;
  void* ctx = nullptr;
};
IterGate*& iter_gate();
inline void gate_point() {
  IterGate* g = iter_gate();
  if (g != nullptr && g->pass != nullptr) g->pass(g->ctx);
}

// ---------------------------------------------------------------- workspace
// Bump allocator over the caller's workspace.  In "measure" mode (base ==
// nullptr) it only accumulates the size, so the same code path computes the
// required bytes and carves the buffers.
struct Arena {
  char* base = nullptr;
  size_t cap = 0;
  size_t used = 0;
  bool overflow = false;
  template <class T>
  T* take(size_t count) {
    size_t off = (used + 255) & ~size_t(255);
    size_t bytes = count * sizeof(T);
    used = off + bytes;
    if (base == nullptr) return nullptr;
    if (used > cap) {
      overflow = true;
      return nullptr;
    }
    return reinterpret_cast<T*>(base + off);
  }
};

// ---------------------------------------------------------------- events
// HIP events owned for one scope: destroyed on every return path.
template <int K>
struct ScopedEvents {
  hipEvent_t e[K] = {};
  int create(unsigned flags = hipEventDefault) {
    for (int i = 0; i < K; ++i) {
      if (hipEventCreateWithFlags(&e[i], flags) != hipSuccess) {
        e[i] = nullptr;
        set_error("hipEventCreate failed");
        return LRFG_EDEVICE;
      }
    }
    return LRFG_OK;
  }
  hipEvent_t& operator[](int i) { return e[i]; }
  ~ScopedEvents() {
    for (int i = 0; i < K; ++i)
      if (e[i] != nullptr) (void)hipEventDestroy(e[i]);
  }
};

// ---------------------------------------------------------------- complex
// The worse of two non-negative solve statuses: OK < RANK_LIMITED <
// NOT_CONVERGED (negative codes are errors and are returned before).
inline int worse_status(int a, int b) {
  auto rank = [](int v) { return v == LRFG_OK ? 0 : (v == LRFG_RANK_LIMITED ? 1 : 2); };
  return rank(a) >= rank(b) ? a : b;
}

__host__ __device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline double2 cadd(double2 a, double2 b) {
  return make_double2(a.x + b.x, a.y + b.y);
}
__host__ __device__ inline double2 csub(double2 a, double2 b) {
  return make_double2(a.x - b.x, a.y - b.y);
}
__host__ __device__ inline double2 cscale(double2 a, double s) {
  return make_double2(a.x * s, a.y * s);
}
__host__ __device__ inline double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
// multiply by i*s
__host__ __device__ inline double2 cmul_i(double2 a, double s) {
  return make_double2(-a.y * s, a.x * s);
}

// Centred frequency of storage index n on an odd axis of length N (FFT order).
__host__ __device__ inline int freq_of(int n, int N) { return n <= (N - 1) / 2 ? n : n - N; }

constexpr double kPi = 3.141592653589793238462643383279502884;

// ---------------------------------------------------------------- reductions
// Block-wide sum of one double; blockDim.x a multiple of 64, <= 1024.
// Result valid in thread 0.  `sh` needs blockDim.x/64 doubles.
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

__device__ inline double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nw; ++i) t += sh[i];
  }
  return t;
}

inline int ceil_div(long long a, long long b) { return int((a + b - 1) / b); }

}  // namespace lrfg
