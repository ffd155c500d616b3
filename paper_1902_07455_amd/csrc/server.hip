// Request loop with continuous batching on one device (host runtime).
//
// Requests are homogenisation queries (a problem, its coefficient in place,
// the fields E).  An admission thread takes queued requests while the
// caller's device pool has room for their workspace (admission by HBM
// footprint, first fit): the oldest request that fits, together with the
// other queued requests of the same problem (and coefficient ranks and
// fields), up to max_batch of them, becomes one session solved as one
// lrfg_solve_batch on a thread and HIP stream of its own.  The sessions
// share `slots` device permits handed out in arrival order: a session holds
// one while it runs a block of iterations and gives it back at every
// iteration gate of the solve, so a request admitted while others run joins
// the rotation at the next block boundary, and a finished one leaves it
// there, instead of waiting for whole solves to end; up to `slots`
// sessions have work on the device at once.  The coefficient data is read
// where the caller keeps it (device pointers stay on the device).
#include <cstring>
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "common.h"
#include "lowrank.h"

namespace lrfg {

IterGate*& iter_gate() {
  thread_local IterGate* g = nullptr;
  return g;
}

namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

struct Request {
  lrfg_problem p;
  lrfg_coeff a;
  std::vector<double> E;  // nE x d, empty = canonical basis
  int nE = 0;
  lrfg_result* out = nullptr;
  uint64_t tag = 0;
  lrfg_plan* plan = nullptr;
  size_t ws_one = 0;
  hipEvent_t ready = nullptr;  // recorded on the submitter's stream: device inputs complete
  Clock::time_point t_submit;
};

// First-fit allocator over [0, size) in 256-byte units.
class Pool {
 public:
  explicit Pool(size_t size) : size_(size) { free_[0] = size; }
  bool alloc(size_t n, size_t* off) {
    n = (n + 255) & ~(size_t)255;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        *off = it->first;
        const size_t rest = it->second - n, at = it->first + n;
        free_.erase(it);
        if (rest) free_[at] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t n) {
    n = (n + 255) & ~(size_t)255;
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t largest() const {
    size_t m = 0;
    for (auto& kv : free_) m = std::max(m, kv.second);
    return m;
  }

 private:
  size_t size_;
  std::map<size_t, size_t> free_;
};

bool same_problem(const lrfg_problem& x, const lrfg_problem& y) {
  return x.d == y.d && x.N[0] == y.N[0] && x.N[1] == y.N[1] && x.N[2] == y.N[2] && x.format == y.format &&
         x.rank_cap == y.rank_cap && x.trunc_tol == y.trunc_tol && x.solver_tol == y.solver_tol &&
         x.max_iter == y.max_iter && x.solver == y.solver && x.precision == y.precision &&
         x.precond_terms == y.precond_terms && x.oversample == y.oversample && x.seed == y.seed &&
         x.coeff_rank == y.coeff_rank && x.flags == y.flags &&
         std::memcmp(x.aniso, y.aniso, sizeof(x.aniso)) == 0 && x.rank_start == y.rank_start &&
         x.discretisation == y.discretisation;
}

bool same_batch_key(const Request& x, const Request& y) {
  if (!same_problem(x.p, y.p)) return false;
  if (x.nE != y.nE || x.E != y.E) return false;
  if (x.p.format == LRFG_FORMAT_FULL) return true;
  const bool xc = x.a.weights != nullptr, yc = y.a.weights != nullptr;
  const bool xk = x.a.tucker_core != nullptr, yk = y.a.tucker_core != nullptr;
  if (xc != yc || xk != yk || x.a.on_device != y.a.on_device) return false;
  if (xc) return x.a.rank == y.a.rank;
  if (xk) {
    for (int j = 0; j < 3; ++j)
      if (x.a.tucker_ranks[j] != y.a.tucker_ranks[j]) return false;
    return true;
  }
  for (int j = 0; j <= x.p.d; ++j)
    if (x.a.tt_ranks[j] != y.a.tt_ranks[j]) return false;
  return true;
}

}  // namespace
}  // namespace lrfg

struct lrfg_server {
  int device = 0;
  int max_batch = 1;
  int slots = 1;
  int max_sessions = 4;
  char* pool_base = nullptr;
  std::unique_ptr<lrfg::Pool> pool;
  size_t pool_bytes = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::unique_ptr<lrfg::Request>> queue;
  std::deque<lrfg_completion> done;
  int running = 0;  // sessions admitted and not yet completed
  uint64_t gates = 0;   // iteration gates passed by the sessions
  bool stopping = false;
  std::thread admitter;
  int worker_error = LRFG_OK;
  // device permits, granted in request order
  std::mutex pmu;
  std::condition_variable pcv;
  int permits = 1;
  std::deque<uint64_t> waiting;
  uint64_t next_ticket = 0;
};

namespace lrfg {
namespace {

// FIFO permits: a thread waits until it is the oldest waiter and a permit
// is free.
void permit_acquire(lrfg_server* S) {
  std::unique_lock<std::mutex> lk(S->pmu);
  const uint64_t me = S->next_ticket++;
  S->waiting.push_back(me);
  S->pcv.wait(lk, [&] { return S->permits > 0 && S->waiting.front() == me; });
  S->waiting.pop_front();
  --S->permits;
  S->pcv.notify_all();
}
void permit_release(lrfg_server* S) {
  std::lock_guard<std::mutex> lk(S->pmu);
  ++S->permits;
  S->pcv.notify_all();
}
// Iteration gate of a session: give the permit back and queue for it again.
void session_gate(void* ctx) {
  auto* S = static_cast<lrfg_server*>(ctx);
  {
    // a block boundary: the admission may let queued requests join here
    std::lock_guard<std::mutex> lk(S->mu);
    ++S->gates;
  }
  S->cv_work.notify_all();
  permit_release(S);
  permit_acquire(S);
}

struct Session {
  std::vector<std::unique_ptr<Request>> batch;
  size_t off = 0, bytes = 0;
};

void session_main(lrfg_server* S, Session* se) {
  std::unique_ptr<Session> own(se);
  auto& batch = se->batch;
  hipStream_t st = nullptr;
  int rc = LRFG_OK;
  Clock::time_point t0 = Clock::now(), t1 = t0;
  if (hipSetDevice(S->device) != hipSuccess || hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
    rc = LRFG_EDEVICE;
  } else {
    IterGate gate;
    gate.pass = session_gate;
    gate.ctx = S;
    iter_gate() = &gate;
    permit_acquire(S);
    t0 = Clock::now();
    std::vector<lrfg_coeff> coeffs(batch.size());
    std::vector<lrfg_result> res(batch.size());
    for (size_t k = 0; k < batch.size(); ++k) {
      coeffs[k] = batch[k]->a;
      res[k] = *batch[k]->out;
    }
    Request& h = *batch[0];
    const double* E = h.E.empty() ? nullptr : h.E.data();
    // the coefficients are read on this session's stream: wait until the
    // work that produced them on the submitters' streams is done
    for (size_t k = 0; k < batch.size(); ++k)
      if (batch[k]->ready != nullptr) (void)hipStreamWaitEvent(st, batch[k]->ready, 0);
    rc = lrfg_solve_batch(h.plan, coeffs.data(), (int)batch.size(), E, h.nE, S->pool_base + se->off, se->bytes, st,
                          res.data());
    t1 = Clock::now();
    permit_release(S);
    iter_gate() = nullptr;
    for (size_t k = 0; k < batch.size(); ++k) *batch[k]->out = res[k];
  }
  if (st != nullptr) (void)hipStreamDestroy(st);
  std::lock_guard<std::mutex> lk(S->mu);
  S->pool->release(se->off, se->bytes);
  const int nE = batch[0]->nE;
  for (size_t k = 0; k < batch.size(); ++k) {
    Request& r = *batch[k];
    lrfg_completion c;
    c.tag = r.tag;
    int st_k = rc;
    if (rc >= 0) {
      st_k = LRFG_OK;
      if (r.out->status != nullptr)
        for (int e = 0; e < nE; ++e)
          st_k = worse_status(st_k, r.out->status[e]);
    }
    c.status = st_k;
    c.batch_size = (int)batch.size();
    c.queue_ms = ms_between(r.t_submit, t0);
    c.run_ms = ms_between(t0, t1);
    c.total_ms = ms_between(r.t_submit, t1);
    c.workspace_bytes = se->bytes;
    S->done.push_back(c);
    lrfg_plan_destroy(r.plan);
    r.plan = nullptr;
    if (r.ready != nullptr) (void)hipEventDestroy(r.ready);
    r.ready = nullptr;
  }
  --S->running;
  // notified under the lock: the server is not released before this
  // thread has let go of it
  S->cv_done.notify_all();
  S->cv_work.notify_all();
}

void admitter_main(lrfg_server* S) {
  std::unique_lock<std::mutex> lk(S->mu);
  uint64_t seen = 0;  // gate count at the last admission
  for (;;) {
    // admission: the oldest request whose batch workspace fits, plus queued
    // requests with the same key.  With a device permit free it happens at
    // once; otherwise at the next iteration gate of a running session (the
    // new session then queues for the permit that gate hands on), so that
    // requests arriving in between are batched together.
    std::unique_ptr<Session> se;
    for (;;) {
      if (S->stopping && S->queue.empty()) break;
      const bool now = S->running < S->slots || S->gates != seen || S->stopping;
      if (now && S->running < S->max_sessions) {
        for (size_t hi = 0; hi < S->queue.size(); ++hi) {
          Request& head = *S->queue[hi];
          if (head.ws_one > S->pool->largest()) continue;
          std::vector<size_t> pick = {hi};
          size_t need = head.ws_one;
          if (head.p.format != LRFG_FORMAT_FULL) {  // Tucker batches run one microstructure at a time
            // a low-rank batch holds at most kMaxSystems correctors
            const int cap = std::max(1, std::min(S->max_batch, kMaxSystems / head.nE));
            for (size_t j = hi + 1; j < S->queue.size() && (int)pick.size() < cap; ++j) {
              if (!same_batch_key(head, *S->queue[j])) continue;
              size_t more = 0;
              if (lrfg_plan_workspace_bytes(head.plan, (int)(pick.size() + 1) * head.nE, &more) != LRFG_OK) break;
              if (more > S->pool->largest()) break;
              pick.push_back(j);
              need = more;
            }
          }
          size_t off = 0;
          if (!S->pool->alloc(need, &off)) continue;
          se.reset(new Session());
          se->off = off;
          se->bytes = need;
          for (size_t k = 0; k < pick.size(); ++k) se->batch.push_back(std::move(S->queue[pick[k]]));
          for (size_t k = pick.size(); k-- > 0;) S->queue.erase(S->queue.begin() + (long)pick[k]);
          break;
        }
      }
      if (se) break;
      S->cv_work.wait(lk);
    }
    if (!se) break;  // stopping and drained
    seen = S->gates;
    ++S->running;
    try {
      std::thread(session_main, S, se.release()).detach();
    } catch (...) {
      --S->running;
      S->worker_error = LRFG_EDEVICE;
      S->cv_done.notify_all();
      break;
    }
  }
}

}  // namespace
}  // namespace lrfg

extern "C" {

int lrfg_server_create(int device, int slots, int max_batch, void* d_pool, size_t pool_bytes, lrfg_server** out) {
  using namespace lrfg;
  clear_error();
  if (out == nullptr || slots < 1 || slots > 16 || max_batch < 1 || d_pool == nullptr ||
      (reinterpret_cast<uintptr_t>(d_pool) & 255) != 0 || pool_bytes < 256) {
    set_error("bad server arguments (slots in [1, 16], max_batch >= 1, 256-aligned pool)");
    return LRFG_EINVAL;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
    set_error("device %d not available", device);
    return LRFG_EDEVICE;
  }
  auto* S = new lrfg_server();
  S->device = device;
  S->max_batch = max_batch;
  S->slots = slots;
  S->permits = slots;
  S->max_sessions = 4 * slots;
  S->pool_base = static_cast<char*>(d_pool);
  S->pool_bytes = pool_bytes;
  S->pool.reset(new Pool(pool_bytes));
  S->admitter = std::thread(admitter_main, S);
  *out = S;
  return LRFG_OK;
}

int lrfg_server_submit(lrfg_server* S, const lrfg_problem* p, const lrfg_coeff* a, const double* E, int nE,
                       lrfg_result* out, uint64_t tag, void* stream) {
  using namespace lrfg;
  clear_error();
  if (S == nullptr || p == nullptr || a == nullptr || out == nullptr) {
    set_error("server, problem, coefficient and result must be non-NULL");
    return LRFG_EINVAL;
  }
  if (nE < 1 || nE > 3 || (E == nullptr && nE != p->d)) {
    set_error("nE must be in [1, 3], and equal d when E is NULL");
    return LRFG_EINVAL;
  }
  std::unique_ptr<Request> r(new Request());
  r->p = *p;
  r->a = *a;
  r->nE = nE;
  if (E != nullptr) r->E.assign(E, E + (size_t)nE * p->d);
  r->out = out;
  r->tag = tag;
  LRFG_TRY(lrfg_plan_create(p, &r->plan));
  if (lrfg_plan_workspace_bytes(r->plan, nE, &r->ws_one) != LRFG_OK || r->ws_one > S->pool_bytes) {
    set_error("request workspace %zu exceeds the server pool %zu", r->ws_one, S->pool_bytes);
    lrfg_plan_destroy(r->plan);
    return LRFG_EWORKSPACE;
  }
  if (a->on_device) {
    // device inputs are read by a worker's stream: order that read after
    // the work already queued on the submitter's stream
    if (hipEventCreateWithFlags(&r->ready, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(r->ready, static_cast<hipStream_t>(stream)) != hipSuccess) {
      if (r->ready != nullptr) (void)hipEventDestroy(r->ready);
      lrfg_plan_destroy(r->plan);
      set_error("could not record the submit event");
      return LRFG_EDEVICE;
    }
  }
  r->t_submit = Clock::now();
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stopping) {
      if (r->ready != nullptr) (void)hipEventDestroy(r->ready);
      lrfg_plan_destroy(r->plan);
      set_error("server is stopping");
      return LRFG_EINVAL;
    }
    S->queue.push_back(std::move(r));
  }
  S->cv_work.notify_one();
  return LRFG_OK;
}

int lrfg_server_poll(lrfg_server* S, lrfg_completion* done, int max, int* n, int timeout_ms) {
  using namespace lrfg;
  clear_error();
  if (S == nullptr || n == nullptr || (max > 0 && done == nullptr)) {
    set_error("bad arguments");
    return LRFG_EINVAL;
  }
  std::unique_lock<std::mutex> lk(S->mu);
  auto ready = [&] { return !S->done.empty() || S->worker_error != LRFG_OK; };
  if (timeout_ms < 0)
    S->cv_done.wait(lk, ready);
  else if (timeout_ms > 0)
    S->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready);
  int k = 0;
  while (k < max && !S->done.empty()) {
    done[k++] = S->done.front();
    S->done.pop_front();
  }
  *n = k;
  if (S->worker_error != LRFG_OK) {
    set_error("a server worker could not start on device %d", S->device);
    return S->worker_error;
  }
  return LRFG_OK;
}

int lrfg_server_pending(lrfg_server* S) {
  if (S == nullptr) return 0;
  std::lock_guard<std::mutex> lk(S->mu);
  return (int)S->queue.size() + S->running;
}

void lrfg_server_destroy(lrfg_server* S) {
  if (S == nullptr) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stopping = true;
  }
  S->cv_work.notify_all();
  S->admitter.join();
  {
    // every admitted session has completed (and let go of the server)
    std::unique_lock<std::mutex> lk(S->mu);
    S->cv_done.wait(lk, [&] { return S->running == 0; });
  }
  for (auto& r : S->queue) {
    if (r->plan) lrfg_plan_destroy(r->plan);
    if (r->ready) (void)hipEventDestroy(r->ready);
  }
  delete S;
}

}  // extern "C"
