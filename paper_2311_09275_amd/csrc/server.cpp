// server.cpp -- continuous-batching request server.
//
// Requests (problem, schedule, replicas, seed, target cut) queue in arrival
// order.  A scheduler thread admits the head of the queue while a slot is
// free and the request's device buffers fit in the server's memory pool,
// then advances every resident request by one chunk of sweeps in a single
// persistent launch.  Spin state, fields and best states stay in device
// memory between chunks (the kernels save and reload each unit's LDS words),
// so a request's trajectory does not depend on how its sweeps are chunked
// or on what else is resident.  A request stops when it has run its whole
// schedule, or -- checked only after a multiple of its own check_every
// sweeps -- when some replica's best cut reaches its target.
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>

#include "runtime.h"

namespace ising {
namespace {

// First-fit allocator over one contiguous range (device memory, or, for the
// null backend, a range of offsets that is never dereferenced).
class Pool {
 public:
  void init(char* base, size_t cap) {
    base_ = base;
    cap_ = cap;
    free_.clear();
    free_[0] = cap;
  }
  char* alloc(size_t bytes) {
    bytes = (bytes + 255) & ~(size_t)255;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        const size_t off = it->first, len = it->second;
        free_.erase(it);
        if (len > bytes) free_[off + bytes] = len - bytes;
        used_[off] = bytes;
        return base_ + off;
      }
    }
    return nullptr;
  }
  void release(char* p) {
    const size_t off = (size_t)(p - base_);
    auto u = used_.find(off);
    if (u == used_.end()) return;
    size_t start = off, len = u->second;
    used_.erase(u);
    auto next = free_.lower_bound(start);
    if (next != free_.end() && next->first == start + len) {
      len += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == start) {
        start = prev->first;
        len += prev->second;
        free_.erase(prev);
      }
    }
    free_[start] = len;
  }
  size_t in_use() const {
    size_t s = 0;
    for (auto& kv : used_) s += kv.second;
    return s;
  }

 private:
  char* base_ = nullptr;
  size_t cap_ = 0;
  std::map<size_t, size_t> free_, used_;
};

struct Request {
  uint64_t ticket = 0;
  ising_problem* p = nullptr;
  Table table;
  int R = 0, S = 0, check_every = 0;
  uint64_t seed = 0;
  int64_t target = 0;
  size_t footprint = 0;
  RunBuffers buf;
  char* mem = nullptr;
  bool prepared = false;
  // Progress as the scheduler thread computes it.  The step functions run
  // without the server lock and write only this; the scheduler copies it
  // into the published fields below under the lock after each step.
  struct Progress {
    int t_done = 0;
    bool done = false;
    bool reached = false;
    int64_t best_cut = 0;
    int best_replica = -1;
    std::vector<int8_t> best_state;
  } work;
  // Published fields: written and read only under the server lock.  A
  // client that sees done == true also sees the final values of the
  // others (they are set in the same critical section).
  int t_done = 0;
  bool done = false;
  int status = ISING_OK;
  bool reached = false;
  int64_t best_cut = 0;
  int best_replica = -1;
  std::vector<int8_t> best_state;
  double t_submit = 0, t_admit = -1, t_finish = -1;
};

using Clock = std::chrono::steady_clock;

}  // namespace
}  // namespace ising

using namespace ising;

struct ising_server {
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<Request>> queue;
  std::vector<std::shared_ptr<Request>> resident;
  std::map<uint64_t, std::shared_ptr<Request>> all;
  uint64_t next_ticket = 1;
  Pool pool;
  DeviceBlock pool_block;
  char* pool_mem = nullptr;
  uint64_t budget = 0;
  int max_slots = 1, chunk = 50, backend = 0, device = -1;
  hipStream_t stream = nullptr;
  PersistentConfig cfg;
  Launcher launcher;
  std::thread th;
  bool stop = false;
  int64_t steps = 0, finished = 0;
  int peak = 0;
  Clock::time_point t0;

  double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
};

namespace {

int next_end(const Request& r, int chunk) {
  const int t_done = r.work.t_done;
  int end = std::min(r.S, t_done + chunk);
  if (r.check_every > 0) end = std::min(end, (t_done / r.check_every + 1) * r.check_every);
  return end;
}

// After a chunk: decide whether the request is finished (scheduler-private
// progress only).
void settle(Request& r, int end) {
  Request::Progress& w = r.work;
  w.t_done = end;
  const bool at_check = r.check_every > 0 && w.t_done % r.check_every == 0;
  if (at_check && w.best_cut >= r.target) {
    w.reached = true;
    w.done = true;
  }
  if (w.t_done >= r.S) {
    w.reached = w.reached || w.best_cut >= r.target;
    w.done = true;
  }
}

// Under the server lock: make the step's progress visible to clients.
void publish(Request& r) {
  const Request::Progress& w = r.work;
  r.t_done = w.t_done;
  r.reached = w.reached;
  r.best_cut = w.best_cut;
  r.best_replica = w.best_replica;
}

// One chunk of sweeps for every resident request on the device.
int step_device(ising_server* s, std::vector<std::shared_ptr<Request>>& batch) {
  std::vector<JobSpec> specs;
  std::vector<int> ends;
  for (auto& r : batch) {
    if (!r->prepared) {
      IRET(upload_graph_once(r->p->g, r->p->dg));
      IRET(prepare_buffers(r->buf, r->p->g, r->table, r->R, s->cfg, s->stream, false, nullptr,
                           r->mem));
      r->prepared = true;
    }
    const int end = next_end(*r, s->chunk);
    ends.push_back(end);
    specs.push_back(JobSpec{&r->p->g, &r->p->dg, &r->buf, r->R, r->seed, r->work.t_done, end});
  }
  TraceRange tr("ising_server_step");
  IRET(run_persistent(s->launcher, specs, s->cfg, s->stream, true));
  ICHK(hipStreamSynchronize(s->stream));
  for (size_t i = 0; i < batch.size(); ++i) {
    Request& r = *batch[i];
    unsigned long long key = 0;
    ICHK(hipMemcpy(&key, r.buf.argmax, sizeof key, hipMemcpyDeviceToHost));
    r.work.best_cut = (int64_t)(int32_t)((uint32_t)(key >> 32) ^ 0x80000000u);
    r.work.best_replica = (int32_t)(0xFFFFFFFFu - (uint32_t)key);
    settle(r, ends[i]);
    if (r.work.done) {
      const HostGraph& g = r.p->g;
      ICHK(launch_gather(r.buf.best, r.buf.layout_best, r.R, g.n_pad, r.work.best_replica,
                         r.p->dg.pos, g.n, r.buf.gather, s->stream));
      std::vector<int32_t> tmp((size_t)g.n);
      ICHK(hipMemcpyAsync(tmp.data(), r.buf.gather, sizeof(int32_t) * g.n, hipMemcpyDeviceToHost,
                          s->stream));
      ICHK(hipStreamSynchronize(s->stream));
      r.work.best_state.assign(tmp.begin(), tmp.end());
    }
  }
  return ISING_OK;
}

// The null backend advances sweep counters only; its "best cut" is the
// number of sweeps done, which makes target checks observable.  Backend 2
// also fails (as a device error would) every step in which a request with
// the seed ISING_NULL_FAIL_SEED is resident.
int step_null(ising_server* s, std::vector<std::shared_ptr<Request>>& batch) {
  if (s->backend == 2)
    for (auto& r : batch)
      if (r->seed == ISING_NULL_FAIL_SEED) {
        set_error("null backend: injected step failure");
        return ISING_ERR_DEVICE;
      }
  for (auto& r : batch) {
    const int end = next_end(*r, s->chunk);
    r->work.best_cut = end;
    r->work.best_replica = 0;
    settle(*r, end);
    if (r->work.done) r->work.best_state.assign((size_t)r->p->g.n, 1);
  }
  return ISING_OK;
}

void scheduler(ising_server* s) {
  if (s->backend == 0) (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    if (s->stop) break;
    while (!s->queue.empty() && (int)s->resident.size() < s->max_slots) {
      auto r = s->queue.front();
      char* mem = s->pool.alloc(r->footprint);
      if (!mem) break;  // the head waits for memory; arrival order is kept
      s->queue.pop_front();
      r->mem = mem;
      r->t_admit = s->now();
      s->resident.push_back(r);
    }
    if (s->resident.empty()) {
      s->cv_work.wait(lk);
      continue;
    }
    std::vector<std::shared_ptr<Request>> batch = s->resident;
    s->peak = std::max(s->peak, (int)batch.size());
    lk.unlock();
    const int rc = s->backend == 0 ? step_device(s, batch) : step_null(s, batch);
    lk.lock();
    ++s->steps;
    std::vector<std::shared_ptr<Request>> keep;
    for (auto& r : s->resident) {
      publish(*r);
      if (rc != ISING_OK) {
        r->status = rc;
        r->work.done = true;
      }
      if (r->work.done) {
        r->best_state.swap(r->work.best_state);
        r->t_finish = s->now();
        r->done = true;
        r->buf.arena.release();
        s->pool.release(r->mem);
        r->mem = nullptr;
        ++s->finished;
      } else {
        keep.push_back(r);
      }
    }
    s->resident.swap(keep);
    s->cv_done.notify_all();
  }
  // shutting down: whatever has not finished is cancelled
  for (auto& r : s->resident) {
    r->status = ISING_ERR_STATE;
    r->done = true;
    r->buf.arena.release();
    s->pool.release(r->mem);
  }
  for (auto& r : s->queue) {
    r->status = ISING_ERR_STATE;
    r->done = true;
  }
  s->resident.clear();
  s->queue.clear();
  s->cv_done.notify_all();
}

PersistentConfig server_config() {
  PersistentConfig c;
  c.path = ISING_PATH_FIELD;
  c.G = 1;
  c.block = 512;
  c.adj = 0;
  return c;
}

}  // namespace

extern "C" {

int ising_server_footprint(const ising_problem* p, const ising_schedule* sched, int32_t n_replicas,
                           uint64_t* bytes) {
  if (!p || !sched || n_replicas < 1 || !bytes) return ISING_ERR_INVALID;
  std::vector<double> beta;
  IRET(eval_schedule(sched, beta));
  Table t;
  IRET(build_table(beta, p->g.kmax, t));
  *bytes = run_bytes(p->g, t, n_replicas, server_config(), false, false);
  return ISING_OK;
}

int ising_server_create(uint64_t hbm_budget, int32_t max_slots, int32_t chunk_sweeps,
                        int32_t backend, void* stream, ising_server** out) {
  if (!out || hbm_budget < 4096 || max_slots < 1 || chunk_sweeps < 1 || backend < 0 || backend > 2)
    return ISING_ERR_INVALID;
  ising_server* s = nullptr;
  try {
    s = new ising_server();
  } catch (...) {
    return ISING_ERR_NOMEM;
  }
  s->budget = hbm_budget;
  s->max_slots = max_slots;
  s->chunk = chunk_sweeps;
  s->backend = backend;
  s->stream = static_cast<hipStream_t>(stream);
  s->cfg = server_config();
  s->t0 = Clock::now();
  if (backend == 0) {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0 || hipGetDevice(&s->device) != hipSuccess) {
      (void)hipGetLastError();
      delete s;
      set_error("no HIP device available");
      return ISING_ERR_DEVICE;
    }
    if (device_alloc(hbm_budget, s->pool_block) != ISING_OK) {
      delete s;
      return ISING_ERR_NOMEM;
    }
    s->pool_mem = static_cast<char*>(s->pool_block.ptr);
    s->pool.init(s->pool_mem, hbm_budget);
  } else {
    // offsets only: a base far from any real mapping, never dereferenced
    s->pool.init(reinterpret_cast<char*>((uintptr_t)1 << 40), hbm_budget);
  }
  try {
    s->th = std::thread(scheduler, s);
  } catch (...) {
    device_free(s->pool_block);
    delete s;
    return ISING_ERR_NOMEM;
  }
  *out = s;
  return ISING_OK;
}

int ising_server_submit(ising_server* s, ising_problem* p, const ising_schedule* sched,
                        int32_t n_replicas, uint64_t seed, int64_t target_cut, int32_t check_every,
                        uint64_t* ticket) {
  if (!s || !p || !sched || n_replicas < 1 || !ticket) return ISING_ERR_INVALID;
  auto r = std::make_shared<Request>();
  std::vector<double> beta;
  IRET(eval_schedule(sched, beta));
  IRET(build_table(beta, p->g.kmax, r->table));
  if (s->backend == 0) IRET(check_config(p->g, r->table, n_replicas, s->cfg));
  r->p = p;
  r->R = n_replicas;
  r->S = r->table.S;
  r->seed = seed;
  r->target = target_cut;
  r->check_every = check_every > 0 ? check_every : 0;
  r->footprint = run_bytes(p->g, r->table, n_replicas, s->cfg, false, false);
  if (r->footprint > s->budget) {
    set_error("request needs %zu bytes, the server budget is %llu", r->footprint,
              (unsigned long long)s->budget);
    return ISING_ERR_NOMEM;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) return ISING_ERR_STATE;
  r->ticket = s->next_ticket++;
  r->t_submit = s->now();
  s->all[r->ticket] = r;
  s->queue.push_back(r);
  s->cv_work.notify_all();
  *ticket = r->ticket;
  return ISING_OK;
}

int ising_server_wait(ising_server* s, uint64_t ticket, double timeout_s, ising_result* out) {
  if (!s || !out) return ISING_ERR_INVALID;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->all.find(ticket);
  if (it == s->all.end()) return ISING_ERR_INVALID;
  std::shared_ptr<Request> r = it->second;
  auto pred = [&] { return r->done; };
  if (timeout_s < 0) {
    s->cv_done.wait(lk, pred);
  } else if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), pred)) {
    return ISING_ERR_TIMEOUT;
  }
  ising_result res;
  memset(&res, 0, sizeof res);
  res.status = r->status;
  res.reached_target = r->reached ? 1 : 0;
  res.sweeps_done = r->t_done;
  res.best_replica = r->best_replica;
  res.best_cut = r->best_cut;
  res.t_submit = r->t_submit;
  res.t_admit = r->t_admit;
  res.t_done = r->t_finish;
  *out = res;
  return ISING_OK;
}

int ising_server_best_state(ising_server* s, uint64_t ticket, int8_t* spins) {
  if (!s || !spins) return ISING_ERR_INVALID;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->all.find(ticket);
  if (it == s->all.end()) return ISING_ERR_INVALID;
  const Request& r = *it->second;
  if (!r.done || r.status != ISING_OK) return ISING_ERR_STATE;
  memcpy(spins, r.best_state.data(), r.best_state.size());
  return ISING_OK;
}

int ising_server_stats(ising_server* s, int64_t* steps, int64_t* finished, int32_t* peak) {
  if (!s) return ISING_ERR_INVALID;
  std::lock_guard<std::mutex> lk(s->mu);
  if (steps) *steps = s->steps;
  if (finished) *finished = s->finished;
  if (peak) *peak = s->peak;
  return ISING_OK;
}

int ising_server_destroy(ising_server* s) {
  if (!s) return ISING_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv_work.notify_all();
  }
  if (s->th.joinable()) s->th.join();
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  {
    DeviceGuard g(s->device);
    for (auto& kv : s->all) kv.second->buf.arena.release();
    device_free(s->pool_block);
  }
  delete s;
  return ISING_OK;
}

}  // extern "C"
