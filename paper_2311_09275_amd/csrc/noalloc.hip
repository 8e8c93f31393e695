// noalloc.hip -- ising_anneal_noalloc: the FIELD anneal of ising_anneal_tuned
// for callers that cannot allocate device memory.  Every device buffer the
// run needs beyond the problem's graph and the caller's result buffers
// (threshold rows, launch structures, the best-state snapshots) lives in
// one fixed array of the library's code object, `scratch`.
#include <string.h>

#include <mutex>

#include "runtime.h"

namespace ising {
namespace {

// One copy per device, created when the code object is loaded there and
// held until the process ends.
static __device__ __align__(256) unsigned char scratch[ISING_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_addr[kMaxDevices] = {nullptr};

// Device address of `scratch` on device dev, which must be current.  In
// host code the array's name is a host-side stand-in, not a device
// address; kernels and copies only ever get the address looked up here.
int scratch_address(int dev, char** out) {
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device %d outside the %d devices the scratch table covers", dev, kMaxDevices);
    return ISING_ERR_DEVICE;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* a = nullptr;
    const hipError_t e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
    if (e != hipSuccess || a == nullptr) {
      (void)hipGetLastError();
      set_error("hipGetSymbolAddress(scratch) on device %d failed: %s", dev,
                hipGetErrorString(e != hipSuccess ? e : hipErrorInvalidSymbol));
      return ISING_ERR_DEVICE;
    }
    g_scratch_addr[dev] = static_cast<char*>(a);
  }
  *out = g_scratch_addr[dev];
  return ISING_OK;
}

// 256-byte aligned pieces of the scratch array, in order.
struct Carve {
  char* base;
  size_t used = 0;
  template <class T>
  T* take(size_t count) {
    T* p = reinterpret_cast<T*>(base + used);
    used += DeviceArena::span(sizeof(T) * count);
    return p;
  }
};

}  // namespace
}  // namespace ising

using namespace ising;

extern "C" int ising_anneal_noalloc(ising_problem* p, const ising_schedule* s, int32_t n_replicas,
                                    uint64_t seed, const ising_tuning* tuning,
                                    const ising_device_results* out, void* stream) {
  if (!p || !s || !out || s->n_sweeps < 1 || n_replicas < 1) return ISING_ERR_INVALID;
  if (!out->best_cut || !out->best_sweep || !out->final_energy || !out->accepts || !out->argmax ||
      !out->best_states) {
    set_error("every result buffer of ising_device_results must be given");
    return ISING_ERR_INVALID;
  }
  TraceRange tr("ising_anneal_noalloc");
  if (p->dg.device < 0) {
    set_error("the problem's graph is not on a device yet: it is uploaded by its first "
              "ising_anneal, ising_anneal_batch or ising_temper");
    return ISING_ERR_STATE;
  }
  int dev = -1;
  ICHK(hipGetDevice(&dev));
  if (dev != p->dg.device) {
    set_error("the current device %d is not the problem's device %d", dev, p->dg.device);
    return ISING_ERR_STATE;
  }
  if (p->init_R > 0 || p->trace) {
    set_error("initial states and energy traces need device copies; this entry point takes none");
    return ISING_ERR_UNSUPPORTED;
  }
  IRET(schedule_table(p, s));
  const Table& table = p->sched.table;
  PersistentConfig cfg;
  IRET(resolve_config(p, table, n_replicas, tuning, cfg));
  if (cfg.path != ISING_PATH_FIELD) {
    set_error("this entry point runs the FIELD path only (the configuration resolved to path %d)",
              cfg.path);
    return ISING_ERR_UNSUPPORTED;
  }
  char* base = nullptr;
  IRET(scratch_address(dev, &base));

  // layout of the scratch array for this run
  const HostGraph& g = p->g;
  auto& na = p->noalloc;
  build_padded_rows(table, na.rows_p);
  build_bond_rows(table, na.rows_b);
  const size_t R = (size_t)n_replicas, np = (size_t)g.n_pad;
  const size_t units_max = R;  // one replica block per unit at most
  const size_t need = DeviceArena::span(R * np) + DeviceArena::span(4 * na.rows_p.size()) +
                      DeviceArena::span(4 * na.rows_b.size()) + DeviceArena::span(sizeof(JobDev)) +
                      DeviceArena::span(sizeof(int2) * units_max) + 2 * DeviceArena::span(64);
  if (need > (size_t)ISING_NOALLOC_SCRATCH_BYTES) {
    set_error("this run needs %zu bytes of scratch (replicas x padded vertices, plus rows); the "
              "fixed maximum is %zu",
              need, (size_t)ISING_NOALLOC_SCRATCH_BYTES);
    return ISING_ERR_UNSUPPORTED;
  }
  Carve c{base};
  RunBuffers& b = na.run;
  b.table = table;  // copy-assign: reuses the capacity of earlier calls
  b.R = n_replicas;
  b.S = table.S;
  b.path = cfg.path;
  b.G = cfg.G;
  b.block = cfg.block;
  b.trace = false;
  b.best = c.take<int8_t>(R * np);
  b.save = nullptr;  // the kernel keeps no final state
  b.tqp = c.take<uint32_t>(na.rows_p.size());
  b.tqb = c.take<uint32_t>(na.rows_b.size());
  JobDev* job_d = c.take<JobDev>(1);
  int2* units_d = c.take<int2>(units_max);
  int32_t* list_off_d = c.take<int32_t>(16);
  int32_t* ctr_d = c.take<int32_t>(16);
  b.best_cut = out->best_cut;
  b.best_sweep = out->best_sweep;
  b.energy = out->final_energy;
  b.accepts = reinterpret_cast<unsigned long long*>(out->accepts);
  b.argmax = reinterpret_cast<unsigned long long*>(out->argmax);
  b.trace_buf = nullptr;
  b.init_dev = nullptr;

  std::vector<JobSpec> js{JobSpec{&g, &p->dg, &b, n_replicas, seed, 0, table.S}};
  PersistentPlan& plan = na.plan;
  IRET(plan_persistent(js, cfg, plan));
  if (plan.units.size() > units_max || plan.jobs.size() != 1) {
    set_error("launch plan larger than its scratch slot");
    return ISING_ERR_UNSUPPORTED;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  ICHK(hipMemcpyAsync(b.tqp, na.rows_p.data(), 4 * na.rows_p.size(), hipMemcpyHostToDevice, st));
  ICHK(hipMemcpyAsync(b.tqb, na.rows_b.data(), 4 * na.rows_b.size(), hipMemcpyHostToDevice, st));
  ICHK(hipMemcpyAsync(job_d, plan.jobs.data(), sizeof(JobDev), hipMemcpyHostToDevice, st));
  ICHK(hipMemcpyAsync(units_d, plan.units.data(), sizeof(int2) * plan.units.size(),
                      hipMemcpyHostToDevice, st));
  ICHK(hipMemcpyAsync(list_off_d, plan.list_off, sizeof(plan.list_off), hipMemcpyHostToDevice, st));
  // the work-list cursors start at zero (the array keeps the last call's)
  ICHK(launch_fill_i32(ctr_d, 0, 8, st));
  LaunchPersistent lp;
  lp.jobs = job_d;
  lp.units = units_d;
  lp.list_off = list_off_d;
  lp.ctr = ctr_d;
  lp.grid = plan.grid;
  lp.lds_bytes = plan.lds;
  lp.planes = plan.planes;
  lp.adj = plan.form;
  ICHK(launch_field(lp, cfg.block, st));
  ICHK(launch_argmax(job_d, 1, st));
  ICHK(launch_gather_states(static_cast<const int8_t*>(b.best), n_replicas, g.n_pad, p->dg.pos, g.n,
                            out->best_states, st));
  return ISING_OK;
}
