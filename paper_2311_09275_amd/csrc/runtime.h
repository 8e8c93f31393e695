// runtime.h -- host runtime of libising (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>
#include <stdint.h>

#include <memory>
#include <string>
#include <vector>

#include "device_types.h"
#include "ising.h"
#include "kernels.h"

namespace ising {

// Thread-local text of the last error (for ising_status_string callers
// that want detail, and for the Python binding's exceptions).
void set_error(const char* fmt, ...);
const char* last_error();

#define ICHK(expr)                                                              \
  do {                                                                          \
    hipError_t e_ = (expr);                                                     \
    if (e_ != hipSuccess) {                                                     \
      ::ising::set_error("%s failed: %s", #expr, hipGetErrorString(e_));        \
      return ISING_ERR_DEVICE;                                                  \
    }                                                                           \
  } while (0)

#define IRET(expr)                  \
  do {                              \
    int rc_ = (expr);               \
    if (rc_ != ISING_OK) return rc_; \
  } while (0)

// A named roctx range for the scope: the library's calls show up in
// rocprofv3 --marker-trace timelines.
struct TraceRange {
  explicit TraceRange(const char* name) { roctxRangePushA(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

// Switches to a device for the scope and restores the caller's device.
struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (dev >= 0 && hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
    else prev = -1;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

// Device memory of the library: hipMalloc, or the caller's allocator
// (ising_set_allocator).  A block remembers how it was obtained, so it is
// returned the same way even if the allocator changes meanwhile.
struct DeviceBlock {
  void* ptr = nullptr;
  size_t bytes = 0;
  int device = -1;
  ising_free_fn free_fn = nullptr;  // null: hipFree
  void* ctx = nullptr;
};
int device_alloc(size_t bytes, DeviceBlock& out);
void device_free(DeviceBlock& b);

// One device allocation carved into 256-byte aligned pieces.
struct DeviceArena {
  char* base = nullptr;
  size_t cap = 0, used = 0;
  int device = -1;
  DeviceBlock block;  // what reserve() obtained (owned memory only)
  bool owned = true;  // false: memory lent by a pool, not freed here
  uint64_t generation = 0;  // bumped whenever the memory behind base changes
  void adopt(char* p, size_t bytes, int dev) {
    release();
    base = p;
    cap = bytes;
    used = 0;
    device = dev;
    owned = false;
    ++generation;
  }
  DeviceArena() = default;
  DeviceArena(const DeviceArena&) = delete;
  DeviceArena& operator=(const DeviceArena&) = delete;
  ~DeviceArena();
  int reserve(size_t bytes);  // reallocates when too small; resets used
  void release();
  template <class T>
  T* take(size_t count) {
    size_t bytes = (count * sizeof(T) + 255) & ~(size_t)255;
    if (bytes == 0) bytes = 256;
    T* p = reinterpret_cast<T*>(base + used);
    used += bytes;
    return p;
  }
  static size_t span(size_t bytes) { return bytes == 0 ? 256 : (bytes + 255) & ~(size_t)255; }
};

// ---------------------------------------------------------------- problem
struct HostGraph {
  int32_t n = 0;
  int64_t m = 0;
  int64_t W = 0;
  int32_t kmax = 0, max_deg = 0;
  bool unit = true;
  // local fields b (ising_set_fields): position order, 0 on padding; kmax
  // is max_v (sum_u |w_vu| + 2 |b_v|)
  bool fields = false;
  std::vector<int32_t> bpos;           // [n_pad]
  std::vector<int64_t> wsum;           // [n] sum_u |w_vu|
  int64_t abs_total = 0;               // sum_v sum_u |w_vu|
  bool deg4 = false;                   // every vertex has degree 4 (tori)
  int32_t C = 0;
  int32_t n_pad = 0;
  std::vector<int32_t> u, v, w;        // original edge list
  std::vector<int32_t> colour;         // [n]
  std::vector<int32_t> pos;            // [n] original id -> position
  std::vector<int32_t> orig;           // [n_pad] position -> id, -1 padding
  std::vector<int32_t> grp;            // [n_pad/4]
  std::vector<int32_t> cls;            // [2C] group ranges
  std::vector<int32_t> row, adj, wgt;  // CSR over positions
  std::vector<uint32_t> adjm;          // (position << 1) | (w > 0)
  std::vector<int32_t> aw;             // [2m][2] {position, w}
  std::vector<int32_t> gbase;          // [n_pad/4] = row[4g]
  std::vector<uint32_t> gdeg;          // [n_pad/4] packed slot degrees
  // degree-4 graphs with at most 2^16 positions: the 48-byte group blocks
  // of the FIELD kernel (kDeg4BlockWords), neighbour entries as 16-bit word
  // indices of the tiled state layout (tile_word)
  std::vector<uint32_t> adj4;
  std::vector<int32_t> lab4;  // [4n] neighbours in label order, with adj4
  // the multispin degree-4 form's blocks (kDeg4MscBlockWords), with adj4
  // when twice the tiled state has at most 2^16 elements
  std::vector<uint32_t> adj4m;
};

int compile_graph(int32_t n, int64_t m, const int32_t* u, const int32_t* v, const int32_t* w,
                  const int32_t* colour, HostGraph& g);

// ---------------------------------------------------------------- schedule
int eval_schedule(const ising_schedule* s, std::vector<double>& beta);
uint64_t threshold_q32(double beta, int64_t k);
struct Table {
  int S = 0, kw = 0;
  int32_t kmax = 0;            // the problem's kmax the rows were built for
  uint64_t id = 0;             // distinct for every table built
  std::vector<uint32_t> tq;    // Tq - 1
  std::vector<int32_t> off, len;
};
constexpr int64_t kMaxTableEntries = int64_t(1) << 26;
int build_table(const std::vector<double>& beta, int32_t kmax, Table& t);

// ---------------------------------------------------------------- device
struct DevGraph {
  DeviceArena arena;
  int device = -1;
  int32_t *row = nullptr, *adj = nullptr, *wgt = nullptr, *grp = nullptr, *cls = nullptr,
          *pos = nullptr, *gbase = nullptr;
  uint32_t *adjm = nullptr, *gdeg = nullptr;
  uint32_t* adj4 = nullptr;
  uint32_t* adj4m = nullptr;
  int2* aw = nullptr;
  int32_t* bf = nullptr;  // [n_pad] local fields, position order
};
int upload_graph(const HostGraph& g, DevGraph& d);

struct PersistentConfig {
  int path = ISING_PATH_FIELD;
  int G = 1;
  int block = 256;
  int adj = 0;  // FIELD adjacency: 0 = decide, 1 = staged in LDS, 2 = read from HBM
};

struct RunBuffers {
  DeviceArena arena;
  int R = 0, S = 0, path = 0, G = 0, block = 0, nw = 0;
  bool trace = false;
  size_t arena_key = 0;
  // state and results
  void* best = nullptr;
  int32_t* save = nullptr;
  int8_t* spins = nullptr;
  int32_t* field = nullptr;
  int32_t *best_cut = nullptr, *best_sweep = nullptr, *energy = nullptr, *eacc = nullptr,
          *snap = nullptr, *trace_buf = nullptr, *gather = nullptr;
  unsigned long long *accepts = nullptr, *argmax = nullptr;
  uint32_t* tq = nullptr;
  int32_t *tq_off = nullptr, *tq_len = nullptr;
  uint32_t* tqp = nullptr;     // FIELD: key rows [S][2 kw + 2]
  uint32_t* tqb = nullptr;     // FIELD: degree-4 rows [S][kBondRowWords]
  std::vector<uint32_t> tqp_host, tqb_host;
  // what the last table upload wrote, so that an unchanged table on an
  // unchanged arena is not uploaded again
  uint64_t up_table = 0, up_generation = 0;
  const void* up_at = nullptr;
  int8_t* init_dev = nullptr;
  JobDev* job_dev = nullptr;
  int layout_best = 0, layout_final = 0, layout_field = -1;
  Table table;                 // host source of the uploaded thresholds
  // what the last run left: its launch configuration, seed and the sweeps
  // done, so that a later range can continue it
  PersistentConfig cfg;
  uint64_t seed = 0;
  int t_done = 0;
  hipStream_t stream = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  bool valid = false;
  ~RunBuffers();
};

// Launch structures of the persistent kernels plus a cached hipGraph.
struct Launcher {
  DeviceArena arena;
  JobDev* jobs_d = nullptr;
  int2* units_d = nullptr;
  int32_t* list_off_d = nullptr;
  int32_t* ctr_d = nullptr;
  size_t jobs_cap = 0, units_cap = 0;
  char* staging = nullptr;  // pinned
  size_t staging_cap = 0;
  hipEvent_t staged = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  std::string graph_key;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  // recorded after every launch: the next launch, on whatever stream, waits
  // for it before it rewrites the shared device launch structures
  hipEvent_t done = nullptr;
  bool done_recorded = false;
  ~Launcher();
};


// One anneal (or a chunk of sweeps of it) ready for the persistent kernels.
struct JobSpec {
  const HostGraph* g;
  const DevGraph* dg;
  const RunBuffers* b;
  int R;
  uint64_t seed;
  int t_begin, t_end;
};

// Parallel tempering of a single job: sweeps [0, S) in segments that end
// at every P-th sweep, each followed by exchange round t_end / P - 1.
struct TemperPlan {
  int S, P;
  const SwapDev* swap;
  const ClusterDev* cluster;  // cluster moves before each round, or null
};

// What one persistent launch needs on the device: the jobs, the units in
// eight per-XCD lists (longest first), and the launch shape.
struct PersistentPlan {
  std::vector<JobDev> jobs;
  std::vector<int2> units;
  int32_t list_off[9] = {0};
  size_t lds = 0;   // dynamic LDS per workgroup
  int form = 0;     // adjacency form (LaunchPersistent::adj)
  int planes = 1;   // MSC bit planes
  int grid = 0;     // workgroups (0 when there are no units)
};
int plan_persistent(const std::vector<JobSpec>& specs, const PersistentConfig& cfg,
                    PersistentPlan& plan);
// FIELD threshold rows of a table: key rows (JobDev::tqp, padded_rows(t)
// words) and degree-4 rows (JobDev::tqb, kBondRowWords per sweep).
size_t padded_rows(const Table& t);
void build_padded_rows(const Table& t, std::vector<uint32_t>& out);
void build_bond_rows(const Table& t, std::vector<uint32_t>& out);
int run_persistent(Launcher& L, const std::vector<JobSpec>& jobs, const PersistentConfig& cfg,
                   hipStream_t stream, bool use_graph, const TemperPlan* pt = nullptr);
// Largest replicas_per_block whose rows a FIELD tempering launch can stage
// (one row per replica of a block).
int temper_max_group(const Table& t);
int prepare_run(ising_problem* p, const Table& table, int R, const PersistentConfig& cfg,
                hipStream_t stream);
// Device bytes of one run's buffers.
size_t run_bytes(const HostGraph& g, const Table& table, int R, const PersistentConfig& cfg,
                 bool trace, bool init_given);
// Lay out a run's buffers (in its own allocation, or in pool memory of at
// least run_bytes) and upload thresholds and initial states.
int prepare_buffers(RunBuffers& b, const HostGraph& g, const Table& table, int R,
                    const PersistentConfig& cfg, hipStream_t stream, bool trace,
                    const int8_t* init, char* pool);
int upload_graph_once(const HostGraph& g, DevGraph& d);
int device_cu_count();
size_t lds_budget(int path);
int check_config(const HostGraph& g, const Table& table, int R, const PersistentConfig& cfg);
PersistentConfig heuristic_config(const HostGraph& g, const Table& table, int R);
JobDev make_job(const HostGraph& g, const DevGraph& d, const RunBuffers& b, int R, uint64_t seed,
                int t_begin, int t_end, const PersistentConfig& cfg);
int msc_planes(int max_deg);

}  // namespace ising

// Parallel tempering state of a problem: the ladder's tables and the
// exchange arrays of the last run.
struct TemperState {
  ising::DeviceArena arena;
  std::vector<double> betas;      // ladder the tables were built for
  ising::Table rows;              // flip thresholds, one row per temperature
  ising::Table swap;              // exchange thresholds, one row per pair
  ising::SwapDev dev{};
  ising::ClusterDev cluster{};
  bool cluster_on = false;
  int32_t K = 0, n_sets = 0, S = 0, P = 0;
  bool valid = false;             // the last run of the problem was tempering
};

struct ising_problem {
  ising::HostGraph g;
  ising::DevGraph dg;
  ising::RunBuffers run;
  ising::Launcher launcher;
  TemperState temper;
  std::vector<int8_t> init;  // [init_R][n] original order
  int32_t init_R = 0;
  bool trace = false;
  // ising_anneal_noalloc: the run's view of the scratch array, and host
  // copies of what it uploads there (kept, so that repeated calls of one
  // shape reuse their capacity)
  struct {
    ising::RunBuffers run;
    std::vector<uint32_t> rows_p, rows_b;
    ising::PersistentPlan plan;
  } noalloc;
  // the thresholds of the last schedule annealed, reused while it repeats
  struct {
    int32_t kind = -1, n_sweeps = 0;
    double beta0 = 0, beta1 = 0;
    std::vector<double> betas;
    ising::Table table;
  } sched;
};

// Local fields of p's device graph, or null when p has none.
const int32_t* fields_or_null(const ising_problem* p);
// Arguments of the per-pass kernels for a run of p in b (anneal.cpp).
ising::PlainDev make_plain(const ising_problem* p, const ising::RunBuffers& b, int R, uint64_t seed);
// Thresholds of schedule s for p (p->sched.table), rebuilt only when s
// differs from the last schedule p annealed with.
int schedule_table(ising_problem* p, const ising_schedule* s);
// Launch configuration of tuning t (NULL or ISING_PATH_AUTO: the tuned or
// heuristic choice), checked against the problem.
int resolve_config(ising_problem* p, const ising::Table& table, int R, const ising_tuning* t,
                   ising::PersistentConfig& cfg);
