// batch.cpp -- batched persistent launches and the launch autotuner.
//
// A batch is many problems of uneven size, each with its own seed and
// replicas, annealed by one persistent launch: the unit list holds every
// (problem, replica block) pair in longest-first order, spread over eight
// lists (one per XCD).  The launch sequence is captured once into a
// hipGraph and replayed while the batch shape is unchanged.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>

#include "runtime.h"

namespace ising {
namespace {

std::mutex g_mu;
Launcher* g_launcher = nullptr;  // shared by ising_anneal_batch callers

Launcher& batch_launcher() {
  if (!g_launcher) g_launcher = new Launcher();
  return *g_launcher;
}

// ---------------------------------------------------------------- tuning cache
std::mutex g_tune_mu;
std::map<std::string, PersistentConfig> g_tune;
bool g_tune_loaded = false;

std::string batch_key(const std::vector<const HostGraph*>& gs, int R, int S) {
  int64_t total = 0;
  int max_pad = 0, max_deg = 0, max_c = 0;
  bool unit = true;
  for (const HostGraph* g : gs) {
    total += g->n_pad;
    max_pad = std::max(max_pad, g->n_pad);
    max_deg = std::max(max_deg, g->max_deg);
    max_c = std::max(max_c, g->C);
    unit = unit && g->unit;
  }
  char buf[160];
  // sizes rounded to 1/8 octaves so that near-identical shapes share an entry
  auto q = [](int64_t x) {
    int b = 0;
    while ((int64_t(1) << (b + 1)) <= x) ++b;
    return (int64_t)((x >> std::max(b - 3, 0)) << std::max(b - 3, 0));
  };
  snprintf(buf, sizeof buf, "b%zu_t%lld_m%lld_R%d_d%d_c%d_u%d_s%d", gs.size(), (long long)q(total),
           (long long)q(max_pad), R, max_deg, max_c, unit ? 1 : 0, S >= 64 ? 64 : S);
  return buf;
}

void load_tune_file() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = getenv("ISING_TUNE_CACHE");
  if (!path) return;
  FILE* f = fopen(path, "r");
  if (!f) return;
  char key[200];
  int a, b, c;
  int d;
  while (fscanf(f, "%199s %d %d %d %d", key, &a, &b, &c, &d) == 5)
    g_tune[key] = PersistentConfig{a, b, c, d};
  fclose(f);
}

void save_tune_file() {
  const char* path = getenv("ISING_TUNE_CACHE");
  if (!path) return;
  FILE* f = fopen(path, "w");
  if (!f) return;
  for (auto& kv : g_tune)
    fprintf(f, "%s %d %d %d %d\n", kv.first.c_str(), kv.second.path, kv.second.G, kv.second.block,
            kv.second.adj);
  fclose(f);
}

// Each problem's threshold table of the schedule: the one it keeps while the
// schedule repeats (so that a repeated batch neither recomputes nor uploads
// it again).
int batch_tables(ising_problem* const* ps, int count, const ising_schedule* s,
                 std::vector<const Table*>& tables) {
  tables.resize((size_t)count);
  for (int i = 0; i < count; ++i) {
    IRET(schedule_table(ps[i], s));
    tables[(size_t)i] = &ps[i]->sched.table;
  }
  return ISING_OK;
}

int ensure_all(ising_problem* const* ps, int count) {
  int dev = -1;
  for (int i = 0; i < count; ++i) {
    ising_problem* p = ps[i];
    if (!p) return ISING_ERR_INVALID;
    if (p->dg.device < 0) {
      int n = 0;
      if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) {
        (void)hipGetLastError();
        set_error("no HIP device available");
        return ISING_ERR_DEVICE;
      }
      IRET(upload_graph(p->g, p->dg));
    }
    if (dev >= 0 && p->dg.device != dev) {
      set_error("all problems of a batch must live on one device");
      return ISING_ERR_INVALID;
    }
    dev = p->dg.device;
  }
  return ISING_OK;
}

int check_all(ising_problem* const* ps, int count, const std::vector<const Table*>& tables, int R,
              const PersistentConfig& c) {
  for (int i = 0; i < count; ++i) IRET(check_config(ps[i]->g, *tables[(size_t)i], R, c));
  return ISING_OK;
}

// Run a batch of problems with one persistent launch.
int run_batch(ising_problem* const* ps, int count, const std::vector<const Table*>& tables, int R,
              const uint64_t* seeds, const PersistentConfig& cfg, hipStream_t st, Launcher& L,
              bool use_graph) {
  if (cfg.path == ISING_PATH_PLAIN) {
    set_error("the plain path has no batched form");
    return ISING_ERR_INVALID;
  }
  for (int i = 0; i < count; ++i) IRET(prepare_run(ps[i], *tables[(size_t)i], R, cfg, st));
  std::vector<JobSpec> specs;
  for (int i = 0; i < count; ++i)
    specs.push_back(JobSpec{&ps[i]->g, &ps[i]->dg, &ps[i]->run, R, seeds[i], 0, tables[(size_t)i]->S});
  for (int i = 0; i < count; ++i) ICHK(hipEventRecord(ps[i]->run.ev0, st));
  IRET(run_persistent(L, specs, cfg, st, use_graph));
  for (int i = 0; i < count; ++i) {
    ICHK(hipEventRecord(ps[i]->run.ev1, st));
    RunBuffers& b = ps[i]->run;
    b.cfg = cfg;
    b.seed = seeds[i];
    b.t_done = tables[(size_t)i]->S;
    b.valid = true;
    ps[i]->temper.valid = false;  // the last run is this anneal
  }
  return ISING_OK;
}

}  // namespace
}  // namespace ising

using namespace ising;

int tune_lookup(const HostGraph& g, const Table& t, int R, PersistentConfig& c) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  load_tune_file();
  auto it = g_tune.find(batch_key({&g}, R, t.S));
  if (it == g_tune.end()) return ISING_ERR_STATE;
  if (check_config(g, t, R, it->second) != ISING_OK) return ISING_ERR_STATE;
  c = it->second;
  return ISING_OK;
}

extern "C" {

int ising_anneal_batch(ising_problem* const* ps, int32_t count, const ising_schedule* s,
                       int32_t n_replicas, const uint64_t* seeds, const ising_tuning* tuning,
                       void* stream) {
  if (!ps || count < 1 || !s || n_replicas < 1 || !seeds) return ISING_ERR_INVALID;
  TraceRange tr("ising_anneal_batch");
  std::vector<const Table*> tables;
  IRET(batch_tables(ps, count, s, tables));
  IRET(ensure_all(ps, count));
  DeviceGuard dg(ps[0]->dg.device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  PersistentConfig cfg;
  if (tuning && tuning->path != ISING_PATH_AUTO) {
    cfg.path = tuning->path;
    cfg.G = tuning->replicas_per_block > 0 ? tuning->replicas_per_block : 1;
    cfg.block = tuning->block_threads > 0 ? tuning->block_threads
                                          : (cfg.path == ISING_PATH_MSC ? 256 : 1024);
    cfg.adj = tuning->lds_adjacency;
  } else {
    std::vector<const HostGraph*> gs;
    for (int i = 0; i < count; ++i) gs.push_back(&ps[i]->g);
    bool found = false;
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      load_tune_file();
      auto it = g_tune.find(batch_key(gs, n_replicas, tables[0]->S));
      if (it != g_tune.end() && check_all(ps, count, tables, n_replicas, it->second) == ISING_OK) {
        cfg = it->second;
        found = true;
      }
    }
    if (!found) {
      // the largest problem decides what fits
      int big = 0;
      for (int i = 1; i < count; ++i)
        if (ps[i]->g.n_pad > ps[big]->g.n_pad) big = i;
      cfg = heuristic_config(ps[big]->g, *tables[(size_t)big], n_replicas);
      if (cfg.path != ISING_PATH_PLAIN) {
        // with many problems the unit count is large already: keep G = 1
        // unless the LDS budget allows more and units stay plentiful
        const int cus = std::max(device_cu_count(), 1);
        while (cfg.G > 1 && (int64_t)count * n_replicas / cfg.G < 4 * cus) cfg.G /= 2;
      }
    }
  }
  if (cfg.path == ISING_PATH_PLAIN) {
    // one plain anneal per problem, back to back on the stream
    Launcher& L = batch_launcher();
    std::lock_guard<std::mutex> lk(g_mu);
    if (!L.ev0) ICHK(hipEventCreate(&L.ev0));
    if (!L.ev1) ICHK(hipEventCreate(&L.ev1));
    ICHK(hipEventRecord(L.ev0, st));
    ising_tuning t{ISING_PATH_PLAIN, 1, 256, 0};
    for (int i = 0; i < count; ++i) IRET(ising_anneal_tuned(ps[i], s, n_replicas, seeds[i], &t, stream));
    ICHK(hipEventRecord(L.ev1, st));
    return ISING_OK;
  }
  IRET(check_all(ps, count, tables, n_replicas, cfg));
  std::lock_guard<std::mutex> lk(g_mu);
  return run_batch(ps, count, tables, n_replicas, seeds, cfg, st, batch_launcher(), st != nullptr);
}

int ising_last_batch_ms(double* ms) {
  if (!ms) return ISING_ERR_INVALID;
  std::lock_guard<std::mutex> lk(g_mu);
  Launcher& L = batch_launcher();
  if (!L.ev0 || !L.ev1) return ISING_ERR_STATE;
  ICHK(hipEventSynchronize(L.ev1));
  float f = 0;
  ICHK(hipEventElapsedTime(&f, L.ev0, L.ev1));
  *ms = f;
  return ISING_OK;
}

int ising_autotune(ising_problem* const* ps, int32_t count, const ising_schedule* s,
                   int32_t n_replicas, int32_t prefix_sweeps, ising_tuning* best, void* stream) {
  if (!ps || count < 1 || !s || n_replicas < 1 || !best) return ISING_ERR_INVALID;
  TraceRange tr("ising_autotune");
  std::vector<double> beta;
  IRET(eval_schedule(s, beta));
  const int S = (int)beta.size();
  const int prefix = prefix_sweeps > 0 ? std::min(prefix_sweeps, S) : std::min(S, 200);
  // The trial anneals take sweeps spread evenly over the real schedule, so
  // that they meet each temperature for the same share of their sweeps: the
  // paths' costs depend on how many moves are accepted.  Every candidate is
  // timed on `prefix` sweeps; the three fastest are timed again on the whole
  // schedule (at most max(5 prefix, 4000) sweeps), since the cost of a
  // launch is not quite proportional to its sweeps (the longest units set
  // the end of a persistent launch).
  // (the trial schedules replace each problem's kept table)
  std::vector<double> pre;
  ising_schedule ps_sched{};
  auto trial_tables = [&](int n, std::vector<const Table*>& tables) {
    pre.assign((size_t)n, 0.0);
    for (int i = 0; i < n; ++i) pre[(size_t)i] = beta[(size_t)((int64_t)i * S / n)];
    ps_sched = ising_schedule{ISING_SCHED_EXPLICIT, n, 0, 0, pre.data()};
    return batch_tables(ps, count, &ps_sched, tables);
  };
  std::vector<const Table*> tables;
  IRET(trial_tables(prefix, tables));
  IRET(ensure_all(ps, count));
  DeviceGuard dg(ps[0]->dg.device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  std::vector<uint64_t> seeds((size_t)count);
  for (int i = 0; i < count; ++i) seeds[(size_t)i] = 0x5EEDull + (uint64_t)i;

  std::vector<PersistentConfig> cands;
  // adjacency: 0 = each problem's staged form unless that costs occupancy
  // (mixed forms in one launch), 1 = staged for every problem, 2 = HBM
  for (int adj : {0, 1, 2})
    for (int block : {256, 512, 1024})
      for (int G : {1, 2, 4, 8, 16}) cands.push_back(PersistentConfig{ISING_PATH_FIELD, G, block, adj});
  for (int block : {256, 512})
    for (int G : {1, 2, 4}) cands.push_back(PersistentConfig{ISING_PATH_MSC, G, block, 0});
  // the multispin degree-4 form, 8, 16 or 32 replicas per unit
  for (int block : {256, 512, 1024})
    for (int G : {8, 16, 32}) cands.push_back(PersistentConfig{ISING_PATH_MSC, G, block, 0});

  Launcher L;
  auto time_config = [&](const std::vector<const Table*>& tb, const PersistentConfig& c, double& ms) {
    ms = 1e300;
    if (check_all(ps, count, tb, n_replicas, c) != ISING_OK) return ISING_OK;
    for (int rep = 0; rep < 2; ++rep) {  // the first run warms caches and code
      int rc = run_batch(ps, count, tb, n_replicas, seeds.data(), c, st, L, false);
      if (rc != ISING_OK) {
        ms = 1e300;
        return ISING_OK;
      }
      ICHK(hipEventSynchronize(L.ev1));
      float f = 0;
      ICHK(hipEventElapsedTime(&f, L.ev0, L.ev1));
      ms = std::min(ms, (double)f);
    }
    return ISING_OK;
  };
  std::vector<std::pair<double, size_t>> timed;
  for (size_t i = 0; i < cands.size(); ++i) {
    double ms;
    IRET(time_config(tables, cands[i], ms));
    if (ms < 1e300) timed.push_back({ms, i});
  }
  PersistentConfig winner{ISING_PATH_PLAIN, 1, 256};
  if (!timed.empty()) {
    std::sort(timed.begin(), timed.end());
    winner = cands[timed[0].second];
    const int longer = std::min(S, std::max(5 * prefix, 4000));
    if (timed.size() > 1 && longer > prefix) {
      std::vector<const Table*> tables2;
      IRET(trial_tables(longer, tables2));
      double best_ms = 1e300;
      for (size_t k = 0; k < std::min<size_t>(3, timed.size()); ++k) {
        double ms;
        IRET(time_config(tables2, cands[timed[k].second], ms));
        if (ms < best_ms) {
          best_ms = ms;
          winner = cands[timed[k].second];
        }
      }
    }
  }
  for (int i = 0; i < count; ++i) ps[i]->run.valid = false;  // prefix results are not results
  best->path = winner.path;
  best->replicas_per_block = winner.G;
  best->block_threads = winner.block;
  best->lds_adjacency = winner.adj;
  std::vector<const HostGraph*> gs;
  for (int i = 0; i < count; ++i) gs.push_back(&ps[i]->g);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_tune_file();
    g_tune[batch_key(gs, n_replicas, S)] = winner;
    save_tune_file();
  }
  return ISING_OK;
}

}  // extern "C"
