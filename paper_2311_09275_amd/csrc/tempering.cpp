// tempering.cpp -- parallel tempering (replica exchange) on the annealing
// kernels: per-replica temperature rows and an exchange kernel between
// segments of sweeps.
#include <math.h>
#include <string.h>

#include <algorithm>

#include "runtime.h"

using namespace ising;

namespace {

// Tables of a ladder: flip thresholds of every temperature (the sweeps'
// rows, one per temperature instead of one per sweep) and exchange
// thresholds of every adjacent pair, for inverse temperature
// betas[k+1] - betas[k] and indexed by the cut difference, up to the
// largest difference two states can have (sum of |w|).
int ladder_tables(ising_problem* p, const std::vector<double>& betas) {
  TemperState& T = p->temper;
  if (T.rows.id != 0 && T.betas == betas) return ISING_OK;
  Table rows, swap;
  IRET(build_table(betas, p->g.kmax, rows));
  int64_t wabs = 0;
  for (int32_t w : p->g.w) wabs += w < 0 ? -(int64_t)w : (int64_t)w;
  std::vector<double> dbeta;
  for (size_t k = 0; k + 1 < betas.size(); ++k) dbeta.push_back(betas[k + 1] - betas[k]);
  IRET(build_table(dbeta, (int32_t)std::max<int64_t>(wabs, 1), swap));
  T.rows = std::move(rows);
  T.swap = std::move(swap);
  T.betas = betas;
  return ISING_OK;
}

}  // namespace

extern "C" {

int ising_temper(ising_problem* p, const ising_tempering* x, uint64_t seed,
                 const ising_tuning* tuning, void* stream) {
  if (!p || !x || !x->betas) return ISING_ERR_INVALID;
  TraceRange tr("ising_temper");
  const int32_t K = x->n_temps, n_sets = x->n_sets, S = x->n_sweeps, P = x->swap_every;
  if (K < 1 || n_sets < 1 || S < 1 || P < 1 || (int64_t)K * n_sets > 0x7FFFFFFF) {
    set_error("tempering needs n_temps, n_sets, n_sweeps, swap_every >= 1");
    return ISING_ERR_INVALID;
  }
  std::vector<double> betas(x->betas, x->betas + K);
  for (int32_t k = 0; k < K; ++k)
    if (!std::isfinite(betas[(size_t)k]) || betas[(size_t)k] < 0 ||
        (k > 0 && betas[(size_t)k] < betas[(size_t)k - 1])) {
      set_error("tempering betas must be finite, >= 0 and non-decreasing");
      return ISING_ERR_INVALID;
    }
  if (p->trace) {
    set_error("energy tracing is not available for tempering");
    return ISING_ERR_UNSUPPORTED;
  }
  const bool cm = x->cluster_moves != 0;
  if (cm && (x->cluster_from < 0 || x->cluster_from > K)) {
    set_error("cluster_from must lie in 0..n_temps");
    return ISING_ERR_INVALID;
  }
  if (cm && p->g.fields) {
    set_error("cluster moves rely on spin-reversal symmetry, which local fields break");
    return ISING_ERR_UNSUPPORTED;
  }
  if (cm && p->g.n_pad > (1 << 18)) {
    set_error("cluster moves keep a bitmask of the positions in LDS: at most 2^18 positions");
    return ISING_ERR_UNSUPPORTED;
  }
  const int R = K * n_sets;
  IRET(ladder_tables(p, betas));
  TemperState& T = p->temper;
  IRET(upload_graph_once(p->g, p->dg));
  DeviceGuard dg(p->dg.device);
  PersistentConfig cfg;
  IRET(resolve_config(p, T.rows, R, tuning, cfg));
  if (cfg.path == ISING_PATH_MSC) {
    if (tuning && tuning->path == ISING_PATH_MSC) {
      set_error("tempering does not run on the multispin path");
      return ISING_ERR_UNSUPPORTED;
    }
    cfg = heuristic_config(p->g, T.rows, R);
  }
  if (cfg.path == ISING_PATH_FIELD && cfg.G > temper_max_group(T.rows)) {
    if (tuning && tuning->path != ISING_PATH_AUTO) {
      set_error("tempering stages one row per replica: at most %d replicas per block",
                temper_max_group(T.rows));
      return ISING_ERR_UNSUPPORTED;
    }
    while (cfg.G > temper_max_group(T.rows)) cfg.G /= 2;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  IRET(prepare_run(p, T.rows, R, cfg, st));
  RunBuffers& b = p->run;

  // exchange state and thresholds
  const size_t pairs = (size_t)n_sets * (size_t)(K - 1);
  // cluster moves: one workgroup per (set pair, temperature >= from)
  const int n_pairs = cm ? n_sets / 2 : 0;
  const int wgs = n_pairs * (K - (cm ? x->cluster_from : K));
  const size_t cl_stats = (size_t)n_pairs * (size_t)K;
  // the BFS queue and the position CSR go to LDS when they fit
  const int n_adj = (int)(2 * p->g.m);
  const bool cl_stage = p->g.n_pad < 65536 && n_adj < 65536 &&
                        houdayer_lds(p->g.n, p->g.n_pad, n_adj, true) <= 150 * 1024;
  const size_t cl_scratch = cl_stage ? 0 : (size_t)wgs * (size_t)p->g.n_pad;
  const size_t bytes = 2 * DeviceArena::span(sizeof(int32_t) * (size_t)R) +
                       DeviceArena::span(sizeof(long long) * pairs) +
                       DeviceArena::span(sizeof(uint32_t) * T.swap.tq.size()) +
                       2 * DeviceArena::span(sizeof(int32_t) * (size_t)T.swap.S) +
                       2 * DeviceArena::span(sizeof(long long) * cl_stats) +
                       DeviceArena::span(sizeof(int32_t) * cl_scratch);
  IRET(T.arena.reserve(bytes));
  SwapDev X;
  memset(&X, 0, sizeof X);
  X.K = K;
  X.n_sets = n_sets;
  X.seed_lo = (uint32_t)seed;
  X.seed_hi = (uint32_t)(seed >> 32);
  X.energy = b.energy;
  X.temp = T.arena.take<int32_t>((size_t)R);
  X.slot = T.arena.take<int32_t>((size_t)R);
  X.swaps = T.arena.take<long long>(pairs);
  uint32_t* tq = T.arena.take<uint32_t>(T.swap.tq.size());
  int32_t* off = T.arena.take<int32_t>((size_t)T.swap.S);
  int32_t* len = T.arena.take<int32_t>((size_t)T.swap.S);
  // small, synchronous: the host tables may change with the next ladder
  ICHK(hipMemcpy(tq, T.swap.tq.data(), sizeof(uint32_t) * T.swap.tq.size(), hipMemcpyHostToDevice));
  if (T.swap.S > 0) {
    ICHK(hipMemcpy(off, T.swap.off.data(), sizeof(int32_t) * T.swap.S, hipMemcpyHostToDevice));
    ICHK(hipMemcpy(len, T.swap.len.data(), sizeof(int32_t) * T.swap.S, hipMemcpyHostToDevice));
  }
  X.tq = tq;
  X.off = off;
  X.len = len;
  T.dev = X;
  ClusterDev Y;
  memset(&Y, 0, sizeof Y);
  Y.K = K;
  Y.n_pairs = n_pairs;
  Y.from = cm ? x->cluster_from : K;
  Y.n = p->g.n;
  Y.n_pad = p->g.n_pad;
  Y.R = R;
  Y.n_adj = n_adj;
  Y.stage = cl_stage ? 1 : 0;
  Y.unit = cl_stage && p->g.unit && p->g.n_pad < 32768 ? 1 : 0;
  Y.seed_lo = X.seed_lo;
  Y.seed_hi = X.seed_hi;
  Y.row = p->dg.row;
  Y.adj = p->dg.adj;
  Y.wgt = p->dg.wgt;
  Y.grp = p->dg.grp;
  Y.pos = p->dg.pos;
  Y.slot = X.slot;
  Y.energy = b.energy;
  if (cfg.path == ISING_PATH_PLAIN) {
    Y.spins = b.spins;
    Y.field = b.field;
    Y.best = static_cast<int8_t*>(b.best);
    Y.snap = b.snap;
  } else {
    Y.packed = b.save;
  }
  Y.moves = T.arena.take<long long>(cl_stats);
  Y.sites = T.arena.take<long long>(cl_stats);
  Y.queue = T.arena.take<int32_t>(cl_scratch);
  T.cluster = Y;
  T.cluster_on = cm;
  T.K = K;
  T.n_sets = n_sets;
  T.S = S;
  T.P = P;
  p->temper.valid = false;

  ICHK(hipEventRecord(b.ev0, st));
  ICHK(launch_pt_init(T.dev, st));
  if (cl_stats) ICHK(launch_fill_i32(reinterpret_cast<int32_t*>(Y.moves), 0, 2 * (int64_t)cl_stats, st));
  if (cl_stats) ICHK(launch_fill_i32(reinterpret_cast<int32_t*>(Y.sites), 0, 2 * (int64_t)cl_stats, st));
  if (cfg.path == ISING_PATH_PLAIN) {
    PlainDev Pd = make_plain(p, b, R, seed);
    Pd.temp = T.dev.temp;
    static thread_local JobDev hjob;
    hjob = make_job(p->g, p->dg, b, R, seed, 0, S, cfg);
    ICHK(hipMemcpy(b.job_dev, &hjob, sizeof(JobDev), hipMemcpyHostToDevice));
    PlainPlan plan{S, p->g.C, p->g.cls.data(), &T.dev, P, cm ? &T.cluster : nullptr};
    ICHK(launch_plain_anneal(Pd, plan, st));
    ICHK(launch_argmax(b.job_dev, 1, st));
  } else {
    std::vector<JobSpec> js{JobSpec{&p->g, &p->dg, &b, R, seed, 0, S}};
    TemperPlan plan{S, P, &T.dev, cm ? &T.cluster : nullptr};
    IRET(run_persistent(p->launcher, js, cfg, st, st != nullptr, &plan));
  }
  ICHK(hipEventRecord(b.ev1, st));
  b.S = S;
  b.valid = true;
  T.valid = true;
  return ISING_OK;
}

int ising_temper_results(ising_problem* p, int32_t* final_temp, int64_t* swaps,
                         int64_t* cluster_moves, int64_t* cluster_sites) {
  if (!p) return ISING_ERR_INVALID;
  TemperState& T = p->temper;
  if (!T.valid || !p->run.valid) {
    set_error("the last run of this problem was not tempering");
    return ISING_ERR_STATE;
  }
  DeviceGuard g(p->dg.device);
  ICHK(hipStreamSynchronize(p->run.stream));
  if (final_temp)
    ICHK(hipMemcpy(final_temp, T.dev.temp, sizeof(int32_t) * (size_t)T.K * T.n_sets,
                   hipMemcpyDeviceToHost));
  const size_t pairs = (size_t)T.n_sets * (size_t)(T.K - 1);
  if (swaps && pairs) {
    std::vector<long long> tmp(pairs);
    ICHK(hipMemcpy(tmp.data(), T.dev.swaps, sizeof(long long) * pairs, hipMemcpyDeviceToHost));
    for (size_t i = 0; i < pairs; ++i) swaps[i] = (int64_t)tmp[i];
  }
  const size_t cl = T.cluster_on ? (size_t)(T.n_sets / 2) * (size_t)T.K : 0;
  if ((cluster_moves || cluster_sites) && !T.cluster_on) {
    set_error("the last tempering run made no cluster moves");
    return ISING_ERR_STATE;
  }
  if (cl) {
    std::vector<long long> tmp(cl);
    if (cluster_moves) {
      ICHK(hipMemcpy(tmp.data(), T.cluster.moves, sizeof(long long) * cl, hipMemcpyDeviceToHost));
      for (size_t i = 0; i < cl; ++i) cluster_moves[i] = (int64_t)tmp[i];
    }
    if (cluster_sites) {
      ICHK(hipMemcpy(tmp.data(), T.cluster.sites, sizeof(long long) * cl, hipMemcpyDeviceToHost));
      for (size_t i = 0; i < cl; ++i) cluster_sites[i] = (int64_t)tmp[i];
    }
  }
  return ISING_OK;
}

}  // extern "C"
