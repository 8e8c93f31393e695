// kernels.h -- host-side entry points of the HIP kernels (kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "device_types.h"

namespace ising {

// Colour classes of one problem for the per-pass launches.
struct PlainPlan {
  int S;             // sweeps
  int C;             // colours
  const int32_t* cls;  // host [2*C] first and end group of each class
  // parallel tempering: an exchange round after every swap_every-th sweep
  // (null = none)
  const SwapDev* swap = nullptr;
  int swap_every = 0;
  const ClusterDev* cluster = nullptr;  // cluster moves before each round
  // sweeps [t_begin, t_end) of the schedule (t_end < 0: to S); the initial
  // state is drawn only when t_begin = 0, else the arrays hold sweep t_begin
  int t_begin = 0, t_end = -1;
};

// One persistent launch (FIELD or MSC) over a unit list.
struct LaunchPersistent {
  const JobDev* jobs;      // device [jobs]
  const int2* units;       // device [units]: (job, replica block)
  const int32_t* list_off; // device [9]: unit lists by XCD
  int32_t* ctr;            // device [8]: list cursors, zero before launch
  int grid;
  size_t lds_bytes;        // dynamic LDS per workgroup
  int planes;              // MSC: bit planes of the unsatisfied-bond counter
  int adj;                 // FIELD: 0 = adjacency in HBM, 1 = staged 16-bit CSR,
                           // 2 = staged degree-4 form (every vertex of degree 4),
                           // 3 = each job's own form (JobDev::adj_form),
                           // 4 = degree-4 blocks read from HBM
  int width = 0;           // MSC: 0 = general form (units of 32-replica words);
                           // 8, 16, 32 = degree-4 form with units of that many replicas
};

hipError_t launch_plain_anneal(const PlainDev& P, const PlainPlan& plan, hipStream_t s);
hipError_t launch_field(const LaunchPersistent& L, int block, hipStream_t s);
hipError_t launch_msc(const LaunchPersistent& L, int block, hipStream_t s);
// Resident workgroups per CU of a persistent kernel (path 2 = FIELD, 3 = MSC;
// adj = the FIELD adjacency form, as in LaunchPersistent, or the MSC width).
int persistent_occupancy(int path, int block, int adj, size_t lds_bytes);
hipError_t set_persistent_lds_limit(int path, int block, size_t lds_bytes);
// Per job: argmax over replicas of best_cut, packed into *argmax as
// (best_cut + 2^31) << 32 | (2^32 - 1 - r): the lowest replica wins ties.
hipError_t launch_argmax(const JobDev* jobs, int n_jobs, hipStream_t s);
hipError_t launch_gather(const void* buf, int layout, int R, int n_pad, int r, const int32_t* pos,
                         int n, int32_t* out, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int32_t value, int64_t count, hipStream_t s);
// Every replica's int8 state: src [R][n_pad] in position order to out
// [R][n] in original order (pos = original id -> position).
hipError_t launch_gather_states(const int8_t* src, int R, int n_pad, const int32_t* pos, int n,
                                int8_t* out, hipStream_t s);
// Parallel tempering: initial ladders, and exchange round m (which also
// zeroes clear8[0..7] when given).
hipError_t launch_pt_init(const SwapDev& X, hipStream_t s);
hipError_t launch_swap(const SwapDev& X, int m, int32_t* clear8, hipStream_t s);
// Houdayer cluster moves of round m, after sweep t (one workgroup per pair
// and temperature from X.from up).
hipError_t launch_houdayer(const ClusterDev& X, int m, int t, hipStream_t s);
// Dynamic LDS of the cluster-move kernel (bitmasks, plus the staged queue
// and CSR when `stage`).
size_t houdayer_lds(int n, int n_pad, int n_adj, bool stage);

// Static LDS of the persistent kernels (bytes), for the LDS budget.
constexpr size_t kFieldStaticLds = 512;
constexpr size_t kMscStaticLds = 4096;

}  // namespace ising
