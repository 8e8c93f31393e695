/*
 * ising.h -- C ABI of libising, an MI355X (gfx950) many-replica Metropolis
 * annealer for sparse Ising / MaxCut problems.
 *
 * Problem (paper Sec. II.A): weighted MaxCut on n variables with integer
 * edge weights, as in the Gset instances (toroidal +-1 spin glasses, sparse
 * random unweighted graphs; Table I).  The library maximises
 *     cut(s) = sum_e w_e (1 - s_u s_v) / 2,   s in {-1,+1}^n,
 * through the Ising energy E(s) = sum_e w_e s_u s_v (couplings J = -w), with
 * cut = (W - E)/2 and W = sum_e w_e.  A solution is reported per variable
 * in the original numbering (the paper's appendices list variables 1..N;
 * here ids are 0-based, and x = (1+s)/2 gives the paper's bits).
 *
 * Method: R independent replicas, each doing single-spin-flip Metropolis
 * sweeps under an annealing schedule beta_t (work is counted in sweeps,
 * Sec. III.A; independent trials, Sec. III.A and II.B).  Inside a sweep the
 * vertices are visited one colour class at a time (a proper colouring, so
 * the updates of one class are independent), each with
 *     k = s_i h_i,  h_i = -sum_j w_ij s_j   (flipping s_i changes E by 2k)
 *     accept iff k <= 0 or u < Tq(beta_t, k),  Tq = floor(2^32 exp(-2 k beta_t))
 * where u is word j of Philox4x32-10(key = seed, counter = (t, run, r, 0)),
 * j being the vertex's rank in its run -- see ising_create for the runs
 * and their numbering.  The best cut of a
 * replica is taken over its initial state and its end-of-sweep states
 * (strict improvement, earliest sweep wins).  Every step is integer
 * arithmetic on the device, so results are bit-identical across kernel
 * variants, batch compositions and runs.
 *
 * Conventions
 *  - Every call returns an int status: ISING_OK (0) or a negative code.
 *  - Out-parameters are written only on success.
 *  - Inputs are copied; the caller keeps ownership of every pointer it
 *    passes.  Output buffers are caller-owned host memory unless a name
 *    says "device".
 *  - A handle is not thread-safe; distinct handles may be used concurrently
 *    from different threads.
 *  - `stream` arguments are hipStream_t values passed as void*; NULL means
 *    the null stream.  Work is enqueued and the call returns; calls that
 *    return results to the host synchronise that stream first.
 *  - No exception crosses the ABI.
 */
#ifndef ISING_H
#define ISING_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status */
#define ISING_OK 0
#define ISING_ERR_INVALID -1     /* argument or problem rejected */
#define ISING_ERR_NOMEM -2       /* host or device allocation failed, or
                                    a request exceeds the server budget */
#define ISING_ERR_DEVICE -3      /* a HIP call failed (no GPU, fault, ...) */
#define ISING_ERR_STATE -4       /* call not valid in the handle's state */
#define ISING_ERR_UNSUPPORTED -5 /* e.g. the multispin path on weights != +-1 */
#define ISING_ERR_TIMEOUT -6     /* server wait timed out */

/* Human-readable text of a status code (static storage). */
const char* ising_status_string(int status);
/* Detail of the last error raised on the calling thread (thread-local
 * storage, valid until the thread's next failing call). */
const char* ising_last_error(void);

/*
 * Device memory (optional).  By default the library takes its device memory
 * (problem graphs, run buffers, launch structures, tempering state, server
 * pools) with hipMalloc and returns it with hipFree.  A caller may route it
 * through its own allocator, e.g. PyTorch's caching allocator:
 *   alloc(bytes, device, ctx) returns device memory of `device` (the
 *   current device at the call), at least `bytes`, 256-byte aligned, or
 *   NULL (the library call then fails with ISING_ERR_NOMEM);
 *   free(ptr, bytes, device, ctx) takes back exactly what alloc returned.
 * Memory is returned through the functions it was obtained with, even
 * after the allocator changes; before calling free the library waits for
 * the device to finish (the allocator may reuse the memory at once).  Both
 * NULL restores hipMalloc/hipFree; one NULL is ISING_ERR_INVALID.  Affects
 * later allocations only.  The functions may be called from the server's
 * scheduler thread.
 */
typedef void* (*ising_alloc_fn)(size_t bytes, int device, void* ctx);
typedef void (*ising_free_fn)(void* ptr, size_t bytes, int device, void* ctx);
int ising_set_allocator(ising_alloc_fn alloc, ising_free_fn free_fn, void* ctx);

/* --------------------------------------------------------------- problem */
typedef struct ising_problem ising_problem;

/*
 * Compile a MaxCut problem (paper Sec. II.A: n variables, m weighted edges).
 *   n        number of vertices, 1 <= n < 2^28
 *   m        number of undirected edges, m >= 0
 *   u, v, w  edge e joins u[e] and v[e] (0-based) with weight w[e]
 *   colour   NULL: greedy first-fit colouring in index order (each vertex
 *            takes the smallest colour not held by a lower-numbered
 *            neighbour; on an even-sided row-major torus this is the
 *            checkerboard).  Otherwise colour[i] in [0, 1024) per vertex; it
 *            must be proper.  Classes are swept in colour order 0, 1, ...
 * Random-number runs: inside each colour class, in ascending vertex id,
 * consecutive runs of four vertices share one Philox block (a class's last
 * run may be shorter).  Runs are numbered 0, 1, ... in class order, then in
 * id order within a class; counter word 1 is that number and the i-th
 * vertex of a run uses output word i.
 * Errors (ISING_ERR_INVALID): n out of range; m < 0; NULL arrays with
 * m > 0; an id out of range; a self loop; a repeated undirected edge;
 * w == 0 or |w| > 32768; 2 * sum_e |w_e| >= 2^30; an improper or
 * out-of-range colouring.  ISING_ERR_NOMEM on allocation failure.
 * This call is host-only; device memory is allocated on first use.
 * *out is library-owned until ising_destroy.
 */
int ising_create(int32_t n, int64_t m, const int32_t* u, const int32_t* v,
                 const int32_t* w, const int32_t* colour, ising_problem** out);

/* Free a problem and all its host and device memory.  NULL is a no-op. */
int ising_destroy(ising_problem* p);

typedef struct {
  int32_t n, n_colours;
  int64_t m;
  int64_t total_weight;   /* W = sum_e w_e */
  int32_t kmax;           /* max_i (sum_j |w_ij| + 2 |b_i|): the largest |k| */
  int32_t max_degree;
  int32_t unit_weights;   /* 1 when every |w| == 1 (multispin path allowed) */
  int32_t n_padded;       /* vertices after padding each class to 4 */
  int32_t fields;         /* 1 when nonzero local fields are set */
} ising_info;

/* Facts about a compiled problem (host-only). */
int ising_problem_info(const ising_problem* p, ising_info* out);
/* The colour of every vertex, original order (host-only).  [n] */
int ising_colouring(const ising_problem* p, int32_t* colour);
/* Edge labels of the degree-4 form (host-only).  For a problem with unit
 * weights, every vertex of degree 4 and a padded state of at most 2^16
 * words (about 65,000 vertices), lab[4 v + e] is v's neighbour with label e, in
 * original ids, such that lab[4 u + (e XOR 1)] == v whenever
 * lab[4 v + e] == u: each edge carries labels 2f and 2f + 1 at its two
 * ends.  The FIELD kernel's degree-4 forms push a flip of v into bit
 * e XOR 1 of neighbour e's bond word, so every push of one label is an
 * XOR of one fixed bit.  [4n], caller-owned.  ISING_ERR_UNSUPPORTED when
 * the problem has no degree-4 form. */
int ising_neighbour_labels(const ising_problem* p, int32_t* lab);
/* MaxCut value of a +-1 assignment in original order (host-only); the
 * plain cut, without the field term. */
int ising_eval_cut(const ising_problem* p, const int8_t* spins, int64_t* cut);
/*
 * Local fields (the paper notes that some sparse Ising problems have them,
 * Sec. II.C): b[v] for every vertex, original order, copied; NULL removes
 * them.  With fields the energy is E(s) = sum_e w_e s_u s_v - 2 sum_v b_v s_v
 * (so h_v = -sum_u w_vu s_u + 2 b_v and k = s_v h_v as before), and every
 * "cut" the library reports (best cuts, per-replica cuts, argmax) is the
 * objective (W - E)/2 = cut(s) + sum_v b_v s_v.  kmax becomes
 * max_v (sum_u |w_vu| + 2 |b_v|).  Applies to later runs; it waits for
 * the problem's own last run, but must not be called while a server holds
 * a request of p (the server reads the same device copy).  Refused with
 * fields: the multispin path and the degree-4 adjacency forms (their state
 * words hold no field; other FIELD forms are chosen), and tempering's
 * cluster moves (ISING_ERR_UNSUPPORTED).  ISING_ERR_INVALID when some
 * |b_v| > 32768 or sum_v (sum_u |w_vu| + 2 |b_v|) >= 2^30.
 */
int ising_set_fields(ising_problem* p, const int32_t* b);

/* -------------------------------------------------------------- schedule */
enum { ISING_SCHED_LINEAR = 0, ISING_SCHED_GEOMETRIC = 1, ISING_SCHED_EXPLICIT = 2 };

/*
 * Annealing schedule of inverse temperatures beta_t, t = 0 .. n_sweeps-1:
 *   LINEAR     beta0 + (beta1 - beta0) * t/(S-1)
 *   GEOMETRIC  beta0 * (beta1/beta0)^(t/(S-1))     (beta0, beta1 > 0)
 *   EXPLICIT   betas[t]
 * (S = 1 gives beta0.)  Every beta_t must be finite and >= 0.
 */
typedef struct {
  int32_t kind;
  int32_t n_sweeps;
  double beta0, beta1;
  const double* betas;
} ising_schedule;

/*
 * The acceptance thresholds the library uses, Tq(beta_t, k) for
 * k = 1..kmax, written to out[t*kmax + (k-1)] as uint64 (2^32 = always).
 * Host-only; used to check the table against an independent computation
 * before any device run.  ISING_ERR_INVALID on a bad schedule or kmax < 1.
 */
int ising_threshold_table(const ising_schedule* s, int32_t kmax, uint64_t* out);

/* ---------------------------------------------------------------- anneal */
enum {
  ISING_PATH_AUTO = 0,  /* the autotuner's (cached) choice, else FIELD with
                           one replica per block and about one thread per
                           group of a colour class (PLAIN if that does not
                           fit) */
  ISING_PATH_PLAIN = 1, /* state in HBM, one launch per colour pass */
  ISING_PATH_FIELD = 2, /* persistent: replica blocks resident in LDS */
  ISING_PATH_MSC = 3    /* persistent multispin: 32 replicas per word */
};

/*
 * Launch choices.  All of them compute identical results.
 *   path                 ISING_PATH_*
 *   replicas_per_block   FIELD: replicas per workgroup (1, 2, 4, 8, 16);
 *                        MSC: 1, 2 or 4 = 32-replica words per workgroup
 *                        (general form, degree <= 31); 8, 16 or 32 =
 *                        replicas per workgroup in the degree-4 form (unit
 *                        weights, every vertex of degree 4, at most 2^15
 *                        padded vertices: the tori), whose state keeps each
 *                        vertex's spins of those replicas as one bit field
 *   block_threads        256, 512 or 1024 (general MSC form: 256 or 512);
 *                        0 = default
 *   lds_adjacency        FIELD: 0 = decide, 1 = stage a 16-bit adjacency in
 *                        LDS (unit weights, fewer than 2^15 vertices; a
 *                        fixed 48-byte-per-group form with bond-word state
 *                        when every vertex has degree 4, else CSR order), 2 = read the adjacency
 *                        from HBM, 3 = stage it in CSR order even when the
 *                        degree-4 form applies, 4 = read the degree-4 form
 *                        from HBM (unit weights, every vertex of degree 4,
 *                        state of at most 2^16 words).  With 0 a graph whose
 *                        degree-4 form does not fit LDS reads it from HBM.
 */
typedef struct {
  int32_t path;
  int32_t replicas_per_block;
  int32_t block_threads;
  int32_t lds_adjacency;
} ising_tuning;

/*
 * Anneal R = n_replicas replicas of p from their initial states (Philox
 * init draws, or the states given by ising_set_initial_state) through the
 * whole schedule.  Enqueued on `stream`; returns without waiting.  Each
 * call starts afresh.  `tuning` NULL = ISING_PATH_AUTO.
 * Errors: ISING_ERR_INVALID (bad schedule, R < 1, tuning out of range, a
 * threshold table over 2^26 entries); ISING_ERR_UNSUPPORTED (MSC on
 * non-unit weights, FIELD with more than 64 colour classes, the LDS paths
 * (FIELD, MSC) on a vertex of degree above 255 or a threshold row longer
 * than 1024 keys (a schedule whose smallest beta accepts some k > 1024 with
 * nonzero probability), or a problem too large for the requested LDS path;
 * ISING_PATH_AUTO then runs PLAIN);
 * ISING_ERR_NOMEM; ISING_ERR_DEVICE.
 */
int ising_anneal(ising_problem* p, const ising_schedule* s, int32_t n_replicas,
                 uint64_t seed, void* stream);
int ising_anneal_tuned(ising_problem* p, const ising_schedule* s,
                       int32_t n_replicas, uint64_t seed,
                       const ising_tuning* tuning, void* stream);

/*
 * Sweeps [t_begin, t_end) of an anneal (0 <= t_begin < t_end <= S).  With
 * t_begin = 0 it starts afresh like ising_anneal_tuned (which is the range
 * [0, S)); otherwise it continues the problem's last run, which must have
 * the same schedule, replica count and seed and have stopped at t_begin
 * (ISING_ERR_STATE otherwise), in that run's launch configuration.  A run
 * cut into ranges gives the same results, bit for bit, as one call; the
 * results of each range (best cuts so far, states) can be read between
 * ranges.  Errors otherwise as ising_anneal_tuned.
 */
int ising_anneal_range(ising_problem* p, const ising_schedule* s, int32_t n_replicas,
                       uint64_t seed, const ising_tuning* tuning, int32_t t_begin,
                       int32_t t_end, void* stream);

/*
 * Checkpoints of an anneal (after ising_anneal or a range of it; not of a
 * tempering run): the whole device state of the run in a caller-owned host
 * buffer of ising_checkpoint_size bytes (synchronises).  ising_checkpoint_load
 * puts such a buffer back into a problem compiled from the same graph, given
 * the same schedule (ISING_ERR_INVALID otherwise) and the same tracing and
 * initial-state settings (ISING_ERR_STATE otherwise); its results can then
 * be read, and ising_anneal_range continues it from the sweep it had reached.
 * The buffer format is private to the library version that wrote it.
 */
int ising_checkpoint_size(const ising_problem* p, uint64_t* bytes);
int ising_checkpoint_save(ising_problem* p, void* buf);
int ising_checkpoint_load(ising_problem* p, const ising_schedule* s, const void* buf,
                          uint64_t bytes, void* stream);

/*
 * Initial states for subsequent anneals: spins[r*n + i] in {-1,+1}, original
 * order, for r < n_replicas; NULL restores the Philox initial draw.  An
 * anneal with a different R than given here is rejected (ISING_ERR_STATE).
 */
int ising_set_initial_state(ising_problem* p, const int8_t* spins,
                            int32_t n_replicas);

/* Record E after every sweep of every replica in the next anneals
 * (enable = 1) or not (0). */
int ising_set_trace(ising_problem* p, int32_t enable);

/*
 * Results of the last anneal (synchronises its stream).
 *   best_cut       the largest best cut over replicas
 *   best_replica   its replica (lowest index on ties)
 *   per_replica    NULL or [R] best cut of each replica
 * ISING_ERR_STATE before any anneal.
 */
int ising_cut(ising_problem* p, int64_t* best_cut, int32_t* best_replica,
              int64_t* per_replica);

/* Best state of the argmax replica, +-1 per vertex, original order [n]. */
int ising_best_state(ising_problem* p, int8_t* spins);

/*
 * Per-replica detail of the last anneal, any pointer may be NULL, each [R]:
 * best_sweep (-1 = the initial state), accepted flips, final energy E.
 */
int ising_replica_results(ising_problem* p, int32_t* best_sweep,
                          int64_t* accepts, int64_t* final_energy);
/* Best and final state of replica r (either NULL), original order [n]. */
int ising_replica_state(ising_problem* p, int32_t r, int8_t* best_spins,
                        int8_t* final_spins);
/* Final local fields h of replica r, original order [n]; available after
 * PLAIN and FIELD anneals (ISING_ERR_UNSUPPORTED after MSC). */
int ising_replica_field(ising_problem* p, int32_t r, int32_t* field);
/* Energy trace of the last anneal, out[r*S + t] (needs ising_set_trace). */
int ising_energy_trace(ising_problem* p, int64_t* out);
/* Device time of the last anneal in milliseconds (HIP events around the
 * enqueued work; synchronises). */
int ising_last_anneal_ms(ising_problem* p, double* ms);
/* Shape of the last anneal (single or batched): replicas, sweeps and the
 * kernel path that ran.  Any pointer may be NULL.  ISING_ERR_STATE before
 * any anneal. */
int ising_last_run_info(const ising_problem* p, int32_t* n_replicas, int32_t* n_sweeps,
                        int32_t* path);

/* ------------------------------------------------- allocation-free anneal */
/*
 * For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: the anneal
 * of ising_anneal_tuned on the FIELD path, with no hipMalloc, hipFree or
 * other allocating call.  Its results go to caller-owned device buffers,
 * and every other device buffer of the run (threshold rows, launch
 * structures, best-state snapshots) is carved from one fixed array of
 * ISING_NOALLOC_SCRATCH_BYTES bytes per device, held by the library's code
 * object until the process ends.  Requirements and limits:
 *  - the problem's graph is already on the current device (its first
 *    ising_anneal, ising_anneal_batch or ising_temper uploads it;
 *    ISING_ERR_STATE otherwise);
 *  - tuning NULL/AUTO or an explicit FIELD tuning; a configuration that is
 *    not FIELD, initial states or an enabled energy trace give
 *    ISING_ERR_UNSUPPORTED;
 *  - R * n_padded bytes of snapshots plus the rows (about
 *    S * (2 kmax + 10) * 4 bytes) and R * 8 bytes of launch structures must
 *    fit the array, else ISING_ERR_UNSUPPORTED with the sizes in
 *    ising_last_error.
 * Results (device pointers, caller-owned, each written once the enqueued
 * work completes), identical to those of ising_anneal_tuned:
 *   best_cut [R], best_sweep [R] (-1 = initial state), final_energy [R]
 *   (int32); accepts [R] (uint64); argmax [1] = (best cut + 2^31) << 32 |
 *   (2^32 - 1 - best replica); best_states [R][n] int8 +-1, original order.
 * Work is enqueued on `stream` and the call returns.  Every call on one
 * device uses that device's single array: calls whose work overlaps on one
 * GPU (other streams, other threads) race and must be serialised by the
 * caller.  The array keeps the last call's contents; this call rewrites
 * every part it reads.  Other errors as ising_anneal_tuned.
 */
#define ISING_NOALLOC_SCRATCH_BYTES (16u << 20)
typedef struct {
  int32_t* best_cut;
  int32_t* best_sweep;
  int32_t* final_energy;
  uint64_t* accepts;
  uint64_t* argmax;
  int8_t* best_states;
} ising_device_results;
int ising_anneal_noalloc(ising_problem* p, const ising_schedule* s,
                         int32_t n_replicas, uint64_t seed,
                         const ising_tuning* tuning,
                         const ising_device_results* out, void* stream);

/* ------------------------------------------------------ parallel tempering */
/*
 * Parallel tempering (replica exchange), which the paper names among the
 * contenders for sparse Ising optimisation (Sec. II.C): replicas run at
 * different temperatures and exchange them.
 *   n_temps     K >= 1 temperatures per set
 *   betas       [K] inverse temperatures, finite, >= 0, non-decreasing
 *               (copied; the caller keeps ownership)
 *   n_sets      independent sets of K replicas; R = n_sets * K, replica r
 *               is in set r / K and starts at temperature r % K
 *   n_sweeps    S >= 1
 *   swap_every  P >= 1: after sweeps P-1, 2P-1, ... exchange round m
 *               (m = 0, 1, ...) tries the pairs (k, k+1) with k of m's
 *               parity in every set
 * Each sweep is the annealing sweep at the replica's current beta (its
 * Philox counters as in ising_anneal, (t, run, r, 0)).  The pair with the
 * replica a at k and b at k+1 exchanges temperatures with the Metropolis
 * probability of the product of Boltzmann weights: always when
 * q = cut(b) - cut(a) <= 0, else when word 0 of Philox(counter
 * (m, k, set, 3), key seed) is below floor(2^32 exp(-2 q (beta_k+1 -
 * beta_k))).
 */
typedef struct {
  int32_t n_temps;
  const double* betas;
  int32_t n_sets;
  int32_t n_sweeps;
  int32_t swap_every;
  int32_t cluster_moves;  /* nonzero: Houdayer cluster moves (below) */
  int32_t cluster_from;   /* ... at temperatures k >= cluster_from (0..K) */
} ising_tempering;

/*
 * Run parallel tempering on p, enqueued on `stream` (returns without
 * waiting).  Best cuts and states are tracked per replica as in an anneal
 * and read with ising_cut, ising_best_state, ising_replica_results and
 * ising_replica_state; the exchange state with ising_temper_results.
 * `tuning` NULL = automatic (FIELD, else PLAIN when it does not fit); the
 * FIELD path runs a launch per P sweeps and an exchange kernel after each,
 * captured into one hipGraph.  Initial states given with
 * ising_set_initial_state apply (for R = n_sets * K replicas).
 * Errors: ISING_ERR_INVALID (bad ladder or sizes, tuning out of range);
 * ISING_ERR_UNSUPPORTED (the MSC path, energy tracing enabled, FIELD with
 * more replicas per block than the rows it can stage, or what ising_anneal
 * rejects); ISING_ERR_STATE (initial states for another R); ISING_ERR_NOMEM;
 * ISING_ERR_DEVICE.
 */
int ising_temper(ising_problem* p, const ising_tempering* pt, uint64_t seed,
                 const ising_tuning* tuning, void* stream);
/*
 * Houdayer cluster moves (replica cluster moves, which the paper names as
 * combinable with parallel tempering, Sec. II.C).  With cluster_moves set,
 * sets 2p and 2p+1 form pair p (an odd last set has no partner).  At every
 * exchange point, before exchange round m, pair p makes one move at each
 * temperature k >= cluster_from between its two replicas a and b there: D
 * = the sites where they disagree (no move when D is empty); the seed is
 * the (u mod |D|)-th site of D in ascending vertex id, u word 0 of
 * Philox(counter (m, k, p, 4), key seed); the connected component of the
 * seed in the subgraph induced by D flips in both replicas.  The move keeps
 * E_a + E_b and is always accepted.  Problems of more than 2^18 padded
 * positions are refused (ISING_ERR_UNSUPPORTED); cluster_from outside
 * 0..K is ISING_ERR_INVALID.
 */

/*
 * Exchange state after the last ising_temper of p (synchronises).  Any
 * pointer may be NULL.
 *   final_temp     [R] temperature index of every replica at the end
 *   swaps          [n_sets][K-1] accepted exchanges of each pair (k, k+1)
 *   cluster_moves  [n_sets/2][K] cluster moves made at each temperature
 *   cluster_sites  [n_sets/2][K] sites flipped by them, summed
 * ISING_ERR_STATE when the last run of p was not tempering, or asks for
 * cluster counts of a run without cluster moves.
 */
int ising_temper_results(ising_problem* p, int32_t* final_temp, int64_t* swaps,
                         int64_t* cluster_moves, int64_t* cluster_sites);

/* --------------------------------------------------------------- batching */
/*
 * Anneal `count` problems in one persistent launch (captured once into a
 * hipGraph and replayed while the batch shape is unchanged).  Problem i uses
 * seeds[i], the shared schedule and R replicas; results are read per
 * problem with ising_cut / ising_best_state / ising_replica_*.  Results
 * equal those of separate ising_anneal calls bit for bit.  `tuning` NULL =
 * autotune.  Errors as ising_anneal.
 */
int ising_anneal_batch(ising_problem* const* ps, int32_t count,
                       const ising_schedule* s, int32_t n_replicas,
                       const uint64_t* seeds, const ising_tuning* tuning,
                       void* stream);
/* Device time of the last batch launch in milliseconds (synchronises). */
int ising_last_batch_ms(double* ms);

/*
 * Autotuner: time each launch candidate on a short trial anneal of the given
 * batch -- prefix_sweeps sweeps whose betas are taken evenly spaced from the
 * schedule -- then the three fastest again on max(5 prefix_sweeps, 4000)
 * sweeps (at most S), and return the fastest of those in *best (also cached in memory
 * and in the file named by $ISING_TUNE_CACHE when set).  prefix_sweeps <= 0
 * picks 200 (or S when smaller).  The trials' results are discarded: each
 * problem needs a new anneal before its results can be read.
 */
int ising_autotune(ising_problem* const* ps, int32_t count,
                   const ising_schedule* s, int32_t n_replicas,
                   int32_t prefix_sweeps, ising_tuning* best, void* stream);

/* ---------------------------------------------------------------- serving */
typedef struct ising_server ising_server;

typedef struct {
  int32_t status;          /* ISING_OK, or the error that ended the request */
  int32_t reached_target;  /* 1 when some replica reached target_cut */
  int32_t sweeps_done;
  int32_t best_replica;
  int64_t best_cut;
  double t_submit, t_admit, t_done; /* seconds on the server's clock */
} ising_result;

/*
 * Continuous-batching server.  Requests are admitted while the device bytes
 * they need (state, graph, tables) fit in hbm_budget and fewer than
 * max_slots are resident; all resident requests advance chunk_sweeps sweeps
 * per step in one persistent launch, finished ones retire and queued ones
 * are admitted between steps.  State stays on the device across steps.
 * backend: 0 = GPU; 1 = host-only null backend that advances sweep counters
 * without computing (to exercise the scheduling logic without a GPU); 2 = the
 * null backend that also fails, with ISING_ERR_DEVICE, every step in which a
 * request submitted with seed ISING_NULL_FAIL_SEED is resident (to exercise
 * the failure path).  A failed step ends every request resident in it with
 * that status, frees their memory and slots, and the server goes on with
 * the queue.
 */
#define ISING_NULL_FAIL_SEED 0xFA11FA11FA11FA11ull
int ising_server_create(uint64_t hbm_budget, int32_t max_slots,
                        int32_t chunk_sweeps, int32_t backend, void* stream,
                        ising_server** out);
/*
 * Queue one anneal of p (the problem must outlive the request).  It stops
 * early, after a multiple of check_every of its own sweeps, once a replica's
 * best cut reaches target_cut (check_every <= 0: never early).  A request
 * whose footprint exceeds the budget returns ISING_ERR_NOMEM.
 */
int ising_server_submit(ising_server* srv, ising_problem* p,
                        const ising_schedule* s, int32_t n_replicas,
                        uint64_t seed, int64_t target_cut, int32_t check_every,
                        uint64_t* ticket);
/* Wait for a request (timeout_s < 0: forever). */
int ising_server_wait(ising_server* srv, uint64_t ticket, double timeout_s,
                      ising_result* out);
/* Best state of a finished request's argmax replica, original order. */
int ising_server_best_state(ising_server* srv, uint64_t ticket, int8_t* spins);
/* Device bytes a request would need (the admission footprint). */
int ising_server_footprint(const ising_problem* p, const ising_schedule* s,
                           int32_t n_replicas, uint64_t* bytes);
/* Running totals: steps launched, requests finished, peak resident. */
int ising_server_stats(ising_server* srv, int64_t* steps, int64_t* finished,
                       int32_t* peak_resident);
int ising_server_destroy(ising_server* srv);

/*
 * Measurement helper for the roofline, not part of the method: issue rates
 * of the integer VALU instructions the anneal kernels are built from, on
 * the current device, in lane-operations per second, from independent
 * register-only chains at eight waves per SIMD.  rates[0..3] =
 * v_mad_u64_u32, v_mul_lo_u32, v_mul_hi_u32, v_xor_b32.  Synchronous; takes
 * a small temporary device buffer.  Errors: ISING_ERR_INVALID (rates NULL),
 * ISING_ERR_DEVICE.
 */
int ising_valu_rates(double* rates);
/*
 * Measurement helper for the roofline, not part of the method: LDS read
 * bandwidth of the current device in bytes per second, from conflict-free
 * 16-byte reads (ds_read_b128) of every lane, four 256-thread workgroups
 * per CU.  Synchronous; takes a small temporary device buffer.  Errors:
 * ISING_ERR_INVALID (bytes_per_s NULL), ISING_ERR_DEVICE.
 */
int ising_lds_rate(double* bytes_per_s);

#ifdef __cplusplus
}
#endif
#endif /* ISING_H */
