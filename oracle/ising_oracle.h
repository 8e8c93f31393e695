/*
 * ising_oracle.h -- plain CPU oracle for many-replica single-spin-flip
 * Metropolis annealing of sparse Ising / MaxCut problems.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, obviously correct
 * definition against which the HIP path is checked.  It shares no code with
 * the HIP library and must never be called by the product path; only the
 * tests, the smoke check and the CPU-baseline leg of the benchmark use it.
 *
 * Problem statement (paper Sec. II.A): weighted MaxCut on n variables with
 * integer edge weights w; the paper poses its toroidal +-1 spin glasses
 * (2D Edwards-Anderson) as weighted MaxCut instances.  Reading used here: the
 * Ising couplings are J = -w, so with s in {-1,+1}^n
 *     E(s)   = sum_e w_e s_u s_v,      cut(s) = sum_e w_e (1 - s_u s_v)/2
 *     cut(s) = (W - E(s)) / 2  with W = sum_e w_e.
 * Work is counted in sweeps (paper Sec. III.A); one sweep here visits every
 * vertex once, colour class by colour class.
 *
 * Local fields (the paper notes that some sparse Ising problems have them,
 * Sec. II.C): with integer b_v,
 *     E(s) = sum_e w_e s_u s_v - 2 sum_v b_v s_v,
 *     h_v  = -sum_u w_vu s_u + 2 b_v,       k = s_v h_v as before,
 * and the reported objective (W - E)/2 becomes cut(s) + sum_v b_v s_v, still
 * an integer.  |b_v| <= 32768 and sum_v (sum_u |w_vu| + 2 |b_v|) < 2^30.
 */
#ifndef ISING_ORACLE_H
#define ISING_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_LINEAR = 0, OR_GEOMETRIC = 1, OR_EXPLICIT = 2 };

typedef struct {
  int32_t n;
  int64_t m;
  const int32_t* u;
  const int32_t* v;
  const int32_t* w;
  const int32_t* colour; /* NULL: greedy first-fit colouring in index order */
  const int32_t* field;  /* NULL, or [n] local fields b (see below) */
} or_graph_in;

typedef struct {
  int32_t kind;          /* OR_LINEAR / OR_GEOMETRIC / OR_EXPLICIT */
  int32_t n_sweeps;
  double beta0, beta1;
  const double* betas;   /* [n_sweeps] for OR_EXPLICIT */
  int32_t n_replicas;
  uint64_t seed;
  const int8_t* init_spins; /* NULL, or [n_replicas][n] +-1 */
  int32_t r_begin, r_end;   /* simulate replicas r_begin .. r_end-1 */
  int32_t n_threads;        /* host threads over replicas (>= 1) */
  int32_t check_every_sweep;/* recompute h and E from scratch each sweep */
  uint64_t shuffle_seed;    /* 0: ascending order inside a colour class */
} or_run_in;

typedef struct { /* per-replica arrays are indexed by r - r_begin */
  int64_t* best_cut;     /* [nr] */
  int32_t* best_sweep;   /* [nr]; -1 = the initial state */
  int64_t* accepts;      /* [nr] accepted flips */
  int64_t* final_energy; /* [nr] */
  int8_t* best_state;    /* [nr][n] or NULL */
  int8_t* final_state;   /* [nr][n] or NULL */
  int32_t* final_field;  /* [nr][n] or NULL */
  int64_t* energy_trace; /* [nr][n_sweeps] or NULL: E after every sweep */
  int64_t check_failures;/* sweeps where maintained h/E != recomputed */
  int64_t* draws;        /* [nr] or NULL: distinct Philox blocks the sweeps
                            needed, i.e. (t, run, r) with a draw */
  int64_t* improvements; /* [nr] or NULL: sweeps that raised the best cut */
  /* measurement tallies (test infrastructure; NULL = not counted): */
  int64_t* tests;        /* [nr] attempts whose acceptance a draw decided
                            (k > 0 and 0 < Tq < 2^32) */
  int64_t* touched;      /* [nr] distinct neighbours whose field a colour
                            pass changed, summed over passes */
} or_run_out;

/* Philox4x32-10 block function (Salmon et al., SC'11). */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                          uint32_t out[4]);
/* beta_t for t = 0 .. S-1.  Returns 0, or -1 on an invalid schedule. */
int oracle_schedule(int32_t kind, int32_t n_sweeps, double beta0, double beta1,
                    const double* betas, double* out);
/* Acceptance threshold Tq(beta, k) = floor(2^32 exp(-2 k beta)), 2^32 when
 * exp(...) >= 1.  Accept a flip with k > 0 iff u32 < Tq. */
uint64_t oracle_threshold(double beta, int64_t k);
/* Greedy first-fit colouring in index order; returns the number of colours
 * or -1 on invalid input. */
int32_t oracle_colouring(int32_t n, int64_t m, const int32_t* u,
                         const int32_t* v, int32_t* colour);
/* The random-number stream of a graph (its colouring as given, or greedy
 * first-fit): inside each colour class, taken in ascending id, consecutive
 * runs of four vertices (the class's last run may be shorter) are numbered
 * 0, 1, ... in class order, then in id order within a class.  run[v] is the
 * ordinal of v's run and rank[v] its place in the run, so v's draw for
 * sweep t, replica r and purpose tag (0 sweep, 1 initial state) is word
 * rank[v] of Philox4x32-10 with counter (t, run[v], r, tag) and key
 * (seed low, seed high).  A different colouring gives a different stream.
 * Returns 0, or -1 on invalid input. */
int oracle_stream_map(const or_graph_in* g, int32_t* run, int32_t* rank);
/* out[v] = that draw for every vertex v (t, r, tag fixed). */
int oracle_draws(const or_graph_in* g, uint64_t seed, uint32_t t, uint32_t r,
                 uint32_t tag, uint32_t* out);
/* MaxCut value of a +-1 assignment. */
int64_t oracle_cut(int32_t n, int64_t m, const int32_t* u, const int32_t* v,
                   const int32_t* w, const int8_t* spins);
/* Validate a problem the way the library does: 0 ok, -1 invalid. */
int oracle_validate(const or_graph_in* g);
/* Run the anneal.  Returns 0, or -1 on invalid input. */
int oracle_anneal(const or_graph_in* g, const or_run_in* run, or_run_out* out);

/*
 * Parallel tempering (replica exchange): the paper names it among the
 * contenders for sparse Ising optimisation (Sec. II.C): replicas simulated at
 * different temperatures exchange their temperatures.  Here a ladder of K
 * inverse temperatures betas[0] <= ... <= betas[K-1] is run by each of
 * n_sets independent sets of K replicas (R = n_sets K; replica r is in set
 * r / K and starts at temperature r % K).  Every sweep is the annealing
 * sweep above at the replica's current beta; after every swap_every-th
 * sweep, swap round m (m = 0, 1, ...) tries the pairs (k, k+1) with k of
 * the parity of m, in every set, as a Metropolis move on the product of the
 * K Boltzmann distributions:
 *     a = replica at k, b = replica at k+1, q = cut(b) - cut(a) = (E_a - E_b)/2
 *     exchange iff q <= 0, or u < Tq(betas[k+1] - betas[k], q)
 * with u word 0 of Philox(counter (m, k, set, 3), key seed) and Tq the
 * threshold function above (exp(-2 q dbeta) = exp(-dbeta (E_a - E_b))).
 * Best cuts and states are tracked per replica as in the anneal.
 */
typedef struct {
  int32_t n_temps;          /* K >= 1 */
  const double* betas;      /* [K], finite, >= 0, non-decreasing */
  int32_t n_sets;           /* >= 1 */
  int32_t n_sweeps;         /* S >= 1 */
  int32_t swap_every;       /* P >= 1 */
  uint64_t seed;
  const int8_t* init_spins; /* NULL, or [R][n] +-1 */
  int32_t n_threads;        /* host threads over sets (>= 1) */
  int32_t set_begin, set_end; /* simulate sets set_begin .. set_end-1 (both
                                 0: all); outputs stay indexed by replica */
  int32_t cluster_moves;    /* 1: Houdayer cluster moves (below) */
  int32_t cluster_from;     /* ... at temperatures k >= cluster_from */
} or_temper_in;

typedef struct {
  int64_t* best_cut;     /* [R] */
  int32_t* best_sweep;   /* [R]; -1 = the initial state */
  int64_t* accepts;      /* [R] accepted flips */
  int64_t* final_energy; /* [R] */
  int32_t* final_temp;   /* [R] temperature index at the end */
  int64_t* swaps;        /* [n_sets][K-1] accepted exchanges of pair (k, k+1) */
  int8_t* best_state;    /* [R][n] or NULL */
  int8_t* final_state;   /* [R][n] or NULL */
  int64_t* temp_energy;  /* [n_sets][S][K] or NULL: E of the replica at
                            temperature k after sweep t and its swap round */
  int64_t* cluster_moves; /* [n_sets/2][K] moves made (with cluster moves) */
  int64_t* cluster_sites; /* [n_sets/2][K] sites flipped, summed over moves */
  int64_t check_failures; /* cluster moves after which E_a + E_b differed */
} or_temper_out;

/*
 * Houdayer cluster moves (replica cluster moves, which the paper names as
 * combinable with parallel tempering, Sec. II.C).  With cluster_moves set,
 * sets 2p and 2p+1 form pair p (an odd last set has no partner).  At every
 * exchange point, before the exchange round m, each pair makes one move at
 * each temperature k >= cluster_from between its two replicas there: D is
 * the set of sites where they disagree; if D is empty there is no move;
 * else the seed is the (u mod |D|)-th site of D in ascending id, u word 0 of
 * Philox(counter (m, k, p, 4), key seed), and the connected component of
 * the seed in the subgraph induced by D is flipped in both replicas.  The
 * move keeps E_a + E_b and is always accepted.  A set range (set_begin,
 * set_end) must then keep pairs whole.
 */
/* The cluster of seed i0 (in_cluster[v] = 1 for its sites, [n]); returns
 * its size, 0 when the replicas agree at i0, -1 on invalid input. */
int64_t oracle_cluster(const or_graph_in* g, const int8_t* sa, const int8_t* sb, int32_t i0,
                       uint8_t* in_cluster);
/* Run parallel tempering.  Returns 0, or -1 on invalid input. */
int oracle_temper(const or_graph_in* g, const or_temper_in* pt, or_temper_out* out);
/* The exchange test of one pair: 1 = exchange.  Ea, Eb are the energies of
 * the replicas at betas[k] and betas[k+1]. */
int oracle_swap_accept(uint64_t seed, uint32_t m, uint32_t k, uint32_t set,
                       int64_t Ea, int64_t Eb, double beta_k, double beta_k1);

#ifdef __cplusplus
}
#endif
#endif
