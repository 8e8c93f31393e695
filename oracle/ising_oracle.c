/*
 * ising_oracle.c -- plain CPU oracle (TEST INFRASTRUCTURE ONLY).
 *
 * Slow on purpose: one replica at a time, one vertex at a time, in the order
 * the method defines.  Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg may call it; the product path never links it.
 *
 * The paper defers the algorithm of its own solver to later work (Sec. I and
 * Sec. III.A), so what is written out here is the classical neighbour it
 * names (Sec. II.C: simulated annealing, replicas) in the form the HIP path
 * computes: many independent replicas, each doing single-spin-flip Metropolis
 * sweeps under an annealing schedule of inverse temperatures, visiting the
 * vertices colour class by colour class, with an incrementally maintained
 * local field.  Readings of everything the paper leaves open are listed in
 * the design notes of the repository; the ones that change numbers are
 * restated next to the code that applies them.
 *
 * Pins (tests/): Philox known-answer vectors; thresholds against a
 * 50-digit exp; colouring properness and the torus checkerboard; fields and
 * energy recomputed from scratch after every sweep; the cut identity; brute
 * force optima for n <= 20; beta = 0 and beta = infinity closed forms; planted
 * and gauge-transformed instances; a Boltzmann chi-square test.  Parallel
 * tempering (below): reductions to the anneal (one temperature, equal
 * temperatures), the odd-even transposition closed form, the exchange
 * test's acceptance frequency, and the stationary energy at every
 * temperature and exchange rate of every pair against exact enumeration.
 */
#include "ising_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw: "Parallel random numbers:  */
/* as easy as 1, 2, 3", SC'11).  Round: two 32x32->64 products of the    */
/* even counter words with fixed multipliers; the high halves are XORed  */
/* with the odd words and the key, the low halves move to the odd slots. */
/* The key is advanced by the Weyl constants between rounds.             */
/* ------------------------------------------------------------------ */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                          uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
    uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
    uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    uint32_t n1 = (uint32_t)p1;
    uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    uint32_t n3 = (uint32_t)p0;
    c0 = n0;
    c1 = n1;
    c2 = n2;
    c3 = n3;
    k0 += PHILOX_W0;
    k1 += PHILOX_W1;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

/* ------------------------------------------------------------------ */
/* Annealing schedule: inverse temperature beta_t for sweep t.           */
/* ------------------------------------------------------------------ */
static double beta_at(int32_t kind, int32_t S, double b0, double b1,
                      const double* betas, int32_t t) {
  if (kind == OR_EXPLICIT) return betas[t];
  if (S == 1) return b0;
  double frac = (double)t / (double)(S - 1);
  if (kind == OR_LINEAR) return b0 + (b1 - b0) * frac;
  return b0 * pow(b1 / b0, frac); /* OR_GEOMETRIC */
}

int oracle_schedule(int32_t kind, int32_t S, double b0, double b1,
                    const double* betas, double* out) {
  if (S <= 0) return -1;
  if (kind != OR_LINEAR && kind != OR_GEOMETRIC && kind != OR_EXPLICIT)
    return -1;
  if (kind == OR_EXPLICIT) {
    if (!betas) return -1;
  } else {
    if (!isfinite(b0) || !isfinite(b1) || b0 < 0 || b1 < 0) return -1;
    if (kind == OR_GEOMETRIC && (b0 <= 0 || b1 <= 0)) return -1;
  }
  for (int32_t t = 0; t < S; ++t) {
    double b = beta_at(kind, S, b0, b1, betas, t);
    if (!isfinite(b) || b < 0) return -1;
    if (out) out[t] = b;
  }
  return 0;
}

/* Metropolis acceptance of a move raising the energy by dE = 2k > 0 has
 * probability exp(-beta dE).  It is quantised to a 32-bit threshold so that
 * the decision is an integer compare of a uniform u32 against Tq. */
uint64_t oracle_threshold(double beta, int64_t k) {
  double x = -2.0 * (double)k;
  x = x * beta;
  double a = exp(x);
  if (a >= 1.0) return (uint64_t)1 << 32;
  return (uint64_t)floor(ldexp(a, 32));
}

/* ------------------------------------------------------------------ */
/* Graph handling                                                        */
/* ------------------------------------------------------------------ */
static int cmp_u64(const void* a, const void* b) {
  uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
  return (x > y) - (x < y);
}

int oracle_validate(const or_graph_in* g) {
  if (g->n <= 0 || g->m < 0) return -1;
  if (g->m > 0 && (!g->u || !g->v || !g->w)) return -1;
  int64_t total = 0;
  uint64_t* keys = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(g->m + 1));
  if (!keys) return -1;
  for (int64_t e = 0; e < g->m; ++e) {
    int32_t a = g->u[e], b = g->v[e], w = g->w[e];
    if (a < 0 || b < 0 || a >= g->n || b >= g->n || a == b || w == 0 ||
        w > 32768 || w < -32768) {
      free(keys);
      return -1;
    }
    total += 2 * (int64_t)(w < 0 ? -w : w);
    uint32_t lo = (uint32_t)(a < b ? a : b), hi = (uint32_t)(a < b ? b : a);
    keys[e] = ((uint64_t)lo << 32) | hi;
  }
  if (g->field)
    for (int32_t i = 0; i < g->n; ++i) {
      const int32_t b = g->field[i];
      if (b > 32768 || b < -32768) {
        free(keys);
        return -1;
      }
      total += 2 * (int64_t)(b < 0 ? -b : b);
    }
  if (total >= ((int64_t)1 << 30)) {
    free(keys);
    return -1;
  }
  qsort(keys, (size_t)g->m, sizeof(uint64_t), cmp_u64);
  for (int64_t e = 1; e < g->m; ++e)
    if (keys[e] == keys[e - 1]) {
      free(keys);
      return -1;
    }
  free(keys);
  if (g->colour) {
    for (int32_t i = 0; i < g->n; ++i)
      if (g->colour[i] < 0 || g->colour[i] >= 1024) return -1;
    for (int64_t e = 0; e < g->m; ++e)
      if (g->colour[g->u[e]] == g->colour[g->v[e]]) return -1;
  }
  return 0;
}

typedef struct {
  int32_t n;
  int64_t m;
  int32_t* row;  /* [n+1] */
  int32_t* nbr;  /* [2m] neighbour id */
  int32_t* wt;   /* [2m] MaxCut weight w of that edge */
  int32_t* bf;   /* [n] local fields b, or NULL */
  int32_t n_colours;
  int32_t* colour;       /* [n] */
  int32_t* class_start;  /* [C+1] into members */
  int32_t* members;      /* [n] vertices of each class, ascending id */
  int32_t* run;          /* [n] RNG counter word 1: ordinal of v's run */
  int32_t* rank;         /* [n] which Philox output word vertex v uses */
  int64_t W;
  int64_t kmax;          /* max_v sum_j |w_vj| */
} or_graph;

static void graph_free(or_graph* G) {
  free(G->bf);
  free(G->row);
  free(G->nbr);
  free(G->wt);
  free(G->colour);
  free(G->class_start);
  free(G->members);
  free(G->run);
  free(G->rank);
}

int32_t oracle_colouring(int32_t n, int64_t m, const int32_t* u,
                         const int32_t* v, int32_t* colour) {
  if (n <= 0 || m < 0) return -1;
  int32_t* deg = (int32_t*)calloc((size_t)n + 1, sizeof(int32_t));
  int32_t* nbr = (int32_t*)malloc(sizeof(int32_t) * (size_t)(2 * m + 1));
  for (int64_t e = 0; e < m; ++e) {
    if (u[e] < 0 || v[e] < 0 || u[e] >= n || v[e] >= n) {
      free(deg);
      free(nbr);
      return -1;
    }
    deg[u[e] + 1]++;
    deg[v[e] + 1]++;
  }
  for (int32_t i = 0; i < n; ++i) deg[i + 1] += deg[i];
  int32_t* fill = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  for (int32_t i = 0; i < n; ++i) fill[i] = deg[i];
  for (int64_t e = 0; e < m; ++e) {
    nbr[fill[u[e]]++] = v[e];
    nbr[fill[v[e]]++] = u[e];
  }
  /* First fit in index order: vertex i takes the smallest colour that no
   * already-coloured neighbour (id < i) holds. */
  int32_t* used = (int32_t*)malloc(sizeof(int32_t) * ((size_t)n + 2));
  for (int32_t i = 0; i < n + 2; ++i) used[i] = -1;
  int32_t C = 0;
  for (int32_t i = 0; i < n; ++i) {
    for (int32_t a = deg[i]; a < deg[i + 1]; ++a)
      if (nbr[a] < i) used[colour[nbr[a]]] = i;
    int32_t c = 0;
    while (used[c] == i) ++c;
    colour[i] = c;
    if (c + 1 > C) C = c + 1;
  }
  free(used);
  free(fill);
  free(nbr);
  free(deg);
  return C;
}

static int graph_build(const or_graph_in* in, or_graph* G) {
  memset(G, 0, sizeof(*G));
  if (oracle_validate(in) != 0) return -1;
  int32_t n = in->n;
  int64_t m = in->m;
  G->n = n;
  G->m = m;
  G->row = (int32_t*)calloc((size_t)n + 1, sizeof(int32_t));
  G->nbr = (int32_t*)malloc(sizeof(int32_t) * (size_t)(2 * m + 1));
  G->wt = (int32_t*)malloc(sizeof(int32_t) * (size_t)(2 * m + 1));
  for (int64_t e = 0; e < m; ++e) {
    G->row[in->u[e] + 1]++;
    G->row[in->v[e] + 1]++;
  }
  for (int32_t i = 0; i < n; ++i) G->row[i + 1] += G->row[i];
  int32_t* fill = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  for (int32_t i = 0; i < n; ++i) fill[i] = G->row[i];
  G->W = 0;
  for (int64_t e = 0; e < m; ++e) {
    int32_t a = in->u[e], b = in->v[e];
    G->nbr[fill[a]] = b;
    G->wt[fill[a]++] = in->w[e];
    G->nbr[fill[b]] = a;
    G->wt[fill[b]++] = in->w[e];
    G->W += in->w[e];
  }
  free(fill);
  if (in->field) {
    G->bf = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    memcpy(G->bf, in->field, sizeof(int32_t) * (size_t)n);
  }
  /* the largest |k|: sum of |w| plus 2 |b| */
  G->kmax = 0;
  for (int32_t i = 0; i < n; ++i) {
    int64_t s = G->bf ? 2 * (int64_t)(G->bf[i] < 0 ? -G->bf[i] : G->bf[i]) : 0;
    for (int32_t a = G->row[i]; a < G->row[i + 1]; ++a)
      s += G->wt[a] < 0 ? -G->wt[a] : G->wt[a];
    if (s > G->kmax) G->kmax = s;
  }
  G->colour = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  if (in->colour) {
    int32_t C = 0;
    for (int32_t i = 0; i < n; ++i) {
      G->colour[i] = in->colour[i];
      if (in->colour[i] + 1 > C) C = in->colour[i] + 1;
    }
    G->n_colours = C;
  } else {
    G->n_colours = oracle_colouring(n, m, in->u, in->v, G->colour);
  }
  int32_t C = G->n_colours;
  G->class_start = (int32_t*)calloc((size_t)C + 1, sizeof(int32_t));
  for (int32_t i = 0; i < n; ++i) G->class_start[G->colour[i] + 1]++;
  for (int32_t c = 0; c < C; ++c) G->class_start[c + 1] += G->class_start[c];
  G->members = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  G->run = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  G->rank = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  int32_t* pos = (int32_t*)malloc(sizeof(int32_t) * ((size_t)C + 1));
  for (int32_t c = 0; c <= C; ++c) pos[c] = G->class_start[c];
  for (int32_t i = 0; i < n; ++i) G->members[pos[G->colour[i]]++] = i;
  free(pos);
  /* Random-number groups: inside each colour class, taken in ascending id
   * order, consecutive runs of four vertices share one Philox block (the
   * last run of a class may be shorter).  Runs are numbered in class order,
   * then in id order within a class; the block's counter names the run by
   * that ordinal, and the i-th vertex of the run uses output word i. */
  int32_t runs_before = 0;
  for (int32_t c = 0; c < C; ++c) {
    for (int32_t idx = G->class_start[c]; idx < G->class_start[c + 1]; ++idx) {
      int32_t local = idx - G->class_start[c];
      int32_t vtx = G->members[idx];
      G->rank[vtx] = local % 4;
      G->run[vtx] = runs_before + local / 4;
    }
    runs_before += (G->class_start[c + 1] - G->class_start[c] + 3) / 4;
  }
  return 0;
}

/* u32 random number for (vertex, sweep, replica, purpose): word rank(v) of
 * Philox4x32-10 with key = seed and counter = (t, run(v), r, tag). */
static uint32_t draw(const or_graph* G, uint64_t seed, int32_t v, uint32_t t,
                     uint32_t r, uint32_t tag) {
  uint32_t ctr[4] = {t, (uint32_t)G->run[v], r, tag};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t out[4];
  oracle_philox4x32_10(ctr, key, out);
  return out[G->rank[v]];
}

int oracle_stream_map(const or_graph_in* gin, int32_t* run, int32_t* rank) {
  if (!gin || !run || !rank) return -1;
  or_graph G;
  if (graph_build(gin, &G) != 0) {
    graph_free(&G);
    return -1;
  }
  memcpy(run, G.run, sizeof(int32_t) * (size_t)G.n);
  memcpy(rank, G.rank, sizeof(int32_t) * (size_t)G.n);
  graph_free(&G);
  return 0;
}

int oracle_draws(const or_graph_in* gin, uint64_t seed, uint32_t t, uint32_t r,
                 uint32_t tag, uint32_t* out) {
  if (!gin || !out) return -1;
  or_graph G;
  if (graph_build(gin, &G) != 0) {
    graph_free(&G);
    return -1;
  }
  for (int32_t v = 0; v < G.n; ++v) out[v] = draw(&G, seed, v, t, r, tag);
  graph_free(&G);
  return 0;
}

int64_t oracle_cut(int32_t n, int64_t m, const int32_t* u, const int32_t* v,
                   const int32_t* w, const int8_t* s) {
  (void)n;
  int64_t cut = 0;
  for (int64_t e = 0; e < m; ++e)
    if (s[u[e]] != s[v[e]]) cut += w[e];
  return cut;
}

/* Local field h_i = sum_j J_ij s_j + 2 b_i = -sum_j w_ij s_j + 2 b_i, from
 * scratch. */
static void fields_from_scratch(const or_graph* G, const int8_t* s,
                                int64_t* h) {
  for (int32_t i = 0; i < G->n; ++i) {
    int64_t acc = G->bf ? 2 * (int64_t)G->bf[i] : 0;
    for (int32_t a = G->row[i]; a < G->row[i + 1]; ++a)
      acc -= (int64_t)G->wt[a] * s[G->nbr[a]];
    h[i] = acc;
  }
}

/* E(s) = sum_e w_e s_u s_v - 2 sum_v b_v s_v, from scratch (each edge seen
 * from both ends). */
static int64_t energy_from_scratch(const or_graph* G, const int8_t* s) {
  int64_t twice = 0;
  for (int32_t i = 0; i < G->n; ++i)
    for (int32_t a = G->row[i]; a < G->row[i + 1]; ++a)
      twice += (int64_t)G->wt[a] * s[i] * s[G->nbr[a]];
  int64_t lin = 0;
  if (G->bf)
    for (int32_t i = 0; i < G->n; ++i) lin += 2 * (int64_t)G->bf[i] * s[i];
  return twice / 2 - lin;
}

static uint64_t splitmix64(uint64_t* x) {
  uint64_t z = (*x += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* One sweep t of replica r: the colour classes in order, each class's
 * vertices in ascending id (or, with shuf, in a random order: inside a class
 * no two vertices are adjacent and every draw is keyed by its own vertex, so
 * the order cannot change the result).  tq[k] for k = 1..kmax holds the
 * sweep's thresholds.  Updates s, h, E and the counters. */
/* Measurement tallies of a sweep (all optional; they never change the
 * sweep): attempts whose acceptance a draw decides, and distinct
 * neighbours whose field a colour pass changed (touched_at[j] holds the
 * last pass that changed h_j). */
typedef struct {
  int64_t* tests;
  int64_t* touched;
  int64_t* touched_at;
} sweep_tally;

static void sweep_once(const or_graph* G, uint64_t seed, int32_t t, int32_t r,
                       const uint64_t* tq, int8_t* s, int64_t* h, int64_t* E,
                       int64_t* accepts, int64_t* draws, int32_t* drawn_at,
                       int32_t* order, uint64_t* shuf, const sweep_tally* tally) {
  for (int32_t c = 0; c < G->n_colours; ++c) {
    const int64_t pass = (int64_t)t * G->n_colours + c;
    const int32_t lo = G->class_start[c], hi = G->class_start[c + 1];
    for (int32_t idx = lo; idx < hi; ++idx) order[idx - lo] = G->members[idx];
    if (shuf) {
      for (int32_t a = hi - lo - 1; a > 0; --a) {
        int32_t b = (int32_t)(splitmix64(shuf) % (uint64_t)(a + 1));
        int32_t tmp = order[a];
        order[a] = order[b];
        order[b] = tmp;
      }
    }
    for (int32_t q = 0; q < hi - lo; ++q) {
      const int32_t i = order[q];
      const int64_t k = s[i] * h[i]; /* flipping s_i changes E by 2k */
      int accept;
      if (k <= 0) {
        accept = 1;
      } else {
        uint32_t u = draw(G, seed, i, (uint32_t)t, (uint32_t)r, 0);
        accept = (uint64_t)u < tq[k];
        /* bookkeeping only: the stream gives the four vertices of a run
         * the four words of one Philox block, so the arithmetic the
         * method needs is one block per (run, sweep) that draws at all;
         * a draw whose threshold is 0 or 2^32 decides nothing and is not
         * counted */
        if (tq[k] != 0 && tq[k] != ((uint64_t)1 << 32) && drawn_at[G->run[i]] != t) {
          drawn_at[G->run[i]] = t;
          ++*draws;
        }
        if (tally && tally->tests && tq[k] != 0 && tq[k] != ((uint64_t)1 << 32)) ++*tally->tests;
      }
      if (accept) {
        s[i] = (int8_t)-s[i];
        *E += 2 * k;
        ++*accepts;
        for (int32_t a = G->row[i]; a < G->row[i + 1]; ++a) {
          h[G->nbr[a]] -= 2 * (int64_t)G->wt[a] * s[i];
          if (tally && tally->touched && tally->touched_at[G->nbr[a]] != pass) {
            tally->touched_at[G->nbr[a]] = pass;
            ++*tally->touched;
          }
        }
      }
    }
  }
}

typedef struct {
  const or_graph* G;
  const or_run_in* run;
  or_run_out* out;
  const double* betas;
  int32_t first, stride; /* replicas first, first+stride, ... of the range */
  int64_t failures;
  int status;
} worker_arg;

static void run_replica(worker_arg* A, int32_t r, int8_t* s, int64_t* h,
                        int64_t* hchk, uint64_t* tq, int32_t* order,
                        int32_t* drawn_at) {
  const or_graph* G = A->G;
  const or_run_in* run = A->run;
  or_run_out* out = A->out;
  const int32_t n = G->n, S = run->n_sweeps;
  const int64_t slot = r - run->r_begin;
  const int64_t kmax = G->kmax;

  /* Initial state: given, or s_v = +1 iff bit 31 of draw(v, 0, r, tag 1). */
  for (int32_t i = 0; i < n; ++i) {
    if (run->init_spins)
      s[i] = run->init_spins[(int64_t)r * n + i];
    else
      s[i] = (draw(G, run->seed, i, 0, (uint32_t)r, 1) >> 31) ? 1 : -1;
  }
  fields_from_scratch(G, s, h);
  int64_t E = energy_from_scratch(G, s);
  int64_t best_cut = (G->W - E) / 2;
  int32_t best_sweep = -1;
  int64_t accepts = 0, draws = 0, improvements = 0, tests = 0, touched = 0;
  for (int32_t i = 0; i < n; ++i) drawn_at[i] = -1;
  sweep_tally tally = {NULL, NULL, NULL};
  int64_t* touched_at = NULL;
  if (out->tests || out->touched) {
    tally.tests = out->tests ? &tests : NULL;
    if (out->touched) {
      touched_at = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
      if (touched_at) {
        for (int32_t i = 0; i < n; ++i) touched_at[i] = -1;
        tally.touched = &touched;
        tally.touched_at = touched_at;
      }
    }
  }
  if (out->best_state) memcpy(out->best_state + slot * n, s, (size_t)n);
  uint64_t shuf = run->shuffle_seed ^ ((uint64_t)r * 0x632BE59BD9B4E019ull);

  for (int32_t t = 0; t < S; ++t) {
    const double beta = A->betas[t];
    for (int64_t k = 1; k <= kmax; ++k) tq[k] = oracle_threshold(beta, k);
    sweep_once(G, run->seed, t, r, tq, s, h, &E, &accepts, &draws, drawn_at, order,
               run->shuffle_seed ? &shuf : NULL, (out->tests || out->touched) ? &tally : NULL);
    /* End of sweep: the best is taken over end-of-sweep states only, strict
     * improvement, so the earliest sweep reaching a value keeps it. */
    int64_t cut = (G->W - E) / 2;
    if (cut > best_cut) {
      best_cut = cut;
      best_sweep = t;
      ++improvements;
      if (out->best_state) memcpy(out->best_state + slot * n, s, (size_t)n);
    }
    if (out->energy_trace) out->energy_trace[slot * S + t] = E;
    if (run->check_every_sweep) {
      fields_from_scratch(G, s, hchk);
      int bad = energy_from_scratch(G, s) != E;
      for (int32_t i = 0; i < n && !bad; ++i) bad = hchk[i] != h[i];
      if (bad) A->failures++;
    }
  }
  out->best_cut[slot] = best_cut;
  out->best_sweep[slot] = best_sweep;
  out->accepts[slot] = accepts;
  out->final_energy[slot] = E;
  if (out->draws) out->draws[slot] = draws;
  if (out->improvements) out->improvements[slot] = improvements;
  if (out->tests) out->tests[slot] = tests;
  if (out->touched) out->touched[slot] = touched;
  free(touched_at);
  if (out->final_state) memcpy(out->final_state + slot * n, s, (size_t)n);
  if (out->final_field)
    for (int32_t i = 0; i < n; ++i) out->final_field[slot * n + i] = (int32_t)h[i];
}

static void* worker(void* p) {
  worker_arg* A = (worker_arg*)p;
  const int32_t n = A->G->n;
  int8_t* s = (int8_t*)malloc((size_t)n);
  int64_t* h = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  int64_t* hchk = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  uint64_t* tq = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(A->G->kmax + 1));
  int32_t* order = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  int32_t* drawn_at = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  if (!s || !h || !hchk || !tq || !order || !drawn_at) {
    A->status = -1;
  } else {
    for (int32_t r = A->run->r_begin + A->first; r < A->run->r_end; r += A->stride)
      run_replica(A, r, s, h, hchk, tq, order, drawn_at);
  }
  free(drawn_at);
  free(s);
  free(h);
  free(hchk);
  free(tq);
  free(order);
  return NULL;
}

int oracle_anneal(const or_graph_in* gin, const or_run_in* run,
                  or_run_out* out) {
  if (!gin || !run || !out) return -1;
  if (run->n_replicas <= 0 || run->r_begin < 0 || run->r_end > run->n_replicas ||
      run->r_begin >= run->r_end)
    return -1;
  double* betas = (double*)malloc(sizeof(double) * (size_t)(run->n_sweeps > 0 ? run->n_sweeps : 1));
  if (oracle_schedule(run->kind, run->n_sweeps, run->beta0, run->beta1,
                      run->betas, betas) != 0) {
    free(betas);
    return -1;
  }
  or_graph G;
  if (graph_build(gin, &G) != 0) {
    free(betas);
    graph_free(&G);
    return -1;
  }
  int32_t nt = run->n_threads < 1 ? 1 : run->n_threads;
  int32_t nr = run->r_end - run->r_begin;
  if (nt > nr) nt = nr;
  worker_arg* args = (worker_arg*)calloc((size_t)nt, sizeof(worker_arg));
  pthread_t* th = (pthread_t*)calloc((size_t)nt, sizeof(pthread_t));
  for (int32_t i = 0; i < nt; ++i) {
    args[i].G = &G;
    args[i].run = run;
    args[i].out = out;
    args[i].betas = betas;
    args[i].first = i;
    args[i].stride = nt;
  }
  if (nt == 1) {
    worker(&args[0]);
  } else {
    for (int32_t i = 0; i < nt; ++i) pthread_create(&th[i], NULL, worker, &args[i]);
    for (int32_t i = 0; i < nt; ++i) pthread_join(th[i], NULL);
  }
  int status = 0;
  out->check_failures = 0;
  for (int32_t i = 0; i < nt; ++i) {
    out->check_failures += args[i].failures;
    if (args[i].status) status = -1;
  }
  free(args);
  free(th);
  free(betas);
  graph_free(&G);
  return status;
}

/* ------------------------------------------------------------------ */
/* Parallel tempering                                                    */
/* ------------------------------------------------------------------ */
/* Exchanging the temperatures of a (at beta_k) and b (at beta_k1 >= beta_k)
 * has Metropolis ratio exp((beta_k1 - beta_k)(E_b - E_a)) on the product of
 * Boltzmann weights exp(-beta E).  The energies differ by an even number
 * (every state's E has the parity of sum_e w_e), so with q = (E_a - E_b)/2
 * the ratio is exp(-2 q dbeta): at least 1 when q <= 0, else the same
 * quantised threshold as a flip of "k = q" at inverse temperature dbeta. */
int oracle_swap_accept(uint64_t seed, uint32_t m, uint32_t k, uint32_t set,
                       int64_t Ea, int64_t Eb, double beta_k, double beta_k1) {
  const int64_t q = (Ea - Eb) / 2;
  if (q <= 0) return 1;
  const double dbeta = beta_k1 - beta_k;
  uint32_t ctr[4] = {m, k, set, 3};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t x[4];
  oracle_philox4x32_10(ctr, key, x);
  return (uint64_t)x[0] < oracle_threshold(dbeta, q);
}

/* Houdayer cluster move (a replica cluster move of the kind the paper
 * names beside parallel tempering, Sec. II.C): two replicas a and b at the
 * same temperature disagree on the sites D = {v : s_a(v) != s_b(v)}.  The
 * connected component of a seed site in the subgraph of the problem graph
 * induced by D is flipped in both replicas.  Along the cluster's boundary
 * every edge ends in a site where the two replicas agree, so the boundary
 * terms of E_a + E_b cancel before and after the flip, and interior edges
 * keep their terms: E_a + E_b is unchanged, and the move (a symmetric
 * proposal) is always accepted. */
static int64_t cluster_bfs(const or_graph* G, const int8_t* sa, const int8_t* sb, int32_t i0,
                           uint8_t* mark, int32_t* queue) {
  if (sa[i0] == sb[i0]) return 0;
  int64_t head = 0, tail = 0;
  queue[tail++] = i0;
  mark[i0] = 1;
  while (head < tail) {
    const int32_t v = queue[head++];
    for (int32_t a = G->row[v]; a < G->row[v + 1]; ++a) {
      const int32_t u = G->nbr[a];
      if (!mark[u] && sa[u] != sb[u]) {
        mark[u] = 1;
        queue[tail++] = u;
      }
    }
  }
  return tail;
}

int64_t oracle_cluster(const or_graph_in* gin, const int8_t* sa, const int8_t* sb, int32_t i0,
                       uint8_t* in_cluster) {
  if (!gin || !sa || !sb || !in_cluster) return -1;
  or_graph G;
  if (graph_build(gin, &G) != 0) {
    graph_free(&G);
    return -1;
  }
  if (i0 < 0 || i0 >= G.n) {
    graph_free(&G);
    return -1;
  }
  int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (size_t)G.n);
  memset(in_cluster, 0, (size_t)G.n);
  const int64_t size = cluster_bfs(&G, sa, sb, i0, in_cluster, queue);
  free(queue);
  graph_free(&G);
  return size;
}

/* One move on the replica pair (sa, sb) at temperature k of pair p in
 * round m: the seed is the (u mod |D|)-th site of D in ascending id, u word
 * 0 of Philox(counter (m, k, p, 4)).  Returns the cluster size (0 when the
 * replicas agree everywhere: no move).  Fields and energies are recomputed
 * from scratch. */
static int64_t houdayer_move(const or_graph* G, uint64_t seed, uint32_t m, uint32_t k, uint32_t p,
                             int8_t* sa, int8_t* sb, int64_t* ha, int64_t* hb, int64_t* Ea,
                             int64_t* Eb, uint8_t* mark, int32_t* queue, int64_t* failures) {
  const int32_t n = G->n;
  int64_t count = 0;
  for (int32_t v = 0; v < n; ++v) count += sa[v] != sb[v];
  if (count == 0) return 0;
  uint32_t ctr[4] = {m, k, p, 4};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t x[4];
  oracle_philox4x32_10(ctr, key, x);
  int64_t j = (int64_t)((uint64_t)x[0] % (uint64_t)count);
  int32_t i0 = 0;
  for (int32_t v = 0; v < n; ++v)
    if (sa[v] != sb[v] && j-- == 0) {
      i0 = v;
      break;
    }
  const int64_t size = cluster_bfs(G, sa, sb, i0, mark, queue);
  for (int32_t v = 0; v < n; ++v)
    if (mark[v]) {
      sa[v] = (int8_t)-sa[v];
      sb[v] = (int8_t)-sb[v];
      mark[v] = 0;
    }
  const int64_t before = *Ea + *Eb;
  fields_from_scratch(G, sa, ha);
  fields_from_scratch(G, sb, hb);
  *Ea = energy_from_scratch(G, sa);
  *Eb = energy_from_scratch(G, sb);
  if (*Ea + *Eb != before) ++*failures;  /* the move keeps E_a + E_b */
  return size;
}

typedef struct {
  const or_graph* G;
  const or_temper_in* pt;
  or_temper_out* out;
  int32_t first, stride; /* groups first, first+stride, ... below end */
  int32_t end;
  int32_t per_group;     /* sets per group: 2 with cluster moves, else 1 */
  int64_t failures;      /* cluster moves that changed E_a + E_b */
  int status;
} temper_arg;

typedef struct { /* scratch of one worker, for groups of up to gK replicas */
  int8_t* s;
  int64_t* h;
  uint64_t* tq;
  int32_t *order, *drawn_at, *best_sweep, *temp, *slot, *queue;
  int64_t *E, *best_cut, *accepts;
  uint8_t* mark;
} temper_scratch;

/* Sets set0 .. set0+ns-1 (ns = 1, or 2 for a cluster-move pair), replicas
 * j = 0 .. ns K - 1 of the group (global replica set0 K + j). */
static void temper_group(temper_arg* A, int32_t set0, int32_t ns, const temper_scratch* W) {
  const or_graph* G = A->G;
  const or_temper_in* pt = A->pt;
  or_temper_out* out = A->out;
  const int32_t n = G->n, K = pt->n_temps, S = pt->n_sweeps;
  const int32_t nr = ns * K;
  const int64_t kmax = G->kmax;
  const int64_t r0 = (int64_t)set0 * K;
  int8_t* s = W->s;
  int64_t *h = W->h, *E = W->E, *best_cut = W->best_cut, *accepts = W->accepts;
  int32_t *temp = W->temp, *slot = W->slot, *best_sweep = W->best_sweep;
  int64_t draws = 0;
  for (int32_t j = 0; j < nr; ++j) {
    const int64_t r = r0 + j;
    int8_t* sj = s + (int64_t)j * n;
    for (int32_t i = 0; i < n; ++i) {
      if (pt->init_spins)
        sj[i] = pt->init_spins[r * n + i];
      else
        sj[i] = (draw(G, pt->seed, i, 0, (uint32_t)r, 1) >> 31) ? 1 : -1;
    }
    fields_from_scratch(G, sj, h + (int64_t)j * n);
    E[j] = energy_from_scratch(G, sj);
    best_cut[j] = (G->W - E[j]) / 2;
    best_sweep[j] = -1;
    accepts[j] = 0;
    temp[j] = j % K;  /* slot[q K + k]: replica of set q of the group at k */
    slot[j] = j;
    if (out->best_state) memcpy(out->best_state + r * n, sj, (size_t)n);
  }
  for (int32_t k = 0; k < K; ++k)
    for (int64_t d = 1; d <= kmax; ++d) W->tq[(int64_t)k * (kmax + 1) + d] = oracle_threshold(pt->betas[k], d);
  for (int32_t t = 0; t < S; ++t) {
    for (int32_t j = 0; j < nr; ++j) {
      int8_t* sj = s + (int64_t)j * n;
      for (int32_t i = 0; i < n; ++i) W->drawn_at[i] = -1;
      sweep_once(G, pt->seed, t, (int32_t)(r0 + j), W->tq + (int64_t)temp[j] * (kmax + 1), sj,
                 h + (int64_t)j * n, &E[j], &accepts[j], &draws, W->drawn_at, W->order, NULL,
                 NULL);
      const int64_t cut = (G->W - E[j]) / 2;
      if (cut > best_cut[j]) {
        best_cut[j] = cut;
        best_sweep[j] = t;
        if (out->best_state) memcpy(out->best_state + (r0 + j) * n, sj, (size_t)n);
      }
    }
    if ((t + 1) % pt->swap_every == 0) {
      const int32_t m = (t + 1) / pt->swap_every - 1;
      /* cluster moves between the two sets of a pair, then the exchanges */
      if (pt->cluster_moves && ns == 2) {
        const int32_t pair = set0 / 2;
        for (int32_t k = pt->cluster_from; k < K; ++k) {
          const int32_t a = slot[k], b = slot[K + k];
          const int64_t size = houdayer_move(G, pt->seed, (uint32_t)m, (uint32_t)k, (uint32_t)pair,
                                             s + (int64_t)a * n, s + (int64_t)b * n, h + (int64_t)a * n,
                                             h + (int64_t)b * n, &E[a], &E[b], W->mark, W->queue,
                                             &A->failures);
          if (size > 0) {
            out->cluster_moves[(int64_t)pair * K + k]++;
            out->cluster_sites[(int64_t)pair * K + k] += size;
          }
        }
      }
      for (int32_t q = 0; q < ns; ++q) {
        int32_t* sl = slot + q * K;
        const int32_t set = set0 + q;
        for (int32_t k = m & 1; k + 1 < K; k += 2) {
          const int32_t a = sl[k], b = sl[k + 1];
          if (oracle_swap_accept(pt->seed, (uint32_t)m, (uint32_t)k, (uint32_t)set, E[a], E[b],
                                 pt->betas[k], pt->betas[k + 1])) {
            sl[k] = b;
            sl[k + 1] = a;
            temp[a] = k + 1;
            temp[b] = k;
            out->swaps[(int64_t)set * (K - 1) + k]++;
          }
        }
      }
    }
    if (out->temp_energy)
      for (int32_t q = 0; q < ns; ++q)
        for (int32_t k = 0; k < K; ++k)
          out->temp_energy[((int64_t)(set0 + q) * S + t) * K + k] = E[slot[q * K + k]];
  }
  for (int32_t j = 0; j < nr; ++j) {
    const int64_t r = r0 + j;
    out->best_cut[r] = best_cut[j];
    out->best_sweep[r] = best_sweep[j];
    out->accepts[r] = accepts[j];
    out->final_energy[r] = E[j];
    out->final_temp[r] = temp[j];
    if (out->final_state) memcpy(out->final_state + r * n, s + (int64_t)j * n, (size_t)n);
  }
}

static void* temper_worker(void* p) {
  temper_arg* A = (temper_arg*)p;
  const int32_t n = A->G->n, K = A->pt->n_temps, g = A->per_group;
  const int64_t kmax = A->G->kmax;
  const size_t nr = (size_t)g * (size_t)K;
  temper_scratch W;
  W.s = (int8_t*)malloc(nr * (size_t)n);
  W.h = (int64_t*)malloc(sizeof(int64_t) * nr * (size_t)n);
  W.tq = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)K * (size_t)(kmax + 1));
  W.order = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  W.drawn_at = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  W.queue = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  W.mark = (uint8_t*)calloc((size_t)n, 1);
  W.E = (int64_t*)malloc(sizeof(int64_t) * nr);
  W.best_cut = (int64_t*)malloc(sizeof(int64_t) * nr);
  W.accepts = (int64_t*)malloc(sizeof(int64_t) * nr);
  W.best_sweep = (int32_t*)malloc(sizeof(int32_t) * nr);
  W.temp = (int32_t*)malloc(sizeof(int32_t) * nr);
  W.slot = (int32_t*)malloc(sizeof(int32_t) * nr);
  if (!W.s || !W.h || !W.tq || !W.order || !W.drawn_at || !W.queue || !W.mark || !W.E ||
      !W.best_cut || !W.accepts || !W.best_sweep || !W.temp || !W.slot) {
    A->status = -1;
  } else {
    for (int32_t grp = A->first; grp < A->end; grp += A->stride) {
      const int32_t set0 = grp * g;
      const int32_t ns = set0 + g <= A->pt->n_sets ? g : A->pt->n_sets - set0;
      temper_group(A, set0, ns, &W);
    }
  }
  free(W.s);
  free(W.h);
  free(W.tq);
  free(W.order);
  free(W.drawn_at);
  free(W.queue);
  free(W.mark);
  free(W.E);
  free(W.best_cut);
  free(W.accepts);
  free(W.best_sweep);
  free(W.temp);
  free(W.slot);
  return NULL;
}

int oracle_temper(const or_graph_in* gin, const or_temper_in* pt, or_temper_out* out) {
  if (!gin || !pt || !out || !out->best_cut || !out->best_sweep || !out->accepts ||
      !out->final_energy || !out->final_temp || !out->swaps)
    return -1;
  if (pt->n_temps < 1 || pt->n_sets < 1 || pt->n_sweeps < 1 || pt->swap_every < 1 || !pt->betas)
    return -1;
  if ((int64_t)pt->n_temps * pt->n_sets > 0x7FFFFFFF) return -1;
  for (int32_t k = 0; k < pt->n_temps; ++k) {
    if (!isfinite(pt->betas[k]) || pt->betas[k] < 0) return -1;
    if (k > 0 && pt->betas[k] < pt->betas[k - 1]) return -1;
  }
  const int32_t g = pt->cluster_moves ? 2 : 1;
  /* cluster moves rely on spin-reversal symmetry, which fields break */
  if (pt->cluster_moves && gin->field) return -1;
  if (pt->cluster_moves &&
      (pt->cluster_from < 0 || pt->cluster_from > pt->n_temps || !out->cluster_moves ||
       !out->cluster_sites))
    return -1;
  int32_t s0 = pt->set_begin, s1 = pt->set_end;
  if (s0 == 0 && s1 == 0) s1 = pt->n_sets;
  if (s0 < 0 || s1 > pt->n_sets || s0 >= s1) return -1;
  /* a cluster-move pair is simulated whole */
  if (g == 2 && (s0 % 2 != 0 || (s1 % 2 != 0 && s1 != pt->n_sets))) return -1;
  or_graph G;
  if (graph_build(gin, &G) != 0) {
    graph_free(&G);
    return -1;
  }
  memset(out->swaps, 0, sizeof(int64_t) * (size_t)pt->n_sets * (size_t)(pt->n_temps - 1));
  if (pt->cluster_moves) {
    const size_t np = (size_t)(pt->n_sets / 2) * (size_t)pt->n_temps;
    memset(out->cluster_moves, 0, sizeof(int64_t) * np);
    memset(out->cluster_sites, 0, sizeof(int64_t) * np);
  }
  const int32_t g0 = s0 / g, g1 = (s1 + g - 1) / g;
  int32_t nt = pt->n_threads < 1 ? 1 : pt->n_threads;
  if (nt > g1 - g0) nt = g1 - g0;
  temper_arg* args = (temper_arg*)calloc((size_t)nt, sizeof(temper_arg));
  pthread_t* th = (pthread_t*)calloc((size_t)nt, sizeof(pthread_t));
  for (int32_t i = 0; i < nt; ++i) {
    args[i].G = &G;
    args[i].pt = pt;
    args[i].out = out;
    args[i].first = g0 + i;
    args[i].stride = nt;
    args[i].end = g1;
    args[i].per_group = g;
  }
  if (nt == 1) {
    temper_worker(&args[0]);
  } else {
    for (int32_t i = 0; i < nt; ++i) pthread_create(&th[i], NULL, temper_worker, &args[i]);
    for (int32_t i = 0; i < nt; ++i) pthread_join(th[i], NULL);
  }
  int status = 0;
  out->check_failures = 0;
  for (int32_t i = 0; i < nt; ++i) {
    if (args[i].status) status = -1;
    out->check_failures += args[i].failures;
  }
  free(args);
  free(th);
  graph_free(&G);
  return status;
}
