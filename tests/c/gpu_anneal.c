/* One anneal through the C ABI from plain C99 (NULL stream), checked
 * against the C oracle element by element: every replica's best cut, best
 * sweep, accepted flips and final energy, the argmax replica and its best
 * state.  Needs a GPU.  Prints "ok" and exits 0 when every check holds. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "ising.h"
#include "ising_oracle.h"

enum { LX = 12, LY = 10, N = LX * LY, M = 2 * N, R = 16, S = 300 };

int main(void) {
  /* +-1 torus from a small linear congruential sequence (an input recipe,
   * shared by both sides) */
  static int32_t u[M], v[M], w[M];
  uint32_t x = 12345u;
  for (int i = 0; i < N; ++i) {
    const int cx = i % LX, cy = i / LX;
    u[2 * i] = i;
    v[2 * i] = cy * LX + (cx + 1) % LX;
    u[2 * i + 1] = i;
    v[2 * i + 1] = ((cy + 1) % LY) * LX + cx;
    for (int e = 0; e < 2; ++e) {
      x = x * 1664525u + 1013904223u;
      w[2 * i + e] = (x >> 31) ? 1 : -1;
    }
  }
  const uint64_t seed = 77;

  ising_problem* p = NULL;
  if (ising_create(N, M, u, v, w, NULL, &p) != ISING_OK) {
    fprintf(stderr, "create: %s\n", ising_last_error());
    return 1;
  }
  ising_schedule sch;
  memset(&sch, 0, sizeof sch);
  sch.kind = 1; /* geometric */
  sch.n_sweeps = S;
  sch.beta0 = 0.1;
  sch.beta1 = 3.0;
  int64_t best = 0, per[R], acc[R], en[R];
  int32_t arg = -1, bs[R];
  static int8_t state[N];
  if (ising_anneal(p, &sch, R, seed, NULL) != ISING_OK ||
      ising_cut(p, &best, &arg, per) != ISING_OK ||
      ising_replica_results(p, bs, acc, en) != ISING_OK ||
      ising_best_state(p, state) != ISING_OK) {
    fprintf(stderr, "device run: %s\n", ising_last_error());
    return 1;
  }

  or_graph_in g = {N, M, u, v, w, NULL, NULL};
  or_run_in run;
  memset(&run, 0, sizeof run);
  run.kind = 1;
  run.n_sweeps = S;
  run.beta0 = 0.1;
  run.beta1 = 3.0;
  run.n_replicas = R;
  run.seed = seed;
  run.r_begin = 0;
  run.r_end = R;
  run.n_threads = 1;
  static int64_t obest[R], oacc[R], oen[R];
  static int32_t obs[R];
  static int8_t ostate[R][N];
  or_run_out out;
  memset(&out, 0, sizeof out);
  out.best_cut = obest;
  out.best_sweep = obs;
  out.accepts = oacc;
  out.final_energy = oen;
  out.best_state = &ostate[0][0];
  if (oracle_anneal(&g, &run, &out) != 0) {
    fprintf(stderr, "oracle failed\n");
    return 1;
  }

  int failures = 0, oarg = 0;
  for (int r = 0; r < R; ++r) {
    if (per[r] != obest[r] || bs[r] != obs[r] || acc[r] != oacc[r] || en[r] != oen[r]) {
      fprintf(stderr, "replica %d: device (%lld %d %lld %lld) oracle (%lld %d %lld %lld)\n", r,
              (long long)per[r], bs[r], (long long)acc[r], (long long)en[r], (long long)obest[r],
              obs[r], (long long)oacc[r], (long long)oen[r]);
      ++failures;
    }
    if (obest[r] > obest[oarg]) oarg = r;
  }
  if (arg != oarg || best != obest[oarg] || memcmp(state, ostate[oarg], N) != 0) {
    fprintf(stderr, "argmax: device %d (%lld), oracle %d (%lld)\n", arg, (long long)best, oarg,
            (long long)obest[oarg]);
    ++failures;
  }
  ising_destroy(p);
  if (failures) return 1;
  printf("ok\n");
  return 0;
}
