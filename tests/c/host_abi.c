/* The C ABI used from plain C99: host-only entry points (problem compile,
 * cut evaluation, colouring, thresholds, errors).  No device work.  Prints
 * "ok" and exits 0 when every check holds. */
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "ising.h"

static int failures = 0;
#define CHECK(cond)                                              \
  do {                                                           \
    if (!(cond)) {                                               \
      fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #cond); \
      ++failures;                                                \
    }                                                            \
  } while (0)

int main(void) {
  /* a triangle with a two-edge tail: W = 9, vertex 2 has degree 3 and
   * sum |w| = 6 */
  const int32_t u[5] = {0, 1, 2, 2, 3}, v[5] = {1, 2, 0, 3, 4}, w[5] = {1, 2, 3, -1, 4};
  ising_problem* p = NULL;
  CHECK(ising_create(5, 5, u, v, w, NULL, &p) == ISING_OK && p != NULL);
  if (!p) return 1;

  ising_info info;
  CHECK(ising_problem_info(p, &info) == ISING_OK);
  CHECK(info.n == 5 && info.m == 5 && info.total_weight == 9);
  CHECK(info.max_degree == 3 && info.kmax == 6 && info.unit_weights == 0 && info.fields == 0);
  CHECK(info.n_padded % 4 == 0 && info.n_padded >= 5);

  int32_t colour[5];
  CHECK(ising_colouring(p, colour) == ISING_OK);
  for (int e = 0; e < 5; ++e) CHECK(colour[u[e]] != colour[v[e]]);

  /* the cut of every state against its definition, sum of w over the
   * edges whose ends differ */
  for (int x = 0; x < 32; ++x) {
    int8_t s[5];
    int64_t ref = 0, got = -1;
    for (int i = 0; i < 5; ++i) s[i] = (int8_t)(((x >> i) & 1) ? 1 : -1);
    for (int e = 0; e < 5; ++e) ref += s[u[e]] != s[v[e]] ? w[e] : 0;
    CHECK(ising_eval_cut(p, s, &got) == ISING_OK && got == ref);
  }
  CHECK(ising_destroy(p) == ISING_OK);
  CHECK(ising_destroy(NULL) == ISING_OK);

  /* rejected inputs leave the out-parameter untouched and explain why */
  const int32_t lu[1] = {1}, lv[1] = {1}, lw[1] = {1};
  ising_problem* q = (ising_problem*)&failures;
  CHECK(ising_create(2, 1, lu, lv, lw, NULL, &q) == ISING_ERR_INVALID);
  CHECK(q == (ising_problem*)&failures);
  CHECK(strlen(ising_last_error()) > 0);
  const int32_t du[2] = {0, 1}, dv[2] = {1, 0}, dw[2] = {1, 1};
  CHECK(ising_create(2, 2, du, dv, dw, NULL, &q) == ISING_ERR_INVALID);
  CHECK(strlen(ising_status_string(ISING_ERR_INVALID)) > 0);

  /* thresholds: beta = 0 always accepts; rows fall with k and with beta */
  ising_schedule sch;
  memset(&sch, 0, sizeof sch);
  sch.kind = 0; /* linear */
  sch.n_sweeps = 3;
  sch.beta0 = 0.0;
  sch.beta1 = 1.0;
  uint64_t tq[3 * 4];
  CHECK(ising_threshold_table(&sch, 4, tq) == ISING_OK);
  for (int k = 0; k < 4; ++k) CHECK(tq[k] == ((uint64_t)1 << 32));
  for (int t = 1; t < 3; ++t)
    for (int k = 0; k < 4; ++k) {
      CHECK(tq[t * 4 + k] < ((uint64_t)1 << 32));
      if (k > 0) CHECK(tq[t * 4 + k] <= tq[t * 4 + k - 1]);
      CHECK(tq[t * 4 + k] <= tq[(t - 1) * 4 + k]);
    }
  sch.n_sweeps = 0;
  CHECK(ising_threshold_table(&sch, 4, tq) == ISING_ERR_INVALID);

  if (failures) return 1;
  printf("ok\n");
  return 0;
}
