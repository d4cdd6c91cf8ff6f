/* A plain C11 program that drives libka through include/ka.h alone (no Python), for the tests:
 *   1. a periodic square lattice L = 8 (Sec. 2.1), 128 replicas, m = 2, rho = 0.5, seed 3,
 *      observed with ka_run at t = 0, 1, 3, 6, then its state and the Sec. 2.2 averages;
 *   2. a random regular graph N = 100, z = 3, graph seed 11, K = 40, m = 1, 64 replicas,
 *      seed 5: five sweeps with ka_sweep, then ka_observe and the state;
 *   3. one argument error (L = 6 is not a multiple of 4).
 * Every result goes to stdout as "key v0 v1 ..." lines; the test compares them with the
 * oracle.  Exit status 0 when every call that should succeed did. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "ka.h"

#define CHECK(call)                                                                   \
  do {                                                                                \
    const int rc_ = (call);                                                           \
    if (rc_ != KA_OK) {                                                               \
      fprintf(stderr, "%s failed: %d (%s)\n", #call, rc_, ka_last_error());           \
      return 1;                                                                       \
    }                                                                                 \
  } while (0)

static void print_i64(const char *key, int row, const int64_t *v, int n)
{
  printf("%s %d", key, row);
  for (int i = 0; i < n; ++i) printf(" %lld", (long long)v[i]);
  printf("\n");
}

static void print_u64(const char *key, const uint64_t *v, int64_t n)
{
  printf("%s", key);
  for (int64_t i = 0; i < n; ++i) printf(" %llu", (unsigned long long)v[i]);
  printf("\n");
}

static int lattice_run(void)
{
  enum { R = 128, W = R / 64, NOBS = 4 };
  ka_graph *g = NULL;
  ka_sim *s = NULL;
  CHECK(ka_graph_lattice(2, 8, &g));
  int64_t N = 0, E = 0, K = 0;
  int z = 0, C = 0;
  CHECK(ka_graph_info(g, &N, &z, &E, &C));
  printf("lattice_graph %lld %d %lld %d\n", (long long)N, z, (long long)E, C);
  CHECK(ka_init(g, 2, 0.5, 3, R, NULL, &s));
  CHECK(ka_sim_info(s, NULL, NULL, &K, NULL, NULL, NULL));
  printf("lattice_K %lld\n", (long long)K);
  const int64_t times[NOBS] = {0, 1, 3, 6};
  int64_t *dens = malloc(sizeof(int64_t) * NOBS * R);
  int64_t *ov = malloc(sizeof(int64_t) * NOBS * R);
  int64_t *pers = malloc(sizeof(int64_t) * NOBS * R);
  uint64_t *n = malloc(sizeof(uint64_t) * (size_t)(W * N));
  uint64_t *f = malloc(sizeof(uint64_t) * (size_t)(W * N));
  if (!dens || !ov || !pers || !n || !f) return 1;
  CHECK(ka_run(s, times, NOBS, dens, ov, pers));
  for (int q = 0; q < NOBS; ++q) {
    print_i64("lattice_density", q, dens + q * R, R);
    print_i64("lattice_overlap", q, ov + q * R, R);
    print_i64("lattice_persistence", q, pers + q * R, R);
  }
  int64_t t = -1;
  CHECK(ka_get_state(s, n, NULL, f, &t));
  printf("lattice_t %lld\n", (long long)t);
  print_u64("lattice_n", n, W * N);
  print_u64("lattice_f", f, W * N);
  double Cq[NOBS], chi4[NOBS], P[NOBS];
  CHECK(ka_derived(N, K, R, NOBS, ov, pers, Cq, chi4, P));
  for (int q = 0; q < NOBS; ++q) printf("lattice_derived %d %.17g %.17g %.17g\n", q, Cq[q], chi4[q], P[q]);
  ka_free(s);
  ka_graph_free(g);
  free(dens);
  free(ov);
  free(pers);
  free(n);
  free(f);
  return 0;
}

static int graph_run(void)
{
  enum { R = 64, NV = 100 };
  ka_graph *g = NULL;
  ka_sim *s = NULL;
  CHECK(ka_graph_rrg(NV, 3, 11, &g));
  CHECK(ka_init_k(g, 1, 40, 5, R, NULL, &s));
  CHECK(ka_sweep(s, 5));
  int64_t t = -1, dens[R], ov[R], pers[R];
  CHECK(ka_observe(s, &t, dens, ov, pers));
  printf("graph_t %lld\n", (long long)t);
  print_i64("graph_density", 0, dens, R);
  print_i64("graph_overlap", 0, ov, R);
  print_i64("graph_persistence", 0, pers, R);
  uint64_t n[NV];
  CHECK(ka_get_state(s, n, NULL, NULL, NULL));
  print_u64("graph_n", n, NV);
  ka_free(s);
  ka_graph_free(g);
  return 0;
}

int main(void)
{
  if (lattice_run() != 0) return 1;
  if (graph_run() != 0) return 1;
  ka_graph *g = NULL;
  const int rc = ka_graph_lattice(2, 6, &g);
  printf("error %d %s\n", rc, g == NULL ? "null" : "set");
  return rc == KA_EINVAL && g == NULL ? 0 : 1;
}
