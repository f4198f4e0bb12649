/*
 * Drives every entry point of the CPU oracle (oracle/vegas_oracle.c) over
 * small and edge-case shapes, so that a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer sees every code path: each integrand at its
 * dimension, one dimension with two bins, 64 dimensions, 4096 bins, event
 * indices across 2^32, refinement with empty bins and empty dimensions,
 * alpha = 0, the combination with a zero sigma, and rejected arguments.
 * Prints "ok" when every call returned what it should.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void vo_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]);
int vo_uniform_grid(int dim, int nb, double *edges);
void vo_map_dim(int nb, const double *e, uint32_t r, double *x, int *k, double *jac);
double vo_rambo4(double sqrt_s, const double *u, double *p);
double vo_integrand(int id, int dim, const double *par, int np, const double *x);
int vo_weights(int dim, int nb, const double *edges, int id, const double *par, int np,
               uint64_t seed, uint32_t t, uint64_t first, int64_t count, double *w_out);
int vo_points(int dim, int nb, const double *edges, uint64_t seed, uint32_t t, uint64_t first,
              int64_t count, double *x_out, int *k_out, double *jac_out);
int vo_iterate(int dim, int nb, const double *edges, int id, const double *par, int np,
               int64_t n_events, uint64_t seed, uint32_t t, double *I, double *sigma,
               double *hist_out, int64_t *n_nonfinite);
int vo_refine(int dim, int nb, const double *edges, const double *hist, double alpha,
              double *new_edges);
int vo_combine(int n, const double *I_t, const double *sigma_t, double *I, double *sigma,
               double *chi2_dof);
int vo_run(int dim, int nb, int id, const double *par, int np, int64_t n_events, uint64_t seed,
           int n_iter, double alpha, double *I_t, double *sigma_t, double *edges_out,
           int64_t *n_nonfinite);

static int failures = 0;
#define CHECK(c)                                                \
  do {                                                          \
    if (!(c)) {                                                 \
      fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      ++failures;                                               \
    }                                                           \
  } while (0)

static double *alloc(size_t n) {
  double *p = (double *)calloc(n ? n : 1, sizeof(double));
  if (!p) exit(2);
  return p;
}

/* iterate, then refine, on a shape; the grid must stay increasing */
static void iterate_refine(int dim, int nb, int id, const double *par, int np, int64_t n,
                           double alpha) {
  double *e = alloc((size_t)dim * (nb + 1)), *e2 = alloc((size_t)dim * (nb + 1));
  double *h = alloc((size_t)dim * nb);
  double I = 0, s = 0;
  int64_t bad = -1;
  CHECK(vo_uniform_grid(dim, nb, e) == 0);
  CHECK(vo_iterate(dim, nb, e, id, par, np, n, 7, 1, &I, &s, h, &bad) == 0);
  CHECK(isfinite(I) && s >= 0.0 && bad >= 0);
  CHECK(vo_refine(dim, nb, e, h, alpha, e2) == 0);
  for (int d = 0; d < dim; ++d)
    for (int i = 0; i < nb; ++i) CHECK(e2[(size_t)d * (nb + 1) + i + 1] > e2[(size_t)d * (nb + 1) + i]);
  free(e);
  free(e2);
  free(h);
}

int main(void) {
  uint32_t ctr[4] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu}, key[2] = {1, 2}, out[4];
  vo_philox4x32_10(ctr, key, out);

  double e1[3] = {0.0, 0.25, 1.0}, x, j;
  int k;
  vo_map_dim(2, e1, 0u, &x, &k, &j);
  CHECK(k == 0 && x > 0.0);
  vo_map_dim(2, e1, 0xFFFFFFFFu, &x, &k, &j);
  CHECK(k == 1 && x < 1.0);

  double u[16], p[16];
  for (int i = 0; i < 16; ++i) u[i] = (i + 0.5) / 16.0;
  CHECK(vo_rambo4(1000.0, u, p) > 0.0);

  /* every integrand at its dimension */
  const double gpar[1] = {0.1}, lpar[4] = {13000.0, 91.19, 2.5, 20.0}, rpar[3] = {1000.0, 0.01, 0.0},
               bpar[2] = {0.5, 0.02};
  iterate_refine(3, 7, 0, NULL, 0, 1000, 1.5);
  iterate_refine(10, 20, 1, NULL, 0, 1000, 1.5);
  iterate_refine(4, 50, 2, gpar, 1, 5000, 1.5);
  iterate_refine(4, 100, 3, lpar, 4, 5000, 1.5);
  iterate_refine(16, 50, 4, rpar, 3, 2000, 1.5);
  iterate_refine(2, 30, 5, bpar, 2, 3000, 0.5);
  /* edge shapes */
  iterate_refine(1, 2, 2, gpar, 1, 2, 1.5);
  iterate_refine(64, 3, 2, gpar, 1, 500, 1.5);
  iterate_refine(1, 4096, 2, gpar, 1, 20000, 1.5);
  iterate_refine(5, 9, 0, NULL, 0, 100, 0.0);

  /* weights and points across the 2^32 boundary of the event index */
  {
    double *e = alloc(3 * 11), *w = alloc(64), *xo = alloc(64 * 3), *jo = alloc(64);
    int *ko = (int *)calloc(64 * 3, sizeof(int));
    CHECK(vo_uniform_grid(3, 10, e) == 0);
    CHECK(vo_weights(3, 10, e, 2, gpar, 1, 5, 2, 0xFFFFFFE0ull, 64, w) == 0);
    CHECK(vo_points(3, 10, e, 5, 2, 0xFFFFFFE0ull, 64, xo, ko, jo) == 0);
    for (int i = 0; i < 64 * 3; ++i) CHECK(ko[i] >= 0 && ko[i] < 10);
    free(e); free(w); free(xo); free(jo); free(ko);
  }

  /* refinement: empty bins, an empty dimension, a single populated bin */
  {
    const int dim = 3, nb = 8;
    double *e = alloc(dim * (nb + 1)), *e2 = alloc(dim * (nb + 1)), *h = alloc(dim * nb);
    CHECK(vo_uniform_grid(dim, nb, e) == 0);
    for (int i = 0; i < nb; ++i) h[i] = (i % 3 == 0) ? 0.0 : 1.0 + i;
    /* dimension 1 stays empty */
    h[2 * nb + 5] = 4.0;
    CHECK(vo_refine(dim, nb, e, h, 1.5, e2) == 0);
    for (int i = 0; i <= nb; ++i) CHECK(e2[nb + 1 + i] == e[nb + 1 + i]);
    free(e); free(e2); free(h);
  }

  /* combination, including a zero sigma */
  {
    double It[3] = {1.0, 1.1, 0.9}, st[3] = {0.1, 0.2, 0.1}, I, s, c;
    CHECK(vo_combine(3, It, st, &I, &s, &c) == 0 && s > 0.0);
    st[1] = 0.0;
    CHECK(vo_combine(3, It, st, &I, &s, &c) == 0 && I == 1.1 && s == 0.0);
    CHECK(vo_combine(0, It, st, &I, &s, &c) != 0);
  }

  /* whole runs */
  {
    double It[4], st[4], *e = alloc(4 * 51);
    int64_t bad = -1;
    CHECK(vo_run(4, 50, 2, gpar, 1, 2000, 0, 4, 1.5, It, st, e, &bad) == 0 && bad == 0);
    CHECK(vo_run(4, 100, 3, lpar, 4, 2000, 0, 3, 1.5, It, st, NULL, NULL) == 0);
    free(e);
  }

  /* rejected arguments */
  {
    double e[3] = {0.0, 0.5, 1.0}, h[2] = {1.0, 1.0}, out3[3], I, s;
    CHECK(vo_uniform_grid(0, 4, NULL) != 0);
    CHECK(vo_uniform_grid(65, 4, NULL) != 0);
    CHECK(vo_iterate(1, 2, e, 2, gpar, 1, 1, 0, 0, &I, &s, NULL, NULL) != 0);
    CHECK(vo_iterate(1, 2, e, 3, lpar, 4, 10, 0, 0, &I, &s, NULL, NULL) != 0);
    CHECK(vo_iterate(1, 2, e, 9, NULL, 0, 10, 0, 0, &I, &s, NULL, NULL) != 0);
    CHECK(vo_refine(1, 2, e, h, -1.0, out3) != 0);
    CHECK(vo_run(1, 1, 2, gpar, 1, 10, 0, 1, 1.5, &I, &s, NULL, NULL) != 0);
  }

  if (failures) return 1;
  printf("ok\n");
  return 0;
}
