/* Exercises every entry point of the FP64 oracle on small volumes (ragged
 * shapes, flat regions, general neighbourhoods, slabs, swarms, differences)
 * so that a build with the address and undefined-behaviour sanitizers sees
 * every loop of the oracle run.  Exit status 0: every call returned 0 and
 * produced finite values. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "pifcm_oracle.h"

static double lcg(uint64_t* s) {
  *s = *s * 6364136223846793005ull + 1442695040888963407ull;
  return (double)(*s >> 11) / 9007199254740992.0;
}

static int finite_all(const double* a, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!isfinite(a[i])) return 0;
  return 1;
}

#define CHECK(expr)                                                  \
  do {                                                               \
    if ((expr) != 0) {                                               \
      fprintf(stderr, "%s:%d: %s failed\n", __FILE__, __LINE__, #expr); \
      return 1;                                                      \
    }                                                                \
  } while (0)

static int one_case(int nx, int ny, int nz, int C, int V, int flags, double m, uint64_t seed) {
  const int64_t n = (int64_t)nx * ny * nz;
  float* raw = malloc(sizeof(float) * n);
  float* x = malloc(sizeof(float) * n);
  double* U = malloc(sizeof(double) * n * C);
  double* U1 = malloc(sizeof(double) * n * C);
  double* H = malloc(sizeof(double) * n * C);
  double* F = malloc(sizeof(double) * n * C);
  uint8_t* lab = malloc(n);
  uint64_t s = seed;
  for (int64_t i = 0; i < n; ++i) raw[i] = (i % 7 == 0) ? 0.5f : (float)lcg(&s);  /* some flat runs */
  CHECK(oracle_normalize(raw, n, x));
  or_params p = {C, V, 6, flags, m, 1.5, 1e-5};
  double c[16], c1[16], J = 0.0, Jh[8];
  for (int j = 0; j < C; ++j) c[j] = (j + 0.5) / C;
  CHECK(oracle_init_memberships(x, n, &p, c, U));
  CHECK(oracle_step(x, nx, ny, nz, &p, 0.3, 0.4, U, c, U1, c1, &J, H, F));
  if (!finite_all(U1, (size_t)n * C) || !isfinite(J)) return 1;
  int32_t it = 0;
  CHECK(oracle_solve(x, nx, ny, nz, &p, 0.6, 0.7, c, U, U1, c1, &J, &it, Jh));
  CHECK(oracle_solve(x, nx, ny, nz, &p, 0.2, 0.1, c, NULL, U1, c1, &J, &it, NULL));
  CHECK(oracle_solve_slab(x, nx, ny, nz, nz / 2, nz / 2 + 1, &p, 0.3, 0.2, c, U, U1, c1, &J, &it, Jh));
  CHECK(oracle_fcm_init(x, nx, ny, nz, &p, U1, c1, &it));
  CHECK(oracle_labels(U1, n, C, lab));
  enum { P = 3, G = 2 };
  double x0[P * 2], v0[P * 2], r1[G * P * 2], r2[G * P * 2];
  for (int i = 0; i < P * 2; ++i) {
    x0[i] = lcg(&s);
    v0[i] = 0.1 * (lcg(&s) - 0.5);
  }
  for (int i = 0; i < G * P * 2; ++i) {
    r1[i] = lcg(&s);
    r2[i] = lcg(&s);
  }
  double bp[2], bf, fh[G * P], ph[G * P * 2];
  CHECK(oracle_pso(x, nx, ny, nz, &p, c1, U1, P, G, x0, v0, r1, r2, 0.7, 1.5, 1.5, bp, &bf, fh, ph));
  CHECK(oracle_pso_interleaved(x, nx, ny, nz, &p, c1, U1, P, G, 2, x0, v0, r1, r2, 0.7, 1.5, 1.5, bp,
                               &bf, fh, ph, U, c));
  double grad[2 + 16];
  CHECK(oracle_fd_grad(x, nx, ny, nz, &p, 0.2, 0.3, c1, U1, 2, 1e-4, &J, grad));
  if (!finite_all(grad, (size_t)(2 + C)) || !finite_all(fh, G * P)) return 1;
  free(raw);
  free(x);
  free(U);
  free(U1);
  free(H);
  free(F);
  free(lab);
  return 0;
}

int main(void) {
  oracle_set_threads(2);
  const int shapes[][3] = {{1, 1, 1}, {2, 1, 3}, {5, 4, 3}, {7, 3, 9}, {4, 4, 2}};
  for (size_t k = 0; k < sizeof shapes / sizeof shapes[0]; ++k) {
    const int* d = shapes[k];
    if (one_case(d[0], d[1], d[2], 3, 1, 0, 2.0, 11 + k)) return 1;
    if (one_case(d[0], d[1], d[2], 4, 2, OR_Q2_SQDIST, 2.5, 23 + k)) return 1;
    if (one_case(d[0], d[1], d[2], 2, 5, OR_SHELL_SQDIST, 1.7, 37 + k)) return 1;
  }
  printf("oracle driver ok\n");
  return 0;
}
