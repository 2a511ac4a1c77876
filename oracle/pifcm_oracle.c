/*
 * pifcm_oracle.c -- FP64 CPU reference of the 3DPIFCM IFCM iteration.
 *
 * TEST INFRASTRUCTURE ONLY (see pifcm_oracle.h): plain, slow, obviously
 * correct loops over the paper's equations in double precision.  OpenMP
 * splits the volume by z-plane; every reduction keeps one partial sum per
 * plane and adds the planes in order, so the result does not depend on the
 * number of threads.
 *
 * Readings of passages the paper leaves open (each one is applied below
 * where it matters):
 *   rings   -- the rings S_r of eqs (5), (7) are Chebyshev shells
 *              r = max(|dX|, |dY|, |dZ|) = 1..V; V = 1 is the 3x3x3 cube,
 *              which is eq (9) with the strict bound and L = 3.  With
 *              OR_SHELL_SQDIST the ring index is the squared distance
 *              dX^2 + dY^2 + dZ^2 = 1..V instead.
 *   q^2     -- eq (8) defines q as a squared distance and eq (7) squares it
 *              again; the literal reading weights a neighbour by q^2.  With
 *              OR_Q2_SQDIST the weight is q.
 *   borders -- only neighbours inside the volume count, in numerators and
 *              denominators alike (eq (9): x_k in I).
 *   sum g=0 -- when every neighbour of a ring has the intensity of the centre
 *              voxel, the ring's ratio in eq (5) is the plain mean of u_kj
 *              (the equal-weight limit); an empty ring contributes 0.
 *   floor   -- d^2 = max(|x - c|^2 (1 - lambda H - xi F), 1e-12) so eq (2)
 *              stays defined when the factor is <= 0 or x equals a centre.
 *   order   -- Jacobi: every H and F of a step reads the step's input U.
 *   J       -- a step reports J of its input state (U, c); eq (3) is applied
 *              as printed, weighted by u^m only.
 *   F power -- eq (7) squares u_kj (exponent 2, not m).
 *   stop    -- stop after iteration t >= 2 when |J(t-1) - J(t-2)| <=
 *              eps * |J(t-2)|; eps = 0 runs max_iter iterations.
 *   W       -- eq (10) is evaluated as exp(-(i-1)/h) / sum exp(-(r-1)/h),
 *              the same ratio with the common factor exp(-1/h) cancelled,
 *              so tiny h cannot underflow both terms to 0.
 */
#include "pifcm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_D_FLOOR 1e-12
#define OR_MAX_C 16
#define OR_MAX_RING 27

typedef struct {
  int dx, dy, dz;
  int ring; /* 1..V */
  double q2;
} or_offset;

int oracle_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

int oracle_get_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

static int params_ok(const or_params* p) {
  if (!p) return 0;
  if (p->C < 2 || p->C > OR_MAX_C) return 0;
  if (!(p->m > 1.0)) return 0;
  if (p->V < 1 || p->V > OR_MAX_RING - 1) return 0;
  if (!(p->h > 0.0)) return 0;
  if (p->max_iter < 0 || !(p->eps >= 0.0)) return 0;
  return 1;
}

/* Neighbourhood of eq (9) with ring indices (eqs (5), (7)) and the spatial
 * weight q^2 of eqs (7), (8).  Returns the number of offsets. */
static int build_offsets(const or_params* p, or_offset** out) {
  int reach = p->V;
  if (p->flags & OR_SHELL_SQDIST) {
    reach = 0;
    while ((reach + 1) * (reach + 1) <= p->V) reach++;
  }
  int side = 2 * reach + 1;
  or_offset* o = (or_offset*)malloc(sizeof(or_offset) * (size_t)side * side * side);
  int n = 0;
  for (int dz = -reach; dz <= reach; ++dz)
    for (int dy = -reach; dy <= reach; ++dy)
      for (int dx = -reach; dx <= reach; ++dx) {
        int s = dx * dx + dy * dy + dz * dz; /* eq (8): q = dX^2 + dY^2 + dZ^2 */
        if (s == 0) continue;                /* eq (9): 0 < distance          */
        int ring;
        if (p->flags & OR_SHELL_SQDIST) {
          if (s > p->V) continue;
          ring = s;
        } else {
          int ax = abs(dx), ay = abs(dy), az = abs(dz);
          ring = ax > ay ? ax : ay;
          ring = ring > az ? ring : az;
        }
        o[n].dx = dx;
        o[n].dy = dy;
        o[n].dz = dz;
        o[n].ring = ring;
        o[n].q2 = (p->flags & OR_Q2_SQDIST) ? (double)s : (double)s * (double)s;
        n++;
      }
  *out = o;
  return n;
}

/* eq (10): W_i = e^{-i/h} / sum_{r=1..V} e^{-r/h}. */
static void ring_weights(const or_params* p, double* W) {
  double total = 0.0;
  for (int r = 1; r <= p->V; ++r) total += exp(-(double)(r - 1) / p->h);
  W[0] = 0.0;
  for (int r = 1; r <= p->V; ++r) W[r] = exp(-(double)(r - 1) / p->h) / total;
}

/* eq (2) from squared distances: u_j = 1 / sum_k (d_j / d_k)^{2/(m-1)}. */
static void memberships_eq2(const double* d2, int C, double m, double* u) {
  double e = 1.0 / (m - 1.0);
  for (int j = 0; j < C; ++j) {
    double s = 0.0;
    for (int k = 0; k < C; ++k) s += pow(d2[j] / d2[k], e);
    u[j] = 1.0 / s;
  }
}

int oracle_normalize(const float* raw, int64_t n, float* out) {
  if (!raw || !out || n <= 0) return -1;
  double mn = 0.0, mx = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double v = (double)raw[i];
    if (!isfinite(v)) return -2;
    if (i == 0 || v < mn) mn = v;
    if (i == 0 || v > mx) mx = v;
  }
  for (int64_t i = 0; i < n; ++i) {
    if (mx == mn)
      out[i] = 0.0f;
    else
      out[i] = (float)(((double)raw[i] - mn) / (mx - mn));
  }
  return 0;
}

/* U^(0) when none is given: eq (2) with the attraction factor equal to 1,
 * i.e. plain FCM memberships of the initial centres. */
int oracle_init_memberships(const float* x, int64_t n, const or_params* p, const double* c,
                            double* U) {
  if (!params_ok(p) || !x || !c || !U) return -1;
  int C = p->C;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double d2[OR_MAX_C];
    for (int j = 0; j < C; ++j) {
      double e = ((double)x[i] - c[j]) * ((double)x[i] - c[j]);
      d2[j] = e > OR_D_FLOOR ? e : OR_D_FLOOR;
    }
    memberships_eq2(d2, C, p->m, U + i * C);
  }
  return 0;
}

/* One IFCM step (section 4, "step function"): from (U, c) compute H, F
 * (eqs (5)-(10)), the modified distances (eq (4)), J of the input state
 * (eq (1)), new memberships (eq (2)) and new centres (eq (3)). */
/* The step over the planes [zbeg, zend) only: memberships of the other
 * planes are copied unchanged to U_out (they act as fixed context), and the
 * centres and J are sums over the active planes (Algorithm 1, step 1:
 * segmenting one slice with its 3D neighbours). */
static int step_range(const float* x, int nx, int ny, int nz, int zbeg, int zend,
                      const or_params* p, double lambda, double xi, const double* U,
                      const double* c, double* U_out, double* c_out, double* J_out,
                      double* H_out, double* F_out) {
  if (!params_ok(p) || !x || !U || !c || nx < 1 || ny < 1 || nz < 1) return -1;
  if (zbeg < 0 || zend > nz || zbeg >= zend) return -1;
  const int C = p->C, V = p->V;
  const double m = p->m;
  or_offset* off = NULL;
  const int noff = build_offsets(p, &off);
  double W[OR_MAX_RING];
  ring_weights(p, W);
  const int stride = 2 * C + 1;
  double* parts = (double*)calloc((size_t)nz * stride, sizeof(double));

  if (U_out)
    for (int z = 0; z < nz; ++z)
      if (z < zbeg || z >= zend)
        memcpy(U_out + (size_t)z * ny * nx * C, U + (size_t)z * ny * nx * C,
               sizeof(double) * (size_t)ny * nx * C);
#pragma omp parallel for schedule(static)
  for (int z = zbeg; z < zend; ++z) {
    double* part = parts + (size_t)z * stride; /* num[C], den[C], J */
    double gs[OR_MAX_RING], qs[OR_MAX_RING];
    int cnt[OR_MAX_RING];
    double hn[OR_MAX_RING][OR_MAX_C], fn[OR_MAX_RING][OR_MAX_C], un[OR_MAX_RING][OR_MAX_C];
    double d2[OR_MAX_C], un_new[OR_MAX_C];
    for (int y = 0; y < ny; ++y) {
      for (int xx = 0; xx < nx; ++xx) {
        const int64_t i = ((int64_t)z * ny + y) * nx + xx;
        const double xv = (double)x[i];
        for (int r = 0; r <= V; ++r) {
          gs[r] = 0.0;
          qs[r] = 0.0;
          cnt[r] = 0;
          for (int j = 0; j < C; ++j) hn[r][j] = fn[r][j] = un[r][j] = 0.0;
        }
        /* Sums over each ring S_r of the in-volume neighbourhood (eq (9)). */
        for (int o = 0; o < noff; ++o) {
          const int X = xx + off[o].dx, Y = y + off[o].dy, Z = z + off[o].dz;
          if (X < 0 || X >= nx || Y < 0 || Y >= ny || Z < 0 || Z >= nz) continue;
          const int64_t k = ((int64_t)Z * ny + Y) * nx + X;
          const double g = fabs(xv - (double)x[k]); /* eq (6) */
          const int r = off[o].ring;
          gs[r] += g;
          qs[r] += off[o].q2;
          cnt[r] += 1;
          for (int j = 0; j < C; ++j) {
            const double u = U[k * C + j];
            hn[r][j] += u * g;              /* numerator of eq (5) */
            fn[r][j] += u * u * off[o].q2;  /* numerator of eq (7) */
            un[r][j] += u;
          }
        }
        double J = 0.0;
        for (int j = 0; j < C; ++j) {
          double H = 0.0, F = 0.0;
          for (int r = 1; r <= V; ++r) {
            if (cnt[r] == 0) continue; /* empty ring */
            const double hr = gs[r] > 0.0 ? hn[r][j] / gs[r] : un[r][j] / (double)cnt[r];
            const double fr = fn[r][j] / qs[r];
            H += W[r] * hr; /* eq (5) */
            F += W[r] * fr; /* eq (7) */
          }
          if (H_out) H_out[i * C + j] = H;
          if (F_out) F_out[i * C + j] = F;
          const double a = 1.0 - lambda * H - xi * F;           /* eq (4) */
          const double e = (xv - c[j]) * (xv - c[j]) * a;
          d2[j] = e > OR_D_FLOOR ? e : OR_D_FLOOR;
          J += pow(U[i * C + j], m) * d2[j]; /* eq (1), input state */
        }
        memberships_eq2(d2, C, m, un_new); /* eq (2) */
        for (int j = 0; j < C; ++j) {
          if (U_out) U_out[i * C + j] = un_new[j];
          const double w = pow(un_new[j], m);
          part[j] += w * xv; /* eq (3) numerator   */
          part[C + j] += w;  /* eq (3) denominator */
        }
        part[2 * C] += J;
      }
    }
  }

  double J = 0.0;
  double num[OR_MAX_C], den[OR_MAX_C];
  for (int j = 0; j < C; ++j) num[j] = den[j] = 0.0;
  for (int z = zbeg; z < zend; ++z) {
    const double* part = parts + (size_t)z * stride;
    for (int j = 0; j < C; ++j) {
      num[j] += part[j];
      den[j] += part[C + j];
    }
    J += part[2 * C];
  }
  if (c_out)
    for (int j = 0; j < C; ++j) c_out[j] = den[j] > 0.0 ? num[j] / den[j] : c[j];
  if (J_out) *J_out = J;
  free(parts);
  free(off);
  return 0;
}

int oracle_step(const float* x, int nx, int ny, int nz, const or_params* p, double lambda,
                double xi, const double* U, const double* c, double* U_out, double* c_out,
                double* J_out, double* H_out, double* F_out) {
  return step_range(x, nx, ny, nz, 0, nz, p, lambda, xi, U, c, U_out, c_out, J_out, H_out, F_out);
}

/* The IFCM solve of Algorithm 1 step 11 (and of every fitness evaluation of
 * steps 4-9): iterate the step until the relative change of J falls to eps
 * or max_iter is reached.  The fitness is J of the final state. */
static int solve_range(const float* x, int nx, int ny, int nz, int zbeg, int zend,
                       const or_params* p, double lambda, double xi, const double* c0,
                       const double* U0, double* U_out, double* c_out, double* J_fit,
                       int32_t* iters, double* J_hist) {
  if (!params_ok(p) || !x || !c0 || !U_out || !c_out) return -1;
  const int C = p->C;
  const int64_t n = (int64_t)nx * ny * nz;
  double* Ua = (double*)malloc(sizeof(double) * (size_t)n * C);
  double* Ub = (double*)malloc(sizeof(double) * (size_t)n * C);
  double ca[OR_MAX_C], cb[OR_MAX_C];
  if (U0)
    memcpy(Ua, U0, sizeof(double) * (size_t)n * C);
  else
    oracle_init_memberships(x, n, p, c0, Ua);
  memcpy(ca, c0, sizeof(double) * C);

  double Jprev2 = 0.0, Jprev1 = 0.0;
  int t = 0;
  for (t = 1; t <= p->max_iter; ++t) {
    double J = 0.0;
    int rc = step_range(x, nx, ny, nz, zbeg, zend, p, lambda, xi, Ua, ca, Ub, cb, &J, NULL, NULL);
    if (rc) {
      free(Ua);
      free(Ub);
      return rc;
    }
    if (J_hist) J_hist[t - 1] = J; /* J of state t-1 */
    double* tmp = Ua;
    Ua = Ub;
    Ub = tmp;
    memcpy(ca, cb, sizeof(double) * C);
    Jprev2 = Jprev1;
    Jprev1 = J;
    if (p->eps > 0.0 && t >= 2 && fabs(Jprev1 - Jprev2) <= p->eps * fabs(Jprev2)) break;
  }
  int T = t > p->max_iter ? p->max_iter : t;
  double Jf = 0.0;
  step_range(x, nx, ny, nz, zbeg, zend, p, lambda, xi, Ua, ca, NULL, NULL, &Jf, NULL, NULL);
  memcpy(U_out, Ua, sizeof(double) * (size_t)n * C);
  memcpy(c_out, ca, sizeof(double) * C);
  if (J_fit) *J_fit = Jf;
  if (iters) *iters = T;
  free(Ua);
  free(Ub);
  return 0;
}

int oracle_solve(const float* x, int nx, int ny, int nz, const or_params* p, double lambda,
                 double xi, const double* c0, const double* U0, double* U_out, double* c_out,
                 double* J_fit, int32_t* iters, double* J_hist) {
  return solve_range(x, nx, ny, nz, 0, nz, p, lambda, xi, c0, U0, U_out, c_out, J_fit, iters,
                     J_hist);
}

/* Slab mode: only the planes [zbeg, zend) are iterated; the memberships of
 * the other planes stay those of U0 (required) and serve as neighbours. */
int oracle_solve_slab(const float* x, int nx, int ny, int nz, int zbeg, int zend,
                      const or_params* p, double lambda, double xi, const double* c0,
                      const double* U0, double* U_out, double* c_out, double* J_fit,
                      int32_t* iters, double* J_hist) {
  if (!U0) return -1;
  return solve_range(x, nx, ny, nz, zbeg, zend, p, lambda, xi, c0, U0, U_out, c_out, J_fit, iters,
                     J_hist);
}

/* Initial centres and memberships (Algorithm 1 step 2): plain FCM from
 * evenly spaced centres c_j = (j + 1/2) / C, i.e. the IFCM solve with
 * lambda = xi = 0 and no U, then the centres sorted ascending (stable) with
 * the membership columns permuted alike.  The paper's Gaussian-mixture
 * seeding is not specified and is not reproduced. */
int oracle_fcm_init(const float* x, int nx, int ny, int nz, const or_params* p, double* U_out,
                    double* c_out, int32_t* iters) {
  if (!params_ok(p) || !x || !U_out || !c_out) return -1;
  const int C = p->C;
  const int64_t n = (int64_t)nx * ny * nz;
  double c0[OR_MAX_C] = {0}, c1[OR_MAX_C] = {0};
  for (int j = 0; j < C; ++j) c0[j] = ((double)j + 0.5) / (double)C;
  double* U = (double*)malloc(sizeof(double) * (size_t)n * C);
  int rc = oracle_solve(x, nx, ny, nz, p, 0.0, 0.0, c0, NULL, U, c1, NULL, iters, NULL);
  if (rc) {
    free(U);
    return rc;
  }
  int perm[OR_MAX_C];
  for (int j = 0; j < C; ++j) perm[j] = j;
  for (int a = 1; a < C; ++a) { /* stable insertion sort of the centres */
    int v = perm[a], b = a - 1;
    while (b >= 0 && c1[perm[b]] > c1[v]) {
      perm[b + 1] = perm[b];
      b--;
    }
    perm[b + 1] = v;
  }
  for (int j = 0; j < C; ++j) c_out[j] = c1[perm[j]];
  for (int64_t i = 0; i < n; ++i)
    for (int j = 0; j < C; ++j) U_out[i * C + j] = U[i * C + perm[j]];
  free(U);
  return 0;
}

/* Hard labels of the final memberships: argmax_j u_ij, ties to the lowest j. */
int oracle_labels(const double* U, int64_t n, int C, uint8_t* labels) {
  if (!U || !labels || C < 1 || C > 255) return -1;
  for (int64_t i = 0; i < n; ++i) {
    int best = 0;
    for (int j = 1; j < C; ++j)
      if (U[i * C + j] > U[i * C + best]) best = j;
    labels[i] = (uint8_t)best;
  }
  return 0;
}

/* Synchronous global-best particle swarm over (lambda, xi) in [0,1]^2
 * (Algorithm 1 steps 3-9).  The fitness of a particle is the J of an IFCM
 * solve from the shared initial state (c0, U0).  The paper's update has no
 * inertia or coefficients and names no neighbourhood topology; this uses
 * v <- w v + c1 r1 (pbest - x) + c2 r2 (gbest - x), x <- clip(x + v, 0, 1),
 * with r1, r2 drawn per particle and dimension by the caller, strict
 * improvement, ties of gbest to the lowest particle index, G generations. */
int oracle_pso(const float* x, int nx, int ny, int nz, const or_params* p, const double* c0,
               const double* U0, int P, int G, const double* x0, const double* v0,
               const double* r1, const double* r2, double w, double c1, double c2,
               double* best_pos, double* best_fit, double* fit_hist, double* pos_hist) {
  if (!params_ok(p) || P < 1 || G < 1 || !x0 || !v0 || !r1 || !r2) return -1;
  const int C = p->C;
  const int64_t n = (int64_t)nx * ny * nz;
  double* pos = (double*)malloc(sizeof(double) * P * 2);
  double* vel = (double*)malloc(sizeof(double) * P * 2);
  double* pb = (double*)malloc(sizeof(double) * P * 2);
  double* pbf = (double*)malloc(sizeof(double) * P);
  double* Ut = (double*)malloc(sizeof(double) * (size_t)n * C);
  double gb[2] = {0.0, 0.0}, gbf = 0.0;
  int have_g = 0;
  memcpy(pos, x0, sizeof(double) * P * 2);
  memcpy(vel, v0, sizeof(double) * P * 2);
  for (int g = 0; g < G; ++g) {
    for (int q = 0; q < P; ++q) {
      double ct[OR_MAX_C], f = 0.0;
      int32_t it = 0;
      oracle_solve(x, nx, ny, nz, p, pos[2 * q], pos[2 * q + 1], c0, U0, Ut, ct, &f, &it, NULL);
      if (fit_hist) fit_hist[(size_t)g * P + q] = f;
      if (pos_hist) {
        pos_hist[((size_t)g * P + q) * 2] = pos[2 * q];
        pos_hist[((size_t)g * P + q) * 2 + 1] = pos[2 * q + 1];
      }
      if (g == 0 || f < pbf[q]) { /* step 5 */
        pbf[q] = f;
        pb[2 * q] = pos[2 * q];
        pb[2 * q + 1] = pos[2 * q + 1];
      }
    }
    for (int q = 0; q < P; ++q) { /* step 6, star topology */
      if (!have_g || pbf[q] < gbf) {
        gbf = pbf[q];
        gb[0] = pb[2 * q];
        gb[1] = pb[2 * q + 1];
        have_g = 1;
      }
    }
    if (g + 1 == G) break;
    for (int q = 0; q < P; ++q) { /* steps 7-8 */
      for (int d = 0; d < 2; ++d) {
        const size_t s = ((size_t)g * P + q) * 2 + d;
        double v = w * vel[2 * q + d] + c1 * r1[s] * (pb[2 * q + d] - pos[2 * q + d]) +
                   c2 * r2[s] * (gb[d] - pos[2 * q + d]);
        double np = pos[2 * q + d] + v;
        vel[2 * q + d] = v;
        pos[2 * q + d] = np < 0.0 ? 0.0 : (np > 1.0 ? 1.0 : np);
      }
    }
  }
  if (best_pos) {
    best_pos[0] = gb[0];
    best_pos[1] = gb[1];
  }
  if (best_fit) *best_fit = gbf;
  free(pos);
  free(vel);
  free(pb);
  free(pbf);
  free(Ut);
  return 0;
}

/* The interleaved reading of the swarm schedule (Algorithm 2, step 11):
 * each particle keeps its own IFCM state (U, c), starting from (U0, c0);
 * in every generation it advances `steps` IFCM iterations at its current
 * (lambda, xi) and its fitness is J of the state it reaches; the swarm then
 * moves exactly as in oracle_pso.  U_best / c_best (optional) receive the
 * state of the particle holding the global best after the last
 * generation. */
int oracle_pso_interleaved(const float* x, int nx, int ny, int nz, const or_params* p,
                           const double* c0, const double* U0, int P, int G, int steps,
                           const double* x0, const double* v0, const double* r1, const double* r2,
                           double w, double c1, double c2, double* best_pos, double* best_fit,
                           double* fit_hist, double* pos_hist, double* U_best, double* c_best) {
  if (!params_ok(p) || P < 1 || G < 1 || steps < 1 || !x0 || !v0 || !r1 || !r2 || !U0 || !c0)
    return -1;
  const int C = p->C;
  const int64_t n = (int64_t)nx * ny * nz;
  or_params q = *p;
  q.eps = 0.0;
  q.max_iter = steps;
  double* U = (double*)malloc(sizeof(double) * (size_t)P * n * C); /* state of each particle */
  double* cs = (double*)malloc(sizeof(double) * (size_t)P * C);
  double* Ut = (double*)malloc(sizeof(double) * (size_t)n * C);
  double* pos = (double*)malloc(sizeof(double) * P * 2);
  double* vel = (double*)malloc(sizeof(double) * P * 2);
  double* pb = (double*)malloc(sizeof(double) * P * 2);
  double* pbf = (double*)malloc(sizeof(double) * P);
  double gb[2] = {0.0, 0.0}, gbf = 0.0;
  int gq = 0;
  for (int k = 0; k < P; ++k) {
    memcpy(U + (size_t)k * n * C, U0, sizeof(double) * (size_t)n * C);
    memcpy(cs + (size_t)k * C, c0, sizeof(double) * C);
  }
  memcpy(pos, x0, sizeof(double) * P * 2);
  memcpy(vel, v0, sizeof(double) * P * 2);
  for (int g = 0; g < G; ++g) {
    for (int k = 0; k < P; ++k) {
      double ct[OR_MAX_C], f = 0.0;
      int32_t it = 0;
      oracle_solve(x, nx, ny, nz, &q, pos[2 * k], pos[2 * k + 1], cs + (size_t)k * C,
                   U + (size_t)k * n * C, Ut, ct, &f, &it, NULL);
      memcpy(U + (size_t)k * n * C, Ut, sizeof(double) * (size_t)n * C);
      memcpy(cs + (size_t)k * C, ct, sizeof(double) * C);
      if (fit_hist) fit_hist[(size_t)g * P + k] = f;
      if (pos_hist) {
        pos_hist[((size_t)g * P + k) * 2] = pos[2 * k];
        pos_hist[((size_t)g * P + k) * 2 + 1] = pos[2 * k + 1];
      }
      if (g == 0 || f < pbf[k]) {
        pbf[k] = f;
        pb[2 * k] = pos[2 * k];
        pb[2 * k + 1] = pos[2 * k + 1];
      }
    }
    for (int k = 0; k < P; ++k) {
      if (k == 0 || pbf[k] < gbf) {
        gbf = pbf[k];
        gb[0] = pb[2 * k];
        gb[1] = pb[2 * k + 1];
        gq = k;
      }
    }
    if (g + 1 == G) break;
    for (int k = 0; k < P; ++k) {
      for (int d = 0; d < 2; ++d) {
        const size_t sidx = ((size_t)g * P + k) * 2 + d;
        double v = w * vel[2 * k + d] + c1 * r1[sidx] * (pb[2 * k + d] - pos[2 * k + d]) +
                   c2 * r2[sidx] * (gb[d] - pos[2 * k + d]);
        double np = pos[2 * k + d] + v;
        vel[2 * k + d] = v;
        pos[2 * k + d] = np < 0.0 ? 0.0 : (np > 1.0 ? 1.0 : np);
      }
    }
  }
  if (best_pos) {
    best_pos[0] = gb[0];
    best_pos[1] = gb[1];
  }
  if (best_fit) *best_fit = gbf;
  if (U_best) memcpy(U_best, U + (size_t)gq * n * C, sizeof(double) * (size_t)n * C);
  if (c_best) memcpy(c_best, cs + (size_t)gq * C, sizeof(double) * C);
  free(U);
  free(cs);
  free(Ut);
  free(pos);
  free(vel);
  free(pb);
  free(pbf);
  return 0;
}

/* Central finite differences of J_K(lambda, xi, c0): the fitness after
 * exactly K IFCM steps from the fixed U0 (eps = 0).  grad = [dJ/dlambda,
 * dJ/dxi, dJ/dc0_0 .. dJ/dc0_{C-1}]. */
int oracle_fd_grad(const float* x, int nx, int ny, int nz, const or_params* p, double lambda,
                   double xi, const double* c0, const double* U0, int K, double step,
                   double* J_out, double* grad) {
  if (!params_ok(p) || !U0 || !c0 || K < 0 || !(step > 0.0) || !grad) return -1;
  or_params q = *p;
  q.eps = 0.0;
  q.max_iter = K;
  const int C = p->C;
  const int64_t n = (int64_t)nx * ny * nz;
  double* Ut = (double*)malloc(sizeof(double) * (size_t)n * C);
  double ct[OR_MAX_C], cc[OR_MAX_C];
  int32_t it = 0;
  double Jp = 0.0, Jm = 0.0;
  if (J_out) oracle_solve(x, nx, ny, nz, &q, lambda, xi, c0, U0, Ut, ct, J_out, &it, NULL);
  oracle_solve(x, nx, ny, nz, &q, lambda + step, xi, c0, U0, Ut, ct, &Jp, &it, NULL);
  oracle_solve(x, nx, ny, nz, &q, lambda - step, xi, c0, U0, Ut, ct, &Jm, &it, NULL);
  grad[0] = (Jp - Jm) / (2.0 * step);
  oracle_solve(x, nx, ny, nz, &q, lambda, xi + step, c0, U0, Ut, ct, &Jp, &it, NULL);
  oracle_solve(x, nx, ny, nz, &q, lambda, xi - step, c0, U0, Ut, ct, &Jm, &it, NULL);
  grad[1] = (Jp - Jm) / (2.0 * step);
  for (int j = 0; j < C; ++j) {
    memcpy(cc, c0, sizeof(double) * C);
    cc[j] = c0[j] + step;
    oracle_solve(x, nx, ny, nz, &q, lambda, xi, cc, U0, Ut, ct, &Jp, &it, NULL);
    cc[j] = c0[j] - step;
    oracle_solve(x, nx, ny, nz, &q, lambda, xi, cc, U0, Ut, ct, &Jm, &it, NULL);
    grad[2 + j] = (Jp - Jm) / (2.0 * step);
  }
  free(Ut);
  return 0;
}
