/*
 * pifcm_oracle.h -- FP64 CPU reference of the 3DPIFCM IFCM iteration.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may include,
 * link or call this code; only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no source, header, table
 * or helper with the GPU path.
 *
 * Every function follows the paper (Agranonik, Herman, Last, "Parallel
 * 3DPIFCM Algorithm for Noisy Brain MRI Images", arXiv 2002.01981) in its own
 * notation, in double precision, with no blocking or fusion:
 *   objective J_m ........................ section 2, eq (1)
 *   memberships .......................... eq (2)
 *   centres .............................. eq (3)
 *   modified distance .................... eq (4)
 *   feature attraction H ................. eq (5), g from eq (6)
 *   neighbourhood attraction F ........... eq (7), q from eq (8)
 *   neighbourhood set NB ................. eq (9)
 *   ring weights W ....................... eq (10)
 *   IFCM loop / PSO ...................... Algorithm 1, Algorithm 2
 *   min-max normalisation ................ Algorithm 2, step 1
 * Readings of passages the paper leaves open are listed beside each function.
 *
 * Pins (what each function is checked against, in tests/test_oracle_*.py):
 *   oracle_normalize ..... exact 0 / 1 at min / max, order preservation,
 *                          power-of-two affine invariance, constant volume
 *   oracle_step .......... textbook FCM at lambda = xi = 0, literal
 *                          set-builder brute force of eq (9) on tiny volumes,
 *                          closed form of a two-voxel volume, uniform-U
 *                          identity, convex-combination bounds of H and F,
 *                          sum-to-one of eq (2), the m = 2 identity
 *   oracle_init_memberships textbook FCM memberships of the centres
 *   oracle_solve ......... FCM descent, constant image, axis flips,
 *                          transposes and centre permutations; the stop
 *                          rule against the first small relative change
 *                          found by hand in a fixed-count run's J list; the
 *                          fitness against J of the last input state of a
 *                          run one iteration longer (and textbook FCM's J
 *                          at lambda = xi = 0)
 *   oracle_solve_slab .... whole-volume slab equals oracle_solve; one-step
 *                          brute force of the active planes; fixed context
 *   oracle_fcm_init ...... sorted centres; equals solve-then-sort
 *   oracle_labels ........ numpy argmax (first maximum)
 *   oracle_pso ........... one hand-derived generation; frozen swarm;
 *                          re-evaluated fitness; pbest monotonicity
 *   oracle_pso_interleaved frozen swarm equals one long solve; steps =
 *                          max_iter with one generation equals oracle_pso
 *   oracle_fd_grad ....... closed-form derivative at K = 0; step-size
 *                          agreement h vs h/2
 */
#ifndef PIFCM_ORACLE_H
#define PIFCM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* flags */
#define OR_SHELL_SQDIST 1 /* rings by squared distance instead of Chebyshev radius */
#define OR_Q2_SQDIST 2    /* weight q instead of q^2 in eq (7)                      */

typedef struct {
  int32_t C;        /* number of clusters c                      */
  int32_t V;        /* depth v: number of rings                  */
  int32_t max_iter; /* iteration cap                             */
  int32_t flags;    /* OR_* readings                             */
  double m;         /* fuzziness m > 1                           */
  double h;         /* exponential decay of eq (10)              */
  double eps;       /* relative stop criterion                   */
} or_params;

int oracle_set_threads(int n);
int oracle_get_threads(void);

int oracle_normalize(const float* raw, int64_t n, float* out);

int oracle_init_memberships(const float* x, int64_t n, const or_params* p, const double* c,
                            double* U);

int oracle_step(const float* x, int nx, int ny, int nz, const or_params* p, double lambda,
                double xi, const double* U, const double* c, double* U_out, double* c_out,
                double* J_out, double* H_out, double* F_out);

int oracle_solve(const float* x, int nx, int ny, int nz, const or_params* p, double lambda,
                 double xi, const double* c0, const double* U0, double* U_out, double* c_out,
                 double* J_fit, int32_t* iters, double* J_hist);

int oracle_solve_slab(const float* x, int nx, int ny, int nz, int zbeg, int zend,
                      const or_params* p, double lambda, double xi, const double* c0,
                      const double* U0, double* U_out, double* c_out, double* J_fit,
                      int32_t* iters, double* J_hist);

int oracle_fcm_init(const float* x, int nx, int ny, int nz, const or_params* p, double* U_out,
                    double* c_out, int32_t* iters);

int oracle_labels(const double* U, int64_t n, int C, uint8_t* labels);

int oracle_pso(const float* x, int nx, int ny, int nz, const or_params* p, const double* c0,
               const double* U0, int P, int G, const double* x0, const double* v0,
               const double* r1, const double* r2, double w, double c1, double c2,
               double* best_pos, double* best_fit, double* fit_hist, double* pos_hist);

int oracle_pso_interleaved(const float* x, int nx, int ny, int nz, const or_params* p,
                           const double* c0, const double* U0, int P, int G, int steps,
                           const double* x0, const double* v0, const double* r1, const double* r2,
                           double w, double c1, double c2, double* best_pos, double* best_fit,
                           double* fit_hist, double* pos_hist, double* U_best, double* c_best);

int oracle_fd_grad(const float* x, int nx, int ny, int nz, const or_params* p, double lambda,
                   double xi, const double* c0, const double* U0, int K, double step,
                   double* J_out, double* grad);

#ifdef __cplusplus
}
#endif
#endif
