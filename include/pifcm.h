/*
 * pifcm.h -- C ABI of libpifcm: the IFCM iteration of 3DPIFCM on AMD MI355X
 * (gfx950).
 *
 * The method is the one of Agranonik, Herman and Last, "Parallel 3DPIFCM
 * Algorithm for Noisy Brain MRI Images" (arXiv 2002.01981): fuzzy c-means
 * whose distance (section 2, eq (4)) is scaled by a feature attraction H
 * (eqs (5), (6)) and a neighbourhood attraction F (eqs (7), (8)) gathered
 * from each voxel's 3D neighbourhood (eq (9)), iterated between memberships
 * (eq (2)) and centres (eq (3)) until the objective (eq (1)) settles, once per
 * particle of a swarm search over the two weights (lambda, xi) (Algorithm 1).
 *
 * Conventions shared by every entry point:
 *   - Volumes are float32, laid out [nz][ny][nx] with x fastest, already
 *     min-max normalised to [0, 1] (pifcm_normalize does that on the GPU).
 *   - Memberships U are float32 [N][C], voxel-major (the C values of one
 *     voxel are contiguous), N = nx * ny * nz.  Device pointers must be
 *     16-byte aligned.  Rows of a caller-supplied U must be memberships:
 *     entries in [0, 1] summing to 1 (within 1e-4); otherwise the call
 *     fails with PIFCM_E_INVALID.
 *   - "device" pointers are HIP device memory (e.g. torch tensors'
 *     data_ptr()); "host" pointers are ordinary CPU memory.  The caller owns
 *     every input and output buffer; the library owns its workspace (kept in
 *     the context and reused until pifcm_destroy).
 *   - Work is ordered after everything already queued on the context's
 *     stream (the stream given to pifcm_create or pifcm_set_stream) and
 *     calls that return host outputs wait for their work to finish.
 *   - Every function returns a pifcm_status and never aborts.  On error the
 *     host outputs are left untouched, device outputs are unspecified,
 *     inputs are never modified, and pifcm_last_error describes the cause.
 *   - Results are deterministic: the same inputs give bit-identical outputs
 *     (all sums are taken in a fixed order; no floating-point atomics).
 *   - A context is used by one host thread at a time.  Separate contexts
 *     (each with its own stream and workspace) may be used from different
 *     threads at once, on one device or several; ifcm_solve_noalloc calls
 *     on one device share that device's scratch array and are serialised
 *     by the library.
 */
#ifndef PIFCM_H
#define PIFCM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PIFCM_OK = 0,
  PIFCM_E_INVALID = -1,     /* null/misaligned pointer, out-of-range value   */
  PIFCM_E_NONFINITE = -2,   /* a NaN or Inf intensity                       */
  PIFCM_E_OOM = -3,         /* workspace allocation failed                  */
  PIFCM_E_HIP = -4,         /* HIP runtime error                            */
  PIFCM_E_UNSUPPORTED = -5  /* valid request outside what is built          */
} pifcm_status;

typedef struct pifcm_ctx pifcm_ctx;

/* Context on HIP device `device`; `hip_stream` is a hipStream_t (NULL: the
 * device's null stream).  The context owns a private non-blocking stream for
 * its work and orders it after / before `hip_stream` with events. */
pifcm_status pifcm_create(int device, void* hip_stream, pifcm_ctx** out);
void pifcm_destroy(pifcm_ctx* ctx);
pifcm_status pifcm_set_stream(pifcm_ctx* ctx, void* hip_stream);
/* Description of the last error on ctx (valid until the next call on ctx);
 * "" if the last call succeeded.  Accepts NULL. */
const char* pifcm_last_error(const pifcm_ctx* ctx);

/* Readings of passages the paper leaves open (flags). */
#define PIFCM_SHELL_SQDIST 1 /* rings of eqs (5), (7), (10) by squared distance
                                dX^2 + dY^2 + dZ^2 = 1..V instead of the
                                Chebyshev shells max(|dX|, |dY|, |dZ|) = 1..V */
#define PIFCM_Q2_SQDIST 2    /* weight q (eq (8)) instead of q^2 in eq (7) */

typedef struct {
  int32_t C;        /* c: number of clusters, 2..16 (Algorithm 1 input)          */
  float m;          /* m: fuzziness, > 1 (Algorithm 1 input)                      */
  int32_t V;        /* v: depth = number of rings; 1 = the 3x3x3 neighbourhood.
                       Chebyshev rings: V <= 3; with PIFCM_SHELL_SQDIST: V <= 15
                       (cells at most 3 apart along each axis)                */
  float h;          /* h: decay of eq (10), W_r ~ exp(-(r - 1) / h), > 0; only
                       matters with more than one ring                         */
  float eps;        /* epsilon: stop after iteration t >= 2 once
                       |J(t-1) - J(t-2)| <= eps * |J(t-2)|; 0 = run max_iter       */
  int32_t max_iter; /* iteration cap, >= 0                                       */
  int32_t flags;    /* PIFCM_* readings                                          */
} pifcm_params;

typedef struct {
  int32_t nx, ny, nz; /* >= 1 each                                               */
  const float* x;     /* device [nz][ny][nx], normalised intensities             */
} pifcm_volume;

/* Min-max normalisation of a raw volume (Algorithm 2, step 1):
 * x_out = (raw - min) / (max - min), evaluated in double precision and
 * rounded to float32; a constant volume gives zeros.  raw and x_out are
 * device [n] and may alias.  PIFCM_E_NONFINITE if any raw value is NaN/Inf. */
pifcm_status pifcm_normalize(pifcm_ctx* ctx, const float* raw, int64_t n, float* x_out);

/* One IFCM solve at fixed (lambda, xi) -- the final step of Algorithm 1
 * (step 11) and the unit of every fitness evaluation (steps 4-9).
 * Starting from centres_in (host [C]) and U_in (device [N][C]; NULL means
 * eq (2) with the attraction factor 1, i.e. FCM memberships of centres_in),
 * iterate eqs (4)-(10), (2), (3) -- every H and F of an iteration reads that
 * iteration's input memberships -- until the stop rule of pifcm_params or
 * max_iter.  lambda = xi = 0 is plain FCM (eqs (1)-(3)).
 * Outputs: U_out (device [N][C], must not alias U_in), centres_out (host
 * [C]), labels_out (device [N] uint8 argmax_j u_ij with ties to the lowest
 * j, or NULL), J_out (host: J of eq (1) at the final state -- the fitness),
 * iters_out (host: iterations performed), J_hist_out (host [max_iter] or
 * NULL: J of the input state of each iteration performed).
 * The squared distance of eq (4) is floored at 1e-12 so eq (2) stays
 * defined when the attraction factor is <= 0 or a voxel equals a centre.
 * lambda and xi may lie outside [0, 1] but must satisfy |.| <= 1000
 * (PIFCM_E_INVALID otherwise).
 * V = 1 without PIFCM_SHELL_SQDIST runs the fused 3x3x3 kernel; other
 * neighbourhoods run a general kernel (one voxel per thread, neighbours read
 * through the caches).  PIFCM_E_UNSUPPORTED beyond the V limits above. */
pifcm_status ifcm_solve(pifcm_ctx* ctx, const pifcm_volume* vol, const pifcm_params* p,
                        float lambda, float xi, const float* centres_in, const float* U_in,
                        float* U_out, float* centres_out, uint8_t* labels_out, double* J_out,
                        int32_t* iters_out, double* J_hist_out);

/* ifcm_solve for callers that cannot allocate device memory (code under HIP
 * graph capture elsewhere in the program, serving loops, harnesses that
 * forbid hipMalloc): the same solve, the same kernels, the same arguments,
 * outputs and decomposition -- results are bit-identical to ifcm_solve's on
 * the same context -- but no hipMalloc, hipFree or other allocating call.
 * Its workspace (g_inv, the second membership buffer, tile sums, solve
 * state, objective history; about 4 * (C + 1) bytes per voxel) lives in a
 * device array of 256 MiB that the library holds on every GPU it runs on
 * until the process ends; a C = 4 volume of up to about 13 million voxels
 * fits.  Its host staging is the pinned buffer pifcm_create allocates.  A solve that needs more fails with PIFCM_E_INVALID (naming the
 * bytes needed) before any work is queued; V > 1 is PIFCM_E_UNSUPPORTED.
 * The array is shared by every call on that GPU and keeps the last call's
 * contents (each call initialises what it reads): calls on one device are
 * serialised inside the library, and every call finishes its work before
 * it returns.  The call synchronises the context's stream, so it cannot
 * itself be captured into a graph.  Unlike the other entry points,
 * J_hist_out is copied straight into the caller's array and may hold
 * partial values if a HIP error ends the call. */
pifcm_status ifcm_solve_noalloc(pifcm_ctx* ctx, const pifcm_volume* vol, const pifcm_params* p,
                                float lambda, float xi, const float* centres_in, const float* U_in,
                                float* U_out, float* centres_out, uint8_t* labels_out, double* J_out,
                                int32_t* iters_out, double* J_hist_out);

/* Slab mode of ifcm_solve -- Algorithm 1 step 1 segments one slice z of the
 * volume with its 3D neighbours: only the planes [zbeg, zend) (e.g. [z,
 * z + 1)) are iterated; the memberships of every other plane stay those of
 * U_in (required) and enter the neighbourhood sums as fixed context.  The
 * centres (eq (3)) and J (eq (1)) are sums over the planes iterated.
 * U_out (device [N][C]) receives the whole volume (context planes copied
 * from U_in), labels_out (device [N] or NULL) its labels; other arguments
 * as ifcm_solve.  0 <= zbeg < zend <= nz. */
pifcm_status ifcm_solve_slab(pifcm_ctx* ctx, const pifcm_volume* vol, int32_t zbeg, int32_t zend,
                             const pifcm_params* p, float lambda, float xi, const float* centres_in,
                             const float* U_in, float* U_out, float* centres_out,
                             uint8_t* labels_out, double* J_out, int32_t* iters_out,
                             double* J_hist_out);

/* Initial state of Algorithm 1 step 2: plain FCM (lambda = xi = 0) from
 * evenly spaced centres c_j = (j + 1/2) / C, then the centres sorted
 * ascending with the membership columns permuted alike.  The paper seeds
 * this with an unspecified Gaussian mixture model, which is not reproduced.
 * Outputs: U0_out (device [N][C]), centres_out (host [C]), iters_out (host,
 * may be NULL). */
pifcm_status pifcm_fcm_init(pifcm_ctx* ctx, const pifcm_volume* vol, const pifcm_params* p,
                            float* U0_out, float* centres_out, int32_t* iters_out);

/* Fitness of every particle on every volume -- Algorithm 1 step 4.
 * vols: host array [B] (volume b holds N_b voxels); particles: host
 * [B][P][2] of (lambda, xi); centres0: host [B][C] and U0: host array of B
 * device pointers [N_b][C] -- the shared initial state of volume b.  Each
 * (b, p) runs one IFCM solve from (centres0[b], U0[b]) exactly as
 * ifcm_solve does, and its fitness is J at the final state.
 * Outputs (host): fitness_out [B][P] (double), centres_out [B][P][C] or
 * NULL, iters_out [B][P] or NULL.
 * mode PIFCM_SWARM_BATCHED runs the whole swarm as one fused launch per
 * iteration, captured in a HIP graph; PIFCM_SWARM_PLAIN launches one kernel
 * per (b, p) per iteration.  Both give bit-identical results under the same
 * tile shape (pifcm_tune may choose another shape, which changes the order
 * of the floating-point sums).
 * B <= 32, 1 <= P, B * P <= 65536. */
#define PIFCM_SWARM_BATCHED 0
#define PIFCM_SWARM_PLAIN 1
pifcm_status swarm_evaluate(pifcm_ctx* ctx, const pifcm_volume* vols, int32_t B,
                            const pifcm_params* p, const float* particles, int32_t P,
                            const float* centres0, const float* const* U0, double* fitness_out,
                            float* centres_out, int32_t* iters_out, int32_t mode);

/* Gradient of J_K = J(U^K, c^K) -- eq (1) after exactly K IFCM iterations
 * from (centres0 (host [C]), U0 (device [N][C])), U0 held constant -- with
 * respect to lambda, xi and the initial centres, by a hand-written adjoint
 * of the K unrolled iterations (1 <= K <= 100000).  Memberships are kept
 * every ckpt_every iterations (1 <= ckpt_every <= K) and recomputed segment
 * by segment; the context's workspace grows to about
 * (K / ckpt_every + ckpt_every + 5) * N * C * 4 bytes.
 * Outputs (host): J_out, dJ_dlambda, dJ_dxi, dJ_dcentres [C].
 * Built for the 3x3x3 neighbourhood (V = 1 without PIFCM_SHELL_SQDIST);
 * PIFCM_E_UNSUPPORTED otherwise. */
pifcm_status ifcm_backward(pifcm_ctx* ctx, const pifcm_volume* vol, const pifcm_params* p,
                           float lambda, float xi, const float* centres0, const float* U0,
                           int32_t K, int32_t ckpt_every, double* J_out, double* dJ_dlambda,
                           double* dJ_dxi, double* dJ_dcentres);

/* Pick the work decomposition of the fused step for these volumes -- waves
 * per work group, planes per tile and, at C = 4 with P >= 2, particles per
 * work item (1 or 2: two particles of a volume share its intensities and
 * the |x_i - x_k| of eq (6)) -- by timing a short batched swarm evaluation
 * (P particles spread over [0, 1]^2, a few iterations from FCM memberships
 * of evenly spaced centres) for each candidate.  A candidate is eligible
 * only if its fitnesses and centres agree with the default decomposition's
 * to 1e-5 relative and its final memberships of the first two particles on
 * the smallest volume agree element by element to 1e-4 of their largest
 * value (tilings change the order of the sums, nothing else).  The choice is
 * kept in ctx for these (C, m == 2, shape) keys and used by later calls.  If
 * the environment variable PIFCM_TUNE_CACHE names a file, a choice stored
 * there for the same device architecture, C, m == 2, V, B, P and shape
 * bucket (total voxels and largest plane count rounded up to powers of two)
 * is applied without timing, and a new choice is added to the file (a JSON
 * object, one entry per line).  best_out (host, may be NULL) receives a short
 * description (best_len bytes).  The general-neighbourhood kernel has a
 * fixed decomposition: for those parameters nothing is timed. */
pifcm_status pifcm_tune(pifcm_ctx* ctx, const pifcm_volume* vols, int32_t B,
                        const pifcm_params* p, int32_t P, char* best_out, int32_t best_len);

/* Set the work decomposition of the fused step for these volumes by hand
 * (what pifcm_tune would otherwise choose): waves per work group (1, 2 or 4),
 * planes per tile (>= 1, clamped to the volume and to the 32-bit offset
 * range; 0 = the default depth: of the depths ceil(nz / k) and 32 that
 * are at least min(nz, 32), the one with the fewest rounds of one pair's
 * tiles on the resident waves times (depth + 4), as a solve without a chosen
 * decomposition uses) and particles per work item (1 or 2; used by batched swarm
 * launches of P >= 2 particles).  Other values than 4 waves and 1 particle
 * are built for C = 4 only (PIFCM_E_UNSUPPORTED otherwise).  Kept in ctx for
 * these (C, m == 2, shape) keys, as a tuned choice is.  Results of every
 * decomposition agree up to the order of floating-point sums; for a given
 * waves and planes choice the particles per item do not change any result
 * bit. */
pifcm_status pifcm_set_decomposition(pifcm_ctx* ctx, const pifcm_volume* vols, int32_t B,
                                     const pifcm_params* p, int32_t waves_per_group,
                                     int32_t planes_per_tile, int32_t particles_per_item);

/* Particle swarm search over (lambda, xi) in [0, 1]^2 -- Algorithm 1 steps
 * 3-9 -- on B volumes at once, each volume with its own swarm of P
 * particles; every generation evaluates all B * P fitnesses with one
 * swarm_evaluate call (mode as there).  The paper's update has no inertia or
 * coefficients and names no topology; this is the synchronous global-best
 * swarm: v <- w v + c1 r1 (pbest - x) + c2 r2 (gbest - x), x <- clip(x + v,
 * 0, 1), per particle and dimension, improvements only when strictly better,
 * ties of the best to the lowest particle index.  All random numbers come
 * from the caller: x0, v0 (host [P][2]) start every volume's swarm; r1, r2
 * (host [G][P][2]) are the coefficients of generation g.  centres0, U0: the
 * shared initial state of each volume (as in swarm_evaluate).
 * Outputs (host): best_pos [B][2], best_fit [B], and optionally fit_hist
 * [B][G][P], pos_hist [B][G][P][2] (positions evaluated) and iters_hist
 * [B][G][P] (IFCM iterations each evaluation ran before its stop rule or
 * max_iter ended it); NULL skips an optional output. */
pifcm_status pifcm_pso(pifcm_ctx* ctx, const pifcm_volume* vols, int32_t B, const pifcm_params* p,
                       int32_t P, int32_t G, const double* x0, const double* v0, const double* r1,
                       const double* r2, double w, double c1, double c2, const float* centres0,
                       const float* const* U0, int32_t mode, double* best_pos, double* best_fit,
                       double* fit_hist, double* pos_hist, int32_t* iters_hist);

/* The interleaved reading of the swarm schedule (Algorithm 2, step 11):
 * every particle carries its own IFCM state.  Particle q of volume b starts
 * from (centres0[b], U0[b]); in generation g it runs `steps` IFCM iterations
 * (no stop rule; p->eps and p->max_iter are not used) at its current
 * (lambda, xi) from the state it reached in generation g - 1, its fitness is
 * J of eq (1) at the new state, and the swarm then moves as in pifcm_pso
 * (same update, same random-number arguments and outputs).  U_best_out
 * (host array [B] of device [N_b][C], may be NULL) and centres_best_out
 * (host [B][C], may be NULL) receive, per volume, the final state of the
 * particle whose personal best is the global best.  The library holds one
 * membership buffer per (volume, particle) for the states. */
pifcm_status pifcm_pso_interleaved(pifcm_ctx* ctx, const pifcm_volume* vols, int32_t B,
                                   const pifcm_params* p, int32_t P, int32_t G, int32_t steps,
                                   const double* x0, const double* v0, const double* r1,
                                   const double* r2, double w, double c1, double c2,
                                   const float* centres0, const float* const* U0, int32_t mode,
                                   double* best_pos, double* best_fit, double* fit_hist,
                                   double* pos_hist, float* const* U_best_out,
                                   float* centres_best_out);

/* Segmentation quality against a reference: confusion counts of labels
 * (device [n] uint8, cluster indices 0..C-1, e.g. from ifcm_solve) against
 * truth (device [n] uint8, classes 0..K-1): counts_out (host [C][K] int64)
 * [j][k] = number of voxels labelled j whose class is k.  With centres sorted
 * ascending and classes numbered by intensity, the misclassification rate
 * of the paper's quality comparisons (section 6) is 1 - trace / n.
 * PIFCM_E_INVALID if a label or class is out of range. */
pifcm_status pifcm_confusion(pifcm_ctx* ctx, const uint8_t* labels, const uint8_t* truth, int64_t n,
                             int32_t C, int32_t K, int64_t* counts_out);

/* Device workspace the context holds (bytes, host outputs; either may be
 * NULL): the sum of its device buffers, which only grow, so this is also the
 * peak since pifcm_create, and its pinned host staging buffer. */
pifcm_status pifcm_workspace_bytes(pifcm_ctx* ctx, int64_t* device_bytes, int64_t* pinned_bytes);

/* Benchmark timing of the fused step launches.  While enabled, ifcm_solve
 * and swarm_evaluate record HIP events on the context's own stream before
 * their first and after their last step launch (the launches are queued back
 * to back when eps == 0) and add the elapsed time and the number of step
 * launches to two counters.  pifcm_get_timing reads them (host outputs;
 * either may be NULL) and, if reset != 0, clears them. */
pifcm_status pifcm_set_timing(pifcm_ctx* ctx, int32_t enable);
pifcm_status pifcm_get_timing(pifcm_ctx* ctx, double* step_ms, int64_t* step_launches,
                              int32_t reset);

#ifdef __cplusplus
}
#endif
#endif /* PIFCM_H */
