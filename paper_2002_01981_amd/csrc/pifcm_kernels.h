// pifcm_kernels.h -- launchers of the HIP kernels (internal to libpifcm).
#pragma once
#include <algorithm>
#include <mutex>
#include <type_traits>

#include "pifcm_device.h"

namespace pifcm {

// Device scratch of the entry point that allocates nothing (scratch.hip):
// kScratchBytes per device.  scratch_region gives this device's address of
// the array (taken once per device, with that device current);
// scratch_call_lock serialises the calls that use it on one device.
constexpr size_t kScratchBytes = size_t(256) << 20;
hipError_t scratch_region(int device, void** ptr);
std::mutex* scratch_call_lock(int device);

// Fused IFCM step (step = true) or objective-only pass (step = false) over
// the tiles of a launch; ty = waves per work group (1, 2 or 4; 4 unless
// C = 4), a.pt = particles per work item (1, or 2 at C = 4).
hipError_t launch_gather(int C, const LaunchArgs& a, int grid, int ty, bool m2, bool step,
                         hipStream_t s);
// Per-pair fp64 sum of the tile slots of the preceding step / objective
// launch and the state update (one work group per pair).
hipError_t launch_finalize(int C, const LaunchArgs& a, int npairs, bool step, hipStream_t s);
// Pointwise FCM step / objective (lambda = xi = 0).
hipError_t launch_fcm(int C, const LaunchArgs& a, int grid, bool m2, bool step, hipStream_t s);
// Waves (one tile each) per work group of the general-neighbourhood kernel
// and of the fused two-ring kernel.
constexpr int kRingWaves = 4;
constexpr int kRing2Waves = 4;
// Fused step for the two Chebyshev rings of the 5x5x5 cube, C <= 4 (reads
// VolDev::rinv, the invariants of launch_ring2_invariants).
hipError_t launch_ring2(int C, const LaunchArgs& a, int grid, bool m2, bool step, hipStream_t s);
int ring2_occupancy(int C, bool m2, bool step);
hipError_t launch_ring2_invariants(const float* x, float* rinv, int nx, int ny, int nz, int q2_sqdist,
                                   hipStream_t s);
// IFCM step / objective for general neighbourhoods (a.ring, a.W).
hipError_t launch_ring(int C, const LaunchArgs& a, int grid, bool m2, bool step, hipStream_t s);
int ring_occupancy(int C, bool m2, bool step);
hipError_t launch_init_u(int C, const float* x, size_t N, const SolveState* st, float m, bool m2,
                         float* U, hipStream_t s);
hipError_t launch_invariants(const float* x, float* invg, int nx, int ny, int nz, int* flag,
                             hipStream_t s);
hipError_t launch_check_rows(const float* U, size_t N, int C, int* flag, hipStream_t s);
hipError_t launch_labels(const float* U, size_t N, int C, uint8_t* out, hipStream_t s);
// counts (device, C * K + 1 entries, zeroed by the caller) += confusion of
// labels against truth; the last entry counts out-of-range pairs.
hipError_t launch_confusion(const uint8_t* labels, const uint8_t* truth, size_t N, int C, int K,
                            unsigned long long* counts, hipStream_t s);
hipError_t launch_permute(const float* U, size_t N, int C, const int32_t* perm, float* out,
                          hipStream_t s);
// Min-max normalisation: exact min/max keys into mm[0..1] (mm preset to
// {0xffffffff, 0}) and a non-finite flag, then the scaling pass.
hipError_t launch_minmax(const float* raw, size_t n, uint32_t* mm, int* flag, hipStream_t s);
hipError_t launch_scale(const float* raw, size_t n, const uint32_t* mm, float* out, hipStream_t s);
// Arguments of the reverse pass of one iteration (adjoint.hip).
struct AdjArgs {
  const float* x;          // [N] normalised intensities
  const float* invg;       // [N] stored g_inv (sign: flat neighbourhood)
  int32_t nx, ny, nz;
  int32_t q2_sqdist;
  float m, lam, xi;
  const float* U;          // U^(t): the iteration's input (or the final state)
  const float* c;          // c^(t) [C]
  const float* Ubar_next;  // dJ/dU^(t+1) [N][C]         (iteration pass)
  const double* cbar_next; // dJ/dc^(t+1) [C]            (iteration pass)
  const float* c_next;     // c^(t+1) [C]                (iteration pass)
  const double* B_next;    // eq (3) denominators of c^(t+1) [C]
  float* PQ;               // [N][C] da, the transpose source (P and Q are formed from it)
  float* Ubar_direct;      // [N][C] direct term of the objective-only pass
  float* partials;         // [adjoint_slots][C + 2] per-wave sums
  int32_t num_cu;          // compute units of the device (grid sizing)
  int32_t zc;              // planes per tile (set per kernel by launch_adjoint)
};
// Reverse of one iteration (eval = false) or of the final objective (eval =
// true): writes dJ/dc of that state to cbar_out[C], adds dJ/dlambda and
// dJ/dxi to acc2[0..1], and, if Ubar_out, dJ/dU of the state to Ubar_out.
hipError_t launch_adjoint(int C, const AdjArgs& a, bool m2, bool eval, float* Ubar_out,
                          double* cbar_out, double* acc2, hipStream_t s);
// Slots of per-wave sums the adjoint's per-voxel kernel writes (upper bound).
size_t adjoint_slots(int nx, int ny, int nz);

// Resident work groups per CU of the gather / pointwise kernels.
int gather_occupancy(int C, int ty, int pt, bool m2, bool step);
int fcm_occupancy(int C, bool m2, bool step);

}  // namespace pifcm
