// pifcm_device.h -- descriptors shared by the HIP kernels and the host
// runtime of libpifcm (not part of the public ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pifcm {

constexpr int kMaxC = 16;         // clusters supported
constexpr int kMaxBatchVols = 32; // volumes in one batched launch
constexpr int kWaveTileX = 16;    // columns of a fused-step tile along x
constexpr int kWaveTileY = 4;     // and along y (16 x 4 = one wavefront)
constexpr float kDFloor = 1e-12f; // floor of the squared distance of eq (4)
constexpr int kFcmVoxPerThread = 8;

// Device-side state of one IFCM run (one volume x one particle).
struct alignas(64) SolveState {
  float c[2][kMaxC];   // centres by iteration parity: c^(t) lives in c[t & 1]
  float lam, xi;       // the particle (lambda, xi)
  float eps;           // relative stop criterion (0: run max_iter)
  int32_t max_iter;
  int32_t iter;        // iterations completed
  int32_t stop;        // 1 once the run has converged or hit max_iter
  uint32_t counter;    // tiles of the current launch that have finished
  int32_t pad0;
  double J_prev1;      // J(t-1): objective of the previous iteration's input
  double J_prev2;      // J(t-2)
  double J_eval;       // J of the final state (fitness)
  double* J_hist;      // optional device [max_iter]: J(t-1) of iteration t
  double* B_hist;      // optional device [max_iter][C]: eq (3) denominators
                       // sum_i u_ij^m of iteration t's new memberships
  float* c_hist;       // optional device [max_iter + 1][C]: c^(t) after
                       // iteration t (row 0 is set by the host)
};

// One volume of a launch.
struct VolDev {
  const float* x;      // [nz][ny][nx] normalised intensities
  const float* invg;   // [nz][ny][nx] 1 / sum_k |x_i - x_k|; -1 / n_valid when
                       // every neighbour has the voxel's intensity; 0 if none
  int32_t nx, ny, nz;
  int32_t zc;          // planes per tile
  int32_t ntx, nty, ntz;
  int32_t tiles;       // ntx * nty * ntz (gather kernels)
  int32_t tiles1d;     // ceil(active voxels / voxels per block) (pointwise kernels)
  int32_t zbeg, zend;  // planes iterated; the others are fixed context
  int32_t pad;
  const float* rinv;   // [nz][ny][nx][4] per-ring g_inv and q_inv (two-ring kernel only)
};

// One (volume, particle) run of a launch.
struct PairDev {
  const float* U0;     // U^(0)
  float* Ua;           // U^(t) for odd t
  float* Ub;           // U^(t) for even t >= 2
  SolveState* st;
  float* partials;     // [tiles][2C + 1] per-tile sums of one launch
};

// General neighbourhoods (rings V >= 1, eqs (5), (7), (9), (10)): offsets
// sorted by ring, at most kMaxReach cells away along each axis.
constexpr int kMaxReach = 3;
constexpr int kMaxRings = 15;
struct RingOff {
  int16_t dx, dy, dz, ring;  // offset and its ring index r (1..V)
  float q2;                  // eq (7) spatial weight of the offset
  float pad;
};

// Arguments of a fused launch over volumes [0, nvol) x particles [0, P).
// Pairs are ordered volume-major: pair (b, p) = pairs[b * P + p]; work items
// are ordered pair-major (particle-group-major for the fused step) then
// tile, so adjacent tiles of one pair are neighbours in item order.
struct LaunchArgs {
  const VolDev* vols;
  const PairDev* pairs;
  int32_t nvol;
  int32_t P;
  int32_t nitems;
  int32_t q2_sqdist;   // 1: eq (7) weight q instead of q^2
  float m;
  int32_t use_1d;      // items are 1D voxel blocks (pointwise kernels)
  int32_t item_begin[kMaxBatchVols + 1];  // first item of each volume
  int32_t xcd_begin[9];  // items [xcd_begin[k], xcd_begin[k + 1]) go to the
                         // work groups with blockIdx.x % 8 == k (one XCD):
                         // contiguous ranges of about equal work
  int32_t* work;         // fused step: [0, 8) next item of each XCD's range,
                         // [8, 16) its waves that have run out of items;
                         // zero between launches (the last wave resets them)
  int32_t handout;       // 1: the fused step may hand out items by counter
  int32_t pad3;
  const RingOff* ring; // general-neighbourhood offsets (ring kernel only)
  int32_t nring;       // number of offsets
  int32_t pad1;
  int32_t pt;          // particles per work item of the fused step (1 or 2):
                       // its items are (volume, group of pt particles, tile)
  int32_t pad2;
  float W[kMaxRings + 1];  // eq (10) weight of ring r at W[r]
};

__host__ __device__ inline const float* u_in_of(const PairDev& pr, int t) {
  // Input of iteration t (1-based): U^(t-1).
  return t == 1 ? pr.U0 : ((t & 1) ? pr.Ub : pr.Ua);
}
__host__ __device__ inline float* u_out_of(const PairDev& pr, int t) {
  return (t & 1) ? pr.Ua : pr.Ub;
}
__host__ __device__ inline const float* u_state_of(const PairDev& pr, int T) {
  // U^(T) after T completed iterations.
  return T == 0 ? pr.U0 : ((T & 1) ? pr.Ua : pr.Ub);
}

}  // namespace pifcm
