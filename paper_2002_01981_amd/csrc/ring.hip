// ring.hip -- the IFCM step for general neighbourhoods: several rings with
// the exponential weights of eq (10), or rings by squared distance.
//
// Each voxel walks the offset table of the launch, which the host sorts by
// ring.  Per ring r it forms the ratio of eq (5) (sum_k u_kj g_ik over
// sum_k g_ik, or the mean of u_kj when every g_ik of the ring is 0, or 0 for
// a ring without in-volume cells) and the ratio of eq (7), and adds them with
// the weight W_r of eq (10).  Then eqs (4), (1), (2) and (3) as in the fused
// 3x3x3 step.  Work is decomposed like the fused step: a wave owns a tile of
// 16 x 4 columns and zc planes and its lanes walk their columns along z, so
// the cells a wave reads (its tile plus the reach of the table in x, y and
// z) stay in the L1 cache while it moves one plane at a time; neighbours are
// read from global memory through the caches.
#include "common.h"
#include "pifcm_kernels.h"

namespace pifcm {

template <int C, bool M2, bool STEP>
__global__ __launch_bounds__(64 * kRingWaves) void k_ifcm_ring(const LaunchArgs a) {
  constexpr int NV = STEP ? 2 * C + 1 : 1;
  constexpr int TX = 16, TY = 4;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int tx = lane & (TX - 1), ty = lane / TX;
  const int xcd = blockIdx.x & 7;
  const int it_end = a.xcd_begin[xcd + 1];
  const int it_step = (gridDim.x >> 3) * kRingWaves;
  for (int it = a.xcd_begin[xcd] + (blockIdx.x >> 3) * kRingWaves + wave; it < it_end; it += it_step) {
    const int b = vol_of_item(a, it);
    const VolDev vd = ld_const(a.vols + b);
    const int r = it - a.item_begin[b];
    const int pidx = r / vd.tiles;
    const int tile = r - pidx * vd.tiles;
    const PairDev pr = ld_const(a.pairs + b * a.P + pidx);
    const SolveState* st = pr.st;
    if (STEP && ld_const(&st->stop)) continue;
    const int t = STEP ? ld_const(&st->iter) + 1 : ld_const(&st->iter);
    const gfloat* Uin = as_global(STEP ? u_in_of(pr, t) : u_state_of(pr, t));
    gfloat* Uout = STEP ? as_global(u_out_of(pr, t)) : nullptr;
    const gfloat* X = as_global(vd.x);
    float cj[C];
#pragma unroll
    for (int j = 0; j < C; ++j) cj[j] = ld_const(&st->c[(STEP ? t - 1 : t) & 1][j]);
    const float lam = ld_const(&st->lam), xi = ld_const(&st->xi);
    const int nx = vd.nx, ny = vd.ny, nz = vd.nz;
    const int txi = tile % vd.ntx;
    const int rest = tile / vd.ntx;
    const int tyi = rest % vd.nty;
    const int tzi = rest / vd.nty;
    const int vx = txi * TX + tx, vy = tyi * TY + ty;
    const bool active = vx < nx && vy < ny;
    const int zlo = vd.zbeg + tzi * vd.zc, zhi = min(zlo + vd.zc, vd.zend);
    float acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = 0.f;
    for (int vz = zlo; vz < zhi && active; ++vz) {
      const size_t i = ((size_t)vz * ny + vy) * nx + vx;
      const float xv = X[i];
      float H[C], F[C];
#pragma unroll
      for (int j = 0; j < C; ++j) H[j] = F[j] = 0.f;
      // Sums of the ring being walked.
      float hn[C], hm[C], fn[C], gsum = 0.f, qsum = 0.f;
      int cnt = 0;
#pragma unroll
      for (int j = 0; j < C; ++j) hn[j] = hm[j] = fn[j] = 0.f;
      int rcur = a.nring > 0 ? (int)ld_const(a.ring).ring : 0;
      auto fold = [&]() __attribute__((always_inline)) {
        const float w = a.W[rcur];
        if (cnt > 0) {
          // eq (5); a ring whose cells all share the voxel's intensity
          // takes the plain mean (the equal-weight limit)
          const float ih = gsum > 0.f ? w / gsum : w / (float)cnt;
          const float iq = w / qsum;  // eq (7); qsum > 0 when cnt > 0
#pragma unroll
          for (int j = 0; j < C; ++j) {
            H[j] = fmaf(gsum > 0.f ? hn[j] : hm[j], ih, H[j]);
            F[j] = fmaf(fn[j], iq, F[j]);
          }
        }
      };
      for (int o = 0; o < a.nring; ++o) {
        const RingOff ro = ld_const(a.ring + o);
        if (ro.ring != rcur) {
          fold();
          gsum = qsum = 0.f;
          cnt = 0;
#pragma unroll
          for (int j = 0; j < C; ++j) hn[j] = hm[j] = fn[j] = 0.f;
          rcur = ro.ring;
        }
        const int kx = vx + ro.dx, ky = vy + ro.dy, kz = vz + ro.dz;
        if (kx < 0 || kx >= nx || ky < 0 || ky >= ny || kz < 0 || kz >= nz) continue;
        const size_t kk = ((size_t)kz * ny + ky) * nx + kx;
        const float g = fabsf(xv - X[kk]);  // eq (6)
        float u[C];
        load_row<C>(Uin + kk * C, u);
        gsum += g;
        qsum += ro.q2;
        ++cnt;
#pragma unroll
        for (int j = 0; j < C; ++j) {
          hn[j] = fmaf(u[j], g, hn[j]);
          hm[j] += u[j];
          fn[j] = fmaf(u[j] * u[j], ro.q2, fn[j]);
        }
      }
      fold();
      float uo[C], d2[C];
      load_row<C>(Uin + i * C, uo);
      float Jv = 0.f;
#pragma unroll
      for (int j = 0; j < C; ++j) {
        const float av = 1.f - lam * H[j] - xi * F[j];  // eq (4) factor
        const float dd = xv - cj[j];
        d2[j] = fmaxf(dd * dd * av, kDFloor);
        Jv = fmaf(pow_m<M2>(uo[j], a.m), d2[j], Jv);  // eq (1)
      }
      if constexpr (STEP) {
        float un[C];
        memberships<C, M2>(d2, a.m, un);  // eq (2)
        store_row<C>(Uout + i * C, un);
#pragma unroll
        for (int j = 0; j < C; ++j) {
          const float w = pow_m<M2>(un[j], a.m);
          acc[j] = fmaf(w, xv, acc[j]);  // eq (3)
          acc[C + j] += w;
        }
        acc[2 * C] += Jv;
      } else {
        acc[0] += Jv;
      }
    }
    wave_tile_store<NV>(pr, tile, acc);
  }
}

template <int C, bool M2>
static hipError_t launch_ring_ct(const LaunchArgs& a, int grid, bool step, hipStream_t s) {
  if (step) hipLaunchKernelGGL((k_ifcm_ring<C, M2, true>), dim3(grid), dim3(64 * kRingWaves), 0, s, a);
  else hipLaunchKernelGGL((k_ifcm_ring<C, M2, false>), dim3(grid), dim3(64 * kRingWaves), 0, s, a);
  return hipGetLastError();
}

template <int C, bool M2>
static int occ_ring_ct(bool step) {
  int n = 0;
  const void* f = step ? reinterpret_cast<const void*>(&k_ifcm_ring<C, M2, true>)
                       : reinterpret_cast<const void*>(&k_ifcm_ring<C, M2, false>);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, 64 * kRingWaves, 0) != hipSuccess) n = 1;
  return std::max(1, n);
}

hipError_t launch_ring(int C, const LaunchArgs& a, int grid, bool m2, bool step, hipStream_t s) {
  switch (C) {
#define PIFCM_RING_CASE(c)                                                       \
  case c:                                                                        \
    return m2 ? launch_ring_ct<c, true>(a, grid, step, s)                        \
              : launch_ring_ct<c, false>(a, grid, step, s);
    PIFCM_RING_CASE(2) PIFCM_RING_CASE(3) PIFCM_RING_CASE(4) PIFCM_RING_CASE(5)
    PIFCM_RING_CASE(6) PIFCM_RING_CASE(7) PIFCM_RING_CASE(8) PIFCM_RING_CASE(9)
    PIFCM_RING_CASE(10) PIFCM_RING_CASE(11) PIFCM_RING_CASE(12) PIFCM_RING_CASE(13)
    PIFCM_RING_CASE(14) PIFCM_RING_CASE(15) PIFCM_RING_CASE(16)
#undef PIFCM_RING_CASE
    default:
      return hipErrorInvalidValue;
  }
}

int ring_occupancy(int C, bool m2, bool step) {
  switch (C) {
#define PIFCM_RING_OCC(c) \
  case c:                 \
    return m2 ? occ_ring_ct<c, true>(step) : occ_ring_ct<c, false>(step);
    PIFCM_RING_OCC(2) PIFCM_RING_OCC(3) PIFCM_RING_OCC(4) PIFCM_RING_OCC(5)
    PIFCM_RING_OCC(6) PIFCM_RING_OCC(7) PIFCM_RING_OCC(8) PIFCM_RING_OCC(9)
    PIFCM_RING_OCC(10) PIFCM_RING_OCC(11) PIFCM_RING_OCC(12) PIFCM_RING_OCC(13)
    PIFCM_RING_OCC(14) PIFCM_RING_OCC(15) PIFCM_RING_OCC(16)
#undef PIFCM_RING_OCC
    default:
      return 1;
  }
}

}  // namespace pifcm
