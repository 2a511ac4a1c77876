// gather.h -- the fused IFCM step kernel (instantiated per cluster count in
// the gather_c*.hip translation units).
//
// The hot path is one IFCM iteration (section 4 of the paper, the "step
// function"): for every voxel i and cluster j the feature attraction H_ij
// (eqs (5), (6)) and neighbourhood attraction F_ij (eqs (7), (8)) over the
// 26-voxel neighbourhood (eq (9) with the 3x3x3 cube, one ring, W_1 = 1 by
// eq (10)), the modified distance (eq (4)), the objective of the input state
// (eq (1)), the new memberships (eq (2)) and the sums of the new centres
// (eq (3)).  All of it is fused into k_ifcm_gather: one HBM pass reads x and
// U^(t) and writes U^(t+1).
//
// Data flow of k_ifcm_gather.  A work item is a tile of 64 (x) by TY (y)
// columns and zc planes of one (volume, particle) pair; each lane owns one
// (x, y) column and walks it along z.  Each plane of the tile plus a
// one-voxel halo is staged once in LDS (double-buffered, one barrier per
// plane) and every lane reads its 3x3 in-plane cells once: they contribute
// to three voxels of its column at the same time -- z-1 (the plane is its
// upper neighbour plane), z (its own plane) and z+1 (lower plane).  The
// partial sums of those three voxels live in a ring of register slots; the
// voxel z-1 is complete after the plane and is finalised right away.  Plane
// data is prefetched two planes ahead into registers.
//
// Arithmetic shortcuts that keep the results those of the equations:
//   * the denominator of eq (5), sum_k |x_i - x_k|, does not change between
//     iterations and is precomputed once per volume (k_invariants);
//   * sum_j H_ij = 1 when the rows of U sum to 1, so the last cluster's H is
//     1 - sum of the others (rows of caller-supplied U are validated);
//   * eq (7)'s weights depend only on the offset class (face, edge, corner
//     in the plane and one plane off), so per plane the squared memberships
//     are summed per class once and weighted afterwards;
//   * the denominator of eq (7) is a function of which neighbours exist,
//     computed from the column position and the plane count.
// Sums over voxels are per-lane in fp32, reduced per tile in a fixed
// butterfly order, and combined over tiles in fp64 by the last tile of the
// pair to finish (no floating-point atomics: results are bit-reproducible).
#pragma once
#include "common.h"

namespace pifcm {

// ------------------------------------------------------------ fused gather
#ifndef PIFCM_GATHER_ATTR
#define PIFCM_GATHER_ATTR
#endif
template <int C, bool M2, int TY, bool STEP>
__global__ __launch_bounds__(64 * TY) PIFCM_GATHER_ATTR void k_ifcm_gather(const LaunchArgs a) {
  constexpr int NT = 64 * TY;
  constexpr int CP = (C + 3) / 4 * 4;
  constexpr int WD = kTX + 2;                // halo tile width
  constexpr int NCELL = WD * (TY + 2);
  constexpr int NHALO = 2 * WD + 2 * TY;
  constexpr int HPT = (NHALO + NT - 1) / NT;  // halo cells per lane
  constexpr int CH = C - 1;                   // clusters whose H is gathered
  constexpr int NV = STEP ? 2 * C + 1 : 1;

  __shared__ float s_x[2][NCELL];
  __shared__ __align__(16) float s_u[2][NCELL * CP];
  __shared__ float s_red[(NT / 64) * NV];
  __shared__ double s_redd[(NT / 64) * NV];
  __shared__ int s_flag;

  const int tid = threadIdx.x;
  const int tx = tid & 63, ty = tid >> 6;
  const int own_cell = (ty + 1) * WD + (tx + 1);
  // eq (7) weights by offset class: in-plane edge / corner (q = 1, 2) and
  // off-plane centre / edge / corner (q = 1, 2, 3); q^2 or q.
  const float wEa = 1.f, wCa = a.q2_sqdist ? 2.f : 4.f;
  const float wPb = 1.f, wEb = a.q2_sqdist ? 2.f : 4.f, wCb = a.q2_sqdist ? 3.f : 9.f;

  int h_cy[HPT], h_cx[HPT];
  bool h_ok[HPT];
#pragma unroll
  for (int k = 0; k < HPT; ++k) {
    const int h = tid + k * NT;
    h_ok[k] = h < NHALO;
    int cy, cx;
    if (h < WD) { cy = 0; cx = h; }
    else if (h < 2 * WD) { cy = TY + 1; cx = h - WD; }
    else if (h < 2 * WD + TY) { cy = 1 + (h - 2 * WD); cx = 0; }
    else { cy = 1 + (h - 2 * WD - TY); cx = WD - 1; }
    h_cy[k] = cy;
    h_cx[k] = cx;
  }

  int first, end, step;
  item_range(a.nitems, first, end, step);
  for (int it = first; it < end; it += step) {
    const int b = vol_of_item(a, it);
    const VolDev vd = a.vols[b];
    const int r = it - a.item_begin[b];
    const int pidx = r / vd.tiles;
    const int tile = r - pidx * vd.tiles;
    const PairDev pr = a.pairs[b * a.P + pidx];
    SolveState* st = pr.st;
    if (STEP && st->stop) continue;
    const int t = STEP ? st->iter + 1 : st->iter;
    const float* __restrict__ Uin = STEP ? u_in_of(pr, t) : u_state_of(pr, t);
    float* __restrict__ Uout = STEP ? u_out_of(pr, t) : nullptr;
    float cj[C];
#pragma unroll
    for (int j = 0; j < C; ++j) cj[j] = st->c[(STEP ? t - 1 : t) & 1][j];
    const float lam = st->lam, xi = st->xi;
    const float* __restrict__ X = vd.x;
    const float* __restrict__ IG = vd.invg;
    const int nx = vd.nx, ny = vd.ny, nz = vd.nz;

    const int txi = tile % vd.ntx;
    const int rest = tile / vd.ntx;
    const int tyi = rest % vd.nty;
    const int tzi = rest / vd.nty;
    const int x0 = txi * kTX, y0 = tyi * TY;
    const int zlo = tzi * vd.zc, zhi = min(zlo + vd.zc, nz);
    const int gx = x0 + tx, gy = y0 + ty;
    const bool active = gx < nx && gy < ny;
    const size_t plane_sz = (size_t)nx * ny;
    const size_t own_xy = (size_t)gy * nx + gx;

    // Denominator of eq (7) for this column: in-plane neighbours give
    // edges e and corners e_x * e_y, each of the az existing off-planes a
    // centre, e edges and e_x * e_y corners.
    float invQ[3];
    {
      const int ex = (gx > 0) + (gx < nx - 1), ey = (gy > 0) + (gy < ny - 1);
      const float e = (float)(ex + ey), co = (float)(ex * ey);
      const float q0 = wEa * e + wCa * co, q1 = wPb + wEb * e + wCb * co;
#pragma unroll
      for (int az = 0; az < 3; ++az) {
        const float q = q0 + (float)az * q1;
        invQ[az] = q > 0.f ? 1.f / q : 0.f;
      }
    }

    // Register sets for planes in flight (two planes ahead).
    float rx[2], rg[2], ru[2][C], rhx[2][HPT], rhu[2][HPT][C];
    auto load_plane = [&](int q, float& ox, float& og, float (&ou)[C], float (&hx)[HPT],
                          float (&hu)[HPT][C]) __attribute__((always_inline)) {
      const bool pv = q >= 0 && q < nz;
      const size_t base = (size_t)q * plane_sz;
      if (pv && active) {
        const size_t i = base + own_xy;
        ox = X[i];
        og = IG[i];
        load_row<C>(Uin + i * C, ou);
      } else {
        ox = 0.f;
        og = 1.f;
#pragma unroll
        for (int j = 0; j < C; ++j) ou[j] = 0.f;
      }
#pragma unroll
      for (int k = 0; k < HPT; ++k) {
        const int hx_ = x0 - 1 + h_cx[k], hy_ = y0 - 1 + h_cy[k];
        const bool ok = pv && h_ok[k] && hx_ >= 0 && hx_ < nx && hy_ >= 0 && hy_ < ny;
        if (ok) {
          const size_t i = base + (size_t)hy_ * nx + hx_;
          hx[k] = X[i];
          load_row<C>(Uin + i * C, hu[k]);
        } else {
          hx[k] = 0.f;
#pragma unroll
          for (int j = 0; j < C; ++j) hu[k][j] = 0.f;
        }
      }
    };
    auto store_plane = [&](int buf, const float& ox, const float (&ou)[C], const float (&hx)[HPT],
                           const float (&hu)[HPT][C]) __attribute__((always_inline)) {
      s_x[buf][own_cell] = ox;
      lds_cell_store<C, CP>(&s_u[buf][own_cell * CP], ou);
#pragma unroll
      for (int k = 0; k < HPT; ++k) {
        if (h_ok[k]) {
          const int cell = h_cy[k] * WD + h_cx[k];
          s_x[buf][cell] = hx[k];
          lds_cell_store<C, CP>(&s_u[buf][cell * CP], hu[k]);
        }
      }
    };

    // Slots of the three voxels in flight.
    float hn[3][CH > 0 ? CH : 1], fn[3][C], xs[3], gs[3], us[3][C];
    float acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = 0.f;

    // Finalise voxel z of slot S: eqs (5)/(7) ratios, (4), (1), (2), (3).
    auto finalize = [&](int z, const float (&h)[CH > 0 ? CH : 1], const float (&f)[C], float xv,
                        float ig, const float (&uo)[C]) __attribute__((always_inline)) {
      if (!active) return;
      const int az = (z > 0) + (z < nz - 1);
      const float iq = invQ[az];
      float H[C];
      if (__builtin_expect(ig >= 0.f, 1)) {
        float sh = 0.f;
#pragma unroll
        for (int j = 0; j < CH; ++j) {
          H[j] = h[j] * ig;
          sh += H[j];
        }
        H[C - 1] = 1.f - sh;
      } else {
        // Every neighbour has the voxel's own intensity: eq (5) in the
        // equal-weight limit, the plain mean of the neighbours' memberships.
        float sum[C];
#pragma unroll
        for (int j = 0; j < C; ++j) sum[j] = 0.f;
        int cnt = 0;
        for (int dz = -1; dz <= 1; ++dz)
          for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
              const int X2 = gx + dx, Y2 = gy + dy, Z2 = z + dz;
              if ((dx | dy | dz) == 0 || X2 < 0 || X2 >= nx || Y2 < 0 || Y2 >= ny || Z2 < 0 ||
                  Z2 >= nz)
                continue;
              float u2[C];
              load_row<C>(Uin + (((size_t)Z2 * ny + Y2) * nx + X2) * C, u2);
#pragma unroll
              for (int j = 0; j < C; ++j) sum[j] += u2[j];
              ++cnt;
            }
        const float ic = cnt > 0 ? 1.f / (float)cnt : 0.f;
#pragma unroll
        for (int j = 0; j < C; ++j) H[j] = sum[j] * ic;
      }
      float d2[C];
      float Jv = 0.f;
#pragma unroll
      for (int j = 0; j < C; ++j) {
        const float av = fmaf(-lam, H[j], fmaf(-xi, f[j] * iq, 1.f));  // eq (4) factor
        const float dd = xv - cj[j];
        d2[j] = fmaxf(dd * dd * av, kDFloor);
        Jv = fmaf(pow_m<M2>(uo[j], a.m), d2[j], Jv);  // eq (1)
      }
      if constexpr (STEP) {
        float un[C];
        memberships<C, M2>(d2, a.m, un);  // eq (2)
        const size_t i = (size_t)z * plane_sz + own_xy;
        store_row<C>(Uout + i * C, un);
#pragma unroll
        for (int j = 0; j < C; ++j) {
          const float w = pow_m<M2>(un[j], a.m);
          acc[j] = fmaf(w, xv, acc[j]);  // eq (3) numerator
          acc[C + j] += w;                // eq (3) denominator
        }
        acc[2 * C] += Jv;
      } else {
        acc[0] += Jv;
      }
    };

    // One plane p: contributions of its 3x3 cells to voxels p-1 (slot SA),
    // p (SB), p+1 (SC); then finalise p-1, stage plane p+1, prefetch p+3.
    auto plane = [&](int p, auto SAc, auto SBc, auto SCc, auto S1c) __attribute__((always_inline)) {
      constexpr int SA = decltype(SAc)::value, SB = decltype(SBc)::value;
      constexpr int SC = decltype(SCc)::value, S1 = decltype(S1c)::value;
      __syncthreads();
      const bool pv = p >= 0 && p < nz;
      const bool doA = p - 1 >= zlo;
      const bool doB = p >= zlo && p < zhi;
      const bool doC = p + 1 < zhi;
      if (pv) {
        const float* __restrict__ sx = s_x[p & 1];
        const float* __restrict__ su = s_u[p & 1];
        float E[C], Co[C], Pc[C];
        float hA[CH > 0 ? CH : 1], hB[CH > 0 ? CH : 1], hC[CH > 0 ? CH : 1];
#pragma unroll
        for (int j = 0; j < C; ++j) E[j] = Co[j] = Pc[j] = 0.f;
#pragma unroll
        for (int j = 0; j < CH; ++j) hA[j] = hB[j] = hC[j] = 0.f;
        const float xA = xs[SA], xB = xs[SB], xC = rx[S1];
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy) {
#pragma unroll
          for (int dx = -1; dx <= 1; ++dx) {
            const int cell = own_cell + dy * WD + dx;
            const float xk = sx[cell];
            float u[C];
            lds_cell_load<C, CP>(su + cell * CP, u);
            const int n = (dx != 0) + (dy != 0);
#pragma unroll
            for (int j = 0; j < C; ++j) {
              if (n == 0) Pc[j] = u[j] * u[j];
              else if (n == 1) E[j] = fmaf(u[j], u[j], E[j]);
              else Co[j] = fmaf(u[j], u[j], Co[j]);
            }
            if (doA) {
              const float g = fabsf(xA - xk);  // eq (6)
#pragma unroll
              for (int j = 0; j < CH; ++j) hA[j] = fmaf(u[j], g, hA[j]);
            }
            if (doB && n != 0) {
              const float g = fabsf(xB - xk);
#pragma unroll
              for (int j = 0; j < CH; ++j) hB[j] = fmaf(u[j], g, hB[j]);
            }
            if (doC) {
              const float g = fabsf(xC - xk);
#pragma unroll
              for (int j = 0; j < CH; ++j) hC[j] = fmaf(u[j], g, hC[j]);
            }
          }
        }
        float Sa[C], Sb[C];
#pragma unroll
        for (int j = 0; j < C; ++j) {
          Sa[j] = fmaf(wCa, Co[j], wEa * E[j]);
          Sb[j] = fmaf(wCb, Co[j], fmaf(wEb, E[j], wPb * Pc[j]));
        }
        if (doA) {
#pragma unroll
          for (int j = 0; j < CH; ++j) hn[SA][j] += hA[j];
#pragma unroll
          for (int j = 0; j < C; ++j) fn[SA][j] += Sb[j];
        }
        if (doB) {
#pragma unroll
          for (int j = 0; j < CH; ++j) hn[SB][j] += hB[j];
#pragma unroll
          for (int j = 0; j < C; ++j) fn[SB][j] += Sa[j];
        }
        if (doC) {
#pragma unroll
          for (int j = 0; j < CH; ++j) hn[SC][j] = hC[j];
#pragma unroll
          for (int j = 0; j < C; ++j) fn[SC][j] = Sb[j];
        }
      } else if (doC) {
#pragma unroll
        for (int j = 0; j < CH; ++j) hn[SC][j] = 0.f;
#pragma unroll
        for (int j = 0; j < C; ++j) fn[SC][j] = 0.f;
      }
      if (doA) finalize(p - 1, hn[SA], fn[SA], xs[SA], gs[SA], us[SA]);
      if (p + 1 <= zhi) {
        store_plane((p + 1) & 1, rx[S1], ru[S1], rhx[S1], rhu[S1]);
        xs[SC] = rx[S1];
        gs[SC] = rg[S1];
#pragma unroll
        for (int j = 0; j < C; ++j) us[SC][j] = ru[S1][j];
        if (p + 3 <= zhi) load_plane(p + 3, rx[S1], rg[S1], ru[S1], rhx[S1], rhu[S1]);
      }
    };

    // Prologue: planes zlo-1 (staged), zlo and zlo+1 (in flight).
    load_plane(zlo - 1, rx[0], rg[0], ru[0], rhx[0], rhu[0]);
    load_plane(zlo, rx[1], rg[1], ru[1], rhx[1], rhu[1]);
    __syncthreads();  // previous item's last plane reads are done
    store_plane((zlo - 1) & 1, rx[0], ru[0], rhx[0], rhu[0]);
    if (zlo + 1 <= zhi) load_plane(zlo + 1, rx[0], rg[0], ru[0], rhx[0], rhu[0]);
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      xs[s] = 0.f;
      gs[s] = 1.f;
#pragma unroll
      for (int j = 0; j < CH; ++j) hn[s][j] = 0.f;
#pragma unroll
      for (int j = 0; j < C; ++j) fn[s][j] = us[s][j] = 0.f;
    }

    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    for (int p = zlo - 1; p <= zhi; p += 6) {
      plane(p, I2{}, I0{}, I1{}, I1{});
      if (p + 1 > zhi) break;
      plane(p + 1, I0{}, I1{}, I2{}, I0{});
      if (p + 2 > zhi) break;
      plane(p + 2, I1{}, I2{}, I0{}, I1{});
      if (p + 3 > zhi) break;
      plane(p + 3, I2{}, I0{}, I1{}, I0{});
      if (p + 4 > zhi) break;
      plane(p + 4, I0{}, I1{}, I2{}, I1{});
      if (p + 5 > zhi) break;
      plane(p + 5, I1{}, I2{}, I0{}, I0{});
    }

    tile_done<C, NT, STEP>(pr, tile, vd.tiles, acc, s_red, s_redd, &s_flag);
  }
}


// Launch / occupancy of one C.  TY (rows per tile) variants exist only where
// ALL_TY is set (the C = 4 fast path); elsewhere TY = 4.
template <int C, bool M2, int TY>
static hipError_t launch_gather_ct(const LaunchArgs& a, int grid, bool step, hipStream_t s) {
  if (step) hipLaunchKernelGGL((k_ifcm_gather<C, M2, TY, true>), dim3(grid), dim3(64 * TY), 0, s, a);
  else hipLaunchKernelGGL((k_ifcm_gather<C, M2, TY, false>), dim3(grid), dim3(64 * TY), 0, s, a);
  return hipGetLastError();
}

template <int C, bool M2, int TY>
static int occ_gather_ct(bool step) {
  int n = 0;
  const void* f = step ? reinterpret_cast<const void*>(&k_ifcm_gather<C, M2, TY, true>)
                       : reinterpret_cast<const void*>(&k_ifcm_gather<C, M2, TY, false>);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, 64 * TY, 0) != hipSuccess) n = 1;
  return std::max(n, 1);
}

template <int C, bool ALL_TY>
static hipError_t launch_gather_one(const LaunchArgs& a, int grid, int ty, bool m2, bool step,
                                    hipStream_t s) {
  if constexpr (ALL_TY) {
    switch (ty) {
      case 2: return m2 ? launch_gather_ct<C, true, 2>(a, grid, step, s) : launch_gather_ct<C, false, 2>(a, grid, step, s);
      case 4: return m2 ? launch_gather_ct<C, true, 4>(a, grid, step, s) : launch_gather_ct<C, false, 4>(a, grid, step, s);
      case 8: return m2 ? launch_gather_ct<C, true, 8>(a, grid, step, s) : launch_gather_ct<C, false, 8>(a, grid, step, s);
      default: return hipErrorInvalidValue;
    }
  } else {
    if (ty != 4) return hipErrorInvalidValue;
    return m2 ? launch_gather_ct<C, true, 4>(a, grid, step, s) : launch_gather_ct<C, false, 4>(a, grid, step, s);
  }
}

template <int C, bool ALL_TY>
static int occ_gather_one(int ty, bool m2, bool step) {
  if constexpr (ALL_TY) {
    switch (ty) {
      case 2: return m2 ? occ_gather_ct<C, true, 2>(step) : occ_gather_ct<C, false, 2>(step);
      case 4: return m2 ? occ_gather_ct<C, true, 4>(step) : occ_gather_ct<C, false, 4>(step);
      case 8: return m2 ? occ_gather_ct<C, true, 8>(step) : occ_gather_ct<C, false, 8>(step);
      default: return 1;
    }
  } else {
    return m2 ? occ_gather_ct<C, true, 4>(step) : occ_gather_ct<C, false, 4>(step);
  }
}

// One translation unit per group of C defines these for its C values.
#define PIFCM_DEFINE_GATHER(c, all_ty)                                                     \
  hipError_t launch_gather_C##c(const LaunchArgs& a, int grid, int ty, bool m2, bool step, \
                                hipStream_t s) {                                           \
    return launch_gather_one<c, all_ty>(a, grid, ty, m2, step, s);                         \
  }                                                                                        \
  int occ_gather_C##c(int ty, bool m2, bool step) { return occ_gather_one<c, all_ty>(ty, m2, step); }

}  // namespace pifcm
