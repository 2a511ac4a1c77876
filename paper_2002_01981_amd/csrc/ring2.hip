// ring2.hip -- the IFCM step for the two Chebyshev rings of the 5x5x5 cube
// (V = 2, eq (10) weights W_1, W_2), fused like the 3x3x3 step, for C <= 4.
//
// Per voxel i and ring r (the cells at Chebyshev distance r):
//   H_ij = sum_r W_r g_inv_ir sum_{k in r} u_kj g_ik    (eqs (5), (6), (10))
//   F_ij = sum_r W_r q_inv_ir sum_{k in r} u_kj^2 q_ik  (eqs (7), (8), (10))
// with g_inv_ir = 1 / sum_{k in r} g_ik and q_inv_ir = 1 / sum_{k in r} q_ik.
// Both depend on x only and are computed once per call (k_ring2_invariants);
// a ring whose cells all share the voxel's intensity stores -1 / n_r and its
// centre value is shifted by -1 when forming g, so every g_ik of it is 1 and
// the ring contributes the mean of its memberships (the equal-weight limit).
//
// Work decomposition: as in the fused step, a wave owns a tile of 16 x 4
// columns and zc planes and walks it along z.  Each plane of the tile plus a
// two-voxel halo (20 x 8 cells of x and U) is staged once in the wave's LDS
// (four plane buffers), and every lane reads its 5 x 5 in-plane cells once:
// they contribute to the five voxels of its column at planes p-2 .. p+2, kept
// in five register slots that move down by one after each plane (a version
// that renames the slots over five unrolled planes needs more than 512
// registers).  For F the squared memberships of the 25
// cells are summed per in-plane offset class once per plane and weighted per
// slot.  The last cluster's H comes from sum_j H_ij = sum_r W_r (rows of U
// sum to 1).  Voxel p-2 is complete after plane p and is finalised: eqs (4),
// (1), (2), (3) as in the fused step.
#include "common.h"
#include "pifcm_kernels.h"

namespace pifcm {

__global__ __launch_bounds__(256) void k_ring2_invariants(const float* __restrict__ x,
                                                          float* __restrict__ rinv, int nx, int ny,
                                                          int nz, int q2_sqdist) {
  const size_t N = (size_t)nx * ny * nz;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (size_t)gridDim.x * blockDim.x) {
    const int gx = (int)(i % nx);
    const size_t rr = i / nx;
    const int gy = (int)(rr % ny);
    const int gz = (int)(rr / ny);
    const float xi = x[i];
    float gs[2] = {0.f, 0.f}, qs[2] = {0.f, 0.f};
    int cnt[2] = {0, 0};
    for (int dz = -2; dz <= 2; ++dz)
      for (int dy = -2; dy <= 2; ++dy)
        for (int dx = -2; dx <= 2; ++dx) {
          const int X2 = gx + dx, Y2 = gy + dy, Z2 = gz + dz;
          if ((dx | dy | dz) == 0 || X2 < 0 || X2 >= nx || Y2 < 0 || Y2 >= ny || Z2 < 0 || Z2 >= nz)
            continue;
          const int r = max(abs(dx), max(abs(dy), abs(dz))) - 1;
          const int s2 = dx * dx + dy * dy + dz * dz;
          gs[r] += fabsf(xi - x[((size_t)Z2 * ny + Y2) * nx + X2]);
          qs[r] += q2_sqdist ? (float)s2 : (float)(s2 * s2);
          ++cnt[r];
        }
    float o[4];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      o[r] = gs[r] > 0.f ? 1.f / gs[r] : (cnt[r] > 0 ? -1.f / (float)cnt[r] : 0.f);
      o[2 + r] = cnt[r] > 0 ? 1.f / qs[r] : 0.f;
    }
    store_row<4>(as_global(rinv) + i * 4, o);
  }
}

hipError_t launch_ring2_invariants(const float* x, float* rinv, int nx, int ny, int nz, int q2_sqdist,
                                   hipStream_t s) {
  const size_t N = (size_t)nx * ny * nz;
  const int grid = (int)std::min<size_t>((N + 255) / 256, 65536);
  hipLaunchKernelGGL(k_ring2_invariants, dim3(grid), dim3(256), 0, s, x, rinv, nx, ny, nz, q2_sqdist);
  return hipGetLastError();
}

namespace r2 {
constexpr int TX = 16, TY = 4, HX = TX + 4, HY = TY + 4;
constexpr int NCELL = HX * HY;  // 160 cells per staged plane
constexpr int NHALO = NCELL - 64;  // 96 halo cells: one per lane, a second for lanes 0..31
constexpr int NBUF = 4;
// In-plane offset classes (|dx|, |dy|) sorted: (0,0) (0,1) (1,1) (0,2) (1,2) (2,2).
__host__ __device__ constexpr int cls(int a, int b) {
  return (a > b ? cls(b, a) : (b < 2 ? a + b : 3 + a));
}
__host__ __device__ constexpr int cls_a(int c) { return c == 2 ? 1 : c == 4 ? 1 : c == 5 ? 2 : 0; }
__host__ __device__ constexpr int cls_b(int c) { return c == 0 ? 0 : c <= 2 ? 1 : 2; }
static_assert(cls(0, 0) == 0 && cls(1, 0) == 1 && cls(1, 1) == 2, "classes");
static_assert(cls(2, 0) == 3 && cls(1, 2) == 4 && cls(2, 2) == 5, "classes");
static_assert(cls_a(4) == 1 && cls_b(4) == 2 && cls_a(3) == 0 && cls_b(3) == 2, "class members");
// Halo cell h (0 .. 95) of the 20 x 8 staged plane: two rows above, two
// below, two columns on each side of the 16 x 4 tile.
__device__ __forceinline__ void halo_cell(int h, int& cx, int& cy) {
  if (h < 2 * HX) {
    cy = h / HX;
    cx = h - cy * HX;
  } else if (h < 4 * HX) {
    const int k = h - 2 * HX;
    cy = TY + 2 + k / HX;
    cx = k % HX;
  } else {
    const int k = h - 4 * HX;  // 0 .. 15
    cy = 2 + ((k & 7) >> 1);
    cx = (k < 8 ? 0 : TX + 2) + (k & 1);
  }
}
// f(integral_constant<int, B>) ... f(integral_constant<int, E - 1>): the
// loop index is a constant expression, so arrays indexed by values derived
// from it stay in registers.
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}
}  // namespace r2

template <int C, bool M2, bool STEP>
__global__ __launch_bounds__(64 * kRing2Waves) void k_ifcm_ring2(const LaunchArgs a) {
  static_assert(C >= 2 && C <= 4, "the fused two-ring step holds C <= 4 clusters");
  using namespace r2;
  constexpr int CP = 4, CH = C - 1, NW = kRing2Waves;
  constexpr int NV = STEP ? 2 * C + 1 : 1;
  // One spare cell takes the second halo load of lanes that have none.
  __shared__ float s_x[NW][NBUF][NCELL + 1];
  __shared__ __align__(16) float s_u[NW][NBUF][(NCELL + 1) * CP];

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int tx = lane & (TX - 1), ty = lane / TX;
  const int own_cell = (ty + 2) * HX + (tx + 2);
  int h0x, h0y, h1x = 0, h1y = 0;
  halo_cell(lane, h0x, h0y);
  const bool has_h1 = lane + 64 < NHALO;
  if (has_h1) halo_cell(lane + 64, h1x, h1y);
  const int h0_cell = h0y * HX + h0x;
  const int h1_dst = has_h1 ? h1y * HX + h1x : NCELL;
  const float W1 = a.W[1], W2 = a.W[2];
  auto qw = [&](int s2) { return a.q2_sqdist ? (float)s2 : (float)(s2 * s2); };

  const int xcd = blockIdx.x & 7;
  const int it_end = a.xcd_begin[xcd + 1];
  const int it_step = (gridDim.x >> 3) * NW;
  for (int it = a.xcd_begin[xcd] + (blockIdx.x >> 3) * NW + wave; it < it_end; it += it_step) {
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
    const gfloat* RI = as_global(vd.rinv);
    float cj[C];
#pragma unroll
    for (int j = 0; j < C; ++j) cj[j] = ld_const(&st->c[(STEP ? t - 1 : t) & 1][j]);
    const float lam = ld_const(&st->lam), xi = ld_const(&st->xi);
    const int nx = vd.nx, ny = vd.ny, nz = vd.nz;
    const int txi = tile % vd.ntx;
    const int rest = tile / vd.ntx;
    const int tyi = rest % vd.nty;
    const int tzi = rest / vd.nty;
    const int x0 = txi * TX, y0 = tyi * TY;
    const int zlo = vd.zbeg + tzi * vd.zc, zhi = min(zlo + vd.zc, vd.zend);
    const int gx = x0 + tx, gy = y0 + ty;
    const bool active = gx < nx && gy < ny;
    auto in_xy = [&](int cx, int cy) {
      const int hx = x0 - 2 + cx, hy = y0 - 2 + cy;
      return hx >= 0 && hx < nx && hy >= 0 && hy < ny;
    };
    const bool v0 = in_xy(h0x, h0y), v1 = has_h1 && in_xy(h1x, h1y);
    const size_t psz = (size_t)nx * ny;
    const size_t own_xy = active ? (size_t)gy * nx + gx : 0;
    const size_t h0_xy = v0 ? (size_t)(y0 - 2 + h0y) * nx + (x0 - 2 + h0x) : 0;
    const size_t h1_xy = v1 ? (size_t)(y0 - 2 + h1y) * nx + (x0 - 2 + h1x) : 0;
    auto bufof = [&](int q) { return (q - zlo + 2) & (NBUF - 1); };

    // Prefetch registers of the next staged plane (own cell, two halo cells)
    // and of the lane's own intensity and ring invariants two planes ahead.
    float px, pu[C], qx0, qu0[C], qx1, qu1[C];
    float ox, ri[4];
    auto load_cells = [&](int q) __attribute__((always_inline)) {
      const bool pv = q >= 0 && q < nz;
      const size_t pofs = pv ? (size_t)q * psz : 0;
      px = qx0 = qx1 = 0.f;
#pragma unroll
      for (int j = 0; j < C; ++j) pu[j] = qu0[j] = qu1[j] = 0.f;
      if (pv && active) {
        px = X[pofs + own_xy];
        load_row<C>(Uin + (pofs + own_xy) * C, pu);
      }
      if (pv && v0) {
        qx0 = X[pofs + h0_xy];
        load_row<C>(Uin + (pofs + h0_xy) * C, qu0);
      }
      if (pv && v1) {
        qx1 = X[pofs + h1_xy];
        load_row<C>(Uin + (pofs + h1_xy) * C, qu1);
      }
    };
    auto load_own = [&](int q) __attribute__((always_inline)) {
      const bool pv = q >= 0 && q < nz;
      ox = 0.f;
      ri[0] = ri[1] = ri[2] = ri[3] = 0.f;
      if (pv && active) {
        const size_t i = (size_t)q * psz + own_xy;
        ox = X[i];
        load_row<4>(RI + i * 4, ri);
      }
    };
    auto store_cells = [&](int buf) __attribute__((always_inline)) {
      float* sx = &s_x[wave][buf][0];
      float* su = &s_u[wave][buf][0];
      sx[own_cell] = px;
      lds_cell_store<C, CP>(su + own_cell * CP, pu);
      sx[h0_cell] = qx0;
      lds_cell_store<C, CP>(su + h0_cell * CP, qu0);
      sx[h1_dst] = qx1;
      lds_cell_store<C, CP>(su + h1_dst * CP, qu1);
    };

    // Slots of the voxels p-2 .. p+2 of the lane's column, per ring: H
    // numerators (first C - 1 clusters), F numerators, and the centre value,
    // g_inv and q_inv of the slot's voxel.
    float hn[5][2][CH], fn[5][2][C], xcs[5][2], gis[5][2], qis[5][2];
    float acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = 0.f;
#pragma unroll
    for (int s5 = 0; s5 < 5; ++s5)
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        xcs[s5][q] = gis[s5][q] = qis[s5][q] = 0.f;
#pragma unroll
        for (int j = 0; j < CH; ++j) hn[s5][q][j] = 0.f;
#pragma unroll
        for (int j = 0; j < C; ++j) fn[s5][q][j] = 0.f;
      }

    auto finalize = [&](int z, auto Sc, int bz) __attribute__((always_inline)) {
      constexpr int S = decltype(Sc)::value;
      const float xv = s_x[wave][bz][own_cell];
      float uo[C];
      lds_cell_load<C, CP>(&s_u[wave][bz][own_cell * CP], uo);
      float H[C], F[C];
#pragma unroll
      for (int j = 0; j < C; ++j) H[j] = F[j] = 0.f;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const float w = q == 0 ? W1 : W2;
        const float gi = gis[S][q];
        float sh = 0.f;
#pragma unroll
        for (int j = 0; j < CH; ++j) {
          const float h = hn[S][q][j] * gi;
          H[j] = fmaf(w, h, H[j]);
          sh += h;
        }
        // The ring's ratios sum to 1 over the clusters (0 for a ring without cells).
        H[C - 1] = fmaf(gi != 0.f ? w : 0.f, 1.f - sh, H[C - 1]);
        const float wq = w * qis[S][q];
#pragma unroll
        for (int j = 0; j < C; ++j) F[j] = fmaf(wq, fn[S][q][j], F[j]);
      }
      float d2[C];
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
        if (active) store_row<C>(Uout + ((size_t)z * psz + own_xy) * C, un);
#pragma unroll
        for (int j = 0; j < C; ++j) {
          const float w = active ? pow_m<M2>(un[j], a.m) : 0.f;
          acc[j] = fmaf(w, xv, acc[j]);  // eq (3)
          acc[C + j] += w;
        }
        acc[2 * C] += Jv;  // 0 for a lane outside: its staged memberships are 0
      } else {
        acc[0] += Jv;
      }
    };

    // One plane p: its 5 x 5 cells added to the voxels p-2 .. p+2 (slots
    // rotated by ROT), the slot of p+2 started, plane p+1 staged, p+2 and the own
    // values of p+3 prefetched, voxel p-2 finalised.  GEN: the tile's first
    // and last planes, with the validity tests.
    auto plane = [&](int p, auto ROTc, auto GENc) __attribute__((always_inline)) {
      constexpr int ROT = decltype(ROTc)::value;
      constexpr bool GEN = decltype(GENc)::value;
      // Slots of voxels p - 2 (finalised) and p + 2 (started).
      constexpr int S0 = ROT % 5, S4 = (4 + ROT) % 5;
      const bool pv = !GEN || (p >= 0 && p < nz);
      // Start voxel p+2 (its own values were prefetched).
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        xcs[S4][q] = ri[q] < 0.f ? ox - 1.f : ox;
        gis[S4][q] = fabsf(ri[q]);
        qis[S4][q] = ri[2 + q];
#pragma unroll
        for (int j = 0; j < CH; ++j) hn[S4][q][j] = 0.f;
#pragma unroll
        for (int j = 0; j < C; ++j) fn[S4][q][j] = 0.f;
      }
      if (pv) {
        const int bp = bufof(p);
        const float* sx = &s_x[wave][bp][own_cell];
        const float* su = &s_u[wave][bp][own_cell * CP];
        float cs[6][C];
#pragma unroll
        for (int c = 0; c < 6; ++c)
#pragma unroll
          for (int j = 0; j < C; ++j) cs[c][j] = 0.f;
        static_for<0, 5>([&](auto yc) {
          constexpr int dy = decltype(yc)::value - 2;
          static_for<0, 5>([&](auto xc) {
            constexpr int dx = decltype(xc)::value - 2;
            constexpr int ad = dx < 0 ? -dx : dx, bd = dy < 0 ? -dy : dy;
            const float xk = sx[dy * HX + dx];
            float u[C];
            lds_cell_load<C, CP>(su + (dy * HX + dx) * CP, u);
            constexpr int c = cls(ad, bd);
#pragma unroll
            for (int j = 0; j < C; ++j) cs[c][j] = fmaf(u[j], u[j], cs[c][j]);
            static_for<0, 5>([&](auto kc) {
              constexpr int k = decltype(kc)::value;
              constexpr int dz = 2 - k, ed = dz < 0 ? -dz : dz;
              if constexpr (!(dx == 0 && dy == 0 && dz == 0)) {
                constexpr int q = (ad > bd ? (ad > ed ? ad : ed) : (bd > ed ? bd : ed)) - 1;
                constexpr int sk = (k + ROT) % 5;
                const float g = fabsf(xcs[sk][q] - xk);  // eq (6)
#pragma unroll
                for (int j = 0; j < CH; ++j) hn[sk][q][j] = fmaf(u[j], g, hn[sk][q][j]);
              }
            });
          });
          // One row of cells at a time: keeps the row's LDS reads, not the
          // whole window's, in registers.
          __builtin_amdgcn_sched_barrier(0);
        });
        // eq (7): the class sums, weighted per slot.
        static_for<0, 5>([&](auto kc) {
          constexpr int k = decltype(kc)::value;
          constexpr int ed = k < 2 ? 2 - k : k - 2, sk = (k + ROT) % 5;
          static_for<0, 6>([&](auto cc) {
            constexpr int c = decltype(cc)::value;
            constexpr int ad = cls_a(c), bd = cls_b(c);
            if constexpr (!(ad == 0 && bd == 0 && ed == 0)) {
              constexpr int q = (ad > bd ? (ad > ed ? ad : ed) : (bd > ed ? bd : ed)) - 1;
              const float wgt = qw(ad * ad + bd * bd + ed * ed);
#pragma unroll
              for (int j = 0; j < C; ++j) fn[sk][q][j] = fmaf(wgt, cs[c][j], fn[sk][q][j]);
            }
          });
        });
      }
      __builtin_amdgcn_sched_barrier(0);
      if (!GEN || p + 1 <= zhi + 1) {
        store_cells(bufof(p + 1));
        if (!GEN || p + 2 <= zhi + 1) load_cells(p + 2);
      }
      if (!GEN || p + 3 <= zhi + 1) load_own(p + 3);
      if (!GEN || (p - 2 >= zlo && p - 2 < zhi)) finalize(p - 2, std::integral_constant<int, S0>{}, bufof(p - 2));
      __builtin_amdgcn_sched_barrier(0);
    };
    auto shift = [&]() __attribute__((always_inline)) {
#pragma unroll
      for (int s5 = 0; s5 < 4; ++s5)
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          xcs[s5][q] = xcs[s5 + 1][q];
          gis[s5][q] = gis[s5 + 1][q];
          qis[s5][q] = qis[s5 + 1][q];
#pragma unroll
          for (int j = 0; j < CH; ++j) hn[s5][q][j] = hn[s5 + 1][q][j];
#pragma unroll
          for (int j = 0; j < C; ++j) fn[s5][q][j] = fn[s5 + 1][q][j];
        }
    };

    using I0 = std::integral_constant<int, 0>;
    using Gen = std::integral_constant<bool, true>;
    using Steady = std::integral_constant<bool, false>;

    // Prologue: plane zlo-2 staged, zlo-1 prefetched, the own values of zlo
    // (the voxel that enters at plane zlo-2) prefetched.
    load_cells(zlo - 2);
    store_cells(bufof(zlo - 2));
    load_cells(zlo - 1);
    load_own(zlo);
    int p = zlo - 2;
    for (; p < zlo + 2; ++p) {
      plane(p, I0{}, Gen{});
      shift();
    }
    // Interior planes: every per-plane test is true (the loads still test
    // the plane range).  tests/test_plane_walk.py replays this walk.
    for (; p + 4 <= zhi; ++p) {
      plane(p, I0{}, Steady{});
      shift();
    }
    for (; p <= zhi + 1; ++p) {
      plane(p, I0{}, Gen{});
      shift();
    }
    wave_tile_store<NV>(pr, tile, acc);
  }
}

template <int C, bool M2>
static hipError_t launch_ring2_ct(const LaunchArgs& a, int grid, bool step, hipStream_t s) {
  if (step) hipLaunchKernelGGL((k_ifcm_ring2<C, M2, true>), dim3(grid), dim3(64 * kRing2Waves), 0, s, a);
  else hipLaunchKernelGGL((k_ifcm_ring2<C, M2, false>), dim3(grid), dim3(64 * kRing2Waves), 0, s, a);
  return hipGetLastError();
}

template <int C, bool M2>
static int occ_ring2_ct(bool step) {
  int n = 0;
  const void* f = step ? reinterpret_cast<const void*>(&k_ifcm_ring2<C, M2, true>)
                       : reinterpret_cast<const void*>(&k_ifcm_ring2<C, M2, false>);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, 64 * kRing2Waves, 0) != hipSuccess) n = 1;
  return std::max(1, n);
}

hipError_t launch_ring2(int C, const LaunchArgs& a, int grid, bool m2, bool step, hipStream_t s) {
  switch (C) {
    case 2: return m2 ? launch_ring2_ct<2, true>(a, grid, step, s) : launch_ring2_ct<2, false>(a, grid, step, s);
    case 3: return m2 ? launch_ring2_ct<3, true>(a, grid, step, s) : launch_ring2_ct<3, false>(a, grid, step, s);
    case 4: return m2 ? launch_ring2_ct<4, true>(a, grid, step, s) : launch_ring2_ct<4, false>(a, grid, step, s);
    default: return hipErrorInvalidValue;
  }
}

int ring2_occupancy(int C, bool m2, bool step) {
  switch (C) {
    case 2: return m2 ? occ_ring2_ct<2, true>(step) : occ_ring2_ct<2, false>(step);
    case 3: return m2 ? occ_ring2_ct<3, true>(step) : occ_ring2_ct<3, false>(step);
    case 4: return m2 ? occ_ring2_ct<4, true>(step) : occ_ring2_ct<4, false>(step);
    default: return 1;
  }
}

}  // namespace pifcm
