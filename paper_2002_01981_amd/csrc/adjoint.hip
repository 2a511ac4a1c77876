// adjoint.hip -- reverse mode of the IFCM iteration (ifcm_backward).
//
// The objective is J_K = J(U^K, c^K) of eq (1) after K iterations from a
// fixed U^0.  One iteration maps (U, c) to (U', c') through eqs (4)-(10),
// (2), (3); with, per voxel i and cluster j,
//   H_ij = g_inv_i sum_k u_kj g_ik        (eq (5); g = 1 and g_inv = 1/n for
//                                          a flat neighbourhood)
//   F_ij = q_inv_i sum_k u_kj^2 q_ik      (eq (7))
//   a_ij = 1 - lambda H_ij - xi F_ij      (eq (4))
//   e_ij = (x_i - c_j)^2 a_ij,  d_ij = max(e_ij, 1e-12)
//   w_ij = d_ij^(-1/(m-1)), s_i = sum_j w_ij, u'_ij = w_ij / s_i   (eq (2))
//   c'_j = A_j / B_j, A_j = sum_i u'_ij^m x_i, B_j = sum_i u'_ij^m  (eq (3))
// the adjoint of one iteration, given dJ/dU' and dJ/dc', is
//   du'_ij  = dJ/du'_ij + m u'_ij^(m-1) (dA_j x_i + dB_j),
//             dA_j = dc'_j / B_j, dB_j = -dc'_j c'_j / B_j
//   dw_ij   = (du'_ij - sum_k du'_ik u'_ik) / s_i
//   dd_ij   = -dw_ij w_ij / ((m-1) d_ij)
//   de_ij   = dd_ij where e_ij > 1e-12, else 0
//   da_ij   = de_ij (x_i - c_j)^2,  dc_j += -2 de_ij a_ij (x_i - c_j)
//   dlambda += -da_ij H_ij,  dxi += -da_ij F_ij
//   dU_kj   = sum_{i in NB(k)} [P_ij g_ik + 2 u_kj Q_ij q_ik]
//             with P_ij = -lambda da_ij g_inv_i, Q_ij = -xi da_ij q_inv_i
// (the neighbourhood is symmetric; g_ik is taken as the centre voxel i uses
// it, so a flat i contributes g = 1).  The objective-only pass at U^K starts
// the chain with dJ/du_ij = m u_ij^(m-1) d_ij and dd_ij = u_ij^m.
// k_adj_point does the per-voxel part (recomputing the forward values from
// (U^t, c^t)), k_adj_transpose_tiled the gather of dU; the sums of dc,
// dlambda and dxi go to per-wave slots that k_adj_finalize adds in fp64.
#include <atomic>

#include "common.h"
#include "pifcm_kernels.h"

namespace pifcm {

// Tiles of both tiled adjoint kernels: a wave owns 16 x 4 columns of a tile
// of AdjArgs::zc planes and walks it along z; each plane plus a one-voxel
// halo is staged once in the wave's LDS.
constexpr int kAdjTX = 16, kAdjTY = 4, kAdjHX = kAdjTX + 2, kAdjHY = kAdjTY + 2;
constexpr int kAdjCells = kAdjHX * kAdjHY;   // 108 cells per staged plane
constexpr int kAdjHalo = kAdjCells - 64;     // 44 halo cells, one per lane
constexpr int kAdjMinZc = 32;                // shallowest tile depth (fewer planes only when nz is)
// Waves per work group: as many (up to 4) as the staged planes of each wave
// leave room for in LDS.
constexpr int kAdjPW = 4;                    // waves per work group of k_adj_point

// Inverse of the denominator of eq (7) for voxel (gx, gy, gz): the weights of
// its in-volume neighbours summed from its position (in-plane edges weigh 1,
// in-plane corners wCa; per existing off-plane the centre 1, edges wEb,
// corners wCb).  The per-voxel kernel forms the three values of its column
// (by the number of existing off-planes: 0, 1, 2) once per tile and picks
// one per plane (adj_qinv_column, adj_qinv_at); the transpose, which needs
// them for its halo cells too, forms each cell's one value as it stages it
// (adj_qinv_cell; measured faster there than carrying six values).  The
// expressions are the same, so the transpose rebuilds Q bit for bit.
struct AdjQinv {
  float v[3];
};
__device__ __forceinline__ AdjQinv adj_qinv_column(int gx, int gy, int nx, int ny, float wCa, float wEb,
                                                   float wCb) {
  const int ex = (gx > 0) + (gx < nx - 1), ey = (gy > 0) + (gy < ny - 1);
  const float e = (float)(ex + ey), co = (float)(ex * ey);
  const float q0 = e + wCa * co, q1 = 1.f + wEb * e + wCb * co;
  AdjQinv r;
  r.v[0] = q0 > 0.f ? 1.f / q0 : 0.f;
  r.v[1] = 1.f / (q0 + q1);
  r.v[2] = 1.f / (q0 + 2.f * q1);
  return r;
}
__device__ __forceinline__ float adj_qinv_at(const AdjQinv& q, int gz, int nz) {
  const int np = (gz > 0) + (gz < nz - 1);
  return np == 2 ? q.v[2] : (np == 1 ? q.v[1] : q.v[0]);
}
__device__ __forceinline__ float adj_qinv_cell(int gx, int gy, int gz, int nx, int ny, int nz, float wCa,
                                               float wEb, float wCb) {
  const int ex = (gx > 0) + (gx < nx - 1), ey = (gy > 0) + (gy < ny - 1);
  const float e = (float)(ex + ey), co = (float)(ex * ey);
  const float q0 = e + wCa * co, q1 = 1.f + wEb * e + wCb * co;
  const int np = (gz > 0) + (gz < nz - 1);
  return np == 2 ? 1.f / (q0 + 2.f * q1) : (np == 1 ? 1.f / (q0 + q1) : (q0 > 0.f ? 1.f / q0 : 0.f));
}

// The per-voxel part of the adjoint of one iteration on wave-private
// z-streaming tiles (the layout of the fused forward step): each plane of a
// tile plus its halo is staged once in the wave's LDS as (x, U) per cell,
// every lane adds its 3 x 3 in-plane cells to the H and F numerators of the
// three voxels of its column the plane touches (for F by offset class first:
// the weights of eq (7) depend only on the class), and a voxel whose three
// planes are done is finalised: it recomputes the forward values of eqs (4),
// (2) from (U^t, c^t) and applies the adjoint formulas above, writing its
// transpose source da (the transpose forms P and Q from it) and adding its
// dJ/dc, dJ/dlambda, dJ/dxi terms to the lane's sums.  Each wave leaves its sums in its own slot.
template <int C, bool M2, bool EVAL>
__global__ __launch_bounds__(64 * kAdjPW) void k_adj_point(const AdjArgs a) {
  constexpr int CP = (C + 3) / 4 * 4;
  constexpr int CW = 4 + CP;   // floats per staged cell: x (+3 pad), U
  constexpr int NV = C + 2;    // dc[C], dlambda, dxi
  __shared__ __align__(16) float s_c[kAdjPW][3][kAdjCells * CW];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int tx = lane & (kAdjTX - 1), ty = lane / kAdjTX;
  const int own_cell = (ty + 1) * kAdjHX + (tx + 1);
  int hcx, hcy;
  if (lane < kAdjHX) { hcy = 0; hcx = lane; }
  else if (lane < 2 * kAdjHX) { hcy = kAdjHY - 1; hcx = lane - kAdjHX; }
  else if (lane < 2 * kAdjHX + kAdjTY) { hcy = 1 + lane - 2 * kAdjHX; hcx = 0; }
  else { hcy = 1 + lane - 2 * kAdjHX - kAdjTY; hcx = kAdjHX - 1; }
  const bool hlane = lane < kAdjHalo;
  const int halo_cell = hlane ? hcy * kAdjHX + hcx : 0;
  // eq (7) weights by offset class (in-plane edge and off-plane centre weigh 1).
  const float wCa = a.q2_sqdist ? 2.f : 4.f;
  const float wEb = a.q2_sqdist ? 2.f : 4.f, wCb = a.q2_sqdist ? 3.f : 9.f;
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const int ntx = (nx + kAdjTX - 1) / kAdjTX, nty = (ny + kAdjTY - 1) / kAdjTY;
  const int zc = a.zc;
  const int ntz = (nz + zc - 1) / zc;
  const int nitems = ntx * nty * ntz;
  const uint32_t psz = (uint32_t)nx * (uint32_t)ny;
  const float m = a.m;

  // Scalars of the adjoint of eq (3) for this step.
  float dA[C], dB[C], cj[C];
#pragma unroll
  for (int j = 0; j < C; ++j) {
    cj[j] = a.c[j];
    if constexpr (!EVAL) {
      const double Bj = a.B_next[j];
      dA[j] = (float)(a.cbar_next[j] / Bj);
      dB[j] = (float)(-a.cbar_next[j] * (double)a.c_next[j] / Bj);
    } else {
      dA[j] = dB[j] = 0.f;
    }
  }
  float acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0.f;

  const int per = (nitems + 7) >> 3;
  const int xcd = blockIdx.x & 7;
  const int it_end = min(nitems, (xcd + 1) * per);
  const int it_step = (gridDim.x >> 3) * kAdjPW;
  for (int it = xcd * per + (blockIdx.x >> 3) * kAdjPW + wave; it < it_end; it += it_step) {
    const int txi = it % ntx;
    const int rest = it / ntx;
    const int tyi = rest % nty;
    const int tzi = rest / nty;
    const int x0 = txi * kAdjTX, y0 = tyi * kAdjTY;
    const int zlo = tzi * zc, zhi = min(zlo + zc, nz);
    const int gx = x0 + tx, gy = y0 + ty;
    const bool active = gx < nx && gy < ny;
    const int hx = x0 - 1 + hcx, hy = y0 - 1 + hcy;
    const bool hvalid = hlane && hx >= 0 && hx < nx && hy >= 0 && hy < ny;
    const size_t own_xy = active ? (size_t)gy * nx + gx : 0;
    const size_t halo_xy = hvalid ? (size_t)hy * nx + hx : 0;
    float* const sc = &s_c[wave][0][0];
    const AdjQinv qcol = adj_qinv_column(gx, gy, nx, ny, wCa, wEb, wCb);

    // Prefetch registers of one plane: own cell (x, g_inv, U, and in the
    // iteration pass dJ/dU^(t+1), which only the voxel itself reads, three
    // planes later) and halo cell.
    float rx, rg, ru[C], rgn[C], hxv, hu[C];
    auto load_plane = [&](int q) __attribute__((always_inline)) {
      const bool pv = q >= 0 && q < nz;
      if (pv && active) {
        const size_t i = (size_t)q * psz + own_xy;
        rx = a.x[i];
        rg = a.invg[i];
        load_row<C>(as_global(a.U) + i * C, ru);
        if constexpr (!EVAL) load_row<C>(as_global(a.Ubar_next) + i * C, rgn);
      } else {
        rx = 0.f;
        rg = 1.f;
#pragma unroll
        for (int j = 0; j < C; ++j) ru[j] = rgn[j] = 0.f;
      }
      if (pv && hvalid) {
        const size_t i = (size_t)q * psz + halo_xy;
        hxv = a.x[i];
        load_row<C>(as_global(a.U) + i * C, hu);
      } else {
        hxv = 0.f;
#pragma unroll
        for (int j = 0; j < C; ++j) hu[j] = 0.f;
      }
    };
    auto store_plane = [&](int buf) __attribute__((always_inline)) {
      float* base = sc + buf * kAdjCells * CW;
      base[own_cell * CW] = rx;
      lds_cell_store<C, CP>(base + own_cell * CW + 4, ru);  // offset 4 keeps the float4s aligned
      if (hlane) {
        base[halo_cell * CW] = hxv;
        lds_cell_store<C, CP>(base + halo_cell * CW + 4, hu);
      }
    };
    auto cell_at = [&](int buf, int dy, int dx) -> const float* {
      return sc + (buf * kAdjCells + own_cell + dy * kAdjHX + dx) * CW;
    };

    // Slots of the voxels p-1, p, p+1 of the lane's column: H numerators of
    // the first C - 1 clusters (the last H is 1 minus their sum, as in the
    // forward step), F numerators, the stored g_inv and (iteration pass)
    // dJ/dU^(t+1).
    constexpr int CH = C - 1;
    float hn[3][C], fn[3][C], gs[3], gns[3][C];
#pragma unroll
    for (int s2 = 0; s2 < 3; ++s2) {
      gs[s2] = 1.f;
#pragma unroll
      for (int j = 0; j < C; ++j) hn[s2][j] = fn[s2][j] = gns[s2][j] = 0.f;
    }

    auto finalize = [&](int z, int S, int bz) __attribute__((always_inline)) {
      const float* own = cell_at(bz, 0, 0);
      const float xv = own[0];
      const float gi = fabsf(gs[S]);
      const float iq = adj_qinv_at(qcol, z, nz);
      float H[C], F[C], av[C], dd[C], e[C], d[C];
      float sh = 0.f;
#pragma unroll
      for (int j = 0; j < CH; ++j) {
        H[j] = hn[S][j] * gi;
        sh += H[j];
      }
      H[CH] = gi != 0.f ? 1.f - sh : 0.f;  // sum_j H_ij = 1 (0 without neighbours)
#pragma unroll
      for (int j = 0; j < C; ++j) {
        F[j] = fn[S][j] * iq;
        av[j] = 1.f - a.lam * H[j] - a.xi * F[j];
        dd[j] = xv - cj[j];
        e[j] = dd[j] * dd[j] * av[j];
        d[j] = fmaxf(e[j], kDFloor);
      }
      const size_t i = (size_t)z * psz + own_xy;
      float dbar[C];
      if constexpr (EVAL) {
        float u[C];
        lds_cell_load<C, CP>(own + 4, u);
        float direct[C];
#pragma unroll
        for (int j = 0; j < C; ++j) {
          const float um1 = M2 ? u[j] : (u[j] > 0.f ? exp2f((m - 1.f) * log2f(u[j])) : 0.f);
          direct[j] = m * um1 * d[j];
          dbar[j] = pow_m<M2>(u[j], m);
        }
        if (active) store_row<C>(as_global(a.Ubar_direct) + i * C, direct);
      } else {
        float w[C], up[C];
        float sw = 0.f;
        if constexpr (M2) {
          // Hardware reciprocals (about 1 ulp): these recomputed forward
          // values only feed the derivative.
#pragma unroll
          for (int j = 0; j < C; ++j) {
            w[j] = __builtin_amdgcn_rcpf(d[j]);
            sw += w[j];
          }
        } else {
          float dmin = d[0];
#pragma unroll
          for (int j = 1; j < C; ++j) dmin = fminf(dmin, d[j]);
          // w_j scaled by dmin^(1/(m-1)): s and dw scale alike, dd is unchanged.
          const float ex = 1.f / (m - 1.f);
#pragma unroll
          for (int j = 0; j < C; ++j) {
            w[j] = exp2f((log2f(dmin) - log2f(d[j])) * ex);
            sw += w[j];
          }
        }
        const float is = M2 ? __builtin_amdgcn_rcpf(sw) : 1.f / sw;
#pragma unroll
        for (int j = 0; j < C; ++j) up[j] = w[j] * is;
        const float* gin = gns[S];  // prefetched with the voxel's plane (0 outside)
        float dup[C];
        float t = 0.f;
#pragma unroll
        for (int j = 0; j < C; ++j) {
          const float um1 = M2 ? up[j] : (up[j] > 0.f ? exp2f((m - 1.f) * log2f(up[j])) : 0.f);
          dup[j] = gin[j] + m * um1 * fmaf(dA[j], xv, dB[j]);
          t = fmaf(dup[j], up[j], t);
        }
#pragma unroll
        for (int j = 0; j < C; ++j) {
          const float dw = (dup[j] - t) * is;
          // m = 2: w_j = 1 / d_j, so w_j / ((m - 1) d_j) = w_j^2
          dbar[j] = M2 ? -dw * w[j] * w[j] : -dw * w[j] / ((m - 1.f) * d[j]);
        }
      }
      // da is the transpose's source: P = -lambda da g_inv, Q = -xi da q_inv
      // are rebuilt there from the voxel's g_inv and position.
      float da[C];
      const float keep = active ? 1.f : 0.f;
#pragma unroll
      for (int j = 0; j < C; ++j) {
        const float de = e[j] > kDFloor ? dbar[j] * keep : 0.f;
        da[j] = de * dd[j] * dd[j];
        acc[j] += -2.f * de * av[j] * dd[j];  // dJ/dc_j
        acc[C] += -da[j] * H[j];             // dJ/dlambda
        acc[C + 1] += -da[j] * F[j];         // dJ/dxi
      }
      if (active) store_row<C>(as_global(a.PQ) + i * C, da);
    };

    auto plane = [&](int p, int SA, int SB, int SC) __attribute__((always_inline)) {
      const int bp = (p - zlo + 1) % 3;
      const int bprev = (p - zlo + 3) % 3;  // plane p-1
      const int bnext = (p - zlo + 2) % 3;
      const bool pv = p >= 0 && p < nz;
      const bool doA = p - 1 >= zlo, doB = p >= zlo && p < zhi, doC = p + 1 < zhi;
      __builtin_amdgcn_wave_barrier();
      // Centre values for g (shifted by -1 for a flat neighbourhood).
      const float xA = doA ? cell_at(bprev, 0, 0)[0] : 0.f;
      const float xcA = gs[SA] < 0.f ? xA - 1.f : xA;
      const float xC = rg < 0.f ? rx - 1.f : rx;  // voxel p+1, prefetched
      float hC[C], E[C], Co[C], Pc[C];
#pragma unroll
      for (int j = 0; j < C; ++j) hC[j] = E[j] = Co[j] = Pc[j] = 0.f;
      if (pv) {
        const float xB = cell_at(bp, 0, 0)[0];
        const float xcB = gs[SB] < 0.f ? xB - 1.f : xB;
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy) {
#pragma unroll
          for (int dx = -1; dx <= 1; ++dx) {
            const float* cell = cell_at(bp, dy, dx);
            const float xk = cell[0];
            float u[C];
            lds_cell_load<C, CP>(cell + 4, u);
            const int n = (dx != 0) + (dy != 0);
#pragma unroll
            for (int j = 0; j < C; ++j) {
              if (n == 0) Pc[j] = u[j] * u[j];
              else if (n == 1) E[j] = fmaf(u[j], u[j], E[j]);
              else Co[j] = fmaf(u[j], u[j], Co[j]);
            }
            const float gA = fabsf(xcA - xk), gC = fabsf(xC - xk);  // eq (6)
#pragma unroll
            for (int j = 0; j < CH; ++j) {
              hn[SA][j] = fmaf(u[j], gA, hn[SA][j]);
              hC[j] = fmaf(u[j], gC, hC[j]);
            }
            if (n != 0) {
              const float gB = fabsf(xcB - xk);
#pragma unroll
              for (int j = 0; j < CH; ++j) hn[SB][j] = fmaf(u[j], gB, hn[SB][j]);
            }
          }
        }
      }
#pragma unroll
      for (int j = 0; j < C; ++j) {
        const float Sa = fmaf(wCa, Co[j], E[j]);
        const float Sb = fmaf(wCb, Co[j], fmaf(wEb, E[j], Pc[j]));
        fn[SA][j] += Sb;
        fn[SB][j] += Sa;
        hn[SC][j] = hC[j];
        fn[SC][j] = Sb;
      }
      __builtin_amdgcn_sched_barrier(0);
      if (p + 1 <= zhi) {
        store_plane(bnext);
        gs[SC] = rg;
#pragma unroll
        for (int j = 0; j < C; ++j) gns[SC][j] = rgn[j];
        if (p + 2 <= zhi) load_plane(p + 2);
      }
      if (doA) finalize(p - 1, SA, bprev);
      (void)doB;
      (void)doC;
      __builtin_amdgcn_sched_barrier(0);
    };

    // Plane walk replayed by tests/test_plane_walk.py.
    load_plane(zlo - 1);
    store_plane(0);
    load_plane(zlo);
    int p = zlo - 1;
    while (p <= zhi) {
      if (p > zlo && p + 4 <= zhi) {
        plane(p, 0, 1, 2);
        plane(p + 1, 1, 2, 0);
        plane(p + 2, 2, 0, 1);
        p += 3;
      } else {
        plane(p, 0, 1, 2);
#pragma unroll
        for (int j = 0; j < C; ++j) {
          hn[0][j] = hn[1][j];
          hn[1][j] = hn[2][j];
          fn[0][j] = fn[1][j];
          fn[1][j] = fn[2][j];
          gns[0][j] = gns[1][j];
          gns[1][j] = gns[2][j];
        }
        gs[0] = gs[1];
        gs[1] = gs[2];
        p += 1;
      }
    }
  }
  PairDev pr{};
  pr.partials = a.partials;
  wave_tile_store<NV>(pr, blockIdx.x * kAdjPW + wave, acc);
}

// The transpose gather on wave-private z-streaming tiles (the layout of the
// fused forward step): a wave owns 16 x 4 columns of a tile of zc planes,
// each plane of the tile plus a one-voxel halo is staged once in the wave's
// LDS as (xc, P, Q) per cell -- xc the cell's intensity as the cell uses it
// in eq (5) (shifted by -1 for a flat neighbourhood), P and Q formed from the
// cell's da, g_inv and position -- and every lane adds
// its 3 x 3 in-plane cells to the three voxels of its column they touch.
// For the Q part the in-plane cells are summed per offset class first (the
// weights of eq (7) depend only on the class).
template <int C>
constexpr int adj_waves() { return C <= 12 ? 4 : 3; }

template <int C, bool EVAL>
__global__ __launch_bounds__(64 * adj_waves<C>()) void k_adj_transpose_tiled(const AdjArgs a, float* Ubar_out) {
  constexpr int kAdjWaves = adj_waves<C>();
  constexpr int CP = (C + 3) / 4 * 4;
  constexpr int CW = 2 * CP;                 // floats per staged cell: P, Q
  // P and Q per cell, the cell's xc in an array of its own (no padding of
  // the float4 rows): three work groups of four waves fit a CU's LDS.
  __shared__ __align__(16) float s_c[kAdjWaves][3][kAdjCells * CW];
  __shared__ float s_xc[kAdjWaves][3][kAdjCells];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int tx = lane & (kAdjTX - 1), ty = lane / kAdjTX;
  const int own_cell = (ty + 1) * kAdjHX + (tx + 1);
  int hcx, hcy;
  if (lane < kAdjHX) { hcy = 0; hcx = lane; }
  else if (lane < 2 * kAdjHX) { hcy = kAdjHY - 1; hcx = lane - kAdjHX; }
  else if (lane < 2 * kAdjHX + kAdjTY) { hcy = 1 + lane - 2 * kAdjHX; hcx = 0; }
  else { hcy = 1 + lane - 2 * kAdjHX - kAdjTY; hcx = kAdjHX - 1; }
  const bool hlane = lane < kAdjHalo;
  const int halo_cell = hlane ? hcy * kAdjHX + hcx : 0;
  const float wCa = a.q2_sqdist ? 2.f : 4.f;  // in-plane corner (edge weighs 1)
  const float wEb = a.q2_sqdist ? 2.f : 4.f, wCb = a.q2_sqdist ? 3.f : 9.f;  // off-plane
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const int ntx = (nx + kAdjTX - 1) / kAdjTX, nty = (ny + kAdjTY - 1) / kAdjTY;
  const int zc = a.zc;
  const int ntz = (nz + zc - 1) / zc;
  const int nitems = ntx * nty * ntz;
  const uint32_t psz = (uint32_t)nx * (uint32_t)ny;

  const int per = (nitems + 7) >> 3;
  const int xcd = blockIdx.x & 7;
  const int it_end = min(nitems, (xcd + 1) * per);
  const int it_step = (gridDim.x >> 3) * kAdjWaves;
  for (int it = xcd * per + (blockIdx.x >> 3) * kAdjWaves + wave; it < it_end; it += it_step) {
    const int txi = it % ntx;
    const int rest = it / ntx;
    const int tyi = rest % nty;
    const int tzi = rest / nty;
    const int x0 = txi * kAdjTX, y0 = tyi * kAdjTY;
    const int zlo = tzi * zc, zhi = min(zlo + zc, nz);
    const int gx = x0 + tx, gy = y0 + ty;
    const bool active = gx < nx && gy < ny;
    const int hx = x0 - 1 + hcx, hy = y0 - 1 + hcy;
    const bool hvalid = hlane && hx >= 0 && hx < nx && hy >= 0 && hy < ny;
    const size_t own_xy = active ? (size_t)gy * nx + gx : 0;
    const size_t halo_xy = hvalid ? (size_t)hy * nx + hx : 0;
    float* const sc = &s_c[wave][0][0];

    // Prefetch registers of one plane: own and halo cell (intensity as the
    // cell uses it in eq (5), its |g_inv| and q_inv, and da).
    // The own cell also brings the voxel's U (and in the objective pass its
    // direct term), which only the voxel's own finalisation reads, three
    // planes later.
    float rxc, rx, rgi, rqi, rd[C], ru[C], rdir[C], hxc, hgi, hqi, hd[C];
    auto load_plane = [&](int q) __attribute__((always_inline)) {
      const bool pv = q >= 0 && q < nz;
      rx = rxc = rgi = rqi = hxc = hgi = hqi = 0.f;
#pragma unroll
      for (int j = 0; j < C; ++j) rd[j] = hd[j] = ru[j] = rdir[j] = 0.f;
      if (pv && active) {
        const size_t i = (size_t)q * psz + own_xy;
        rx = a.x[i];
        const float g = a.invg[i];
        rxc = g < 0.f ? rx - 1.f : rx;
        rgi = fabsf(g);
        rqi = adj_qinv_cell(gx, gy, q, nx, ny, nz, wCa, wEb, wCb);
        load_row<C>(as_global(a.PQ) + i * C, rd);
        load_row<C>(as_global(a.U) + i * C, ru);
        if constexpr (EVAL) load_row<C>(as_global(a.Ubar_direct) + i * C, rdir);
      }
      if (pv && hvalid) {
        const size_t i = (size_t)q * psz + halo_xy;
        const float xh = a.x[i];
        const float g = a.invg[i];
        hxc = g < 0.f ? xh - 1.f : xh;
        hgi = fabsf(g);
        hqi = adj_qinv_cell(hx, hy, q, nx, ny, nz, wCa, wEb, wCb);
        load_row<C>(as_global(a.PQ) + i * C, hd);
      }
    };
    // P = -lambda da g_inv and Q = -xi da q_inv of the cell (the products the
    // per-voxel kernel would have formed).
    auto store_cell = [&](float* cell, float* xcell, float xc, float gi, float qi, const float (&dav)[C])
        __attribute__((always_inline)) {
      *xcell = xc;
      float P[C], Q[C];
#pragma unroll
      for (int j = 0; j < C; ++j) {
        P[j] = -a.lam * dav[j] * gi;
        Q[j] = -a.xi * dav[j] * qi;
      }
      lds_cell_store<C, CP>(cell, P);
      lds_cell_store<C, CP>(cell + CP, Q);
    };
    float* const sxw = &s_xc[wave][0][0];
    auto store_plane = [&](int buf) __attribute__((always_inline)) {
      float* base = sc + buf * kAdjCells * CW;
      float* xb = sxw + buf * kAdjCells;
      store_cell(base + own_cell * CW, xb + own_cell, rxc, rgi, rqi, rd);
      if (hlane) store_cell(base + halo_cell * CW, xb + halo_cell, hxc, hgi, hqi, hd);
    };

    // Target slots (voxels p-1, p, p+1 of the lane's column): P-part and
    // class-weighted Q sums, and the target's own intensity.
    float hP[3][C], fQ[3][C], xt[3], us[3][C], ds[3][C];
#pragma unroll
    for (int s2 = 0; s2 < 3; ++s2) {
      xt[s2] = 0.f;
#pragma unroll
      for (int j = 0; j < C; ++j) hP[s2][j] = fQ[s2][j] = us[s2][j] = ds[s2][j] = 0.f;
    }
    auto finalize = [&](int z, int S) __attribute__((always_inline)) {
      if (!active) return;
      const size_t k = (size_t)z * psz + own_xy;
      float out[C];
#pragma unroll
      for (int j = 0; j < C; ++j) {
        const float t = hP[S][j] + 2.f * us[S][j] * fQ[S][j];
        out[j] = EVAL ? ds[S][j] + t : t;
      }
      store_row<C>(as_global(Ubar_out) + k * C, out);
    };

    auto cell_at = [&](int buf, int dy, int dx) -> const float* {
      return sc + (buf * kAdjCells + own_cell + dy * kAdjHX + dx) * CW;
    };
    auto plane = [&](int p, int SA, int SB, int SC) __attribute__((always_inline)) {
      const int bp = (p - zlo + 1) % 3;
      const int bnext = (p - zlo + 2) % 3;
      const bool pv = p >= 0 && p < nz;
      const bool doA = p - 1 >= zlo, doB = p >= zlo && p < zhi, doC = p + 1 < zhi;
      __builtin_amdgcn_wave_barrier();
      const float xA = xt[SA], xB = xt[SB], xC = rx;  // plain target intensities
      float hC[C], E[C], Co[C], Pc[C];
#pragma unroll
      for (int j = 0; j < C; ++j) hC[j] = E[j] = Co[j] = Pc[j] = 0.f;
      if (pv) {
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy) {
#pragma unroll
          for (int dx = -1; dx <= 1; ++dx) {
            const float* cell = cell_at(bp, dy, dx);
            const float xc = sxw[bp * kAdjCells + own_cell + dy * kAdjHX + dx];
            float P[C], Q[C];
            lds_cell_load<C, CP>(cell, P);
            lds_cell_load<C, CP>(cell + CP, Q);
            const int n = (dx != 0) + (dy != 0);
#pragma unroll
            for (int j = 0; j < C; ++j) {
              if (n == 0) Pc[j] = Q[j];
              else if (n == 1) E[j] += Q[j];
              else Co[j] += Q[j];
            }
            const float gA = fabsf(xc - xA), gC = fabsf(xc - xC);
#pragma unroll
            for (int j = 0; j < C; ++j) {
              hP[SA][j] = fmaf(P[j], gA, hP[SA][j]);
              hC[j] = fmaf(P[j], gC, hC[j]);
            }
            if (n != 0) {
              const float gB = fabsf(xc - xB);
#pragma unroll
              for (int j = 0; j < C; ++j) hP[SB][j] = fmaf(P[j], gB, hP[SB][j]);
            }
          }
        }
      }
#pragma unroll
      for (int j = 0; j < C; ++j) {
        const float Sa = fmaf(wCa, Co[j], E[j]);
        const float Sb = fmaf(wCb, Co[j], fmaf(wEb, E[j], Pc[j]));
        fQ[SA][j] += Sb;
        fQ[SB][j] += Sa;
        hP[SC][j] = hC[j];
        fQ[SC][j] = Sb;
      }
      __builtin_amdgcn_sched_barrier(0);
      if (p + 1 <= zhi) {
        store_plane(bnext);
        xt[SC] = rx;
#pragma unroll
        for (int j = 0; j < C; ++j) {
          us[SC][j] = ru[j];
          if constexpr (EVAL) ds[SC][j] = rdir[j];
        }
        if (p + 2 <= zhi) load_plane(p + 2);
      }
      if (doA) finalize(p - 1, SA);
      (void)doB;
      (void)doC;
      __builtin_amdgcn_sched_barrier(0);
    };

    // Plane walk replayed by tests/test_plane_walk.py.
    load_plane(zlo - 1);
    store_plane(0);
    load_plane(zlo);
    // Slot ring: rotating indices (runtime: the arrays stay in registers only
    // through full unrolling of the three-plane body below).
    int p = zlo - 1;
    while (p <= zhi) {
      if (p > zlo && p + 4 <= zhi) {
        plane(p, 0, 1, 2);
        plane(p + 1, 1, 2, 0);
        plane(p + 2, 2, 0, 1);
        p += 3;
      } else {
        plane(p, 0, 1, 2);
#pragma unroll
        for (int j = 0; j < C; ++j) {
          hP[0][j] = hP[1][j];
          hP[1][j] = hP[2][j];
          fQ[0][j] = fQ[1][j];
          fQ[1][j] = fQ[2][j];
          us[0][j] = us[1][j];
          us[1][j] = us[2][j];
          ds[0][j] = ds[1][j];
          ds[1][j] = ds[2][j];
        }
        xt[0] = xt[1];
        xt[1] = xt[2];
        p += 1;
      }
    }
  }
}

// Fixed-order fp64 sum of the adjoint block slots: out[0..C) = dJ/dc (this
// step), acc2[0..1] += dJ/dlambda, dJ/dxi.
template <int C>
__global__ __launch_bounds__(1024) void k_adj_finalize(const float* parts, int nslots, double* out,
                                                       double* acc2) {
  constexpr int NV = C + 2;
  constexpr int NWF = 1024 / 64;
  __shared__ double s_red[NWF * NV];
  double d[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) d[k] = 0.0;
  // Slots s, s + 1024, ... added in that order, four loaded at once.
  constexpr int kU = 4;
  int s = threadIdx.x;
  for (; s + (kU - 1) * 1024 < nslots; s += kU * 1024) {
    float v[kU][NV];
#pragma unroll
    for (int u = 0; u < kU; ++u)
#pragma unroll
      for (int k = 0; k < NV; ++k) v[u][k] = parts[(size_t)(s + u * 1024) * NV + k];
#pragma unroll
    for (int u = 0; u < kU; ++u)
#pragma unroll
      for (int k = 0; k < NV; ++k) d[k] += (double)v[u][k];
  }
  for (; s < nslots; s += 1024) {
#pragma unroll
    for (int k = 0; k < NV; ++k) d[k] += (double)parts[(size_t)s * NV + k];
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double v = d[k];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    d[k] = v;
  }
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) s_red[wave * NV + k] = d[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double t = 0.0;
      for (int w = 0; w < NWF; ++w) t += s_red[w * NV + k];
      if (k < C) out[k] = t;
      else acc2[k - C] += t;
    }
  }
}

// Planes per tile of a tiled adjoint kernel whose resident work groups hold
// `resident` waves: among the depths ceil(nz / k) of at least
// min(nz, kAdjMinZc) planes, the one whose tiles take the fewest rounds of
// the resident waves times (depth + 3) (a tile also stages its two halo
// planes and fills its pipeline); the deepest of equal ones.  A shallower
// tile spreads a volume over more waves when one tile per column leaves
// wave slots empty.
static int adj_depth(int nx, int ny, int nz, long resident) {
  const long txy = (long)((nx + kAdjTX - 1) / kAdjTX) * ((ny + kAdjTY - 1) / kAdjTY);
  const int floor_zc = std::min(nz, kAdjMinZc);
  resident = std::max(1L, resident);
  int best = nz;
  long best_cost = -1;
  for (int k = 1; k <= nz; ++k) {
    const int d = (nz + k - 1) / k;
    if (d < floor_zc) break;
    if (k > 1 && d == (nz + k - 2) / (k - 1)) continue;  // same depth as k - 1
    const long items = txy * ((nz + d - 1) / d);
    const long cost = (items + resident - 1) / resident * (d + 3);
    if (best_cost < 0 || cost < best_cost) {
      best_cost = cost;
      best = d;
    }
  }
  return best;
}

// Persistent grid of a tiled adjoint kernel with `waves` waves per work
// group: one tile per wave while that fits in 8 rounds of the resident work
// groups, else the resident work groups; a multiple of 8 (one share per
// XCD), at least 8.
static long adj_grid(const AdjArgs& a, int waves, int occ) {
  const long ntiles = (long)((a.nx + kAdjTX - 1) / kAdjTX) * ((a.ny + kAdjTY - 1) / kAdjTY) *
                      ((a.nz + a.zc - 1) / a.zc);
  const long want = (ntiles + waves - 1) / waves;
  const long resident = (long)std::max(occ, 1) * std::max(1, a.num_cu);
  const long g = want <= 8 * resident ? (want + 7) / 8 * 8 : resident / 8 * 8;
  return std::max<long>(8, g);
}

static int occupancy_of(const void* f, int threads) {
  int o = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, f, threads, 0) != hipSuccess || o < 1) o = 1;
  return o;
}

template <int C>
static hipError_t launch_adj_c(const AdjArgs& a, bool m2, bool eval, float* Ubar_out,
                               double* cbar_out, double* acc2, hipStream_t s) {
  // Per-voxel part: each wave leaves its sums in slot (block, wave).
  {
    // Occupancy of each variant, found once (any thread may store it: the
    // value is the same).
    static std::atomic<int> occ[4] = {0, 0, 0, 0};
    const void* f = eval ? (m2 ? reinterpret_cast<const void*>(&k_adj_point<C, true, true>)
                               : reinterpret_cast<const void*>(&k_adj_point<C, false, true>))
                         : (m2 ? reinterpret_cast<const void*>(&k_adj_point<C, true, false>)
                               : reinterpret_cast<const void*>(&k_adj_point<C, false, false>));
    std::atomic<int>& oc = occ[(eval ? 2 : 0) + (m2 ? 1 : 0)];
    int o = oc.load(std::memory_order_relaxed);
    if (!o) {
      o = occupancy_of(f, 64 * kAdjPW);
      oc.store(o, std::memory_order_relaxed);
    }
    AdjArgs ap = a;
    ap.zc = adj_depth(a.nx, a.ny, a.nz, (long)o * std::max(1, a.num_cu) * kAdjPW);
    const int g = (int)adj_grid(ap, kAdjPW, o);
    if (eval) {
      if (m2) hipLaunchKernelGGL((k_adj_point<C, true, true>), dim3(g), dim3(64 * kAdjPW), 0, s, ap);
      else hipLaunchKernelGGL((k_adj_point<C, false, true>), dim3(g), dim3(64 * kAdjPW), 0, s, ap);
    } else {
      if (m2) hipLaunchKernelGGL((k_adj_point<C, true, false>), dim3(g), dim3(64 * kAdjPW), 0, s, ap);
      else hipLaunchKernelGGL((k_adj_point<C, false, false>), dim3(g), dim3(64 * kAdjPW), 0, s, ap);
    }
    hipLaunchKernelGGL((k_adj_finalize<C>), dim3(1), dim3(1024), 0, s, a.partials, g * kAdjPW, cbar_out,
                       acc2);
  }
  if (Ubar_out) {
    // Tiled transpose: one wave per tile, a persistent grid.
    static std::atomic<int> occ[2] = {0, 0};
    std::atomic<int>& oc = occ[eval ? 1 : 0];
    int o = oc.load(std::memory_order_relaxed);
    if (!o) {
      o = occupancy_of(eval ? reinterpret_cast<const void*>(&k_adj_transpose_tiled<C, true>)
                            : reinterpret_cast<const void*>(&k_adj_transpose_tiled<C, false>),
                       64 * adj_waves<C>());
      oc.store(o, std::memory_order_relaxed);
    }
    AdjArgs at = a;
    at.zc = adj_depth(a.nx, a.ny, a.nz, (long)o * std::max(1, a.num_cu) * adj_waves<C>());
    const long g = adj_grid(at, adj_waves<C>(), o);
    if (eval)
      hipLaunchKernelGGL((k_adj_transpose_tiled<C, true>), dim3((int)g), dim3(64 * adj_waves<C>()), 0, s, at,
                         Ubar_out);
    else
      hipLaunchKernelGGL((k_adj_transpose_tiled<C, false>), dim3((int)g), dim3(64 * adj_waves<C>()), 0, s, at,
                         Ubar_out);
  }
  return hipGetLastError();
}

#define PIFCM_FOR_EACH_C(X) \
  X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)

hipError_t launch_adjoint(int C, const AdjArgs& a, bool m2, bool eval, float* Ubar_out,
                          double* cbar_out, double* acc2, hipStream_t s) {
  switch (C) {
#define CASE(c) \
  case c: return launch_adj_c<c>(a, m2, eval, Ubar_out, cbar_out, acc2, s);
    PIFCM_FOR_EACH_C(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

// Upper bound of the slots k_adj_point writes (its grid never exceeds the
// one-tile-per-wave grid of the shallowest depth, at least 8 work groups).
size_t adjoint_slots(int nx, int ny, int nz) {
  const int zmin = std::max(1, std::min(nz, kAdjMinZc));
  const long ntiles = (long)((nx + kAdjTX - 1) / kAdjTX) * ((ny + kAdjTY - 1) / kAdjTY) *
                      ((nz + zmin - 1) / zmin);
  const long want = (ntiles + kAdjPW - 1) / kAdjPW;
  return (size_t)std::max<long>(8, (want + 7) / 8 * 8) * kAdjPW;
}

}  // namespace pifcm
