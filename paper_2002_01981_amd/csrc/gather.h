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
// Work decomposition.  A work item is a tile of 16 (x) by 4 (y) columns and
// zc planes of one (volume, particle) pair, owned by ONE wavefront: each
// lane owns one (x, y) column and walks it along z.  Waves never wait for
// each other -- each has a private LDS region -- so there is no work-group
// barrier anywhere in the kernel.  Each plane of the tile plus a one-voxel
// halo (18 x 6 cells) is staged once in the wave's LDS (triple-buffered) and
// every lane reads its 3x3 in-plane cells once: they contribute to three
// voxels of its column at the same time -- z-1 (the plane is its upper
// neighbour plane), z (its own plane) and z+1 (lower plane).  The partial
// sums of those voxels live in a ring of three register slots; voxel z-1 is
// complete after the plane and is finalised right away.  The next plane is
// prefetched into registers while the current one is processed.  Planes away
// from the tile's first and last ones run a branch-free body unrolled three
// times so the slot ring rotates by renaming instead of register moves.
//
// Particle sharing.  A work item may hold PT particles (two) of the same
// volume: the intensities, g_inv and every g_ik = |x_i - x_k| depend on the
// volume only, so they are loaded, staged and formed once and applied to
// each particle's memberships, which are staged side by side in the wave's
// LDS.  Each particle keeps its own slots, sums, centres and output.  A
// particle past the end of the swarm, or one that has stopped, is computed
// from a duplicate and its stores are skipped.
//
// Arithmetic shortcuts that keep the results those of the equations:
//   * the denominator of eq (5), sum_k |x_i - x_k|, does not change between
//     iterations: it is precomputed once per volume as its inverse g_inv;
//   * sum_j H_ij = 1 when the rows of U sum to 1, so the last cluster's H is
//     1 - sum of the others (rows of caller-supplied U are validated);
//   * a voxel whose neighbours all share its intensity takes the mean of
//     their memberships in eq (5); it is stored with g_inv = -1 / n_valid and
//     its centre value shifted by -1 when forming g, so every g_ik of it is
//     exactly 1 and the gather yields the mean with no branch;
//   * eq (7)'s weights depend only on the offset class (face, edge, corner
//     in the plane and one plane off), so per plane the squared memberships
//     are summed per class once and weighted afterwards;
//   * the denominator of eq (7) depends only on which neighbours exist and is
//     formed from the column position and the plane index;
//   * cells outside the volume are staged with u = 0, so they add nothing to
//     any sum.
// Sums over voxels are per-lane in fp32, reduced per tile in a fixed
// butterfly order into the tile's own slot; k_finalize then adds the slots of
// each pair in fp64 in tile order (no floating-point atomics: results are
// bit-reproducible).
#pragma once
#include "common.h"

namespace pifcm {

constexpr int kWX = 16, kWY = 4;               // wave tile (columns)
constexpr int kHX = kWX + 2, kHY = kWY + 2;    // staged plane with halo
constexpr int kNCell = kHX * kHY;              // 108 cells
constexpr int kNHalo = kNCell - 64;            // 44 halo cells, one per lane

template <int C, bool M2, int NW, bool STEP, int PT>
__global__ __launch_bounds__(64 * NW) void k_ifcm_gather(const LaunchArgs a) {
  constexpr int CP = (C + 3) / 4 * 4;
  constexpr int CH = C - 1;  // clusters whose H is gathered
  constexpr int NV = STEP ? 2 * C + 1 : 1;

  // Three plane buffers per wave: the plane being read, the one before it
  // (own cells of the voxel being finalised), and the one being staged; the
  // memberships of the PT particles side by side.
  __shared__ float s_x[NW][3][kNCell];
  __shared__ __align__(16) float s_u[NW][3][PT][kNCell * CP];

  const int lane = threadIdx.x & 63;
  // The wave index is uniform across the wave; say so, so that every value
  // derived from it (the work item, its pointers and parameters) stays in
  // scalar registers.
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int tx = lane & (kWX - 1), ty = lane / kWX;
  const int own_cell = (ty + 1) * kHX + (tx + 1);
  int hcx, hcy;
  if (lane < kHX) { hcy = 0; hcx = lane; }
  else if (lane < 2 * kHX) { hcy = kHY - 1; hcx = lane - kHX; }
  else if (lane < 2 * kHX + kWY) { hcy = 1 + lane - 2 * kHX; hcx = 0; }
  else { hcy = 1 + lane - 2 * kHX - kWY; hcx = kHX - 1; }
  const bool hlane = lane < kNHalo;
  const int halo_cell = hlane ? hcy * kHX + hcx : 0;
  // eq (7) weights by offset class: in-plane edge / corner (q = 1, 2) and
  // off-plane centre / edge / corner (q = 1, 2, 3); q^2 or q.  The weight
  // of q = 1 is 1 in both readings.
  constexpr float wEa = 1.f, wPb = 1.f;
  const float wCa = a.q2_sqdist ? 2.f : 4.f;
  const float wEb = a.q2_sqdist ? 2.f : 4.f, wCb = a.q2_sqdist ? 3.f : 9.f;

  // Items: 8 contiguous ranges of about equal work, one per XCD (work groups
  // go to the XCDs round-robin), walked in order by that XCD's waves, so
  // neighbouring tiles run together and share L2: wave w of the W takes
  // items w, w + W, w + 2W, ...  Without a stop rule (a.handout), a range
  // holding more items than the XCD has waves is walked that way for its
  // first nine tenths only; the last tenth is handed out one item at a time
  // to whichever wave is free (a counter per XCD), which keeps the tail of
  // the launch balanced while the counter sees few requests.  Under a stop
  // rule the items of stopped pairs cost nothing and waves running through
  // them would queue on a counter, so those launches keep the plain walk.
  // The last wave of the XCD to run out resets the counters for the next
  // launch.
  const int xcd = blockIdx.x & 7;
  const int waves = (int)((gridDim.x - xcd + 7) >> 3) * NW;  // this XCD's waves
  const int widx = (int)(blockIdx.x >> 3) * NW + wave;       // this wave among them
  const int it_beg = a.xcd_begin[xcd], it_end = a.xcd_begin[xcd + 1];
  const int n_it = it_end - it_beg;
  const bool handout = a.handout && n_it > waves;
  // items each wave takes by index: without hand-out, all of its share
  const int spw = handout ? max(1, (int)((long)n_it * 9 / 10 / waves)) : (n_it + waves - 1) / waves;
  const int it_dyn = it_beg + spw * waves;                                    // first handed-out item
  // The ticket for the wave's first handed-out item is drawn when its last
  // item by index starts (then at each handed-out item's start) and read
  // when that item ends, so the atomic's round trip hides behind the item.
  int ticket = 0;
  int k = 0;
  for (int it = it_beg + widx; it < it_end;
       it = ++k < spw ? it_beg + widx + k * waves
                      : (handout ? it_dyn + __builtin_amdgcn_readfirstlane(ticket) : it_end)) {
    if (handout && k + 1 >= spw && lane == 0) ticket = atomicAdd(a.work + xcd, 1);
    const int b = vol_of_item(a, it);
    const VolDev vd = ld_const(a.vols + b);
    const int r = it - a.item_begin[b];
    const int grp = r / vd.tiles;
    const int tile = r - grp * vd.tiles;
    // The PT particles of the item: a slot past the swarm repeats the last
    // particle, and it and a particle that has stopped store nothing.
    PairDev pr[PT];
    bool live[PT];
    bool any = false;
#pragma unroll
    for (int k = 0; k < PT; ++k) {
      const int q = grp * PT + k;
      pr[k] = ld_const(a.pairs + b * a.P + min(q, a.P - 1));
      live[k] = q < a.P && !(STEP && ld_const(&pr[k].st->stop));
      any = any || live[k];
    }
    if (!any) continue;
    const float* Uin[PT];
    float* Uout[PT];
    float cj[PT][C], lam[PT], xi[PT];
#pragma unroll
    for (int k = 0; k < PT; ++k) {
      const SolveState* st = pr[k].st;
      const int t = STEP ? ld_const(&st->iter) + 1 : ld_const(&st->iter);
      Uin[k] = uniform_ptr(STEP ? u_in_of(pr[k], t) : u_state_of(pr[k], t));
      Uout[k] = STEP ? uniform_ptr(u_out_of(pr[k], t)) : nullptr;
#pragma unroll
      for (int j = 0; j < C; ++j) cj[k][j] = ld_const(&st->c[(STEP ? t - 1 : t) & 1][j]);
      lam[k] = ld_const(&st->lam);
      xi[k] = ld_const(&st->xi);
    }
    const int nx = vd.nx, ny = vd.ny, nz = vd.nz;

    const int txi = tile % vd.ntx;
    const int rest = tile / vd.ntx;
    const int tyi = rest % vd.nty;
    const int tzi = rest / vd.nty;
    const int x0 = txi * kWX, y0 = tyi * kWY;
    const int zlo = vd.zbeg + tzi * vd.zc, zhi = min(zlo + vd.zc, vd.zend);
    const int gx = x0 + tx, gy = y0 + ty;
    const bool active = gx < nx && gy < ny;
    const float amask = active ? 1.f : 0.f;
    const int hx = x0 - 1 + hcx, hy = y0 - 1 + hcy;
    const bool hvalid = hlane && hx >= 0 && hx < nx && hy >= 0 && hy < ny;
    // 32-bit offsets from the first staged plane of the tile (the host keeps
    // (zc + 2) * nx * ny * C * 4 below 2^31).
    const uint32_t psz = (uint32_t)nx * (uint32_t)ny;
    const int zb = max(zlo - 1, 0);
    const gfloat* Xb = as_global(vd.x) + (size_t)zb * psz;
    const gfloat* Gb = as_global(vd.invg) + (size_t)zb * psz;
    const gfloat* Ub[PT];
    gfloat* Ob[PT];
#pragma unroll
    for (int k = 0; k < PT; ++k) {
      Ub[k] = as_global(Uin[k]) + (size_t)zb * psz * C;
      Ob[k] = STEP ? as_global(Uout[k]) + (size_t)zb * psz * C : nullptr;
    }
    // Lane byte offsets within a plane of x / g_inv (4 B per voxel); U rows
    // are C times that.  Per plane, the base moves in scalar registers.
    uint32_t own_ofs = active ? ((uint32_t)gy * nx + gx) * 4u : 0u;
    uint32_t halo_ofs = hvalid ? ((uint32_t)hy * nx + hx) * 4u : 0u;
    uint32_t own_ofs_u = own_ofs * C, halo_ofs_u = halo_ofs * C;

    // Denominator of eq (7): in-plane edges e and corners e_x * e_y, plus for
    // each of the az existing off-planes a centre, e edges and e_x * e_y
    // corners.
    float invQ0, invQ1, invQ2;  // by the number of existing off-planes
    {
      const int ex = (gx > 0) + (gx < nx - 1), ey = (gy > 0) + (gy < ny - 1);
      const float e = (float)(ex + ey), co = (float)(ex * ey);
      const float q0 = wEa * e + wCa * co, q1 = wPb + wEb * e + wCb * co;
      invQ0 = q0 > 0.f ? 1.f / q0 : 0.f;
      invQ1 = 1.f / (q0 + q1);
      invQ2 = 1.f / (q0 + 2.f * q1);
    }

    // Plane q lives in buffer (q - zlo + 1) % 3: the tile's first staged
    // plane (zlo - 1) in buffer 0.  In the unrolled interior loop the buffer of
    // every access is a compile-time constant, so LDS addresses are one lane
    // base plus immediate offsets.
    float* const sxw = &s_x[wave][0][0] + own_cell;
    float* const suw = &s_u[wave][0][0][0] + own_cell * CP;
    auto bufof = [&](int q) { return (q - zlo + 1) % 3; };
    auto sx_at = [&](int buf, int dy, int dx) -> float {
      return sxw[buf * kNCell + dy * kHX + dx];
    };
    auto su_at = [&](int buf, int k, int dy, int dx, float (&u)[C]) {
      lds_cell_load<C, CP>(suw + ((buf * PT + k) * kNCell + dy * kHX + dx) * CP, u);
    };

    // Prefetch registers of the next plane.  A lane whose column lies outside
    // the volume (in x or y) does so for the whole tile: the tile's first
    // planes (full form) stage zeros for its cells in all three buffers, and
    // the interior planes (LIGHT form) neither load nor store them.
    float rx, rg, ru[PT][C], rhx, rhu[PT][C];
    auto zero_prefetch = [&]() __attribute__((always_inline)) {
      rx = 0.f;
      rg = 1.f;
      rhx = 0.f;
#pragma unroll
      for (int k = 0; k < PT; ++k)
#pragma unroll
        for (int j = 0; j < C; ++j) ru[k][j] = rhu[k][j] = 0.f;
    };
    auto load_plane = [&](int q, auto LIGHTc) __attribute__((always_inline)) {
      constexpr bool LIGHT = decltype(LIGHTc)::value;
      const bool pv = q >= 0 && q < nz;
      const uint32_t pb = (uint32_t)(q - zb) * psz * 4u;
      const gfloat* Xq = opaque_base(at_byte(Xb, pb));
      const gfloat* Gq = opaque_base(at_byte(Gb, pb));
      if constexpr (LIGHT) {
        if (!pv) {
          zero_prefetch();
          return;
        }
      }
      if (pv && active) {
        rx = *at_lane(Xq, own_ofs);
        rg = *at_lane(Gq, own_ofs);
#pragma unroll
        for (int k = 0; k < PT; ++k) {
          const gfloat* Uq = opaque_base(at_byte(Ub[k], pb * C));
          load_row<C>(at_lane(Uq, own_ofs_u), ru[k]);
        }
      } else if (!LIGHT) {
        rx = 0.f;
        rg = 1.f;
#pragma unroll
        for (int k = 0; k < PT; ++k)
#pragma unroll
          for (int j = 0; j < C; ++j) ru[k][j] = 0.f;
      }
      if (pv && hvalid) {
        rhx = *at_lane(Xq, halo_ofs);
#pragma unroll
        for (int k = 0; k < PT; ++k) {
          const gfloat* Uq = opaque_base(at_byte(Ub[k], pb * C));
          load_row<C>(at_lane(Uq, halo_ofs_u), rhu[k]);
        }
      } else if (!LIGHT) {
        rhx = 0.f;
#pragma unroll
        for (int k = 0; k < PT; ++k)
#pragma unroll
          for (int j = 0; j < C; ++j) rhu[k][j] = 0.f;
      }
    };
    auto store_plane = [&](int buf, auto LIGHTc) __attribute__((always_inline)) {
      constexpr bool LIGHT = decltype(LIGHTc)::value;
      float* sx = &s_x[wave][buf][0];
      // The light form skips the cells of lanes outside the volume: they
      // hold the zeros the full form staged.
      if (!LIGHT || active) {
        sx[own_cell] = rx;
#pragma unroll
        for (int k = 0; k < PT; ++k) lds_cell_store<C, CP>(&s_u[wave][buf][k][0] + own_cell * CP, ru[k]);
      }
      if (LIGHT ? hvalid : hlane) {
        sx[halo_cell] = rhx;
#pragma unroll
        for (int k = 0; k < PT; ++k) lds_cell_store<C, CP>(&s_u[wave][buf][k][0] + halo_cell * CP, rhu[k]);
      }
    };

    // Slots of the three voxels in flight: gathered H numerators, F class
    // sums (per particle), the stored g_inv (its sign marks a flat
    // neighbourhood) and the centre value that forms g (shifted by -1 for a
    // flat neighbourhood).
    float hn[3][PT][CH], fn[3][PT][C], gs[3], xs[3];
    float acc[PT][NV];
#pragma unroll
    for (int k = 0; k < PT; ++k)
#pragma unroll
      for (int v = 0; v < NV; ++v) acc[k][v] = 0.f;
#pragma unroll
    for (int s2 = 0; s2 < 3; ++s2) {
      gs[s2] = 1.f;
      xs[s2] = 0.f;
#pragma unroll
      for (int k = 0; k < PT; ++k) {
#pragma unroll
        for (int j = 0; j < CH; ++j) hn[s2][k][j] = 0.f;
#pragma unroll
        for (int j = 0; j < C; ++j) fn[s2][k][j] = 0.f;
      }
    }

    // Finalise voxel z of slot S; its own cell is in buffer bz:
    // eqs (5)/(7) ratios, (4), (1), (2), (3), per particle.
    auto finalize = [&](int z, auto Sc, int bz) __attribute__((always_inline)) {
      constexpr int S = decltype(Sc)::value;
      // Computed by every lane (a lane outside the volume sees staged zeros
      // and finite distances); only its store and its sums are masked, so no
      // conditional block holds the arithmetic.
      const float xv = sx_at(bz, 0, 0);
      const float iq = (z > 0 && z < nz - 1) ? invQ2 : ((z > 0 || z < nz - 1) ? invQ1 : invQ0);
      const float g = fabsf(gs[S]);
#pragma unroll
      for (int k = 0; k < PT; ++k) {
        float uo[C];
        su_at(bz, k, 0, 0, uo);
        // a_j = 1 - lambda H_j - xi F_j with H_j = hn_j * g, F_j = fn_j * iq.
        const float lg = -lam[k] * g, xq = -xi[k] * iq;
        float sh = hn[S][k][0];
#pragma unroll
        for (int j = 1; j < CH; ++j) sh += hn[S][k][j];
        // Last cluster by sum_j H_ij = 1 (0 when the voxel has no neighbour).
        const float hlast = g != 0.f ? fmaf(-g, sh, 1.f) : 0.f;
        float d2[C];
        float Jv = 0.f;
#pragma unroll
        for (int j = 0; j < C; ++j) {
          const float ah =
              j < CH ? fmaf(lg, hn[S][k][j < CH ? j : 0], 1.f) : fmaf(-lam[k], hlast, 1.f);
          const float av = fmaf(xq, fn[S][k][j], ah);  // eq (4) factor
          const float dd = xv - cj[k][j];
          d2[j] = fmaxf(dd * dd * av, kDFloor);
          Jv = fmaf(pow_m<M2>(uo[j], a.m), d2[j], Jv);  // eq (1)
        }
        if constexpr (STEP) {
          // eq (2); a lane outside the volume gets zeros (scale 0), so its
          // terms vanish from the sums of eq (3) with no masking.
          float un[C];
          memberships<C, M2>(d2, a.m, un, amask);
          if (active && live[k]) {
            gfloat* Oz = opaque_base(at_byte(Ob[k], (uint32_t)(z - zb) * psz * (4u * C)));
            store_row<C>(at_lane(Oz, own_ofs_u), un);
          }
#pragma unroll
          for (int j = 0; j < C; ++j) {
            const float w = pow_m<M2>(un[j], a.m);
            acc[k][j] = fmaf(w, xv, acc[k][j]);  // eq (3) numerator
            acc[k][C + j] += w;                   // eq (3) denominator
          }
          acc[k][2 * C] += Jv;  // 0 for a lane outside: its staged memberships are 0
        } else {
          acc[k][0] += Jv;
        }
      }
    };

    // One plane p: contributions of its 3x3 cells to voxels p-1 (slot SA),
    // p (SB) and p+1 (SC); finalise p-1; stage plane p+1; prefetch p+2.
    // BP: buffer of plane p (-1: computed at run time); GEN: the tile's
    // first / last planes, with the validity tests.
    auto plane = [&](int p, auto SAc, auto SBc, auto SCc, auto BPc, auto GENc) __attribute__((always_inline)) {
      constexpr int SA = decltype(SAc)::value, SB = decltype(SBc)::value;
      constexpr int SC = decltype(SCc)::value;
      constexpr int BPS = decltype(BPc)::value;
      constexpr bool GEN = decltype(GENc)::value;
      const int bp = BPS >= 0 ? BPS : bufof(p);
      const int bprev = BPS >= 0 ? (BPS + 2) % 3 : bufof(p + 2);  // plane p-1
      const int bnext = BPS >= 0 ? (BPS + 1) % 3 : bufof(p + 1);  // plane p+1
      const bool pv = !GEN || (p >= 0 && p < nz);
      const bool doA = !GEN || p - 1 >= zlo;
      const bool doB = !GEN || (p >= zlo && p < zhi);
      const bool doC = !GEN || p + 1 < zhi;
      __builtin_amdgcn_wave_barrier();
      // Centre values for g: voxels p-1 and p from their slots, p+1 from the
      // prefetch registers.
      const float xcA = xs[SA];
      const float xC = rg < 0.f ? rx - 1.f : rx;
      if (pv) {
        float E[PT][C], Co[PT][C], Pc[PT][C];
        // H gathers accumulate straight into the slots of voxels p-1 and p.
        float hC[PT][CH];
#pragma unroll
        for (int k = 0; k < PT; ++k) {
#pragma unroll
          for (int j = 0; j < C; ++j) E[k][j] = Co[k][j] = Pc[k][j] = 0.f;
#pragma unroll
          for (int j = 0; j < CH; ++j) hC[k][j] = 0.f;
        }
        const float xcB = xs[SB];
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy) {
#pragma unroll
          for (int dx = -1; dx <= 1; ++dx) {
            const float xk = sx_at(bp, dy, dx);
            const int n = (dx != 0) + (dy != 0);
            // eq (6), formed once for all particles
            const float gA = fabsf(xcA - xk), gB = fabsf(xcB - xk), gC = fabsf(xC - xk);
#pragma unroll
            for (int k = 0; k < PT; ++k) {
              float u[C];
              su_at(bp, k, dy, dx, u);
#pragma unroll
              for (int j = 0; j < C; ++j) {
                if (n == 0) Pc[k][j] = u[j] * u[j];
                else if (n == 1) E[k][j] = fmaf(u[j], u[j], E[k][j]);
                else Co[k][j] = fmaf(u[j], u[j], Co[k][j]);
              }
              if (doA) {
#pragma unroll
                for (int j = 0; j < CH; ++j) hn[SA][k][j] = fmaf(u[j], gA, hn[SA][k][j]);
              }
              if (doB && n != 0) {
#pragma unroll
                for (int j = 0; j < CH; ++j) hn[SB][k][j] = fmaf(u[j], gB, hn[SB][k][j]);
              }
              if (doC) {
#pragma unroll
                for (int j = 0; j < CH; ++j) hC[k][j] = fmaf(u[j], gC, hC[k][j]);
              }
            }
          }
          // With two particles, one row of cells at a time: keeps the row's
          // LDS reads, not the whole window's, in registers.
          if constexpr (PT > 1) __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int k = 0; k < PT; ++k) {
          float Sa[C], Sb[C];
#pragma unroll
          for (int j = 0; j < C; ++j) {
            Sa[j] = fmaf(wCa, Co[k][j], wEa * E[k][j]);
            Sb[j] = fmaf(wCb, Co[k][j], fmaf(wEb, E[k][j], wPb * Pc[k][j]));
          }
          if (doA) {
#pragma unroll
            for (int j = 0; j < C; ++j) fn[SA][k][j] += Sb[j];
          }
          if (doB) {
#pragma unroll
            for (int j = 0; j < C; ++j) fn[SB][k][j] += Sa[j];
          }
          if (doC) {
#pragma unroll
            for (int j = 0; j < CH; ++j) hn[SC][k][j] = hC[k][j];
#pragma unroll
            for (int j = 0; j < C; ++j) fn[SC][k][j] = Sb[j];
          }
        }
        // The gathers are complete here: the compiler may not sink them past
        // the staging below (which waits on the prefetch loads).
#pragma unroll
        for (int s2 = 0; s2 < 3; ++s2) {
#pragma unroll
          for (int k = 0; k < PT; ++k) {
#pragma unroll
            for (int j = 0; j < CH; ++j) asm volatile("" : "+v"(hn[s2][k][j]));
#pragma unroll
            for (int j = 0; j < C; ++j) asm volatile("" : "+v"(fn[s2][k][j]));
          }
        }
      } else if (doC) {
#pragma unroll
        for (int k = 0; k < PT; ++k) {
#pragma unroll
          for (int j = 0; j < CH; ++j) hn[SC][k][j] = 0.f;
#pragma unroll
          for (int j = 0; j < C; ++j) fn[SC][k][j] = 0.f;
        }
      }
      // Stage plane p+1 and prefetch p+2 before finalising p-1: the global
      // store of p-1's memberships then has a whole plane of work to drain
      // before the next wait on the prefetch loads.  The fence keeps the
      // staging (and its wait for the prefetch) after this plane's gathers.
      __builtin_amdgcn_sched_barrier(0);
      if (!GEN || p + 1 <= zhi) {
        store_plane(bnext, std::integral_constant<bool, !GEN>{});
        gs[SC] = rg;
        xs[SC] = xC;
        if (!GEN || p + 2 <= zhi) load_plane(p + 2, std::integral_constant<bool, !GEN>{});
      }
      if (doA) finalize(p - 1, SAc, bprev);
      // Keep the next plane's gathers after this plane's store.
      __builtin_amdgcn_sched_barrier(0);
    };

    // Canonical slot ring: slot 0 = voxel p-1, 1 = p, 2 = p+1.  After a plane
    // processed with the canonical slots, move the ring down by one.
    auto shift = [&]() __attribute__((always_inline)) {
#pragma unroll
      for (int s2 = 0; s2 < 2; ++s2) {
        gs[s2] = gs[s2 + 1];
        xs[s2] = xs[s2 + 1];
#pragma unroll
        for (int k = 0; k < PT; ++k) {
#pragma unroll
          for (int j = 0; j < CH; ++j) hn[s2][k][j] = hn[s2 + 1][k][j];
#pragma unroll
          for (int j = 0; j < C; ++j) fn[s2][k][j] = fn[s2 + 1][k][j];
        }
      }
    };

    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using Bdyn = std::integral_constant<int, -1>;
    using Gen = std::integral_constant<bool, true>;
    using Steady = std::integral_constant<bool, false>;
    using Full = std::integral_constant<bool, false>;  // staging forms

    // Prologue: stage plane zlo-1 (zeros outside the volume) in buffer 0,
    // prefetch zlo.
    load_plane(zlo - 1, Full{});
    store_plane(0, Full{});
    load_plane(zlo, Full{});
    // The tile's first two planes, the interior in groups of three, the
    // rest.  Three loops rather than one, so the interior loop's back edge
    // carries the slots in the registers they entered with (no copies).
    // The interior's last prefetch reads plane p + 4 <= zhi, which is nz
    // when the tile ends at the volume's last plane: load_plane keeps its
    // plane-range test.  tests/test_plane_walk.py replays this walk.
    int p = zlo - 1;
    for (; p <= zlo && p <= zhi; ++p) {
      plane(p, I0{}, I1{}, I2{}, Bdyn{}, Gen{});
      shift();
    }
    // Interior planes (entered at p = zlo + 1 + 3k, whose plane sits in
    // buffer 2): every test is true, slots rotate by name.
    for (; p + 4 <= zhi; p += 3) {
      plane(p, I0{}, I1{}, I2{}, I2{}, Steady{});
      plane(p + 1, I1{}, I2{}, I0{}, I0{}, Steady{});
      plane(p + 2, I2{}, I0{}, I1{}, I1{}, Steady{});
    }
    for (; p <= zhi; ++p) {
      plane(p, I0{}, I1{}, I2{}, Bdyn{}, Gen{});
      shift();
    }

#pragma unroll
    for (int k = 0; k < PT; ++k)
      if (live[k]) wave_tile_store<NV>(pr[k], tile, acc[k]);
  }
  if (handout && lane == 0) {
    __threadfence();
    if (atomicAdd(a.work + 8 + xcd, 1) == waves - 1) {
      atomicExch(a.work + xcd, 0);
      atomicExch(a.work + 8 + xcd, 0);
    }
  }
}

// Launch / occupancy of one C with NW waves per work group and PT particles
// per work item.  NW and PT variants exist only where ALL_NW is set (the
// C = 4 fast path); elsewhere NW = 4 and PT = 1.
template <int C, bool M2, int NW, int PT>
static hipError_t launch_gather_ct(const LaunchArgs& a, int grid, bool step, hipStream_t s) {
  if (step) hipLaunchKernelGGL((k_ifcm_gather<C, M2, NW, true, PT>), dim3(grid), dim3(64 * NW), 0, s, a);
  else hipLaunchKernelGGL((k_ifcm_gather<C, M2, NW, false, PT>), dim3(grid), dim3(64 * NW), 0, s, a);
  return hipGetLastError();
}

template <int C, bool M2, int NW, int PT>
static int occ_gather_ct(bool step) {
  int n = 0;
  const void* f = step ? reinterpret_cast<const void*>(&k_ifcm_gather<C, M2, NW, true, PT>)
                       : reinterpret_cast<const void*>(&k_ifcm_gather<C, M2, NW, false, PT>);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, 64 * NW, 0) != hipSuccess) n = 1;
  return std::max(n, 1);
}

template <int C, int NW, int PT>
static hipError_t launch_gather_m(const LaunchArgs& a, int grid, bool m2, bool step, hipStream_t s) {
  return m2 ? launch_gather_ct<C, true, NW, PT>(a, grid, step, s) : launch_gather_ct<C, false, NW, PT>(a, grid, step, s);
}

template <int C, int NW, int PT>
static int occ_gather_m(bool m2, bool step) {
  return m2 ? occ_gather_ct<C, true, NW, PT>(step) : occ_gather_ct<C, false, NW, PT>(step);
}

template <int C, bool ALL_NW>
static hipError_t launch_gather_one(const LaunchArgs& a, int grid, int nw, bool m2, bool step,
                                    hipStream_t s) {
  if constexpr (ALL_NW) {
    if (a.pt == 2) {
      switch (nw) {
        case 1: return launch_gather_m<C, 1, 2>(a, grid, m2, step, s);
        case 2: return launch_gather_m<C, 2, 2>(a, grid, m2, step, s);
        case 4: return launch_gather_m<C, 4, 2>(a, grid, m2, step, s);
        default: return hipErrorInvalidValue;
      }
    }
    if (a.pt != 1) return hipErrorInvalidValue;
    switch (nw) {
      case 1: return launch_gather_m<C, 1, 1>(a, grid, m2, step, s);
      case 2: return launch_gather_m<C, 2, 1>(a, grid, m2, step, s);
      case 4: return launch_gather_m<C, 4, 1>(a, grid, m2, step, s);
      default: return hipErrorInvalidValue;
    }
  } else {
    if (nw != 4 || a.pt != 1) return hipErrorInvalidValue;
    return launch_gather_m<C, 4, 1>(a, grid, m2, step, s);
  }
}

template <int C, bool ALL_NW>
static int occ_gather_one(int nw, int pt, bool m2, bool step) {
  if constexpr (ALL_NW) {
    if (pt == 2) {
      switch (nw) {
        case 1: return occ_gather_m<C, 1, 2>(m2, step);
        case 2: return occ_gather_m<C, 2, 2>(m2, step);
        case 4: return occ_gather_m<C, 4, 2>(m2, step);
        default: return 1;
      }
    }
    switch (nw) {
      case 1: return occ_gather_m<C, 1, 1>(m2, step);
      case 2: return occ_gather_m<C, 2, 1>(m2, step);
      case 4: return occ_gather_m<C, 4, 1>(m2, step);
      default: return 1;
    }
  } else {
    return occ_gather_m<C, 4, 1>(m2, step);
  }
}

// One translation unit per group of C defines these for its C values.
#define PIFCM_DEFINE_GATHER(c, all_nw)                                                     \
  hipError_t launch_gather_C##c(const LaunchArgs& a, int grid, int nw, bool m2, bool step, \
                                hipStream_t s) {                                           \
    return launch_gather_one<c, all_nw>(a, grid, nw, m2, step, s);                         \
  }                                                                                        \
  int occ_gather_C##c(int nw, int pt, bool m2, bool step) { return occ_gather_one<c, all_nw>(nw, pt, m2, step); }

}  // namespace pifcm
