// common.h -- device helpers shared by the kernels of libpifcm.
#pragma once
#include <algorithm>
#include <type_traits>

#include "pifcm_device.h"

namespace pifcm {

__device__ __forceinline__ float frcp(float v) { return __builtin_amdgcn_rcpf(v); }

// Items of a launch are split into 8 contiguous ranges, one per XCD (work
// groups are dealt to the 8 XCDs round-robin), so tiles that share halos run
// on the same XCD and meet in its L2.
__device__ __forceinline__ void item_range(int nitems, int& first, int& end, int& step) {
  const int per = (nitems + 7) >> 3;
  const int xcd = blockIdx.x & 7;
  first = xcd * per + (blockIdx.x >> 3);
  end = min(nitems, (xcd + 1) * per);
  step = gridDim.x >> 3;
}

__device__ __forceinline__ int vol_of_item(const LaunchArgs& a, int it) {
  int b = 0;
  while (b + 1 < a.nvol && it >= a.item_begin[b + 1]) ++b;
  return b;
}

template <int C>
__device__ __forceinline__ void load_row(const float* __restrict__ p, float (&u)[C]) {
  if constexpr (C % 4 == 0) {
#pragma unroll
    for (int q = 0; q < C / 4; ++q) {
      const float4 v = reinterpret_cast<const float4*>(p)[q];
      u[4 * q] = v.x;
      u[4 * q + 1] = v.y;
      u[4 * q + 2] = v.z;
      u[4 * q + 3] = v.w;
    }
  } else if constexpr (C % 2 == 0) {
#pragma unroll
    for (int q = 0; q < C / 2; ++q) {
      const float2 v = reinterpret_cast<const float2*>(p)[q];
      u[2 * q] = v.x;
      u[2 * q + 1] = v.y;
    }
  } else {
#pragma unroll
    for (int j = 0; j < C; ++j) u[j] = p[j];
  }
}

template <int C>
__device__ __forceinline__ void store_row(float* __restrict__ p, const float (&u)[C]) {
  if constexpr (C % 4 == 0) {
#pragma unroll
    for (int q = 0; q < C / 4; ++q)
      reinterpret_cast<float4*>(p)[q] = make_float4(u[4 * q], u[4 * q + 1], u[4 * q + 2], u[4 * q + 3]);
  } else if constexpr (C % 2 == 0) {
#pragma unroll
    for (int q = 0; q < C / 2; ++q)
      reinterpret_cast<float2*>(p)[q] = make_float2(u[2 * q], u[2 * q + 1]);
  } else {
#pragma unroll
    for (int j = 0; j < C; ++j) p[j] = u[j];
  }
}

// LDS cell of CP floats (C padded to a multiple of 4) read as float4s.
template <int C, int CP>
__device__ __forceinline__ void lds_cell_load(const float* __restrict__ s, float (&u)[C]) {
#pragma unroll
  for (int q = 0; q < CP / 4; ++q) {
    const float4 v = reinterpret_cast<const float4*>(s)[q];
    if (4 * q < C) u[4 * q] = v.x;
    if (4 * q + 1 < C) u[4 * q + 1] = v.y;
    if (4 * q + 2 < C) u[4 * q + 2] = v.z;
    if (4 * q + 3 < C) u[4 * q + 3] = v.w;
  }
}

template <int C, int CP>
__device__ __forceinline__ void lds_cell_store(float* __restrict__ s, const float (&u)[C]) {
#pragma unroll
  for (int q = 0; q < CP / 4; ++q) {
    float4 v;
    v.x = (4 * q < C) ? u[4 * q] : 0.f;
    v.y = (4 * q + 1 < C) ? u[4 * q + 1] : 0.f;
    v.z = (4 * q + 2 < C) ? u[4 * q + 2] : 0.f;
    v.w = (4 * q + 3 < C) ? u[4 * q + 3] : 0.f;
    reinterpret_cast<float4*>(s)[q] = v;
  }
}

// w = u^m for the centre sums of eq (3) and the objective of eq (1).
template <bool M2>
__device__ __forceinline__ float pow_m(float u, float m) {
  if constexpr (M2) return u * u;
  else return u > 0.f ? exp2f(m * log2f(u)) : 0.f;
}

// Memberships of eq (2) from squared distances d2[0..C), d2 > 0.
// m == 2: u_j = (1/d2_j) / sum_k (1/d2_k).  Otherwise u_j is proportional to
// (d2_min / d2_j)^(1/(m-1)), which is eq (2) scaled so no term overflows.
template <int C, bool M2>
__device__ __forceinline__ void memberships(const float (&d2)[C], float m, float (&u)[C]) {
  if constexpr (M2) {
    float s = 0.f;
#pragma unroll
    for (int j = 0; j < C; ++j) {
      u[j] = frcp(d2[j]);
      s += u[j];
    }
    const float r = frcp(s);
#pragma unroll
    for (int j = 0; j < C; ++j) u[j] *= r;
  } else {
    float dmin = d2[0];
#pragma unroll
    for (int j = 1; j < C; ++j) dmin = fminf(dmin, d2[j]);
    const float e = 1.f / (m - 1.f);
    const float lmin = log2f(dmin);
    float s = 0.f;
#pragma unroll
    for (int j = 0; j < C; ++j) {
      u[j] = exp2f((lmin - log2f(d2[j])) * e);
      s += u[j];
    }
    const float r = 1.f / s;
#pragma unroll
    for (int j = 0; j < C; ++j) u[j] *= r;
  }
}

// ---------------------------------------------------------------- tile end
// Reduce NV per-lane sums over the work group (fixed butterfly, then waves in
// order), store them in the pair's slot for this tile, and let the last tile
// of the pair to finish combine all slots in fp64 and advance the state.
template <int C, int NT, bool STEP>
__device__ __forceinline__ void tile_done(const PairDev& pr, int tile, int tiles,
                                          float (&acc)[STEP ? 2 * C + 1 : 1], float* s_red,
                                          double* s_redd, int* s_flag) {
  constexpr int NV = STEP ? 2 * C + 1 : 1;
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    float v = acc[k];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    acc[k] = v;
  }
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) s_red[wave * NV + k] = acc[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    float* slot = pr.partials + (size_t)tile * NV;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      float s = 0.f;
#pragma unroll
      for (int w = 0; w < NW; ++w) s += s_red[w * NV + k];
      slot[k] = s;
    }
    __threadfence();
    const uint32_t prev = atomicAdd(&pr.st->counter, 1u);
    *s_flag = (prev == (uint32_t)(tiles - 1));
  }
  __syncthreads();
  if (*s_flag) {
    __threadfence();
    double d[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) d[k] = 0.0;
    for (int s = threadIdx.x; s < tiles; s += NT) {
      const float* slot = pr.partials + (size_t)s * NV;
#pragma unroll
      for (int k = 0; k < NV; ++k) d[k] += (double)__builtin_nontemporal_load(slot + k);
    }
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double v = d[k];
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
      d[k] = v;
    }
    if (lane == 0) {
#pragma unroll
      for (int k = 0; k < NV; ++k) s_redd[wave * NV + k] = d[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double tot[NV];
#pragma unroll
      for (int k = 0; k < NV; ++k) {
        tot[k] = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) tot[k] += s_redd[w * NV + k];
      }
      SolveState* st = pr.st;
      if constexpr (STEP) {
        const int t = st->iter + 1;
        const int par = t & 1;
#pragma unroll
        for (int j = 0; j < C; ++j) {
          const double den = tot[C + j];
          st->c[par][j] = den > 0.0 ? (float)(tot[j] / den) : st->c[par ^ 1][j];  // eq (3)
        }
        const double J = tot[2 * C];  // eq (1) of the iteration's input state
        if (st->J_hist) st->J_hist[t - 1] = J;
        int stop = 0;
        if (t >= 2 && st->eps > 0.f && fabs(J - st->J_prev1) <= (double)st->eps * fabs(st->J_prev1))
          stop = 1;
        if (t >= st->max_iter) stop = 1;
        st->J_prev2 = st->J_prev1;
        st->J_prev1 = J;
        st->iter = t;
        st->stop = stop;
      } else {
        st->J_eval = tot[0];
      }
      st->counter = 0u;
    }
  }
  __syncthreads();
}

}  // namespace pifcm
