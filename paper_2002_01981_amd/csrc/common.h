// common.h -- device helpers shared by the kernels of libpifcm.
#pragma once
#include <algorithm>
#include <type_traits>

#include "pifcm_device.h"

namespace pifcm {

// Global-memory views of pointers read from descriptor tables: loads and
// stores through them are global (not flat) instructions.
typedef __attribute__((address_space(1))) float gfloat;
__device__ __forceinline__ const gfloat* as_global(const float* p) { return (const gfloat*)p; }
__device__ __forceinline__ gfloat* as_global(float* p) { return (gfloat*)p; }

// base + a 32-bit byte offset: with a uniform base this is the scalar-base
// plus vector-offset form of the global instructions (no 64-bit address math).
__device__ __forceinline__ const gfloat* at_byte(const gfloat* base, uint32_t off) {
  return (const gfloat*)((const __attribute__((address_space(1))) char*)base + off);
}
__device__ __forceinline__ gfloat* at_byte(gfloat* base, uint32_t off) {
  return (gfloat*)((__attribute__((address_space(1))) char*)base + off);
}

// Read-only descriptor data (tables, particle state) through the constant
// address space: uniform reads become scalar loads.
template <typename T>
__device__ __forceinline__ T ld_const(const T* p) {
  static_assert(sizeof(T) % 4 == 0, "word-sized descriptors only");
  typedef const __attribute__((address_space(4))) uint32_t CW;
  T out;
  uint32_t* o = reinterpret_cast<uint32_t*>(&out);
  CW* q = (CW*)p;
#pragma unroll
  for (unsigned i = 0; i < sizeof(T) / 4; ++i) o[i] = q[i];
  return out;
}

typedef float f4v __attribute__((ext_vector_type(4)));
typedef float f2v __attribute__((ext_vector_type(2)));

__device__ __forceinline__ float frcp(float v) { return __builtin_amdgcn_rcpf(v); }

// A pointer that is the same in every lane, pinned to scalar registers (a
// select of descriptor fields can otherwise leave it in vector registers, to
// be read back before every memory instruction that uses it as a base).
template <typename T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return reinterpret_cast<T*>(((uint64_t)hi << 32) | lo);
}

// A uniform base the optimiser may not re-associate with a lane offset: kept
// in scalar registers, so base + 32-bit lane offset stays one memory
// instruction with no vector address arithmetic.
template <typename T>
__device__ __forceinline__ T* opaque_base(T* p) {
  asm("" : "+s"(p));
  return p;
}
// base + a lane offset held in a variable that is redefined (in place, no
// code) at each use: its widening then stays next to the access instead of
// being hoisted out of the loop as a 64-bit vector address.
__device__ __forceinline__ const gfloat* at_lane(const gfloat* base, uint32_t& off) {
  asm("" : "+v"(off));
  return at_byte(base, off);
}
__device__ __forceinline__ gfloat* at_lane(gfloat* base, uint32_t& off) {
  asm("" : "+v"(off));
  return at_byte(base, off);
}

__device__ __forceinline__ int vol_of_item(const LaunchArgs& a, int it) {
  int b = 0;
  while (b + 1 < a.nvol && it >= a.item_begin[b + 1]) ++b;
  return b;
}

// Row of C memberships in global memory (16-byte aligned when C % 4 == 0).
template <int C>
__device__ __forceinline__ void load_row(const gfloat* p, float (&u)[C]) {
  typedef __attribute__((address_space(1))) const f4v G4;
  typedef __attribute__((address_space(1))) const f2v G2;
  if constexpr (C % 4 == 0) {
#pragma unroll
    for (int q = 0; q < C / 4; ++q) {
      const f4v v = reinterpret_cast<G4*>(p)[q];
      u[4 * q] = v.x;
      u[4 * q + 1] = v.y;
      u[4 * q + 2] = v.z;
      u[4 * q + 3] = v.w;
    }
  } else if constexpr (C % 2 == 0) {
#pragma unroll
    for (int q = 0; q < C / 2; ++q) {
      const f2v v = reinterpret_cast<G2*>(p)[q];
      u[2 * q] = v.x;
      u[2 * q + 1] = v.y;
    }
  } else {
#pragma unroll
    for (int j = 0; j < C; ++j) u[j] = p[j];
  }
}

template <int C>
__device__ __forceinline__ void store_row(gfloat* p, const float (&u)[C]) {
  typedef __attribute__((address_space(1))) f4v G4;
  typedef __attribute__((address_space(1))) f2v G2;
  if constexpr (C % 4 == 0) {
#pragma unroll
    for (int q = 0; q < C / 4; ++q) {
      f4v v;
      v.x = u[4 * q];
      v.y = u[4 * q + 1];
      v.z = u[4 * q + 2];
      v.w = u[4 * q + 3];
      reinterpret_cast<G4*>(p)[q] = v;
    }
  } else if constexpr (C % 2 == 0) {
#pragma unroll
    for (int q = 0; q < C / 2; ++q) {
      f2v v;
      v.x = u[2 * q];
      v.y = u[2 * q + 1];
      reinterpret_cast<G2*>(p)[q] = v;
    }
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

// Memberships of eq (2) from squared distances d2[0..C), d2 > 0, times
// scale (1, or 0 to zero a row).
// m == 2: u_j = (1/d2_j) / sum_k (1/d2_k).  Otherwise u_j is proportional to
// (d2_min / d2_j)^(1/(m-1)), which is eq (2) scaled so no term overflows.
template <int C, bool M2>
__device__ __forceinline__ void memberships(const float (&d2)[C], float m, float (&u)[C],
                                            float scale = 1.f) {
  if constexpr (M2 && C <= 4) {
    // u_j = P_j / sum_k P_k with P_j the product of the other d2: one
    // reciprocal.  d2 lies in [1e-12, 2e3] (|lambda|, |xi| <= 1e3), so the
    // products of at most three stay within float32's normal range.
    float P[C];
    if constexpr (C == 2) {
      P[0] = d2[1];
      P[1] = d2[0];
    } else if constexpr (C == 3) {
      P[0] = d2[1] * d2[2];
      P[1] = d2[0] * d2[2];
      P[2] = d2[0] * d2[1];
    } else {
      const float d01 = d2[0] * d2[1], d23 = d2[2] * d2[3];
      P[0] = d2[1] * d23;
      P[1] = d2[0] * d23;
      P[2] = d2[3] * d01;
      P[3] = d2[2] * d01;
    }
    float s = 0.f;
#pragma unroll
    for (int j = 0; j < C; ++j) s += P[j];
    const float r = frcp(s) * scale;
#pragma unroll
    for (int j = 0; j < C; ++j) u[j] = P[j] * r;
  } else if constexpr (M2) {
    float s = 0.f;
#pragma unroll
    for (int j = 0; j < C; ++j) {
      u[j] = frcp(d2[j]);
      s += u[j];
    }
    const float r = frcp(s) * scale;
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
    const float r = scale / s;
#pragma unroll
    for (int j = 0; j < C; ++j) u[j] *= r;
  }
}

// ------------------------------------------------------------ tile sums
// Every tile of a launch leaves NV fp32 sums in its own slot of the pair's
// partials ([tile][NV]); a per-pair finalise kernel launched right after adds
// the slots in fp64 in tile order.  Both reductions have a fixed order, so
// the results do not depend on scheduling.

// Wave owning a tile: butterfly over the 64 lanes, lane 0 stores the slot.
template <int NV>
__device__ __forceinline__ void wave_tile_store(const PairDev& pr, int tile, float (&acc)[NV]) {
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    float v = acc[k];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    acc[k] = v;
  }
  if ((threadIdx.x & 63) == 0) {
    gfloat* slot = as_global(pr.partials) + (size_t)tile * NV;
#pragma unroll
    for (int k = 0; k < NV; ++k) slot[k] = acc[k];
  }
}

// Work group owning a tile: butterfly per wave, waves in order through LDS.
template <int NV, int NT>
__device__ __forceinline__ void block_tile_store(const PairDev& pr, int tile, float (&acc)[NV],
                                                 float* s_red) {
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
  if (threadIdx.x < NV) {
    float s = 0.f;
#pragma unroll
    for (int w = 0; w < NW; ++w) s += s_red[w * NV + threadIdx.x];
    as_global(pr.partials)[(size_t)tile * NV + threadIdx.x] = s;
  }
  __syncthreads();
}

// Advance the state of a pair from its fp64 totals (one thread): new centres
// (eq (3)), J of the iteration's input state (eq (1)) and the stop rule; or,
// for the objective-only pass, the fitness.
template <int C, bool STEP>
__device__ __forceinline__ void finish_pair(SolveState* st, const double* tot) {
  if constexpr (STEP) {
    const int t = st->iter + 1;
    const int par = t & 1;
#pragma unroll
    for (int j = 0; j < C; ++j) {
      const double den = tot[C + j];
      st->c[par][j] = den > 0.0 ? (float)(tot[j] / den) : st->c[par ^ 1][j];
    }
    if (st->B_hist)
      for (int j = 0; j < C; ++j) st->B_hist[(size_t)(t - 1) * C + j] = tot[C + j];
    if (st->c_hist)
      for (int j = 0; j < C; ++j) st->c_hist[(size_t)t * C + j] = st->c[par][j];
    const double J = tot[2 * C];
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
}

// One work group per pair: add the pair's tile slots in fp64 (thread t takes
// tiles t, t + 256, ...; then a fixed butterfly and the waves in order) and
// advance its state.  Pairs that have stopped are left alone.
template <int C, bool STEP>
__global__ __launch_bounds__(256) void k_finalize(const LaunchArgs a) {
  constexpr int NV = STEP ? 2 * C + 1 : 1;
  __shared__ double s_red[4 * NV];
  const int pair = blockIdx.x;
  const PairDev pr = a.pairs[pair];
  SolveState* st = pr.st;
  if (STEP && st->stop) return;
  const VolDev vd = a.vols[pair / a.P];
  const int tiles = a.use_1d ? vd.tiles1d : vd.tiles;
  double d[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) d[k] = 0.0;
  const gfloat* parts = as_global(pr.partials);
  // Each thread adds the slots s, s + 256, s + 512, ... in that order; eight
  // of them are loaded at once so their latencies overlap (the order of the
  // additions, and so the result, is that of the plain strided loop).
  constexpr int kU = 8;
  int s = threadIdx.x;
  for (; s + (kU - 1) * 256 < tiles; s += kU * 256) {
    float v[kU][NV];
#pragma unroll
    for (int u = 0; u < kU; ++u)
#pragma unroll
      for (int k = 0; k < NV; ++k) v[u][k] = parts[(size_t)(s + u * 256) * NV + k];
#pragma unroll
    for (int u = 0; u < kU; ++u)
#pragma unroll
      for (int k = 0; k < NV; ++k) d[k] += (double)v[u][k];
  }
  for (; s < tiles; s += 256) {
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
    double tot[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k)
      tot[k] = ((s_red[k] + s_red[NV + k]) + s_red[2 * NV + k]) + s_red[3 * NV + k];
    finish_pair<C, STEP>(st, tot);
  }
}

}  // namespace pifcm
