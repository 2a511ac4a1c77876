// pointwise.hip -- the per-voxel kernels of libpifcm (plain FCM step for
// lambda = xi = 0, initial memberships, iteration invariants, labels,
// normalisation, checks) and the dispatchers over the cluster count.
#include "common.h"
#include "pifcm_kernels.h"

namespace pifcm {

// ------------------------------------------------ pointwise FCM (lambda=xi=0)
// With lambda = xi = 0 the attraction factor of eq (4) is exactly 1, so H and
// F are not needed and the step is plain FCM (eqs (1)-(3)).
template <int C, bool M2, bool STEP>
__global__ __launch_bounds__(256) void k_fcm_point(const LaunchArgs a) {
  constexpr int NT = 256;
  constexpr int NV = STEP ? 2 * C + 1 : 1;
  __shared__ float s_red[(NT / 64) * NV];
  const int xcd = blockIdx.x & 7;
  const int it_end = a.xcd_begin[xcd + 1];
  for (int it = a.xcd_begin[xcd] + (blockIdx.x >> 3); it < it_end; it += gridDim.x >> 3) {
    const int b = vol_of_item(a, it);
    const VolDev vd = ld_const(a.vols + b);
    const int r = it - a.item_begin[b];
    const int pidx = r / vd.tiles1d;
    const int tile = r - pidx * vd.tiles1d;
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
    const size_t psz = (size_t)vd.nx * vd.ny;
    const size_t N = (size_t)vd.zend * psz;  // end of the planes iterated
    float acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = 0.f;
    const size_t base = (size_t)vd.zbeg * psz + (size_t)tile * NT * kFcmVoxPerThread;
#pragma unroll 2
    for (int k = 0; k < kFcmVoxPerThread; ++k) {
      const size_t i = base + (size_t)k * NT + threadIdx.x;
      if (i >= N) break;
      const float xv = X[i];
      float uo[C], d2[C];
      load_row<C>(Uin + i * C, uo);
      float Jv = 0.f;
#pragma unroll
      for (int j = 0; j < C; ++j) {
        const float dd = xv - cj[j];
        d2[j] = fmaxf(dd * dd, kDFloor);
        Jv = fmaf(pow_m<M2>(uo[j], a.m), d2[j], Jv);
      }
      if constexpr (STEP) {
        float un[C];
        memberships<C, M2>(d2, a.m, un);
        store_row<C>(Uout + i * C, un);
#pragma unroll
        for (int j = 0; j < C; ++j) {
          const float w = pow_m<M2>(un[j], a.m);
          acc[j] = fmaf(w, xv, acc[j]);
          acc[C + j] += w;
        }
        acc[2 * C] += Jv;
      } else {
        acc[0] += Jv;
      }
    }
    block_tile_store<NV, NT>(pr, tile, acc, s_red);
  }
}

// ----------------------------------------------------------- small kernels
// Iteration invariants of one volume: g_inv = 1 / sum_k |x_i - x_k| over the
// in-volume 3x3x3 neighbourhood (denominator of eq (5)); for a voxel whose
// neighbours all have its intensity, -1 / (number of neighbours), which the
// fused step turns into the equal-weight mean; 0 for a voxel without
// neighbours.  Also flags non-finite intensities.
// A work group covers 64 x 4 columns of the volume (the x-y tile of
// blockIdx.x) and walks planes blockIdx.y, blockIdx.y + gridDim.y, ...: the
// voxel position comes from the launch shape, not from dividing a flat
// index.  The neighbours are read through the caches in a fixed order.
__global__ __launch_bounds__(256) void k_invariants(const float* __restrict__ x, float* __restrict__ invg,
                                                    int nx, int ny, int nz, int* __restrict__ flag) {
  const int ntx = (nx + 63) >> 6;
  const int gx = (int)(blockIdx.x % ntx) * 64 + (int)(threadIdx.x & 63);
  const int gy = (int)(blockIdx.x / ntx) * 4 + (int)(threadIdx.x >> 6);
  if (gx >= nx || gy >= ny) return;
  bool bad = false;
  for (int gz = blockIdx.y; gz < nz; gz += gridDim.y) {
    const size_t i = ((size_t)gz * ny + gy) * nx + gx;
    const float xi = x[i];
    bad = bad || !isfinite(xi);
    float gsum = 0.f;
    int cnt = 0;
    for (int dz = -1; dz <= 1; ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          const int X2 = gx + dx, Y2 = gy + dy, Z2 = gz + dz;
          if ((dx | dy | dz) == 0 || X2 < 0 || X2 >= nx || Y2 < 0 || Y2 >= ny || Z2 < 0 || Z2 >= nz)
            continue;
          gsum += fabsf(xi - x[((size_t)Z2 * ny + Y2) * nx + X2]);
          ++cnt;
        }
    invg[i] = gsum > 0.f ? 1.f / gsum : (cnt > 0 ? -1.f / (float)cnt : 0.f);
  }
  if (bad) atomicOr(flag, 1);
}

// U^(0) from centres (eq (2) with the attraction factor 1).
template <int C, bool M2>
__global__ __launch_bounds__(256) void k_init_u(const float* __restrict__ x, size_t N,
                                                const SolveState* __restrict__ st, float m,
                                                float* __restrict__ U) {
  float cj[C];
#pragma unroll
  for (int j = 0; j < C; ++j) cj[j] = st->c[0][j];
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (size_t)gridDim.x * blockDim.x) {
    const float xv = x[i];
    float d2[C], u[C];
#pragma unroll
    for (int j = 0; j < C; ++j) {
      const float dd = xv - cj[j];
      d2[j] = fmaxf(dd * dd, kDFloor);
    }
    memberships<C, M2>(d2, m, u);
    store_row<C>(as_global(U) + i * C, u);
  }
}

// Rows of a caller's U must be memberships: finite, in [0, 1], sum 1 +- 1e-4.
__global__ __launch_bounds__(256) void k_check_rows(const float* __restrict__ U, size_t N, int C,
                                                    int* __restrict__ flag) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (size_t)gridDim.x * blockDim.x) {
    float s = 0.f;
    bool ok = true;
    for (int j = 0; j < C; ++j) {
      const float u = U[i * C + j];
      ok = ok && isfinite(u) && u >= 0.f && u <= 1.f + 1e-6f;
      s += u;
    }
    if (!ok || fabsf(s - 1.f) > 1e-4f) atomicOr(flag, 1);
  }
}

// Labels: argmax_j u_ij, ties to the lowest j.
__global__ __launch_bounds__(256) void k_labels(const float* __restrict__ U, size_t N, int C,
                                                uint8_t* __restrict__ out) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (size_t)gridDim.x * blockDim.x) {
    int best = 0;
    float bv = U[i * C];
    for (int j = 1; j < C; ++j) {
      const float v = U[i * C + j];
      if (v > bv) {
        bv = v;
        best = j;
      }
    }
    out[i] = (uint8_t)best;
  }
}

// Confusion counts of labels (0..C-1) against reference classes (0..K-1):
// counts[j * K + k] += #{i : labels_i = j, truth_i = k}; pairs outside the
// ranges go to counts[C * K].  Per-block LDS histogram, then one atomic add
// per bin (integer sums: the result does not depend on the order).
__global__ __launch_bounds__(256) void k_confusion(const uint8_t* __restrict__ labels,
                                                   const uint8_t* __restrict__ truth, size_t N,
                                                   int C, int K, unsigned long long* counts) {
  __shared__ uint32_t h[kMaxC * kMaxC + 1];
  const int nb = C * K + 1;
  for (int t = threadIdx.x; t < nb; t += blockDim.x) h[t] = 0u;
  __syncthreads();
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (size_t)gridDim.x * blockDim.x) {
    const int j = labels[i], k = truth[i];
    atomicAdd(&h[(j < C && k < K) ? j * K + k : C * K], 1u);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < nb; t += blockDim.x)
    if (h[t]) atomicAdd(&counts[t], (unsigned long long)h[t]);
}

struct Perm {
  int32_t p[kMaxC];
};
// In place allowed: each row is read whole before it is written.
__global__ __launch_bounds__(256) void k_permute(const float* U, size_t N, int C, Perm perm,
                                                 float* out) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (size_t)gridDim.x * blockDim.x) {
    float row[kMaxC];
    for (int j = 0; j < C; ++j) row[j] = U[i * C + perm.p[j]];
    for (int j = 0; j < C; ++j) out[i * C + j] = row[j];
  }
}

// Min-max normalisation (Algorithm 2 step 1).  Floats are mapped to
// order-preserving unsigned keys so min/max are exact integer atomics.
__device__ __forceinline__ uint32_t fkey(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float kinv(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}
__global__ __launch_bounds__(256) void k_minmax(const float* __restrict__ raw, size_t n,
                                                uint32_t* __restrict__ mm, int* __restrict__ flag) {
  uint32_t lo = 0xffffffffu, hi = 0u;
  bool bad = false;
  auto take = [&](float v) {
    bad = bad || !isfinite(v);
    const uint32_t k = fkey(v);
    lo = min(lo, k);
    hi = max(hi, k);
  };
  // Four independent loads in flight per thread, then the remainder.
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    const float v0 = raw[i], v1 = raw[i + stride], v2 = raw[i + 2 * stride], v3 = raw[i + 3 * stride];
    take(v0);
    take(v1);
    take(v2);
    take(v3);
  }
  for (; i < n; i += stride) take(raw[i]);
  // Wave, then work group, then one atomic per work group and key (min and
  // max of the keys do not depend on the order).
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    lo = min(lo, (uint32_t)__shfl_xor((int)lo, o, 64));
    hi = max(hi, (uint32_t)__shfl_xor((int)hi, o, 64));
  }
  __shared__ uint32_t s_lo[4], s_hi[4];
  __shared__ int s_bad;
  if (threadIdx.x == 0) s_bad = 0;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    s_lo[threadIdx.x >> 6] = lo;
    s_hi[threadIdx.x >> 6] = hi;
  }
  if (bad) s_bad = 1;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 4; ++w) {
      lo = min(lo, s_lo[w]);
      hi = max(hi, s_hi[w]);
    }
    atomicMin(&mm[0], lo);
    atomicMax(&mm[1], hi);
    if (s_bad) atomicOr(flag, 1);
  }
}
__global__ __launch_bounds__(256) void k_normalize(const float* raw, size_t n,
                                                   const uint32_t* __restrict__ mm, float* out) {
  const double mn = (double)kinv(mm[0]), mx = (double)kinv(mm[1]);
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    out[i] = mx == mn ? 0.f : (float)(((double)raw[i] - mn) / (mx - mn));
  }
}

// ------------------------------------------------------------- dispatchers
template <int C>
static hipError_t launch_fcm_c(const LaunchArgs& a, int grid, bool m2, bool step, hipStream_t s) {
  if (m2) {
    if (step) hipLaunchKernelGGL((k_fcm_point<C, true, true>), dim3(grid), dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_fcm_point<C, true, false>), dim3(grid), dim3(256), 0, s, a);
  } else {
    if (step) hipLaunchKernelGGL((k_fcm_point<C, false, true>), dim3(grid), dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_fcm_point<C, false, false>), dim3(grid), dim3(256), 0, s, a);
  }
  return hipGetLastError();
}

template <int C>
static hipError_t launch_finalize_c(const LaunchArgs& a, int npairs, bool step, hipStream_t s) {
  if (step) hipLaunchKernelGGL((k_finalize<C, true>), dim3(npairs), dim3(256), 0, s, a);
  else hipLaunchKernelGGL((k_finalize<C, false>), dim3(npairs), dim3(256), 0, s, a);
  return hipGetLastError();
}

template <int C>
static hipError_t launch_init_c(const float* x, size_t N, const SolveState* st, float m, bool m2,
                                float* U, hipStream_t s) {
  const int grid = (int)std::min<size_t>((N + 255) / 256, 65536);
  if (m2) hipLaunchKernelGGL((k_init_u<C, true>), dim3(grid), dim3(256), 0, s, x, N, st, m, U);
  else hipLaunchKernelGGL((k_init_u<C, false>), dim3(grid), dim3(256), 0, s, x, N, st, m, U);
  return hipGetLastError();
}

#define PIFCM_FOR_EACH_C(X) \
  X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)

#define DECL(c)                                                                              \
  hipError_t launch_gather_C##c(const LaunchArgs& a, int grid, int ty, bool m2, bool step, \
                                hipStream_t s);                                            \
  int occ_gather_C##c(int ty, int pt, bool m2, bool step);
PIFCM_FOR_EACH_C(DECL)
#undef DECL

hipError_t launch_gather(int C, const LaunchArgs& a, int grid, int ty, bool m2, bool step,
                         hipStream_t s) {
  switch (C) {
#define CASE(c) \
  case c: return launch_gather_C##c(a, grid, ty, m2, step, s);
    PIFCM_FOR_EACH_C(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

int gather_occupancy(int C, int ty, int pt, bool m2, bool step) {
  switch (C) {
#define CASE(c) \
  case c: return occ_gather_C##c(ty, pt, m2, step);
    PIFCM_FOR_EACH_C(CASE)
#undef CASE
    default: return 1;
  }
}

hipError_t launch_fcm(int C, const LaunchArgs& a, int grid, bool m2, bool step, hipStream_t s) {
  switch (C) {
#define CASE(c) \
  case c: return launch_fcm_c<c>(a, grid, m2, step, s);
    PIFCM_FOR_EACH_C(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_finalize(int C, const LaunchArgs& a, int npairs, bool step, hipStream_t s) {
  switch (C) {
#define CASE(c) \
  case c: return launch_finalize_c<c>(a, npairs, step, s);
    PIFCM_FOR_EACH_C(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_init_u(int C, const float* x, size_t N, const SolveState* st, float m, bool m2,
                         float* U, hipStream_t s) {
  switch (C) {
#define CASE(c) \
  case c: return launch_init_c<c>(x, N, st, m, m2, U, s);
    PIFCM_FOR_EACH_C(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

static int small_grid(size_t n) { return (int)std::max<size_t>(1, std::min<size_t>((n + 255) / 256, 65536)); }

hipError_t launch_invariants(const float* x, float* invg, int nx, int ny, int nz, int* flag,
                             hipStream_t s) {
  const long tiles = (long)((nx + 63) / 64) * ((ny + 3) / 4);
  if (tiles > 0x7fffffffL) return hipErrorInvalidValue;
  const int planes = std::max(1, std::min(nz, 65535));
  hipLaunchKernelGGL(k_invariants, dim3((unsigned)tiles, (unsigned)planes), dim3(256), 0, s, x, invg, nx, ny,
                     nz, flag);
  return hipGetLastError();
}

hipError_t launch_check_rows(const float* U, size_t N, int C, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_check_rows, dim3(small_grid(N)), dim3(256), 0, s, U, N, C, flag);
  return hipGetLastError();
}

hipError_t launch_labels(const float* U, size_t N, int C, uint8_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_labels, dim3(small_grid(N)), dim3(256), 0, s, U, N, C, out);
  return hipGetLastError();
}

hipError_t launch_confusion(const uint8_t* labels, const uint8_t* truth, size_t N, int C, int K,
                            unsigned long long* counts, hipStream_t s) {
  hipLaunchKernelGGL(k_confusion, dim3(small_grid(N)), dim3(256), 0, s, labels, truth, N, C, K, counts);
  return hipGetLastError();
}

hipError_t launch_permute(const float* U, size_t N, int C, const int32_t* perm, float* out,
                          hipStream_t s) {
  Perm p{};
  for (int j = 0; j < C; ++j) p.p[j] = perm[j];
  hipLaunchKernelGGL(k_permute, dim3(small_grid(N)), dim3(256), 0, s, U, N, C, p, out);
  return hipGetLastError();
}

hipError_t launch_minmax(const float* raw, size_t n, uint32_t* mm, int* flag, hipStream_t s) {
  // 256 threads per work group (the reduction above assumes four waves)
  const int g = std::min(small_grid(n), 1024);
  hipLaunchKernelGGL(k_minmax, dim3(g), dim3(256), 0, s, raw, n, mm, flag);
  return hipGetLastError();
}

hipError_t launch_scale(const float* raw, size_t n, const uint32_t* mm, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_normalize, dim3(small_grid(n)), dim3(256), 0, s, raw, n, mm, out);
  return hipGetLastError();
}

template <int C>
static int occ_fcm_c(bool m2, bool step) {
  int n = 0;
  const void* f;
  if (m2) f = step ? reinterpret_cast<const void*>(&k_fcm_point<C, true, true>)
                   : reinterpret_cast<const void*>(&k_fcm_point<C, true, false>);
  else f = step ? reinterpret_cast<const void*>(&k_fcm_point<C, false, true>)
                : reinterpret_cast<const void*>(&k_fcm_point<C, false, false>);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, 256, 0) != hipSuccess) n = 1;
  return std::max(n, 1);
}

int fcm_occupancy(int C, bool m2, bool step) {
  switch (C) {
#define CASE(c) \
  case c: return occ_fcm_c<c>(m2, step);
    PIFCM_FOR_EACH_C(CASE)
#undef CASE
    default: return 1;
  }
}

}  // namespace pifcm
