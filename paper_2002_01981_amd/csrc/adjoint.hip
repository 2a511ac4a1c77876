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
// (U^t, c^t)), k_adj_transpose the gather of dU; per-block sums of dc,
// dlambda and dxi go to slots that k_adj_finalize adds in fp64.
#include "common.h"
#include "pifcm_kernels.h"

namespace pifcm {

constexpr int kAdjThreads = 256;

// Per-voxel stencil view of the 3x3x3 cube: coordinates from the linear
// index (32-bit: volumes hold fewer than 2^32 voxels) and, per axis, whether
// the -1 and +1 neighbours exist.
struct Nbr {
  int nx, ny, nz;
  int gx, gy, gz;
  bool vxm, vxp, vym, vyp, vzm, vzp;
  __device__ __forceinline__ Nbr(int nx_, int ny_, int nz_, size_t i) : nx(nx_), ny(ny_), nz(nz_) {
    const uint32_t ii = (uint32_t)i;
    gx = (int)(ii % (uint32_t)nx);
    const uint32_t r = ii / (uint32_t)nx;
    gy = (int)(r % (uint32_t)ny);
    gz = (int)(r / (uint32_t)ny);
    vxm = gx > 0;
    vxp = gx < nx - 1;
    vym = gy > 0;
    vyp = gy < ny - 1;
    vzm = gz > 0;
    vzp = gz < nz - 1;
  }
  // Neighbour (dx, dy, dz) exists (offsets are compile-time constants).
  __device__ __forceinline__ bool valid(int dx, int dy, int dz) const {
    return (dx < 0 ? vxm : (dx > 0 ? vxp : true)) && (dy < 0 ? vym : (dy > 0 ? vyp : true)) &&
           (dz < 0 ? vzm : (dz > 0 ? vzp : true));
  }
  // Linear index of neighbour (dx, dy, dz) of voxel i.
  __device__ __forceinline__ size_t at(size_t i, int dx, int dy, int dz) const {
    return (size_t)((long long)i + ((long long)dz * ny + dy) * nx + dx);
  }
};

// eq (7) weight of an offset with n non-zero components: n^2, or n.
__device__ __forceinline__ float qweight(int n, bool q2_sqdist) {
  return q2_sqdist ? (float)n : (float)(n * n);
}

template <int C, bool M2, bool EVAL>
__global__ __launch_bounds__(kAdjThreads) void k_adj_point(const AdjArgs a) {
  constexpr int NV = C + 2;  // dc[C], dlambda, dxi
  __shared__ float s_red[(kAdjThreads / 64) * NV];
  const size_t N = (size_t)a.nx * a.ny * a.nz;
  const size_t i = (size_t)blockIdx.x * kAdjThreads + threadIdx.x;
  const float m = a.m;
  float acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0.f;
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
  if (i < N) {
    const Nbr nb(a.nx, a.ny, a.nz, i);
    const float xv = a.x[i];
    const float ig = a.invg[i];
    const float gi = fabsf(ig);
    const float xc = ig < 0.f ? xv - 1.f : xv;
    float Gn[C], Fn[C];
#pragma unroll
    for (int j = 0; j < C; ++j) Gn[j] = Fn[j] = 0.f;
    float qs = 0.f;
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
          if ((dx | dy | dz) == 0 || !nb.valid(dx, dy, dz)) continue;
          const size_t k = nb.at(i, dx, dy, dz);
          const float g = fabsf(xc - a.x[k]);
          const float q = qweight((dx != 0) + (dy != 0) + (dz != 0), a.q2_sqdist);
          qs += q;
          float u[C];
          load_row<C>(as_global(a.U) + k * C, u);
#pragma unroll
          for (int j = 0; j < C; ++j) {
            Gn[j] = fmaf(u[j], g, Gn[j]);
            Fn[j] = fmaf(u[j] * u[j], q, Fn[j]);
          }
        }
    const float iq = qs > 0.f ? 1.f / qs : 0.f;
    float H[C], F[C], av[C], dd[C], e[C], d[C];
#pragma unroll
    for (int j = 0; j < C; ++j) {
      H[j] = Gn[j] * gi;
      F[j] = Fn[j] * iq;
      av[j] = 1.f - a.lam * H[j] - a.xi * F[j];
      dd[j] = xv - cj[j];
      e[j] = dd[j] * dd[j] * av[j];
      d[j] = fmaxf(e[j], kDFloor);
    }
    float dbar[C];
    if constexpr (EVAL) {
      float u[C];
      load_row<C>(as_global(a.U) + i * C, u);
      float direct[C];
#pragma unroll
      for (int j = 0; j < C; ++j) {
        const float um1 = M2 ? u[j] : (u[j] > 0.f ? exp2f((m - 1.f) * log2f(u[j])) : 0.f);
        direct[j] = m * um1 * d[j];
        dbar[j] = pow_m<M2>(u[j], m);
      }
      store_row<C>(as_global(a.Ubar_direct) + i * C, direct);
    } else {
      float w[C], up[C];
      float sw = 0.f;
      if constexpr (M2) {
#pragma unroll
        for (int j = 0; j < C; ++j) {
          w[j] = 1.f / d[j];
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
      const float is = 1.f / sw;
#pragma unroll
      for (int j = 0; j < C; ++j) up[j] = w[j] * is;
      float gin[C];
      load_row<C>(as_global(a.Ubar_next) + i * C, gin);
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
        dbar[j] = -dw * w[j] / ((m - 1.f) * d[j]);
      }
    }
    float pq[2 * C];
#pragma unroll
    for (int j = 0; j < C; ++j) {
      const float de = e[j] > kDFloor ? dbar[j] : 0.f;
      const float da = de * dd[j] * dd[j];
      acc[j] += -2.f * de * av[j] * dd[j];  // dJ/dc_j
      acc[C] += -da * H[j];                // dJ/dlambda
      acc[C + 1] += -da * F[j];            // dJ/dxi
      pq[j] = -a.lam * da * gi;
      pq[C + j] = -a.xi * da * iq;
    }
    gfloat* PQ = as_global(a.PQ) + i * (2 * C);
#pragma unroll
    for (int j = 0; j < 2 * C; ++j) PQ[j] = pq[j];
  }
  // Block sums (fixed order) into this block's slot.
  PairDev pr{};
  pr.partials = a.partials;
  block_tile_store<NV, kAdjThreads>(pr, blockIdx.x, acc, s_red);
}

template <int C, bool EVAL>
__global__ __launch_bounds__(kAdjThreads) void k_adj_transpose(const AdjArgs a, float* Ubar_out) {
  const size_t N = (size_t)a.nx * a.ny * a.nz;
  const size_t k = (size_t)blockIdx.x * kAdjThreads + threadIdx.x;
  if (k >= N) return;
  const Nbr nb(a.nx, a.ny, a.nz, k);
  const float xk = a.x[k];
  float u[C], out[C];
  load_row<C>(as_global(a.U) + k * C, u);
  if constexpr (EVAL) load_row<C>(as_global(a.Ubar_direct) + k * C, out);
  else {
#pragma unroll
    for (int j = 0; j < C; ++j) out[j] = 0.f;
  }
#pragma unroll
  for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        if ((dx | dy | dz) == 0 || !nb.valid(dx, dy, dz)) continue;
        const size_t i = nb.at(k, dx, dy, dz);
        const float igi = a.invg[i];
        const float xci = igi < 0.f ? a.x[i] - 1.f : a.x[i];
        const float g = fabsf(xci - xk);  // g_ik as voxel i uses it
        const float q = qweight((dx != 0) + (dy != 0) + (dz != 0), a.q2_sqdist);
        const gfloat* PQ = as_global(a.PQ) + i * (2 * C);
#pragma unroll
        for (int j = 0; j < C; ++j) out[j] = fmaf(PQ[j], g, fmaf(2.f * u[j] * PQ[C + j], q, out[j]));
      }
  store_row<C>(as_global(Ubar_out) + k * C, out);
}

// Fixed-order fp64 sum of the adjoint block slots: out[0..C) = dJ/dc (this
// step), acc2[0..1] += dJ/dlambda, dJ/dxi.
template <int C>
__global__ __launch_bounds__(256) void k_adj_finalize(const float* parts, int nslots, double* out,
                                                      double* acc2) {
  constexpr int NV = C + 2;
  __shared__ double s_red[4 * NV];
  double d[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) d[k] = 0.0;
  for (int s = threadIdx.x; s < nslots; s += 256) {
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
      const double t = ((s_red[k] + s_red[NV + k]) + s_red[2 * NV + k]) + s_red[3 * NV + k];
      if (k < C) out[k] = t;
      else acc2[k - C] += t;
    }
  }
}

template <int C>
static hipError_t launch_adj_c(const AdjArgs& a, bool m2, bool eval, float* Ubar_out,
                               double* cbar_out, double* acc2, hipStream_t s) {
  const size_t N = (size_t)a.nx * a.ny * a.nz;
  const int grid = (int)((N + kAdjThreads - 1) / kAdjThreads);
  if (eval) {
    if (m2) hipLaunchKernelGGL((k_adj_point<C, true, true>), dim3(grid), dim3(kAdjThreads), 0, s, a);
    else hipLaunchKernelGGL((k_adj_point<C, false, true>), dim3(grid), dim3(kAdjThreads), 0, s, a);
  } else {
    if (m2) hipLaunchKernelGGL((k_adj_point<C, true, false>), dim3(grid), dim3(kAdjThreads), 0, s, a);
    else hipLaunchKernelGGL((k_adj_point<C, false, false>), dim3(grid), dim3(kAdjThreads), 0, s, a);
  }
  hipLaunchKernelGGL((k_adj_finalize<C>), dim3(1), dim3(256), 0, s, a.partials, grid, cbar_out, acc2);
  if (Ubar_out) {
    if (eval) hipLaunchKernelGGL((k_adj_transpose<C, true>), dim3(grid), dim3(kAdjThreads), 0, s, a, Ubar_out);
    else hipLaunchKernelGGL((k_adj_transpose<C, false>), dim3(grid), dim3(kAdjThreads), 0, s, a, Ubar_out);
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

size_t adjoint_slots(size_t N) { return (N + kAdjThreads - 1) / kAdjThreads; }

}  // namespace pifcm
