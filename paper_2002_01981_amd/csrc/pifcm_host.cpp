// pifcm_host.cpp -- host runtime of libpifcm: context, argument checks,
// workspace, the IFCM solve loop, the swarm evaluation (batched launches
// captured in a HIP graph, or one launch per particle), the tuner, and the
// C ABI of include/pifcm.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "pifcm.h"
#include "pifcm_device.h"
#include "pifcm_kernels.h"

using namespace pifcm;

namespace {

struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
};

struct GraphCache {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<char> key;
};

struct TileShape {
  int nw = 4;   // wavefronts per work group of the fused step
  int zc = 0;   // planes per tile (0: the volume's default, default_zc)
  int pt = 1;   // particles per work item of the batched fused step (C = 4: 1 or 2)
};

constexpr int kChunk = 8;            // iterations between stop-flag reads
// Host staging of one solve: its state, pair and volume records.
constexpr size_t kStageBytes = (sizeof(SolveState) + sizeof(PairDev) + sizeof(VolDev) + 64 + 255) / 256 * 256;
constexpr float kMaxWeight = 1000.f; // |lambda|, |xi| accepted
constexpr int kMaxPairs = 65536;

}  // namespace

struct pifcm_ctx {
  int device = 0;
  hipStream_t user = nullptr;
  hipStream_t s = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  std::string err;
  int num_cu = 256;
  DevBuf invg, rinv, ubuf, partials, states, jhist, tvol, tpair, flags;
  DevBuf adj_ck, adj_seg, adj_bar, adj_pq, adj_misc, adj_rs;  // ifcm_backward workspace
  DevBuf tune_u0, tune_state, tune_ref;                // pifcm_tune workspace
  DevBuf ring_tab;                                     // general-neighbourhood offsets
  DevBuf conf;                                         // pifcm_confusion counts
  DevBuf pso_state;                                    // pifcm_pso_interleaved states
  DevBuf work;                                         // fused step's item counters (16 ints)
  int ring_n = 0;                                      // offsets in ring_tab
  int ring_gen = 0;                                    // rebuilds of ring_tab
  int ring_key[3] = {0, -1, 0};                        // (V, flags, bits of h) of ring_tab
  float ring_W[kMaxRings + 1] = {};                    // eq (10) weights by ring
  void* pinned = nullptr;
  size_t pinned_cap = 0;
  GraphCache graph;
  bool timing = false;
  hipEvent_t tm0 = nullptr, tm1 = nullptr;
  double step_ms = 0.0;
  int64_t step_launches = 0;
  std::map<std::tuple<int, int, int, int, int>, TileShape> tuned;  // (C, m2, nx, ny, nz)
  int occ_gather[kMaxC + 1][2] = {};  // resident work groups per CU of the fused step (4 waves)
  char arch[64] = "unknown";  // device architecture (tuning cache key)
};

namespace {

pifcm_status fail(pifcm_ctx* ctx, pifcm_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (ctx) ctx->err = buf;
  return st;
}

#define HIPCHK(call)                                                                         \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess) return fail(ctx, PIFCM_E_HIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
  } while (0)

pifcm_status ensure(pifcm_ctx* ctx, DevBuf& b, size_t bytes, const char* what) {
  if (bytes == 0) bytes = 256;
  if (b.cap >= bytes) return PIFCM_OK;
  if (b.p) {
    HIPCHK(hipStreamSynchronize(ctx->s));
    HIPCHK(hipFree(b.p));
    b.p = nullptr;
    b.cap = 0;
  }
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, PIFCM_E_OOM, "cannot allocate %zu bytes of workspace for %s", bytes, what);
  }
  b.p = p;
  b.cap = bytes;
  return PIFCM_OK;
}

pifcm_status ensure_pinned(pifcm_ctx* ctx, size_t bytes) {
  if (ctx->pinned_cap >= bytes) return PIFCM_OK;
  if (ctx->pinned) {
    HIPCHK(hipStreamSynchronize(ctx->s));
    HIPCHK(hipHostFree(ctx->pinned));
    ctx->pinned = nullptr;
    ctx->pinned_cap = 0;
  }
  if (hipHostMalloc(&ctx->pinned, bytes, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    ctx->pinned = nullptr;
    return fail(ctx, PIFCM_E_OOM, "cannot allocate %zu bytes of pinned host memory", bytes);
  }
  ctx->pinned_cap = bytes;
  return PIFCM_OK;
}

#define TRY(expr)                       \
  do {                                  \
    pifcm_status s_ = (expr);           \
    if (s_ != PIFCM_OK) return s_;      \
  } while (0)

pifcm_status begin(pifcm_ctx* ctx) {
  HIPCHK(hipSetDevice(ctx->device));
  HIPCHK(hipEventRecord(ctx->ev_in, ctx->user));
  HIPCHK(hipStreamWaitEvent(ctx->s, ctx->ev_in, 0));
  // The fused step's item counters start every call at zero (each launch
  // also leaves them at zero).
  HIPCHK(hipMemsetAsync(ctx->work.p, 0, 16 * sizeof(int32_t), ctx->s));
  return PIFCM_OK;
}

pifcm_status finish(pifcm_ctx* ctx) {
  HIPCHK(hipEventRecord(ctx->ev_out, ctx->s));
  HIPCHK(hipStreamWaitEvent(ctx->user, ctx->ev_out, 0));
  return PIFCM_OK;
}

pifcm_status timing_begin(pifcm_ctx* ctx) {
  if (ctx->timing) HIPCHK(hipEventRecord(ctx->tm0, ctx->s));
  return PIFCM_OK;
}

pifcm_status timing_end(pifcm_ctx* ctx) {
  if (ctx->timing) HIPCHK(hipEventRecord(ctx->tm1, ctx->s));
  return PIFCM_OK;
}

// After the stream has been synchronised: add the bracketed time.
pifcm_status timing_collect(pifcm_ctx* ctx, int64_t launches) {
  if (!ctx->timing || launches <= 0) return PIFCM_OK;
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, ctx->tm0, ctx->tm1));
  ctx->step_ms += ms;
  ctx->step_launches += launches;
  return PIFCM_OK;
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

pifcm_status check_params(pifcm_ctx* ctx, const pifcm_params* p) {
  if (!p) return fail(ctx, PIFCM_E_INVALID, "params is NULL");
  if (p->C < 2 || p->C > kMaxC) return fail(ctx, PIFCM_E_INVALID, "C = %d outside [2, %d]", p->C, kMaxC);
  if (!std::isfinite(p->m) || !(p->m > 1.f)) return fail(ctx, PIFCM_E_INVALID, "m = %g must be finite and > 1", p->m);
  if (p->V < 1) return fail(ctx, PIFCM_E_INVALID, "V = %d must be >= 1", p->V);
  if (!std::isfinite(p->h) || !(p->h > 0.f)) return fail(ctx, PIFCM_E_INVALID, "h = %g must be finite and > 0", p->h);
  if (!std::isfinite(p->eps) || p->eps < 0.f) return fail(ctx, PIFCM_E_INVALID, "eps = %g must be finite and >= 0", p->eps);
  if (p->max_iter < 0 || p->max_iter > 1000000) return fail(ctx, PIFCM_E_INVALID, "max_iter = %d outside [0, 1e6]", p->max_iter);
  if (p->flags & ~(PIFCM_Q2_SQDIST | PIFCM_SHELL_SQDIST))
    return fail(ctx, PIFCM_E_INVALID, "unknown flags 0x%x", p->flags);
  if ((p->flags & PIFCM_SHELL_SQDIST) && p->V > kMaxRings)
    return fail(ctx, PIFCM_E_UNSUPPORTED, "V = %d: squared-distance rings are built up to V = %d", p->V,
                kMaxRings);
  if (!(p->flags & PIFCM_SHELL_SQDIST) && p->V > kMaxReach)
    return fail(ctx, PIFCM_E_UNSUPPORTED, "V = %d: Chebyshev rings are built up to V = %d", p->V, kMaxReach);
  return PIFCM_OK;
}

// (C: the cluster count of the call, from validated params.)
pifcm_status check_volume(pifcm_ctx* ctx, const pifcm_volume* v, int C) {
  if (!v) return fail(ctx, PIFCM_E_INVALID, "volume is NULL");
  if (!v->x) return fail(ctx, PIFCM_E_INVALID, "volume intensities are NULL");
  if (v->nx < 1 || v->ny < 1 || v->nz < 1)
    return fail(ctx, PIFCM_E_INVALID, "volume dims %d x %d x %d must be >= 1", v->nx, v->ny, v->nz);
  const double n = (double)v->nx * v->ny * v->nz;
  if (n > 4.0e9) return fail(ctx, PIFCM_E_INVALID, "volume of %.0f voxels is too large", n);
  // The kernels address the planes of a tile with 32-bit byte offsets: three
  // planes of memberships must stay below 2^31 bytes.
  if (3.0 * v->nx * v->ny * C * 4.0 >= 2147483648.0)
    return fail(ctx, PIFCM_E_INVALID, "planes of %d x %d voxels are too large for C = %d", v->nx, v->ny, C);
  return PIFCM_OK;
}

size_t nvox(const pifcm_volume& v) { return (size_t)v.nx * v.ny * v.nz; }

// Largest plane count per tile such that the 32-bit in-tile offsets of the
// fused step stay below 2^31 bytes: (zc + 2) * nx * ny * C * 4 < 2^31.
int max_zc(const pifcm_volume& v, int C) {
  const double per_plane = (double)v.nx * v.ny * C * 4.0;
  const double z = std::floor((2147483647.0 / per_plane)) - 2.0;
  return (int)std::max(0.0, std::min(z, (double)v.nz));
}

// Planes per tile when no shape was chosen for the volume.  A solve of one
// pair runs ceil(tiles / R) rounds of tiles on the R waves the fused step
// keeps resident (4 waves per work group), and a tile costs about zc + 4
// plane passes (its two halo planes and the start of its walk): among the
// depths ceil(nz / k) and 32 that are at least min(nz, 32) deep, take the
// one with the fewest rounds * (zc + 4), the deeper one on a tie.  Batched
// swarm launches hold many pairs and want deep tiles (fewer tile starts and
// halo planes), hence the floor; the depth does not depend on the launch, so
// every launch mode gives the same bits.  On the 181-plane brain volume this
// is 46 planes (four tiles per column, one round) rather than 32 (six per
// column, 1.3 rounds).
int default_zc(pifcm_ctx* ctx, int C, bool m2, const pifcm_volume& v) {
  int& occ = ctx->occ_gather[std::max(0, std::min(C, kMaxC))][m2 ? 1 : 0];
  if (occ == 0) occ = std::max(1, gather_occupancy(C, 4, 1, m2, true));
  const long R = (long)occ * ctx->num_cu * 4;
  const long txy = (long)((v.nx + kWaveTileX - 1) / kWaveTileX) * ((v.ny + kWaveTileY - 1) / kWaveTileY);
  const int floor_zc = std::min(v.nz, 32);
  int best = v.nz;
  long best_cost = -1;
  auto consider = [&](int zc) {
    const long tiles = txy * ((v.nz + zc - 1) / zc);
    const long cost = (tiles + R - 1) / R * (zc + 4);
    if (best_cost < 0 || cost < best_cost || (cost == best_cost && zc > best)) {
      best_cost = cost;
      best = zc;
    }
  };
  for (int k = 1; k <= v.nz; ++k) {
    const int zc = (v.nz + k - 1) / k;
    if (zc < floor_zc) break;
    consider(zc);
  }
  consider(floor_zc);
  return best;
}

TileShape shape_for(pifcm_ctx* ctx, int C, bool m2, const pifcm_volume& v) {
  TileShape t;
  auto it = ctx->tuned.find(std::make_tuple(C, (int)m2, v.nx, v.ny, v.nz));
  if (it != ctx->tuned.end()) t = it->second;
  if (t.zc <= 0) t.zc = default_zc(ctx, C, m2, v);
  t.zc = std::max(1, std::min(t.zc, max_zc(v, C)));
  return t;
}

// Launch descriptor of a volume whose planes [zbeg, zend) are iterated
// (zend < 0: all planes).
VolDev make_vol(const pifcm_volume& v, const float* invg, TileShape ts, int zbeg = 0, int zend = -1,
                const float* rinv = nullptr) {
  if (zend < 0) zend = v.nz;
  VolDev d{};
  d.x = v.x;
  d.invg = invg;
  d.rinv = rinv;
  d.nx = v.nx;
  d.ny = v.ny;
  d.nz = v.nz;
  d.zbeg = zbeg;
  d.zend = zend;
  const int nact = zend - zbeg;
  d.zc = std::max(1, std::min(ts.zc, nact));
  d.ntx = (v.nx + kWaveTileX - 1) / kWaveTileX;
  d.nty = (v.ny + kWaveTileY - 1) / kWaveTileY;
  d.ntz = (nact + d.zc - 1) / d.zc;
  d.tiles = d.ntx * d.nty * d.ntz;
  const size_t per = (size_t)256 * kFcmVoxPerThread;
  d.tiles1d = (int)(((size_t)v.nx * v.ny * nact + per - 1) / per);
  return d;
}

// Work groups for `nitems` work items, `per_group` items in flight per work
// group (waves of the fused step, 1 for the pointwise kernels): one item per
// slot when they all fit in 8 waves of resident groups, else a persistent
// grid of the resident groups.  Always a multiple of 8 (one share per XCD).
int grid_for(pifcm_ctx* ctx, int nitems, int occupancy, int per_group = 1) {
  const long resident = (long)occupancy * ctx->num_cu;
  const long groups = ((long)nitems + per_group - 1) / per_group;
  long g;
  if (groups <= 8 * resident) g = (groups + 7) / 8 * 8;
  else g = resident / 8 * 8;
  return (int)std::max<long>(8, g);
}

// g_inv of `nv` volumes into invg (volume b at invg + invg_off[b]), the
// intensity check, and the row check of caller U0 pointers (optional), with
// flags (device, 2 ints) and stage (host, 2 ints) as workspace.
pifcm_status run_invariants(pifcm_ctx* ctx, const pifcm_volume* vols, int nv, int C,
                            const float* const* U0s, float* invg, const size_t* invg_off, int* flags,
                            int* stage) {
  HIPCHK(hipMemsetAsync(flags, 0, 2 * sizeof(int), ctx->s));
  for (int b = 0; b < nv; ++b) {
    HIPCHK(launch_invariants(vols[b].x, invg + invg_off[b], vols[b].nx, vols[b].ny, vols[b].nz,
                             flags, ctx->s));
    if (U0s && U0s[b]) HIPCHK(launch_check_rows(U0s[b], nvox(vols[b]), C, flags + 1, ctx->s));
  }
  HIPCHK(hipMemcpyAsync(stage, flags, 2 * sizeof(int), hipMemcpyDeviceToHost, ctx->s));
  HIPCHK(hipStreamSynchronize(ctx->s));
  if (stage[0]) return fail(ctx, PIFCM_E_NONFINITE, "a volume holds a NaN or Inf intensity");
  if (stage[1])
    return fail(ctx, PIFCM_E_INVALID,
                "initial memberships must be finite, in [0, 1] and sum to 1 (+-1e-4) per voxel");
  return PIFCM_OK;
}

// Set up invariants of `nv` volumes into ctx->invg (concatenated) and check
// intensities; optionally check rows of caller U0 pointers.
pifcm_status prepare_volumes(pifcm_ctx* ctx, const pifcm_volume* vols, int nv, int C,
                             const float* const* U0s, std::vector<size_t>& invg_off,
                             const pifcm_params* ring2 = nullptr) {
  size_t total = 0;
  invg_off.resize(nv);
  for (int b = 0; b < nv; ++b) {
    invg_off[b] = total;
    total += (nvox(vols[b]) + 63) / 64 * 64;
  }
  TRY(ensure(ctx, ctx->invg, total * sizeof(float), "iteration invariants"));
  if (ring2) {
    // Per-ring invariants of the fused two-ring kernel (4 floats per voxel,
    // at 4 x the offsets of g_inv).
    TRY(ensure(ctx, ctx->rinv, total * 4 * sizeof(float), "ring invariants"));
    for (int b = 0; b < nv; ++b)
      HIPCHK(launch_ring2_invariants(vols[b].x, (float*)ctx->rinv.p + 4 * invg_off[b], vols[b].nx,
                                     vols[b].ny, vols[b].nz, (ring2->flags & PIFCM_Q2_SQDIST) ? 1 : 0,
                                     ctx->s));
  }
  TRY(ensure(ctx, ctx->flags, 64, "flags"));
  TRY(ensure_pinned(ctx, 4096));
  return run_invariants(ctx, vols, nv, C, U0s, (float*)ctx->invg.p, invg_off.data(), (int*)ctx->flags.p,
                        (int*)ctx->pinned);
}

SolveState init_state(const float* c0, int C, float lam, float xi, const pifcm_params* p,
                      double* jhist) {
  SolveState s;
  std::memset(&s, 0, sizeof s);
  for (int j = 0; j < C; ++j) s.c[0][j] = s.c[1][j] = c0[j];
  s.lam = lam;
  s.xi = xi;
  s.eps = p->eps;
  s.max_iter = p->max_iter;
  s.iter = 0;
  s.stop = p->max_iter == 0 ? 1 : 0;
  s.counter = 0;
  s.J_hist = jhist;
  return s;
}

// Which step kernel a launch uses.
enum Kind { kGather = 0, kFcm = 1, kRing = 2, kRing2 = 3 };

bool ring_params(const pifcm_params* p) { return p->V > 1 || (p->flags & PIFCM_SHELL_SQDIST); }
// The two Chebyshev rings of the 5x5x5 cube with C <= 4 run the fused
// two-ring kernel; other general neighbourhoods walk the offset table.
bool ring2_params(const pifcm_params* p) {
  return p->V == 2 && !(p->flags & PIFCM_SHELL_SQDIST) && p->C <= 4;
}
bool is_ring(int kind) { return kind == kRing || kind == kRing2; }

// lambda = xi = 0 makes the attraction factor of eq (4) exactly 1 for every
// neighbourhood: plain FCM.
int kind_of(const pifcm_params* p, bool zero_weights) {
  if (zero_weights) return kFcm;
  return ring_params(p) ? (ring2_params(p) ? kRing2 : kRing) : kGather;
}

int occupancy_of(int kind, int C, int nw, bool m2, bool step, int pt = 1) {
  if (kind == kFcm) return fcm_occupancy(C, m2, step);
  if (kind == kRing) return ring_occupancy(C, m2, step);
  if (kind == kRing2) return ring2_occupancy(C, m2, step);
  return gather_occupancy(C, nw, pt, m2, step);
}

// Particles per work item a launch of `kind` over P particles uses: the
// shape's pt for the fused step of a swarm at C = 4, else 1.
int pt_for(int kind, int C, int P, const TileShape& ts) {
  return (kind == kGather && C == 4 && P >= 2) ? std::max(1, std::min(ts.pt, 2)) : 1;
}

// Work items in flight per work group.
// Work items a work group takes at a time: one per wave for the tiled
// kernels, one for the pointwise kernels.
int items_per_group(int kind, int nw) {
  return kind == kGather ? nw : kind == kRing ? kRingWaves : kind == kRing2 ? kRing2Waves : 1;
}

// Offsets of the general neighbourhood (eq (9) up to the reach of V), sorted
// by ring (Chebyshev shell, or squared distance with PIFCM_SHELL_SQDIST) with
// their eq (7) weights, and the ring weights of eq (10), uploaded once per
// (V, flags, h).
pifcm_status prepare_ring(pifcm_ctx* ctx, const pifcm_params* p) {
  const int fl = p->flags & (PIFCM_SHELL_SQDIST | PIFCM_Q2_SQDIST);
  int hb;
  std::memcpy(&hb, &p->h, sizeof hb);
  if (ctx->ring_tab.p && ctx->ring_key[0] == p->V && ctx->ring_key[1] == fl && ctx->ring_key[2] == hb)
    return PIFCM_OK;
  const bool sq = fl & PIFCM_SHELL_SQDIST;
  int reach = p->V;
  if (sq) {
    reach = 0;
    while ((reach + 1) * (reach + 1) <= p->V) ++reach;
  }
  std::vector<RingOff> offs;
  for (int r = 1; r <= p->V; ++r)
    for (int dz = -reach; dz <= reach; ++dz)
      for (int dy = -reach; dy <= reach; ++dy)
        for (int dx = -reach; dx <= reach; ++dx) {
          const int s2 = dx * dx + dy * dy + dz * dz;
          if (s2 == 0) continue;
          const int ring = sq ? s2 : std::max(std::abs(dx), std::max(std::abs(dy), std::abs(dz)));
          if (ring != r) continue;
          RingOff o{};
          o.dx = (int16_t)dx;
          o.dy = (int16_t)dy;
          o.dz = (int16_t)dz;
          o.ring = (int16_t)r;
          o.q2 = (fl & PIFCM_Q2_SQDIST) ? (float)s2 : (float)(s2 * s2);
          offs.push_back(o);
        }
  double total = 0.0;
  for (int r = 1; r <= p->V; ++r) total += std::exp(-(double)(r - 1) / (double)p->h);
  for (int r = 0; r <= kMaxRings; ++r)
    ctx->ring_W[r] = (r >= 1 && r <= p->V) ? (float)(std::exp(-(double)(r - 1) / (double)p->h) / total) : 0.f;
  TRY(ensure(ctx, ctx->ring_tab, offs.size() * sizeof(RingOff), "neighbourhood table"));
  HIPCHK(hipMemcpyAsync(ctx->ring_tab.p, offs.data(), offs.size() * sizeof(RingOff), hipMemcpyHostToDevice,
                        ctx->s));
  HIPCHK(hipStreamSynchronize(ctx->s));
  ctx->ring_n = (int)offs.size();
  ctx->ring_key[0] = p->V;
  ctx->ring_key[1] = fl;
  ctx->ring_key[2] = hb;
  ++ctx->ring_gen;
  return PIFCM_OK;
}

// One iteration (step) or the objective-only pass: the tile kernel, then the
// per-pair finalise that adds the tile sums and advances the state.
// A grid with a wave slot for every item of an even split by count (each XCD
// runs its range in one pass) keeps that split: ranges balanced by work
// would hand some XCD more items than it has waves.  A persistent grid,
// whose waves walk several items each, takes the balanced ranges.
hipError_t launch_step(int C, const LaunchArgs& a, int grid, int nw, bool m2, int kind, bool step,
                       hipStream_t s) {
  LaunchArgs b = a;
  const long per = ((long)a.nitems + 7) / 8;
  if ((long)(grid / 8) * items_per_group(kind, nw) >= per)
    for (int k = 0; k <= 8; ++k) b.xcd_begin[k] = (int32_t)std::min<long>(a.nitems, per * k);
  hipError_t e = kind == kFcm     ? launch_fcm(C, b, grid, m2, step, s)
                 : kind == kRing  ? launch_ring(C, b, grid, m2, step, s)
                 : kind == kRing2 ? launch_ring2(C, b, grid, m2, step, s)
                                  : launch_gather(C, b, grid, nw, m2, step, s);
  if (e != hipSuccess) return e;
  return launch_finalize(C, b, b.nvol * b.P, step, s);
}

// The 8 XCD ranges of a launch's items (LaunchArgs::xcd_begin): contiguous,
// cut where the running work reaches k / 8 of the total.  A tile item's work
// is the planes its tile walks plus 3 (the two halo planes and the start of
// the walk); a pointwise item counts 1.  Items run volume by volume, particle
// group by group, and within a group tile rows of equal depth follow each
// other (tiles are numbered x, then y, then z), so the cuts are found per
// volume and per tile row without visiting every item.  With volumes of
// different depths in one launch an even split by count leaves some XCDs
// with up to 15 % more work than the mean.
void split_items(LaunchArgs& a, const VolDev* vh, int nvol) {
  const int groups = (a.P + a.pt - 1) / a.pt;
  auto depth = [&](const VolDev& v, int tz) { return std::min(v.zc, v.zend - v.zbeg - tz * v.zc); };
  double total = 0.0;
  for (int b = 0; b < nvol; ++b) {
    const VolDev& v = vh[b];
    double per_group = 0.0;
    if (a.use_1d) per_group = v.tiles1d;
    else
      for (int tz = 0; tz < v.ntz; ++tz) per_group += (double)v.ntx * v.nty * (depth(v, tz) + 3);
    total += per_group * groups;
  }
  a.xcd_begin[0] = 0;
  int k = 1;
  double cum = 0.0;
  for (int b = 0; b < nvol && k < 8; ++b) {
    const VolDev& v = vh[b];
    const long txy = (long)v.ntx * v.nty;
    const int nrow = a.use_1d ? 1 : v.ntz;  // runs of equal-cost items in a group
    auto row_items = [&](int r) -> long { return a.use_1d ? (long)v.tiles1d : txy; };
    auto row_cost = [&](int r) -> double { return a.use_1d ? 1.0 : (double)(depth(v, r) + 3); };
    double per_group = 0.0;
    for (int r = 0; r < nrow; ++r) per_group += row_items(r) * row_cost(r);
    const double vol_end = cum + per_group * groups;
    while (k < 8 && total * k / 8.0 < vol_end) {
      const double target = total * k / 8.0;
      const long g = std::min<long>(groups - 1, (long)((target - cum) / per_group));
      double c = cum + per_group * g;
      long item = a.item_begin[b] + g * (a.use_1d ? (long)v.tiles1d : (long)v.tiles);
      for (int r = 0; r < nrow; ++r) {
        const double rc = row_items(r) * row_cost(r);
        if (c + rc >= target) {
          item += std::min<long>(row_items(r), (long)std::ceil((target - c) / row_cost(r)));
          break;
        }
        c += rc;
        item += row_items(r);
      }
      a.xcd_begin[k++] = (int32_t)std::min<long>(item, a.nitems);
    }
    cum = vol_end;
  }
  while (k <= 8) a.xcd_begin[k++] = a.nitems;
  for (int i = 1; i <= 8; ++i) a.xcd_begin[i] = std::max(a.xcd_begin[i], a.xcd_begin[i - 1]);
}

LaunchArgs make_args(const pifcm_ctx* ctx, const VolDev* vols_dev, const PairDev* pairs_dev,
                     const VolDev* vh, int nvol, int P, int kind, const pifcm_params* p,
                     int pt = 1) {
  LaunchArgs a;
  std::memset(&a, 0, sizeof a);
  a.vols = vols_dev;
  a.pairs = pairs_dev;
  a.nvol = nvol;
  a.P = P;
  a.q2_sqdist = (p->flags & PIFCM_Q2_SQDIST) ? 1 : 0;
  a.m = p->m;
  a.use_1d = kind == kFcm ? 1 : 0;  // the pointwise kernel's 1D tiles
  a.work = (int32_t*)ctx->work.p;
  // Items are handed out by counter only when every pair runs every
  // iteration: under a stop rule the items of stopped pairs cost nothing,
  // and waves running through them would queue on the counter.
  a.handout = p->eps == 0.f ? 1 : 0;
  if (is_ring(kind)) {
    a.ring = (const RingOff*)ctx->ring_tab.p;
    a.nring = ctx->ring_n;
    a.pad1 = ctx->ring_gen;  // part of the graph cache key
    for (int r = 0; r <= kMaxRings; ++r) a.W[r] = ctx->ring_W[r];
  }
  // Fused-step items are (volume, group of pt particles, tile).
  a.pt = kind == kGather ? std::max(1, pt) : 1;
  const int groups = (P + a.pt - 1) / a.pt;
  int acc = 0;
  for (int b = 0; b < nvol; ++b) {
    a.item_begin[b] = acc;
    acc += groups * (a.use_1d ? vh[b].tiles1d : vh[b].tiles);
  }
  a.item_begin[nvol] = acc;
  a.nitems = acc;
  split_items(a, vh, nvol);
  return a;
}

LaunchArgs make_args(const pifcm_ctx* ctx, const VolDev* vols_dev, const PairDev* pairs_dev,
                     const std::vector<VolDev>& vh, int nvol, int P, int kind,
                     const pifcm_params* p, int pt = 1) {
  return make_args(ctx, vols_dev, pairs_dev, vh.data(), nvol, P, kind, p, pt);
}

bool ranges_overlap(const void* a, size_t na, const void* b, size_t nb) {
  const char* pa = (const char*)a;
  const char* pb = (const char*)b;
  return pa < pb + nb && pb < pa + na;
}

// ------------------------------------------------------------ tuning cache
// The tuner's choices are kept, if PIFCM_TUNE_CACHE names a file, as a JSON
// object with one entry per line:
//   "gfx950|C4|m2|V1|B6|P64|N2^25|Z2^7": {"nw": 4, "zc": 128, "pt": 2, "step_ms": 14.5},
// keyed by device architecture, C, m == 2, V, the batch size, the particle
// count and the total voxel count and largest plane count rounded up to
// powers of two.
int ceil_log2(double v) {
  int k = 0;
  while (std::ldexp(1.0, k) < v) ++k;
  return k;
}

std::string tune_key(const pifcm_ctx* ctx, const pifcm_volume* vols, int B, const pifcm_params* p, int P) {
  double n = 0.0;
  int z = 1;
  for (int b = 0; b < B; ++b) {
    n += (double)nvox(vols[b]);
    z = std::max(z, vols[b].nz);
  }
  char k[160];
  snprintf(k, sizeof k, "%s|C%d|m%s|V%d|B%d|P%d|N2^%d|Z2^%d", ctx->arch, p->C, p->m == 2.0f ? "2" : "x", p->V, B,
           P, ceil_log2(n), ceil_log2((double)z));
  return k;
}

// Entries of the cache file as (key, rest of the line).
std::vector<std::pair<std::string, std::string>> tune_cache_read(const char* path) {
  std::vector<std::pair<std::string, std::string>> out;
  FILE* f = std::fopen(path, "r");
  if (!f) return out;
  char line[512];
  while (std::fgets(line, sizeof line, f)) {
    const char* a = std::strchr(line, '"');
    if (!a) continue;
    const char* b = std::strchr(a + 1, '"');
    const char* c = b ? std::strchr(b, '{') : nullptr;
    const char* d = c ? std::strchr(c, '}') : nullptr;
    if (!d) continue;
    out.emplace_back(std::string(a + 1, b), std::string(c, d + 1));
  }
  std::fclose(f);
  return out;
}

bool tune_cache_get(const char* path, const std::string& key, TileShape& t, double& ms) {
  for (const auto& e : tune_cache_read(path)) {
    if (e.first != key) continue;
    int nw = 0, zc = 0, pt = 0;
    double m = 0.0;
    if (std::sscanf(e.second.c_str(), "{\"nw\": %d, \"zc\": %d, \"pt\": %d, \"step_ms\": %lf}", &nw, &zc, &pt,
                    &m) != 4)
      return false;
    if ((nw != 1 && nw != 2 && nw != 4) || zc < 0 || (pt != 1 && pt != 2)) return false;
    t.nw = nw;
    t.zc = zc;
    t.pt = pt;
    ms = m;
    return true;
  }
  return false;
}

// Add or replace `key` (written to a temporary file, then renamed).
void tune_cache_put(const char* path, const std::string& key, const TileShape& t, double ms) {
  auto entries = tune_cache_read(path);
  char val[160];
  snprintf(val, sizeof val, "{\"nw\": %d, \"zc\": %d, \"pt\": %d, \"step_ms\": %.4f}", t.nw, t.zc, t.pt, ms);
  bool found = false;
  for (auto& e : entries)
    if (e.first == key) {
      e.second = val;
      found = true;
    }
  if (!found) entries.emplace_back(key, val);
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return;
  std::fprintf(f, "{\n");
  for (size_t i = 0; i < entries.size(); ++i)
    std::fprintf(f, "\"%s\": %s%s\n", entries[i].first.c_str(), entries[i].second.c_str(),
                 i + 1 < entries.size() ? "," : "");
  std::fprintf(f, "}\n");
  if (std::fclose(f) == 0) std::rename(tmp.c_str(), path);
}

}  // namespace

// ===================================================================== ABI
extern "C" {

pifcm_status pifcm_create(int device, void* hip_stream, pifcm_ctx** out) {
  if (!out) return PIFCM_E_INVALID;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
    (void)hipGetLastError();
    return PIFCM_E_INVALID;
  }
  pifcm_ctx* ctx = new pifcm_ctx();
  ctx->device = device;
  ctx->user = (hipStream_t)hip_stream;
  if (hipSetDevice(device) != hipSuccess ||
      hipStreamCreateWithFlags(&ctx->s, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->ev_in, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->ev_out, hipEventDisableTiming) != hipSuccess ||
      hipEventCreate(&ctx->tm0) != hipSuccess || hipEventCreate(&ctx->tm1) != hipSuccess) {
    (void)hipGetLastError();
    pifcm_destroy(ctx);
    return PIFCM_E_HIP;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
    ctx->num_cu = prop.multiProcessorCount;
    // "gfx950:sramecc+:xnack-" -> "gfx950"
    size_t n = 0;
    while (n + 1 < sizeof ctx->arch && prop.gcnArchName[n] && prop.gcnArchName[n] != ':') {
      ctx->arch[n] = prop.gcnArchName[n];
      ++n;
    }
    ctx->arch[n] = 0;
  }
  ensure(ctx, ctx->tvol, sizeof(VolDev) * kMaxBatchVols, "volume table");
  ensure(ctx, ctx->tpair, sizeof(PairDev) * kMaxPairs, "pair table");
  if (ensure(ctx, ctx->work, 16 * sizeof(int32_t), "item counters") != PIFCM_OK ||
      hipMemset(ctx->work.p, 0, 16 * sizeof(int32_t)) != hipSuccess) {
    (void)hipGetLastError();
    pifcm_destroy(ctx);
    return PIFCM_E_OOM;
  }
  // The device address of the no-allocation scratch, once per device (a
  // failure here is reported by ifcm_solve_noalloc, which asks again), and
  // the pinned host staging that solve uses (it only ever grows).
  void* sp = nullptr;
  if (scratch_region(device, &sp) != hipSuccess) (void)hipGetLastError();
  if (ensure_pinned(ctx, kStageBytes + 4096) != PIFCM_OK) {
    pifcm_destroy(ctx);
    return PIFCM_E_OOM;
  }
  *out = ctx;
  return PIFCM_OK;
}

void pifcm_destroy(pifcm_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  if (ctx->s) (void)hipStreamSynchronize(ctx->s);
  if (ctx->graph.exec) (void)hipGraphExecDestroy(ctx->graph.exec);
  if (ctx->graph.graph) (void)hipGraphDestroy(ctx->graph.graph);
  for (DevBuf* b : {&ctx->invg, &ctx->rinv, &ctx->ubuf, &ctx->partials, &ctx->states, &ctx->jhist, &ctx->tvol,
                    &ctx->tpair, &ctx->flags, &ctx->adj_ck, &ctx->adj_seg, &ctx->adj_bar,
                    &ctx->adj_pq, &ctx->adj_misc, &ctx->adj_rs, &ctx->tune_u0, &ctx->tune_state, &ctx->tune_ref, &ctx->ring_tab,
                    &ctx->conf, &ctx->pso_state, &ctx->work})
    if (b->p) (void)hipFree(b->p);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  if (ctx->ev_in) (void)hipEventDestroy(ctx->ev_in);
  if (ctx->ev_out) (void)hipEventDestroy(ctx->ev_out);
  if (ctx->tm0) (void)hipEventDestroy(ctx->tm0);
  if (ctx->tm1) (void)hipEventDestroy(ctx->tm1);
  if (ctx->s) (void)hipStreamDestroy(ctx->s);
  delete ctx;
}

pifcm_status pifcm_set_stream(pifcm_ctx* ctx, void* hip_stream) {
  if (!ctx) return PIFCM_E_INVALID;
  ctx->user = (hipStream_t)hip_stream;
  ctx->err.clear();
  return PIFCM_OK;
}

const char* pifcm_last_error(const pifcm_ctx* ctx) { return ctx ? ctx->err.c_str() : ""; }

pifcm_status pifcm_set_timing(pifcm_ctx* ctx, int32_t enable) {
  if (!ctx) return PIFCM_E_INVALID;
  ctx->err.clear();
  ctx->timing = enable != 0;
  return PIFCM_OK;
}

pifcm_status pifcm_get_timing(pifcm_ctx* ctx, double* step_ms, int64_t* step_launches,
                              int32_t reset) {
  if (!ctx) return PIFCM_E_INVALID;
  ctx->err.clear();
  if (step_ms) *step_ms = ctx->step_ms;
  if (step_launches) *step_launches = ctx->step_launches;
  if (reset) {
    ctx->step_ms = 0.0;
    ctx->step_launches = 0;
  }
  return PIFCM_OK;
}

pifcm_status pifcm_workspace_bytes(pifcm_ctx* ctx, int64_t* device_bytes, int64_t* pinned_bytes) {
  if (!ctx) return PIFCM_E_INVALID;
  ctx->err.clear();
  int64_t d = 0;
  for (const DevBuf* b : {&ctx->invg, &ctx->rinv, &ctx->ubuf, &ctx->partials, &ctx->states, &ctx->jhist,
                          &ctx->tvol, &ctx->tpair, &ctx->flags, &ctx->adj_ck, &ctx->adj_seg,
                          &ctx->adj_bar, &ctx->adj_pq, &ctx->adj_misc, &ctx->adj_rs, &ctx->tune_u0,
                          &ctx->tune_state, &ctx->tune_ref, &ctx->ring_tab, &ctx->conf, &ctx->pso_state,
                          &ctx->work})
    d += (int64_t)b->cap;
  if (device_bytes) *device_bytes = d;
  if (pinned_bytes) *pinned_bytes = (int64_t)ctx->pinned_cap;
  return PIFCM_OK;
}

pifcm_status pifcm_confusion(pifcm_ctx* ctx, const uint8_t* labels, const uint8_t* truth, int64_t n,
                             int32_t C, int32_t K, int64_t* counts_out) {
  if (!ctx) return PIFCM_E_INVALID;
  ctx->err.clear();
  if (!labels || !truth || !counts_out) return fail(ctx, PIFCM_E_INVALID, "labels, truth and counts_out must be non-NULL");
  if (n < 1) return fail(ctx, PIFCM_E_INVALID, "n = %lld must be >= 1", (long long)n);
  if (C < 1 || C > kMaxC || K < 1 || K > kMaxC)
    return fail(ctx, PIFCM_E_INVALID, "C = %d, K = %d outside [1, %d]", C, K, kMaxC);
  const size_t nb = (size_t)C * K + 1;
  TRY(begin(ctx));
  TRY(ensure(ctx, ctx->conf, nb * sizeof(unsigned long long), "confusion counts"));
  TRY(ensure_pinned(ctx, nb * sizeof(unsigned long long)));
  HIPCHK(hipMemsetAsync(ctx->conf.p, 0, nb * sizeof(unsigned long long), ctx->s));
  HIPCHK(launch_confusion(labels, truth, (size_t)n, C, K, (unsigned long long*)ctx->conf.p, ctx->s));
  HIPCHK(hipMemcpyAsync(ctx->pinned, ctx->conf.p, nb * sizeof(unsigned long long), hipMemcpyDeviceToHost, ctx->s));
  HIPCHK(hipStreamSynchronize(ctx->s));
  TRY(finish(ctx));
  const unsigned long long* h = (const unsigned long long*)ctx->pinned;
  if (h[nb - 1]) return fail(ctx, PIFCM_E_INVALID, "%llu labels or classes out of range", h[nb - 1]);
  for (size_t t = 0; t + 1 < nb; ++t) counts_out[t] = (int64_t)h[t];
  return PIFCM_OK;
}

pifcm_status pifcm_normalize(pifcm_ctx* ctx, const float* raw, int64_t n, float* x_out) {
  if (!ctx) return PIFCM_E_INVALID;
  ctx->err.clear();
  if (!raw || !x_out) return fail(ctx, PIFCM_E_INVALID, "raw and x_out must be non-NULL");
  if (n < 1) return fail(ctx, PIFCM_E_INVALID, "n = %lld must be >= 1", (long long)n);
  TRY(begin(ctx));
  TRY(ensure(ctx, ctx->flags, 64, "flags"));
  uint32_t* mm = (uint32_t*)ctx->flags.p + 4;
  int* flag = (int*)ctx->flags.p;
  const uint32_t init[2] = {0xffffffffu, 0u};
  TRY(ensure_pinned(ctx, 4096));
  std::memcpy(ctx->pinned, init, sizeof init);
  HIPCHK(hipMemsetAsync(flag, 0, sizeof(int), ctx->s));
  HIPCHK(hipMemcpyAsync(mm, ctx->pinned, sizeof init, hipMemcpyHostToDevice, ctx->s));
  // The flag is checked before x_out is written so an error leaves it alone.
  HIPCHK(launch_minmax(raw, (size_t)n, mm, flag, ctx->s));
  HIPCHK(hipMemcpyAsync((char*)ctx->pinned + 64, flag, sizeof(int), hipMemcpyDeviceToHost, ctx->s));
  HIPCHK(hipStreamSynchronize(ctx->s));
  if (*(int*)((char*)ctx->pinned + 64))
    return fail(ctx, PIFCM_E_NONFINITE, "the raw volume holds a NaN or Inf");
  HIPCHK(launch_scale(raw, (size_t)n, mm, x_out, ctx->s));
  TRY(finish(ctx));
  return PIFCM_OK;
}

}  // extern "C"

namespace {

// Memory one IFCM solve of a single volume works in.
struct SolveWs {
  float* invg = nullptr;       // device [N] g_inv
  float* rinv = nullptr;       // device [N][4] ring invariants (two-ring kernel only)
  float* ubuf = nullptr;       // device [N][C] second membership buffer
  float* partials = nullptr;   // device [tiles][2C + 1] tile sums
  SolveState* st = nullptr;    // device, one
  PairDev* tpair = nullptr;    // device, one
  VolDev* tvol = nullptr;      // device, one
  double* jhist = nullptr;     // device [max(1, max_iter)]
  int* flags = nullptr;        // device, 2 ints
  char* stage = nullptr;       // host, kStageBytes (pinned or pageable)
  double* jh_stage = nullptr;  // host [max_iter] staging of the J history, or NULL to copy
                               // it straight into the caller's array
};

// Tile slots of a solve over planes [zbeg, zend) (the larger of the tiled and
// pointwise decompositions).
int solve_slots(pifcm_ctx* ctx, const pifcm_volume* vol, const pifcm_params* p, int zbeg, int zend) {
  const VolDev v = make_vol(*vol, nullptr, shape_for(ctx, p->C, p->m == 2.0f, *vol), zbeg, zend);
  return std::max(v.tiles, v.tiles1d);
}

// One IFCM solve on the context's stream in the workspace ws.  U_out
// receives U^(T); host outputs optional.
pifcm_status solve_run(pifcm_ctx* ctx, const SolveWs& ws, const pifcm_volume* vol,
                       const pifcm_params* p, float lambda, float xi, const float* centres_in,
                       const float* U_in, float* U_out, float* centres_out, uint8_t* labels_out,
                       double* J_out, int32_t* iters_out, double* J_hist_out, int zbeg, int zend) {
  const bool slab = zbeg > 0 || zend < vol->nz;
  const int C = p->C;
  const bool m2 = p->m == 2.0f;
  const int kind = kind_of(p, lambda == 0.0f && xi == 0.0f);
  const size_t N = nvox(*vol);
  if (kind == kRing2)
    HIPCHK(launch_ring2_invariants(vol->x, ws.rinv, vol->nx, vol->ny, vol->nz,
                                   (p->flags & PIFCM_Q2_SQDIST) ? 1 : 0, ctx->s));
  const size_t off0 = 0;
  const float* u0s[1] = {U_in};
  TRY(run_invariants(ctx, vol, 1, C, u0s, ws.invg, &off0, ws.flags, (int*)ws.stage));
  const TileShape ts = shape_for(ctx, C, m2, *vol);
  const VolDev vh = make_vol(*vol, ws.invg, ts, zbeg, zend, kind == kRing2 ? ws.rinv : nullptr);
  PairDev pr{};
  pr.U0 = U_in ? U_in : ws.ubuf;
  pr.Ua = U_out;
  pr.Ub = ws.ubuf;
  // Odd iterations write Ua, even ones Ub: when the run is expected to end
  // on an even iteration (no stop rule, an even count) and ws.ubuf is free
  // at the start (U_in given), the buffers swap so the last state lands in
  // U_out without a copy.
  if (U_in && p->eps == 0.f && (p->max_iter & 1) == 0) std::swap(pr.Ua, pr.Ub);
  pr.st = ws.st;
  pr.partials = ws.partials;

  char* pin = ws.stage;
  SolveState hs = init_state(centres_in, C, lambda, xi, p, ws.jhist);
  std::memcpy(pin, &hs, sizeof hs);
  std::memcpy(pin + sizeof(SolveState), &pr, sizeof pr);
  std::memcpy(pin + sizeof(SolveState) + sizeof(PairDev), &vh, sizeof(VolDev));
  HIPCHK(hipMemcpyAsync(ws.st, pin, sizeof hs, hipMemcpyHostToDevice, ctx->s));
  HIPCHK(hipMemcpyAsync(ws.tpair, pin + sizeof(SolveState), sizeof pr, hipMemcpyHostToDevice, ctx->s));
  HIPCHK(hipMemcpyAsync(ws.tvol, pin + sizeof(SolveState) + sizeof(PairDev), sizeof(VolDev),
                        hipMemcpyHostToDevice, ctx->s));
  if (!U_in) HIPCHK(launch_init_u(C, vol->x, N, ws.st, p->m, m2, ws.ubuf, ctx->s));
  if (slab) {
    // Planes outside the slab keep U_in in both iteration buffers.
    HIPCHK(hipMemcpyAsync(U_out, U_in, N * C * sizeof(float), hipMemcpyDeviceToDevice, ctx->s));
    HIPCHK(hipMemcpyAsync(ws.ubuf, U_in, N * C * sizeof(float), hipMemcpyDeviceToDevice, ctx->s));
  }

  LaunchArgs a = make_args(ctx, ws.tvol, ws.tpair, &vh, 1, 1, kind, p);
  const int occ = occupancy_of(kind, C, ts.nw, m2, true);
  const int grid = grid_for(ctx, a.nitems, occ, items_per_group(kind, ts.nw));
  int t = 0;
  SolveState* hst = (SolveState*)pin;
  TRY(timing_begin(ctx));
  while (t < p->max_iter) {
    const int k = p->eps > 0.f ? std::min(kChunk, p->max_iter - t) : p->max_iter - t;
    for (int i = 0; i < k; ++i) HIPCHK(launch_step(C, a, grid, ts.nw, m2, kind, true, ctx->s));
    t += k;
    if (p->eps > 0.f && t < p->max_iter) {
      HIPCHK(hipMemcpyAsync(hst, ws.st, sizeof(SolveState), hipMemcpyDeviceToHost, ctx->s));
      HIPCHK(hipStreamSynchronize(ctx->s));
      if (hst->stop) break;
    }
  }
  TRY(timing_end(ctx));
  // Objective of the final state (the fitness).
  LaunchArgs ae = a;
  const int occe = occupancy_of(kind, C, ts.nw, m2, false);
  HIPCHK(launch_step(C, ae, grid_for(ctx, a.nitems, occe, items_per_group(kind, ts.nw)), ts.nw, m2,
                     kind, false, ctx->s));
  HIPCHK(hipMemcpyAsync(hst, ws.st, sizeof(SolveState), hipMemcpyDeviceToHost, ctx->s));
  HIPCHK(hipStreamSynchronize(ctx->s));
  const int T = hst->iter;
  TRY(timing_collect(ctx, t));
  const float* Ufin = u_state_of(pr, T);
  if (labels_out) HIPCHK(launch_labels(Ufin, N, C, labels_out, ctx->s));
  if (Ufin != U_out) HIPCHK(hipMemcpyAsync(U_out, Ufin, N * C * sizeof(float), hipMemcpyDeviceToDevice, ctx->s));
  double* jh = ws.jh_stage ? ws.jh_stage : J_hist_out;
  if (J_hist_out && T > 0)
    HIPCHK(hipMemcpyAsync(jh, ws.jhist, (size_t)T * sizeof(double), hipMemcpyDeviceToHost, ctx->s));
  HIPCHK(hipStreamSynchronize(ctx->s));
  if (centres_out)
    for (int j = 0; j < C; ++j) centres_out[j] = hst->c[T & 1][j];
  if (J_out) *J_out = hst->J_eval;
  if (iters_out) *iters_out = T;
  if (J_hist_out && T > 0 && ws.jh_stage) std::memcpy(J_hist_out, jh, (size_t)T * sizeof(double));
  return PIFCM_OK;
}

// One IFCM solve in the context's workspace (allocated or grown here);
// shared by ifcm_solve, ifcm_solve_slab and pifcm_fcm_init.
pifcm_status solve_impl(pifcm_ctx* ctx, const pifcm_volume* vol, const pifcm_params* p,
                        float lambda, float xi, const float* centres_in, const float* U_in,
                        float* U_out, float* centres_out, uint8_t* labels_out, double* J_out,
                        int32_t* iters_out, double* J_hist_out, int zbeg = 0, int zend = -1) {
  if (zend < 0) zend = vol->nz;
  const int C = p->C;
  const int kind = kind_of(p, lambda == 0.0f && xi == 0.0f);
  const size_t N = nvox(*vol);
  const size_t Np = (N + 63) / 64 * 64;
  if (is_ring(kind)) TRY(prepare_ring(ctx, p));
  const int slots = solve_slots(ctx, vol, p, zbeg, zend);
  TRY(ensure(ctx, ctx->invg, Np * sizeof(float), "iteration invariants"));
  if (kind == kRing2) TRY(ensure(ctx, ctx->rinv, Np * 4 * sizeof(float), "ring invariants"));
  TRY(ensure(ctx, ctx->flags, 64, "flags"));
  TRY(ensure(ctx, ctx->ubuf, N * C * sizeof(float), "memberships"));
  TRY(ensure(ctx, ctx->partials, (size_t)slots * (2 * C + 1) * sizeof(float), "tile sums"));
  TRY(ensure(ctx, ctx->states, sizeof(SolveState), "solve state"));
  TRY(ensure(ctx, ctx->jhist, (size_t)std::max(1, p->max_iter) * sizeof(double), "objective history"));
  TRY(ensure_pinned(ctx, kStageBytes + (size_t)std::max(1, p->max_iter) * sizeof(double) + 4096));
  SolveWs ws;
  ws.invg = (float*)ctx->invg.p;
  ws.rinv = kind == kRing2 ? (float*)ctx->rinv.p : nullptr;
  ws.ubuf = (float*)ctx->ubuf.p;
  ws.partials = (float*)ctx->partials.p;
  ws.st = (SolveState*)ctx->states.p;
  ws.tpair = (PairDev*)ctx->tpair.p;
  ws.tvol = (VolDev*)ctx->tvol.p;
  ws.jhist = (double*)ctx->jhist.p;
  ws.flags = (int*)ctx->flags.p;
  ws.stage = (char*)ctx->pinned;
  ws.jh_stage = (double*)((char*)ctx->pinned + kStageBytes);
  return solve_run(ctx, ws, vol, p, lambda, xi, centres_in, U_in, U_out, centres_out, labels_out, J_out,
                   iters_out, J_hist_out, zbeg, zend);
}

pifcm_status check_solve_args(pifcm_ctx* ctx, const pifcm_volume* vol, const pifcm_params* p,
                              float lambda, float xi, const float* centres_in, const float* U_in,
                              const float* U_out) {
  TRY(check_params(ctx, p));
  TRY(check_volume(ctx, vol, p->C));
  if (!(std::fabs(lambda) <= kMaxWeight) || !(std::fabs(xi) <= kMaxWeight))
    return fail(ctx, PIFCM_E_INVALID, "lambda and xi must be finite with magnitude <= %g", kMaxWeight);
  if (!centres_in) return fail(ctx, PIFCM_E_INVALID, "centres_in is NULL");
  for (int j = 0; j < p->C; ++j)
    if (!std::isfinite(centres_in[j])) return fail(ctx, PIFCM_E_INVALID, "centres_in[%d] is not finite", j);
  if (!U_out) return fail(ctx, PIFCM_E_INVALID, "U_out is NULL");
  if (!aligned16(U_out) || (U_in && !aligned16(U_in)))
    return fail(ctx, PIFCM_E_INVALID, "membership buffers must be 16-byte aligned");
  const size_t bytes = nvox(*vol) * p->C * sizeof(float);
  if (U_in && ranges_overlap(U_in, bytes, U_out, bytes))
    return fail(ctx, PIFCM_E_INVALID, "U_out must not overlap U_in");
  return PIFCM_OK;
}

}  // namespace

extern "C" {

pifcm_status ifcm_solve(pifcm_ctx* ctx, const pifcm_volume* vol, const pifcm_params* p,
                        float lambda, float xi, const float* centres_in, const float* U_in,
                        float* U_out, float* centres_out, uint8_t* labels_out, double* J_out,
                        int32_t* iters_out, double* J_hist_out) {
  if (!ctx) return PIFCM_E_INVALID;
  ctx->err.clear();
  TRY(check_solve_args(ctx, vol, p, lambda, xi, centres_in, U_in, U_out));
  TRY(begin(ctx));
  float c_tmp[kMaxC];
  double J = 0.0;
  int32_t T = 0;
  std::vector<double> jh((size_t)std::max(1, p->max_iter));
  TRY(solve_impl(ctx, vol, p, lambda, xi, centres_in, U_in, U_out, c_tmp, labels_out, &J, &T,
                 J_hist_out ? jh.data() : nullptr));
  TRY(finish(ctx));
  if (centres_out) std::memcpy(centres_out, c_tmp, sizeof(float) * p->C);
  if (J_out) *J_out = J;
  if (iters_out) *iters_out = T;
  if (J_hist_out) std::memcpy(J_hist_out, jh.data(), sizeof(double) * (size_t)T);
  return PIFCM_OK;
}

pifcm_status ifcm_solve_noalloc(pifcm_ctx* ctx, const pifcm_volume* vol, const pifcm_params* p,
                                float lambda, float xi, const float* centres_in, const float* U_in,
                                float* U_out, float* centres_out, uint8_t* labels_out, double* J_out,
                                int32_t* iters_out, double* J_hist_out) {
  if (!ctx) return PIFCM_E_INVALID;
  ctx->err.clear();
  TRY(check_solve_args(ctx, vol, p, lambda, xi, centres_in, U_in, U_out));
  if (ring_params(p))
    return fail(ctx, PIFCM_E_UNSUPPORTED, "ifcm_solve_noalloc covers the 3x3x3 neighbourhood (V = 1) only");
  // The workspace of solve_run, carved out of this device's scratch array.
  const int C = p->C;
  const size_t N = nvox(*vol);
  const size_t Np = (N + 63) / 64 * 64;
  const int slots = solve_slots(ctx, vol, p, 0, vol->nz);
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t o_invg = 0;
  const size_t o_ubuf = o_invg + al(Np * sizeof(float));
  const size_t o_part = o_ubuf + al(N * C * sizeof(float));
  const size_t o_st = o_part + al((size_t)slots * (2 * C + 1) * sizeof(float));
  const size_t o_pair = o_st + al(sizeof(SolveState));
  const size_t o_vol = o_pair + al(sizeof(PairDev));
  const size_t o_jh = o_vol + al(sizeof(VolDev));
  const size_t o_flags = o_jh + al((size_t)std::max(1, p->max_iter) * sizeof(double));
  const size_t need = o_flags + al(2 * sizeof(int));
  if (need > kScratchBytes)
    return fail(ctx, PIFCM_E_INVALID,
                "ifcm_solve_noalloc: this solve needs %zu bytes of scratch (N = %zu, C = %d, max_iter = %d), "
                "more than the %zu bytes the library holds per device; use ifcm_solve",
                need, N, C, p->max_iter, kScratchBytes);
  std::mutex* mu = scratch_call_lock(ctx->device);
  if (!mu) return fail(ctx, PIFCM_E_UNSUPPORTED, "device %d is beyond the scratch table", ctx->device);
  std::lock_guard<std::mutex> lock(*mu);
  TRY(begin(ctx));
  void* base = nullptr;
  HIPCHK(scratch_region(ctx->device, &base));
  char* sc = (char*)base;
  SolveWs ws;
  ws.invg = (float*)(sc + o_invg);
  ws.ubuf = (float*)(sc + o_ubuf);
  ws.partials = (float*)(sc + o_part);
  ws.st = (SolveState*)(sc + o_st);
  ws.tpair = (PairDev*)(sc + o_pair);
  ws.tvol = (VolDev*)(sc + o_vol);
  ws.jhist = (double*)(sc + o_jh);
  ws.flags = (int*)(sc + o_flags);
  ws.stage = (char*)ctx->pinned;  // allocated at pifcm_create, at least kStageBytes
  ws.jh_stage = nullptr;          // the J history goes straight to J_hist_out
  float c_tmp[kMaxC];
  double J = 0.0;
  int32_t T = 0;
  TRY(solve_run(ctx, ws, vol, p, lambda, xi, centres_in, U_in, U_out, c_tmp, labels_out, &J, &T,
                J_hist_out, 0, vol->nz));
  TRY(finish(ctx));
  if (centres_out) std::memcpy(centres_out, c_tmp, sizeof(float) * C);
  if (J_out) *J_out = J;
  if (iters_out) *iters_out = T;
  return PIFCM_OK;
}

pifcm_status ifcm_solve_slab(pifcm_ctx* ctx, const pifcm_volume* vol, int32_t zbeg, int32_t zend,
                             const pifcm_params* p, float lambda, float xi, const float* centres_in,
                             const float* U_in, float* U_out, float* centres_out,
                             uint8_t* labels_out, double* J_out, int32_t* iters_out,
                             double* J_hist_out) {
  if (!ctx) return PIFCM_E_INVALID;
  ctx->err.clear();
  TRY(check_solve_args(ctx, vol, p, lambda, xi, centres_in, U_in, U_out));
  if (!U_in) return fail(ctx, PIFCM_E_INVALID, "slab mode needs U_in (the context memberships)");
  if (zbeg < 0 || zend > vol->nz || zbeg >= zend)
    return fail(ctx, PIFCM_E_INVALID, "planes [%d, %d) outside [0, %d)", zbeg, zend, vol->nz);
  TRY(begin(ctx));
  float c_tmp[kMaxC];
  double J = 0.0;
  int32_t T = 0;
  std::vector<double> jh((size_t)std::max(1, p->max_iter));
  TRY(solve_impl(ctx, vol, p, lambda, xi, centres_in, U_in, U_out, c_tmp, labels_out, &J, &T,
                 J_hist_out ? jh.data() : nullptr, zbeg, zend));
  TRY(finish(ctx));
  if (centres_out) std::memcpy(centres_out, c_tmp, sizeof(float) * p->C);
  if (J_out) *J_out = J;
  if (iters_out) *iters_out = T;
  if (J_hist_out) std::memcpy(J_hist_out, jh.data(), sizeof(double) * (size_t)T);
  return PIFCM_OK;
}

pifcm_status pifcm_fcm_init(pifcm_ctx* ctx, const pifcm_volume* vol, const pifcm_params* p,
                            float* U0_out, float* centres_out, int32_t* iters_out) {
  if (!ctx) return PIFCM_E_INVALID;
  ctx->err.clear();
  if (!p) return fail(ctx, PIFCM_E_INVALID, "params is NULL");
  float c0[kMaxC];
  const int C = std::max(2, std::min(p->C, kMaxC));
  for (int j = 0; j < C; ++j) c0[j] = (float)(((double)j + 0.5) / (double)p->C);
  TRY(check_solve_args(ctx, vol, p, 0.f, 0.f, c0, nullptr, U0_out));
  if (!centres_out) return fail(ctx, PIFCM_E_INVALID, "centres_out is NULL");
  TRY(begin(ctx));
  float c1[kMaxC];
  int32_t T = 0;
  TRY(solve_impl(ctx, vol, p, 0.f, 0.f, c0, nullptr, U0_out, c1, nullptr, nullptr, &T, nullptr));
  int32_t perm[kMaxC];
  for (int j = 0; j < C; ++j) perm[j] = j;
  std::stable_sort(perm, perm + C, [&](int a, int b) { return c1[a] < c1[b]; });
  HIPCHK(launch_permute(U0_out, nvox(*vol), C, perm, U0_out, ctx->s));
  HIPCHK(hipStreamSynchronize(ctx->s));
  TRY(finish(ctx));
  for (int j = 0; j < C; ++j) centres_out[j] = c1[perm[j]];
  if (iters_out) *iters_out = T;
  return PIFCM_OK;
}

}  // extern "C"

namespace {

// The swarm evaluation proper: B volumes x P particles, pair k = b * P + q
// starting from (centres_pp[k], U0_pp[k]); U0_check (per volume, may be
// NULL) are validated as memberships.  If state_out is given, the final
// memberships of pair k are copied to state_out[k] (device [N_b][C]).
pifcm_status swarm_core(pifcm_ctx* ctx, const pifcm_volume* vols, int32_t B, const pifcm_params* p,
                        const float* particles, int32_t P, const float* centres_pp,
                        const float* const* U0_pp, const float* const* U0_check,
                        float* const* state_out, double* fitness_out, float* centres_out,
                        int32_t* iters_out, int32_t mode) {
  const int C = p->C;
  const bool m2 = p->m == 2.0f;
  TRY(begin(ctx));
  // lambda = xi = 0 for every particle: plain FCM kernels.
  bool zero = true;
  for (long k = 0; k < 2L * B * P; ++k) zero = zero && particles[k] == 0.0f;
  const int kind = kind_of(p, zero);
  std::vector<size_t> off;
  TRY(prepare_volumes(ctx, vols, B, C, U0_check, off, kind == kRing2 ? p : nullptr));

  // Tile shape: one per launch (the batched kernel has one TY).
  const TileShape ts0 = shape_for(ctx, C, m2, vols[0]);
  std::vector<VolDev> vh(B);
  size_t ubytes = 0, slots = 0;
  std::vector<size_t> uoff(B), soff(B);
  for (int b = 0; b < B; ++b) {
    TileShape ts = shape_for(ctx, C, m2, vols[b]);
    ts.nw = ts0.nw;
    vh[b] = make_vol(vols[b], (const float*)ctx->invg.p + off[b], ts);
    uoff[b] = ubytes;
    ubytes += (size_t)P * 2 * ((nvox(vols[b]) * C + 63) / 64 * 64) * sizeof(float);
    soff[b] = slots;
    slots += (size_t)P * std::max(vh[b].tiles, vh[b].tiles1d);
  }
  const size_t npairs = (size_t)B * P;
  // Work items are numbered in 32 bits (their memberships alone would
  // outgrow the device long before), with room above the last one for the
  // fused step's hand-out, whose final tickets run up to one per wave past
  // the end of a range.
  if (slots > (size_t)INT32_MAX - ((size_t)1 << 20))
    return fail(ctx, PIFCM_E_UNSUPPORTED, "%zu tiles in one launch: more than 2^31 - 2^20", slots);
  TRY(ensure(ctx, ctx->ubuf, ubytes, "swarm memberships"));
  TRY(ensure(ctx, ctx->partials, slots * (2 * C + 1) * sizeof(float), "tile sums"));
  TRY(ensure(ctx, ctx->states, npairs * sizeof(SolveState), "solve states"));
  const size_t pin_bytes = npairs * (sizeof(SolveState) + sizeof(PairDev)) + sizeof(VolDev) * B + 4096;
  TRY(ensure_pinned(ctx, pin_bytes));
  for (int b = 0; b < B; ++b) {
    vh[b].invg = (const float*)ctx->invg.p + off[b];
    vh[b].rinv = kind == kRing2 ? (const float*)ctx->rinv.p + 4 * off[b] : nullptr;
  }

  char* pin = (char*)ctx->pinned;
  SolveState* hs = (SolveState*)pin;
  PairDev* hp = (PairDev*)(pin + npairs * sizeof(SolveState));
  VolDev* hv = (VolDev*)(pin + npairs * (sizeof(SolveState) + sizeof(PairDev)));
  SolveState* st_dev = (SolveState*)ctx->states.p;
  for (int b = 0; b < B; ++b) {
    hv[b] = vh[b];
    const size_t Nb = nvox(vols[b]);
    const size_t ustride = (Nb * C + 63) / 64 * 64;
    const int tb = std::max(vh[b].tiles, vh[b].tiles1d);
    for (int q = 0; q < P; ++q) {
      const size_t k = (size_t)b * P + q;
      hs[k] = init_state(centres_pp + k * C, C, particles[2 * k], particles[2 * k + 1], p, nullptr);
      PairDev& pr = hp[k];
      pr.U0 = U0_pp[k];
      pr.Ua = (float*)((char*)ctx->ubuf.p + uoff[b]) + (size_t)q * 2 * ustride;
      pr.Ub = pr.Ua + ustride;
      pr.st = st_dev + k;
      pr.partials = (float*)ctx->partials.p + (soff[b] + (size_t)q * tb) * (2 * C + 1);
    }
  }
  HIPCHK(hipMemcpyAsync(st_dev, hs, npairs * sizeof(SolveState), hipMemcpyHostToDevice, ctx->s));
  HIPCHK(hipMemcpyAsync(ctx->tpair.p, hp, npairs * sizeof(PairDev), hipMemcpyHostToDevice, ctx->s));
  HIPCHK(hipMemcpyAsync(ctx->tvol.p, hv, B * sizeof(VolDev), hipMemcpyHostToDevice, ctx->s));

  if (is_ring(kind)) TRY(prepare_ring(ctx, p));
  const VolDev* vdev = (const VolDev*)ctx->tvol.p;
  const PairDev* pdev = (const PairDev*)ctx->tpair.p;
  // Particles per work item of the batched launch (the per-pair launches of
  // the plain mode hold one particle).
  const int pt = mode == PIFCM_SWARM_BATCHED ? pt_for(kind, C, P, ts0) : 1;
  const int occ = occupancy_of(kind, C, ts0.nw, m2, true, pt);
  const int occe = occupancy_of(kind, C, ts0.nw, m2, false, pt);
  const int ipg = items_per_group(kind, ts0.nw);

  int64_t launches = 0;
  auto all_stopped = [&](bool& done) -> pifcm_status {
    HIPCHK(hipMemcpyAsync(hs, st_dev, npairs * sizeof(SolveState), hipMemcpyDeviceToHost, ctx->s));
    HIPCHK(hipStreamSynchronize(ctx->s));
    done = true;
    for (size_t k = 0; k < npairs; ++k) done = done && hs[k].stop;
    return PIFCM_OK;
  };

  if (mode == PIFCM_SWARM_BATCHED) {
    LaunchArgs a = make_args(ctx, vdev, pdev, vh, B, P, kind, p, pt);
    const int grid = grid_for(ctx, a.nitems, occ, ipg);
    const int chunk = p->eps > 0.f ? std::min(kChunk, std::max(1, p->max_iter)) : std::max(1, p->max_iter);
    // Capture `chunk` fused launches once; replay until every pair stops.
    std::vector<char> key(sizeof(LaunchArgs) + 5 * sizeof(int));
    std::memcpy(key.data(), &a, sizeof a);
    const int extra[5] = {grid, ts0.nw, C * 2 + (int)m2, kind, chunk};
    std::memcpy(key.data() + sizeof a, extra, sizeof extra);
    if (ctx->graph.key != key || !ctx->graph.exec) {
      if (ctx->graph.exec) HIPCHK(hipGraphExecDestroy(ctx->graph.exec));
      if (ctx->graph.graph) HIPCHK(hipGraphDestroy(ctx->graph.graph));
      ctx->graph.exec = nullptr;
      ctx->graph.graph = nullptr;
      ctx->graph.key.clear();
      HIPCHK(hipStreamBeginCapture(ctx->s, hipStreamCaptureModeThreadLocal));
      for (int i = 0; i < chunk; ++i) {
        hipError_t e = launch_step(C, a, grid, ts0.nw, m2, kind, true, ctx->s);
        if (e != hipSuccess) {
          hipGraph_t g = nullptr;
          (void)hipStreamEndCapture(ctx->s, &g);
          if (g) (void)hipGraphDestroy(g);
          return fail(ctx, PIFCM_E_HIP, "capture of the swarm step failed: %s", hipGetErrorString(e));
        }
      }
      HIPCHK(hipStreamEndCapture(ctx->s, &ctx->graph.graph));
      HIPCHK(hipGraphInstantiate(&ctx->graph.exec, ctx->graph.graph, nullptr, nullptr, 0));
      ctx->graph.key = key;
    }
    int t = 0;
    TRY(timing_begin(ctx));
    while (t < p->max_iter) {
      HIPCHK(hipGraphLaunch(ctx->graph.exec, ctx->s));
      t += chunk;
      if (t < p->max_iter) {
        bool done = false;
        TRY(all_stopped(done));
        if (done) break;
      }
    }
    TRY(timing_end(ctx));
    launches = t;
    HIPCHK(launch_step(C, a, grid_for(ctx, a.nitems, occe, ipg), ts0.nw, m2, kind, false, ctx->s));
  } else {
    // One launch per (volume, particle) per iteration.
    std::vector<LaunchArgs> args(npairs);
    std::vector<int> grids(npairs), gride(npairs);
    for (int b = 0; b < B; ++b) {
      std::vector<VolDev> one{vh[b]};
      for (int q = 0; q < P; ++q) {
        const size_t k = (size_t)b * P + q;
        args[k] = make_args(ctx, vdev + b, pdev + k, one, 1, 1, kind, p);
        grids[k] = grid_for(ctx, args[k].nitems, occ, ipg);
        gride[k] = grid_for(ctx, args[k].nitems, occe, ipg);
      }
    }
    int t = 0;
    TRY(timing_begin(ctx));
    while (t < p->max_iter) {
      const int k = p->eps > 0.f ? std::min(kChunk, p->max_iter - t) : p->max_iter - t;
      for (int i = 0; i < k; ++i)
        for (size_t q = 0; q < npairs; ++q)
          HIPCHK(launch_step(C, args[q], grids[q], ts0.nw, m2, kind, true, ctx->s));
      t += k;
      if (t < p->max_iter) {
        bool done = false;
        TRY(all_stopped(done));
        if (done) break;
      }
    }
    TRY(timing_end(ctx));
    launches = (int64_t)t * (int64_t)npairs;
    for (size_t q = 0; q < npairs; ++q)
      HIPCHK(launch_step(C, args[q], gride[q], ts0.nw, m2, kind, false, ctx->s));
  }
  HIPCHK(hipMemcpyAsync(hs, st_dev, npairs * sizeof(SolveState), hipMemcpyDeviceToHost, ctx->s));
  HIPCHK(hipStreamSynchronize(ctx->s));
  TRY(timing_collect(ctx, launches));
  if (state_out) {
    for (int b = 0; b < B; ++b)
      for (int q = 0; q < P; ++q) {
        const size_t k = (size_t)b * P + q;
        const float* fin = u_state_of(hp[k], hs[k].iter);
        if (fin != state_out[k])
          HIPCHK(hipMemcpyAsync(state_out[k], fin, nvox(vols[b]) * C * sizeof(float), hipMemcpyDeviceToDevice,
                                ctx->s));
      }
    HIPCHK(hipStreamSynchronize(ctx->s));
  }
  TRY(finish(ctx));
  for (size_t k = 0; k < npairs; ++k) {
    const int T = hs[k].iter;
    fitness_out[k] = hs[k].J_eval;
    if (centres_out)
      for (int j = 0; j < C; ++j) centres_out[k * C + j] = hs[k].c[T & 1][j];
    if (iters_out) iters_out[k] = T;
  }
  return PIFCM_OK;
}

}  // namespace

extern "C" {

pifcm_status swarm_evaluate(pifcm_ctx* ctx, const pifcm_volume* vols, int32_t B,
                            const pifcm_params* p, const float* particles, int32_t P,
                            const float* centres0, const float* const* U0, double* fitness_out,
                            float* centres_out, int32_t* iters_out, int32_t mode) {
  if (!ctx) return PIFCM_E_INVALID;
  ctx->err.clear();
  if (!vols || B < 1 || B > kMaxBatchVols)
    return fail(ctx, PIFCM_E_INVALID, "B = %d outside [1, %d]", B, kMaxBatchVols);
  if (P < 1 || (long)B * P > kMaxPairs)
    return fail(ctx, PIFCM_E_INVALID, "P = %d: need 1 <= P and B * P <= %d", P, kMaxPairs);
  if (mode != PIFCM_SWARM_BATCHED && mode != PIFCM_SWARM_PLAIN)
    return fail(ctx, PIFCM_E_INVALID, "unknown mode %d", mode);
  TRY(check_params(ctx, p));
  if (!particles || !centres0 || !U0 || !fitness_out)
    return fail(ctx, PIFCM_E_INVALID, "particles, centres0, U0 and fitness_out must be non-NULL");
  const int C = p->C;
  for (int b = 0; b < B; ++b) {
    TRY(check_volume(ctx, &vols[b], C));
    if (!U0[b] || !aligned16(U0[b])) return fail(ctx, PIFCM_E_INVALID, "U0[%d] is NULL or not 16-byte aligned", b);
    for (int j = 0; j < C; ++j)
      if (!std::isfinite(centres0[b * C + j])) return fail(ctx, PIFCM_E_INVALID, "centres0[%d][%d] is not finite", b, j);
  }
  for (long k = 0; k < 2L * B * P; ++k)
    if (!(std::fabs(particles[k]) <= kMaxWeight))
      return fail(ctx, PIFCM_E_INVALID, "particle value %ld is not finite or exceeds %g", k, kMaxWeight);
  std::vector<float> cpp((size_t)B * P * C);
  std::vector<const float*> upp((size_t)B * P);
  for (int b = 0; b < B; ++b)
    for (int q = 0; q < P; ++q) {
      upp[(size_t)b * P + q] = U0[b];
      for (int j = 0; j < C; ++j) cpp[((size_t)b * P + q) * C + j] = centres0[b * C + j];
    }
  return swarm_core(ctx, vols, B, p, particles, P, cpp.data(), upp.data(), U0, nullptr, fitness_out,
                    centres_out, iters_out, mode);
}

pifcm_status ifcm_backward(pifcm_ctx* ctx, const pifcm_volume* vol, const pifcm_params* p,
                           float lambda, float xi, const float* centres0, const float* U0,
                           int32_t K, int32_t ckpt_every, double* J_out, double* dJ_dlambda,
                           double* dJ_dxi, double* dJ_dcentres) {
  if (!ctx) return PIFCM_E_INVALID;
  ctx->err.clear();
  TRY(check_params(ctx, p));
  TRY(check_volume(ctx, vol, p->C));
  if (ring_params(p))
    return fail(ctx, PIFCM_E_UNSUPPORTED, "the adjoint is built for the 3x3x3 neighbourhood (V = 1)");
  if (!(std::fabs(lambda) <= kMaxWeight) || !(std::fabs(xi) <= kMaxWeight))
    return fail(ctx, PIFCM_E_INVALID, "lambda and xi must be finite with magnitude <= %g", kMaxWeight);
  if (!centres0 || !U0 || !dJ_dlambda || !dJ_dxi || !dJ_dcentres)
    return fail(ctx, PIFCM_E_INVALID, "centres0, U0 and the gradient outputs must be non-NULL");
  for (int j = 0; j < p->C; ++j)
    if (!std::isfinite(centres0[j])) return fail(ctx, PIFCM_E_INVALID, "centres0[%d] is not finite", j);
  if (!aligned16(U0)) return fail(ctx, PIFCM_E_INVALID, "U0 must be 16-byte aligned");
  if (K < 1 || K > 100000) return fail(ctx, PIFCM_E_INVALID, "K = %d outside [1, 1e5]", K);
  if (ckpt_every < 1 || ckpt_every > K)
    return fail(ctx, PIFCM_E_INVALID, "ckpt_every = %d outside [1, K = %d]", ckpt_every, K);
  const int C = p->C, S = ckpt_every;
  const bool m2 = p->m == 2.0f;
  const int kind = kind_of(p, lambda == 0.0f && xi == 0.0f);
  const size_t N = nvox(*vol);
  if (is_ring(kind)) TRY(prepare_ring(ctx, p));
  const size_t UB = N * C * sizeof(float);
  TRY(begin(ctx));
  std::vector<size_t> off;
  const float* u0s[1] = {U0};
  TRY(prepare_volumes(ctx, vol, 1, C, u0s, off));
  const TileShape ts = shape_for(ctx, C, m2, *vol);
  std::vector<VolDev> vh{make_vol(*vol, (const float*)ctx->invg.p, ts)};
  const int slots = std::max(vh[0].tiles, vh[0].tiles1d);
  // Workspace: forward ping-pong, checkpoints at t = S, 2S, ... <= K - 1,
  // the S - 1 recomputed states of a segment, two adjoint buffers, the
  // transpose sources, slots and small histories.
  const int nck = (K - 1) / S;
  const size_t hist_doubles = (size_t)(K + 1) * C * 2 + (size_t)K + 2;
  const size_t adj_slots = adjoint_slots(vol->nx, vol->ny, vol->nz) * (C + 2);
  TRY(ensure(ctx, ctx->ubuf, 2 * UB, "memberships"));
  TRY(ensure(ctx, ctx->adj_ck, (size_t)std::max(nck, 1) * UB, "checkpoints"));
  TRY(ensure(ctx, ctx->adj_seg, (size_t)std::max(S - 1, 1) * UB, "segment states"));
  TRY(ensure(ctx, ctx->adj_bar, 2 * UB, "adjoint memberships"));
  TRY(ensure(ctx, ctx->adj_pq, UB, "transpose sources"));
  TRY(ensure(ctx, ctx->adj_misc, adj_slots * sizeof(float) + hist_doubles * sizeof(double) +
                                     (size_t)(K + 1) * C * sizeof(float) + 1024, "adjoint sums"));
  TRY(ensure(ctx, ctx->partials, (size_t)slots * (2 * C + 1) * sizeof(float), "tile sums"));
  TRY(ensure(ctx, ctx->states, 2 * sizeof(SolveState), "solve states"));
  TRY(ensure(ctx, ctx->jhist, (size_t)K * sizeof(double), "objective history"));
  // Every recomputed step of the backward pass gets its own state and pair
  // record: R of them (S - 1 per full segment), uploaded in one copy.
  int R = 0;
  for (int t0 = 0; t0 < K; t0 += S) R += std::min(S, K - t0) - 1;
  const size_t rs_states = ((size_t)std::max(R, 1) * sizeof(SolveState) + 255) / 256 * 256;
  const size_t rs_bytes = rs_states + (size_t)std::max(R, 1) * sizeof(PairDev);
  TRY(ensure(ctx, ctx->adj_rs, rs_bytes, "recompute states"));
  TRY(ensure(ctx, ctx->tpair, (size_t)K * sizeof(PairDev), "pair records"));
  const size_t pin_fixed = (size_t)(S + 2) * (sizeof(SolveState) + sizeof(PairDev)) + sizeof(VolDev) +
                           (size_t)(K + 1) * C * sizeof(float) + 64 * sizeof(double) + 4096;
  const size_t pin_rs = (pin_fixed + 255) / 256 * 256;  // pinned copy of the recompute records
  const size_t pin_fwd = (pin_rs + rs_bytes + 255) / 256 * 256;  // ... and of the forward's
  const size_t pin_need = pin_fwd + (size_t)K * sizeof(PairDev);
  TRY(ensure_pinned(ctx, pin_need));
  char* misc = (char*)ctx->adj_misc.p;
  float* adj_parts = (float*)misc;
  double* cbar = (double*)(misc + ((adj_slots * sizeof(float) + 255) / 256) * 256);
  double* acc2 = cbar + (size_t)(K + 1) * C;
  double* B_hist = acc2 + 2;
  float* c_hist = (float*)(B_hist + (size_t)K * C);
  float* ubA = (float*)ctx->ubuf.p;
  float* ubB = (float*)((char*)ctx->ubuf.p + UB);
  SolveState* st_dev = (SolveState*)ctx->states.p;
  PairDev* tp = (PairDev*)ctx->tpair.p;
  char* pin = (char*)ctx->pinned;

  // ---------------------------------------------------------------- forward
  pifcm_params pf = *p;
  pf.eps = 0.f;
  pf.max_iter = K;
  SolveState hs = init_state(centres0, C, lambda, xi, &pf, (double*)ctx->jhist.p);
  hs.B_hist = B_hist;
  hs.c_hist = c_hist;
  // Iteration t (1-based) reads state t - 1 and writes state t.  A state
  // t = S, 2S, ... <= K - 1 is written straight into its checkpoint; the
  // others alternate between ubA (odd t) and ubB (even t), so no iteration
  // writes the buffer it reads.  Each iteration has its own pair record,
  // with its input and output in the fields the kernels read for the
  // iteration's parity (u_in_of, u_out_of).
  auto ckpt = [&](int t) -> float* { return (float*)((char*)ctx->adj_ck.p + (size_t)(t / S - 1) * UB); };
  // States of the last segment (t0_last < t < K) go straight into the
  // segment buffers the reverse sweep would recompute them into.
  auto seg_state = [&](int i) -> float* { return (float*)((char*)ctx->adj_seg.p + (size_t)(i - 1) * UB); };
  const int t0_last = ((K - 1) / S) * S;
  auto fwd_out = [&](int t) -> float* {
    if (t % S == 0 && t <= K - 1) return ckpt(t);
    if (t > t0_last && t < K) return seg_state(t - t0_last);
    return (t & 1) ? ubA : ubB;
  };
  PairDev* hrec = (PairDev*)(pin + pin_fwd);
  for (int t = 1; t <= K; ++t) {
    PairDev q{};
    q.st = st_dev;
    q.partials = (float*)ctx->partials.p;
    float* in = t == 1 ? nullptr : fwd_out(t - 1);
    q.U0 = t == 1 ? U0 : in;
    q.Ua = (t & 1) ? fwd_out(t) : in;
    q.Ub = (t & 1) ? (t == 1 ? fwd_out(t) : in) : fwd_out(t);
    hrec[t - 1] = q;
  }
  std::memcpy(pin, &hs, sizeof hs);
  std::memcpy(pin + sizeof(SolveState) + sizeof(PairDev), &vh[0], sizeof(VolDev));
  std::memcpy(pin + sizeof(SolveState) + sizeof(PairDev) + sizeof(VolDev), centres0, C * sizeof(float));
  HIPCHK(hipMemcpyAsync(st_dev, pin, sizeof hs, hipMemcpyHostToDevice, ctx->s));
  HIPCHK(hipMemcpyAsync(tp, hrec, (size_t)K * sizeof(PairDev), hipMemcpyHostToDevice, ctx->s));
  HIPCHK(hipMemcpyAsync(ctx->tvol.p, pin + sizeof(SolveState) + sizeof(PairDev), sizeof(VolDev),
                        hipMemcpyHostToDevice, ctx->s));
  HIPCHK(hipMemcpyAsync(c_hist, pin + sizeof(SolveState) + sizeof(PairDev) + sizeof(VolDev),
                        C * sizeof(float), hipMemcpyHostToDevice, ctx->s));
  LaunchArgs a = make_args(ctx, (const VolDev*)ctx->tvol.p, tp, vh, 1, 1, kind, p);
  const int occ = occupancy_of(kind, C, ts.nw, m2, true);
  const int grid = grid_for(ctx, a.nitems, occ, items_per_group(kind, ts.nw));
  const int occe = occupancy_of(kind, C, ts.nw, m2, false);
  const int gride = grid_for(ctx, a.nitems, occe, items_per_group(kind, ts.nw));
  for (int t = 1; t <= K; ++t) {
    a.pairs = tp + (t - 1);
    HIPCHK(launch_step(C, a, grid, ts.nw, m2, kind, true, ctx->s));
  }
  // The objective of state K, through the last iteration's record.
  HIPCHK(launch_step(C, a, gride, ts.nw, m2, kind, false, ctx->s));
  SolveState* hst = (SolveState*)pin;
  float* hc = (float*)(pin + (size_t)(S + 2) * (sizeof(SolveState) + sizeof(PairDev)) + sizeof(VolDev));
  HIPCHK(hipMemcpyAsync(hst, st_dev, sizeof(SolveState), hipMemcpyDeviceToHost, ctx->s));
  HIPCHK(hipMemcpyAsync(hc, c_hist, (size_t)(K + 1) * C * sizeof(float), hipMemcpyDeviceToHost, ctx->s));
  HIPCHK(hipStreamSynchronize(ctx->s));
  const double J = hst->J_eval;
  const float* UK = fwd_out(K);
  std::vector<float> chost(hc, hc + (size_t)(K + 1) * C);

  // --------------------------------------------------------------- backward
  HIPCHK(hipMemsetAsync(acc2, 0, 2 * sizeof(double), ctx->s));
  float* bar0 = (float*)ctx->adj_bar.p;
  float* bar1 = (float*)((char*)ctx->adj_bar.p + UB);
  AdjArgs ad{};
  ad.x = vol->x;
  ad.invg = (const float*)ctx->invg.p;
  ad.nx = vol->nx;
  ad.ny = vol->ny;
  ad.nz = vol->nz;
  ad.q2_sqdist = (p->flags & PIFCM_Q2_SQDIST) ? 1 : 0;
  ad.m = p->m;
  ad.lam = lambda;
  ad.xi = xi;
  ad.PQ = (float*)ctx->adj_pq.p;
  ad.partials = adj_parts;
  ad.num_cu = ctx->num_cu;
  // The objective at the final state.
  ad.U = UK;
  ad.c = c_hist + (size_t)K * C;
  ad.Ubar_direct = bar1;
  HIPCHK(launch_adjoint(C, ad, m2, true, bar0, cbar + (size_t)K * C, acc2, ctx->s));
  float* cur = bar0;
  float* other = bar1;
  // Recomputed states of the current segment: seg[i] = U^(t0 + i), computed
  // by one forward iteration U^(t0+i-1) -> U^(t0+i) with c^(t0+i-1) each
  // (the last segment's are still there from the forward pass).  Their state
  // and pair records are written once, here, and uploaded in one copy, so
  // the reverse sweep below only enqueues work.
  SolveState* rs_st = (SolveState*)ctx->adj_rs.p;
  PairDev* rs_pr = (PairDev*)((char*)ctx->adj_rs.p + rs_states);
  {
    char* hrs = pin + pin_rs;
    SolveState* hs_rs = (SolveState*)hrs;
    PairDev* hp_rs = (PairDev*)(hrs + rs_states);
    int r = 0;
    for (int t0 = 0; t0 < K; t0 += S) {
      const int len = std::min(S, K - t0);
      for (int i = 1; i < len; ++i, ++r) {
        pifcm_params p1 = *p;
        p1.eps = 0.f;
        p1.max_iter = 1;
        hs_rs[r] = init_state(&chost[(size_t)(t0 + i - 1) * C], C, lambda, xi, &p1, nullptr);
        PairDev q{};
        q.U0 = i == 1 ? (t0 == 0 ? U0 : ckpt(t0)) : seg_state(i - 1);
        q.Ua = seg_state(i);
        q.Ub = q.Ua;
        q.st = rs_st + r;
        q.partials = (float*)ctx->partials.p;
        hp_rs[r] = q;
      }
    }
    if (R > 0) HIPCHK(hipMemcpyAsync(ctx->adj_rs.p, hrs, rs_bytes, hipMemcpyHostToDevice, ctx->s));
  }
  std::vector<const float*> seg(S, nullptr);
  int seg_t0 = -1, seg_r = 0;
  for (int t = K - 1; t >= 0; --t) {
    const int t0 = (t / S) * S;
    if (t0 != seg_t0) {
      // First record of segment t0: the segments before it use t0 / S * (S - 1).
      seg_r = (t0 / S) * (S - 1);
      seg[0] = t0 == 0 ? U0 : ckpt(t0);
      const int len = std::min(S, K - t0);
      for (int i = 1; i < len; ++i) {
        if (t0 != t0_last) {
          const LaunchArgs ar =
              make_args(ctx, (const VolDev*)ctx->tvol.p, rs_pr + seg_r + (i - 1), vh, 1, 1, kind, p);
          HIPCHK(launch_step(C, ar, grid, ts.nw, m2, kind, true, ctx->s));
        }
        seg[i] = seg_state(i);
      }
      seg_t0 = t0;
    }
    ad.U = seg[t - t0];
    ad.c = c_hist + (size_t)t * C;
    ad.Ubar_next = cur;
    ad.cbar_next = cbar + (size_t)(t + 1) * C;
    ad.c_next = c_hist + (size_t)(t + 1) * C;
    ad.B_next = B_hist + (size_t)t * C;
    HIPCHK(launch_adjoint(C, ad, m2, false, t > 0 ? other : nullptr, cbar + (size_t)t * C, acc2, ctx->s));
    std::swap(cur, other);
  }
  double* hout = (double*)(pin + pin_fixed - 64 * sizeof(double) - 4096);
  HIPCHK(hipMemcpyAsync(hout, cbar, C * sizeof(double), hipMemcpyDeviceToHost, ctx->s));
  HIPCHK(hipMemcpyAsync(hout + C, acc2, 2 * sizeof(double), hipMemcpyDeviceToHost, ctx->s));
  HIPCHK(hipStreamSynchronize(ctx->s));
  TRY(finish(ctx));
  if (J_out) *J_out = J;
  *dJ_dlambda = hout[C];
  *dJ_dxi = hout[C + 1];
  for (int j = 0; j < C; ++j) dJ_dcentres[j] = hout[j];
  return PIFCM_OK;
}

pifcm_status pifcm_set_decomposition(pifcm_ctx* ctx, const pifcm_volume* vols, int32_t B,
                                     const pifcm_params* p, int32_t waves_per_group,
                                     int32_t planes_per_tile, int32_t particles_per_item) {
  if (!ctx) return PIFCM_E_INVALID;
  ctx->err.clear();
  if (!vols || B < 1 || B > kMaxBatchVols) return fail(ctx, PIFCM_E_INVALID, "B = %d outside [1, %d]", B, kMaxBatchVols);
  TRY(check_params(ctx, p));
  for (int b = 0; b < B; ++b) TRY(check_volume(ctx, &vols[b], p->C));
  const int nw = waves_per_group, zc = planes_per_tile, pt = particles_per_item;
  if (nw != 1 && nw != 2 && nw != 4) return fail(ctx, PIFCM_E_INVALID, "waves_per_group = %d: 1, 2 or 4", nw);
  if (p->C != 4 && nw != 4) return fail(ctx, PIFCM_E_UNSUPPORTED, "waves_per_group = %d is built for C = 4 only", nw);
  if (zc < 0) return fail(ctx, PIFCM_E_INVALID, "planes_per_tile = %d must be >= 0 (0: the default)", zc);
  if (pt != 1 && pt != 2) return fail(ctx, PIFCM_E_INVALID, "particles_per_item = %d: 1 or 2", pt);
  if (p->C != 4 && pt != 1) return fail(ctx, PIFCM_E_UNSUPPORTED, "particles_per_item = 2 is built for C = 4 only");
  for (int b = 0; b < B; ++b)
    ctx->tuned[std::make_tuple(p->C, (int)(p->m == 2.0f), vols[b].nx, vols[b].ny, vols[b].nz)] = TileShape{nw, zc, pt};
  return PIFCM_OK;
}

pifcm_status pifcm_tune(pifcm_ctx* ctx, const pifcm_volume* vols, int32_t B, const pifcm_params* p,
                        int32_t P, char* best_out, int32_t best_len) {
  if (!ctx) return PIFCM_E_INVALID;
  ctx->err.clear();
  if (!vols || B < 1 || B > kMaxBatchVols) return fail(ctx, PIFCM_E_INVALID, "B = %d outside [1, %d]", B, kMaxBatchVols);
  if (P < 1 || (long)B * P > kMaxPairs) return fail(ctx, PIFCM_E_INVALID, "P = %d out of range", P);
  TRY(check_params(ctx, p));
  auto describe = [&](const char* text) {
    if (best_out && best_len > 0) {
      std::strncpy(best_out, text, (size_t)best_len - 1);
      best_out[best_len - 1] = 0;
    }
  };
  if (ring_params(p)) {
    describe("general neighbourhood: fixed decomposition, nothing timed");
    return PIFCM_OK;
  }
  const int C = p->C;
  for (int b = 0; b < B; ++b) TRY(check_volume(ctx, &vols[b], C));
  const bool m2 = p->m == 2.0f;
  auto apply = [&](const TileShape& t) {
    for (int b = 0; b < B; ++b) ctx->tuned[std::make_tuple(C, (int)m2, vols[b].nx, vols[b].ny, vols[b].nz)] = t;
  };
  // A choice kept in the cache file for this device, parameters and shape
  // bucket is applied without timing.
  const std::string key = tune_key(ctx, vols, B, p, P);
  const char* cache = std::getenv("PIFCM_TUNE_CACHE");
  if (cache && *cache) {
    TileShape t;
    double ms = 0.0;
    if (tune_cache_get(cache, key, t, ms)) {
      apply(t);
      char tz[16];
      if (t.zc > 0) snprintf(tz, sizeof tz, "%d", t.zc);
      else snprintf(tz, sizeof tz, "auto");
      char desc[512];
      snprintf(desc, sizeof desc, "waves_per_group=%d planes_per_tile=%s particles_per_item=%d step_ms=%.4f cached [%s]",
               t.nw, tz, t.pt, ms, key.c_str());
      describe(desc);
      return PIFCM_OK;
    }
  }
  // Initial memberships: eq (2) with the attraction factor 1 for evenly
  // spaced centres, one buffer per volume.
  size_t total = 0;
  std::vector<size_t> uoff(B);
  int bmin = 0;  // the smallest volume: element-wise membership check
  for (int b = 0; b < B; ++b) {
    uoff[b] = total;
    total += (nvox(vols[b]) * C + 63) / 64 * 64;
    if (nvox(vols[b]) < nvox(vols[bmin])) bmin = b;
  }
  const size_t nmin = nvox(vols[bmin]) * C;
  const size_t nmin_pad = (nmin + 63) / 64 * 64;
  const int Pc = std::min(P, 2);  // particles of the membership check
  TRY(begin(ctx));
  TRY(ensure(ctx, ctx->tune_u0, total * sizeof(float), "tuning memberships"));
  TRY(ensure(ctx, ctx->tune_state, sizeof(SolveState), "tuning state"));
  TRY(ensure(ctx, ctx->tune_ref, 2 * (size_t)Pc * nmin_pad * sizeof(float), "tuning reference memberships"));
  TRY(ensure_pinned(ctx, std::max<size_t>(sizeof(SolveState), 2 * (size_t)Pc * nmin_pad * sizeof(float)) + 4096));
  std::vector<float> c0((size_t)B * C);
  for (int b = 0; b < B; ++b)
    for (int j = 0; j < C; ++j) c0[(size_t)b * C + j] = (float)(((double)j + 0.5) / C);
  SolveState hs = init_state(c0.data(), C, 0.f, 0.f, p, nullptr);
  std::memcpy(ctx->pinned, &hs, sizeof hs);
  HIPCHK(hipMemcpyAsync(ctx->tune_state.p, ctx->pinned, sizeof hs, hipMemcpyHostToDevice, ctx->s));
  std::vector<const float*> U0(B);
  for (int b = 0; b < B; ++b) {
    float* u = (float*)ctx->tune_u0.p + uoff[b];
    HIPCHK(launch_init_u(C, vols[b].x, nvox(vols[b]), (const SolveState*)ctx->tune_state.p, p->m, m2, u,
                         ctx->s));
    U0[b] = u;
  }
  HIPCHK(hipStreamSynchronize(ctx->s));
  TRY(finish(ctx));
  // Particles on a regular grid over [0.05, 0.95]^2.
  std::vector<float> parts((size_t)B * P * 2);
  const int side = std::max(1, (int)std::ceil(std::sqrt((double)P)));
  for (int q = 0; q < P; ++q) {
    const float l = 0.05f + 0.9f * (float)(q % side) / (float)std::max(1, side - 1);
    const float x = 0.05f + 0.9f * (float)(q / side) / (float)std::max(1, side - 1);
    for (int b = 0; b < B; ++b) {
      parts[((size_t)b * P + q) * 2] = l;
      parts[((size_t)b * P + q) * 2 + 1] = x;
    }
  }
  pifcm_params pt = *p;
  pt.eps = 0.f;
  pt.max_iter = std::max(2, std::min(p->max_iter, 4));
  int maxz = 1;
  for (int b = 0; b < B; ++b) maxz = std::max(maxz, vols[b].nz);
  std::vector<TileShape> cands;
  // Candidate 0, the reference of the parity gate, is the default
  // decomposition (4 waves, each volume's default depth, one particle per
  // item); zc = 0 below stands for the default depth.
  cands.push_back(TileShape{4, 0, 1});
  const int nws[3] = {1, 2, 4};
  const int zcs[6] = {0, 8, 16, 32, 64, 128};
  const int maxpt = (C == 4 && P >= 2) ? 2 : 1;
  for (int ptc = 1; ptc <= maxpt; ++ptc)
    for (int nw : nws) {
      if (C != 4 && nw != 4) continue;
      for (int zc : zcs) {
        if (zc / 2 >= maxz && zc != 8) continue;  // one candidate covers the whole column
        if (nw == 4 && zc == 0 && ptc == 1) continue;
        if (zc == 0 && nw != 4) continue;
        cands.push_back(TileShape{nw, zc, ptc});
      }
    }
  const bool was_timing = ctx->timing;
  const auto saved = ctx->tuned;
  std::vector<double> fit_ref((size_t)B * P), fit((size_t)B * P);
  std::vector<float> cen_ref((size_t)B * P * C), cen((size_t)B * P * C);
  // Final memberships of the check: reference (candidate 0) in the first Pc
  // buffers, the candidate's in the next Pc.
  float* uref[2] = {(float*)ctx->tune_ref.p, (float*)ctx->tune_ref.p + nmin_pad};
  float* ucand[2] = {(float*)ctx->tune_ref.p + Pc * nmin_pad, (float*)ctx->tune_ref.p + (Pc + 1) * nmin_pad};
  const float* U0min[2] = {U0[bmin], U0[bmin]};
  std::vector<float> cmin((size_t)Pc * C);
  for (int q = 0; q < Pc; ++q)
    for (int j = 0; j < C; ++j) cmin[(size_t)q * C + j] = c0[(size_t)bmin * C + j];
  std::vector<double> fchk(Pc);
  double best_ms = 1e300;
  TileShape best = cands[0];
  std::string tried;
  for (size_t ci = 0; ci < cands.size(); ++ci) {
    apply(cands[ci]);
    ctx->timing = false;
    pifcm_status st = swarm_evaluate(ctx, vols, B, &pt, parts.data(), P, c0.data(), U0.data(),
                                     fit.data(), cen.data(), nullptr, PIFCM_SWARM_BATCHED);
    double ms = 0.0;
    if (st == PIFCM_OK) {
      ctx->timing = true;
      const double ms0 = ctx->step_ms;
      const int64_t n0 = ctx->step_launches;
      st = swarm_evaluate(ctx, vols, B, &pt, parts.data(), P, c0.data(), U0.data(), fit.data(),
                          cen.data(), nullptr, PIFCM_SWARM_BATCHED);
      ms = (ctx->step_ms - ms0) / std::max<int64_t>(1, ctx->step_launches - n0);
      ctx->step_ms = ms0;
      ctx->step_launches = n0;
    }
    // Memberships of the first particles on the smallest volume, element
    // by element (the same decomposition as the timed launch).
    if (st == PIFCM_OK) {
      ctx->timing = false;
      st = swarm_core(ctx, &vols[bmin], 1, &pt, parts.data() + (size_t)bmin * P * 2, Pc, cmin.data(), U0min,
                      nullptr, ci == 0 ? uref : ucand, fchk.data(), nullptr, nullptr, PIFCM_SWARM_BATCHED);
    }
    if (st != PIFCM_OK) {
      if (ci == 0) {
        ctx->timing = was_timing;
        ctx->tuned = saved;
        return st;
      }
      continue;
    }
    bool ok = true;
    double du = 0.0;
    if (ci == 0) {
      fit_ref = fit;
      cen_ref = cen;
    } else {
      for (size_t k = 0; k < fit.size(); ++k)
        ok = ok && std::fabs(fit[k] - fit_ref[k]) <= 1e-5 * std::fabs(fit_ref[k]);
      for (size_t k = 0; k < cen.size(); ++k)
        ok = ok && std::fabs(cen[k] - cen_ref[k]) <= 1e-5f * std::max(1e-3f, std::fabs(cen_ref[k]));
      float* hu = (float*)ctx->pinned;
      HIPCHK(hipMemcpyAsync(hu, ctx->tune_ref.p, 2 * (size_t)Pc * nmin_pad * sizeof(float), hipMemcpyDeviceToHost,
                            ctx->s));
      HIPCHK(hipStreamSynchronize(ctx->s));
      double dmax = 0.0, rmax = 0.0;
      for (int q = 0; q < Pc; ++q)
        for (size_t i = 0; i < nmin; ++i) {
          const double r = hu[q * nmin_pad + i], c = hu[(Pc + q) * nmin_pad + i];
          dmax = std::max(dmax, std::fabs(c - r));
          rmax = std::max(rmax, std::fabs(r));
        }
      du = dmax / std::max(rmax, 1e-30);
      ok = ok && du <= 1e-4;
    }
    char one[64];
    char zs[16];
    if (cands[ci].zc > 0) snprintf(zs, sizeof zs, "%d", cands[ci].zc);
    else snprintf(zs, sizeof zs, "auto");
    snprintf(one, sizeof one, "%s%dx%sx%d:%.3f%s", tried.empty() ? "" : " ", cands[ci].nw, zs,
             cands[ci].pt, ms, ok ? "" : "(differs)");
    tried += one;
    if (ok && ms < best_ms) {
      best_ms = ms;
      best = cands[ci];
    }
  }
  ctx->timing = was_timing;
  ctx->tuned = saved;
  apply(best);
  if (cache && *cache) tune_cache_put(cache, key, best, best_ms);
  // The depth reported is the one chosen (each volume clamps it to its
  // plane count); "auto" is each volume's default depth.
  char bz[16];
  if (best.zc > 0) snprintf(bz, sizeof bz, "%d", best.zc);
  else snprintf(bz, sizeof bz, "auto");
  char desc[1024];
  snprintf(desc, sizeof desc,
           "waves_per_group=%d planes_per_tile=%s particles_per_item=%d step_ms=%.4f candidates=%zu [%s]", best.nw,
           bz, best.pt, best_ms, cands.size(), tried.c_str());
  describe(desc);
  ctx->err.clear();
  return PIFCM_OK;
}

}  // extern "C"

namespace {

// Synchronous global-best swarm bookkeeping (Algorithm 1, steps 5-8) around
// an evaluation callback eval(g, particles [B][P][2] as float, fitness).
// best_k (may be NULL) receives, per volume, the particle holding the best.
pifcm_status pso_run(pifcm_ctx* ctx, int32_t B, int32_t P, int32_t G, const double* x0,
                     const double* v0, const double* r1, const double* r2, double w, double c1,
                     double c2, const std::function<pifcm_status(int, const float*, double*)>& eval,
                     double* best_pos, double* best_fit, double* fit_hist, double* pos_hist,
                     int* best_k) {
  if (B < 1 || B > kMaxBatchVols || P < 1 || G < 1 || (long)B * P > kMaxPairs)
    return fail(ctx, PIFCM_E_INVALID, "B = %d, P = %d, G = %d out of range", B, P, G);
  if (!x0 || !v0 || !r1 || !r2 || !best_pos || !best_fit)
    return fail(ctx, PIFCM_E_INVALID, "x0, v0, r1, r2, best_pos and best_fit must be non-NULL");
  if (!std::isfinite(w) || !std::isfinite(c1) || !std::isfinite(c2))
    return fail(ctx, PIFCM_E_INVALID, "w, c1, c2 must be finite");
  std::vector<double> pos((size_t)B * P * 2), vel((size_t)B * P * 2), pb((size_t)B * P * 2);
  std::vector<double> pbf((size_t)B * P), gb((size_t)B * 2), gbf(B);
  std::vector<int> gk(B, 0);
  std::vector<float> parts((size_t)B * P * 2);
  std::vector<double> fit((size_t)B * P);
  for (int b = 0; b < B; ++b)
    for (int k = 0; k < P * 2; ++k) {
      pos[(size_t)b * P * 2 + k] = x0[k];
      vel[(size_t)b * P * 2 + k] = v0[k];
    }
  for (int g = 0; g < G; ++g) {
    for (size_t k = 0; k < parts.size(); ++k) parts[k] = (float)pos[k];
    TRY(eval(g, parts.data(), fit.data()));
    for (int b = 0; b < B; ++b) {
      for (int q = 0; q < P; ++q) {
        const size_t k = (size_t)b * P + q;
        if (fit_hist) fit_hist[((size_t)b * G + g) * P + q] = fit[k];
        if (pos_hist) {
          pos_hist[(((size_t)b * G + g) * P + q) * 2] = pos[k * 2];
          pos_hist[(((size_t)b * G + g) * P + q) * 2 + 1] = pos[k * 2 + 1];
        }
        if (g == 0 || fit[k] < pbf[k]) {  // step 5
          pbf[k] = fit[k];
          pb[k * 2] = pos[k * 2];
          pb[k * 2 + 1] = pos[k * 2 + 1];
        }
      }
      bool have = false;  // step 6, global best over the personal bests
      for (int q = 0; q < P; ++q) {
        const size_t k = (size_t)b * P + q;
        if (!have || pbf[k] < gbf[b]) {
          gbf[b] = pbf[k];
          gb[b * 2] = pb[k * 2];
          gb[b * 2 + 1] = pb[k * 2 + 1];
          gk[b] = q;
          have = true;
        }
      }
    }
    if (g + 1 == G) break;
    for (int b = 0; b < B; ++b)  // steps 7-8
      for (int q = 0; q < P; ++q)
        for (int d = 0; d < 2; ++d) {
          const size_t k = ((size_t)b * P + q) * 2 + d;
          const size_t s = ((size_t)g * P + q) * 2 + d;
          const double v = w * vel[k] + c1 * r1[s] * (pb[k] - pos[k]) + c2 * r2[s] * (gb[b * 2 + d] - pos[k]);
          const double np = pos[k] + v;
          vel[k] = v;
          pos[k] = np < 0.0 ? 0.0 : (np > 1.0 ? 1.0 : np);
        }
  }
  for (int b = 0; b < B; ++b) {
    best_pos[b * 2] = gb[b * 2];
    best_pos[b * 2 + 1] = gb[b * 2 + 1];
    best_fit[b] = gbf[b];
    if (best_k) best_k[b] = gk[b];
  }
  return PIFCM_OK;
}

}  // namespace

extern "C" {

pifcm_status pifcm_pso(pifcm_ctx* ctx, const pifcm_volume* vols, int32_t B, const pifcm_params* p,
                       int32_t P, int32_t G, const double* x0, const double* v0, const double* r1,
                       const double* r2, double w, double c1, double c2, const float* centres0,
                       const float* const* U0, int32_t mode, double* best_pos, double* best_fit,
                       double* fit_hist, double* pos_hist, int32_t* iters_hist) {
  if (!ctx) return PIFCM_E_INVALID;
  ctx->err.clear();
  std::vector<int32_t> its(iters_hist && B > 0 && P > 0 ? (size_t)B * P : 0);
  auto eval = [&](int g, const float* parts, double* fit) -> pifcm_status {
    TRY(swarm_evaluate(ctx, vols, B, p, parts, P, centres0, U0, fit, nullptr,
                       iters_hist ? its.data() : nullptr, mode));
    if (iters_hist)
      for (int b = 0; b < B; ++b)
        for (int q = 0; q < P; ++q) iters_hist[((size_t)b * G + g) * P + q] = its[(size_t)b * P + q];
    return PIFCM_OK;
  };
  return pso_run(ctx, B, P, G, x0, v0, r1, r2, w, c1, c2, eval, best_pos, best_fit, fit_hist,
                 pos_hist, nullptr);
}

pifcm_status pifcm_pso_interleaved(pifcm_ctx* ctx, const pifcm_volume* vols, int32_t B,
                                   const pifcm_params* p, int32_t P, int32_t G, int32_t steps,
                                   const double* x0, const double* v0, const double* r1,
                                   const double* r2, double w, double c1, double c2,
                                   const float* centres0, const float* const* U0, int32_t mode,
                                   double* best_pos, double* best_fit, double* fit_hist,
                                   double* pos_hist, float* const* U_best_out,
                                   float* centres_best_out) {
  if (!ctx) return PIFCM_E_INVALID;
  ctx->err.clear();
  if (steps < 1 || steps > 1000000) return fail(ctx, PIFCM_E_INVALID, "steps = %d must be in [1, 1e6]", steps);
  if (!vols || B < 1 || B > kMaxBatchVols || P < 1 || (long)B * P > kMaxPairs)
    return fail(ctx, PIFCM_E_INVALID, "B = %d, P = %d out of range", B, P);
  TRY(check_params(ctx, p));
  if (!centres0 || !U0) return fail(ctx, PIFCM_E_INVALID, "centres0 and U0 must be non-NULL");
  const int C = p->C;
  for (int b = 0; b < B; ++b) {
    TRY(check_volume(ctx, &vols[b], C));
    if (!U0[b] || !aligned16(U0[b])) return fail(ctx, PIFCM_E_INVALID, "U0[%d] is NULL or not 16-byte aligned", b);
    if (U_best_out && (!U_best_out[b] || !aligned16(U_best_out[b])))
      return fail(ctx, PIFCM_E_INVALID, "U_best_out[%d] is NULL or not 16-byte aligned", b);
  }
  // Per-particle states, one membership buffer per (volume, particle).
  std::vector<size_t> soff((size_t)B * P);
  size_t total = 0;
  for (int b = 0; b < B; ++b)
    for (int q = 0; q < P; ++q) {
      soff[(size_t)b * P + q] = total;
      total += (nvox(vols[b]) * C + 63) / 64 * 64;
    }
  TRY(begin(ctx));
  TRY(ensure(ctx, ctx->pso_state, total * sizeof(float), "particle states"));
  std::vector<float*> st((size_t)B * P);
  std::vector<float> cen((size_t)B * P * C), cnext((size_t)B * P * C);
  for (int b = 0; b < B; ++b)
    for (int q = 0; q < P; ++q) {
      const size_t k = (size_t)b * P + q;
      st[k] = (float*)ctx->pso_state.p + soff[k];
      HIPCHK(hipMemcpyAsync(st[k], U0[b], nvox(vols[b]) * C * sizeof(float), hipMemcpyDeviceToDevice, ctx->s));
      for (int j = 0; j < C; ++j) cen[k * C + j] = centres0[b * C + j];
    }
  HIPCHK(hipStreamSynchronize(ctx->s));
  pifcm_params ps = *p;
  ps.max_iter = steps;
  ps.eps = 0.f;
  std::vector<const float*> stc(st.begin(), st.end());
  auto eval = [&](int g, const float* parts, double* fit) -> pifcm_status {
    for (long k = 0; k < 2L * B * P; ++k)
      if (!(std::fabs(parts[k]) <= kMaxWeight))
        return fail(ctx, PIFCM_E_INVALID, "particle value %ld is not finite or exceeds %g", k, kMaxWeight);
    TRY(swarm_core(ctx, vols, B, &ps, parts, P, cen.data(), stc.data(), g == 0 ? U0 : nullptr,
                   st.data(), fit, cnext.data(), nullptr, mode));
    cen.swap(cnext);
    return PIFCM_OK;
  };
  std::vector<int> bk(B);
  TRY(pso_run(ctx, B, P, G, x0, v0, r1, r2, w, c1, c2, eval, best_pos, best_fit, fit_hist, pos_hist,
              bk.data()));
  for (int b = 0; b < B; ++b) {
    const size_t k = (size_t)b * P + bk[b];
    if (U_best_out)
      HIPCHK(hipMemcpyAsync(U_best_out[b], st[k], nvox(vols[b]) * C * sizeof(float), hipMemcpyDeviceToDevice,
                            ctx->s));
    if (centres_best_out)
      for (int j = 0; j < C; ++j) centres_best_out[b * C + j] = cen[k * C + j];
  }
  HIPCHK(hipStreamSynchronize(ctx->s));
  TRY(finish(ctx));
  return PIFCM_OK;
}

}  // extern "C"
