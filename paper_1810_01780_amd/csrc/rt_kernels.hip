// Eikonal ray tracing on gfx950 (MI355X), FP64: the general 3-D trace
// kernel, the set-up, compaction and resume kernels, and the host launcher
// (raytrace_launch, raytrace_launch_static).  The trace loop itself is in
// rt_trace.hpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <optional>

#include "rt_trace.hpp"

namespace rt {

// Persistent trace kernel of the general 3-D gradient body (analytic media
// along any axis, anomalies, grids), two waves per SIMD with the registers
// it wants.  Gridded media were once held to three waves despite ~120
// spilled VGPRs, while their node gathers mostly missed L2 (a third hit);
// with the primaries handed out by source and direction two thirds hit, and
// two waves without spills are faster.  EV: the instance also writes event
// records (launched only when the caller asks for them, so that the others
// carry none of that code).  The stratified kernel is in rt_strat.hip.
template <int MODEL, bool EV>
__global__ void __launch_bounds__(256) trace_general_kernel(KParams P) {
  trace_body<MODEL, 1, EV>(P);
}

// Record slots in use: [0, min(tail, capacity)).
__device__ __forceinline__ int64_t used_slots(const KParams& P) {
  const uint64_t tail = P.q->tail;
  return tail < (uint64_t)P.capacity ? (int64_t)tail : P.capacity;
}

// Queue counters and statistics to their launch values.
__global__ void reset_kernel(KParams P) {
  const int i = threadIdx.x;
  unsigned long long* s64 = reinterpret_cast<unsigned long long*>(P.stats);
  if (i < (int)(sizeof(rt_stats) / 8)) s64[i] = 0;
  if (i == 0) {
    P.q->head = 0;
    P.q->tail = (uint64_t)P.n_primary;
    P.q->gq_head = 0;
    P.q->gq_tail = 0;
    P.q->finished = 0;
    P.q->dropped = 0;
    P.q->fix_a = 0;
    P.q->fix_b = 0;
    P.q->steps = 0;
    P.q->stop = 0;
    P.q->holes = 0;
    P.q->ev_tail = 0;
  }
}

// Resuming an interrupted launch: the queue counters and statistics carry
// on; the overflow queue is rebuilt from the slots that hold rays still to
// trace (parked rays, and queued secondaries or primaries already handed
// out), so that no ray waits on a ticket or a ring that ended with the
// interrupted launch.  Fresh primaries stay with q->head.
__global__ void resume_reset_kernel(KParams P) {
  if (threadIdx.x == 0) {
    P.q->gq_head = 0;
    P.q->gq_tail = 0;
    P.q->fix_a = 0;
    P.q->fix_b = 0;
    P.q->holes = 0;
    P.q->steps = 0;
    P.q->stop = 0;
    P.stats->interrupted = 0;
  }
}

__global__ void resume_clear_kernel(KParams P) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s < P.capacity) P.gq[s] = -1;
}

__global__ void resume_queue_kernel(KParams P) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t M = used_slots(P);
  const uint64_t head = P.q->head;
  // slot s: a parked ray, or a queued secondary (after resume_fix_kernel
  // M is the number of occupied slots)
  bool pending = false;
  if (s < M) {
    const int32_t st = P.pool.status[s];
    pending = st == RT_ST_PARKED || (st == RT_ST_QUEUED && s >= P.n_primary);
  }
  if (__ballot(pending)) {
    if (pending) {
      const uint64_t e = wave_append(&P.q->gq_tail);
      if (e < (uint64_t)P.capacity) P.gq[e] = (int32_t)s;
    }
  }
  // ticket s: a primary handed out before the interruption and still queued
  int32_t slot = -1;
  if (s < P.n_primary && (uint64_t)s < head) {
    slot = P.perm[s];
    if (P.pool.status[slot] != RT_ST_QUEUED) slot = -1;
  }
  if (__ballot(slot >= 0)) {
    if (slot >= 0) {
      const uint64_t e = wave_append(&P.q->gq_tail);
      if (e < (uint64_t)P.capacity) P.gq[e] = slot;
    }
  }
}

// Slot compaction after a launch with chunked reservations, and before a
// resumed one: with M = min(tail, capacity) and H the empty slots among the
// secondaries in [n_primary, M) (holes left by chunks), every empty slot
// below N = M - H receives a record (finished, parked or queued) from a slot
// at or above N, so the occupied slots become [0, N).  The two lists live in
// the overflow queue, which is free at these points: holes at gq[0, ...),
// records to move at gq[capacity/2, ...); both hold at most
// min(N, capacity - N) <= capacity/2 entries.  Nothing refers to a slot
// index across these kernels (queued rays are found again by their status).
__global__ void compact_count_kernel(KParams P) {
  if (P.q->stop) return;  // interrupted: compacted when resumed
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool hole = s >= P.n_primary && s < used_slots(P) && P.pool.status[s] == RT_ST_EMPTY;
  const uint64_t m = __ballot(hole);
  if (m && (int)__lane_id() == __ffsll((unsigned long long)m) - 1)
    __hip_atomic_fetch_add(&P.q->holes, (uint64_t)__popcll(m), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void compact_scan_kernel(KParams P) {
  if (P.q->stop) return;
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t M = used_slots(P);
  const int64_t N = M - (int64_t)P.q->holes;
  const int32_t st = s < M ? P.pool.status[s] : RT_ST_EMPTY;
  const bool hole = s < M && s < N && st == RT_ST_EMPTY;
  const bool mover = s < M && s >= N && st != RT_ST_EMPTY;
  const uint64_t half = (uint64_t)P.capacity / 2;
  if (__ballot(hole)) {
    if (hole) {
      const uint64_t e = wave_append(&P.q->fix_a);
      if (e < half) P.gq[e] = (int32_t)s;
    }
  }
  if (__ballot(mover)) {
    if (mover) {
      const uint64_t e = wave_append(&P.q->fix_b);
      if (e < half) P.gq[half + e] = (int32_t)s;
    }
  }
}

__global__ void compact_move_kernel(KParams P) {
  if (P.q->stop) return;
  const int64_t half = P.capacity / 2;
  const int64_t n = min(min((int64_t)P.q->fix_a, (int64_t)P.q->fix_b), half);
  const Pool& Q = P.pool;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t d = P.gq[i], s = P.gq[half + i];
    double* const f64[] = {Q.x, Q.y, Q.z, Q.ux, Q.uy, Q.uz, Q.s, Q.t,
                           Q.as_re, Q.as_im, Q.ap_re, Q.ap_im, Q.h};
#pragma unroll
    for (int f = 0; f < 13; ++f) f64[f][d] = f64[f][s];
    Q.key[d] = Q.key[s];
    Q.parent[d] = Q.parent[s];
    int32_t* const i32[] = {Q.gen, Q.status, Q.n_acc, Q.n_rej, Q.n_ev, Q.region};
#pragma unroll
    for (int f = 0; f < 6; ++f) i32[f][d] = i32[f][s];
    Q.side[d] = Q.side[s];
    Q.status[s] = RT_ST_EMPTY;
  }
}

// After compacting for a resumed launch: the holes were counted as finished
// when their waves published them; both counts drop by the hole count.
__global__ void resume_fix_kernel(KParams P) {
  if (threadIdx.x == 0) {
    const uint64_t h = P.q->holes;
    P.q->tail -= h;
    P.q->finished -= h;
    P.q->holes = 0;
    P.q->fix_a = 0;
    P.q->fix_b = 0;
  }
}

// Records the launch needs: primaries + every secondary cast; when some
// found no slot, plus the slots chunks may leave unused, so that a relaunch
// with that capacity holds them all.
__global__ void finish_kernel(KParams P) {
  if (threadIdx.x == 0) {
    P.stats->needed = P.n_primary + P.stats->spawned + (P.q->dropped ? (int64_t)P.reserve : 0);
    P.stats->interrupted = P.q->stop ? 1 : 0;
    const uint64_t ev = P.q->ev_tail;
    P.stats->events_lost =
        ev > (uint64_t)P.ev_capacity ? (int64_t)(ev - (uint64_t)P.ev_capacity) : 0;
  }
}

// Hand-out order of the primaries: deepest sources first, and rays of one
// source by a Morton code of the direction's octahedral map (9 bits per
// axis), so that the lanes of a wave trace neighbouring directions.  In two
// steps: within each chunk of kOrderChunk consecutive rays, a bitonic sort of
// 64-bit keys (source depth descending, direction code, index) in LDS
// (128 KiB of the 160 KiB of a CU); then the full chunks are put in the
// order of their first keys (chunk_order_kernel, up to kOrderChunk chunks)
// and the permutation is applied (apply_order_kernel).  Deepest first
// measured 4-5 % faster than source-index order on the two-layer workload:
// the rays of the shallow sources, handed out last, leave a shorter tail of
// lone waves.  Only the order in which lanes take the rays changes: every
// ray keeps its record slot and its result.
constexpr int kOrderChunk = 16384;

// 32 high bits of a key that decreases with the depth z (IEEE order made
// monotone: sign flipped for z >= 0, all bits for z < 0; then complemented).
__device__ __forceinline__ uint32_t depth_key(double z) {
  const uint64_t b = (uint64_t)__double_as_longlong(z);
  const uint64_t up = (b >> 63) ? ~b : (b | 0x8000000000000000ull);
  return (uint32_t)(~up >> 32);
}

__device__ __forceinline__ uint32_t spread9(uint32_t v) {  // bits 0..8 -> even bits
  v &= 0x1ffu;
  v = (v | (v << 8)) & 0x00ff00ffu;
  v = (v | (v << 4)) & 0x0f0f0f0fu;
  v = (v | (v << 2)) & 0x33333333u;
  v = (v | (v << 1)) & 0x55555555u;
  return v;
}

__global__ void __launch_bounds__(1024) order_kernel(KParams P,
                                                     const double* __restrict__ src_xyz,
                                                     int32_t n_src,
                                                     const double* __restrict__ dir_xyz,
                                                     const int32_t* __restrict__ ray_src,
                                                     int32_t* __restrict__ perm0,
                                                     uint64_t* __restrict__ chunk_key) {
  __shared__ unsigned long long key[kOrderChunk];
  const int64_t base = (int64_t)blockIdx.x * kOrderChunk;
  const int n = (int)min((int64_t)kOrderChunk, P.n_primary - base);
  for (int j = threadIdx.x; j < kOrderChunk; j += blockDim.x) {
    unsigned long long k = ~0ull;
    if (j < n) {
      const int64_t i = base + j;
      const double dx = dir_xyz[3 * i], dy = dir_xyz[3 * i + 1], dz = dir_xyz[3 * i + 2];
      const double l1 = fabs(dx) + fabs(dy) + fabs(dz);
      double ox = 0.0, oy = 0.0;
      if (l1 > 0.0 && isfinite(l1)) {
        ox = dx / l1;
        oy = dy / l1;
        if (dz < 0.0) {  // fold the lower hemisphere onto the corners
          const double fx = (1.0 - fabs(oy)) * copysign(1.0, ox);
          oy = (1.0 - fabs(ox)) * copysign(1.0, oy);
          ox = fx;
        }
      }
      const uint32_t ix = min(511u, (uint32_t)((ox + 1.0) * 256.0));
      const uint32_t iy = min(511u, (uint32_t)((oy + 1.0) * 256.0));
      const uint32_t code = spread9(ix) | (spread9(iy) << 1);
      const int32_t s = ray_src[i];  // a ray of no valid source is invalid: any place
      const uint32_t dk = (s >= 0 && s < n_src) ? depth_key(src_xyz[3 * (int64_t)s + 2]) : 0u;
      k = ((unsigned long long)dk << 32) | ((unsigned long long)code << 14) |
          (unsigned long long)j;
    }
    key[j] = k;
  }
  __syncthreads();
  for (int size = 2; size <= kOrderChunk; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = threadIdx.x; t < kOrderChunk; t += blockDim.x) {
        const int u = t ^ stride;
        if (u > t) {
          const unsigned long long a = key[t], b = key[u];
          if ((a > b) == ((t & size) == 0)) {
            key[t] = b;
            key[u] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int j = threadIdx.x; j < n; j += blockDim.x)
    perm0[base + j] = (int32_t)(base + (int64_t)(key[j] & 0x3fffu));
  if (threadIdx.x == 0)
    chunk_key[blockIdx.x] = (key[0] & 0xffffffff00000000ull) | (unsigned long long)blockIdx.x;
}

// The full chunks in the order of their first keys (one block; keys padded
// to a power of two): chunk_key[c] = the c-th chunk to hand out.
__global__ void __launch_bounds__(1024) chunk_order_kernel(uint64_t* __restrict__ chunk_key,
                                                           int n_full) {
  __shared__ unsigned long long key[kOrderChunk];
  int np = 1;
  while (np < n_full) np <<= 1;
  for (int j = threadIdx.x; j < np; j += blockDim.x) key[j] = j < n_full ? chunk_key[j] : ~0ull;
  __syncthreads();
  for (int size = 2; size <= np; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = threadIdx.x; t < np; t += blockDim.x) {
        const int u = t ^ stride;
        if (u > t) {
          const unsigned long long a = key[t], b = key[u];
          if ((a > b) == ((t & size) == 0)) {
            key[t] = b;
            key[u] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int j = threadIdx.x; j < n_full; j += blockDim.x) chunk_key[j] = key[j];
}

// Ticket t -> slot: the (t / kOrderChunk)-th chunk of the chunk order, at
// its (t % kOrderChunk)-th sorted position; a partial last chunk stays last.
__global__ void apply_order_kernel(KParams P, const int32_t* __restrict__ perm0,
                                   const uint64_t* __restrict__ chunk_key, int n_full) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= P.n_primary) return;
  const int64_t c = t / kOrderChunk;
  const int64_t src = c < n_full
                          ? (int64_t)(chunk_key[c] & 0xffffffffull) * kOrderChunk + t % kOrderChunk
                          : t;
  P.perm[t] = perm0[src];
}

// FP32 grid -> float4 nodes (n, Dx, Dy, Dz): D is the central difference of
// the neighbours, or twice the one-sided difference at an edge, so that
// grad n = D / (2 spacing) everywhere.  The FP32 differences are exact for
// values within a factor of two of each other (Sterbenz).
__global__ void grid_prep_kernel(const float* __restrict__ n, float4* __restrict__ out, int nx,
                                 int ny, int nz, int bx, int by) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)nx * ny * nz;
  if (id >= total) return;
  const int i = (int)(id % nx);
  const int j = (int)((id / nx) % ny);
  const int k = (int)(id / ((int64_t)nx * ny));
  const int64_t sy = nx, sz = (int64_t)nx * ny;
  const float c = n[id];
  float dx, dy, dz;
  if (i == 0) dx = 2.0f * (n[id + 1] - c);
  else if (i == nx - 1) dx = 2.0f * (c - n[id - 1]);
  else dx = n[id + 1] - n[id - 1];
  if (j == 0) dy = 2.0f * (n[id + sy] - c);
  else if (j == ny - 1) dy = 2.0f * (c - n[id - sy]);
  else dy = n[id + sy] - n[id - sy];
  if (k == 0) dz = 2.0f * (n[id + sz] - c);
  else if (k == nz - 1) dz = 2.0f * (c - n[id - sz]);
  else dz = n[id + sz] - n[id - sz];
  out[node_index(i, j, k, bx, by)] = make_float4(c, dx, dy, dz);
}

// ---------------------------------------------------------------------------
// Primary rays into the record slots; empty status for the rest.
__global__ void init_kernel(KParams P, const double* __restrict__ src_xyz, int32_t n_src,
                            const double* __restrict__ dir_xyz, const int32_t* __restrict__ ray_src,
                            double h0) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const Pool& Q = P.pool;
  if (i >= P.capacity) return;
  P.gq[i] = -1;
  if (i >= P.n_primary) {
    Q.status[i] = RT_ST_EMPTY;
    return;
  }
  const int32_t sidx = ray_src[i];
  bool ok = sidx >= 0 && sidx < n_src;
  double r[3] = {0.0, 0.0, 0.0}, d[3];
  for (int a = 0; a < 3; ++a) {
    d[a] = dir_xyz[3 * i + a];
    if (ok) r[a] = src_xyz[3 * sidx + a];
  }
  const double d2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
  ok = ok && isfinite(d2) && d2 > 0.0 && isfinite(r[0]) && isfinite(r[1]) && isfinite(r[2]);
  uint32_t side = 0;
  int32_t region = 0;
  for (int g = P.n_regions - 1; g >= 0; --g)  // first region containing the depth
    if (r[2] >= P.reg[g].z_top && r[2] < P.reg[g].z_bot) region = g;
  for (int k = 0; k < P.n_bnd; ++k) {
    const KBnd& B = P.bnd[k];
    if (B.kind == B_TIME) continue;
    const double g = bnd_value(B, r);
    if (B.kind == B_BOX) ok = ok && g > 0.0;
    else ok = ok && fabs(g) > 1e-9;
    if (g > 0.0) side |= 1u << k;
  }
  Q.x[i] = r[0];
  Q.y[i] = r[1];
  Q.z[i] = r[2];
  Q.ux[i] = d[0];
  Q.uy[i] = d[1];
  Q.uz[i] = d[2];
  Q.s[i] = 0.0;
  Q.t[i] = 0.0;
  Q.h[i] = h0;
  Q.as_re[i] = 1.0;
  Q.as_im[i] = 0.0;
  Q.ap_re[i] = 1.0;
  Q.ap_im[i] = 0.0;
  Q.key[i] = (uint64_t)i << 24;
  Q.parent[i] = ~(uint64_t)0;
  Q.gen[i] = 0;
  Q.region[i] = region;
  Q.side[i] = side;
  Q.n_acc[i] = 0;
  Q.n_rej[i] = 0;
  Q.n_ev[i] = 0;
  Q.status[i] = ok ? RT_ST_QUEUED : RT_ST_INVALID;
  if (!ok) atomicAdd(reinterpret_cast<unsigned long long*>(&P.stats->invalid), 1ull);
}


// ===========================================================================
// Host launcher.
namespace {

struct DeviceInfo {
  int device = -1;
  int n_cu = 0;
};
thread_local DeviceInfo g_dev;

// Kinds of launch: 0 stratified, 1 general analytic, 2 gridded (both on the
// general kernel); plus 3 for the instances that write event records.
template <int MODEL, int KIND>
void* trace_kernel_ptr() {
  constexpr bool EV = KIND >= 3;
  return reinterpret_cast<void*>(&trace_general_kernel<MODEL, EV>);
}

template <int MODEL, int FIELD>
int max_blocks_per_cu(int block) {
  if constexpr (FIELD % 3 == 0) return strat_blocks_per_cu(MODEL, FIELD >= 3, block);
  static thread_local int cached[5] = {};
  int& c = cached[block / 64];
  if (c == 0) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, trace_kernel_ptr<MODEL, FIELD>(), block,
                                                     0) != hipSuccess ||
        nb < 1)
      nb = 1;
    c = nb;
  }
  return c;
}

template <int MODEL, int KIND>
hipError_t launch_trace(const KParams& P, int grid, int block, hipStream_t s) {
  constexpr bool EV = KIND >= 3;
  if constexpr (KIND % 3 != 0) {
    hipLaunchKernelGGL((trace_general_kernel<MODEL, EV>), dim3(grid), dim3(block), 0, s, P);
    return hipGetLastError();
  } else {
    return launch_strat(MODEL, EV, P, grid, block, s);
  }
}

template <int MODEL>
int blocks_per_cu(int kind, int block) {
  switch (kind) {
    case 5: return max_blocks_per_cu<MODEL, 5>(block);
    case 4: return max_blocks_per_cu<MODEL, 4>(block);
    case 3: return max_blocks_per_cu<MODEL, 3>(block);
    case 2: return max_blocks_per_cu<MODEL, 2>(block);
    case 1: return max_blocks_per_cu<MODEL, 1>(block);
    default: return max_blocks_per_cu<MODEL, 0>(block);
  }
}

template <int MODEL>
hipError_t launch_kind(int kind, const KParams& P, int grid, int block, hipStream_t s) {
  switch (kind) {
    case 5: return launch_trace<MODEL, 5>(P, grid, block, s);
    case 4: return launch_trace<MODEL, 4>(P, grid, block, s);
    case 3: return launch_trace<MODEL, 3>(P, grid, block, s);
    case 2: return launch_trace<MODEL, 2>(P, grid, block, s);
    case 1: return launch_trace<MODEL, 1>(P, grid, block, s);
    default: return launch_trace<MODEL, 0>(P, grid, block, s);
  }
}

hipError_t launch_compaction(const KParams& P, unsigned cap_blocks, hipStream_t s) {
  hipLaunchKernelGGL(compact_count_kernel, dim3(cap_blocks), dim3(256), 0, s, P);
  hipLaunchKernelGGL(compact_scan_kernel, dim3(cap_blocks), dim3(256), 0, s, P);
  hipLaunchKernelGGL(compact_move_kernel, dim3(std::min(cap_blocks, 1024u)), dim3(256), 0, s, P);
  return hipGetLastError();
}

}  // namespace
}  // namespace rt

#define HIP_TRY(expr)                                                         \
  do {                                                                        \
    hipError_t e_ = (expr);                                                   \
    if (e_ != hipSuccess) {                                                   \
      rt::set_last_error("%s: %s", #expr, hipGetErrorString(e_));             \
      return RT_ERR_DEVICE;                                                   \
    }                                                                         \
  } while (0)

namespace rt {
namespace {

// Body of raytrace_launch and raytrace_launch_static: everything after the
// caller's scratch memory has been chosen.
rt_status launch_trace(const rt_field* field, const rt_boundaries* bnd, const rt_sources* src,
                       const rt_directions* dirs, double tol, const rt_step_limits* L,
                       rt_outputs* out, void* workspace, size_t workspace_bytes, void* stream,
                       const rt_tuning* tuning) {
  rt_status st = validate(field, bnd, src, dirs, tol, L);
  if (st != RT_OK) return st;
  if (!out || !out->stats || !workspace) {
    set_last_error("null outputs, stats or workspace");
    return RT_ERR_INVALID_ARG;
  }
  const double* const* f64[] = {&out->x, &out->y, &out->z, &out->ux, &out->uy, &out->uz, &out->s,
                                &out->t, &out->as_re, &out->as_im, &out->ap_re, &out->ap_im,
                                &out->h};
  for (auto p : f64)
    if (!*p) {
      set_last_error("null output array");
      return RT_ERR_INVALID_ARG;
    }
  if (!out->key || !out->parent || !out->gen || !out->status || !out->n_acc || !out->n_rej ||
      !out->n_ev || !out->region || !out->side) {
    set_last_error("null output array");
    return RT_ERR_INVALID_ARG;
  }
  if (out->capacity < dirs->n || out->capacity > (int64_t)0x7fffffff) {
    set_last_error("capacity must be >= number of rays and < 2^31");
    return RT_ERR_INVALID_ARG;
  }
  if (out->ev_capacity < 0 || (out->ev_capacity > 0 && !out->events)) {
    set_last_error("ev_capacity must be >= 0, with an events array when > 0");
    return RT_ERR_INVALID_ARG;
  }
  size_t need = 0;
  st = rt_workspace_bytes(field, out->capacity, &need);
  if (st != RT_OK) return st;
  if (workspace_bytes < need) {
    set_last_error("workspace of %zu bytes < %zu needed", workspace_bytes, need);
    return RT_ERR_INVALID_ARG;
  }
  const int block = tuning && tuning->block_size ? tuning->block_size : 256;
  if (block < 64 || block > 256 || block % 64) {
    set_last_error("block_size must be 64, 128, 192 or 256");
    return RT_ERR_INVALID_ARG;
  }
  // default refill threshold: 32 idle lanes, 48 for gridded media (whose
  // trial waits on node gathers: fewer, larger refills measured 2 % faster)
  const int refill = tuning && tuning->refill_threshold ? tuning->refill_threshold
                     : field_uses_grid(field)             ? 48
                                                          : 32;
  if (refill < 1 || refill > 64) {
    set_last_error("refill_threshold must be 1..64");
    return RT_ERR_INVALID_ARG;
  }
  int local = tuning && tuning->local_queue ? tuning->local_queue : 256;
  if (local == -1) local = 0;
  if (local < 0 || local > (int)kRing) {
    set_last_error("local_queue must be -1, 0 or 1..%d", (int)kRing);
    return RT_ERR_INVALID_ARG;
  }

  KParams P;
  memset(&P, 0, sizeof P);
  P.n_regions = field->n_regions;
  for (int i = 0; i < field->n_regions; ++i) {
    const rt_region& r = field->regions[i];
    KRegion& k = P.reg[i];
    k.a = r.a;
    k.b = r.b;
    k.dn = r.dn;
    k.inv_z0 = r.dn != 0.0 ? 1.0 / r.z0 : 0.0;
    k.dn_inv_z0 = r.dn != 0.0 ? r.dn / r.z0 : 0.0;
    k.z_top = r.z_top;
    k.z_bot = r.z_bot;
    k.use_grid = r.use_grid ? 1 : 0;
    const double len = sqrt(r.axis[0] * r.axis[0] + r.axis[1] * r.axis[1] +
                            r.axis[2] * r.axis[2]);
    for (int a = 0; a < 3; ++a) k.ax[a] = len > 0.0 ? r.axis[a] / len : (a == 2 ? 1.0 : 0.0);
  }
  P.n_anom = field->n_anomalies;
  for (int j = 0; j < field->n_anomalies; ++j) {
    const rt_anomaly& q = field->anomalies[j];
    KAnom& A = P.anom[j];
    for (int a = 0; a < 3; ++a) A.c[a] = q.centre[a];
    A.amp = q.amplitude;
    A.k = 1.0 / (2.0 * q.sigma * q.sigma);
    A.region = q.region;
  }
  int nb = 0;
  for (int i = 0; i < bnd->n_planes; ++i) {
    const rt_plane& p = bnd->planes[i];
    KBnd& b = P.bnd[nb++];
    b.shape = p.shape;
    if (p.shape == RT_SHAPE_PLANE) {
      const double len = sqrt(p.normal[0] * p.normal[0] + p.normal[1] * p.normal[1] +
                              p.normal[2] * p.normal[2]);
      for (int a = 0; a < 3; ++a) b.nrm[a] = p.normal[a] / len;
      b.d = p.point[0] * b.nrm[0] + p.point[1] * b.nrm[1] + p.point[2] * b.nrm[2];
    } else {  // centre or vertex, radius or curvature
      for (int a = 0; a < 3; ++a) b.nrm[a] = p.point[a];
      b.d = p.param;
    }
    b.kind = p.kind == RT_PLANE_ABSORB ? B_ABSORB : B_FRESNEL;
    b.reg_pos = p.region_pos;
    b.reg_neg = p.region_neg;
  }
  if (bnd->has_box) {
    for (int a = 0; a < 3; ++a)
      for (int hi = 0; hi < 2; ++hi) {
        KBnd& b = P.bnd[nb++];
        b.nrm[a] = hi ? -1.0 : 1.0;  // inside of the box is g > 0
        b.d = hi ? -bnd->box_hi[a] : bnd->box_lo[a];
        b.kind = B_BOX;
        b.reg_pos = b.reg_neg = -1;
      }
  }
  if (L->t_max > 0.0) P.bnd[nb++].kind = B_TIME;
  P.n_bnd = nb;
  P.model = L->model;
  P.max_gen = L->max_generations;
  P.refill = refill;
  P.local_limit = (uint32_t)local;
  P.tol = tol;
  P.inv_tol = 1.0 / tol;
  P.h_min = L->h_min;
  P.h_max = L->h_max;
  P.h_init = L->h_init > 0.0 ? L->h_init : L->h_max;
  P.s_max = L->s_max;
  P.t_max = L->t_max;
  P.amp_min = L->amp_min;
  P.max_steps = L->max_steps_per_ray;
  P.budget = L->max_steps_per_launch;
  P.pool = Pool{out->x,     out->y,     out->z,     out->ux,    out->uy,    out->uz,
                out->s,     out->t,     out->as_re, out->as_im, out->ap_re, out->ap_im,
                out->h,     out->key,   out->parent, out->gen,  out->status, out->n_acc,
                out->n_rej, out->n_ev,  out->region, out->side};
  P.capacity = out->capacity;
  P.n_primary = dirs->n;
  P.events = out->events;
  P.ev_capacity = out->ev_capacity;
  P.q = static_cast<QueueCounters*>(workspace);
  P.gq = reinterpret_cast<int32_t*>(static_cast<char*>(workspace) + 4096);
  const size_t gq_bytes = ((size_t)out->capacity * 4 + 4095) / 4096 * 4096;
  P.perm = reinterpret_cast<int32_t*>(static_cast<char*>(workspace) + 4096 + gq_bytes);
  // per-chunk sorted order and the chunks' keys (order_kernel)
  int32_t* perm0 = reinterpret_cast<int32_t*>(static_cast<char*>(workspace) + 4096 + 2 * gq_bytes);
  uint64_t* chunk_key =
      reinterpret_cast<uint64_t*>(static_cast<char*>(workspace) + 4096 + 3 * gq_bytes);
  const size_t ck_bytes = ((size_t)(out->capacity / kOrderChunk + 1) * 8 + 4095) / 4096 * 4096;
  P.stats = out->stats;
  const bool has_grid = field_uses_grid(field);
  const int kind = (has_grid ? 2 : field_is_general(field) ? 1 : 0) + (P.ev_capacity > 0 ? 3 : 0);
  if (has_grid) {
    const rt_grid& g = field->grid;
    P.nodes = static_cast<char*>(workspace) + 4096 + 3 * gq_bytes + ck_bytes;
    P.gnx = g.nx;
    P.gny = g.ny;
    P.gnz = g.nz;
    P.gbx = (g.nx + 1) / 2;
    P.gby = (g.ny + 1) / 2;
    P.gbz = (g.nz + 1) / 2;
    const int dims[3] = {g.nx, g.ny, g.nz};
    for (int a = 0; a < 3; ++a) {
      P.gorg[a] = g.origin[a];
      P.ginv[a] = 1.0 / g.spacing[a];
      P.gmax[a] = (double)(dims[a] - 1);
      P.ghalf[a] = 1.0 / (2.0 * g.spacing[a]);
    }
  }

  hipStream_t s = static_cast<hipStream_t>(stream);
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (g_dev.device != dev) {
    int ncu = 0;
    HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    g_dev.device = dev;
    g_dev.n_cu = ncu;
  }

  const unsigned cap_blocks = (unsigned)((out->capacity + 255) / 256);
  std::optional<Range> range;  // the enqueue phases, for a profiler's timeline
  range.emplace("raytrace_launch: reset, init, order");
  if (L->resume) {
    hipLaunchKernelGGL(resume_reset_kernel, dim3(1), dim3(64), 0, s, P);
    HIP_TRY(hipGetLastError());
    if (out->capacity > 0) {
      HIP_TRY(launch_compaction(P, cap_blocks, s));
      hipLaunchKernelGGL(resume_fix_kernel, dim3(1), dim3(64), 0, s, P);
      HIP_TRY(hipGetLastError());
      hipLaunchKernelGGL(resume_clear_kernel, dim3(cap_blocks), dim3(256), 0, s, P);
      HIP_TRY(hipGetLastError());
      hipLaunchKernelGGL(resume_queue_kernel, dim3(cap_blocks), dim3(256), 0, s, P);
      HIP_TRY(hipGetLastError());
    }
  } else {
    hipLaunchKernelGGL(reset_kernel, dim3(1), dim3(64), 0, s, P);
    HIP_TRY(hipGetLastError());
  }
  if (has_grid) {
    const int64_t total = (int64_t)field->grid.nx * field->grid.ny * field->grid.nz;
    hipLaunchKernelGGL(grid_prep_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                       field->grid.n, static_cast<float4*>(const_cast<void*>(P.nodes)),
                       field->grid.nx, field->grid.ny, field->grid.nz, P.gbx, P.gby);
    HIP_TRY(hipGetLastError());
  }
  if (out->capacity > 0 && !L->resume) {
    hipLaunchKernelGGL(init_kernel, dim3((unsigned)((out->capacity + 255) / 256)), dim3(256), 0,
                       s, P, src->xyz, src->n, dirs->xyz, dirs->src, P.h_init);
    HIP_TRY(hipGetLastError());
  }
  if (dirs->n > 0 && !L->resume) {  // a resumed launch keeps the order it had
    const int64_t chunks = (dirs->n + kOrderChunk - 1) / kOrderChunk;
    hipLaunchKernelGGL(order_kernel, dim3((unsigned)chunks), dim3(1024), 0, s, P, src->xyz,
                       src->n, dirs->xyz, dirs->src, perm0, chunk_key);
    HIP_TRY(hipGetLastError());
    int n_full = (int)(dirs->n / kOrderChunk);
    if (n_full > kOrderChunk) n_full = 0;  // beyond one block's sort: chunks in input order
    if (n_full >= 2) {
      hipLaunchKernelGGL(chunk_order_kernel, dim3(1), dim3(1024), 0, s, chunk_key, n_full);
      HIP_TRY(hipGetLastError());
    } else {
      n_full = 0;
    }
    hipLaunchKernelGGL(apply_order_kernel, dim3((unsigned)((dirs->n + 255) / 256)), dim3(256), 0,
                       s, P, perm0, chunk_key, n_full);
    HIP_TRY(hipGetLastError());
  }


  // persistent grid: every CU filled to its occupancy, fewer blocks for
  // small launches
  int bpc = 0;
  if (L->model == RT_MODEL_PAPER)
    bpc = blocks_per_cu<RT_MODEL_PAPER>(kind, block);
  else
    bpc = blocks_per_cu<RT_MODEL_EXACT>(kind, block);
  if (tuning && tuning->blocks_per_cu > 0) bpc = std::min(bpc, (int)tuning->blocks_per_cu);
  int64_t nblk = (int64_t)g_dev.n_cu * bpc;
  const int64_t by_rays = std::max<int64_t>(1, (dirs->n + block - 1) / block);
  nblk = std::max<int64_t>(1, std::min(nblk, by_rays));
  // chunked secondary slots when the capacity leaves room for the chunks'
  // unused rests (at most one chunk per wave) and for the compaction lists
  const int64_t waves = nblk * (block / 64);
  const int64_t reserve = waves * kChunk;
  const bool chunked = L->max_generations > 1 && out->capacity >= dirs->n + 4 * reserve;
  P.chunk = chunked ? (uint32_t)kChunk : 0u;
  P.chunk_limit = chunked ? (uint64_t)(out->capacity - reserve) : 0;
  P.reserve = chunked ? (uint64_t)reserve : 0;

  range.reset();
  range.emplace("raytrace_launch: trace, compaction");
  if (tuning && tuning->ev_trace_begin)
    HIP_TRY(hipEventRecord(static_cast<hipEvent_t>(tuning->ev_trace_begin), s));
  hipError_t e;
  if (L->model == RT_MODEL_PAPER)
    e = launch_kind<RT_MODEL_PAPER>(kind, P, (int)nblk, block, s);
  else
    e = launch_kind<RT_MODEL_EXACT>(kind, P, (int)nblk, block, s);
  HIP_TRY(e);
  if (tuning && tuning->ev_trace_end)
    HIP_TRY(hipEventRecord(static_cast<hipEvent_t>(tuning->ev_trace_end), s));
  if (chunked && out->capacity > 0) HIP_TRY(launch_compaction(P, cap_blocks, s));
  hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(64), 0, s, P);
  HIP_TRY(hipGetLastError());
  return RT_OK;
}

// Scratch memory of raytrace_launch_static, a file-scope device array: every
// GPU the library runs on holds its own copy, at its own address, until the
// process ends.  In host code 'scratch' names a host-side stand-in, never the
// device memory: the device address comes from hipGetSymbolAddress, taken
// once per device with that device current.
__device__ __align__(256) unsigned char scratch[RT_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

rt_status static_scratch(void** ptr) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_last_error("device %d beyond the %d devices the static scratch supports", dev,
                   kMaxDevices);
    return RT_ERR_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) {
      set_last_error("hipGetSymbolAddress returned no address for the static scratch");
      return RT_ERR_DEVICE;
    }
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  return RT_OK;
}

}  // namespace
}  // namespace rt

extern "C" rt_status raytrace_launch(const rt_field* field, const rt_boundaries* bnd,
                                     const rt_sources* src, const rt_directions* dirs, double tol,
                                     const rt_step_limits* L, rt_outputs* out, void* workspace,
                                     size_t workspace_bytes, void* stream,
                                     const rt_tuning* tuning) {
  return rt::launch_trace(field, bnd, src, dirs, tol, L, out, workspace, workspace_bytes, stream,
                          tuning);
}

extern "C" rt_status raytrace_launch_static(const rt_field* field, const rt_boundaries* bnd,
                                            const rt_sources* src, const rt_directions* dirs,
                                            double tol, const rt_step_limits* L,
                                            rt_outputs* out, void* stream,
                                            const rt_tuning* tuning) {
  using namespace rt;
  rt_status st = validate(field, bnd, src, dirs, tol, L);
  if (st != RT_OK) return st;
  if (!out) {
    set_last_error("null outputs");
    return RT_ERR_INVALID_ARG;
  }
  size_t need = 0;
  st = rt_workspace_bytes(field, out->capacity, &need);
  if (st != RT_OK) return st;
  if (need > (size_t)RT_STATIC_SCRATCH_BYTES) {
    set_last_error("launch needs %zu bytes of scratch; the static scratch holds %zu "
                   "(use raytrace_launch with a workspace)",
                   need, (size_t)RT_STATIC_SCRATCH_BYTES);
    return RT_ERR_UNSUPPORTED;
  }
  void* ws = nullptr;
  st = static_scratch(&ws);
  if (st != RT_OK) return st;
  return launch_trace(field, bnd, src, dirs, tol, L, out, ws, need, stream, tuning);
}
