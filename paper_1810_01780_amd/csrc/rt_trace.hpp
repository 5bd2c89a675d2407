// The persistent trace: scheduler, per-lane ray state, boundary events and
// the loop that runs one Cash-Karp trial per busy lane and iteration
// (trace_body), shared by the stratified kernel (rt_strat.hip) and the
// general 3-D kernel (rt_kernels.hip), which are compiled apart.
//
// Method: RadioPropa (arXiv:1810.01780) section 2 -- the ray equation (eq. 2,
// locally paraxial; or eq. 1, full eikonal) integrated by the Cash-Karp
// embedded Runge-Kutta 4(5) pair with adaptive steps, and boundary surfaces
// (planes, spheres, paraboloids) handled apart from the propagation: the ray
// reflects and a refracted secondary is cast from the crossing point, with
// Fresnel amplitudes.
//
// Execution model: one ray per lane, state in registers.  A persistent grid
// of waves pulls rays from a queue whose slots are the caller's output
// records; secondaries are appended to the same queue.  Every loop iteration
// runs exactly one Cash-Karp trial step in every busy lane -- a normal step,
// or one iterate of the crossing search -- so the expensive arithmetic never
// diverges; only the cheap bookkeeping after the trial does.  A launch can
// stop at a step budget, parking its rays in their slots for a resumed one.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "rt_device.hpp"

namespace rt {

// Per-wave statistics of the trace kernel, indexed like the fields of
// rt_stats.
enum : int {
  S_ACC = 0, S_REJ, S_RELOC, S_FORCED, S_EVENTS, S_SPAWNED, S_SUPP_GEN, S_SUPP_AMP,
  S_RECORDS, S_NEEDED, S_NONFINITE, S_MAXGEN, S_INVALID, S_REFILLS, S_SCHED, S_SPILLED,
  S_FIN,   // rays finished here and not yet added to q->finished (not a stat)
  S_MAXQ,  // largest backlog on this wave's ring (rt_stats.max_queue)
  S_COUNT
};

// Secondaries stay with the wave that cast them: a ring of record-slot
// indices per wave in LDS.  Producer and consumer are the same wave, so a
// workgroup-scope fence orders the child's record stores before the lane
// that later takes the child reads them; no cross-CU coherence is needed
// (the L2s of the eight XCDs are not coherent with each other, and
// publishing through them would mean L2 write-backs).
constexpr uint32_t kRing = 1024;  // LDS ring entries per wave (>= any local limit)
constexpr int64_t kChunk = 64;    // secondary record slots a wave reserves at once
// Batching of boundary events in the stratified kernel (see trace_body):
// 6 lanes, 16 iterations, event-dense below 16 trials between events
// (measured on the two-layer workload: 13 % faster; the curved workload,
// whose trapped rays meet events every few trials, unchanged).
constexpr uint32_t kEvBatch = 6, kEvWait = 16;
constexpr int32_t kEvDense = 16;
struct WaveQueue {
  int32_t* ring;   // kRing slot indices
  uint32_t* head;  // next index to take
  uint32_t* tail;  // next index to fill
};

// Per-lane ray data that boundary events read and update, kept in LDS (one
// entry per thread) instead of being re-read from the record pool: the
// Fresnel amplitudes and the ray key.  An event then issues no global load
// whose completion it would wait for; the pool receives the amplitudes when
// the record is written.
__shared__ double s_as_re[256], s_as_im[256], s_ap_re[256], s_ap_im[256];
__shared__ uint64_t s_key[256];
// Accepted and rejected steps of the rays each lane has finished: the
// launch totals are the sums of the records' step counts, so the step loop
// keeps no counters of its own.
__shared__ unsigned long long s_nacc[256], s_nrej[256];

// Record slots of secondaries.  A wave reserves slots in chunks of P.chunk
// consecutive indices (one atomic per chunk rather than per spawning
// iteration: a single counter bumped by every wave is a contended address),
// which also keeps each wave's children in cache lines of their own.  The
// unused rest of a wave's chunk is published as finished while the wave is
// idle, so that finished == tail still means that no ray is running; the
// wave takes that count back before it hands out such a slot.  Slots left
// unused at the end are filled by moving the last records into them
// (compact_*_kernel), so the records stay dense.  Near the capacity waves
// switch to one reservation per child.
__shared__ unsigned long long s_cnext[4], s_cend[4];
__shared__ uint32_t s_cphant[4], s_cmode[4];

__device__ __forceinline__ uint64_t wave_slot(const KParams& P, int wv) {
  const uint64_t m = __ballot(1);
  const int leader = __ffsll((unsigned long long)m) - 1;
  const uint32_t cnt = (uint32_t)__popcll(m);
  const uint32_t rank = (uint32_t)__popcll(m & lanemask_lt());
  unsigned long long b1 = 0, b2 = 0, t1 = 0;
  if ((int)__lane_id() == leader) {
    unsigned long long nx = s_cnext[wv], en = s_cend[wv];
    t1 = min((unsigned long long)cnt, en - nx);
    b1 = nx;
    nx += t1;
    const uint32_t rest = cnt - (uint32_t)t1;
    if (rest > 0) {
      if (s_cmode[wv]) {  // a fresh chunk (P.chunk >= 64 covers any rest)
        const uint64_t b = __hip_atomic_fetch_add(&P.q->tail, (uint64_t)P.chunk, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
        b2 = b;
        nx = b + rest;
        en = b + P.chunk;
        if (b + 2 * (uint64_t)P.chunk > P.chunk_limit) s_cmode[wv] = 0;
      } else {
        b2 = __hip_atomic_fetch_add(&P.q->tail, (uint64_t)rest, __ATOMIC_RELAXED,
                                    __HIP_MEMORY_SCOPE_AGENT);
        nx = en = 0;
      }
    }
    s_cnext[wv] = nx;
    s_cend[wv] = en;
    // slots published as finished by an idle phase are running rays now
    const uint32_t unused = (uint32_t)(en - nx);
    if (s_cphant[wv] > unused) {
      __hip_atomic_fetch_add(&P.q->finished, (uint64_t)unused - s_cphant[wv], __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
      s_cphant[wv] = unused;
    }
  }
  b1 = __shfl(b1, leader);
  b2 = __shfl(b2, leader);
  t1 = __shfl(t1, leader);
  return rank < t1 ? b1 + rank : b2 + (rank - t1);
}

// Event-record array and its capacity, copied into LDS at kernel start.
__shared__ rt_event* s_ev_base;
__shared__ unsigned long long s_ev_cap;

// Reserve consecutive entries of a counter for the calling wave's active
// lanes (one atomic per wave); returns this lane's index.
__device__ __forceinline__ uint64_t wave_append(uint64_t* tail) {
  const uint64_t m = __ballot(1);
  const int leader = __ffsll((unsigned long long)m) - 1;
  unsigned long long base = 0;
  if ((int)__lane_id() == leader)
    base = __hip_atomic_fetch_add(tail, (uint64_t)__popcll(m), __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
  base = __shfl(base, leader);
  return base + (uint64_t)__popcll(m & lanemask_lt());
}

__device__ __forceinline__ void write_record(const KParams& P, const Ray& R, int32_t status,
                                             const Counters& C) {
  const Pool& Q = P.pool;
  const int i = R.slot;
  const double il = rsqrt_nr(fma(R.y[3], R.y[3], fma(R.y[4], R.y[4], R.y[5] * R.y[5])));
  Q.x[i] = R.y[0];
  Q.y[i] = R.y[1];
  Q.z[i] = R.y[2];
  Q.ux[i] = R.y[3] * il;
  Q.uy[i] = R.y[4] * il;
  Q.uz[i] = R.y[5] * il;
  Q.s[i] = R.s;
  Q.t[i] = R.y[6];
  Q.h[i] = R.h;
  const int t = (int)threadIdx.x;
  s_nacc[t] += (unsigned long long)R.n_acc;
  s_nrej[t] += (unsigned long long)R.n_rej;
  Q.as_re[i] = s_as_re[t];
  Q.as_im[i] = s_as_im[t];
  Q.ap_re[i] = s_ap_re[t];
  Q.ap_im[i] = s_ap_im[t];
  Q.n_acc[i] = R.n_acc;
  Q.n_rej[i] = R.n_rej;
  Q.n_ev[i] = R.n_ev;
  Q.region[i] = R.region;
  Q.side[i] = R.side;
  Q.status[i] = status;
  C.bump(S_RECORDS);
  C.bump(S_FIN);
}

// Load the queued ray of a slot into a lane.
template <int MODEL, int FIELD>
__device__ __forceinline__ void load_ray(const KParams& P, int32_t slot, Ray& R, const Counters& C) {
  const Pool& Q = P.pool;
  R.slot = slot;
  R.y[0] = Q.x[slot];
  R.y[1] = Q.y[slot];
  R.y[2] = Q.z[slot];
  R.y[6] = Q.t[slot];
  R.s = Q.s[slot];
  R.h = Q.h[slot];
  R.gen = Q.gen[slot];
  R.region = Q.region[slot];
  R.side = Q.side[slot];
  R.n_acc = Q.n_acc[slot];
  R.n_rej = Q.n_rej[slot];
  R.n_ev = Q.n_ev[slot];
  const int t = (int)threadIdx.x;
  s_as_re[t] = Q.as_re[slot];
  s_as_im[t] = Q.as_im[slot];
  s_ap_re[t] = Q.ap_re[slot];
  s_ap_im[t] = Q.ap_im[slot];
  s_key[t] = Q.key[slot];
  if (Q.status[slot] == RT_ST_PARKED) {  // the exact direction state it had
    R.y[3] = Q.ux[slot];
    R.y[4] = Q.uy[slot];
    R.y[5] = Q.uz[slot];
  } else {
    set_direction<MODEL, FIELD>(P, R, Q.ux[slot], Q.uy[slot], Q.uz[slot]);
  }
  C.max(S_MAXGEN, (unsigned long long)R.gen);
}

// Park a ray in flight when the launch's step budget is reached: its whole
// state goes into its record slot (the direction state as it is, not
// normalised) with status RT_ST_PARKED, and a resumed launch continues it
// bit for bit.  A ray that was locating a crossing redoes that step: its
// state is still the step's start, and the accepted step is uncounted.
__device__ __forceinline__ void park_ray(const KParams& P, Ray& R, int mode) {
  const Pool& Q = P.pool;
  const int i = R.slot;
  const int t = (int)threadIdx.x;
  if (mode == 1) R.n_acc--;
  Q.x[i] = R.y[0];
  Q.y[i] = R.y[1];
  Q.z[i] = R.y[2];
  Q.ux[i] = R.y[3];
  Q.uy[i] = R.y[4];
  Q.uz[i] = R.y[5];
  Q.s[i] = R.s;
  Q.t[i] = R.y[6];
  Q.h[i] = R.h;
  Q.as_re[i] = s_as_re[t];
  Q.as_im[i] = s_as_im[t];
  Q.ap_re[i] = s_ap_re[t];
  Q.ap_im[i] = s_ap_im[t];
  Q.n_acc[i] = R.n_acc;
  Q.n_rej[i] = R.n_rej;
  Q.n_ev[i] = R.n_ev;
  Q.region[i] = R.region;
  Q.side[i] = R.side;
  Q.status[i] = RT_ST_PARKED;
}

// Checks made before every normal trial step; returns a final status or 0.
__device__ __forceinline__ int32_t pretrial_status(const KParams& P, const Ray& R) {
  if (R.s >= P.s_max) return RT_ST_PATH;
  if ((int64_t)R.n_acc + R.n_rej >= P.max_steps) return RT_ST_STEPCAP;
  return 0;
}

// Boundary event at the located state ys (boundary k, at sigma along the
// step); returns the final status of the ray or 0 when it continues.
template <int MODEL, int FIELD, bool EV>
__device__ __forceinline__ int32_t boundary_event(const KParams& P, Ray& R, int k, double sig,
                                                  double ys[7], double h_next, const Counters& C,
                                                  const WaveQueue& WQ) {
  const KBnd& B = s_bnd[k];
  if (B.kind != B_TIME) bnd_snap(B, ys);  // onto the boundary
#pragma unroll
  for (int i = 0; i < 7; ++i) R.y[i] = ys[i];
  set_direction<MODEL, FIELD>(P, R, ys[3], ys[4], ys[5]);
  R.s = R.s + sig;
  R.h = h_next;
  if (B.kind == B_BOX) return RT_ST_BOX;
  if (B.kind == B_TIME) return RT_ST_TIME;
  if (B.kind == B_ABSORB) return RT_ST_ABSORB;
  if (R.n_ev >= kMaxEvents) return RT_ST_STEPCAP;
  R.n_ev++;
  C.bump(S_EVENTS);

  const double sg = ((R.side >> k) & 1u) ? 1.0 : -1.0;
  double nb[3];
  bnd_normal(B, R.y, nb);
  const double nin[3] = {sg * nb[0], sg * nb[1], sg * nb[2]};
  const double il = rsqrt_nr(fma(R.y[3], R.y[3], fma(R.y[4], R.y[4], R.y[5] * R.y[5])));
  const double u[3] = {R.y[3] * il, R.y[4] * il, R.y[5] * il};
  double ci = -fma(u[2], nin[2], fma(u[1], nin[1], u[0] * nin[0]));
  ci = fmax(ci, 0.0);
  const int reg_out = sg > 0.0 ? B.reg_neg : B.reg_pos;
  const Medium Mo = medium_of(P, reg_out);
  const double n1 = field_n<MODEL, FIELD>(P, medium_of(P, R.region), R.y);
  const double n2 = field_n<MODEL, FIELD>(P, Mo, R.y);
  double rt[8], ct;
  const bool tir = fresnel(n1, n2, ci, rt, ct);

  const Pool& Q = P.pool;
  const int tl = (int)threadIdx.x;
  const double as_re = s_as_re[tl], as_im = s_as_im[tl];
  const double ap_re = s_ap_re[tl], ap_im = s_ap_im[tl];
  int32_t outcome = tir ? RT_EV_TIR : RT_EV_GEN;
  if (!tir) {
    if (R.gen + 1 < P.max_gen) {
      const double cs_re = as_re * rt[4] - as_im * rt[5];
      const double cs_im = as_re * rt[5] + as_im * rt[4];
      const double cp_re = ap_re * rt[6] - ap_im * rt[7];
      const double cp_im = ap_re * rt[7] + ap_im * rt[6];
      const double amax = fmax(hypot(cs_re, cs_im), hypot(cp_re, cp_im));
      if (P.amp_min > 0.0 && amax < P.amp_min) {
        C.bump(S_SUPP_AMP);
        outcome = RT_EV_AMP;
      } else {
        C.bump(S_SPAWNED);
        outcome = RT_EV_SPAWNED;
        const uint64_t c = wave_slot(P, (int)threadIdx.x / 64);
        if (c >= (uint64_t)P.capacity) {
          C.bump(S_FIN);  // no record slot: reported via stats.needed
          __hip_atomic_fetch_add(&P.q->dropped, (uint64_t)1, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
        } else {
          const double eta = n1 / n2;
          const double f = eta * ci - ct;
          const uint64_t key = s_key[tl];
          Q.x[c] = R.y[0];
          Q.y[c] = R.y[1];
          Q.z[c] = R.y[2];
          Q.ux[c] = fma(eta, u[0], f * nin[0]);
          Q.uy[c] = fma(eta, u[1], f * nin[1]);
          Q.uz[c] = fma(eta, u[2], f * nin[2]);
          Q.s[c] = R.s;
          Q.t[c] = R.y[6];
          Q.h[c] = R.h;
          Q.as_re[c] = cs_re;
          Q.as_im[c] = cs_im;
          Q.ap_re[c] = cp_re;
          Q.ap_im[c] = cp_im;
          Q.key[c] = key | ((uint64_t)R.n_ev << (8 * (2 - R.gen)));
          Q.parent[c] = key;
          Q.gen[c] = R.gen + 1;
          Q.region[c] = reg_out;
          Q.side[c] = R.side ^ (1u << k);
          Q.n_acc[c] = 0;
          Q.n_rej[c] = 0;
          Q.n_ev[c] = 0;
          Q.status[c] = RT_ST_QUEUED;
          // Queue the child on this wave while its backlog is short; beyond
          // local_limit queued rays, publish it on the global overflow queue
          // so that idle waves elsewhere share a large ray tree.
          const uint64_t m = __ballot(1);
          const uint32_t h = *WQ.head, t = *WQ.tail;
          const uint32_t rank = (uint32_t)__popcll(m & lanemask_lt());
          const uint32_t room = (t - h) < P.local_limit ? P.local_limit - (t - h) : 0u;
          const uint32_t np = min((uint32_t)__popcll(m), room);
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
          if (rank < np) WQ.ring[(t + rank) % kRing] = (int32_t)c;
          if ((int)__lane_id() == __ffsll((unsigned long long)m) - 1) {
            *WQ.tail = t + np;
            C.max(S_MAXQ, t + np - h);
          }
          // The agent-scope release below writes back this XCD's L2; the
          // wave-uniform guard keeps it off the path when no lane spills.
          if (__ballot(rank >= np) != 0) {
            if (rank >= np) {
              const uint64_t e = wave_append(&P.q->gq_tail);
              __hip_atomic_store(&P.gq[e], (int32_t)c, __ATOMIC_RELEASE,
                                 __HIP_MEMORY_SCOPE_AGENT);
              C.bump(S_SPILLED);
            }
          }
        }
      }
    } else {
      C.bump(S_SUPP_GEN);
    }
  }
  if constexpr (EV) {  // instances that record events run only with ev_capacity > 0
    // the array and its size come from LDS: kept as kernel arguments they
    // would occupy scalar registers for the whole step loop
    const uint64_t e = wave_append(&P.q->ev_tail);
    if (e < s_ev_cap) {
      rt_event* E = s_ev_base + e;
      E->key = s_key[tl];
      E->ordinal = R.n_ev;
      E->boundary = k;
      E->outcome = outcome;
      E->gen = R.gen;
      E->region_in = R.region;
      E->region_out = reg_out;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        E->pos[a] = R.y[a];
        E->dir[a] = u[a];
      }
      E->s = R.s;
      E->t = R.y[6];
      E->cos_i = ci;
      E->n1 = n1;
      E->n2 = n2;
      E->amp[0] = as_re;
      E->amp[1] = as_im;
      E->amp[2] = ap_re;
      E->amp[3] = ap_im;
#pragma unroll
      for (int a = 0; a < 8; ++a) E->coef[a] = rt[a];
    }
  }
  // the parent continues as the reflected ray
  const double rs_re = as_re * rt[0] - as_im * rt[1];
  const double rs_im = as_re * rt[1] + as_im * rt[0];
  const double rp_re = ap_re * rt[2] - ap_im * rt[3];
  const double rp_im = ap_re * rt[3] + ap_im * rt[2];
  s_as_re[tl] = rs_re;
  s_as_im[tl] = rs_im;
  s_ap_re[tl] = rp_re;
  s_ap_im[tl] = rp_im;
  const double c2 = 2.0 * ci;
  set_direction<MODEL, FIELD>(P, R, fma(c2, nin[0], u[0]), fma(c2, nin[1], u[1]),
                              fma(c2, nin[2], u[2]));
  if (P.amp_min > 0.0 && fmax(hypot(rs_re, rs_im), hypot(rp_re, rp_im)) < P.amp_min)
    return RT_ST_AMP;
  return 0;
}

// Publish a wave's finished rays and the unused rest of its slot chunk
// (lane 0; the chunk count replaces what was published before).
__device__ __forceinline__ void publish_idle(const KParams& P, const Counters& C, int wv) {
  if ((int)__lane_id() != 0) return;
  const unsigned long long f = C.c[S_FIN];
  const uint32_t unused = (uint32_t)(s_cend[wv] - s_cnext[wv]);
  const unsigned long long d = f + (unused - s_cphant[wv]);  // unused >= s_cphant
  if (d) {
    C.c[S_FIN] = 0;
    s_cphant[wv] = unused;
    __hip_atomic_fetch_add(&P.q->finished, (uint64_t)d, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
  }
}

// ---------------------------------------------------------------------------
// Persistent trace kernel.
template <int MODEL, int FIELD, bool EV>
__device__ __forceinline__ void trace_body(const KParams& P) {
  for (int i = threadIdx.x; i < P.n_regions; i += blockDim.x) s_reg[i] = P.reg[i];
  for (int i = threadIdx.x; i < P.n_bnd; i += blockDim.x) s_bnd[i] = P.bnd[i];
  const int lane = (int)__lane_id();
  const int tid = (int)threadIdx.x;
  __shared__ unsigned long long s_cnt[4][S_COUNT];
  const Counters C{s_cnt[tid / 64]};
  if (lane < S_COUNT) C.c[lane] = 0;
  // Crossing-search state of each lane, kept in LDS (one entry per thread,
  // structure of arrays) so that it does not occupy registers in the step
  // loop: bracket [a, b] with its function values, the full step length, the
  // controller's proposal for the step after the event, the boundary being
  // searched and (pass << 16 | iterations << 2 | last side + 1).
  //
  // A ray passes a boundary only by going through it.  One that starts on
  // the boundary (on_boundary(G0)) and heads into it passes it at sigma = 0;
  // one that starts on it and leaves it (the reflected ray and the
  // secondary after an event) passes it only where it comes back, e.g. at
  // the far end of a short chord through a sphere.  Its bracket starts with
  // a positive value for G(0) (departure_start) in place of G(0) ~ 0, which
  // would draw the iterates to the departure point.
  __shared__ double s_a[256], s_Ga[256], s_b[256], s_Gb[256], s_hp[256], s_hn[256];
  __shared__ int32_t s_k[256], s_meta[256];
  if (EV && tid == 0) {
    s_ev_base = P.events;
    s_ev_cap = (unsigned long long)P.ev_capacity;
  }
  __syncthreads();

  s_nacc[tid] = 0;
  s_nrej[tid] = 0;
  Ray R;
  R.slot = -1;
  R.s = R.h = 0.0;
  R.region = R.gen = R.n_acc = R.n_rej = R.n_ev = 0;
  R.side = 0;
#pragma unroll
  for (int i = 0; i < 7; ++i) R.y[i] = 0.0;
  int mode = 0;     // 0: normal step, 1: searching a crossing, 2: crossing located
  double lc = 0.0;  // search iterate (mode 1) or located sigma (mode 2)

  // Scheduler.
  //  * Primaries (record slots [0, n_primary)) are handed out by ticket, one
  //    fetch_add on q->head per wave refill, ticket t taking slot P.perm[t]:
  //    rays of one source with neighbouring directions (order_kernel), so
  //    that the lanes of a wave follow nearby paths (shared cache lines of
  //    a gridded field, alike branches).
  //  * A secondary gets its record slot from q->tail.  Up to local_limit
  //    wait on the wave that cast them (ring in LDS; producer and consumer
  //    are the same wave, so a workgroup-scope fence suffices).  Beyond that
  //    they are published on a global overflow queue (release store of the
  //    slot index into P.gq), from which waves without local work take
  //    tickets, one fetch_add on q->gq_head per refill; a ticket whose entry
  //    is not published yet waits.
  //  * Idle lanes take, in this order: queued children of their wave,
  //    primaries, overflow tickets.  Finished rays are counted per wave and
  //    added to q->finished when the wave has nothing to step; the launch is
  //    over when finished == tail (only running rays create new ones).
  __shared__ int32_t s_ring[4][kRing];
  __shared__ uint32_t s_rh[4], s_rt[4];
  const int wv = tid / 64;
  const WaveQueue WQ{s_ring[wv], &s_rh[wv], &s_rt[wv]};
  if (lane == 0) {
    s_rh[wv] = 0;
    s_rt[wv] = 0;
    s_cnext[wv] = 0;
    s_cend[wv] = 0;
    s_cphant[wv] = 0;
    s_cmode[wv] = P.chunk > 0 ? 1u : 0u;
  }
  bool prim_done = false;  // wave-uniform: no primaries left to claim
  // Step budget of the launch, per wave in LDS (no registers in the loop):
  // trial steps not yet added to q->steps, iterations, and the stop flag.
  __shared__ unsigned long long s_bsteps[4];
  __shared__ uint32_t s_biter[4], s_bstop[4];
  if (lane == 0) {
    s_bsteps[wv] = 0;
    s_biter[wv] = 0;
    s_bstop[wv] = 0;
  }
  __shared__ uint32_t s_evwait[4];  // iterations the wave's events have waited
  if (lane == 0) s_evwait[wv] = 0;
  int32_t since_ev = kEvDense;  // trials of this lane since its last event
  int32_t ticket = -1;     // overflow ticket: -1 none, -2 exhausted, else entry
  uint32_t sleeps = 0;
  const Pool& Q = P.pool;

  for (;;) {
    // ---- boundary events located in earlier iterations ----
    // An event runs its code (Fresnel coefficients, spawn, event record)
    // for the lanes that have one while the others wait, so a wave handles
    // the events of several lanes at once: in the stratified kernel a lane
    // with a located crossing waits (no trial) until kEvBatch lanes have
    // one, until the pending lanes are a sixteenth of the busy ones (a
    // draining wave), until the oldest has waited kEvWait iterations or the
    // step budget stops the wave -- unless a pending lane met its previous
    // event fewer than kEvDense trials before (a ray in an event-dense
    // stretch, e.g. bouncing inside a void, does not wait).  Which lanes
    // trace together changes, not any ray's arithmetic.  The general kernel
    // handles events at once (batching measured slower there).
    bool ev_go = false;
    if constexpr (FIELD == 0) {
      const uint64_t pend = __ballot(mode == 2);
      if (pend) {
        const uint32_t np = (uint32_t)__popcll(pend);
        const uint32_t nb = (uint32_t)__popcll(__ballot(R.slot >= 0));
        const bool dense = __ballot(mode == 2 && since_ev < kEvDense) != 0;
        ev_go = dense || np >= kEvBatch || np * 16u >= nb || s_evwait[wv] >= kEvWait ||
                (P.budget > 0 && s_bstop[wv]);
        if (lane == 0) s_evwait[wv] = ev_go ? 0u : s_evwait[wv] + 1u;
      }
    } else {
      ev_go = true;
    }
    if (ev_go && mode == 2) {
      since_ev = 0;
      mode = 0;
      int32_t fin = boundary_event<MODEL, FIELD, EV>(P, R, s_k[tid], lc, R.y, s_hn[tid], C, WQ);
      if (!fin) fin = pretrial_status(P, R);
      if (fin) {
        write_record(P, R, fin, C);
        R.slot = -1;
      }
    }
    // ---- step budget reached: leave (the rays in flight are parked below) ----
    if (P.budget > 0 && s_bstop[wv]) break;
    // ---- refill idle lanes ----
    const bool lane_idle = R.slot < 0 && ticket == -1;
    const uint64_t idle = __ballot(lane_idle);
    const uint32_t nidle = (uint32_t)__popcll(idle);
    const uint32_t rank = (uint32_t)__popcll(idle & lanemask_lt());
    uint32_t nr = 0;
    if (nidle > 0) {
      // (1) children queued on this wave
      const uint32_t h = *WQ.head, t = *WQ.tail;
      nr = min(nidle, t - h);
      if (nr > 0) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        if (lane_idle && rank < nr) {
          load_ray<MODEL, FIELD>(P, WQ.ring[(h + rank) % kRing], R, C);
          mode = 0;
        }
        if (lane == 0) *WQ.head = h + nr;
      }
      // (2) primaries
      const uint32_t nleft = nidle - nr;
      if (!prim_done && nleft > 0 && (nleft >= (uint32_t)P.refill || nleft == 64)) {
        unsigned long long base = 0;
        if (lane == 0) {
          base = __hip_atomic_fetch_add(&P.q->head, (uint64_t)nleft, __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT);
          atomicAdd(&C.c[S_REFILLS], 1ull);
        }
        base = __shfl(base, 0);
        if (base + nleft >= (uint64_t)P.n_primary) prim_done = true;
        if (lane_idle && rank >= nr) {
          const uint64_t ti = base + (rank - nr);
          if (ti < (uint64_t)P.n_primary) {
            const int32_t slot = P.perm[ti];
            if (Q.status[slot] == RT_ST_QUEUED) {
              load_ray<MODEL, FIELD>(P, slot, R, C);
              mode = 0;
            } else {
              C.bump(S_FIN);  // an invalid primary: its record is already final
            }
          }
        }
      }
      // (3) overflow tickets, once the wave has nothing else to take
      const bool lane_idle2 = R.slot < 0 && ticket == -1;
      const uint64_t idle2 = __ballot(lane_idle2);
      const uint32_t n2 = (uint32_t)__popcll(idle2);
      if (prim_done && n2 > 0 && *WQ.head == *WQ.tail &&
          (n2 >= (uint32_t)P.refill || n2 == 64)) {
        unsigned long long base = 0;
        if (lane == 0)
          base = __hip_atomic_fetch_add(&P.q->gq_head, (uint64_t)n2, __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT);
        base = __shfl(base, 0);
        if (lane_idle2) {
          const uint64_t e = base + (uint64_t)__popcll(idle2 & lanemask_lt());
          ticket = e < (uint64_t)P.capacity ? (int32_t)e : -2;
        }
      }
    }
    // (4) lanes holding an overflow ticket take the ray once it is published
    // (wave-uniform guards keep the agent-scope acquire, an L2 invalidate,
    // off the common path)
    if (__ballot(R.slot < 0 && ticket >= 0) != 0) {
      int32_t c = -1;
      if (R.slot < 0 && ticket >= 0)
        c = __hip_atomic_load(&P.gq[ticket], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (__ballot(c >= 0) != 0) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        if (c >= 0) {
          load_ray<MODEL, FIELD>(P, c, R, C);
          mode = 0;
          ticket = -1;
        }
      }
    }
    // a ray may end before its first step (path limit reached, no steps left)
    if (R.slot >= 0 && mode == 0 && R.n_acc + R.n_rej == 0) {
      const int32_t fst = pretrial_status(P, R);
      if (fst) {
        write_record(P, R, fst, C);
        R.slot = -1;
      }
    }
    if (__ballot(R.slot >= 0) == 0) {
      // nothing to step: publish finished counts and the unused slots of
      // the wave's chunk, stop once no work can come or the budget is spent
      publish_idle(P, C, wv);
      if (P.budget > 0) {
        unsigned long long stop = 0;
        if (lane == 0)
          stop = __hip_atomic_load(&P.q->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (__shfl(stop, 0)) break;
      }
      if (*WQ.head == *WQ.tail && prim_done) {
        if (__ballot(ticket == -2) == ~0ull) break;  // no work can reach this wave
        unsigned long long done = 0;
        if (lane == 0) {
          const uint64_t fin_g =
              __hip_atomic_load(&P.q->finished, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          const uint64_t tail_g =
              __hip_atomic_load(&P.q->tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          done = fin_g == tail_g;
        }
        if (__shfl(done, 0)) break;
        if (++sleeps > (1u << 26)) {  // guard: never expected
          if (lane == 0) atomicAdd(&C.c[S_SCHED], 1ull);
          break;
        }
        __builtin_amdgcn_s_sleep(4);
      }
      continue;
    }
    if (P.budget > 0) {
      const uint32_t busy = (uint32_t)__popcll(__ballot(R.slot >= 0));
      if (lane == 0) {
        s_bsteps[wv] += busy;
        if ((++s_biter[wv] & 63u) == 0) {
          const unsigned long long w = s_bsteps[wv];
          const unsigned long long tot =
              __hip_atomic_fetch_add(&P.q->steps, (uint64_t)w, __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_AGENT) + w;
          s_bsteps[wv] = 0;
          if (tot >= (unsigned long long)P.budget) {
            s_bstop[wv] = 1;
            __hip_atomic_store(&P.q->stop, (uint64_t)1, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
          }
        }
      }
    }
    if (R.slot < 0 || mode == 2) continue;  // idle, or waiting with an event
    since_ev = since_ev < 0x7fffffff ? since_ev + 1 : since_ev;

    // ---- one Cash-Karp trial in every busy lane ----
    const bool stepping = mode == 0;
    const bool clipped = P.s_max - R.s <= R.h;
    const double ht = stepping ? (clipped ? P.s_max - R.s : R.h) : lc;
    double y5[7], err;
    trial<MODEL, FIELD>(P, R, ht, y5, err);

    int32_t fin = 0;
    bool located = false;
    double sig = 0.0;
    if (stepping) {
      bool finite = isfinite(err);
#pragma unroll
      for (int i = 0; i < 7; ++i) finite = finite && isfinite(y5[i]);
      const bool accept = err <= 1.0 || ht <= P.h_min;
      // a full-length step whose error allows growth stays at h_max (the
      // controller's factor is at least 1.03 for err <= 1/2): the power of
      // the error is skipped, the result is the same
      double hn = P.h_max;
      if (!(accept && err <= 0.5 && ht >= P.h_max))
        hn = clamp_h(P, ht * step_factor(err, accept));
      if (!finite) {
        C.bump(S_NONFINITE);
        fin = RT_ST_NONFINITE;
      } else if (!accept) {
        R.n_rej++;
        R.h = hn;
      } else {
        R.n_acc++;
        if (err > 1.0) C.bump(S_FORCED);
        if constexpr (MODEL == RT_MODEL_PAPER) {
          const double il = rsqrt_nr(fma(y5[3], y5[3], fma(y5[4], y5[4], y5[5] * y5[5])));
          y5[3] *= il;
          y5[4] *= il;
          y5[5] *= il;
        }
        double G0 = 0.0, G1 = 0.0;
        const int k = pick_crossing(P, R.side, R.y, y5, ht, -1, G0, G1);
        if (k < 0) {
#pragma unroll
          for (int i = 0; i < 7; ++i) R.y[i] = y5[i];
          R.s = clipped ? P.s_max : R.s + ht;
          R.h = hn;
          if (clipped) fin = RT_ST_PATH;
        } else {
          // start the crossing search on [0, ht] (rare)
          s_hp[tid] = ht;
          s_hn[tid] = hn;
          s_k[tid] = k;
          const bool on = on_boundary(G0);
          double rate = 0.0, Gd = 0.0;
          if (__builtin_expect(on, 0)) {
            rate = bnd_rate(s_bnd[k], k, R.side, R.y);
            Gd = departure_start(s_bnd[k], k, R.side, rate, ht, G1);
          }
          if (on && !(rate > 0.0)) {  // on the boundary, heading in
            s_meta[tid] = 1;  // pass 0, no iterations, last side 0
            located = true;
            sig = 0.0;
#pragma unroll
            for (int i = 0; i < 7; ++i) y5[i] = R.y[i];
          } else {
            const double Ga = on ? Gd : G0;
            s_a[tid] = 0.0;
            s_Ga[tid] = Ga;
            s_b[tid] = ht;
            s_Gb[tid] = G1;
            s_meta[tid] = 1;
            lc = ht - G1 * ht / (G1 - Ga);
            mode = 1;
          }
        }
      }
    } else {
      // one iterate of the Illinois search (state in LDS)
      C.bump(S_RELOC);
      const int k = s_k[tid];
      int meta = s_meta[tid];
      int last = (meta & 3) - 1;
      const int it = ((meta >> 2) & 0xff) + 1;
      double a = s_a[tid], Ga = s_Ga[tid], b = s_b[tid], Gb = s_Gb[tid];
      const double Gc = bnd_G(P, s_bnd[k], k, R.side, y5);
      bool done = fabs(Gc) <= kLocGTol;
      if (!done) {
        if (Gc < 0.0) {
          b = lc;
          Gb = Gc;
          if (last == -1) Ga *= 0.5;
          last = -1;
        } else {
          a = lc;
          Ga = Gc;
          if (last == 1) Gb *= 0.5;
          last = 1;
        }
        if (b - a <= kLocWRel * s_hp[tid] || it >= kLocMaxIt) done = true;
      }
      if (done) {
        located = true;
        sig = lc;
      } else {
        s_a[tid] = a;
        s_Ga[tid] = Ga;
        s_b[tid] = b;
        s_Gb[tid] = Gb;
        lc = b - Gb * (b - a) / (Gb - Ga);
      }
      s_meta[tid] = (meta & ~0x3ff) | (it << 2) | (last + 1);
    }

    // ---- a crossing was located: look for an earlier one, else act on it ----
    if (located) {
      int k = s_k[tid];
      int pass = s_meta[tid] >> 16;
      for (;;) {
        double H0 = 0.0, H1 = 0.0;
        const int j = pass < kLocMaxPass ? pick_crossing(P, R.side, R.y, y5, sig, k, H0, H1) : -1;
        if (j < 0) {
          // the event itself runs at the top of the next iteration, outside
          // the post-trial branches
          s_k[tid] = k;
          mode = 2;
          lc = sig;
#pragma unroll
          for (int i = 0; i < 7; ++i) R.y[i] = y5[i];
          break;
        }
        ++pass;
        k = j;
        const bool on = on_boundary(H0);
        double rate = 0.0, Hd = 0.0;
        if (__builtin_expect(on, 0)) {
          rate = bnd_rate(s_bnd[k], k, R.side, R.y);
          Hd = departure_start(s_bnd[k], k, R.side, rate, sig, H1);
        }
        if (on && !(rate > 0.0)) {
          sig = 0.0;
#pragma unroll
          for (int i = 0; i < 7; ++i) y5[i] = R.y[i];
          continue;
        }
        const double Ha = on ? Hd : H0;
        s_k[tid] = k;
        s_a[tid] = 0.0;
        s_Ga[tid] = Ha;
        s_b[tid] = sig;
        s_Gb[tid] = H1;
        s_meta[tid] = (pass << 16) | 1;
        lc = sig - H1 * sig / (H1 - Ha);
        mode = 1;
        break;
      }
    }

    if (!fin && mode == 0) fin = pretrial_status(P, R);
    if (fin) {
      write_record(P, R, fin, C);
      R.slot = -1;
      mode = 0;
    }
  }

  // A wave that stopped at the step budget parks its rays; it (and any
  // other) publishes its finished count and unused chunk slots.
  if (R.slot >= 0) park_ray(P, R, mode);
  publish_idle(P, C, wv);

  // ---- per-wave statistics into the launch's rt_stats ----
  {
    unsigned long long a = s_nacc[tid], r = s_nrej[tid];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      a += __shfl_xor(a, o);
      r += __shfl_xor(r, o);
    }
    if (lane == 0) {
      C.c[S_ACC] += a;
      C.c[S_REJ] += r;
    }
  }
  if (lane == 0) {
    unsigned long long* s64 = reinterpret_cast<unsigned long long*>(P.stats);
    for (int i = 0; i < S_FIN; ++i) {
      if (i == S_NEEDED || i == S_INVALID || C.c[i] == 0) continue;
      if (i == S_MAXGEN) atomicMax(&s64[i], C.c[i]);
      else atomicAdd(&s64[i], C.c[i]);
    }
    if (C.c[S_MAXQ]) atomicMax(&s64[offsetof(rt_stats, max_queue) / 8], C.c[S_MAXQ]);
  }
}


// Launch helpers of the stratified trace kernel, defined in rt_strat.hip
// (its own translation unit, compiled with its own code-generation flags).
int strat_blocks_per_cu(int model, bool ev, int block);
hipError_t launch_strat(int model, bool ev, const KParams& P, int grid, int block,
                        hipStream_t s);

}  // namespace rt
