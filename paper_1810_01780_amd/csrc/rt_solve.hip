// Emitter -> receiver solves by shooting, for gfx950 (MI355X), FP64.
//
// Receiver and emitter locations are among the set-ups the method of
// RadioPropa (arXiv:1810.01780, section 2) supports; the rays connecting a
// source and a receiver are found here by shooting.  A shot is one ray,
// integrated exactly as in the trace kernel (Cash-Karp 4(5) steps with the
// same controller and crossing search), that follows a single branch at the
// planes and ends at the receiver plane x = dist.
//
// Execution model.  One shot per lane; a persistent grid of waves takes work
// items ("tasks") from a ticket counter, one fetch_add per wave refill, and
// every loop iteration runs one Cash-Karp trial in every busy lane (a normal
// step or one iterate of a crossing search), as in the trace kernel.  A solve
// is three such launches and a selection:
//   scan    task = (pair, family, angle k): one shot at (k + 1/2) pi / n_scan;
//   refine  task = (bracket b, pair, family): the b-th sign change of the
//           scan's misses, refined by Illinois false position; the lane runs
//           the shots of its bracket one after another;
//   select  one thread per (pair, family): the admissible root with the
//           smallest travel time.
// The scan's shots are independent, so the scan is as parallel as the trace;
// only the short refinement chains are sequential.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "radiotrace_solve.h"
#include "radiotrace_mlp.h"
#include "rt_device.hpp"
#include "rt_solve_internal.hpp"

namespace rt {

constexpr double kPi = 3.14159265358979323846;
constexpr double kMissAbove = -1.0e6;  // touched the surface: passed above the receiver
constexpr double kMissLost = 1.0e6;    // never met the receiver plane
constexpr double kBisectAbove = 1.0e5; // |miss| from which an end counts as a failed shot
// Refinement of a bracket stops below kBracketMin (rad), or when its end
// misses cannot belong to a root: a miss continuous on [a, b] with slope at
// most slope_max (m/rad) and a zero inside has |m(a)| + |m(b)| <=
// slope_max (b - a); failed-shot ends (|miss| >= kBisectAbove) count zero.
// Brackets around jumps of the miss (surface contact or loss setting in,
// total reflection at a layer) end this way.
constexpr double kBracketMin = 1e-9;
constexpr int kRecv = kMaxBnd;         // boundary index of the receiver plane

// Statistics rows, in the order of rt_solve_stats.
enum : int {
  V_SHOTS = 0, V_ACC, V_REJ, V_RELOC, V_FORCED, V_EVENTS, V_BRACKETS, V_FOUND, V_INVALID,
  V_COUNT
};
static_assert(sizeof(rt_solve_stats) == 8 * V_COUNT, "rt_solve_stats layout");

enum : int { PH_LIST = 0, PH_SCAN = 1, PH_REFINE = 2, PH_SEEDED = 3, PH_FUSED = 4 };

// The fused solve (PH_FUSED): scan, refinement and selection in one
// persistent launch.  Each wave holds up to kFEnt entries (pair, family) in
// LDS.  Idle lanes take, in this order, queued brackets, then the next scan
// angles of the wave's scanning entries (oldest entry first); when those
// cannot occupy them the wave claims new entries with one fetch_add.  A scan
// shot's miss goes to the entry's row of the scan table in HBM; the lane
// whose shot completes the scan finds the sign changes and queues the
// brackets; the lane that finishes the entry's last bracket writes its
// result.  A wave depends on no other wave, so the launch ends when every
// wave has finished its entries and no entry is left to claim.  Each shot
// and each bracket is computed exactly as in the three launches (scan,
// refine, select), so the results are the same.  It is not the default: on
// the 65,536-pair solve it took 76 ms against 69 ms for the three launches
// (the same shots in ~4 % more wave iterations, each dearer: the table
// logic runs between trials and the kernel holds more registers); the
// autotuner still tries it.
constexpr int kFEnt = 16;   // entries a wave holds
constexpr int kFScan = 64;  // largest n_scan of a fused solve
constexpr int kFBr = 4;     // largest max_brackets of a fused solve
constexpr int kFQ = kFEnt * kFBr;
constexpr int32_t kFBracket = 1 << 16;  // lane task: bracket (else scan angle)
static_assert(kFEnt <= 32 && kFScan <= 128 && kFBr <= 16, "fused table encodings");
struct FusedWave {
  int64_t pf[kFEnt];       // entry: 2 pair + family
  int32_t done[kFEnt];     // scan shots finished
  int32_t open[kFEnt];     // brackets still refining
  int32_t nb[kFEnt];       // brackets found
  int32_t klast[kFEnt];    // scan index of the last bracket's upper end
  int32_t bshots[kFEnt];   // refinement shots of its finished brackets
  int32_t roots[kFEnt];    // admissible roots so far
  int32_t best_b[kFEnt];   // bracket of the first arrival so far, -1 none
  double best_t[kFEnt];    // its travel time
  int8_t bk[kFEnt][kFBr];  // scan index of each bracket's upper end
  int8_t sq[kFEnt];        // ring: entries with scan angles left, oldest first
  uint16_t q[kFQ];         // ring: brackets to refine, entry << 4 | bracket
  uint32_t used;           // entry slots in use (bit e)
  uint32_t sh, st;         // scan ring head and tail
  int32_t sk;              // next angle of the entry at the scan ring's head
  uint32_t qh, qt;         // bracket ring head and tail
};

struct KSolve {
  const double *zs, *zr, *dist;  // per pair (scan, refine, select) or per shot (list)
  const double* theta;           // list: launch angles
  const int32_t* family;         // list: families
  int64_t n;                     // pairs or shots
  int64_t n_tasks;
  int32_t n_scan, max_iter, max_brackets, refill;
  int32_t scan_chunk;            // scan: entries whose angles interleave
  double miss_tol, accept_tol, slope_max, dtheta;
  uint64_t* tickets;  // one counter per phase
  double* scan_miss;  // [2 n][n_scan]
  // per bracket, [max_brackets][2 n]; b_status -1 = no such bracket
  double *b_theta, *b_miss, *b_t, *b_s, *b_as_re, *b_as_im, *b_ap_re, *b_ap_im;
  int32_t *b_status, *b_shots, *b_k;
  rt_shot_outputs lo;
  rt_solve_outputs so;
  unsigned long long* stats;
  // pair count read on the device (a compacted list whose length is known
  // only there); NULL = n
  const int64_t* n_dev;
  // seeded phase: per entry [2 n] the first angle and whether to try it;
  // verify[2 n] receives 1 (verified solution) or 0 (not verified)
  const double* seed;
  const int32_t* seed_try;
  int32_t* verify;
  double verify_tol, dseed;
  int32_t max_shots;
  // scan and refine: per pair, bit f set = solve family f; NULL = both
  // (the other family's entries are left as no solution)
  const uint8_t* fam_mask;
};

// A pair can be shot if its values are finite, the distance is positive and
// the source is not within 1e-9 m of a plane.
__device__ __forceinline__ bool pair_ok(const KParams& P, double zs, double zr, double D) {
  if (!isfinite(zs) || !isfinite(zr) || !isfinite(D) || !(D > 0.0)) return false;
  for (int k = 0; k < P.n_bnd; ++k)
    if (fabs(zs * P.bnd[k].nrm[2] - P.bnd[k].d) <= 1e-9) return false;
  return true;
}

// Boundary function of boundary k (a plane, or the receiver plane, where
// g = D - x is positive on the source side).
__device__ __forceinline__ double shot_G(const KParams& P, int k, uint32_t side, double D,
                                         const double y[7]) {
  if (k == kRecv) return D - y[0];
  return bnd_G(P, s_bnd[k], k, side, y);
}

// Earliest crossing of a step among the planes and the receiver plane (the
// receiver is the last candidate: a tie goes to the plane).
__device__ __forceinline__ int pick_crossing_shot(const KParams& P, uint32_t side, double D,
                                                  const double y0[7], const double y1[7],
                                                  double len, int skip, double& G0o,
                                                  double& G1o) {
  int best = pick_crossing(P, side, y0, y1, len, skip, G0o, G1o);
  if (skip != kRecv) {
    const double G1 = D - y1[0];
    if (G1 <= 0.0) {
      const double G0 = D - y0[0];
      const double sig = G0 <= 0.0 ? 0.0 : len * G0 / (G0 - G1);
      const double best_sig = best < 0 ? 0.0 : (G0o <= 0.0 ? 0.0 : len * G0o / (G0o - G1o));
      if (best < 0 || sig < best_sig) {
        best = kRecv;
        G0o = G0;
        G1o = G1;
      }
    }
  }
  return best;
}

// Shot state of a lane beyond the ray itself.
struct Shot {
  double D, smax;      // receiver distance, path limit of the shot
  int32_t pair, fam;   // pair (or list entry) index, family
  int32_t nrefl;       // surface reflections so far
};

// Start a shot from (0, 0, zs) at angle theta from the upward vertical.
template <int MODEL>
__device__ __forceinline__ void start_shot(const KParams& P, Ray& R, Shot& S, double zs,
                                           double zr, double theta, double amp[4]) {
  R.y[0] = 0.0;
  R.y[1] = 0.0;
  R.y[2] = zs;
  R.y[6] = 0.0;
  R.s = 0.0;
  R.h = P.h_init;
  R.n_acc = R.n_rej = R.n_ev = 0;
  int32_t region = 0;
  for (int g = P.n_regions - 1; g >= 0; --g)  // first region containing the depth
    if (zs >= P.reg[g].z_top && zs < P.reg[g].z_bot) region = g;
  R.region = region;
  uint32_t side = 0;
  for (int k = 0; k < P.n_bnd; ++k)
    if (zs * P.bnd[k].nrm[2] - P.bnd[k].d > 0.0) side |= 1u << k;
  R.side = side;
  S.smax = 2.0 * (S.D + zs + zr) + 1000.0;
  S.nrefl = 0;
  amp[0] = 1.0;
  amp[1] = 0.0;
  amp[2] = 1.0;
  amp[3] = 0.0;
  double sn, cs;
  sincos(theta, &sn, &cs);
  set_direction<MODEL, 0>(P, R, sn, 0.0, -cs);
}

// Result of a finished shot.
struct ShotEnd {
  int32_t status;
  double miss;
};

// Crossing located at R.y (already the located state) on boundary k after
// sigma: snap, then act.  Returns status >= 0 when the shot ends.
template <int MODEL>
__device__ __forceinline__ ShotEnd shot_event(const KParams& P, const KSolve& V, Ray& R,
                                              Shot& S, int k, double sig, double h_next,
                                              double* amp, const Counters& C) {
  double* y = R.y;
  if (k == kRecv) {
    y[0] += S.D - y[0];  // onto x = D
  } else {
    const KBnd& B = s_bnd[k];
    const double g = fma(y[2], B.nrm[2], fma(y[1], B.nrm[1], y[0] * B.nrm[0])) - B.d;
    y[0] -= g * B.nrm[0];
    y[1] -= g * B.nrm[1];
    y[2] -= g * B.nrm[2];
  }
  set_direction<MODEL, 0>(P, R, y[3], y[4], y[5]);
  R.s = R.s + sig;
  R.h = h_next;
  C.bump(V_EVENTS);
  if (k == kRecv) {
    double z = y[2];
    if (S.fam == RT_FAMILY_REFLECTED && S.nrefl == 0) {
      // before its reflection: the mirror image in the surface
      const double z_surf = P.bnd[0].d * P.bnd[0].nrm[2];
      z = 2.0 * z_surf - z;
    }
    return ShotEnd{RT_SHOT_RECEIVER, z - V.zr[S.pair]};
  }
  const KBnd& B = s_bnd[k];
  if (B.kind != B_FRESNEL) return ShotEnd{RT_SHOT_LOST, kMissLost};
  const bool surface = k == 0;
  if (surface && (S.fam == RT_FAMILY_DIRECT || S.nrefl > 0))
    return ShotEnd{RT_SHOT_SURFACE, kMissAbove};
  const double sg = ((R.side >> k) & 1u) ? 1.0 : -1.0;
  const double nin[3] = {sg * B.nrm[0], sg * B.nrm[1], sg * B.nrm[2]};
  const double il = rsqrt_nr(fma(y[3], y[3], fma(y[4], y[4], y[5] * y[5])));
  const double u[3] = {y[3] * il, y[4] * il, y[5] * il};
  const double ci = fmax(-fma(u[2], nin[2], fma(u[1], nin[1], u[0] * nin[0])), 0.0);
  const int reg_out = sg > 0.0 ? B.reg_neg : B.reg_pos;
  const double n1 = field_n<MODEL, 0>(P, medium_of(P, R.region), y);
  const double n2 = field_n<MODEL, 0>(P, medium_of(P, reg_out), y);
  double rt[8], ct;
  const bool tir = fresnel(n1, n2, ci, rt, ct);
  const int o = (surface || tir) ? 0 : 4;  // reflected or transmitted factors
  const double s_re = amp[0] * rt[o] - amp[1] * rt[o + 1];
  const double s_im = amp[0] * rt[o + 1] + amp[1] * rt[o];
  const double p_re = amp[2] * rt[o + 2] - amp[3] * rt[o + 3];
  const double p_im = amp[2] * rt[o + 3] + amp[3] * rt[o + 2];
  amp[0] = s_re;
  amp[1] = s_im;
  amp[2] = p_re;
  amp[3] = p_im;
  if (surface || tir) {
    const double c2 = 2.0 * ci;
    set_direction<MODEL, 0>(P, R, fma(c2, nin[0], u[0]), fma(c2, nin[1], u[1]),
                            fma(c2, nin[2], u[2]));
    if (surface) S.nrefl++;
  } else {
    const double eta = n1 / n2;
    const double f = eta * ci - ct;
    R.region = reg_out;
    R.side ^= 1u << k;
    set_direction<MODEL, 0>(P, R, fma(eta, u[0], f * nin[0]), fma(eta, u[1], f * nin[1]),
                            fma(eta, u[2], f * nin[2]));
  }
  return ShotEnd{-1, 0.0};
}

__device__ __forceinline__ int miss_sign(double m) { return m < 0.0 ? -1 : 1; }
__device__ __forceinline__ double finite_miss(double m) {
  return fabs(m) < kBisectAbove ? fabs(m) : 0.0;
}

// Next Illinois iterate of a bracket (bisection while an end is a failed
// shot).
__device__ __forceinline__ double illinois_next(double a, double Ga, double b, double Gb) {
  if (fabs(Ga) >= kBisectAbove || fabs(Gb) >= kBisectAbove) return 0.5 * (a + b);
  return b - Gb * (b - a) / (Gb - Ga);
}

// Fused solve: entry slot e of a wave has no bracket left; write what the
// select phase writes (the first arrival's fields are already in place) and
// free the slot.
__device__ __forceinline__ void fused_finish(const KSolve& V, FusedWave& F, int e,
                                             const Counters& C) {
  const rt_solve_outputs& O = V.so;
  const int64_t pf = F.pf[e];
  const int nb = F.nb[e];
  const bool found = F.best_b[e] >= 0;
  O.shots[pf] = (nb >= V.max_brackets ? F.klast[e] + 1 : V.n_scan) + F.bshots[e];
  O.found[pf] = found ? 1 : 0;
  O.roots[pf] = F.roots[e];
  if (found) {
    atomicAdd(&C.c[V_FOUND], 1ull);
  } else {
    O.theta[pf] = O.miss[pf] = O.t[pf] = O.s[pf] = 0.0;
    O.as_re[pf] = O.as_im[pf] = O.ap_re[pf] = O.ap_im[pf] = 0.0;
  }
  __hip_atomic_fetch_and(&F.used, ~(1u << e), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

template <int MODEL, int PHASE>
__device__ __forceinline__ void shot_body(const KParams& P, const KSolve& V) {
  for (int i = threadIdx.x; i < P.n_regions; i += blockDim.x) s_reg[i] = P.reg[i];
  for (int i = threadIdx.x; i < P.n_bnd; i += blockDim.x) s_bnd[i] = P.bnd[i];
  const int lane = (int)__lane_id();
  const int tid = (int)threadIdx.x;
  __shared__ unsigned long long s_cnt[4][V_COUNT];
  const Counters C{s_cnt[tid / 64]};
  if (lane < V_COUNT) C.c[lane] = 0;
  // accepted and rejected steps of the shots each lane has finished (added
  // to the statistics at the end: the step loop keeps no counters)
  __shared__ unsigned long long s_sacc[256], s_srej[256];
  s_sacc[tid] = 0;
  s_srej[tid] = 0;
  // crossing search of each lane (as in the trace kernel)
  __shared__ double s_a[256], s_Ga[256], s_b[256], s_Gb[256], s_hp[256], s_hn[256];
  __shared__ int32_t s_k[256], s_meta[256];
  // amplitudes (s re, s im, p re, p im) of each lane's shot
  __shared__ double s_amp[4][256];
  // refinement state of each lane: bracket [ra, rb] with misses, the angle
  // being shot, and (iterations << 2 | last side + 1)
  // (the seeded phase keeps its previous angle and miss in s_ra, s_rGa and
  // the shots taken in s_rm)
  constexpr int kR = (PHASE == PH_REFINE || PHASE == PH_SEEDED || PHASE == PH_FUSED) ? 256 : 1;
  __shared__ double s_ra[kR], s_rGa[kR];
  __shared__ double s_rb[kR], s_rGb[kR];
  __shared__ double s_rc[kR];
  __shared__ double s_rma[kR], s_rmb[kR];
  __shared__ int32_t s_rm[kR];
  // fused solve: the entries each wave holds
  __shared__ FusedWave s_fw[PHASE == PH_FUSED ? 4 : 1];
  FusedWave& F = s_fw[PHASE == PH_FUSED ? tid / 64 : 0];
  if (PHASE == PH_FUSED && lane == 0) {
    F.used = 0;
    F.sh = F.st = F.qh = F.qt = 0;
    F.sk = 0;
  }
  __syncthreads();
  int64_t n_pairs = V.n, n_tasks = V.n_tasks;
  if (V.n_dev) {
    n_pairs = *V.n_dev;
    n_tasks = PHASE == PH_SCAN     ? 2 * n_pairs * V.n_scan
              : PHASE == PH_REFINE ? 2 * n_pairs * V.max_brackets
                                   : 2 * n_pairs;
  }

  Ray R;
  R.slot = -1;  // task index, -1 = idle
  R.s = R.h = 0.0;
  R.region = R.gen = R.n_acc = R.n_rej = R.n_ev = 0;
  R.side = 0;
#pragma unroll
  for (int i = 0; i < 7; ++i) R.y[i] = 0.0;
  Shot S{0.0, 0.0, 0, 0, 0};
  int mode = 0;     // 0: normal step, 1: searching a crossing, 2: crossing located
  double lc = 0.0;  // search iterate (mode 1) or located sigma (mode 2)
  bool exhausted = false;  // wave-uniform: the ticket counter is past n_tasks
  ShotEnd fin{-1, 0.0};

  for (;;) {
    // ---- crossing located in the previous iteration ----
    if (mode == 2) {
      mode = 0;
      double a4[4] = {s_amp[0][tid], s_amp[1][tid], s_amp[2][tid], s_amp[3][tid]};
      fin = shot_event<MODEL>(P, V, R, S, s_k[tid], lc, s_hn[tid], a4, C);
#pragma unroll
      for (int i = 0; i < 4; ++i) s_amp[i][tid] = a4[i];
      if (fin.status < 0 &&
          (R.s >= S.smax || (int64_t)R.n_acc + R.n_rej >= P.max_steps))
        fin = ShotEnd{RT_SHOT_LOST, kMissLost};
    }
    // ---- a shot ended: record it, or continue its bracket ----
    if (fin.status >= 0) {
      C.bump(V_SHOTS);
      s_sacc[tid] += (unsigned long long)R.n_acc;
      s_srej[tid] += (unsigned long long)R.n_rej;
      const int64_t t = R.slot;
      if constexpr (PHASE == PH_LIST) {
        const rt_shot_outputs& O = V.lo;
        O.status[t] = fin.status;
        O.n_acc[t] = R.n_acc;
        O.n_rej[t] = R.n_rej;
        O.miss[t] = fin.miss;
        O.t[t] = R.y[6];
        O.s[t] = R.s;
        O.as_re[t] = s_amp[0][tid];
        O.as_im[t] = s_amp[1][tid];
        O.ap_re[t] = s_amp[2][tid];
        O.ap_im[t] = s_amp[3][tid];
        R.slot = -1;
      } else if constexpr (PHASE == PH_SCAN) {
        V.scan_miss[t] = fin.miss;
        R.slot = -1;
      } else if constexpr (PHASE == PH_SEEDED) {
        // seeded secant: the seed, the seed + dseed, then secant steps; the
        // entry is solved once a shot meets the receiver plane within
        // verify_tol
        const int shots = s_rm[tid] + 1;
        const double c = s_rc[tid];
        const bool recv = fin.status == RT_SHOT_RECEIVER;
        const bool success = recv && fabs(fin.miss) <= V.verify_tol;
        bool done = success || !recv || shots >= V.max_shots;
        double cn = 0.0;
        if (!done) {
          if (shots == 1) {
            cn = c + V.dseed < kPi ? c + V.dseed : c - V.dseed;
          } else {
            const double cp = s_ra[tid], mp = s_rGa[tid];
            cn = c - fin.miss * (c - cp) / (fin.miss - mp);
          }
          if (!(cn > 0.0 && cn < kPi)) done = true;  // also a non-finite step
        }
        if (done) {
          const rt_solve_outputs& O = V.so;
          O.found[t] = success ? 1 : 0;
          O.shots[t] = shots;
          O.roots[t] = success ? 1 : 0;
          O.theta[t] = success ? c : 0.0;
          O.miss[t] = success ? fin.miss : 0.0;
          O.t[t] = success ? R.y[6] : 0.0;
          O.s[t] = success ? R.s : 0.0;
          O.as_re[t] = success ? s_amp[0][tid] : 0.0;
          O.as_im[t] = success ? s_amp[1][tid] : 0.0;
          O.ap_re[t] = success ? s_amp[2][tid] : 0.0;
          O.ap_im[t] = success ? s_amp[3][tid] : 0.0;
          V.verify[t] = success ? 1 : 0;
          if (success) C.bump(V_FOUND);
          R.slot = -1;
        } else {
          s_ra[tid] = c;
          s_rGa[tid] = fin.miss;
          s_rc[tid] = cn;
          s_rm[tid] = shots;
          double a4[4];
          start_shot<MODEL>(P, R, S, V.zs[S.pair], V.zr[S.pair], cn, a4);
#pragma unroll
          for (int i = 0; i < 4; ++i) s_amp[i][tid] = a4[i];
          mode = 0;
        }
      } else if (PHASE == PH_FUSED && !(t & kFBracket)) {
        // fused: a scan shot of entry slot e, angle k; the shot that
        // completes the scan turns the entry's sign changes into brackets
        const int e = (int)((t >> 8) & 0xff), k = (int)(t & 0xff);
        const double* m = V.scan_miss + F.pf[e] * V.n_scan;
        V.scan_miss[F.pf[e] * V.n_scan + k] = fin.miss;
        // the miss is visible to the wave's lanes before the count moves
        // (an entry's shots and its completion all run in one wave, so
        // work-group scope orders them; agent scope would write back and
        // invalidate the XCD's L2 at each shot)
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        const int before = __hip_atomic_fetch_add(&F.done[e], 1, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_WORKGROUP);
        if (before + 1 == V.n_scan) {
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
          int nb = 0, klast = -1;
          double prev = m[0];
          for (int j = 1; j < V.n_scan && nb < V.max_brackets; ++j) {
            const double cur = m[j];
            if (miss_sign(cur) != miss_sign(prev)) {
              F.bk[e][nb] = (int8_t)j;
              klast = j;
              ++nb;
            }
            prev = cur;
          }
          F.nb[e] = nb;
          F.klast[e] = klast;
          F.open[e] = nb;
          if (nb == 0) {
            fused_finish(V, F, e, C);
          } else {
            atomicAdd(&C.c[V_BRACKETS], (unsigned long long)nb);
            const uint32_t q0 = __hip_atomic_fetch_add(&F.qt, (uint32_t)nb, __ATOMIC_ACQ_REL,
                                                       __HIP_MEMORY_SCOPE_WORKGROUP);
            for (int b = 0; b < nb; ++b) F.q[(q0 + b) % kFQ] = (uint16_t)((e << 4) | b);
          }
        }
        R.slot = -1;
      } else {
        // one Illinois iteration of a bracket (refine phase, or a bracket of
        // the fused solve)
        int meta = s_rm[tid];
        int last = (meta & 3) - 1;
        const int it = (meta >> 2) + 1;
        double a = s_ra[tid], Ga = s_rGa[tid], b = s_rb[tid], Gb = s_rGb[tid];
        double ma = s_rma[tid], mb = s_rmb[tid];
        const double c = s_rc[tid];
        bool done = fin.status == RT_SHOT_RECEIVER && fabs(fin.miss) <= V.miss_tol;
        if (!done) {
          if (miss_sign(fin.miss) == miss_sign(Ga)) {
            a = c;
            Ga = ma = fin.miss;
            if (last == 1) Gb *= 0.5;
            last = 1;
          } else {
            b = c;
            Gb = mb = fin.miss;
            if (last == -1) Ga *= 0.5;
            last = -1;
          }
          if (fabs(b - a) <= kBracketMin || it >= V.max_iter ||
              (V.slope_max > 0.0 &&
               finite_miss(ma) + finite_miss(mb) > V.slope_max * fabs(b - a)))
            done = true;
        }
        if (done) {
          if constexpr (PHASE == PH_FUSED) {
            // the bracket's root into its entry, one lane of the wave at a
            // time; the first arrival so far is written to the outputs
            const int e = (int)((t >> 8) & 0xff), bi = (int)(t & 0xf);
            const bool adm = fin.status == RT_SHOT_RECEIVER && fabs(fin.miss) <= V.accept_tol;
            for (uint64_t m = __ballot(1); m; m &= m - 1) {
              if (lane == __ffsll((unsigned long long)m) - 1) {
                F.bshots[e] += it;
                if (adm) {
                  F.roots[e]++;
                  const double tt = R.y[6];
                  if (F.best_b[e] < 0 || tt < F.best_t[e] ||
                      (tt == F.best_t[e] && bi < F.best_b[e])) {
                    F.best_b[e] = bi;
                    F.best_t[e] = tt;
                    const rt_solve_outputs& O = V.so;
                    const int64_t pf = F.pf[e];
                    O.theta[pf] = c;
                    O.miss[pf] = fin.miss;
                    O.t[pf] = tt;
                    O.s[pf] = R.s;
                    O.as_re[pf] = s_amp[0][tid];
                    O.as_im[pf] = s_amp[1][tid];
                    O.ap_re[pf] = s_amp[2][tid];
                    O.ap_im[pf] = s_amp[3][tid];
                  }
                }
                if (--F.open[e] == 0) fused_finish(V, F, e, C);
              }
              __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
              __builtin_amdgcn_wave_barrier();
              __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            }
          } else {
            V.b_theta[t] = c;
            V.b_miss[t] = fin.miss;
            V.b_t[t] = R.y[6];
            V.b_s[t] = R.s;
            V.b_as_re[t] = s_amp[0][tid];
            V.b_as_im[t] = s_amp[1][tid];
            V.b_ap_re[t] = s_amp[2][tid];
            V.b_ap_im[t] = s_amp[3][tid];
            V.b_status[t] = fin.status;
            V.b_shots[t] = it;
          }
          R.slot = -1;
        } else {
          s_ra[tid] = a;
          s_rGa[tid] = Ga;
          s_rb[tid] = b;
          s_rGb[tid] = Gb;
          s_rma[tid] = ma;
          s_rmb[tid] = mb;
          s_rm[tid] = (it << 2) | (last + 1);
          const double cn = illinois_next(a, Ga, b, Gb);
          s_rc[tid] = cn;
          double a4[4];
          start_shot<MODEL>(P, R, S, V.zs[S.pair], V.zr[S.pair], cn, a4);
#pragma unroll
          for (int i = 0; i < 4; ++i) s_amp[i][tid] = a4[i];
          mode = 0;
        }
      }
      fin.status = -1;
    }
    // ---- idle lanes take tasks ----
    if constexpr (PHASE == PH_FUSED) {
      // Every lane reads the wave's table (LDS of this wave only, updated
      // above) and computes the same claims and hand-out; lane 0 writes the
      // table back.
      const bool lane_idle = R.slot < 0;
      const uint64_t idle = __ballot(lane_idle);
      const uint32_t nidle = (uint32_t)__popcll(idle);
      if (nidle > 0 && (nidle >= (uint32_t)V.refill || nidle == 64)) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        const uint32_t ns = (uint32_t)V.n_scan;
        const uint32_t qh = F.qh, nq = F.qt - qh;
        uint32_t sh = F.sh, st = F.st, used = F.used;
        uint32_t sk = (uint32_t)F.sk;
        uint32_t avail = nq + (sh != st ? ns - sk + (st - sh - 1) * ns : 0u);
        // claim entries while the wave's work cannot occupy the idle lanes
        if (!exhausted && avail < nidle) {
          const uint32_t c = min((uint32_t)(kFEnt - __popc(used)), (nidle - avail + ns - 1) / ns);
          if (c > 0) {
            const int64_t n_ent = 2 * n_pairs;
            unsigned long long base = 0;
            if (lane == 0)
              base = __hip_atomic_fetch_add(&V.tickets[PHASE], (uint64_t)c, __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT);
            base = __shfl(base, 0);
            if (base + c >= (uint64_t)n_ent) exhausted = true;
            const uint32_t was = used;
            for (uint32_t i = 0; i < c && base + i < (uint64_t)n_ent; ++i) {
              const int64_t pf = (int64_t)(base + i);
              const int32_t pair = (int32_t)(pf >> 1), fam = (int32_t)(pf & 1);
              const bool ok = pair_ok(P, V.zs[pair], V.zr[pair], V.dist[pair]);
              const bool want = !V.fam_mask || ((V.fam_mask[pair] >> fam) & 1);
              if (!ok || !want) {
                // no scan: an invalid pair, or a family not asked for
                if (lane == 0) {
                  const rt_solve_outputs& O = V.so;
                  O.found[pf] = 0;
                  O.shots[pf] = ok ? V.n_scan : 0;
                  O.roots[pf] = 0;
                  O.theta[pf] = O.miss[pf] = O.t[pf] = O.s[pf] = 0.0;
                  O.as_re[pf] = O.as_im[pf] = O.ap_re[pf] = O.ap_im[pf] = 0.0;
                  if (!ok && fam == 0) atomicAdd(&C.c[V_INVALID], 1ull);
                }
                continue;
              }
              const int e = __builtin_ctz(~used);  // c <= free slots
              used |= 1u << e;
              if (lane == 0) {
                F.pf[e] = pf;
                F.done[e] = 0;
                F.open[e] = 0;
                F.nb[e] = 0;
                F.klast[e] = -1;
                F.bshots[e] = 0;
                F.roots[e] = 0;
                F.best_b[e] = -1;
                F.sq[st % kFEnt] = (int8_t)e;
              }
              if (sh == st) sk = 0;
              ++st;
              avail += ns;
            }
            if (lane == 0 && used != was)
              __hip_atomic_fetch_or(&F.used, used & ~was, __ATOMIC_RELAXED,
                                    __HIP_MEMORY_SCOPE_WORKGROUP);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
          }
        }
        // hand out: queued brackets first, then scan angles, oldest entry first
        const uint32_t rank = (uint32_t)__popcll(idle & lanemask_lt());
        const uint32_t nbk = min(nq, nidle);
        int32_t task = -1;
        if (lane_idle && rank < nbk) {
          const int32_t qe = (int32_t)F.q[(qh + rank) % kFQ];
          task = kFBracket | ((qe >> 4) << 8) | (qe & 0xf);
        }
        uint32_t given = nbk;
        while (given < nidle && sh != st) {
          const int32_t e = F.sq[sh % kFEnt];
          const uint32_t take = min(ns - sk, nidle - given);
          if (lane_idle && rank >= given && rank < given + take)
            task = (e << 8) | (int32_t)(sk + rank - given);
          given += take;
          sk += take;
          if (sk == ns) {
            ++sh;
            sk = 0;
          }
        }
        if (lane == 0) {
          F.qh = qh + nbk;
          F.sh = sh;
          F.st = st;
          F.sk = (int32_t)sk;
        }
        if (task >= 0) {
          const int e = (task >> 8) & 0xff;
          const int64_t pf = F.pf[e];
          S.pair = (int32_t)(pf >> 1);
          S.fam = (int32_t)(pf & 1);
          S.D = V.dist[S.pair];
          const double zs = V.zs[S.pair], zr = V.zr[S.pair];
          double theta;
          if (task & kFBracket) {
            const int bi = task & 0xf;
            const int k = F.bk[e][bi];
            const double* m = V.scan_miss + pf * V.n_scan;
            const double a = ((double)(k - 1) + 0.5) * V.dtheta;
            const double bb = ((double)k + 0.5) * V.dtheta;
            const double Ga = m[k - 1], Gb = m[k];
            s_ra[tid] = a;
            s_rGa[tid] = Ga;
            s_rb[tid] = bb;
            s_rGb[tid] = Gb;
            s_rma[tid] = Ga;
            s_rmb[tid] = Gb;
            s_rm[tid] = 1;  // no iterations, last side 0
            theta = illinois_next(a, Ga, bb, Gb);
            s_rc[tid] = theta;
          } else {
            theta = ((double)(task & 0xff) + 0.5) * V.dtheta;
          }
          R.slot = task;
          double a4[4];
          start_shot<MODEL>(P, R, S, zs, zr, theta, a4);
#pragma unroll
          for (int i = 0; i < 4; ++i) s_amp[i][tid] = a4[i];
          mode = 0;
        }
      }
      if (__ballot(R.slot >= 0) == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        if (exhausted && F.used == 0) break;
        continue;
      }
    } else if (!exhausted) {
      const bool lane_idle = R.slot < 0;
      const uint64_t idle = __ballot(lane_idle);
      const uint32_t nidle = (uint32_t)__popcll(idle);
      if (nidle > 0 && (nidle >= (uint32_t)V.refill || nidle == 64)) {
        unsigned long long base = 0;
        if (lane == 0)
          base = __hip_atomic_fetch_add(&V.tickets[PHASE], (uint64_t)nidle, __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT);
        base = __shfl(base, 0);
        if (base + nidle >= (uint64_t)n_tasks) exhausted = true;
        const uint64_t task = base + (uint64_t)__popcll(idle & lanemask_lt());
        if (lane_idle && task < (uint64_t)n_tasks) {
          int64_t t = (int64_t)task;
          double zs = 0.0, zr = 0.0, theta = 0.0;
          bool go = false;
          if constexpr (PHASE == PH_LIST) {
            S.pair = (int32_t)t;
            S.fam = V.family[t];
            S.D = V.dist[t];
            zs = V.zs[t];
            zr = V.zr[t];
            theta = V.theta[t];
            go = pair_ok(P, zs, zr, S.D) && theta > 0.0 && theta < kPi &&
                 (S.fam == RT_FAMILY_DIRECT || S.fam == RT_FAMILY_REFLECTED);
            if (!go) {
              const rt_shot_outputs& O = V.lo;
              O.status[t] = RT_SHOT_INVALID;
              O.n_acc[t] = O.n_rej[t] = 0;
              O.miss[t] = O.t[t] = O.s[t] = 0.0;
              O.as_re[t] = O.as_im[t] = O.ap_re[t] = O.ap_im[t] = 0.0;
              C.bump(V_INVALID);
            }
          } else if constexpr (PHASE == PH_SCAN) {
            // tasks in chunks of scan_chunk entries: within a chunk the
            // angle varies slowest, so consecutive lanes shoot one angle for
            // neighbouring entries (the last chunk may be short)
            const int64_t C = V.scan_chunk, n2 = 2 * n_pairs;
            const int64_t ch = t / (C * V.n_scan), r = t - ch * C * V.n_scan;
            const int64_t ne = min(C, n2 - ch * C);
            const int64_t pf = ch * C + r % ne;
            const int k = (int)(r / ne);
            t = pf * V.n_scan + k;  // the scan's miss array is [entry][angle]
            S.pair = (int32_t)(pf >> 1);
            S.fam = (int32_t)(pf & 1);
            S.D = V.dist[S.pair];
            zs = V.zs[S.pair];
            zr = V.zr[S.pair];
            theta = ((double)k + 0.5) * V.dtheta;
            go = pair_ok(P, zs, zr, S.D) &&
                 (!V.fam_mask || ((V.fam_mask[S.pair] >> S.fam) & 1));
            if (!go) V.scan_miss[t] = 0.0;  // no sign change: no bracket
          } else if constexpr (PHASE == PH_SEEDED) {
            S.pair = (int32_t)(t >> 1);
            S.fam = (int32_t)(t & 1);
            S.D = V.dist[S.pair];
            zs = V.zs[S.pair];
            zr = V.zr[S.pair];
            if (V.seed_try[t]) {
              theta = V.seed[t];
              go = pair_ok(P, zs, zr, S.D) && theta > 0.0 && theta < kPi;
              if (go) {
                s_rc[tid] = theta;
                s_rm[tid] = 0;
              } else {
                const rt_solve_outputs& O = V.so;
                O.found[t] = 0;
                O.shots[t] = 0;
                O.roots[t] = 0;
                O.theta[t] = O.miss[t] = O.t[t] = O.s[t] = 0.0;
                O.as_re[t] = O.as_im[t] = O.ap_re[t] = O.ap_im[t] = 0.0;
                V.verify[t] = 0;
              }
            }
          } else {
            const int64_t n2 = 2 * n_pairs;
            const int b = (int)(t / n2);
            const int64_t pf = t - (int64_t)b * n2;
            S.pair = (int32_t)(pf >> 1);
            S.fam = (int32_t)(pf & 1);
            S.D = V.dist[S.pair];
            zs = V.zs[S.pair];
            zr = V.zr[S.pair];
            // the b-th sign change of the scanned misses
            const double* m = V.scan_miss + pf * V.n_scan;
            int found_k = -1, count = 0;
            if (pair_ok(P, zs, zr, S.D)) {
              double prev = m[0];
              for (int k = 1; k < V.n_scan; ++k) {
                const double cur = m[k];
                if (miss_sign(cur) != miss_sign(prev)) {
                  if (count == b) {
                    found_k = k;
                    break;
                  }
                  ++count;
                }
                prev = cur;
              }
            }
            if (found_k < 0) {
              V.b_status[t] = -1;
            } else {
              C.bump(V_BRACKETS);
              const double a = ((double)(found_k - 1) + 0.5) * V.dtheta;
              const double bb = ((double)found_k + 0.5) * V.dtheta;
              const double Ga = m[found_k - 1], Gb = m[found_k];
              s_ra[tid] = a;
              s_rGa[tid] = Ga;
              s_rb[tid] = bb;
              s_rGb[tid] = Gb;
              s_rma[tid] = Ga;
              s_rmb[tid] = Gb;
              s_rm[tid] = 1;  // no iterations, last side 0
              theta = illinois_next(a, Ga, bb, Gb);
              s_rc[tid] = theta;
              V.b_k[t] = found_k;
              go = true;
            }
          }
          if (go) {
            R.slot = (int32_t)t;
            double a4[4];
            start_shot<MODEL>(P, R, S, zs, zr, theta, a4);
#pragma unroll
            for (int i = 0; i < 4; ++i) s_amp[i][tid] = a4[i];
            mode = 0;
          }
        }
      }
    }
    if (__ballot(R.slot >= 0) == 0) {
      if (exhausted) break;
      continue;
    }
    if (R.slot < 0) continue;

    // ---- one Cash-Karp trial in every busy lane ----
    const bool stepping = mode == 0;
    const bool clipped = S.smax - R.s <= R.h;
    const double ht = stepping ? (clipped ? S.smax - R.s : R.h) : lc;
    double y5[7], err;
    trial<MODEL, 0>(P, R, ht, y5, err);

    bool located = false;
    double sig = 0.0;
    if (stepping) {
      bool finite = isfinite(err);
#pragma unroll
      for (int i = 0; i < 7; ++i) finite = finite && isfinite(y5[i]);
      const bool accept = err <= 1.0 || ht <= P.h_min;
      // as in the trace: a full-length step whose error allows growth stays
      // at h_max without the controller's power (same result)
      double hn = P.h_max;
      if (!(accept && err <= 0.5 && ht >= P.h_max))
        hn = clamp_h(P, ht * step_factor(err, accept));
      if (!finite) {
        fin = ShotEnd{RT_SHOT_LOST, kMissLost};
      } else if (!accept) {
        R.n_rej++;
        R.h = hn;
      } else {
        R.n_acc++;
        if (err > 1.0) C.bump(V_FORCED);
        if constexpr (MODEL == RT_MODEL_PAPER) {
          const double il = rsqrt_nr(fma(y5[3], y5[3], fma(y5[4], y5[4], y5[5] * y5[5])));
          y5[3] *= il;
          y5[4] *= il;
          y5[5] *= il;
        }
        double G0 = 0.0, G1 = 0.0;
        const int k = pick_crossing_shot(P, R.side, S.D, R.y, y5, ht, -1, G0, G1);
        if (k < 0) {
#pragma unroll
          for (int i = 0; i < 7; ++i) R.y[i] = y5[i];
          R.s = clipped ? S.smax : R.s + ht;
          R.h = hn;
        } else {
          s_hp[tid] = ht;
          s_hn[tid] = hn;
          s_k[tid] = k;
          s_meta[tid] = 1;
          // as in the trace: a shot standing on a plane and leaving it (after
          // a transmission or reflection) searches for its return from the
          // bracket value rate * len; the receiver plane is never left
          const bool on = on_boundary(G0);
          double rate = -1.0;
          if (__builtin_expect(on, 0) && k != kRecv)
            rate = bnd_rate(s_bnd[k], k, R.side, R.y);
          if (on && !(rate > 0.0)) {
            located = true;
            sig = 0.0;
#pragma unroll
            for (int i = 0; i < 7; ++i) y5[i] = R.y[i];
          } else {
            const double Ga = on ? rate * ht : G0;
            s_a[tid] = 0.0;
            s_Ga[tid] = Ga;
            s_b[tid] = ht;
            s_Gb[tid] = G1;
            lc = ht - G1 * ht / (G1 - Ga);
            mode = 1;
          }
        }
      }
    } else {
      // one iterate of the Illinois crossing search
      C.bump(V_RELOC);
      const int k = s_k[tid];
      const int meta = s_meta[tid];
      int last = (meta & 3) - 1;
      const int it = ((meta >> 2) & 0xff) + 1;
      double a = s_a[tid], Ga = s_Ga[tid], b = s_b[tid], Gb = s_Gb[tid];
      const double Gc = shot_G(P, k, R.side, S.D, y5);
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
        const int j = pass < kLocMaxPass
                          ? pick_crossing_shot(P, R.side, S.D, R.y, y5, sig, k, H0, H1)
                          : -1;
        if (j < 0) {
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
        double rate = -1.0;
        if (__builtin_expect(on, 0) && k != kRecv) rate = bnd_rate(s_bnd[k], k, R.side, R.y);
        if (on && !(rate > 0.0)) {
          sig = 0.0;
#pragma unroll
          for (int i = 0; i < 7; ++i) y5[i] = R.y[i];
          continue;
        }
        const double Ha = on ? rate * sig : H0;
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

    if (fin.status < 0 && mode == 0 &&
        (R.s >= S.smax || (int64_t)R.n_acc + R.n_rej >= P.max_steps))
      fin = ShotEnd{RT_SHOT_LOST, kMissLost};
    if (fin.status >= 0) mode = 0;
  }

  {
    unsigned long long a = s_sacc[tid], r = s_srej[tid];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      a += __shfl_xor(a, o);
      r += __shfl_xor(r, o);
    }
    if (lane == 0) {
      C.c[V_ACC] += a;
      C.c[V_REJ] += r;
    }
  }
  if (lane == 0) {
    for (int i = 0; i < V_COUNT; ++i)
      if (C.c[i]) atomicAdd(&V.stats[i], C.c[i]);
  }
}

template <int MODEL, int PHASE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
shot_kernel(KParams P, KSolve V) {
  shot_body<MODEL, PHASE>(P, V);
}

// Counters and statistics to their launch values.
__global__ void solve_reset_kernel(KSolve V) {
  const int i = threadIdx.x;
  if (i < V_COUNT) V.stats[i] = 0;
  if (i < 5) V.tickets[i] = 0;
}

// The admissible refined root with the smallest travel time, per (pair,
// family).
__global__ void select_kernel(KParams P, KSolve V) {
  const int64_t pf = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = V.n_dev ? *V.n_dev : V.n;
  if (pf >= 2 * n) return;
  const rt_solve_outputs& O = V.so;
  const int32_t pair = (int32_t)(pf >> 1);
  const int64_t n2 = 2 * n;
  int best = -1, nb = 0, last_k = -1, refine_shots = 0, roots = 0;
  double best_t = 0.0;
  const bool ok = pair_ok(P, V.zs[pair], V.zr[pair], V.dist[pair]);
  if (ok) {
    for (int b = 0; b < V.max_brackets; ++b) {
      const int64_t i = (int64_t)b * n2 + pf;
      const int32_t st = V.b_status[i];
      if (st < 0) break;
      ++nb;
      last_k = V.b_k[i];
      refine_shots += V.b_shots[i];
      const bool admissible = st == RT_SHOT_RECEIVER && fabs(V.b_miss[i]) <= V.accept_tol;
      roots += admissible ? 1 : 0;
      if (admissible && (best < 0 || V.b_t[i] < best_t)) {
        best = b;
        best_t = V.b_t[i];
      }
    }
  } else if ((pf & 1) == 0) {
    atomicAdd(&V.stats[V_INVALID], 1ull);
  }
  // shots of the sequential procedure: its scan stops at the bracket that
  // reaches max_brackets
  const int scan_shots = nb >= V.max_brackets ? last_k + 1 : V.n_scan;
  O.shots[pf] = ok ? scan_shots + refine_shots : 0;
  O.roots[pf] = roots;
  O.found[pf] = best >= 0;
  if (best >= 0) {
    const int64_t i = (int64_t)best * n2 + pf;
    O.theta[pf] = V.b_theta[i];
    O.miss[pf] = V.b_miss[i];
    O.t[pf] = V.b_t[i];
    O.s[pf] = V.b_s[i];
    O.as_re[pf] = V.b_as_re[i];
    O.as_im[pf] = V.b_as_im[i];
    O.ap_re[pf] = V.b_ap_re[i];
    O.ap_im[pf] = V.b_ap_im[i];
    atomicAdd(&V.stats[V_FOUND], 1ull);
  } else {
    O.theta[pf] = O.miss[pf] = O.t[pf] = O.s[pf] = 0.0;
    O.as_re[pf] = O.as_im[pf] = O.ap_re[pf] = O.ap_im[pf] = 0.0;
  }
}

// ===========================================================================
// Host side.
namespace {

template <int MODEL, int PHASE>
int shot_blocks_per_cu(int block) {
  static thread_local int cached[5] = {};
  int& c = cached[block / 64];
  if (c == 0) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nb, reinterpret_cast<const void*>(&shot_kernel<MODEL, PHASE>), block, 0) !=
            hipSuccess ||
        nb < 1)
      nb = 1;
    c = nb;
  }
  return c;
}

template <int PHASE>
int blocks_per_cu(int model, int block) {
  return model == RT_MODEL_PAPER ? shot_blocks_per_cu<RT_MODEL_PAPER, PHASE>(block)
                                 : shot_blocks_per_cu<RT_MODEL_EXACT, PHASE>(block);
}

template <int PHASE>
hipError_t launch_shots(const KParams& P, const KSolve& V, int n_cu, int block,
                        hipStream_t s) {
  if (V.n_tasks == 0) return hipSuccess;
  int64_t nblk = (int64_t)n_cu * blocks_per_cu<PHASE>(P.model, block);
  nblk = std::max<int64_t>(1, std::min(nblk, (V.n_tasks + block - 1) / block));
  if (P.model == RT_MODEL_PAPER)
    hipLaunchKernelGGL((shot_kernel<RT_MODEL_PAPER, PHASE>), dim3((unsigned)nblk), dim3(block),
                       0, s, P, V);
  else
    hipLaunchKernelGGL((shot_kernel<RT_MODEL_EXACT, PHASE>), dim3((unsigned)nblk), dim3(block),
                       0, s, P, V);
  return hipGetLastError();
}

// Stratified fields only: the shot kernels are built for the analytic media.
rt_status pack_params(const rt_field* field, const rt_boundaries* bnd, double tol,
                      const rt_step_limits* L, KParams& P) {
  if (field_uses_grid(field)) {
    set_last_error("solves support stratified (analytic) fields only");
    return RT_ERR_UNSUPPORTED;
  }
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
    k.use_grid = 0;
  }
  for (int i = 0; i < bnd->n_planes; ++i) {
    const rt_plane& p = bnd->planes[i];
    KBnd& b = P.bnd[i];
    const double len = sqrt(p.normal[0] * p.normal[0] + p.normal[1] * p.normal[1] +
                            p.normal[2] * p.normal[2]);
    for (int a = 0; a < 3; ++a) b.nrm[a] = p.normal[a] / len;
    b.d = p.point[0] * b.nrm[0] + p.point[1] * b.nrm[1] + p.point[2] * b.nrm[2];
    b.kind = p.kind == RT_PLANE_ABSORB ? B_ABSORB : B_FRESNEL;
    b.reg_pos = p.region_pos;
    b.reg_neg = p.region_neg;
  }
  P.n_bnd = bnd->n_planes;
  P.model = L->model;
  P.max_gen = 1;
  P.tol = tol;
  P.inv_tol = 1.0 / tol;
  P.h_min = L->h_min;
  P.h_max = L->h_max;
  P.h_init = L->h_init > 0.0 ? L->h_init : L->h_max;
  P.max_steps = L->max_steps_per_ray;
  return RT_OK;
}

struct DeviceCU {
  int device = -1;
  int n_cu = 0;
};
thread_local DeviceCU g_cu;

rt_status device_cus(int& n_cu) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess && g_cu.device != dev) {
    int ncu = 0;
    e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) {
      g_cu.device = dev;
      g_cu.n_cu = ncu;
    }
  }
  if (e != hipSuccess) {
    set_last_error("device query: %s", hipGetErrorString(e));
    return RT_ERR_DEVICE;
  }
  n_cu = g_cu.n_cu;
  return RT_OK;
}

rt_status check_pairs_outputs(const rt_pairs* pairs, const rt_solve_outputs* out) {
  if (pairs->n < 0 || pairs->n > ((int64_t)1 << 28)) {
    set_last_error("pair count must be 0..2^28");
    return RT_ERR_INVALID_ARG;
  }
  if (pairs->n > 0 && (!pairs->zs || !pairs->zr || !pairs->dist)) {
    set_last_error("null pair array");
    return RT_ERR_INVALID_ARG;
  }
  if (pairs->n > 0 && (!out->found || !out->shots || !out->roots || !out->theta || !out->miss ||
                       !out->t || !out->s || !out->as_re || !out->as_im || !out->ap_re ||
                       !out->ap_im)) {
    set_last_error("null output array");
    return RT_ERR_INVALID_ARG;
  }
  return RT_OK;
}

rt_status tuning_of(const rt_tuning* tuning, int& block, int& refill, int& chunk,
                    int* fused = nullptr) {
  block = tuning && tuning->block_size ? tuning->block_size : 256;
  if (block < 64 || block > 256 || block % 64) {
    set_last_error("block_size must be 64, 128, 192 or 256");
    return RT_ERR_INVALID_ARG;
  }
  refill = tuning && tuning->refill_threshold ? tuning->refill_threshold : 16;
  if (refill < 1 || refill > 64) {
    set_last_error("refill_threshold must be 1..64");
    return RT_ERR_INVALID_ARG;
  }
  chunk = tuning && tuning->scan_chunk ? tuning->scan_chunk : 1;
  if (chunk < 1 || chunk > 4096) {
    set_last_error("scan_chunk must be 1..4096");
    return RT_ERR_INVALID_ARG;
  }
  const int sf = tuning ? tuning->solve_fused : 0;
  if (sf != 0 && sf != 1) {
    set_last_error("solve_fused must be 0 (three launches) or 1 (one fused launch)");
    return RT_ERR_INVALID_ARG;
  }
  if (fused) *fused = sf;
  return RT_OK;
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

// Enqueue a solve of up to n_cap pairs (the number read on the device from
// *n_dev when n_dev is not NULL); arguments already validated.
rt_status solve_enqueue(const rt_field* field, const rt_boundaries* bnd, double tol,
                        const rt_step_limits* L, const rt_pairs* pairs, int64_t n_cap,
                        const int64_t* n_dev, const uint8_t* fam_mask,
                        const rt_solve_params* prm, const rt_solve_outputs* out, void* workspace,
                        void* stream, const rt_tuning* tuning) {
  rt_status st;
  int block = 0, refill = 0, chunk = 0, want_fused = 0, n_cu = 0;
  if ((st = tuning_of(tuning, block, refill, chunk, &want_fused)) != RT_OK) return st;
  KParams P;
  if ((st = pack_params(field, bnd, tol, L, P)) != RT_OK) return st;
  if ((st = device_cus(n_cu)) != RT_OK) return st;

  const int64_t n = n_cap, K = prm->n_scan, B = prm->max_brackets;
  const bool fused = want_fused && K <= kFScan && B <= kFBr;
  // a lane holds its task index in 32 bits
  if (2 * n * std::max(K, B) > (int64_t)0x7fffffff) {
    set_last_error("pairs x 2 x max(n_scan, max_brackets) = %lld exceeds 2^31 - 1 tasks",
                   (long long)(2 * n * std::max(K, B)));
    return RT_ERR_UNSUPPORTED;
  }
  KSolve V;
  memset(&V, 0, sizeof V);
  V.zs = pairs->zs;
  V.zr = pairs->zr;
  V.dist = pairs->dist;
  V.n = n;
  V.n_dev = n_dev;
  V.fam_mask = fam_mask;
  V.scan_chunk = chunk;
  V.n_scan = prm->n_scan;
  V.max_iter = prm->max_iter;
  V.max_brackets = prm->max_brackets;
  V.refill = refill;
  V.miss_tol = prm->miss_tol;
  V.accept_tol = prm->accept_tol;
  V.slope_max = prm->slope_max;
  V.dtheta = kPi / (double)prm->n_scan;
  char* w = static_cast<char*>(workspace);
  V.tickets = reinterpret_cast<uint64_t*>(w);
  V.stats = reinterpret_cast<unsigned long long*>(out->stats);
  size_t off = 4096;
  V.scan_miss = reinterpret_cast<double*>(w + off);
  off += ((size_t)(2 * n * K) * 8 + 4095) / 4096 * 4096;
  const size_t nb = (size_t)(2 * n * B);
  double** f64[] = {&V.b_theta, &V.b_miss, &V.b_t, &V.b_s,
                    &V.b_as_re, &V.b_as_im, &V.b_ap_re, &V.b_ap_im};
  for (double** p : f64) {
    *p = reinterpret_cast<double*>(w + off);
    off += nb * 8;
  }
  int32_t** i32[] = {&V.b_status, &V.b_shots, &V.b_k};
  for (int32_t** p : i32) {
    *p = reinterpret_cast<int32_t*>(w + off);
    off += nb * 4;
  }
  V.so = *out;

  hipStream_t s = static_cast<hipStream_t>(stream);
  Range range("raytrace_solve: scan, refine, select");
  hipLaunchKernelGGL(solve_reset_kernel, dim3(1), dim3(64), 0, s, V);
  HIP_TRY(hipGetLastError());
  if (n == 0) return RT_OK;
  V.n_tasks = 2 * n * K;
  if (tuning && tuning->ev_trace_begin)
    HIP_TRY(hipEventRecord(static_cast<hipEvent_t>(tuning->ev_trace_begin), s));
  if (fused) {
    HIP_TRY(launch_shots<PH_FUSED>(P, V, n_cu, block, s));
    if (tuning && tuning->ev_trace_end)
      HIP_TRY(hipEventRecord(static_cast<hipEvent_t>(tuning->ev_trace_end), s));
    return RT_OK;
  }
  HIP_TRY(launch_shots<PH_SCAN>(P, V, n_cu, block, s));
  V.n_tasks = 2 * n * B;
  HIP_TRY(launch_shots<PH_REFINE>(P, V, n_cu, block, s));
  if (tuning && tuning->ev_trace_end)
    HIP_TRY(hipEventRecord(static_cast<hipEvent_t>(tuning->ev_trace_end), s));
  hipLaunchKernelGGL(select_kernel, dim3((unsigned)((2 * n + 255) / 256)), dim3(256), 0, s, P,
                     V);
  HIP_TRY(hipGetLastError());
  return RT_OK;
}

// Enqueue the seeded secant of every entry [2 n] with seed_try set; results
// into out (found = verified), verify[2 n] = 1 / 0 for the tried entries.
// The workspace needs 4 KiB.
rt_status seeded_enqueue(const rt_field* field, const rt_boundaries* bnd, double tol,
                         const rt_step_limits* L, const rt_pairs* pairs, const double* seed,
                         const int32_t* seed_try, const rt_surrogate_params* sp,
                         const rt_solve_outputs* out, int32_t* verify, void* workspace,
                         void* stream, const rt_tuning* tuning) {
  rt_status st;
  int block = 0, refill = 0, chunk = 0, n_cu = 0;
  if ((st = tuning_of(tuning, block, refill, chunk)) != RT_OK) return st;
  KParams P;
  if ((st = pack_params(field, bnd, tol, L, P)) != RT_OK) return st;
  if ((st = device_cus(n_cu)) != RT_OK) return st;
  KSolve V;
  memset(&V, 0, sizeof V);
  V.zs = pairs->zs;
  V.zr = pairs->zr;
  V.dist = pairs->dist;
  V.n = pairs->n;
  V.n_tasks = 2 * pairs->n;
  V.refill = refill;
  V.tickets = static_cast<uint64_t*>(workspace);
  V.stats = reinterpret_cast<unsigned long long*>(out->stats);
  V.so = *out;
  V.seed = seed;
  V.seed_try = seed_try;
  V.verify = verify;
  V.verify_tol = sp->verify_tol;
  V.dseed = sp->dseed;
  V.max_shots = sp->max_shots;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Range range("raytrace_solve_seeded: seeded secant");
  hipLaunchKernelGGL(solve_reset_kernel, dim3(1), dim3(64), 0, s, V);
  HIP_TRY(hipGetLastError());
  HIP_TRY(launch_shots<PH_SEEDED>(P, V, n_cu, block, s));
  return RT_OK;
}

}  // namespace rt

extern "C" rt_status raytrace_solve(const rt_field* field, const rt_boundaries* bnd, double tol,
                                    const rt_step_limits* L, const rt_pairs* pairs,
                                    const rt_solve_params* prm, rt_solve_outputs* out,
                                    void* workspace, size_t workspace_bytes, void* stream,
                                    const rt_tuning* tuning) {
  using namespace rt;
  rt_status st = rt_solve_validate(field, bnd, tol, L, prm);
  if (st != RT_OK) return st;
  if (!prm || !pairs || !out || !out->stats || !workspace) {
    set_last_error("null params, pairs, outputs, stats or workspace");
    return RT_ERR_INVALID_ARG;
  }
  if ((st = check_pairs_outputs(pairs, out)) != RT_OK) return st;
  size_t need = 0;
  st = rt_solve_workspace_bytes(field, pairs->n, prm, &need);
  if (st != RT_OK) return st;
  if (workspace_bytes < need) {
    set_last_error("workspace of %zu bytes < %zu needed", workspace_bytes, need);
    return RT_ERR_INVALID_ARG;
  }
  return solve_enqueue(field, bnd, tol, L, pairs, pairs->n, nullptr, nullptr, prm, out,
                       workspace, stream, tuning);
}

extern "C" rt_status raytrace_solve_seeded(const rt_field* field, const rt_boundaries* bnd,
                                           double tol, const rt_step_limits* L,
                                           const rt_pairs* pairs, const double* seed,
                                           const int32_t* seed_try,
                                           const rt_surrogate_params* sp, rt_solve_outputs* out,
                                           int32_t* verify, void* workspace,
                                           size_t workspace_bytes, void* stream,
                                           const rt_tuning* tuning) {
  using namespace rt;
  rt_status st = rt_solve_validate(field, bnd, tol, L, nullptr);
  if (st != RT_OK) return st;
  if (!pairs || !out || !out->stats || !workspace || !sp) {
    set_last_error("null pairs, params, outputs, stats or workspace");
    return RT_ERR_INVALID_ARG;
  }
  if ((st = check_pairs_outputs(pairs, out)) != RT_OK) return st;
  if ((st = check_surrogate_params(sp)) != RT_OK) return st;
  if (pairs->n > 0 && (!seed || !seed_try || !verify)) {
    set_last_error("null seed, seed_try or verify array");
    return RT_ERR_INVALID_ARG;
  }
  if (workspace_bytes < 4096) {
    set_last_error("workspace of %zu bytes < 4096 needed", workspace_bytes);
    return RT_ERR_INVALID_ARG;
  }
  return seeded_enqueue(field, bnd, tol, L, pairs, seed, seed_try, sp, out, verify, workspace,
                        stream, tuning);
}

extern "C" rt_status raytrace_shoot(const rt_field* field, const rt_boundaries* bnd, double tol,
                                    const rt_step_limits* L, const rt_shots* shots,
                                    rt_shot_outputs* out, void* workspace,
                                    size_t workspace_bytes, void* stream,
                                    const rt_tuning* tuning) {
  using namespace rt;
  rt_status st = rt_solve_validate(field, bnd, tol, L, nullptr);
  if (st != RT_OK) return st;
  if (!shots || !out || !out->stats || !workspace) {
    set_last_error("null shots, outputs, stats or workspace");
    return RT_ERR_INVALID_ARG;
  }
  if (shots->n < 0 || shots->n > (int64_t)0x7fffffff) {
    set_last_error("shot count must be 0..2^31-1");
    return RT_ERR_INVALID_ARG;
  }
  if (shots->n > 0 && (!shots->zs || !shots->zr || !shots->dist || !shots->theta ||
                       !shots->family || !out->status || !out->n_acc || !out->n_rej ||
                       !out->miss || !out->t || !out->s || !out->as_re || !out->as_im ||
                       !out->ap_re || !out->ap_im)) {
    set_last_error("null shot or output array");
    return RT_ERR_INVALID_ARG;
  }
  size_t need = 0;
  st = rt_solve_workspace_bytes(field, 0, nullptr, &need);
  if (st != RT_OK) return st;
  if (workspace_bytes < need) {
    set_last_error("workspace of %zu bytes < %zu needed", workspace_bytes, need);
    return RT_ERR_INVALID_ARG;
  }
  int block = 0, refill = 0, chunk = 0, n_cu = 0;
  if ((st = tuning_of(tuning, block, refill, chunk)) != RT_OK) return st;
  KParams P;
  if ((st = pack_params(field, bnd, tol, L, P)) != RT_OK) return st;
  if ((st = device_cus(n_cu)) != RT_OK) return st;

  KSolve V;
  memset(&V, 0, sizeof V);
  V.zs = shots->zs;
  V.zr = shots->zr;
  V.dist = shots->dist;
  V.theta = shots->theta;
  V.family = shots->family;
  V.n = shots->n;
  V.n_tasks = shots->n;
  V.refill = refill;
  V.tickets = static_cast<uint64_t*>(workspace);
  V.stats = reinterpret_cast<unsigned long long*>(out->stats);
  V.lo = *out;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(solve_reset_kernel, dim3(1), dim3(64), 0, s, V);
  HIP_TRY(hipGetLastError());
  if (tuning && tuning->ev_trace_begin)
    HIP_TRY(hipEventRecord(static_cast<hipEvent_t>(tuning->ev_trace_begin), s));
  HIP_TRY(launch_shots<PH_LIST>(P, V, n_cu, block, s));
  if (tuning && tuning->ev_trace_end)
    HIP_TRY(hipEventRecord(static_cast<hipEvent_t>(tuning->ev_trace_end), s));
  return RT_OK;
}

extern "C" rt_status rt_solve_autotune(const rt_field* field, const rt_boundaries* bnd,
                                       double tol, const rt_step_limits* L,
                                       const rt_pairs* pairs, const rt_solve_params* prm,
                                       rt_solve_outputs* out, void* workspace,
                                       size_t workspace_bytes, void* stream, rt_tuning* best,
                                       float* best_ms) {
  using namespace rt;
  if (!best) {
    set_last_error("null tuning output");
    return RT_ERR_INVALID_ARG;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    set_last_error("hipEventCreate failed");
    return RT_ERR_DEVICE;
  }
  static const int kBlocks[] = {64, 128, 192, 256};
  static const int kRefill[] = {4, 16, 32, 64};
  static const int kChunks[] = {1, 4, 16, 64};
  rt_status st = RT_OK;
  float best_t = -1.0f;
  rt_tuning cand;
  memset(&cand, 0, sizeof cand);
  // one untimed call first (code load, caches)
  cand.block_size = 256;
  cand.refill_threshold = 16;
  cand.scan_chunk = 1;
  st = raytrace_solve(field, bnd, tol, L, pairs, prm, out, workspace, workspace_bytes, stream,
                      &cand);
  // each candidate is timed twice and its faster run counts (the launch
  // tunings differ by a few per cent, about the spread of single runs)
  auto trial = [&](const rt_tuning& c) {
    float best_c = -1.0f;
    for (int rep = 0; rep < 2 && st == RT_OK; ++rep) {
      hipError_t e = hipEventRecord(e0, s);
      if (e == hipSuccess)
        st = raytrace_solve(field, bnd, tol, L, pairs, prm, out, workspace, workspace_bytes,
                            stream, &c);
      if (e == hipSuccess && st == RT_OK) e = hipEventRecord(e1, s);
      if (e == hipSuccess && st == RT_OK) e = hipEventSynchronize(e1);
      float ms = 0.0f;
      if (e == hipSuccess && st == RT_OK) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) {
        set_last_error("autotune timing: %s", hipGetErrorString(e));
        st = RT_ERR_DEVICE;
        return;
      }
      if (st == RT_OK && (best_c < 0.0f || ms < best_c)) best_c = ms;
    }
    if (st == RT_OK && (best_t < 0.0f || best_c < best_t)) {
      best_t = best_c;
      *best = c;
    }
  };
  // three launches: block size x refill threshold with each entry's scan
  // in one piece, then the scan interleave at the best of those; then the
  // fused launch at each block size (where the scan fits it)
  for (int bi = 0; st == RT_OK && bi < 4; ++bi)
    for (int ri = 0; st == RT_OK && ri < 4; ++ri) {
      cand.block_size = kBlocks[bi];
      cand.refill_threshold = kRefill[ri];
      trial(cand);
    }
  for (int ci = 1; st == RT_OK && ci < 4; ++ci) {
    cand = *best;
    cand.scan_chunk = kChunks[ci];
    trial(cand);
  }
  const bool fusable = prm && prm->n_scan <= kFScan && prm->max_brackets <= kFBr;
  for (int bi = 0; st == RT_OK && fusable && bi < 4; ++bi) {
    memset(&cand, 0, sizeof cand);
    cand.block_size = kBlocks[bi];
    cand.refill_threshold = 16;
    cand.solve_fused = 1;
    trial(cand);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st == RT_OK && best_ms) *best_ms = best_t;
  return st;
}
