// Launch parameters shared by the host launcher and the kernels.  Passed to
// the kernels by value (kernel-argument segment), so every field is plain data.
#pragma once
#include <stdint.h>

#include "radiotrace.h"

namespace rt {

// user planes, then 6 box faces, then the travel-time pseudo-boundary
constexpr int kMaxBnd = RT_MAX_PLANES + 6 + 1;
enum BndKind : int32_t { B_FRESNEL = 0, B_ABSORB = 1, B_BOX = 2, B_TIME = 3 };

// n = a + b zeta - dn exp(-zeta / z0), zeta = ax . r (unit axis; depth in the
// stratified kernel); exp is skipped when dn == 0
struct KRegion {
  double a, b, dn, inv_z0, dn_inv_z0;
  double z_top, z_bot;  // launch-region lookup: z_top <= z < z_bot
  int32_t use_grid, pad;
  double ax[3];
};

// Gaussian anomaly amp exp(-k |r - c|^2), k = 1 / (2 sigma^2), in one region
struct KAnom {
  double c[3];
  double amp, k;
  int32_t region, pad;
};

// Boundary surface, positive g on the region_pos side:
//   plane       g = r . nrm - d (unit normal)
//   sphere      g = |r - nrm| - d (centre nrm, radius d)
//   paraboloid  g = z - nrm[2] - d ((x - nrm[0])^2 + (y - nrm[1])^2)
//               (vertex nrm, curvature d)
enum ShapeKind : int32_t { SH_PLANE = 0, SH_SPHERE = 1, SH_PARABOLOID = 2 };
struct KBnd {
  double nrm[3];
  double d;
  int32_t kind, reg_pos, reg_neg, shape;
};

struct Pool {
  double *x, *y, *z, *ux, *uy, *uz, *s, *t;
  double *as_re, *as_im, *ap_re, *ap_im, *h;
  uint64_t *key, *parent;
  int32_t *gen, *status, *n_acc, *n_rej, *n_ev, *region;
  uint32_t* side;
};

struct QueueCounters {
  uint64_t head;      // next primary to hand out
  uint64_t tail;      // record slots reserved so far (primaries, secondaries, chunks)
  uint64_t gq_head;   // next overflow-queue ticket
  uint64_t gq_tail;   // overflow-queue entries reserved
  uint64_t finished;  // rays finished plus reserved slots idle waves will not use
  uint64_t dropped;   // secondaries that found no slot below capacity
  uint64_t fix_a;     // slot compaction: holes below the record count
  uint64_t fix_b;     // slot compaction: records at or above it
  uint64_t steps;     // trial steps of this launch (added every 64 wave iterations)
  uint64_t stop;      // 1 once the step budget is reached
  uint64_t holes;     // slot compaction: empty slots among the secondaries
  uint64_t ev_tail;   // event records reserved so far
};

struct KParams {
  KRegion reg[RT_MAX_REGIONS];
  KBnd bnd[kMaxBnd];
  int32_t n_regions, n_bnd;
  int32_t model, max_gen;
  KAnom anom[RT_MAX_ANOMALIES];
  int32_t n_anom, pad_anom;
  // grid: float4 nodes (n, Dx, Dy, Dz) with grad n = D / (2 spacing)
  const void* nodes;
  int32_t gnx, gny, gnz, refill;
  int32_t gbx, gby, gbz, pad_g;  // bricks of 2 x 2 x 2 nodes along x, y, z
  uint32_t local_limit;  // children a wave keeps before publishing globally
  uint32_t chunk;        // secondary slots a wave reserves at once (0: one per child)
  uint64_t chunk_limit;  // waves stop taking chunks once they reach this slot
  uint64_t reserve;      // slots chunks can leave unused (waves x chunk)
  double gorg[3], ginv[3], gmax[3], ghalf[3];
  // limits
  double tol, inv_tol, h_min, h_max, h_init, s_max, t_max, amp_min;
  int64_t max_steps;
  int64_t budget;  // trial steps per launch, 0 = no limit
  // record pool (= caller's outputs)
  Pool pool;
  int64_t capacity, n_primary;
  rt_event* events;     // optional event records (ev_capacity > 0)
  int64_t ev_capacity;
  QueueCounters* q;
  int32_t* gq;  // overflow queue: record slots of published secondaries, -1 = not yet
  int32_t* perm;  // hand-out order of the primaries: ticket -> record slot
  rt_stats* stats;
};

// A ROCTx range over a host scope (rocprofv3 --marker-trace shows it on the
// calling thread's timeline): the enqueue phases of the entry points.
struct Range {
  explicit Range(const char* name);
  ~Range();
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};

// Host helpers shared by the launcher (rt_launch.hip) and rt_host.cpp.
void set_last_error(const char* fmt, ...);
rt_status validate(const rt_field* field, const rt_boundaries* boundaries,
                   const rt_sources* sources, const rt_directions* directions,
                   double tol, const rt_step_limits* limits);
bool field_uses_grid(const rt_field* field);
// true unless every region is analytic along +z and there are no anomalies
bool field_is_general(const rt_field* field);

}  // namespace rt
