/*
 * radiotrace -- FP64 eikonal ray tracing on MI355X (gfx950).
 *
 * C ABI of the GPU library.  It traces very many rays through an analytic
 * (stratified along any axis, with Gaussian anomalies) or gridded
 * refractive-index field with adaptive Cash-Karp Runge-Kutta 4(5) steps, and
 * handles media boundaries (planes, spheres, paraboloids) where a ray is
 * reflected and a refracted secondary ray is cast, both carrying Fresnel
 * amplitudes.  This is the method of RadioPropa (T. Winchen,
 * arXiv:1810.01780), section 2:
 *   - eq. 2, the locally paraxial ray equation n d2r/ds2 = grad n, is the
 *     default model (RT_MODEL_PAPER); eq. 1, the full eikonal
 *     d/ds (n dr/ds) = grad n, is RT_MODEL_EXACT;
 *   - the Cash-Karp solver with a tolerance and a minimum step length as the
 *     free accuracy parameters (section 2, accuracy discussion);
 *   - boundaries defined explicitly and handled apart from the propagation:
 *     reflection, a refracted secondary cast from the intersection point,
 *     Fresnel amplitudes (section 2, boundary paragraph); gridded data,
 *     fields given by formulas and curved boundaries (section 2, set-ups
 *     after the example);
 *   - travel-time and amplitude limits (Fig. 1 example); amplitudes are not
 *     corrected for path length (Fig. 1 caption).
 *
 * Coordinates: right-handed, z is DEPTH (positive downward); the surface of
 * the example media is the plane z = 0 with air at z < 0.  Lengths in metres,
 * times in seconds.
 *
 * Conventions for every entry point:
 *   - Descriptor structs are read on the host during the call and not kept.
 *   - Array pointers inside descriptors are DEVICE pointers (hipMalloc'ed or
 *     torch CUDA tensors) unless the field comment says "host".
 *   - The caller owns every buffer.  The library never allocates memory the
 *     caller can see; raytrace_launch allocates nothing at all (its scratch
 *     memory is the caller-provided workspace).
 *   - No C++ exception crosses the ABI.  Functions return rt_status; on a
 *     non-OK status rt_last_error() holds a message for the calling thread.
 */
#ifndef RADIOTRACE_H
#define RADIOTRACE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RT_ABI_VERSION 8
#define RT_MAX_REGIONS 8
#define RT_MAX_PLANES 16
#define RT_MAX_ANOMALIES 8
#define RT_MAX_GENERATIONS 4 /* ray keys hold three 8-bit event ordinals */

typedef enum {
  RT_OK = 0,
  RT_ERR_INVALID_ARG = 1, /* bad descriptor, or rays flagged RT_ST_INVALID */
  RT_ERR_CAPACITY = 2,    /* more records than out->capacity; see stats.needed */
  RT_ERR_DEVICE = 3,      /* a HIP call failed; message in rt_last_error() */
  RT_ERR_UNSUPPORTED = 4, /* e.g. more than RT_MAX_GENERATIONS generations */
  RT_INTERRUPTED = 5      /* the launch reached max_steps_per_launch; relaunch
                             with resume = 1 to continue */
} rt_status;

enum { RT_MODEL_PAPER = 0, RT_MODEL_EXACT = 1 };
enum { RT_PLANE_FRESNEL = 0, RT_PLANE_ABSORB = 1 };
enum { RT_SHAPE_PLANE = 0, RT_SHAPE_SPHERE = 1, RT_SHAPE_PARABOLOID = 2 };

/* Per-record status (out->status). */
enum {
  RT_ST_PARKED = -2,   /* internal: a ray stopped mid-flight by an
                          interrupted launch, resumed by the next one */
  RT_ST_QUEUED = -1,   /* internal: slot holds a ray waiting to be traced */
  RT_ST_EMPTY = 0,     /* internal: slot not written */
  RT_ST_PATH = 1,      /* reached the path-length limit s_max */
  RT_ST_BOX = 2,       /* crossed a face of the bounding box */
  RT_ST_TIME = 3,      /* reached the travel-time limit t_max */
  RT_ST_AMP = 4,       /* max(|A_s|, |A_p|) fell below amp_min */
  RT_ST_ABSORB = 5,    /* crossed an RT_PLANE_ABSORB plane */
  RT_ST_STEPCAP = 6,   /* step budget or 255 boundary events exhausted */
  RT_ST_NONFINITE = 7, /* NaN or Inf appeared in the state */
  RT_ST_INVALID = 8    /* bad input ray: zero/non-finite direction, source
                          index out of range, source within 1e-9 m of a plane
                          or outside the box; not traced */
};

/* One medium.  Analytic: n = a + b*zeta - dn*exp(-zeta/z0) with
 * zeta = k . r, k = axis/|axis| the stratification direction; an all-zero
 * axis means depth, zeta = z.  This covers the paper's firn profile
 * n0 - dn*exp(-depth/z0) (section 2), linear and constant media, and layers
 * stratified along any direction (section 2 lists analytic fields beyond
 * depth profiles).  use_grid != 0: n comes from rt_field.grid (axis
 * unused).  Gaussian anomalies (rt_field.anomalies) naming the region add
 * to either.  [z_top, z_bot) is used only to pick the region a primary ray
 * starts in, by its depth z. */
typedef struct {
  double a, b, dn, z0;
  double z_top, z_bot;
  int32_t use_grid;
  double axis[3];
} rt_region;

/* Gaussian refractive-index anomaly amplitude * exp(-|r - centre|^2 /
 * (2 sigma^2)), added to the index of one region (a lens where amplitude >
 * 0, a low-index pocket where it is < 0).  sigma > 0. */
typedef struct {
  double centre[3];
  double amplitude, sigma;
  int32_t region;
} rt_anomaly;

/* Gridded refractive index (section 2 mentions gridded data): FP32 values
 * n[k][j][i] at origin + (i, j, k) * spacing, x fastest.  n is trilinearly
 * interpolated; grad n is the trilinear interpolation of node gradients
 * taken by central differences (one-sided at the edges).  The node
 * differences are formed in FP32, which is exact when all values lie within
 * a factor of two of each other (true for refractive indices in [1, 2)).
 * Positions outside the grid are clamped onto it.  nx, ny, nz >= 2, and
 * the prepared nodes (16 bytes each, in 2 x 2 x 2 bricks) under 4 GiB:
 * ceil(nx/2) ceil(ny/2) ceil(nz/2) x 128 < 2^32 (about 2.7e8 nodes;
 * RT_ERR_UNSUPPORTED beyond). */
typedef struct {
  const float* n; /* device, nz*ny*nx floats */
  int32_t nx, ny, nz;
  double origin[3], spacing[3];
} rt_grid;

/* Fields that are not stratified in depth (a grid, an axis other than
 * +z, anomalies) run on the general 3-D gradient kernel; depth-stratified
 * fields on the kernel specialised for them.  Solves take depth-stratified
 * fields only. */
typedef struct {
  int32_t n_regions;          /* 1..RT_MAX_REGIONS */
  const rt_region* regions;   /* host */
  rt_grid grid;               /* used when any region has use_grid */
  int32_t n_anomalies;        /* 0..RT_MAX_ANOMALIES */
  const rt_anomaly* anomalies; /* host; may be NULL when n_anomalies == 0 */
} rt_field;

/* A boundary surface (section 2: boundaries are defined explicitly; curved
 * boundaries are among the supported shapes).  region_pos is the medium on
 * the side its normal points to, region_neg the other one; a ray refracted
 * through it continues in the other medium.  Stage evaluations of a step
 * always use the ray's own medium, extended smoothly across the surface;
 * the crossing itself is found by the event search, and the reflection and
 * refraction use the local normal at the crossing.
 *   RT_SHAPE_PLANE       through point with normal (any length > 0)
 *   RT_SHAPE_SPHERE      centre point, radius param > 0; region_pos outside
 *   RT_SHAPE_PARABOLOID  z = point[2] + param ((x - point[0])^2 +
 *                        (y - point[1])^2), param != 0; region_pos below it
 *                        (larger depth); normal unused for curved shapes.
 * A zero-initialised shape/param gives a plane. */
typedef struct {
  double point[3], normal[3];
  int32_t region_pos, region_neg;
  int32_t kind;  /* RT_PLANE_FRESNEL or RT_PLANE_ABSORB */
  int32_t shape; /* RT_SHAPE_* */
  double param;  /* sphere radius or paraboloid curvature (1/m) */
} rt_plane;

typedef struct {
  int32_t n_planes;       /* 0..RT_MAX_PLANES */
  const rt_plane* planes; /* host */
  int32_t has_box;        /* rays end (RT_ST_BOX) on leaving [box_lo, box_hi] */
  double box_lo[3], box_hi[3];
} rt_boundaries;

typedef struct {
  const double* xyz; /* device, [n][3] source positions */
  int32_t n;
} rt_sources;

typedef struct {
  const double* xyz;  /* device, [n][3] launch directions (any length > 0) */
  const int32_t* src; /* device, [n] source index of each ray */
  int64_t n;          /* number of primary rays, >= 0 */
} rt_directions;

typedef struct {
  double h_min;   /* minimum step: a trial at h <= h_min is always accepted */
  double h_max;   /* maximum step */
  double h_init;  /* first step of a primary ray; 0 means h_max */
  double s_max;   /* path-length limit (> 0) */
  double t_max;   /* travel-time limit, 0 = off */
  double amp_min; /* amplitude cut, 0 = off */
  int32_t max_generations; /* 1 = primaries only ... 4 */
  int32_t model;           /* RT_MODEL_PAPER or RT_MODEL_EXACT */
  int64_t max_steps_per_ray; /* accepted + rejected trials per ray, >= 1 */
  int64_t max_steps_per_launch; /* 0 = off; else the launch stops after about
                                   this many trial steps (the waves check
                                   every 64 iterations), parks the rays in
                                   flight in their record slots and reports
                                   RT_INTERRUPTED */
  int32_t resume; /* 1: continue an interrupted launch: same descriptors,
                     outputs and workspace, none of them changed since; the
                     records and statistics then accumulate as if the launches
                     were one.  Results equal those of an uninterrupted launch
                     bit for bit. */
} rt_step_limits;

/* Launch statistics, accumulated on the device into out->stats. */
typedef struct {
  int64_t accepted;   /* accepted steps (the throughput unit) */
  int64_t rejected;   /* rejected trial steps */
  int64_t relocation; /* trial steps spent locating boundary crossings */
  int64_t forced;     /* steps accepted at h_min above tolerance */
  int64_t events;     /* Fresnel boundary events */
  int64_t spawned;    /* refracted secondaries created */
  int64_t suppressed_gen; /* secondaries not created: generation limit */
  int64_t suppressed_amp; /* secondaries not created: amplitude cut */
  int64_t records;    /* records written (rays finished) */
  int64_t needed;     /* records the launch needs: primaries + spawned; when
                         some secondaries found no slot below capacity, plus
                         the scheduler's reserve (64 slots per wave of the
                         launch), which a relaunch with capacity >= needed
                         always holds */
  int64_t nonfinite;  /* rays ended RT_ST_NONFINITE */
  int64_t max_gen;    /* highest generation traced */
  int64_t invalid;    /* primary rays flagged RT_ST_INVALID */
  int64_t refills;    /* wave refill operations of the scheduler */
  int64_t sched_errors; /* scheduler waits that timed out (must stay 0) */
  int64_t spilled;    /* secondaries handed to other waves (global queue) */
  int64_t interrupted; /* 1: this launch stopped at max_steps_per_launch */
  int64_t events_lost; /* event records that did not fit out->ev_capacity */
  int64_t max_queue;  /* largest backlog of secondaries waiting on one wave's
                         own queue (at most the local queue length) */
} rt_stats;

/* Outcome of a Fresnel event for its transmitted branch. */
enum {
  RT_EV_SPAWNED = 0, /* a refracted secondary was cast */
  RT_EV_TIR = 1,     /* total internal reflection: nothing is transmitted */
  RT_EV_GEN = 2,     /* not cast: the secondary would exceed max_generations */
  RT_EV_AMP = 3      /* not cast: its amplitude is below amp_min */
};

/* Optional record of one Fresnel boundary event, the interaction section 2
 * describes for a ray passing a boundary: the ray is reflected (it keeps its
 * key and continues) and a refracted secondary is cast from the crossing
 * point, both with amplitudes scaled by Fresnel's coefficients.  Events at
 * absorbing boundaries, box faces and the travel-time limit end the ray and
 * are not recorded here (the final record holds them).  216 bytes. */
typedef struct {
  uint64_t key;       /* key of the ray that met the boundary */
  int32_t ordinal;    /* its event count including this event, 1..255; a
                         secondary cast here has key
                         key | ordinal << (8 * (2 - gen)) */
  int32_t boundary;   /* index into rt_boundaries.planes */
  int32_t outcome;    /* RT_EV_* */
  int32_t gen;        /* generation of the ray */
  int32_t region_in;  /* medium of the ray */
  int32_t region_out; /* medium beyond the boundary */
  double pos[3];      /* crossing point, on the boundary */
  double dir[3];      /* incident unit direction */
  double s, t;        /* path length and travel time at the crossing */
  double cos_i;       /* cosine of the angle of incidence */
  double n1, n2;      /* refractive index of region_in and region_out there */
  double amp[4];      /* incident amplitudes: as_re, as_im, ap_re, ap_im */
  double coef[8];     /* Fresnel coefficients as (re, im) pairs: r_s, r_p,
                         t_s, t_p (t = 0 under total internal reflection);
                         the reflected ray's amplitudes are amp * r, the
                         secondary's amp * t */
} rt_event;

/* Caller-owned output records, one per ray (primary or secondary), in no
 * particular order, in slots [0, records + invalid) (primaries first, in
 * slots [0, n)); 'key' identifies a ray deterministically: bits 24..55
 * hold the primary index, bits 16..23 / 8..15 / 0..7 the parent's event
 * ordinal (1..255) at which the generation-1 / -2 / -3 ancestor was cast.
 * All arrays are device arrays of 'capacity' elements.  x,y,z: final
 * position; ux,uy,uz: final unit direction; s: path length; t: travel time;
 * as_*, ap_*: complex s- and p-polarised amplitude factors (start 1 + 0i);
 * h: last proposed step; parent: key of the ray that cast it (~0 for
 * primaries); gen: generation (0 = primary); n_acc/n_rej: accepted/rejected
 * steps of this ray; n_ev: its Fresnel events; region: medium at the end;
 * side: bit k set when the ray is on the +normal side of boundary k. */
typedef struct {
  double *x, *y, *z, *ux, *uy, *uz, *s, *t;
  double *as_re, *as_im, *ap_re, *ap_im, *h;
  uint64_t *key, *parent;
  int32_t *gen, *status, *n_acc, *n_rej, *n_ev, *region;
  uint32_t* side;
  int64_t capacity; /* >= number of primary rays */
  rt_stats* stats;  /* device, one struct; overwritten by each launch */
  rt_event* events; /* device, ev_capacity event records in no particular
                       order, or NULL; the first min(stats.events,
                       ev_capacity) entries are written */
  int64_t ev_capacity; /* 0 = no event records (events may be NULL) */
} rt_outputs;

/* Optional launch tuning; NULL selects the defaults. */
typedef struct {
  int32_t block_size;       /* threads per block: 64, 128, 192 or 256; 0 = 256 */
  int32_t blocks_per_cu;    /* resident blocks per CU; 0 = occupancy maximum */
  int32_t refill_threshold; /* a wave refills when at least this many of its
                               64 lanes are idle (1..64); 0 = 32 for traces
                               (48 for gridded media), 16 for solves */
  void* ev_trace_begin;     /* hipEvent_t recorded just before the trace
                               kernel, or NULL */
  void* ev_trace_end;       /* hipEvent_t recorded just after it, or NULL */
  int32_t local_queue;      /* secondaries a wave keeps for itself before it
                               hands further ones to other waves: 0 = 256,
                               -1 = none, else 1..1024 */
  int32_t scan_chunk;       /* solves: entries (pair, family) whose angle
                               scans are interleaved in the task order, so
                               that consecutive tasks shoot one angle for
                               scan_chunk entries (1..4096); 0 = 1: each
                               entry's angles consecutively.  Traces ignore it.
                               Results do not depend on it. */
  int32_t solve_fused;      /* solves: 0 = scan, refinement and selection as
                               three launches; 1 = one fused persistent
                               launch when n_scan <= 64 and max_brackets <= 4
                               (else the three).  Same results either way. */
} rt_tuning;

/* ABI version (RT_ABI_VERSION of the built library).  Plumbing: no
 * counterpart in the paper. */
int32_t rt_abi_version(void);

/* Host-only validation of the descriptors of a trace (the media, boundaries
 * and limits of section 2's set-ups: refractive-index fields, boundaries,
 * tolerance and minimum step of the accuracy discussion, the travel-time
 * and amplitude limits of the Fig. 1 example): null pointers, counts and
 * limits (1 <= n_regions <= RT_MAX_REGIONS, n_planes <= RT_MAX_PLANES, region
 * indices in range, a zero plane normal, tol > 0, 0 < h_min <= h_max,
 * h_init >= 0, s_max > 0, t_max >= 0, amp_min >= 0, 1 <= max_generations <=
 * RT_MAX_GENERATIONS, model known, max_steps >= 1, grid dims >= 2 and
 * spacing > 0 when a region uses the grid, box lo < hi).  Reads only host
 * memory: the descriptor structs and the host tables they point to.
 * Returns RT_OK or RT_ERR_INVALID_ARG / RT_ERR_UNSUPPORTED with a message in
 * rt_last_error().
 * The checks of single rays -- a zero or non-finite direction, a source
 * index out of range, a source within 1e-9 m of a boundary or outside the
 * box -- are not made here: sources and directions are device arrays, which
 * this host-only call never reads (a copy to the host would serialise the
 * caller's stream).  raytrace_launch makes them on the device, per ray: such
 * a ray is not traced, its record gets RT_ST_INVALID, stats.invalid counts
 * it and rt_collect reports RT_ERR_INVALID_ARG. */
rt_status rt_validate(const rt_field* field, const rt_boundaries* boundaries,
                      const rt_sources* sources,
                      const rt_directions* directions, double tol,
                      const rt_step_limits* limits);

/* Bytes of device workspace raytrace_launch needs for this field and record
 * capacity: queue counters, a queue of record indices (4 bytes per record,
 * for secondaries shared between waves), the order in which the primaries
 * are handed out (4 bytes per record: by source, then by direction, so that
 * the lanes of a wave follow nearby paths), plus the prepared grid (16 bytes
 * per node) for gridded fields.  Plumbing of the persistent scheduler, no
 * counterpart in the paper; it takes the field and the record capacity
 * because nothing else sets the size (the ray count only bounds the
 * capacity from below).  RT_ERR_INVALID_ARG for a null field or bytes, a
 * negative capacity, or grid dims below 2. */
rt_status rt_workspace_bytes(const rt_field* field, int64_t capacity, size_t* bytes);

/* Trace all primary rays and every secondary they cast: section 2 of the
 * paper -- the ray equation (eq. 2, or eq. 1 with RT_MODEL_EXACT)
 * integrated by the Cash-Karp method with adaptive steps set by tol and the
 * minimum step; at every boundary a ray passes, reflection of the ray and a
 * refracted secondary cast from the intersection point, both with Fresnel
 * amplitudes (boundary paragraph); the limits of the Fig. 1 example.  The
 * record of each ray (final position and direction, path length, travel
 * time, amplitudes, step and event counts) goes to caller-owned device
 * arrays in 'out' (SoA, see rt_outputs).  Asynchronous on
 * 'stream' (a hipStream_t; NULL = the default stream): it validates the
 * descriptors, prepares the grid, writes the primaries into the record slots
 * and runs the persistent trace kernel, then returns RT_OK.  Conditions found
 * on the device land in out->stats; after synchronising, copy the stats to
 * the host and pass them to rt_collect.  'workspace' is device memory of at
 * least rt_workspace_bytes; it is overwritten.  Launches sharing a
 * workspace or outputs must not overlap.  With out->ev_capacity > 0 every
 * Fresnel event also appends an rt_event to out->events (RT_ERR_INVALID_ARG
 * for a negative ev_capacity, or a positive one with events NULL). */
rt_status raytrace_launch(const rt_field* field,
                          const rt_boundaries* boundaries,
                          const rt_sources* sources,
                          const rt_directions* directions, double tol,
                          const rt_step_limits* limits, rt_outputs* out,
                          void* workspace, size_t workspace_bytes,
                          void* stream, const rt_tuning* tuning);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * launch as raytrace_launch with the same arguments and results, minus the
 * workspace.  Its scratch memory (queue counters, the shared queue of
 * record slots, the hand-out order and, for gridded fields, the prepared
 * grid: rt_workspace_bytes of it) is a device array of
 * RT_STATIC_SCRATCH_BYTES inside the library, one per GPU, held from the
 * first call on that GPU until the process ends.  The call allocates
 * nothing: no hipMalloc, no hipFree, no allocating library routine; it
 * enqueues kernels on 'stream' like raytrace_launch.  A launch whose
 * rt_workspace_bytes(field, out->capacity) exceeds RT_STATIC_SCRATCH_BYTES
 * (about 5.5 million record slots for analytic fields, fewer with a grid)
 * returns RT_ERR_UNSUPPORTED without enqueuing anything.  Every call on a GPU
 * shares that GPU's array, which keeps the last call's contents (each launch
 * re-initialises what it reads): calls that overlap on one GPU, on any
 * streams, race and must not be issued; resume = 1 continues the last
 * static launch on that GPU, so no other static launch may run on it in
 * between.  The first call on a device looks up the array's device address
 * (hipGetSymbolAddress) with that device current; RT_ERR_DEVICE when that
 * fails. */
#define RT_STATIC_SCRATCH_BYTES (64ull << 20)
rt_status raytrace_launch_static(const rt_field* field,
                                 const rt_boundaries* boundaries,
                                 const rt_sources* sources,
                                 const rt_directions* directions, double tol,
                                 const rt_step_limits* limits, rt_outputs* out,
                                 void* stream, const rt_tuning* tuning);

/* Plumbing, no counterpart in the paper.  Map the statistics of a finished
 * launch to a status: RT_ERR_DEVICE when
 * the scheduler reported an error, RT_ERR_INVALID_ARG when input rays were
 * invalid, RT_ERR_CAPACITY when stats.needed exceeds
 * capacity (records of the slots below capacity are still valid; relaunch
 * with a capacity of at least stats.needed) or when event records were lost
 * (stats.events_lost > 0; the ev_capacity records written are valid, which
 * events they hold is unspecified; relaunch with ev_capacity >=
 * stats.events), RT_INTERRUPTED when the launch
 * stopped at its step budget (the slots then hold finished records, parked
 * and queued rays and unused slots; continue with resume = 1), else RT_OK.
 * Rays that ended RT_ST_NONFINITE are per-ray results and do not fail the
 * launch. */
rt_status rt_collect(const rt_stats* host_stats, int64_t capacity);

/* Message for the last non-OK status returned on the calling thread (a
 * thread-local buffer owned by the library, valid until the thread's next
 * call).  Plumbing, no counterpart in the paper. */
const char* rt_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* RADIOTRACE_H */
