/*
 * CPU oracle for the eikonal ray tracer (test infrastructure only).
 *
 * This is a plain, scalar, FP64 implementation of the method of RadioPropa
 * (Winchen, arXiv:1810.01780) section 2: adaptive Cash-Karp integration of the
 * ray equation (eq. 2 by default, eq. 1 on request) with planar media
 * boundaries that reflect the ray and cast a refracted secondary carrying
 * Fresnel amplitudes.  It exists to judge the GPU path; only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header or constant with the GPU library.
 *
 * Coordinates: z is depth (positive downward), the surface is z = 0.
 * Besides stratified media n(z) it evaluates non-stratified analytic media
 * (a stratification axis other than depth, Gaussian index anomalies) and
 * gridded data, which section 2 names among the supported fields.
 */
#ifndef RT_ORACLE_H
#define RT_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_MODEL_PAPER = 0, ORC_MODEL_EXACT = 1 };
enum { ORC_PLANE_FRESNEL = 0, ORC_PLANE_ABSORB = 1 };
enum {
  ORC_ST_PATH = 1,      /* reached the path-length limit */
  ORC_ST_BOX = 2,       /* left the bounding box */
  ORC_ST_TIME = 3,      /* reached the travel-time limit */
  ORC_ST_AMP = 4,       /* amplitude fell below the cut */
  ORC_ST_ABSORB = 5,    /* hit an absorbing plane */
  ORC_ST_STEPCAP = 6,   /* step or event budget exhausted */
  ORC_ST_NONFINITE = 7  /* NaN or Inf in the state */
};

/* n = a + b zeta - dn exp(-zeta/z0) with zeta = k . r, k the unit vector
 * along axis (axis all zero: k = (0, 0, 1), i.e. zeta = depth z); or the grid
 * when use_grid != 0.  Gaussian anomalies of the region are added to either.
 * [z_top, z_bot) picks the region a primary ray starts in. */
typedef struct {
  double a, b, dn, z0, z_top, z_bot;
  int32_t use_grid;
  double axis[3];
} orc_region;

/* amplitude exp(-|r - centre|^2 / (2 sigma^2)) added to n inside region */
typedef struct {
  double centre[3];
  double amplitude, sigma;
  int32_t region;
} orc_anomaly;

/* Boundary surfaces (shape): plane through point with normal; sphere with
 * centre point and radius param (g = |r - c| - R, region_pos outside);
 * paraboloid z = z_v + param ((x - x_v)^2 + (y - y_v)^2) with vertex point
 * (g = z - z_v - param rho^2, region_pos below, i.e. at larger depth). */
enum { ORC_SHAPE_PLANE = 0, ORC_SHAPE_SPHERE = 1, ORC_SHAPE_PARABOLOID = 2 };

typedef struct {
  double point[3], normal[3];      /* normal need not be unit length */
  int32_t region_pos, region_neg;  /* region on the +normal / -normal side */
  int32_t kind;
  int32_t shape;
  double param;
} orc_plane;

typedef struct {
  int32_t n_regions;
  const orc_region* regions;
  int32_t n_planes;
  const orc_plane* planes;
  int32_t has_box;
  double box_lo[3], box_hi[3];
  const float* grid; /* [nz][ny][nx], x fastest; may be NULL */
  int32_t nx, ny, nz;
  double origin[3], spacing[3];
  int32_t n_sources;
  const double* src_xyz;  /* [S][3] */
  int64_t n_rays;
  const double* dir_xyz;  /* [N][3] */
  const int32_t* ray_src; /* [N] */
  double tol, h_min, h_max, h_init, s_max, t_max, amp_min;
  int32_t max_gen, model;
  int64_t max_steps;
  int32_t n_anomalies;
  const orc_anomaly* anomalies;
} orc_problem;

typedef struct {
  double *x, *y, *z, *ux, *uy, *uz, *s, *t, *as_re, *as_im, *ap_re, *ap_im, *h;
  uint64_t *key, *parent;
  int32_t *gen, *status, *n_acc, *n_rej, *n_ev, *region;
  int64_t capacity;
} orc_records;

typedef struct {
  int64_t accepted, rejected, relocation, forced, events, spawned;
  int64_t suppressed_gen, suppressed_amp, records, needed, nonfinite, max_gen;
} orc_stats;

/* Trace the root rays listed in roots (all rays when roots == NULL) with
 * n_threads host threads.  Records are written in no particular order; each
 * carries its key.  Returns 0, or -1 when the record capacity was too small
 * (stats->needed then holds the required count). */
int orc_trace(const orc_problem* P, const int64_t* roots, int64_t n_roots,
              orc_records* out, orc_stats* stats, int n_threads);

/* One record per Fresnel boundary event (section 2, boundary paragraph):
 * where the ray met which boundary, how it arrived, the two media, the
 * Fresnel coefficients and what became of the refracted branch. */
enum {
  ORC_EV_SPAWNED = 0, /* a refracted secondary was cast */
  ORC_EV_TIR = 1,     /* total internal reflection: nothing transmitted */
  ORC_EV_GEN = 2,     /* transmitted branch beyond the generation limit */
  ORC_EV_AMP = 3      /* transmitted branch below the amplitude cut */
};
typedef struct {
  uint64_t* key;      /* the ray that met the boundary */
  int32_t* ordinal;   /* its event count including this event, 1..255 */
  int32_t* boundary;  /* index of the boundary in the problem's list */
  int32_t* outcome;   /* ORC_EV_* */
  int32_t* gen;       /* generation of the ray */
  int32_t *region_in, *region_out; /* medium of the ray / beyond the boundary */
  double* pos;        /* [cap][3] crossing point (on the boundary) */
  double* dir;        /* [cap][3] incident unit direction */
  double *s, *t;      /* path length and travel time there */
  double *cos_i, *n1, *n2; /* incidence cosine, index before / beyond */
  double* amp;        /* [cap][4] incident amplitudes as_re, as_im, ap_re, ap_im */
  double* coef;       /* [cap][8] r_s, r_p, t_s, t_p as (re, im) pairs */
  int64_t capacity;
} orc_events;

/* orc_trace that also writes the event records (in no particular order);
 * *n_events receives the number of events.  Returns -3 when the event
 * capacity was too small, else as orc_trace. */
int orc_trace_events(const orc_problem* P, const int64_t* roots, int64_t n_roots,
                     orc_records* out, orc_stats* stats, orc_events* ev,
                     int64_t* n_events, int n_threads);

/* The step controller's record of the trials of a trace (test
 * instrumentation: the controller is a convention the paper does not fix,
 * and its constants are checked against the order of the method).  Every
 * trial step of the normal stepping (not of the crossing search) appends its
 * length, its error ratio (error norm / tol) and its outcome (0 rejected, 1
 * accepted, 2 forced at h_min), while n < cap. */
typedef struct {
  double* h;
  double* err;
  int32_t* outcome;
  int64_t cap, n;
} orc_trial_log;

/* orc_trace of the listed roots on one thread, logging their trials in
 * order (one root's whole tree, then the next). */
int orc_trace_log(const orc_problem* P, const int64_t* roots, int64_t n_roots,
                  orc_records* out, orc_stats* stats, orc_trial_log* log);

/* Single Cash-Karp trial step of the ray ODE from y0 (7 components) with step
 * h in region reg: writes the 5th-order result and the embedded error vector. */
void orc_ck_trial(const orc_problem* P, int32_t reg, const double y0[7],
                  double h, double y5[7], double err_vec[7]);

/* Refractive index and gradient of region reg at r. */
void orc_field(const orc_problem* P, int32_t reg, const double r[3], double* n,
               double grad[3]);

/* Fresnel coefficients for incidence from n1 into n2 with cos(theta_i) = ci.
 * out = {rs_re, rs_im, rp_re, rp_im, ts_re, ts_im, tp_re, tp_im, cos_t};
 * returns 1 on total internal reflection (t = 0, cos_t = 0). */
int orc_fresnel(double n1, double n2, double ci, double out[9]);

/* Emitter -> receiver solves (shooting).  Source at (0, 0, zs[i]), receiver
 * at (dist[i], 0, zr[i]); planes[0] of the problem is the surface, the other
 * planes are transmitted (reflected under total internal reflection).  For
 * each pair two families are solved: DIRECT (the ray may not touch the
 * surface) and REFLECTED (exactly one surface reflection). */
enum { ORC_FAMILY_DIRECT = 0, ORC_FAMILY_REFLECTED = 1 };
typedef struct {
  const double *zs, *zr, *dist;
  int32_t n_scan;       /* launch angles scanned per family */
  int32_t max_iter;     /* refinement shots per bracket */
  int32_t max_brackets; /* sign changes refined per family */
  double miss_tol;      /* refinement stops at |miss| <= miss_tol (m) */
  double accept_tol;    /* a root is a solution if |miss| <= accept_tol (m) */
  double slope_max;     /* bracket stop: finite end misses above slope_max *
                           width (m/rad) hold no root; 0 = off */
} orc_solve_spec;

/* Outputs indexed [2 * pair + family].  roots: refined brackets whose last
 * shot met the receiver plane within accept_tol (the solution is the first
 * arrival among them); the seeded secant reports 1 for a verified entry. */
typedef struct {
  int32_t *found, *shots, *roots;
  double *theta, *miss, *t, *s, *as_re, *as_im, *ap_re, *ap_im;
} orc_solve_out;

int orc_solve(const orc_problem* P, const orc_solve_spec* spec, const int64_t* pairs,
              int64_t n_pairs, orc_solve_out* out, int n_threads);

/* Single shots: status 0 = reached the receiver plane (miss = depth - zr,
 * mirrored before the surface reflection for the reflected family), 1 =
 * touched the surface where the family forbids it (miss = -1e6), 2 = never
 * reached the receiver plane (miss = +1e6), 3 = invalid input. */
typedef struct {
  int32_t *status, *n_acc, *n_rej;
  double *miss, *t, *s, *as_re, *as_im, *ap_re, *ap_im;
} orc_shot_out;

int orc_shoot(const orc_problem* P, const double* zs, const double* zr, const double* dist,
              const double* theta, const int32_t* family, int64_t n, orc_shot_out* out,
              int n_threads);

/* Seeded secant per entry [2 pair + family] with try_[e] != 0: shots at the
 * seed, at seed + dseed (seed - dseed if that leaves (0, pi)), then secant
 * steps; solved by the first shot that meets the receiver plane with
 * |miss| <= verify_tol; fails at a shot that does not, a step outside
 * (0, pi), or after max_shots shots.  verify[e] = 1 / 0 for tried entries. */
typedef struct {
  double verify_tol, dseed;
  int32_t max_shots;
} orc_seed_spec;

int orc_solve_seeded(const orc_problem* P, const double* zs, const double* zr,
                     const double* dist, int64_t n_pairs, const double* seed,
                     const int32_t* try_, const orc_seed_spec* spec, orc_solve_out* out,
                     int32_t* verify, int n_threads);

#ifdef __cplusplus
}
#endif
#endif
