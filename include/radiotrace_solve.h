/*
 * radiotrace -- emitter -> receiver solves (shooting) on MI355X (gfx950).
 *
 * Section 2 of RadioPropa (arXiv:1810.01780) lists receiver and emitter
 * locations among the set-ups the method supports (paragraph after the
 * Fig. 1 example).  For a source and a receiver the rays that connect them
 * are found here by shooting: a ray launched at angle theta is traced with
 * the same integrator and boundary handling as raytrace_launch (no
 * secondaries are cast; the ray follows one branch), and the launch angle is
 * adjusted until the ray meets the receiver.  The construction is this
 * library's (the paper describes no solver):
 *
 *   Geometry.  Source at (0, 0, zs), receiver at (dist, 0, zr), both below
 *   the surface; the vertical plane y = 0 contains both.  A ray launched at
 *   angle theta from the upward vertical towards the receiver has direction
 *   (sin theta, 0, -cos theta); theta in (0, pi).  The receiver plane x = dist
 *   ends every ray ("shot"); the miss is the depth at which the shot meets
 *   it minus zr.
 *
 *   Families.  boundaries->planes[0] is the surface.
 *     DIRECT    (family 0): the ray may not touch the surface.
 *     REFLECTED (family 1): the ray is reflected exactly once at the surface;
 *               until that reflection its miss is measured in the mirror
 *               image of the surface (2 z_surface - z), so that the miss is
 *               continuous across rays that do and do not reach it.
 *   At every other plane the ray is transmitted (refracted; reflected under
 *   total internal reflection).  Amplitudes multiply by the Fresnel factor
 *   of the branch taken.  A shot that touches the surface where its family
 *   forbids it ends with miss = -1e6 (it passed above the receiver); a shot
 *   that never reaches the receiver plane (path 2 (dist + zs + zr) + 1000 m,
 *   the step budget, an absorbing plane, a non-finite state) ends with
 *   miss = +1e6.
 *
 *   Solve.  Per pair and family: shots at theta_k = (k + 1/2) pi / n_scan,
 *   k = 0 .. n_scan-1; each sign change of the miss between neighbours is a
 *   bracket (the first max_brackets, in k order, are refined).  A bracket is
 *   refined by Illinois false position on the miss (bisection while an end
 *   has |miss| >= 1e5), stopping when a shot reaches the receiver plane with
 *   |miss| <= miss_tol, when the bracket is narrower than 1e-9 rad, after
 *   max_iter shots, or when the bracket cannot hold a root: a miss that is
 *   continuous with slope at most slope_max (m/rad) and vanishes in [a, b]
 *   has |miss(a)| + |miss(b)| <= slope_max (b - a) (ends with |miss| >= 1e5
 *   count zero); brackets around jumps of the miss -- shots starting to
 *   touch the surface or to get lost, total reflection setting in at a
 *   layer -- end this way.  1e7 m/rad (10 m of miss per mrad of launch
 *   angle, about 900 times the longest shot path) is the suggested value.  A refined root is a solution if its last shot reached
 *   the receiver plane with |miss| <= accept_tol; the solution reported is
 *   the one with the smallest travel time (the first in bracket order among
 *   equal times).
 *
 * Conventions are those of radiotrace.h: descriptors are read during the call,
 * arrays are device arrays owned by the caller, work is enqueued on 'stream'
 * and nothing is allocated (scratch lives in the caller's workspace); the
 * calls enqueue only kernel launches, so they may be captured into a HIP
 * graph (hipStreamBeginCapture / torch.cuda.graph) and replayed.
 */
#ifndef RADIOTRACE_SOLVE_H
#define RADIOTRACE_SOLVE_H

#include "radiotrace.h"

#ifdef __cplusplus
extern "C" {
#endif

enum { RT_FAMILY_DIRECT = 0, RT_FAMILY_REFLECTED = 1 };

/* How a shot ended. */
enum {
  RT_SHOT_RECEIVER = 0, /* met the receiver plane; miss = depth - zr */
  RT_SHOT_SURFACE = 1,  /* touched the surface where its family forbids it */
  RT_SHOT_LOST = 2,     /* never met the receiver plane */
  RT_SHOT_INVALID = 3   /* bad input (non-finite value, dist <= 0, source
                           within 1e-9 m of a plane, theta outside (0, pi),
                           unknown family); not traced */
};

/* Source/receiver pairs: device arrays of n elements. */
typedef struct {
  const double* zs;   /* source depth */
  const double* zr;   /* receiver depth */
  const double* dist; /* horizontal distance, > 0 */
  int64_t n;          /* >= 0 */
} rt_pairs;

typedef struct {
  int32_t n_scan;       /* launch angles scanned per family, 2..4096 */
  int32_t max_iter;     /* refinement shots per bracket, 1..1000 */
  int32_t max_brackets; /* brackets refined per family, 1..16 */
  double miss_tol;      /* refinement stops at |miss| <= miss_tol (m), > 0 */
  double accept_tol;    /* solution if |miss| <= accept_tol (m), >= miss_tol */
  double slope_max;     /* bracket stop (m/rad, see above); 0 = off */
} rt_solve_params;

/* Device-side totals of a solve or shoot call. */
typedef struct {
  int64_t shots;      /* shots traced (scan + refinement, or the list) */
  int64_t accepted;   /* accepted Cash-Karp steps over all shots */
  int64_t rejected;   /* rejected trial steps */
  int64_t relocation; /* trial steps spent locating crossings */
  int64_t forced;     /* steps accepted at h_min above tolerance */
  int64_t events;     /* boundary events (surface, layers, receiver plane) */
  int64_t brackets;   /* brackets refined */
  int64_t found;      /* (pair, family) entries with a solution */
  int64_t invalid;    /* invalid shots or pairs */
} rt_solve_stats;

/* Results, indexed [2 * pair + family], device arrays of 2 n elements.
 * found: 1 if a solution was found (the other fields are then those of its
 * last shot; all zero otherwise).  shots: shots the sequential procedure
 * above takes for this entry (the scan stops after the max_brackets-th
 * bracket there; the device scans all n_scan angles in parallel and counts
 * its actual work in stats.shots).  theta: launch angle; miss: depth at the
 * receiver plane minus zr; t: travel time; s: path length; as_*, ap_*:
 * complex s/p amplitude factors (start 1 + 0i).  roots: refined brackets
 * whose last shot met the receiver plane within accept_tol (the solution is
 * the first arrival among them; 1 for an entry verified by the seeded
 * secant, 0 without a solution). */
typedef struct {
  int32_t *found, *shots, *roots;
  double *theta, *miss, *t, *s, *as_re, *as_im, *ap_re, *ap_im;
  rt_solve_stats* stats; /* device, one struct; overwritten by each call */
} rt_solve_outputs;

/* An explicit list of shots: device arrays of n elements. */
typedef struct {
  const double *zs, *zr, *dist, *theta;
  const int32_t* family;
  int64_t n;
} rt_shots;

/* Per-shot results, device arrays of n elements.  status: RT_SHOT_*; miss,
 * t, s, amplitudes at the end of the shot (miss +-1e6 as described above);
 * n_acc / n_rej: accepted / rejected steps of the shot. */
typedef struct {
  int32_t *status, *n_acc, *n_rej;
  double *miss, *t, *s, *as_re, *as_im, *ap_re, *ap_im;
  rt_solve_stats* stats; /* device, one struct; overwritten by each call */
} rt_shot_outputs;

/* Emitter -> receiver solves: section 2 lists receiver and emitter
 * locations among the set-ups the software supports; the paper gives no
 * solver, and the shooting method here (scan of launch angles, Illinois
 * refinement of the miss at the receiver, first-arrival selection) is this
 * library's construction on top of the trace of section 2.
 * Host-only checks of a solve or shoot set-up: the field, boundaries and
 * limits as in rt_validate (t_max must be 0 and has_box 0: shots end at the
 * receiver plane; s_max, amp_min and max_generations are not used), at
 * least one plane, planes[0] of kind RT_PLANE_FRESNEL (the surface), and
 * params within the ranges above (params may be NULL for shoot).  Gridded
 * fields give RT_ERR_UNSUPPORTED: solves run in stratified media. */
rt_status rt_solve_validate(const rt_field* field, const rt_boundaries* boundaries, double tol,
                            const rt_step_limits* limits, const rt_solve_params* params);

/* Plumbing of the solver, no counterpart in the paper.  Device workspace
 * bytes for a solve of n_pairs pairs: counters, the scan's
 * miss table (8 bytes per pair, family and angle) and the per-bracket
 * results (80 bytes per pair, family and bracket), plus the prepared grid
 * (16 bytes per node) for gridded fields.  shoot needs the same with
 * n_pairs = 0. */
rt_status rt_solve_workspace_bytes(const rt_field* field, int64_t n_pairs,
                                   const rt_solve_params* params, size_t* bytes);

/* Solve every pair for both families (the receiver/emitter set-up of
 * section 2, by shooting).  Caller-owned device arrays in and out; results
 * [2 * pair + family].  Asynchronous on 'stream': a counter reset, then
 * three launches, the scan and the refinement (persistent: one shot per
 * lane, lanes take new shots from a ticket counter) and the selection; or,
 * with tuning->solve_fused = 1 and n_scan <= 64, max_brackets <= 4, one
 * fused persistent launch (each wave holds up to 16 (pair, family)
 * entries, shoots their scans, refines their brackets and writes their
 * results).  The results are the same bit for bit either way and for every
 * tuning.  Outputs and the workspace must not be shared with an
 * overlapping call.  tuning: block_size and refill_threshold as in
 * raytrace_launch; scan_chunk; solve_fused; other fields unused; NULL =
 * defaults. */
rt_status raytrace_solve(const rt_field* field, const rt_boundaries* boundaries, double tol,
                         const rt_step_limits* limits, const rt_pairs* pairs,
                         const rt_solve_params* params, rt_solve_outputs* out, void* workspace,
                         size_t workspace_bytes, void* stream, const rt_tuning* tuning);

/* Trace an explicit list of shots (the building block of raytrace_solve):
 * single-branch traces of section 2 from an emitter at a launch angle to the
 * receiver plane.
 * Asynchronous on 'stream'; same workspace rules with n_pairs = 0. */
rt_status raytrace_shoot(const rt_field* field, const rt_boundaries* boundaries, double tol,
                         const rt_step_limits* limits, const rt_shots* shots,
                         rt_shot_outputs* out, void* workspace, size_t workspace_bytes,
                         void* stream, const rt_tuning* tuning);

/* Plumbing, no counterpart in the paper.  Pick launch tuning for
 * raytrace_solve by measurement: every combination of
 * block_size in {64, 128, 192, 256} and refill_threshold in {4, 16, 32, 64}
 * in three launches (scan_chunk 1), then scan_chunk in {4, 16, 64} at the
 * best of those, then the fused launch (solve_fused 1) at each block size
 * and refill_threshold 16 when n_scan <= 64 and max_brackets <= 4; each
 * runs raytrace_solve twice on 'pairs' (a representative sample; its results
 * land in 'out' and are overwritten by each candidate), after one untimed
 * call for the whole search, timed with HIP events on 'stream', its faster
 * run counting; the fastest candidate is written to *best
 * (other fields zero) and its time in ms to *best_ms (may be NULL).  This
 * call blocks the host until each candidate finishes, so it cannot be
 * captured into a graph: tune first, then capture raytrace_solve with the
 * result. */
rt_status rt_solve_autotune(const rt_field* field, const rt_boundaries* boundaries, double tol,
                            const rt_step_limits* limits, const rt_pairs* pairs,
                            const rt_solve_params* params, rt_solve_outputs* out,
                            void* workspace, size_t workspace_bytes, void* stream,
                            rt_tuning* best, float* best_ms);

#ifdef __cplusplus
}
#endif
#endif /* RADIOTRACE_SOLVE_H */
