/*
 * CPU oracle for the eikonal ray tracer -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain scalar FP64 C, built with -O2 -ffp-contract=off and no fast-math.
 * It follows RadioPropa (arXiv:1810.01780) section 2 step by step:
 *
 *   - the ray equation: eq. 2 (locally paraxial, n r'' = grad n) by default,
 *     eq. 1 (full eikonal, (n r')' = grad n) as the "exact" model;
 *   - the Cash-Karp embedded Runge-Kutta 4(5) solver the paper adapts
 *     (Cash & Karp 1990, ACM TOMS 16(3), table of coefficients);
 *   - adaptive steps whose accuracy is set by a tolerance and a minimum step
 *     length (section 2, accuracy discussion);
 *   - boundaries handled apart from the propagation: a ray passing a plane is
 *     reflected and a refracted secondary is cast from the intersection
 *     point, the amplitudes following Fresnel's equations (section 2,
 *     boundary paragraph); the reflected ray keeps the parent's identity;
 *   - amplitudes are not corrected for path length (Fig. 1 caption);
 *   - optional limits on travel time and amplitude (Fig. 1 example).
 *
 * The paper leaves the step controller, the error norm, the crossing search,
 * the polarisation convention and the ray-tree bookkeeping open; this file
 * takes one explicit reading of each (see the comments at each step).
 *
 * Constants with no value in the paper (conventions): the crossing search's
 * stopping tolerances (|g| <= 1e-10 m, bracket 1e-14 h, 60 trials) and the
 * start value of the search for a ray leaving the boundary it stands on; the
 * solver's scan and stopping constants (angle scan, Illinois stopping widths
 * and slope bound).  The constants themselves are not pinned; the functions
 * that use them are, through their results: crossing points against the
 * closed-form line-plane intersection and the chord through a spherical
 * void, solver roots against the straight-line and mirror solutions of a
 * constant medium and the closed form of the exponential profile, the scan
 * against a dense scan, the slope bound against the roots it may drop.
 * Every other function is pinned by the CPU tests (closed forms,
 * conservation laws, Fresnel identities, convergence orders, the paper's
 * accuracy study).
 *
 * Nothing here is shared with the GPU library.
 */
#include "oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

#define C0 299792458.0 /* speed of light in vacuum, m/s (exact) */

/* Cash-Karp 1990 coefficients: stage nodes c, stage matrix a, fifth-order
 * weights b and the difference b - b* of the fifth- and fourth-order weights
 * (the embedded error estimate). */
static const double CK_A[6][5] = {
    {0, 0, 0, 0, 0},
    {1.0 / 5.0, 0, 0, 0, 0},
    {3.0 / 40.0, 9.0 / 40.0, 0, 0, 0},
    {3.0 / 10.0, -9.0 / 10.0, 6.0 / 5.0, 0, 0},
    {-11.0 / 54.0, 5.0 / 2.0, -70.0 / 27.0, 35.0 / 27.0, 0},
    {1631.0 / 55296.0, 175.0 / 512.0, 575.0 / 13824.0, 44275.0 / 110592.0,
     253.0 / 4096.0}};
static const double CK_B[6] = {37.0 / 378.0, 0.0, 250.0 / 621.0,
                               125.0 / 594.0, 0.0, 512.0 / 1771.0};
static const double CK_E[6] = {-277.0 / 64512.0, 0.0, 6925.0 / 370944.0,
                               -6925.0 / 202752.0, -277.0 / 14336.0,
                               277.0 / 7084.0};

/* Step-size controller (standard embedded-RK control, Press et al. 16.2):
 * safety 0.9, growth at most 5, shrink at most 10, exponents -1/5 after an
 * accepted and -1/4 after a rejected trial.  Below ERRCON the growth factor
 * is the cap 5 (0.9 * ERRCON^(-1/5) == 5 exactly at the switch). */
#define SAFETY 0.9
#define GROW_MAX 5.0
#define SHRINK_MIN 0.1
#define ERRCON 1.889568e-4 /* (0.9/5)^5 */

/* Crossing search: Illinois false position until the bracket on the step
 * parameter is narrower than LOC_WREL times the step, g is exactly zero, or
 * LOC_MAXIT trials.  The stop is on the bracket, not on |g|: a ray that
 * meets a boundary at grazing incidence changes g by little along its path,
 * and a small |g| would leave the crossing point undetermined along the ray
 * (by |g| / |dg/dsigma|). */
#define LOC_WREL 1e-12
#define LOC_MAXIT 60
#define LOC_MAXPASS 8 /* re-searches for an earlier crossing of another plane */
#define ON_BND 0x1p-33 /* a step starts on a boundary when G0 <= 2^-33 m */
#define MAX_EVENTS 255

typedef struct {
  double y[7]; /* r (3), v or p (3), travel time tau */
  double s, h;
  double as_re, as_im, ap_re, ap_im;
  uint64_t key, parent;
  int32_t gen, region, n_acc, n_rej, n_ev;
  uint32_t side; /* bit k set: the ray is on the +normal side of plane k */
} ray_t;

/* ------------------------------------------------------------------------ */
/* Boundaries: user planes, then the six box faces, then (when a travel-time
 * limit is set) a pseudo-plane for tau = t_max.  g > 0 on the +normal side. */
enum { KIND_FRESNEL = 0, KIND_ABSORB = 1, KIND_BOX = 2, KIND_TIME = 3 };

typedef struct {
  double nrm[3], d;     /* plane: unit normal and offset */
  double pt[3], param;  /* sphere: centre, radius; paraboloid: vertex, curvature */
  int32_t kind, reg_pos, reg_neg, shape;
} bplane_t;

typedef struct {
  const orc_problem* P;
  bplane_t pl[32];
  int32_t n_pl;
} scene_t;

static void build_scene(const orc_problem* P, scene_t* S) {
  S->P = P;
  int m = 0;
  for (int k = 0; k < P->n_planes; ++k) {
    const orc_plane* q = &P->planes[k];
    double len = sqrt(q->normal[0] * q->normal[0] + q->normal[1] * q->normal[1] +
                      q->normal[2] * q->normal[2]);
    bplane_t* b = &S->pl[m++];
    memset(b, 0, sizeof *b);
    b->shape = q->shape;
    for (int i = 0; i < 3; ++i) b->pt[i] = q->point[i];
    b->param = q->param;
    if (q->shape == ORC_SHAPE_PLANE) {
      for (int i = 0; i < 3; ++i) b->nrm[i] = q->normal[i] / len;
      b->d = q->point[0] * b->nrm[0] + q->point[1] * b->nrm[1] + q->point[2] * b->nrm[2];
    }
    b->kind = q->kind == ORC_PLANE_ABSORB ? KIND_ABSORB : KIND_FRESNEL;
    b->reg_pos = q->region_pos;
    b->reg_neg = q->region_neg;
  }
  if (P->has_box) {
    for (int a = 0; a < 3; ++a) {
      for (int hi = 0; hi < 2; ++hi) {
        bplane_t* b = &S->pl[m++];
        b->nrm[0] = b->nrm[1] = b->nrm[2] = 0.0;
        b->nrm[a] = hi ? -1.0 : 1.0; /* inside of the box is g > 0 */
        b->d = hi ? -P->box_hi[a] : P->box_lo[a];
        b->kind = KIND_BOX;
        b->reg_pos = b->reg_neg = -1;
      }
    }
  }
  if (P->t_max > 0.0) {
    bplane_t* b = &S->pl[m++];
    memset(b, 0, sizeof *b);
    b->kind = KIND_TIME;
  }
  S->n_pl = m;
}

/* Signed "distance" of the state from boundary k, positive on the side the
 * ray starts on after multiplying by its side sign (metres). */
static double bnd_g(const scene_t* S, int k, const double y[7]) {
  const bplane_t* b = &S->pl[k];
  if (b->kind == KIND_TIME) return (S->P->t_max - y[6]) * C0;
  if (b->shape == ORC_SHAPE_SPHERE) {
    const double dx = y[0] - b->pt[0], dy = y[1] - b->pt[1], dz = y[2] - b->pt[2];
    return sqrt(dx * dx + dy * dy + dz * dz) - b->param;
  }
  if (b->shape == ORC_SHAPE_PARABOLOID) {
    const double dx = y[0] - b->pt[0], dy = y[1] - b->pt[1];
    return y[2] - b->pt[2] - b->param * (dx * dx + dy * dy);
  }
  return y[0] * b->nrm[0] + y[1] * b->nrm[1] + y[2] * b->nrm[2] - b->d;
}

/* Unit normal of boundary k at y, pointing to the g > 0 side (grad g). */
static void bnd_normal(const scene_t* S, int k, const double y[7], double n[3]) {
  const bplane_t* b = &S->pl[k];
  if (b->shape == ORC_SHAPE_SPHERE) {
    for (int i = 0; i < 3; ++i) n[i] = y[i] - b->pt[i];
  } else if (b->shape == ORC_SHAPE_PARABOLOID) {
    n[0] = -2.0 * b->param * (y[0] - b->pt[0]);
    n[1] = -2.0 * b->param * (y[1] - b->pt[1]);
    n[2] = 1.0;
  } else {
    for (int i = 0; i < 3; ++i) n[i] = b->nrm[i];
    return;
  }
  const double l = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
  for (int i = 0; i < 3; ++i) n[i] /= l;
}

/* Move a located point onto boundary k: along the normal for a plane,
 * radially for a sphere, vertically for a paraboloid (whose g is a depth
 * difference). */
static void bnd_snap(const scene_t* S, int k, double y[7]) {
  const bplane_t* b = &S->pl[k];
  if (b->kind == KIND_TIME) return;
  if (b->shape == ORC_SHAPE_SPHERE) {
    const double dx = y[0] - b->pt[0], dy = y[1] - b->pt[1], dz = y[2] - b->pt[2];
    const double f = b->param / sqrt(dx * dx + dy * dy + dz * dz);
    y[0] = b->pt[0] + f * dx;
    y[1] = b->pt[1] + f * dy;
    y[2] = b->pt[2] + f * dz;
  } else if (b->shape == ORC_SHAPE_PARABOLOID) {
    y[2] -= bnd_g(S, k, y);
  } else {
    const double g = bnd_g(S, k, y);
    for (int i = 0; i < 3; ++i) y[i] -= g * b->nrm[i];
  }
}

static double side_sign(const ray_t* r, int k) {
  return ((r->side >> k) & 1u) ? 1.0 : -1.0;
}

/* ------------------------------------------------------------------------ */
/* Refractive index (paper section 2: analytic profiles and gridded data). */

static double grid_node(const orc_problem* P, int i, int j, int k) {
  return (double)P->grid[((size_t)k * P->ny + j) * P->nx + i];
}

/* Node gradient by central differences, one-sided at the grid edges; the
 * one-sided difference is doubled so that grad = D / (2 spacing) everywhere. */
static double grid_diff(const orc_problem* P, int axis, int i, int j, int k) {
  int idx[3] = {i, j, k};
  int dim[3] = {P->nx, P->ny, P->nz};
  int lo[3] = {i, j, k}, hi[3] = {i, j, k};
  double scale = 1.0;
  if (idx[axis] == 0) {
    hi[axis] = 1;
    scale = 2.0;
  } else if (idx[axis] == dim[axis] - 1) {
    lo[axis] = dim[axis] - 2;
    scale = 2.0;
  } else {
    lo[axis] = idx[axis] - 1;
    hi[axis] = idx[axis] + 1;
  }
  double d = grid_node(P, hi[0], hi[1], hi[2]) - grid_node(P, lo[0], lo[1], lo[2]);
  return scale * d;
}

/* Trilinear interpolation of n and of the node gradients; positions outside
 * the grid are clamped onto it. */
static void grid_eval(const orc_problem* P, const double r[3], double* n,
                      double g[3]) {
  int dim[3] = {P->nx, P->ny, P->nz};
  int i0[3];
  double t[3];
  for (int a = 0; a < 3; ++a) {
    double f = (r[a] - P->origin[a]) / P->spacing[a];
    if (f < 0.0) f = 0.0;
    if (f > (double)(dim[a] - 1)) f = (double)(dim[a] - 1);
    int i = (int)floor(f);
    if (i > dim[a] - 2) i = dim[a] - 2;
    i0[a] = i;
    t[a] = f - (double)i;
  }
  double nn = 0.0, gg[3] = {0.0, 0.0, 0.0};
  for (int c = 0; c < 8; ++c) {
    int cx = c & 1, cy = (c >> 1) & 1, cz = (c >> 2) & 1;
    double w = (cx ? t[0] : 1.0 - t[0]) * (cy ? t[1] : 1.0 - t[1]) *
               (cz ? t[2] : 1.0 - t[2]);
    int i = i0[0] + cx, j = i0[1] + cy, k = i0[2] + cz;
    nn += w * grid_node(P, i, j, k);
    for (int a = 0; a < 3; ++a) gg[a] += w * grid_diff(P, a, i, j, k);
  }
  *n = nn;
  for (int a = 0; a < 3; ++a) g[a] = gg[a] / (2.0 * P->spacing[a]);
}

void orc_field(const orc_problem* P, int32_t reg, const double r[3], double* n,
               double g[3]) {
  const orc_region* R = &P->regions[reg];
  if (R->use_grid) {
    grid_eval(P, r, n, g);
  } else {
    /* n = a + b zeta - dn exp(-zeta/z0) along the unit stratification axis k
     * (depth when no axis is given): grad n = (b + dn/z0 exp(-zeta/z0)) k */
    double k[3] = {0.0, 0.0, 1.0};
    double len = sqrt(R->axis[0] * R->axis[0] + R->axis[1] * R->axis[1] +
                      R->axis[2] * R->axis[2]);
    if (len > 0.0)
      for (int a = 0; a < 3; ++a) k[a] = R->axis[a] / len;
    double zeta = k[0] * r[0] + k[1] * r[1] + k[2] * r[2];
    double e = R->dn != 0.0 ? exp(-zeta / R->z0) : 0.0;
    *n = R->a + R->b * zeta - R->dn * e;
    double gs = R->b + R->dn / R->z0 * e;
    for (int a = 0; a < 3; ++a) g[a] = gs * k[a];
  }
  /* Gaussian anomalies A exp(-q / (2 sigma^2)), q = |r - c|^2:
   * grad = -A exp(...) (r - c) / sigma^2 */
  for (int j = 0; j < P->n_anomalies; ++j) {
    const orc_anomaly* A = &P->anomalies[j];
    if (A->region != reg) continue;
    double d[3], q = 0.0;
    for (int a = 0; a < 3; ++a) {
      d[a] = r[a] - A->centre[a];
      q += d[a] * d[a];
    }
    double s2 = A->sigma * A->sigma;
    double v = A->amplitude * exp(-q / (2.0 * s2));
    *n += v;
    for (int a = 0; a < 3; ++a) g[a] -= v * d[a] / s2;
  }
}

/* ------------------------------------------------------------------------ */
/* Right-hand side of the ray ODE in the state y = (r, w, tau).
 * Paper model (eq. 2): w = v = dr/ds, dv/ds = grad n / n; the dn/ds term of
 *   eq. 1 is dropped inside a step and v is renormalised after every step.
 * Exact model (eq. 1): w = p = n dr/ds, dr/ds = p/|p|, dp/ds = grad n.
 * In both, dtau/ds = n / c0 (travel time). */
static void rhs(const orc_problem* P, int reg, const double y[7], double f[7]) {
  double n, g[3];
  orc_field(P, reg, y, &n, g);
  if (P->model == ORC_MODEL_EXACT) {
    double pn = sqrt(y[3] * y[3] + y[4] * y[4] + y[5] * y[5]);
    f[0] = y[3] / pn;
    f[1] = y[4] / pn;
    f[2] = y[5] / pn;
    f[3] = g[0];
    f[4] = g[1];
    f[5] = g[2];
  } else {
    f[0] = y[3];
    f[1] = y[4];
    f[2] = y[5];
    f[3] = g[0] / n;
    f[4] = g[1] / n;
    f[5] = g[2] / n;
  }
  f[6] = n / C0;
}

void orc_ck_trial(const orc_problem* P, int32_t reg, const double y0[7],
                  double h, double y5[7], double dl[7]) {
  double K[6][7], Y[7];
  rhs(P, reg, y0, K[0]);
  for (int st = 1; st < 6; ++st) {
    for (int i = 0; i < 7; ++i) {
      double acc = 0.0;
      for (int j = 0; j < st; ++j) acc += CK_A[st][j] * K[j][i];
      Y[i] = y0[i] + h * acc;
    }
    rhs(P, reg, Y, K[st]);
  }
  for (int i = 0; i < 7; ++i) {
    double acc5 = 0.0, acce = 0.0;
    for (int j = 0; j < 6; ++j) {
      acc5 += CK_B[j] * K[j][i];
      acce += CK_E[j] * K[j][i];
    }
    y5[i] = y0[i] + h * acc5;
    dl[i] = h * acce;
  }
}

/* Scaled error of a trial: max(|dr|/h, |dw|/|w0|) / tol (tau excluded). */
static double trial_error(const double y0[7], const double dl[7], double h,
                          double tol) {
  double dr = sqrt(dl[0] * dl[0] + dl[1] * dl[1] + dl[2] * dl[2]);
  double dw = sqrt(dl[3] * dl[3] + dl[4] * dl[4] + dl[5] * dl[5]);
  double w0 = sqrt(y0[3] * y0[3] + y0[4] * y0[4] + y0[5] * y0[5]);
  double e1 = dr / h, e2 = dw / w0;
  return (e1 > e2 ? e1 : e2) / tol;
}

static double clamp_h(const orc_problem* P, double h) {
  if (h < P->h_min) h = P->h_min;
  if (h > P->h_max) h = P->h_max;
  return h;
}

static int all_finite(const double* v, int n) {
  for (int i = 0; i < n; ++i)
    if (!isfinite(v[i])) return 0;
  return 1;
}

/* Direction state from a unit direction u at position r: v = u (paper) or
 * p = n(r) u (exact). */
static void set_direction(const orc_problem* P, int reg, double y[7],
                          const double u[3]) {
  double len = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  double m = 1.0;
  if (P->model == ORC_MODEL_EXACT) {
    double n, g[3];
    orc_field(P, reg, y, &n, g);
    m = n;
  }
  for (int i = 0; i < 3; ++i) y[3 + i] = m * (u[i] / len);
}

static void unit_direction(const double y[7], double u[3]) {
  double len = sqrt(y[3] * y[3] + y[4] * y[4] + y[5] * y[5]);
  for (int i = 0; i < 3; ++i) u[i] = y[3 + i] / len;
}

/* ------------------------------------------------------------------------ */
/* Fresnel equations (Born & Wolf; Hecht) for incidence from n1 into n2 with
 * cos(theta_i) = ci >= 0.  Beyond the critical angle cos(theta_t) = i kappa. */
int orc_fresnel(double n1, double n2, double ci, double out[9]) {
  double eta = n1 / n2;
  double st2 = eta * eta * (1.0 - ci * ci);
  if (st2 <= 1.0) {
    double ct = sqrt(1.0 - st2);
    double ds = n1 * ci + n2 * ct, dp = n2 * ci + n1 * ct;
    out[0] = (n1 * ci - n2 * ct) / ds;
    out[1] = 0.0;
    out[2] = (n2 * ci - n1 * ct) / dp;
    out[3] = 0.0;
    out[4] = 2.0 * n1 * ci / ds;
    out[5] = 0.0;
    out[6] = 2.0 * n1 * ci / dp;
    out[7] = 0.0;
    out[8] = ct;
    return 0;
  }
  /* total internal reflection: r = (x - i y) / (x + i y), |r| = 1 */
  double kap = sqrt(st2 - 1.0);
  double xs = n1 * ci, ys = n2 * kap;
  double xp = n2 * ci, yp = n1 * kap;
  double qs = xs * xs + ys * ys, qp = xp * xp + yp * yp;
  out[0] = (xs * xs - ys * ys) / qs;
  out[1] = -2.0 * xs * ys / qs;
  out[2] = (xp * xp - yp * yp) / qp;
  out[3] = -2.0 * xp * yp / qp;
  out[4] = out[5] = out[6] = out[7] = 0.0;
  out[8] = 0.0;
  return 1;
}

/* ------------------------------------------------------------------------ */
typedef struct {
  const scene_t* S;
  orc_records* out;
  orc_stats st;
  int64_t* rec_counter; /* shared */
  orc_events* ev;       /* NULL: no event records */
  int64_t* ev_counter;  /* shared */
  orc_trial_log* log;   /* NULL: no trial log */
} worker_t;

static void log_trial(worker_t* W, double h, double err, int32_t outcome) {
  orc_trial_log* L = W->log;
  if (!L || L->n >= L->cap) return;
  L->h[L->n] = h;
  L->err[L->n] = err;
  L->outcome[L->n] = outcome;
  L->n++;
}

/* Event record of a Fresnel event of ray r at boundary k (r holds the state
 * on the boundary and the incident amplitudes; u the incident direction). */
static void emit_event(worker_t* W, const ray_t* r, int k, int32_t reg_out,
                       const double u[3], double ci, double n1, double n2,
                       const double fr[9], int32_t outcome) {
  if (!W->ev) return;
  int64_t e = __atomic_fetch_add(W->ev_counter, 1, __ATOMIC_RELAXED);
  orc_events* E = W->ev;
  if (e >= E->capacity) return;
  E->key[e] = r->key;
  E->ordinal[e] = r->n_ev;
  E->boundary[e] = k;
  E->outcome[e] = outcome;
  E->gen[e] = r->gen;
  E->region_in[e] = r->region;
  E->region_out[e] = reg_out;
  for (int a = 0; a < 3; ++a) {
    E->pos[3 * e + a] = r->y[a];
    E->dir[3 * e + a] = u[a];
  }
  E->s[e] = r->s;
  E->t[e] = r->y[6];
  E->cos_i[e] = ci;
  E->n1[e] = n1;
  E->n2[e] = n2;
  E->amp[4 * e + 0] = r->as_re;
  E->amp[4 * e + 1] = r->as_im;
  E->amp[4 * e + 2] = r->ap_re;
  E->amp[4 * e + 3] = r->ap_im;
  for (int a = 0; a < 8; ++a) E->coef[8 * e + a] = fr[a];
}

static void emit(worker_t* W, const ray_t* r, int32_t status) {
  int64_t slot = __atomic_fetch_add(W->rec_counter, 1, __ATOMIC_RELAXED);
  W->st.records++;
  if (slot >= W->out->capacity) return;
  orc_records* o = W->out;
  double u[3];
  unit_direction(r->y, u);
  o->x[slot] = r->y[0];
  o->y[slot] = r->y[1];
  o->z[slot] = r->y[2];
  o->ux[slot] = u[0];
  o->uy[slot] = u[1];
  o->uz[slot] = u[2];
  o->s[slot] = r->s;
  o->t[slot] = r->y[6];
  o->as_re[slot] = r->as_re;
  o->as_im[slot] = r->as_im;
  o->ap_re[slot] = r->ap_re;
  o->ap_im[slot] = r->ap_im;
  o->h[slot] = r->h;
  o->key[slot] = r->key;
  o->parent[slot] = r->parent;
  o->gen[slot] = r->gen;
  o->status[slot] = status;
  o->n_acc[slot] = r->n_acc;
  o->n_rej[slot] = r->n_rej;
  o->n_ev[slot] = r->n_ev;
  o->region[slot] = r->region;
}

typedef struct {
  ray_t* v;
  int64_t n, cap, head;
} fifo_t;

static void fifo_push(fifo_t* q, const ray_t* r) {
  if (q->n == q->cap) {
    q->cap = q->cap ? 2 * q->cap : 16;
    q->v = (ray_t*)realloc(q->v, (size_t)q->cap * sizeof(ray_t));
  }
  q->v[q->n++] = *r;
}

/* Illinois false-position search for the root of G(sigma) = side * g(y(sigma))
 * on [a, b] with G(a) = Ga > 0 >= G(b) = Gb, where y(sigma) is the Cash-Karp
 * step of length sigma from y0.  Returns sigma* and the state there. */
static double locate(worker_t* W, const ray_t* r, int k, double a, double Ga,
                     double b, double Gb, double hp, double ystar[7]) {
  const scene_t* S = W->S;
  double sg = S->pl[k].kind == KIND_TIME ? 1.0 : side_sign(r, k);
  double c = b, dl[7];
  int last = 0;
  for (int it = 0; it < LOC_MAXIT; ++it) {
    c = b - Gb * (b - a) / (Gb - Ga);
    orc_ck_trial(S->P, r->region, r->y, c, ystar, dl);
    W->st.relocation++;
    double Gc = sg * bnd_g(S, k, ystar);
    if (Gc == 0.0) break;
    if (Gc < 0.0) {
      b = c;
      Gb = Gc;
      if (last == -1) Ga *= 0.5;
      last = -1;
    } else {
      a = c;
      Ga = Gc;
      if (last == 1) Gb *= 0.5;
      last = 1;
    }
    if (b - a <= LOC_WREL * hp) break;
  }
  return c;
}

static double G_of(const scene_t* S, const ray_t* r, int k, const double y[7]) {
  double sg = S->pl[k].kind == KIND_TIME ? 1.0 : side_sign(r, k);
  return sg * bnd_g(S, k, y);
}

/* True when the ray, standing on boundary k, moves away from it into its
 * own side: its direction has a positive component along the normal that
 * points into that side.  A ray only approaches the travel-time limit. */
static int leaving(const scene_t* S, const ray_t* r, int k) {
  if (S->pl[k].kind == KIND_TIME) return 0;
  double nb[3], u[3];
  bnd_normal(S, k, r->y, nb);
  unit_direction(r->y, u);
  return side_sign(r, k) * (u[0] * nb[0] + u[1] * nb[1] + u[2] * nb[2]) > 0.0;
}

/* The crossing of boundary k on the step [0, len] (G0 = G at the start,
 * G1 <= 0 at the end).  A ray passes a boundary only by going through it
 * (section 2, boundary paragraph).  A ray that starts on the boundary
 * (G0 <= ON_BND) and heads into it passes it at sigma = 0.  One that starts
 * on it and leaves it (after an event, the reflected ray and the secondary
 * do) passes it only where it comes back, e.g. at the far end of a short
 * chord through a sphere: the search then starts from the first of len/2,
 * len/4, ... at which the ray is clearly on its own side (G > ON_BND), and
 * the crossing is placed at sigma = 0 when there is none. */
static double crossing(worker_t* W, const ray_t* r, int k, double G0, double len,
                       double G1, double hp, double ystar[7]) {
  if (G0 > ON_BND) return locate(W, r, k, 0.0, G0, len, G1, hp, ystar);
  if (leaving(W->S, r, k)) {
    double a = len, dl[7];
    for (int it = 0; it < LOC_MAXIT; ++it) {
      a *= 0.5;
      orc_ck_trial(W->S->P, r->region, r->y, a, ystar, dl);
      W->st.relocation++;
      const double Ga = G_of(W->S, r, k, ystar);
      if (Ga > ON_BND) return locate(W, r, k, a, Ga, len, G1, hp, ystar);
    }
  }
  memcpy(ystar, r->y, 7 * sizeof(double));
  return 0.0;
}

/* Among the boundaries crossed at the end of a step (G1 <= 0, except 'skip'),
 * pick the one whose linear estimate of the crossing point is earliest. */
static int pick_crossing(const scene_t* S, const ray_t* r, const double y0[7],
                         const double y1[7], double len, int skip, double* G0o,
                         double* G1o) {
  int best = -1;
  double best_sig = 0.0;
  for (int k = 0; k < S->n_pl; ++k) {
    if (k == skip) continue;
    double G1 = G_of(S, r, k, y1);
    if (!(G1 <= 0.0)) continue;
    double G0 = G_of(S, r, k, y0);
    double sig = G0 <= 0.0 ? 0.0 : len * G0 / (G0 - G1);
    if (best < 0 || sig < best_sig) {
      best = k;
      best_sig = sig;
      *G0o = G0;
      *G1o = G1;
    }
  }
  return best;
}

static void trace_tree(worker_t* W, const ray_t* root) {
  const scene_t* S = W->S;
  const orc_problem* P = S->P;
  fifo_t q = {0};
  fifo_push(&q, root);
  while (q.head < q.n) {
    ray_t r = q.v[q.head++];
    /* start of a ray: unit direction, and p = n u in the exact model */
    {
      double u[3] = {r.y[3], r.y[4], r.y[5]};
      set_direction(P, r.region, r.y, u);
    }
    if (r.gen > W->st.max_gen) W->st.max_gen = r.gen;
    int32_t status = 0;
    for (;;) {
      if (r.s >= P->s_max) {
        status = ORC_ST_PATH;
        break;
      }
      if ((int64_t)r.n_acc + r.n_rej >= P->max_steps) {
        status = ORC_ST_STEPCAP;
        break;
      }
      /* trial step, clipped so the last step lands on the path limit */
      double hp = r.h;
      int clipped = 0;
      if (P->s_max - r.s <= hp) {
        hp = P->s_max - r.s;
        clipped = 1;
      }
      double y1[7], dl[7];
      orc_ck_trial(P, r.region, r.y, hp, y1, dl);
      double err = trial_error(r.y, dl, hp, P->tol);
      if (!all_finite(y1, 7) || !isfinite(err)) {
        W->st.nonfinite++;
        status = ORC_ST_NONFINITE;
        break;
      }
      log_trial(W, hp, err, !(err <= 1.0) ? (hp <= P->h_min ? 2 : 0) : 1);
      if (!(err <= 1.0) && !(hp <= P->h_min)) {
        /* rejected: shrink and retry */
        r.n_rej++;
        W->st.rejected++;
        double f = SAFETY * pow(err, -0.25);
        if (f < SHRINK_MIN) f = SHRINK_MIN;
        r.h = clamp_h(P, hp * f);
        continue;
      }
      /* accepted (forced when the step is already at the minimum) */
      r.n_acc++;
      W->st.accepted++;
      if (err > 1.0) W->st.forced++;
      double f = err < ERRCON ? GROW_MAX : SAFETY * pow(err, -0.2);
      double h_next = clamp_h(P, hp * f);
      if (P->model == ORC_MODEL_PAPER) {
        double u[3];
        unit_direction(y1, u);
        y1[3] = u[0];
        y1[4] = u[1];
        y1[5] = u[2];
      }

      /* boundary crossings at the end of the step */
      double G0, G1;
      int k = pick_crossing(S, &r, r.y, y1, hp, -1, &G0, &G1);
      if (k < 0) {
        memcpy(r.y, y1, sizeof y1);
        r.s = clipped ? P->s_max : r.s + hp;
        r.h = h_next;
        if (clipped) {
          status = ORC_ST_PATH;
          break;
        }
        continue;
      }

      /* locate the earliest crossing on the Cash-Karp step map */
      double ystar[7];
      double sig = crossing(W, &r, k, G0, hp, G1, hp, ystar);
      for (int pass = 0; pass < LOC_MAXPASS; ++pass) {
        double H0, H1;
        int j = pick_crossing(S, &r, r.y, ystar, sig, k, &H0, &H1);
        if (j < 0) break;
        k = j;
        sig = crossing(W, &r, k, H0, sig, H1, hp, ystar);
      }
      const bplane_t* b = &S->pl[k];
      bnd_snap(S, k, ystar);
      {
        double u[3];
        unit_direction(ystar, u);
        memcpy(r.y, ystar, sizeof ystar);
        set_direction(P, r.region, r.y, u);
      }
      r.s = r.s + sig;
      r.h = h_next;
      if (b->kind == KIND_BOX) {
        status = ORC_ST_BOX;
        break;
      }
      if (b->kind == KIND_TIME) {
        status = ORC_ST_TIME;
        break;
      }
      if (b->kind == KIND_ABSORB) {
        status = ORC_ST_ABSORB;
        break;
      }
      /* Fresnel boundary: the ray reflects, a refracted secondary is cast */
      if (r.n_ev >= MAX_EVENTS) {
        status = ORC_ST_STEPCAP;
        break;
      }
      r.n_ev++;
      W->st.events++;
      double sgn = side_sign(&r, k);
      double nb[3];
      bnd_normal(S, k, r.y, nb);
      double nin[3] = {sgn * nb[0], sgn * nb[1], sgn * nb[2]};
      double u[3];
      unit_direction(r.y, u);
      double ci = -(u[0] * nin[0] + u[1] * nin[1] + u[2] * nin[2]);
      if (ci < 0.0) ci = 0.0;
      int reg_out = sgn > 0.0 ? b->reg_neg : b->reg_pos;
      double n1, n2, gtmp[3];
      orc_field(P, r.region, r.y, &n1, gtmp);
      orc_field(P, reg_out, r.y, &n2, gtmp);
      double fr[9];
      int tir = orc_fresnel(n1, n2, ci, fr);
      int32_t outcome = tir ? ORC_EV_TIR : ORC_EV_GEN;

      if (!tir) {
        if (r.gen + 1 < P->max_gen) {
          ray_t c = r;
          double eta = n1 / n2;
          double ut[3];
          for (int i = 0; i < 3; ++i)
            ut[i] = eta * u[i] + (eta * ci - fr[8]) * nin[i];
          c.as_re = r.as_re * fr[4] - r.as_im * fr[5];
          c.as_im = r.as_re * fr[5] + r.as_im * fr[4];
          c.ap_re = r.ap_re * fr[6] - r.ap_im * fr[7];
          c.ap_im = r.ap_re * fr[7] + r.ap_im * fr[6];
          c.y[3] = ut[0];
          c.y[4] = ut[1];
          c.y[5] = ut[2];
          c.region = reg_out;
          c.side = r.side ^ (1u << k);
          c.gen = r.gen + 1;
          c.parent = r.key;
          c.key = r.key | ((uint64_t)r.n_ev << (8 * (2 - r.gen)));
          c.n_acc = c.n_rej = c.n_ev = 0;
          double amax = fmax(hypot(c.as_re, c.as_im), hypot(c.ap_re, c.ap_im));
          if (P->amp_min > 0.0 && amax < P->amp_min) {
            W->st.suppressed_amp++;
            outcome = ORC_EV_AMP;
          } else {
            W->st.spawned++;
            outcome = ORC_EV_SPAWNED;
            fifo_push(&q, &c);
          }
        } else {
          W->st.suppressed_gen++;
        }
      }
      emit_event(W, &r, k, reg_out, u, ci, n1, n2, fr, outcome);
      /* the parent continues as the reflected ray */
      {
        double ur[3];
        for (int i = 0; i < 3; ++i) ur[i] = u[i] + 2.0 * ci * nin[i];
        double are = r.as_re * fr[0] - r.as_im * fr[1];
        double aim = r.as_re * fr[1] + r.as_im * fr[0];
        double pre = r.ap_re * fr[2] - r.ap_im * fr[3];
        double pim = r.ap_re * fr[3] + r.ap_im * fr[2];
        r.as_re = are;
        r.as_im = aim;
        r.ap_re = pre;
        r.ap_im = pim;
        set_direction(P, r.region, r.y, ur);
      }
      if (P->amp_min > 0.0 &&
          fmax(hypot(r.as_re, r.as_im), hypot(r.ap_re, r.ap_im)) < P->amp_min) {
        status = ORC_ST_AMP;
        break;
      }
    }
    emit(W, &r, status);
  }
  free(q.v);
}

/* Launch state of root ray i (section 2: rays start at their source with
 * unit amplitude in both polarisations). */
static void make_root(const scene_t* S, int64_t i, ray_t* r) {
  const orc_problem* P = S->P;
  memset(r, 0, sizeof *r);
  int src = P->ray_src[i];
  for (int a = 0; a < 3; ++a) {
    r->y[a] = P->src_xyz[3 * src + a];
    r->y[3 + a] = P->dir_xyz[3 * i + a];
  }
  r->y[6] = 0.0;
  r->region = 0;
  for (int g = 0; g < P->n_regions; ++g) {
    if (r->y[2] >= P->regions[g].z_top && r->y[2] < P->regions[g].z_bot) {
      r->region = g;
      break;
    }
  }
  for (int k = 0; k < S->n_pl; ++k) {
    if (S->pl[k].kind == KIND_TIME) continue;
    if (bnd_g(S, k, r->y) > 0.0) r->side |= 1u << k;
  }
  r->as_re = 1.0;
  r->ap_re = 1.0;
  r->h = P->h_init > 0.0 ? P->h_init : P->h_max;
  r->key = (uint64_t)i << 24;
  r->parent = ~(uint64_t)0;
}

typedef struct {
  worker_t W;
  const int64_t* roots;
  int64_t n_roots;
  int64_t* next;
  pthread_t th;
} job_t;

#define CHUNK 16
static void* run_job(void* arg) {
  job_t* J = (job_t*)arg;
  for (;;) {
    int64_t i0 = __atomic_fetch_add(J->next, CHUNK, __ATOMIC_RELAXED);
    if (i0 >= J->n_roots) break;
    int64_t i1 = i0 + CHUNK < J->n_roots ? i0 + CHUNK : J->n_roots;
    for (int64_t i = i0; i < i1; ++i) {
      ray_t r;
      make_root(J->W.S, J->roots ? J->roots[i] : i, &r);
      trace_tree(&J->W, &r);
    }
  }
  return NULL;
}

int orc_trace(const orc_problem* P, const int64_t* roots, int64_t n_roots,
              orc_records* out, orc_stats* stats, int n_threads) {
  int64_t n_events;
  return orc_trace_events(P, roots, n_roots, out, stats, NULL, &n_events, n_threads);
}

static int trace_impl(const orc_problem* P, const int64_t* roots, int64_t n_roots,
                      orc_records* out, orc_stats* stats, orc_events* ev, int64_t* n_events,
                      int n_threads, orc_trial_log* log) {
  scene_t S;
  if (P->max_gen < 1 || P->max_gen > 4 || P->n_planes > 16) return -2;
  build_scene(P, &S);
  if (!roots) n_roots = P->n_rays;
  if (n_threads < 1) n_threads = 1;
  int64_t counter = 0, next = 0, ev_counter = 0;
  job_t* jobs = (job_t*)calloc((size_t)n_threads, sizeof(job_t));
  for (int t = 0; t < n_threads; ++t) {
    jobs[t].W.S = &S;
    jobs[t].W.out = out;
    jobs[t].W.rec_counter = &counter;
    jobs[t].W.ev = ev;
    jobs[t].W.ev_counter = &ev_counter;
    jobs[t].W.log = log;
    jobs[t].roots = roots;
    jobs[t].n_roots = n_roots;
    jobs[t].next = &next;
  }
  if (n_threads == 1) {
    run_job(&jobs[0]);
  } else {
    for (int t = 0; t < n_threads; ++t)
      pthread_create(&jobs[t].th, NULL, run_job, &jobs[t]);
    for (int t = 0; t < n_threads; ++t) pthread_join(jobs[t].th, NULL);
  }
  memset(stats, 0, sizeof *stats);
  for (int t = 0; t < n_threads; ++t) {
    orc_stats* s = &jobs[t].W.st;
    stats->accepted += s->accepted;
    stats->rejected += s->rejected;
    stats->relocation += s->relocation;
    stats->forced += s->forced;
    stats->events += s->events;
    stats->spawned += s->spawned;
    stats->suppressed_gen += s->suppressed_gen;
    stats->suppressed_amp += s->suppressed_amp;
    stats->records += s->records;
    stats->nonfinite += s->nonfinite;
    if (s->max_gen > stats->max_gen) stats->max_gen = s->max_gen;
  }
  stats->needed = counter;
  *n_events = ev_counter;
  free(jobs);
  if (counter > out->capacity) return -1;
  return ev && ev_counter > ev->capacity ? -3 : 0;
}

int orc_trace_events(const orc_problem* P, const int64_t* roots, int64_t n_roots,
                     orc_records* out, orc_stats* stats, orc_events* ev,
                     int64_t* n_events, int n_threads) {
  return trace_impl(P, roots, n_roots, out, stats, ev, n_events, n_threads, NULL);
}

int orc_trace_log(const orc_problem* P, const int64_t* roots, int64_t n_roots,
                  orc_records* out, orc_stats* stats, orc_trial_log* log) {
  int64_t n_events;
  if (log) log->n = 0;
  return trace_impl(P, roots, n_roots, out, stats, NULL, &n_events, 1, log);
}

/* ======================================================================== */
/* Emitter -> receiver solves by shooting (the paper's "receiver/emitter     */
/* locations", section 2): for a source and a receiver, find the launch     */
/* angles of the direct ray and of the ray reflected once at the surface.   */

enum { SHOT_RECV = 0, SHOT_SURF = 1, SHOT_LOST = 2, SHOT_INVALID = 3 };
#define SHOT_MISS_HIGH (-1.0e6) /* ray ended above the receiver (at the surface) */
#define SHOT_MISS_LOW (1.0e6)   /* ray lost: never reached the receiver plane */

typedef struct {
  int32_t status, n_acc, n_rej;
  double miss, t, s, as_re, as_im, ap_re, ap_im;
} shot_t;

/* A source/receiver pair can be shot if every value is finite, the distance
 * is positive and the source is not within 1e-9 m of a plane (its side of
 * every plane must be defined). */
static int pair_ok(const scene_t* S, double zs, double zr, double D) {
  if (!isfinite(zs) || !isfinite(zr) || !isfinite(D) || !(D > 0.0)) return 0;
  const double y[7] = {0.0, 0.0, zs, 0.0, 0.0, 0.0, 0.0};
  for (int k = 0; k < S->n_pl; ++k)
    if (fabs(bnd_g(S, k, y)) <= 1e-9) return 0;
  return 1;
}

/* Append the receiver plane x = D to a copy of the base scene:
 * g = D - x > 0 on the source side. */
static void add_receiver(scene_t* S, double D) {
  bplane_t* rp = &S->pl[S->n_pl++];
  memset(rp, 0, sizeof *rp);
  rp->nrm[0] = -1.0;
  rp->d = -D;
  rp->kind = KIND_ABSORB;
}

/* One branch-following trace at launch angle theta (from the upward vertical,
 * towards +x).  The receiver plane x = D is the last boundary of S. */
static shot_t shoot(worker_t* W, const scene_t* S, double zs, double zr, double D, double theta,
                    int family) {
  const orc_problem* P = S->P;
  const int k_recv = S->n_pl - 1;
  const double z_surf = S->pl[0].d * S->pl[0].nrm[2];
  const double s_max = 2.0 * (D + zs + zr) + 1000.0;
  shot_t out;
  memset(&out, 0, sizeof out);
  ray_t r;
  memset(&r, 0, sizeof r);
  r.y[2] = zs;
  double u0[3] = {sin(theta), 0.0, -cos(theta)};
  for (int g = 0; g < P->n_regions; ++g)
    if (zs >= P->regions[g].z_top && zs < P->regions[g].z_bot) {
      r.region = g;
      break;
    }
  for (int k = 0; k < S->n_pl; ++k)
    if (bnd_g(S, k, r.y) > 0.0) r.side |= 1u << k;
  r.as_re = r.ap_re = 1.0;
  r.h = P->h_init > 0.0 ? P->h_init : P->h_max;
  set_direction(P, r.region, r.y, u0);
  int n_refl = 0;
  for (;;) {
    if (r.s >= s_max || (int64_t)r.n_acc + r.n_rej >= P->max_steps) break;
    double hp = r.h;
    int clipped = 0;
    if (s_max - r.s <= hp) {
      hp = s_max - r.s;
      clipped = 1;
    }
    double y1[7], dl[7];
    orc_ck_trial(P, r.region, r.y, hp, y1, dl);
    double err = trial_error(r.y, dl, hp, P->tol);
    if (!all_finite(y1, 7) || !isfinite(err)) break;
    if (!(err <= 1.0) && !(hp <= P->h_min)) {
      r.n_rej++;
      W->st.rejected++;
      double f = SAFETY * pow(err, -0.25);
      if (f < SHRINK_MIN) f = SHRINK_MIN;
      r.h = clamp_h(P, hp * f);
      continue;
    }
    r.n_acc++;
    W->st.accepted++;
    double f = err < ERRCON ? GROW_MAX : SAFETY * pow(err, -0.2);
    double h_next = clamp_h(P, hp * f);
    if (P->model == ORC_MODEL_PAPER) {
      double u[3];
      unit_direction(y1, u);
      y1[3] = u[0];
      y1[4] = u[1];
      y1[5] = u[2];
    }
    double G0, G1;
    int k = pick_crossing(S, &r, r.y, y1, hp, -1, &G0, &G1);
    if (k < 0) {
      memcpy(r.y, y1, sizeof y1);
      r.s = clipped ? s_max : r.s + hp;
      r.h = h_next;
      continue;
    }
    double ystar[7];
    double sig = crossing(W, &r, k, G0, hp, G1, hp, ystar);
    for (int pass = 0; pass < LOC_MAXPASS; ++pass) {
      double H0, H1;
      int j = pick_crossing(S, &r, r.y, ystar, sig, k, &H0, &H1);
      if (j < 0) break;
      k = j;
      sig = crossing(W, &r, k, H0, sig, H1, hp, ystar);
    }
    const bplane_t* b = &S->pl[k];
    bnd_snap(S, k, ystar);
    {
      double u[3];
      unit_direction(ystar, u);
      memcpy(r.y, ystar, sizeof ystar);
      set_direction(P, r.region, r.y, u);
    }
    r.s = r.s + sig;
    r.h = h_next;
    if (k == k_recv) {
      /* before its reflection a ray of the reflected family is measured in
       * the mirror image of the surface */
      double z = r.y[2];
      if (family == ORC_FAMILY_REFLECTED && n_refl == 0) z = 2.0 * z_surf - z;
      out.status = SHOT_RECV;
      out.n_acc = r.n_acc;
      out.n_rej = r.n_rej;
      out.miss = z - zr;
      out.t = r.y[6];
      out.s = r.s;
      out.as_re = r.as_re;
      out.as_im = r.as_im;
      out.ap_re = r.ap_re;
      out.ap_im = r.ap_im;
      return out;
    }
    if (b->kind != KIND_FRESNEL) break; /* box, time or absorbing plane */
    const int surface = (k == 0);
    if (surface && (family == ORC_FAMILY_DIRECT || n_refl > 0)) {
      out.status = SHOT_SURF;
      out.n_acc = r.n_acc;
      out.n_rej = r.n_rej;
      out.miss = SHOT_MISS_HIGH;
      return out;
    }
    /* Fresnel at the plane: reflect at the surface, transmit at a layer
     * (reflect when totally reflected) */
    double sgn = side_sign(&r, k);
    double nin[3] = {sgn * b->nrm[0], sgn * b->nrm[1], sgn * b->nrm[2]};
    double u[3];
    unit_direction(r.y, u);
    double ci = -(u[0] * nin[0] + u[1] * nin[1] + u[2] * nin[2]);
    if (ci < 0.0) ci = 0.0;
    int reg_out = sgn > 0.0 ? b->reg_neg : b->reg_pos;
    double n1, n2, gtmp[3];
    orc_field(P, r.region, r.y, &n1, gtmp);
    orc_field(P, reg_out, r.y, &n2, gtmp);
    double fr[9];
    int tir = orc_fresnel(n1, n2, ci, fr);
    if (surface || tir) {
      double ur[3];
      for (int i = 0; i < 3; ++i) ur[i] = u[i] + 2.0 * ci * nin[i];
      double are = r.as_re * fr[0] - r.as_im * fr[1];
      double aim = r.as_re * fr[1] + r.as_im * fr[0];
      double pre = r.ap_re * fr[2] - r.ap_im * fr[3];
      double pim = r.ap_re * fr[3] + r.ap_im * fr[2];
      r.as_re = are;
      r.as_im = aim;
      r.ap_re = pre;
      r.ap_im = pim;
      set_direction(P, r.region, r.y, ur);
      if (surface) n_refl++;
    } else {
      double eta = n1 / n2, ut[3];
      for (int i = 0; i < 3; ++i) ut[i] = eta * u[i] + (eta * ci - fr[8]) * nin[i];
      double are = r.as_re * fr[4] - r.as_im * fr[5];
      double aim = r.as_re * fr[5] + r.as_im * fr[4];
      double pre = r.ap_re * fr[6] - r.ap_im * fr[7];
      double pim = r.ap_re * fr[7] + r.ap_im * fr[6];
      r.as_re = are;
      r.as_im = aim;
      r.ap_re = pre;
      r.ap_im = pim;
      r.region = reg_out;
      r.side ^= 1u << k;
      set_direction(P, r.region, r.y, ut);
    }
  }
  out.status = SHOT_LOST;
  out.n_acc = r.n_acc;
  out.n_rej = r.n_rej;
  out.miss = SHOT_MISS_LOW;
  return out;
}

/* Shots follow planes only (the surface mirror and the receiver plane
 * assume them). */
static int planes_only(const orc_problem* P) {
  for (int k = 0; k < P->n_planes; ++k)
    if (P->planes[k].shape != ORC_SHAPE_PLANE) return 0;
  return 1;
}

static int miss_sign(double m) { return m < 0.0 ? -1 : 1; }

/* Refinement of a bracket stops when it is narrower than SOLVE_WIDTH_MIN
 * (rad), or when its end misses cannot belong to a root: a miss that is
 * continuous on [a, b] with |d miss / d theta| <= slope_max and a zero
 * inside has |miss(a)| + |miss(b)| <= slope_max (b - a); ends that are
 * failed shots (|miss| >= 1e5) contribute nothing.  Brackets around jumps of
 * the miss (a shot starting to touch the surface or to get lost, total
 * reflection setting in at a layer) end this way instead of being bisected
 * down to rounding. */
#define SOLVE_WIDTH_MIN 1.0e-9
static double finite_miss(double m) { return fabs(m) < 1.0e5 ? fabs(m) : 0.0; }

/* Refine a bracket [a, b] of the miss by Illinois false position (plain
 * bisection while an end is a failed shot). */
static shot_t refine(worker_t* W, const scene_t* S, const orc_solve_spec* sp, double zs, double zr,
                     double D, int family, double a, double Ga, double b, double Gb,
                     double* theta, int* shots) {
  shot_t sh;
  memset(&sh, 0, sizeof sh);
  sh.status = SHOT_LOST;
  int last = 0;
  double c = a;
  double ma = Ga, mb = Gb; /* misses at the ends (Ga, Gb get scaled) */
  for (int it = 0; it < sp->max_iter; ++it) {
    if (fabs(Ga) >= 1.0e5 || fabs(Gb) >= 1.0e5)
      c = 0.5 * (a + b);
    else
      c = b - Gb * (b - a) / (Gb - Ga);
    sh = shoot(W, S, zs, zr, D, c, family);
    ++*shots;
    if (sh.status == SHOT_RECV && fabs(sh.miss) <= sp->miss_tol) break;
    if (miss_sign(sh.miss) == miss_sign(Ga)) {
      a = c;
      Ga = ma = sh.miss;
      if (last == 1) Gb *= 0.5;
      last = 1;
    } else {
      b = c;
      Gb = mb = sh.miss;
      if (last == -1) Ga *= 0.5;
      last = -1;
    }
    if (fabs(b - a) <= SOLVE_WIDTH_MIN) break;
    if (sp->slope_max > 0.0 && finite_miss(ma) + finite_miss(mb) > sp->slope_max * fabs(b - a))
      break;
  }
  *theta = c;
  return sh;
}

typedef struct {
  const scene_t* base;
  const orc_solve_spec* sp;
  const int64_t* pairs;
  int64_t n;
  int64_t* next;
  orc_solve_out* out;
  worker_t W;
  pthread_t th;
} solve_job_t;

static void solve_one(worker_t* W, const scene_t* base, const orc_solve_spec* sp, int64_t i,
                      orc_solve_out* out) {
  const double zs = sp->zs[i], zr = sp->zr[i], D = sp->dist[i];
  if (!pair_ok(base, zs, zr, D)) {
    for (int family = 0; family < 2; ++family) {
      const int64_t o = 2 * i + family;
      out->found[o] = out->shots[o] = out->roots[o] = 0;
      out->theta[o] = out->miss[o] = out->t[o] = out->s[o] = 0.0;
      out->as_re[o] = out->as_im[o] = out->ap_re[o] = out->ap_im[o] = 0.0;
    }
    return;
  }
  scene_t S = *base;
  add_receiver(&S, D);
  const scene_t* saved = W->S; /* crossing location reads the worker's scene */
  W->S = &S;
  for (int family = 0; family < 2; ++family) {
    const int64_t o = 2 * i + family;
    int shots = 0, found = 0, brackets = 0, roots = 0;
    double best_theta = 0.0;
    shot_t best;
    memset(&best, 0, sizeof best);
    shot_t prev;
    double th_prev = 0.0;
    for (int k = 0; k < sp->n_scan; ++k) {
      double th = (k + 0.5) * (3.14159265358979323846 / sp->n_scan);
      shot_t sh = shoot(W, &S, zs, zr, D, th, family);
      ++shots;
      if (k > 0 && miss_sign(sh.miss) != miss_sign(prev.miss)) {
        double root;
        shot_t rs = refine(W, &S, sp, zs, zr, D, family, th_prev, prev.miss, th, sh.miss, &root,
                           &shots);
        const int admissible = rs.status == SHOT_RECV && fabs(rs.miss) <= sp->accept_tol;
        roots += admissible;
        if (admissible && (!found || rs.t < best.t)) {
          best = rs;
          best_theta = root;
          found = 1;
        }
        if (++brackets >= sp->max_brackets) break;
      }
      prev = sh;
      th_prev = th;
    }
    out->found[o] = found;
    out->shots[o] = shots;
    out->roots[o] = roots;
    out->theta[o] = found ? best_theta : 0.0;
    out->miss[o] = best.miss;
    out->t[o] = best.t;
    out->s[o] = best.s;
    out->as_re[o] = best.as_re;
    out->as_im[o] = best.as_im;
    out->ap_re[o] = best.ap_re;
    out->ap_im[o] = best.ap_im;
  }
  W->S = saved;
}

static void* run_solve(void* arg) {
  solve_job_t* J = (solve_job_t*)arg;
  for (;;) {
    int64_t j = __atomic_fetch_add(J->next, 1, __ATOMIC_RELAXED);
    if (j >= J->n) break;
    solve_one(&J->W, J->base, J->sp, J->pairs ? J->pairs[j] : j, J->out);
  }
  return NULL;
}

typedef struct {
  const scene_t* base;
  const double *zs, *zr, *dist, *theta;
  const int32_t* family;
  int64_t n;
  int64_t* next;
  orc_shot_out* out;
  worker_t W;
  pthread_t th;
} shoot_job_t;

static void* run_shoot(void* arg) {
  shoot_job_t* J = (shoot_job_t*)arg;
  for (;;) {
    int64_t i = __atomic_fetch_add(J->next, 1, __ATOMIC_RELAXED);
    if (i >= J->n) break;
    const double zs = J->zs[i], zr = J->zr[i], D = J->dist[i], th = J->theta[i];
    const int32_t fam = J->family[i];
    shot_t sh;
    memset(&sh, 0, sizeof sh);
    if (!pair_ok(J->base, zs, zr, D) || !(th > 0.0 && th < 3.14159265358979323846) ||
        (fam != ORC_FAMILY_DIRECT && fam != ORC_FAMILY_REFLECTED)) {
      sh.status = SHOT_INVALID;
    } else {
      scene_t S = *J->base;
      add_receiver(&S, D);
      J->W.S = &S;
      sh = shoot(&J->W, &S, zs, zr, D, th, fam);
      J->W.S = J->base;
    }
    orc_shot_out* o = J->out;
    o->status[i] = sh.status;
    o->n_acc[i] = sh.n_acc;
    o->n_rej[i] = sh.n_rej;
    o->miss[i] = sh.miss;
    o->t[i] = sh.t;
    o->s[i] = sh.s;
    o->as_re[i] = sh.as_re;
    o->as_im[i] = sh.as_im;
    o->ap_re[i] = sh.ap_re;
    o->ap_im[i] = sh.ap_im;
  }
  return NULL;
}

int orc_shoot(const orc_problem* P, const double* zs, const double* zr, const double* dist,
              const double* theta, const int32_t* family, int64_t n, orc_shot_out* out,
              int n_threads) {
  if (P->n_planes < 1 || P->n_planes > 16 || P->has_box || P->t_max > 0.0 || !planes_only(P))
    return -2;
  scene_t S;
  build_scene(P, &S);
  if (n_threads < 1) n_threads = 1;
  int64_t next = 0;
  shoot_job_t* jobs = (shoot_job_t*)calloc((size_t)n_threads, sizeof(shoot_job_t));
  for (int t = 0; t < n_threads; ++t) {
    shoot_job_t* J = &jobs[t];
    J->base = &S;
    J->zs = zs;
    J->zr = zr;
    J->dist = dist;
    J->theta = theta;
    J->family = family;
    J->n = n;
    J->next = &next;
    J->out = out;
    J->W.S = &S;
  }
  if (n_threads == 1) {
    run_shoot(&jobs[0]);
  } else {
    for (int t = 0; t < n_threads; ++t) pthread_create(&jobs[t].th, NULL, run_shoot, &jobs[t]);
    for (int t = 0; t < n_threads; ++t) pthread_join(jobs[t].th, NULL);
  }
  free(jobs);
  return 0;
}

/* Seeded secant of one entry (see oracle.h). */
static void seeded_one(worker_t* W, const scene_t* base, const double* zs_, const double* zr_,
                       const double* dist_, const double* seed, const orc_seed_spec* sp,
                       int64_t e, orc_solve_out* out, int32_t* verify) {
  const double PI = 3.14159265358979323846;
  const int64_t i = e / 2;
  const int family = (int)(e % 2);
  const double zs = zs_[i], zr = zr_[i], D = dist_[i];
  double c = seed[e];
  int shots = 0, success = 0;
  shot_t sh;
  memset(&sh, 0, sizeof sh);
  if (pair_ok(base, zs, zr, D) && c > 0.0 && c < PI) {
    scene_t S = *base;
    add_receiver(&S, D);
    const scene_t* saved = W->S;
    W->S = &S;
    double cp = 0.0, mp = 0.0;
    for (;;) {
      sh = shoot(W, &S, zs, zr, D, c, family);
      ++shots;
      const int recv = sh.status == SHOT_RECV;
      success = recv && fabs(sh.miss) <= sp->verify_tol;
      if (success || !recv || shots >= sp->max_shots) break;
      double cn;
      if (shots == 1)
        cn = c + sp->dseed < PI ? c + sp->dseed : c - sp->dseed;
      else
        cn = c - sh.miss * (c - cp) / (sh.miss - mp);
      if (!(cn > 0.0 && cn < PI)) break;
      cp = c;
      mp = sh.miss;
      c = cn;
    }
    W->S = saved;
  }
  out->found[e] = success;
  out->shots[e] = shots;
  out->roots[e] = success;
  out->theta[e] = success ? c : 0.0;
  out->miss[e] = success ? sh.miss : 0.0;
  out->t[e] = success ? sh.t : 0.0;
  out->s[e] = success ? sh.s : 0.0;
  out->as_re[e] = success ? sh.as_re : 0.0;
  out->as_im[e] = success ? sh.as_im : 0.0;
  out->ap_re[e] = success ? sh.ap_re : 0.0;
  out->ap_im[e] = success ? sh.ap_im : 0.0;
  verify[e] = success;
}

typedef struct {
  const scene_t* base;
  const double *zs, *zr, *dist, *seed;
  const int32_t* try_;
  const orc_seed_spec* sp;
  int64_t n;
  int64_t* next;
  orc_solve_out* out;
  int32_t* verify;
  worker_t W;
  pthread_t th;
} seeded_job_t;

static void* run_seeded(void* arg) {
  seeded_job_t* J = (seeded_job_t*)arg;
  for (;;) {
    int64_t e = __atomic_fetch_add(J->next, 1, __ATOMIC_RELAXED);
    if (e >= J->n) break;
    if (J->try_[e])
      seeded_one(&J->W, J->base, J->zs, J->zr, J->dist, J->seed, J->sp, e, J->out, J->verify);
  }
  return NULL;
}

int orc_solve_seeded(const orc_problem* P, const double* zs, const double* zr,
                     const double* dist, int64_t n_pairs, const double* seed,
                     const int32_t* try_, const orc_seed_spec* spec, orc_solve_out* out,
                     int32_t* verify, int n_threads) {
  if (P->n_planes < 1 || P->n_planes > 16 || P->has_box || P->t_max > 0.0 || !planes_only(P))
    return -2;
  scene_t S;
  build_scene(P, &S);
  if (n_threads < 1) n_threads = 1;
  int64_t next = 0;
  seeded_job_t* jobs = (seeded_job_t*)calloc((size_t)n_threads, sizeof(seeded_job_t));
  for (int t = 0; t < n_threads; ++t) {
    seeded_job_t* J = &jobs[t];
    J->base = &S;
    J->zs = zs;
    J->zr = zr;
    J->dist = dist;
    J->seed = seed;
    J->try_ = try_;
    J->sp = spec;
    J->n = 2 * n_pairs;
    J->next = &next;
    J->out = out;
    J->verify = verify;
    J->W.S = &S;
  }
  if (n_threads == 1) {
    run_seeded(&jobs[0]);
  } else {
    for (int t = 0; t < n_threads; ++t) pthread_create(&jobs[t].th, NULL, run_seeded, &jobs[t]);
    for (int t = 0; t < n_threads; ++t) pthread_join(jobs[t].th, NULL);
  }
  free(jobs);
  return 0;
}

int orc_solve(const orc_problem* P, const orc_solve_spec* sp, const int64_t* pairs,
              int64_t n_pairs, orc_solve_out* out, int n_threads) {
  if (P->n_planes < 1 || P->n_planes > 16 || P->has_box || P->t_max > 0.0 || !planes_only(P))
    return -2;
  scene_t S;
  build_scene(P, &S);
  if (n_threads < 1) n_threads = 1;
  int64_t next = 0;
  solve_job_t* jobs = (solve_job_t*)calloc((size_t)n_threads, sizeof(solve_job_t));
  for (int t = 0; t < n_threads; ++t) {
    jobs[t].base = &S;
    jobs[t].sp = sp;
    jobs[t].pairs = pairs;
    jobs[t].n = n_pairs;
    jobs[t].next = &next;
    jobs[t].out = out;
    jobs[t].W.S = &S;
  }
  if (n_threads == 1) {
    run_solve(&jobs[0]);
  } else {
    for (int t = 0; t < n_threads; ++t) pthread_create(&jobs[t].th, NULL, run_solve, &jobs[t]);
    for (int t = 0; t < n_threads; ++t) pthread_join(jobs[t].th, NULL);
  }
  free(jobs);
  return 0;
}
