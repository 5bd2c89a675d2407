// Host-only parts of the C ABI: validation, workspace sizing, status
// collection and the per-thread error message.  No device access here.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "radiotrace_mlp.h"
#include "radiotrace_solve.h"
#include "rt_params.hpp"
#include "rt_solve_internal.hpp"

namespace rt {

static thread_local char g_err[512];

Range::Range(const char* name) { roctxRangePushA(name); }
Range::~Range() { roctxRangePop(); }

void set_last_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
}

bool field_uses_grid(const rt_field* f) {
  for (int i = 0; i < f->n_regions; ++i)
    if (f->regions[i].use_grid) return true;
  return false;
}

static bool finite3(const double* v) {
  return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]);
}

bool field_is_general(const rt_field* f) {
  if (f->n_anomalies > 0) return true;
  for (int i = 0; i < f->n_regions; ++i) {
    const rt_region& r = f->regions[i];
    if (r.use_grid) return true;
    // an axis along +z (any length) or all zero is depth
    if (r.axis[0] != 0.0 || r.axis[1] != 0.0 || r.axis[2] < 0.0) return true;
  }
  return false;
}

#define FAIL(code, ...)            \
  do {                             \
    set_last_error(__VA_ARGS__);   \
    return code;                   \
  } while (0)

rt_status validate(const rt_field* field, const rt_boundaries* bnd, const rt_sources* src,
                   const rt_directions* dirs, double tol, const rt_step_limits* L) {
  if (!field || !bnd || !src || !dirs || !L) FAIL(RT_ERR_INVALID_ARG, "null descriptor");
  if (field->n_regions < 1 || field->n_regions > RT_MAX_REGIONS || !field->regions)
    FAIL(RT_ERR_INVALID_ARG, "n_regions must be 1..%d with a region array", RT_MAX_REGIONS);
  for (int i = 0; i < field->n_regions; ++i) {
    const rt_region& r = field->regions[i];
    if (!std::isfinite(r.a) || !std::isfinite(r.b) || !std::isfinite(r.dn))
      FAIL(RT_ERR_INVALID_ARG, "region %d: non-finite coefficient", i);
    if (r.dn != 0.0 && !(std::isfinite(r.z0) && r.z0 != 0.0))
      FAIL(RT_ERR_INVALID_ARG, "region %d: z0 must be finite and non-zero when dn != 0", i);
    if (std::isnan(r.z_top) || std::isnan(r.z_bot) || !(r.z_top <= r.z_bot))
      FAIL(RT_ERR_INVALID_ARG, "region %d: need z_top <= z_bot", i);
    if (!finite3(r.axis)) FAIL(RT_ERR_INVALID_ARG, "region %d: non-finite axis", i);
  }
  if (field->n_anomalies < 0 || field->n_anomalies > RT_MAX_ANOMALIES ||
      (field->n_anomalies > 0 && !field->anomalies))
    FAIL(RT_ERR_INVALID_ARG, "n_anomalies must be 0..%d with an anomaly array",
         RT_MAX_ANOMALIES);
  for (int j = 0; j < field->n_anomalies; ++j) {
    const rt_anomaly& q = field->anomalies[j];
    if (!finite3(q.centre) || !std::isfinite(q.amplitude))
      FAIL(RT_ERR_INVALID_ARG, "anomaly %d: non-finite centre or amplitude", j);
    if (!(q.sigma > 0.0) || !std::isfinite(q.sigma) || !std::isfinite(1.0 / (q.sigma * q.sigma)))
      FAIL(RT_ERR_INVALID_ARG, "anomaly %d: sigma must be > 0 (and not tiny)", j);
    if (q.region < 0 || q.region >= field->n_regions)
      FAIL(RT_ERR_INVALID_ARG, "anomaly %d: region index out of range", j);
  }
  if (field_uses_grid(field)) {
    const rt_grid& g = field->grid;
    if (!g.n) FAIL(RT_ERR_INVALID_ARG, "grid: null data pointer");
    if (g.nx < 2 || g.ny < 2 || g.nz < 2) FAIL(RT_ERR_INVALID_ARG, "grid: dims must be >= 2");
    // the prepared nodes (2 x 2 x 2 bricks of 128 bytes) are addressed with
    // 32-bit byte offsets
    if ((double)((g.nx + 1) / 2) * ((g.ny + 1) / 2) * ((g.nz + 1) / 2) * 128.0 > 4294967295.0)
      FAIL(RT_ERR_UNSUPPORTED, "grid: the prepared nodes would exceed 4 GiB (about 2.7e8 nodes)");
    for (int a = 0; a < 3; ++a) {
      if (!(g.spacing[a] > 0.0) || !std::isfinite(g.spacing[a]))
        FAIL(RT_ERR_INVALID_ARG, "grid: spacing must be > 0");
      if (!std::isfinite(g.origin[a])) FAIL(RT_ERR_INVALID_ARG, "grid: non-finite origin");
    }
  }
  if (bnd->n_planes < 0 || bnd->n_planes > RT_MAX_PLANES)
    FAIL(RT_ERR_INVALID_ARG, "n_planes must be 0..%d", RT_MAX_PLANES);
  if (bnd->n_planes > 0 && !bnd->planes) FAIL(RT_ERR_INVALID_ARG, "null plane array");
  for (int k = 0; k < bnd->n_planes; ++k) {
    const rt_plane& p = bnd->planes[k];
    if (!finite3(p.point) || !finite3(p.normal))
      FAIL(RT_ERR_INVALID_ARG, "plane %d: non-finite point or normal", k);
    const double l2 = p.normal[0] * p.normal[0] + p.normal[1] * p.normal[1] +
                      p.normal[2] * p.normal[2];
    if (p.shape == RT_SHAPE_PLANE && !(l2 > 0.0))
      FAIL(RT_ERR_INVALID_ARG, "plane %d: zero normal", k);
    if (p.shape != RT_SHAPE_PLANE && p.shape != RT_SHAPE_SPHERE &&
        p.shape != RT_SHAPE_PARABOLOID)
      FAIL(RT_ERR_INVALID_ARG, "plane %d: unknown shape %d", k, p.shape);
    if (p.shape == RT_SHAPE_SPHERE && !(p.param > 0.0 && std::isfinite(p.param)))
      FAIL(RT_ERR_INVALID_ARG, "plane %d: sphere radius must be > 0", k);
    if (p.shape == RT_SHAPE_PARABOLOID && !(p.param != 0.0 && std::isfinite(p.param)))
      FAIL(RT_ERR_INVALID_ARG, "plane %d: paraboloid curvature must be finite and non-zero", k);
    if (p.kind != RT_PLANE_FRESNEL && p.kind != RT_PLANE_ABSORB)
      FAIL(RT_ERR_INVALID_ARG, "plane %d: unknown kind %d", k, p.kind);
    if (p.region_pos < 0 || p.region_pos >= field->n_regions || p.region_neg < 0 ||
        p.region_neg >= field->n_regions)
      FAIL(RT_ERR_INVALID_ARG, "plane %d: region index out of range", k);
  }
  if (bnd->has_box) {
    if (!finite3(bnd->box_lo) || !finite3(bnd->box_hi))
      FAIL(RT_ERR_INVALID_ARG, "box: non-finite bounds");
    for (int a = 0; a < 3; ++a)
      if (!(bnd->box_lo[a] < bnd->box_hi[a])) FAIL(RT_ERR_INVALID_ARG, "box: need lo < hi");
  }
  if (src->n < 0 || (src->n > 0 && !src->xyz)) FAIL(RT_ERR_INVALID_ARG, "bad sources");
  if (dirs->n < 0) FAIL(RT_ERR_INVALID_ARG, "negative ray count");
  if (dirs->n > 0 && (!dirs->xyz || !dirs->src || src->n < 1))
    FAIL(RT_ERR_INVALID_ARG, "rays need direction and source arrays and >= 1 source");
  if (dirs->n > (int64_t)0x7fffffff) FAIL(RT_ERR_UNSUPPORTED, "more than 2^31-1 rays");
  if (!(tol > 0.0) || !std::isfinite(tol)) FAIL(RT_ERR_INVALID_ARG, "tol must be > 0");
  if (!(L->h_min > 0.0) || !(L->h_min <= L->h_max) || !std::isfinite(L->h_max))
    FAIL(RT_ERR_INVALID_ARG, "need 0 < h_min <= h_max");
  if (!(L->h_init >= 0.0) || !std::isfinite(L->h_init))
    FAIL(RT_ERR_INVALID_ARG, "h_init must be >= 0");
  if (!(L->s_max > 0.0) || !std::isfinite(L->s_max)) FAIL(RT_ERR_INVALID_ARG, "s_max must be > 0");
  if (!(L->t_max >= 0.0) || !std::isfinite(L->t_max)) FAIL(RT_ERR_INVALID_ARG, "t_max must be >= 0");
  if (!(L->amp_min >= 0.0) || !std::isfinite(L->amp_min))
    FAIL(RT_ERR_INVALID_ARG, "amp_min must be >= 0");
  if (L->max_generations < 1) FAIL(RT_ERR_INVALID_ARG, "max_generations must be >= 1");
  if (L->max_generations > RT_MAX_GENERATIONS)
    FAIL(RT_ERR_UNSUPPORTED, "max_generations above %d", RT_MAX_GENERATIONS);
  if (L->model != RT_MODEL_PAPER && L->model != RT_MODEL_EXACT)
    FAIL(RT_ERR_INVALID_ARG, "unknown model %d", L->model);
  if (L->max_steps_per_ray < 1) FAIL(RT_ERR_INVALID_ARG, "max_steps_per_ray must be >= 1");
  if (L->max_steps_per_launch < 0)
    FAIL(RT_ERR_INVALID_ARG, "max_steps_per_launch must be >= 0 (0 = no limit)");
  if (L->resume != 0 && L->resume != 1) FAIL(RT_ERR_INVALID_ARG, "resume must be 0 or 1");
  return RT_OK;
}

rt_status check_surrogate_params(const rt_surrogate_params* sp) {
  if (!sp) FAIL(RT_ERR_INVALID_ARG, "null surrogate params");
  if (!(sp->verify_tol > 0.0) || !std::isfinite(sp->verify_tol))
    FAIL(RT_ERR_INVALID_ARG, "verify_tol must be > 0");
  if (!(sp->dseed > 0.0) || !(sp->dseed < 0.5)) FAIL(RT_ERR_INVALID_ARG, "need 0 < dseed < 0.5");
  if (sp->max_shots < 2 || sp->max_shots > 64) FAIL(RT_ERR_INVALID_ARG, "max_shots must be 2..64");
  if (!std::isfinite(sp->z0) || !std::isfinite(sp->dn) || std::isnan(sp->absent_logit) ||
      std::isnan(sp->multi_logit))
    FAIL(RT_ERR_INVALID_ARG, "non-finite profile features or NaN logit threshold");
  return RT_OK;
}

}  // namespace rt

extern "C" {

int32_t rt_abi_version(void) { return RT_ABI_VERSION; }

rt_status rt_validate(const rt_field* field, const rt_boundaries* boundaries,
                      const rt_sources* sources, const rt_directions* directions, double tol,
                      const rt_step_limits* limits) {
  return rt::validate(field, boundaries, sources, directions, tol, limits);
}

rt_status rt_workspace_bytes(const rt_field* field, int64_t capacity, size_t* bytes) {
  if (!field || !bytes) {
    rt::set_last_error("null argument");
    return RT_ERR_INVALID_ARG;
  }
  if (capacity < 0) {
    rt::set_last_error("negative capacity");
    return RT_ERR_INVALID_ARG;
  }
  size_t b = 4096;                                      // queue counters, padded
  b += ((size_t)capacity * 4 + 4095) / 4096 * 4096;     // overflow queue
  b += ((size_t)capacity * 4 + 4095) / 4096 * 4096;     // hand-out order of the primaries
  b += ((size_t)capacity * 4 + 4095) / 4096 * 4096;     // its per-chunk sorted order
  b += ((size_t)(capacity / 16384 + 1) * 8 + 4095) / 4096 * 4096;  // chunk keys
  if (field->n_regions > 0 && field->regions && rt::field_uses_grid(field)) {
    const rt_grid& g = field->grid;
    if (g.nx < 2 || g.ny < 2 || g.nz < 2) {
      rt::set_last_error("grid: dims must be >= 2");
      return RT_ERR_INVALID_ARG;
    }
    // float4 nodes in bricks of 2 x 2 x 2 (one 128-byte line each)
    b += (size_t)((g.nx + 1) / 2) * ((g.ny + 1) / 2) * ((g.nz + 1) / 2) * 128;
  }
  *bytes = b;
  return RT_OK;
}

rt_status rt_collect(const rt_stats* s, int64_t capacity) {
  rt::Range range("rt_collect");
  if (!s) {
    rt::set_last_error("null stats");
    return RT_ERR_INVALID_ARG;
  }
  if (s->sched_errors > 0) {
    rt::set_last_error("scheduler: %lld queue waits timed out", (long long)s->sched_errors);
    return RT_ERR_DEVICE;
  }
  if (s->invalid > 0) {
    rt::set_last_error("%lld input rays invalid (status RT_ST_INVALID)", (long long)s->invalid);
    return RT_ERR_INVALID_ARG;
  }
  if (s->needed > capacity) {
    rt::set_last_error("record capacity %lld < needed %lld", (long long)capacity,
                       (long long)s->needed);
    return RT_ERR_CAPACITY;
  }
  if (s->events_lost > 0) {
    rt::set_last_error("%lld of %lld event records did not fit; relaunch with ev_capacity >= %lld",
                       (long long)s->events_lost, (long long)s->events, (long long)s->events);
    return RT_ERR_CAPACITY;
  }
  if (s->interrupted) {
    rt::set_last_error("step budget reached; relaunch with resume = 1 to continue");
    return RT_INTERRUPTED;
  }
  return RT_OK;
}

rt_status rt_solve_validate(const rt_field* field, const rt_boundaries* bnd, double tol,
                            const rt_step_limits* L, const rt_solve_params* prm) {
  if (!field || !bnd || !L) {
    rt::set_last_error("null descriptor");
    return RT_ERR_INVALID_ARG;
  }
  // shots have no sources, directions, path limit, amplitude cut or
  // secondaries: check the rest as for a trace
  if (L->max_steps_per_launch != 0 || L->resume != 0) {
    rt::set_last_error("solves take no step budget per launch and no resume");
    return RT_ERR_INVALID_ARG;
  }
  rt_step_limits lim = *L;
  lim.s_max = 1.0;
  lim.amp_min = 0.0;
  lim.max_generations = 1;
  const rt_sources no_src = {nullptr, 0};
  const rt_directions no_dirs = {nullptr, nullptr, 0};
  rt_status st = rt::validate(field, bnd, &no_src, &no_dirs, tol, &lim);
  if (st != RT_OK) return st;
  if (rt::field_is_general(field)) {
    rt::set_last_error("solves support depth-stratified analytic fields only "
                       "(no grid, axis, or anomalies)");
    return RT_ERR_UNSUPPORTED;
  }
  if (L->t_max != 0.0) {
    rt::set_last_error("solves need t_max = 0 (shots end at the receiver plane)");
    return RT_ERR_INVALID_ARG;
  }
  if (bnd->has_box) {
    rt::set_last_error("solves need has_box = 0 (shots end at the receiver plane)");
    return RT_ERR_INVALID_ARG;
  }
  if (bnd->n_planes < 1 || bnd->planes[0].kind != RT_PLANE_FRESNEL) {
    rt::set_last_error("solves need planes[0] = the surface, of kind RT_PLANE_FRESNEL");
    return RT_ERR_INVALID_ARG;
  }
  for (int k = 0; k < bnd->n_planes; ++k)
    if (bnd->planes[k].shape != RT_SHAPE_PLANE) {
      rt::set_last_error("solves follow planar boundaries only (plane %d is curved)", k);
      return RT_ERR_UNSUPPORTED;
    }
  if (prm) {
    if (prm->n_scan < 2 || prm->n_scan > 4096 || prm->max_iter < 1 || prm->max_iter > 1000 ||
        prm->max_brackets < 1 || prm->max_brackets > 16) {
      rt::set_last_error("need 2 <= n_scan <= 4096, 1 <= max_iter <= 1000, "
                         "1 <= max_brackets <= 16");
      return RT_ERR_INVALID_ARG;
    }
    if (!(prm->slope_max >= 0.0) || !std::isfinite(prm->slope_max)) {
      rt::set_last_error("slope_max must be >= 0 (0 = off)");
      return RT_ERR_INVALID_ARG;
    }
    if (!(prm->miss_tol > 0.0) || !(prm->accept_tol >= prm->miss_tol) ||
        !std::isfinite(prm->accept_tol)) {
      rt::set_last_error("need 0 < miss_tol <= accept_tol < inf");
      return RT_ERR_INVALID_ARG;
    }
  }
  return RT_OK;
}

rt_status rt_solve_workspace_bytes(const rt_field* field, int64_t n_pairs,
                                   const rt_solve_params* prm, size_t* bytes) {
  if (!field || !bytes || (n_pairs > 0 && !prm)) {
    rt::set_last_error("null argument");
    return RT_ERR_INVALID_ARG;
  }
  if (n_pairs < 0) {
    rt::set_last_error("negative pair count");
    return RT_ERR_INVALID_ARG;
  }
  size_t b = 4096;  // counters, padded
  if (n_pairs > 0) {
    const size_t pf = 2 * (size_t)n_pairs;
    b += (pf * (size_t)prm->n_scan * 8 + 4095) / 4096 * 4096;       // scan misses
    b += (pf * (size_t)prm->max_brackets * 80 + 4095) / 4096 * 4096; // bracket results
  }
  if (field->n_regions > 0 && field->regions && rt::field_uses_grid(field)) {
    const rt_grid& g = field->grid;
    if (g.nx < 2 || g.ny < 2 || g.nz < 2) {
      rt::set_last_error("grid: dims must be >= 2");
      return RT_ERR_INVALID_ARG;
    }
    b += (size_t)g.nx * g.ny * g.nz * 16;
  }
  *bytes = b;
  return RT_OK;
}

const char* rt_last_error(void) { return rt::g_err; }

}  // extern "C"
