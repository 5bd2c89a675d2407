// Surrogate-seeded emitter -> receiver solves, gfx950 (MI355X).
//
// The network's predicted launch angles seed a short secant per (pair,
// family) entry whose last shot verifies the solution; pairs with an entry
// that could not be verified are solved again by the tracer's full solve.
// Everything runs on the device: the fallback pairs are compacted into a
// list whose length only the device knows, and the solve kernels read that
// length themselves.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "radiotrace_mlp.h"
#include "radiotrace_solve.h"
#include "rt_params.hpp"
#include "rt_solve_internal.hpp"

namespace rt {
namespace surr {

constexpr double kPi = 3.14159265358979323846;
constexpr double kC0 = 299792458.0;
constexpr int kStats = (int)(sizeof(rt_solve_stats) / 8);

__global__ void features_kernel(const double* __restrict__ zs, const double* __restrict__ zr,
                                const double* __restrict__ dist, int64_t n, double z0, double dn,
                                float* __restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float* o = x + i * RT_MLP_IN;
  o[0] = (float)((zs[i] - 1025.0) / 975.0);
  o[1] = (float)((zr[i] - 100.0) / 100.0);
  o[2] = (float)((dist[i] - 1505.0) / 1495.0);
  o[3] = (float)((z0 - 80.0) / 40.0);
  o[4] = (float)((dn - 0.425) / 0.075);
}

__global__ void targets_kernel(rt_solve_outputs S, int64_t n, float* __restrict__ t,
                               float* __restrict__ m) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int f = 0; f < 2; ++f) {
    const int64_t e = 2 * i + f;
    const bool ok = S.found[e] != 0;
    const double A = sqrt(0.5 * (S.as_re[e] * S.as_re[e] + S.as_im[e] * S.as_im[e] +
                                 S.ap_re[e] * S.ap_re[e] + S.ap_im[e] * S.ap_im[e]));
    float* o = t + i * RT_MLP_TARGETS + 4 * f;
    o[0] = ok ? (float)(S.theta[e] / (0.5 * kPi) - 1.0) : 0.0f;
    o[1] = ok ? (float)(kC0 * S.t[e] / 3000.0 - 1.0) : 0.0f;
    o[2] = ok ? (float)(S.s[e] / 3000.0 - 1.0) : 0.0f;
    o[3] = ok ? (float)(2.0 * A - 1.0) : 0.0f;
    m[i * RT_MLP_LABELS + f] = ok ? 1.0f : 0.0f;
    m[i * RT_MLP_LABELS + 2 + f] = S.roots[e] >= 2 ? 1.0f : 0.0f;
  }
}

__global__ void reset_kernel(int64_t* count) {
  if (threadIdx.x == 0) *count = 0;
}

// Network outputs -> seed angle and decision per entry: an entry whose
// existence logit is at or below absent_logit, or whose several-roots logit
// is above multi_logit, is not seeded (the tracer solves it).
__global__ void decode_kernel(const float* __restrict__ y, int64_t n, float absent_logit,
                              float multi_logit, double* __restrict__ seed,
                              int32_t* __restrict__ seed_try, int32_t* __restrict__ verify,
                              int32_t* __restrict__ path) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 2 * n) return;
  const int64_t i = e >> 1;
  const int f = (int)(e & 1);
  const double th = 0.5 * kPi * (1.0 + (double)y[i * RT_MLP_OUT + 4 * f]);
  seed[e] = fmin(fmax(th, 1e-6), kPi - 1e-6);
  const bool tried = y[i * RT_MLP_OUT + 8 + f] > absent_logit &&
                     !(y[i * RT_MLP_OUT + 10 + f] > multi_logit);
  seed_try[e] = tried ? 1 : 0;
  verify[e] = -1;
  path[e] = RT_PATH_SURROGATE;
}

// Pairs with an entry that is not verified (not seeded, or its seed failed)
// -> fallback list, with the families to solve (bit f = family f).
__global__ void flag_kernel(const int32_t* __restrict__ verify, int64_t n,
                            int64_t* __restrict__ count, int64_t* __restrict__ idx,
                            uint8_t* __restrict__ fam) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint8_t m = (uint8_t)((verify[2 * i] != 1 ? 1 : 0) | (verify[2 * i + 1] != 1 ? 2 : 0));
  if (m) {
    const unsigned long long k = atomicAdd(reinterpret_cast<unsigned long long*>(count), 1ull);
    idx[k] = i;
    fam[k] = m;
  }
}

__global__ void gather_kernel(const int64_t* __restrict__ idx, const int64_t* __restrict__ count,
                              int64_t n, const double* __restrict__ zs,
                              const double* __restrict__ zr, const double* __restrict__ dist,
                              double* __restrict__ czs, double* __restrict__ czr,
                              double* __restrict__ cdist) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || i >= *count) return;
  const int64_t p = idx[i];
  czs[i] = zs[p];
  czr[i] = zr[p];
  cdist[i] = dist[p];
}

// The tracer's results of the fallback entries into place.
__global__ void scatter_kernel(const int64_t* __restrict__ idx, const int64_t* __restrict__ count,
                               const uint8_t* __restrict__ fam, int64_t n, rt_solve_outputs C,
                               rt_solve_outputs O, int32_t* __restrict__ path) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || i >= *count) return;
  const int64_t p = idx[i];
  for (int f = 0; f < 2; ++f) {
    if (!((fam[i] >> f) & 1)) continue;
    const int64_t a = 2 * i + f, e = 2 * p + f;
    O.found[e] = C.found[a];
    O.shots[e] = C.shots[a];
    O.roots[e] = C.roots[a];
    O.theta[e] = C.theta[a];
    O.miss[e] = C.miss[a];
    O.t[e] = C.t[a];
    O.s[e] = C.s[a];
    O.as_re[e] = C.as_re[a];
    O.as_im[e] = C.as_im[a];
    O.ap_re[e] = C.ap_re[a];
    O.ap_im[e] = C.ap_im[a];
    path[e] = RT_PATH_TRACER;
  }
}

// out->stats += fallback stats; *fallback_pairs = count.
__global__ void finish_kernel(const int64_t* __restrict__ count,
                              const int64_t* __restrict__ fb_stats, int64_t* __restrict__ stats,
                              int64_t* __restrict__ fallback_pairs) {
  const int i = threadIdx.x;
  if (i < kStats) stats[i] += fb_stats[i];
  if (i == 0) *fallback_pairs = *count;
}

// Workspace layout of raytrace_solve_surrogate for n pairs.
struct Layout {
  int64_t* count;
  int64_t* fb_stats;
  void* tickets;  // seeded phase counters (4 KiB region)
  void* mlp_ws;
  size_t mlp_bytes;
  float *x, *y;
  double* seed;
  int32_t *seed_try, *verify;
  int64_t* idx;
  uint8_t* fam;
  double *czs, *czr, *cdist;
  int32_t *c_found, *c_shots, *c_roots;
  double* c_f64[8];
  void* solve_ws;
  size_t solve_bytes;
  size_t bytes;
};

size_t up(size_t x) { return (x + 4095) / 4096 * 4096; }

rt_status layout(const rt_field* field, int64_t n, const rt_solve_params* fb, char* base,
                 Layout& L) {
  memset(&L, 0, sizeof L);
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = base ? base + off : nullptr;
    off += up(bytes);
    return p;
  };
  char* head = take(4096);  // seeded tickets | count | fallback stats
  if (base) {
    L.tickets = head;
    L.count = reinterpret_cast<int64_t*>(head + 2048);
    L.fb_stats = reinterpret_cast<int64_t*>(head + 2560);
  }
  const int64_t nb = std::max<int64_t>(n, 1);
  if (rt_mlp_workspace_bytes(nb, 0, &L.mlp_bytes) != RT_OK) return RT_ERR_INVALID_ARG;
  L.mlp_ws = take(L.mlp_bytes);
  L.x = reinterpret_cast<float*>(take((size_t)nb * RT_MLP_IN * 4));
  L.y = reinterpret_cast<float*>(take((size_t)nb * RT_MLP_OUT * 4));
  L.seed = reinterpret_cast<double*>(take((size_t)nb * 16));
  L.seed_try = reinterpret_cast<int32_t*>(take((size_t)nb * 8));
  L.verify = reinterpret_cast<int32_t*>(take((size_t)nb * 8));
  L.idx = reinterpret_cast<int64_t*>(take((size_t)nb * 8));
  L.fam = reinterpret_cast<uint8_t*>(take((size_t)nb));
  L.czs = reinterpret_cast<double*>(take((size_t)nb * 8));
  L.czr = reinterpret_cast<double*>(take((size_t)nb * 8));
  L.cdist = reinterpret_cast<double*>(take((size_t)nb * 8));
  L.c_found = reinterpret_cast<int32_t*>(take((size_t)nb * 8));
  L.c_shots = reinterpret_cast<int32_t*>(take((size_t)nb * 8));
  L.c_roots = reinterpret_cast<int32_t*>(take((size_t)nb * 8));
  for (int k = 0; k < 8; ++k) L.c_f64[k] = reinterpret_cast<double*>(take((size_t)nb * 16));
  rt_status st = rt_solve_workspace_bytes(field, nb, fb, &L.solve_bytes);
  if (st != RT_OK) return st;
  L.solve_ws = take(L.solve_bytes);
  L.bytes = off;
  return RT_OK;
}

}  // namespace surr
}  // namespace rt

#define HIP_TRY(expr)                                                         \
  do {                                                                        \
    hipError_t e_ = (expr);                                                   \
    if (e_ != hipSuccess) {                                                   \
      rt::set_last_error("%s: %s", #expr, hipGetErrorString(e_));             \
      return RT_ERR_DEVICE;                                                   \
    }                                                                         \
  } while (0)

extern "C" rt_status rt_surrogate_features(const rt_pairs* pairs, double z0, double dn, float* x,
                                           void* stream) {
  if (!pairs || pairs->n < 0 || (pairs->n > 0 && (!pairs->zs || !pairs->zr || !pairs->dist ||
                                                  !x))) {
    rt::set_last_error("null or invalid pairs or features array");
    return RT_ERR_INVALID_ARG;
  }
  if (pairs->n == 0) return RT_OK;
  hipLaunchKernelGGL(rt::surr::features_kernel, dim3((unsigned)((pairs->n + 255) / 256)),
                     dim3(256), 0, static_cast<hipStream_t>(stream), pairs->zs, pairs->zr,
                     pairs->dist, pairs->n, z0, dn, x);
  HIP_TRY(hipGetLastError());
  return RT_OK;
}

extern "C" rt_status rt_surrogate_targets(const rt_solve_outputs* solved, int64_t n,
                                          float* targets, float* mask, void* stream) {
  if (!solved || n < 0 || (n > 0 && (!targets || !mask || !solved->found || !solved->roots ||
                                     !solved->theta ||
                                     !solved->t || !solved->s || !solved->as_re ||
                                     !solved->as_im || !solved->ap_re || !solved->ap_im))) {
    rt::set_last_error("null or invalid solve outputs, targets or labels");
    return RT_ERR_INVALID_ARG;
  }
  if (n == 0) return RT_OK;
  hipLaunchKernelGGL(rt::surr::targets_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), *solved, n, targets, mask);
  HIP_TRY(hipGetLastError());
  return RT_OK;
}

extern "C" rt_status rt_surrogate_workspace_bytes(const rt_field* field, int64_t n_pairs,
                                                  const rt_solve_params* fb, size_t* bytes) {
  if (!field || !fb || !bytes || n_pairs < 0 || n_pairs > ((int64_t)1 << 24)) {
    rt::set_last_error("null argument or pair count outside 0..2^24");
    return RT_ERR_INVALID_ARG;
  }
  rt::surr::Layout L;
  rt_status st = rt::surr::layout(field, n_pairs, fb, nullptr, L);
  if (st != RT_OK) return st;
  *bytes = L.bytes;
  return RT_OK;
}

extern "C" rt_status raytrace_solve_surrogate(const rt_field* field, const rt_boundaries* bnd,
                                              double tol, const rt_step_limits* lim,
                                              const rt_pairs* pairs,
                                              const rt_solve_params* fb,
                                              const rt_surrogate_params* sp,
                                              const float* mlp_params, rt_solve_outputs* out,
                                              int32_t* path, int64_t* fallback_pairs,
                                              void* workspace, size_t workspace_bytes,
                                              void* stream, const rt_tuning* tuning) {
  using namespace rt;
  using namespace rt::surr;
  rt_status st = rt_solve_validate(field, bnd, tol, lim, fb);
  if (st != RT_OK) return st;
  if ((st = check_surrogate_params(sp)) != RT_OK) return st;
  if (!fb || !pairs || !out || !out->stats || !workspace || !mlp_params || !path ||
      !fallback_pairs) {
    set_last_error("null fallback params, pairs, outputs, network, path or workspace");
    return RT_ERR_INVALID_ARG;
  }
  if (pairs->n < 0 || pairs->n > ((int64_t)1 << 24)) {
    set_last_error("pair count must be 0..2^24");
    return RT_ERR_INVALID_ARG;
  }
  if (pairs->n > 0 && (!pairs->zs || !pairs->zr || !pairs->dist || !out->found || !out->shots ||
                       !out->roots ||
                       !out->theta || !out->miss || !out->t || !out->s || !out->as_re ||
                       !out->as_im || !out->ap_re || !out->ap_im)) {
    set_last_error("null pair or output array");
    return RT_ERR_INVALID_ARG;
  }
  Layout L;
  if ((st = layout(field, pairs->n, fb, nullptr, L)) != RT_OK) return st;
  if (workspace_bytes < L.bytes) {
    set_last_error("workspace of %zu bytes < %zu needed", workspace_bytes, L.bytes);
    return RT_ERR_INVALID_ARG;
  }
  layout(field, pairs->n, fb, static_cast<char*>(workspace), L);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t n = pairs->n;
  const unsigned g1 = (unsigned)((std::max<int64_t>(n, 1) + 255) / 256);
  const unsigned g2 = (unsigned)((std::max<int64_t>(2 * n, 1) + 255) / 256);

  Range range("raytrace_solve_surrogate");
  hipLaunchKernelGGL(reset_kernel, dim3(1), dim3(64), 0, s, L.count);
  HIP_TRY(hipGetLastError());
  // 1. network: features -> outputs
  if (n > 0) {
    hipLaunchKernelGGL(features_kernel, dim3(g1), dim3(256), 0, s, pairs->zs, pairs->zr,
                       pairs->dist, n, sp->z0, sp->dn, L.x);
    HIP_TRY(hipGetLastError());
    if ((st = rt_mlp_pack(mlp_params, L.mlp_ws, L.mlp_bytes, stream)) != RT_OK) return st;
    if ((st = rt_mlp_forward(mlp_params, L.x, n, L.y, L.mlp_ws, L.mlp_bytes, stream)) != RT_OK)
      return st;
    hipLaunchKernelGGL(decode_kernel, dim3(g2), dim3(256), 0, s, L.y, n, sp->absent_logit,
                       sp->multi_logit, L.seed, L.seed_try, L.verify, path);
    HIP_TRY(hipGetLastError());
  }
  // 2. seeded secant of the tried entries (stats into out->stats)
  if ((st = seeded_enqueue(field, bnd, tol, lim, pairs, L.seed, L.seed_try, sp, out, L.verify,
                           L.tickets, stream, tuning)) != RT_OK)
    return st;
  // 3. fallback pairs, compacted on the device, through the full solve
  rt_solve_outputs C;
  memset(&C, 0, sizeof C);
  C.found = L.c_found;
  C.shots = L.c_shots;
  C.roots = L.c_roots;
  double** f[] = {&C.theta, &C.miss, &C.t, &C.s, &C.as_re, &C.as_im, &C.ap_re, &C.ap_im};
  for (int k = 0; k < 8; ++k) *f[k] = L.c_f64[k];
  C.stats = reinterpret_cast<rt_solve_stats*>(L.fb_stats);
  if (n > 0) {
    hipLaunchKernelGGL(flag_kernel, dim3(g1), dim3(256), 0, s, L.verify, n, L.count, L.idx,
                       L.fam);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(gather_kernel, dim3(g1), dim3(256), 0, s, L.idx, L.count, n, pairs->zs,
                       pairs->zr, pairs->dist, L.czs, L.czr, L.cdist);
    HIP_TRY(hipGetLastError());
  }
  const rt_pairs cp = {L.czs, L.czr, L.cdist, n};
  // the caller's launch tuning serves the tracer's solve too (block size,
  // refill threshold, scan interleave, fused launch); its events are not
  // recorded by this call
  rt_tuning ft;
  memset(&ft, 0, sizeof ft);
  if (tuning) {
    ft = *tuning;
    ft.ev_trace_begin = ft.ev_trace_end = nullptr;
  }
  if ((st = solve_enqueue(field, bnd, tol, lim, &cp, n, L.count, L.fam, fb, &C, L.solve_ws,
                          stream, tuning ? &ft : nullptr)) != RT_OK)
    return st;
  if (n > 0) {
    hipLaunchKernelGGL(scatter_kernel, dim3(g1), dim3(256), 0, s, L.idx, L.count, L.fam, n, C,
                       *out, path);
    HIP_TRY(hipGetLastError());
  }
  hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(64), 0, s, L.count, L.fb_stats,
                     reinterpret_cast<int64_t*>(out->stats), fallback_pairs);
  HIP_TRY(hipGetLastError());
  return RT_OK;
}
