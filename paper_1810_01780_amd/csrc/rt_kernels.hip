// Eikonal ray tracing kernels for gfx950 (MI355X), FP64.
//
// Method: RadioPropa (arXiv:1810.01780) section 2 -- the ray equation (eq. 2,
// locally paraxial; or eq. 1, full eikonal) integrated by the Cash-Karp
// embedded Runge-Kutta 4(5) pair with adaptive steps, and planar boundaries
// handled apart from the propagation: the ray reflects and a refracted
// secondary is cast from the crossing point, with Fresnel amplitudes.
//
// Execution model: one ray per lane, state in registers.  A persistent grid
// of waves pulls rays from a queue whose slots are the caller's output
// records; secondaries are appended to the same queue.  Every loop iteration
// runs exactly one Cash-Karp trial step in every busy lane -- a normal step,
// or one iterate of the crossing search -- so the expensive arithmetic never
// diverges; only the cheap bookkeeping after the trial does.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "rt_params.hpp"

namespace rt {

constexpr double kInvC0 = 1.0 / 299792458.0;  // 1 / speed of light (m/s)

// Cash-Karp (1990) tableau: stage matrix, fifth-order weights, and the
// difference of the fifth- and fourth-order weights.
__device__ constexpr double ck_a(int i, int j) {
  return i == 1 ? (1.0 / 5.0)
       : i == 2 ? (j == 0 ? 3.0 / 40.0 : 9.0 / 40.0)
       : i == 3 ? (j == 0 ? 3.0 / 10.0 : j == 1 ? -9.0 / 10.0 : 6.0 / 5.0)
       : i == 4 ? (j == 0 ? -11.0 / 54.0 : j == 1 ? 5.0 / 2.0
                   : j == 2 ? -70.0 / 27.0 : 35.0 / 27.0)
       : (j == 0 ? 1631.0 / 55296.0 : j == 1 ? 175.0 / 512.0
          : j == 2 ? 575.0 / 13824.0 : j == 3 ? 44275.0 / 110592.0
          : 253.0 / 4096.0);
}
constexpr double kB1 = 37.0 / 378.0, kB3 = 250.0 / 621.0,
                 kB4 = 125.0 / 594.0, kB6 = 512.0 / 1771.0;
constexpr double kE1 = -277.0 / 64512.0, kE3 = 6925.0 / 370944.0,
                 kE4 = -6925.0 / 202752.0, kE5 = -277.0 / 14336.0,
                 kE6 = 277.0 / 7084.0;

// y0 + h * sum_j a[S][j] k[j]
template <int S>
__device__ __forceinline__ double stage_in(double y0, double h, const double (&k)[6]) {
  double acc = ck_a(S, 0) * k[0];
#pragma unroll
  for (int j = 1; j < S; ++j) acc = fma(ck_a(S, j), k[j], acc);
  return fma(h, acc, y0);
}
__device__ __forceinline__ double b_sum(const double (&k)[6]) {
  return fma(kB6, k[5], fma(kB4, k[3], fma(kB3, k[2], kB1 * k[0])));
}
__device__ __forceinline__ double e_sum(const double (&k)[6]) {
  return fma(kE6, k[5], fma(kE5, k[4], fma(kE4, k[3], fma(kE3, k[2], kE1 * k[0]))));
}

// ---------------------------------------------------------------------------
// FP64 helpers: hardware estimates refined by Newton steps to within an ulp or
// two of the correctly rounded result.

// 1/x for finite non-zero x.
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// 1/sqrt(x) for finite x > 0.
__device__ __forceinline__ double rsqrt_nr(double x) {
  double r = __builtin_amdgcn_rsq(x);
  const double hx = 0.5 * x;
  double e = fma(-hx * r, r, 0.5);
  r = fma(r, e, r);
  e = fma(-hx * r, r, 0.5);
  return fma(r, e, r);
}

// x^(-1/K) for x > 0: FP32 log2/exp2 seed, then two Newton steps on
// y^-K = x, i.e. y <- y ((K + 1) - x y^K) / K.  Values beyond the FP32 range
// give 0 (the callers clamp the resulting step).
template <int K>
__device__ __forceinline__ double pow_neg_inv(double x) {
  const float l = __builtin_amdgcn_logf((float)x);
  double y = (double)__builtin_amdgcn_exp2f(l * (-1.0f / K));
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const double y2 = y * y;
    const double yk = K == 4 ? y2 * y2 : y2 * y2 * y;
    y = y * fma(-x, yk, (double)(K + 1)) * (1.0 / K);
  }
  return y;
}

// e^x for |x| <= 0.25: Taylor polynomial to degree 11 (truncation below
// 2^-52 relative), Horner form.
__device__ __forceinline__ double exp_small(double x) {
  double p = 1.0 / 39916800.0;
  p = fma(p, x, 1.0 / 3628800.0);
  p = fma(p, x, 1.0 / 362880.0);
  p = fma(p, x, 1.0 / 40320.0);
  p = fma(p, x, 1.0 / 5040.0);
  p = fma(p, x, 1.0 / 720.0);
  p = fma(p, x, 1.0 / 120.0);
  p = fma(p, x, 1.0 / 24.0);
  p = fma(p, x, 1.0 / 6.0);
  p = fma(p, x, 0.5);
  p = fma(p, x, 1.0);
  return fma(p, x, 1.0);
}

// Medium of one ray, kept in registers: n(z) = a + b z - dn exp(-z/z0).
struct Medium {
  double a, b, dn, inv_z0, dn_inv_z0;
  int use_grid;
};

// Media and boundary tables indexed per lane (by a ray's medium or by the
// boundary it is searching): copied into LDS at kernel start.  Loops over all
// boundaries use the uniform copy in the kernel arguments instead.
__shared__ KRegion s_reg[RT_MAX_REGIONS];
__shared__ KBnd s_bnd[kMaxBnd];

__device__ __forceinline__ Medium medium_of(const KParams& P, int r) {
  (void)P;
  const KRegion& R = s_reg[r];
  return Medium{R.a, R.b, R.dn, R.inv_z0, R.dn_inv_z0, R.use_grid};
}

__device__ __forceinline__ void strat_field(const Medium& M, double z, double& n, double& gz) {
  double e = 0.0;
  if (M.dn != 0.0) e = exp(-z * M.inv_z0);
  n = fma(M.b, z, M.a) - M.dn * e;
  gz = fma(M.dn_inv_z0, e, M.b);
}

// Same at a stage point z = z0 + dz of a step starting at z0, where
// E0 = exp(-z0/z0_medium): exp(-z/z0) = E0 exp(-dz/z0), and the second factor
// is a short polynomial because a step moves at most a fraction of z0.
__device__ __forceinline__ void strat_field_rel(const Medium& M, double z0, double dz, double E0,
                                                double& n, double& gz) {
  const double z = z0 + dz;
  double e = 0.0;
  if (M.dn != 0.0) {
    const double x = -dz * M.inv_z0;
    e = fabs(x) <= 0.25 ? E0 * exp_small(x) : exp(-z * M.inv_z0);
  }
  n = fma(M.b, z, M.a) - M.dn * e;
  gz = fma(M.dn_inv_z0, e, M.b);
}

// Trilinear n and gradient from float4 nodes (n, Dx, Dy, Dz); positions
// outside the grid are clamped onto it; grad n = D / (2 spacing).
__device__ __forceinline__ void grid_field(const KParams& P, double x, double y, double z,
                                           double& n, double g[3]) {
  const float4* __restrict__ nodes = static_cast<const float4*>(P.nodes);
  double f[3] = {(x - P.gorg[0]) * P.ginv[0], (y - P.gorg[1]) * P.ginv[1],
                 (z - P.gorg[2]) * P.ginv[2]};
  int i0[3];
  double t[3];
  const int dims[3] = {P.gnx, P.gny, P.gnz};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double v = fmin(fmax(f[a], 0.0), P.gmax[a]);
    int i = (int)floor(v);
    i = min(i, dims[a] - 2);
    i0[a] = i;
    t[a] = v - (double)i;
  }
  const size_t sx = 1, sy = (size_t)P.gnx, sz = (size_t)P.gnx * P.gny;
  const size_t base = (size_t)i0[2] * sz + (size_t)i0[1] * sy + (size_t)i0[0];
  float4 c[8];
#pragma unroll
  for (int q = 0; q < 8; ++q)
    c[q] = nodes[base + ((q & 1) ? sx : 0) + ((q & 2) ? sy : 0) + ((q & 4) ? sz : 0)];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    double w = ((q & 1) ? t[0] : 1.0 - t[0]) * ((q & 2) ? t[1] : 1.0 - t[1]) *
               ((q & 4) ? t[2] : 1.0 - t[2]);
    acc[0] = fma(w, (double)c[q].x, acc[0]);
    acc[1] = fma(w, (double)c[q].y, acc[1]);
    acc[2] = fma(w, (double)c[q].z, acc[2]);
    acc[3] = fma(w, (double)c[q].w, acc[3]);
  }
  n = acc[0];
  g[0] = acc[1] * P.ghalf[0];
  g[1] = acc[2] * P.ghalf[1];
  g[2] = acc[3] * P.ghalf[2];
}

// ---------------------------------------------------------------------------
// One Cash-Karp trial step of length h from state y = (r, w, tau):
// y5 = fifth-order result, err = max(|dr|/h, |dw|/|w0|) / tol.
// Paper model (eq. 2): w = unit velocity, r' = w, w' = grad n / n.
// Exact model (eq. 1): w = p, r' = p / |p|, p' = grad n.   tau' = n / c0.
//
// Stratified media (grad n along z): in the paper model w_x, w_y are constant
// within a step and only z, w_z, tau need stage values.
template <int S>
__device__ __forceinline__ double stage_inc(double h, const double (&k)[6]) {
  double acc = ck_a(S, 0) * k[0];
#pragma unroll
  for (int j = 1; j < S; ++j) acc = fma(ck_a(S, j), k[j], acc);
  return h * acc;
}

template <int MODEL>
__device__ __forceinline__ void trial_strat(const Medium& M, const double y[7], double h,
                                            double inv_tol, double y5[7], double& err) {
  const double E0 = M.dn != 0.0 ? exp(-y[2] * M.inv_z0) : 0.0;
  if constexpr (MODEL == RT_MODEL_PAPER) {
    // w = unit velocity, renormalised after every accepted step (|w| = 1)
    double kz[6], kw[6];
    double tsum = 0.0;  // sum_j b_j n_j / c0
#pragma unroll
    for (int st = 0; st < 6; ++st) {
      double dz = 0.0, ws = y[5];
      if (st == 1) { dz = stage_inc<1>(h, kz); ws = stage_in<1>(y[5], h, kw); }
      if (st == 2) { dz = stage_inc<2>(h, kz); ws = stage_in<2>(y[5], h, kw); }
      if (st == 3) { dz = stage_inc<3>(h, kz); ws = stage_in<3>(y[5], h, kw); }
      if (st == 4) { dz = stage_inc<4>(h, kz); ws = stage_in<4>(y[5], h, kw); }
      if (st == 5) { dz = stage_inc<5>(h, kz); ws = stage_in<5>(y[5], h, kw); }
      double n, gz;
      strat_field_rel(M, y[2], dz, E0, n, gz);
      kz[st] = ws;
      kw[st] = gz * rcp_nr(n);
      if (st == 0) tsum = kB1 * n;
      if (st == 2) tsum = fma(kB3, n, tsum);
      if (st == 3) tsum = fma(kB4, n, tsum);
      if (st == 5) tsum = fma(kB6, n, tsum);
    }
    y5[0] = fma(h, y[3], y[0]);
    y5[1] = fma(h, y[4], y[1]);
    y5[2] = fma(h, b_sum(kz), y[2]);
    y5[3] = y[3];
    y5[4] = y[4];
    y5[5] = fma(h, b_sum(kw), y[5]);
    y5[6] = fma(h * kInvC0, tsum, y[6]);
    // max(|dr|/h, |dw|/|w0|) / tol with |w0| = 1
    err = fmax(fabs(e_sum(kz)), fabs(h * e_sum(kw))) * inv_tol;
  } else {
    // w = p = n dr/ds; p_x, p_y are constant in a stratified medium
    const double px = y[3], py = y[4];
    const double pxy2 = fma(px, px, py * py);
    double kx[6], ky[6], kz[6], kp[6], kt[6];
#pragma unroll
    for (int st = 0; st < 6; ++st) {
      double dz = 0.0, ps = y[5];
      if (st == 1) { dz = stage_inc<1>(h, kz); ps = stage_in<1>(y[5], h, kp); }
      if (st == 2) { dz = stage_inc<2>(h, kz); ps = stage_in<2>(y[5], h, kp); }
      if (st == 3) { dz = stage_inc<3>(h, kz); ps = stage_in<3>(y[5], h, kp); }
      if (st == 4) { dz = stage_inc<4>(h, kz); ps = stage_in<4>(y[5], h, kp); }
      if (st == 5) { dz = stage_inc<5>(h, kz); ps = stage_in<5>(y[5], h, kp); }
      double n, gz;
      strat_field_rel(M, y[2], dz, E0, n, gz);
      const double ip = rsqrt_nr(fma(ps, ps, pxy2));
      kx[st] = px * ip;
      ky[st] = py * ip;
      kz[st] = ps * ip;
      kp[st] = gz;
      kt[st] = n * kInvC0;
    }
    y5[0] = fma(h, b_sum(kx), y[0]);
    y5[1] = fma(h, b_sum(ky), y[1]);
    y5[2] = fma(h, b_sum(kz), y[2]);
    y5[3] = px;
    y5[4] = py;
    y5[5] = fma(h, b_sum(kp), y[5]);
    y5[6] = fma(h, b_sum(kt), y[6]);
    const double ex = e_sum(kx), ey = e_sum(ky), ez = e_sum(kz);
    const double dr_h = sqrt(fma(ex, ex, fma(ey, ey, ez * ez)));  // |dr| / h
    const double dp = h * e_sum(kp);
    err = fmax(dr_h, fabs(dp) * rsqrt_nr(fma(y[5], y[5], pxy2))) * inv_tol;
  }
}

// General 3-D gradient (gridded media, or analytic media inside the grid
// kernel).
template <int MODEL>
__device__ __forceinline__ void field3(const KParams& P, const Medium& M, double x, double y,
                                       double z, double& n, double g[3]) {
  if (M.use_grid) {
    grid_field(P, x, y, z, n, g);
  } else {
    double gz;
    strat_field(M, z, n, gz);
    g[0] = 0.0;
    g[1] = 0.0;
    g[2] = gz;
  }
}

template <int S>
__device__ __forceinline__ void stage_vec(const double y[7], double h, const double (&k)[6][6],
                                          double ys[6]) {
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    double kc[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) kc[j] = k[c][j];
    ys[c] = stage_in<S>(y[c], h, kc);
  }
}

template <int MODEL>
__device__ __forceinline__ void trial_3d(const KParams& P, const Medium& M, const double y[7],
                                         double h, double inv_tol, double y5[7], double& err) {
  double k[6][6];  // [component][stage] for r (0..2) and w (3..5)
  double kt[6];
#pragma unroll
  for (int st = 0; st < 6; ++st) {
    double ys[6];
    if (st == 0) {
#pragma unroll
      for (int c = 0; c < 6; ++c) ys[c] = y[c];
    }
    if (st == 1) stage_vec<1>(y, h, k, ys);
    if (st == 2) stage_vec<2>(y, h, k, ys);
    if (st == 3) stage_vec<3>(y, h, k, ys);
    if (st == 4) stage_vec<4>(y, h, k, ys);
    if (st == 5) stage_vec<5>(y, h, k, ys);
    double n, g[3];
    field3<MODEL>(P, M, ys[0], ys[1], ys[2], n, g);
    if constexpr (MODEL == RT_MODEL_PAPER) {
      const double in = rcp_nr(n);
      k[0][st] = ys[3];
      k[1][st] = ys[4];
      k[2][st] = ys[5];
      k[3][st] = g[0] * in;
      k[4][st] = g[1] * in;
      k[5][st] = g[2] * in;
    } else {
      const double ip = rsqrt_nr(fma(ys[3], ys[3], fma(ys[4], ys[4], ys[5] * ys[5])));
      k[0][st] = ys[3] * ip;
      k[1][st] = ys[4] * ip;
      k[2][st] = ys[5] * ip;
      k[3][st] = g[0];
      k[4][st] = g[1];
      k[5][st] = g[2];
    }
    kt[st] = n * kInvC0;
  }
  double d[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    double kc[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) kc[j] = k[c][j];
    y5[c] = fma(h, b_sum(kc), y[c]);
    d[c] = e_sum(kc);  // error vector / h
  }
  y5[6] = fma(h, b_sum(kt), y[6]);
  // max(|dr|/h, |dw|/|w0|) / tol
  const double dr_h = sqrt(fma(d[0], d[0], fma(d[1], d[1], d[2] * d[2])));
  const double dw_h = sqrt(fma(d[3], d[3], fma(d[4], d[4], d[5] * d[5])));
  const double iw0 = rsqrt_nr(fma(y[3], y[3], fma(y[4], y[4], y[5] * y[5])));
  err = fmax(dr_h, h * dw_h * iw0) * inv_tol;
}

// ---------------------------------------------------------------------------
// Step-size controller (standard embedded-RK control): safety 0.9, growth
// at most 5 (exactly 5 below err = (0.9/5)^5), shrink at most 10, exponents
// -1/5 after an accepted and -1/4 after a rejected trial, clamp to
// [h_min, h_max].
constexpr double kSafety = 0.9, kGrowMax = 5.0, kShrinkMin = 0.1;
constexpr double kErrCon = 1.889568e-4;
// Crossing search (Illinois false position) limits.
constexpr double kLocGTol = 1e-10, kLocWRel = 1e-14;
constexpr int kLocMaxIt = 60, kLocMaxPass = 8, kMaxEvents = 255;

__device__ __forceinline__ double clamp_h(const KParams& P, double h) {
  return fmin(fmax(h, P.h_min), P.h_max);
}

// Boundary function with the ray's side sign applied: > 0 before crossing.
__device__ __forceinline__ double bnd_G(const KParams& P, const KBnd& B, int k, uint32_t side,
                                        const double y[7]) {
  if (B.kind == B_TIME) return (P.t_max - y[6]) * 299792458.0;
  double g = fma(y[2], B.nrm[2], fma(y[1], B.nrm[1], y[0] * B.nrm[0])) - B.d;
  return ((side >> k) & 1u) ? g : -g;
}

// Earliest (by linear estimate) boundary crossed at the end of a step of
// length len from y0 to y1, skipping boundary 'skip'; -1 if none.
__device__ __forceinline__ int pick_crossing(const KParams& P, uint32_t side, const double y0[7],
                                             const double y1[7], double len, int skip,
                                             double& G0o, double& G1o) {
  int best = -1;
  double best_sig = 0.0;
  for (int k = 0; k < P.n_bnd; ++k) {
    if (k == skip) continue;
    double G1 = bnd_G(P, P.bnd[k], k, side, y1);
    if (!(G1 <= 0.0)) continue;
    double G0 = bnd_G(P, P.bnd[k], k, side, y0);
    double sig = G0 <= 0.0 ? 0.0 : len * G0 / (G0 - G1);
    if (best < 0 || sig < best_sig) {
      best = k;
      best_sig = sig;
      G0o = G0;
      G1o = G1;
    }
  }
  return best;
}

// Fresnel equations for incidence from n1 into n2, cos(theta_i) = ci >= 0.
// r/t = (rs, rp, ts, tp) as (re, im); returns true on total reflection.
__device__ __forceinline__ bool fresnel(double n1, double n2, double ci, double rt[8],
                                        double& ct) {
  double eta = n1 / n2;
  double st2 = eta * eta * (1.0 - ci * ci);
  if (st2 <= 1.0) {
    ct = sqrt(1.0 - st2);
    double a1 = n1 * ci, a2 = n2 * ct, b1 = n2 * ci, b2 = n1 * ct;
    double is = 1.0 / (a1 + a2), ip = 1.0 / (b1 + b2);
    rt[0] = (a1 - a2) * is;
    rt[1] = 0.0;
    rt[2] = (b1 - b2) * ip;
    rt[3] = 0.0;
    rt[4] = 2.0 * a1 * is;
    rt[5] = 0.0;
    rt[6] = 2.0 * a1 * ip;
    rt[7] = 0.0;
    return false;
  }
  // beyond the critical angle: cos(theta_t) = i kappa, r = (x - i y)/(x + i y)
  double kap = sqrt(st2 - 1.0);
  double xs = n1 * ci, ys = n2 * kap, xp = n2 * ci, yp = n1 * kap;
  double qs = 1.0 / fma(xs, xs, ys * ys), qp = 1.0 / fma(xp, xp, yp * yp);
  rt[0] = (xs * xs - ys * ys) * qs;
  rt[1] = -2.0 * xs * ys * qs;
  rt[2] = (xp * xp - yp * yp) * qp;
  rt[3] = -2.0 * xp * yp * qp;
  rt[4] = rt[5] = rt[6] = rt[7] = 0.0;
  ct = 0.0;
  return true;
}

// Per-wave statistics in LDS, indexed like the fields of rt_stats.  bump()
// adds the number of lanes calling it (one LDS atomic by the first of them),
// so it may be used inside divergent code.
enum : int {
  S_ACC = 0, S_REJ, S_RELOC, S_FORCED, S_EVENTS, S_SPAWNED, S_SUPP_GEN, S_SUPP_AMP,
  S_RECORDS, S_NEEDED, S_NONFINITE, S_MAXGEN, S_INVALID, S_REFILLS, S_SCHED, S_SPILLED,
  S_FIN,  // rays finished here and not yet added to q->finished (not a stat)
  S_COUNT
};
struct Counters {
  unsigned long long* c;  // this wave's row
  __device__ __forceinline__ void bump(int i) const {
    const uint64_t m = __ballot(1);
    if ((int)__lane_id() == __ffsll((unsigned long long)m) - 1)
      atomicAdd(&c[i], (unsigned long long)__popcll(m));
  }
  __device__ __forceinline__ void max_gen(int g) const {
    atomicMax(&c[S_MAXGEN], (unsigned long long)g);
  }
};

__device__ __forceinline__ uint64_t lanemask_lt() {
  return __lanemask_lt();
}

// Secondaries stay with the wave that cast them: a ring of record-slot
// indices per wave in LDS.  Producer and consumer are the same wave, so a
// workgroup-scope fence orders the child's record stores before the lane
// that later takes the child reads them; no cross-CU coherence is needed
// (the L2s of the eight XCDs are not coherent with each other, and
// publishing through them would mean L2 write-backs).
constexpr uint32_t kRing = 1024;  // LDS ring entries per wave (>= any local limit)
struct WaveQueue {
  int32_t* ring;   // kRing slot indices
  uint32_t* head;  // next index to take
  uint32_t* tail;  // next index to fill
};

// Reserve consecutive record slots for the calling wave's active lanes (one
// atomic per wave); returns this lane's slot index.
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

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// ---------------------------------------------------------------------------
// Ray held by one lane.
struct Ray {
  double y[7];  // x, y, z, w (v or p), tau
  double s, h;
  int32_t slot, region, gen, n_acc, n_rej, n_ev;
  uint32_t side;
};

// Direction state from a direction u: v = u/|u| (paper) or p = n(r) u/|u|.
template <int MODEL, int FIELD>
__device__ __forceinline__ void set_direction(const KParams& P, Ray& R, double ux, double uy,
                                              double uz) {
  const double il = rsqrt_nr(fma(ux, ux, fma(uy, uy, uz * uz)));
  double m = il;
  if constexpr (MODEL == RT_MODEL_EXACT) {
    double n, g[3];
    if constexpr (FIELD == 1) {
      field3<MODEL>(P, medium_of(P, R.region), R.y[0], R.y[1], R.y[2], n, g);
    } else {
      strat_field(medium_of(P, R.region), R.y[2], n, g[2]);
    }
    m = n * il;
  }
  R.y[3] = ux * m;
  R.y[4] = uy * m;
  R.y[5] = uz * m;
}

template <int MODEL, int FIELD>
__device__ __forceinline__ double field_n(const KParams& P, const Medium& M, const double y[7]) {
  double n, g[3];
  if constexpr (FIELD == 1) {
    field3<MODEL>(P, M, y[0], y[1], y[2], n, g);
  } else {
    strat_field(M, y[2], n, g[2]);
  }
  return n;
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
  R.n_acc = R.n_rej = R.n_ev = 0;
  set_direction<MODEL, FIELD>(P, R, Q.ux[slot], Q.uy[slot], Q.uz[slot]);
  C.max_gen(R.gen);
}

// Checks made before every normal trial step; returns a final status or 0.
__device__ __forceinline__ int32_t pretrial_status(const KParams& P, const Ray& R) {
  if (R.s >= P.s_max) return RT_ST_PATH;
  if ((int64_t)R.n_acc + R.n_rej >= P.max_steps) return RT_ST_STEPCAP;
  return 0;
}

// ---------------------------------------------------------------------------
template <int MODEL, int FIELD>
__device__ __forceinline__ void trial(const KParams& P, const Ray& R, double h, double y5[7],
                                      double& err) {
  if constexpr (FIELD == 1) {
    trial_3d<MODEL>(P, medium_of(P, R.region), R.y, h, P.inv_tol, y5, err);
  } else {
    trial_strat<MODEL>(medium_of(P, R.region), R.y, h, P.inv_tol, y5, err);
  }
}

// Boundary event at the located state ys (boundary k, at sigma along the
// step); returns the final status of the ray or 0 when it continues.
template <int MODEL, int FIELD>
__device__ __forceinline__ int32_t boundary_event(const KParams& P, Ray& R, int k, double sig,
                                                  double ys[7], double h_next, const Counters& C,
                                                  const WaveQueue& WQ) {
  const KBnd& B = s_bnd[k];
  if (B.kind != B_TIME) {
    // snap onto the plane
    double g = fma(ys[2], B.nrm[2], fma(ys[1], B.nrm[1], ys[0] * B.nrm[0])) - B.d;
    ys[0] -= g * B.nrm[0];
    ys[1] -= g * B.nrm[1];
    ys[2] -= g * B.nrm[2];
  }
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
  const double nin[3] = {sg * B.nrm[0], sg * B.nrm[1], sg * B.nrm[2]};
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
  const int i = R.slot;
  const double as_re = Q.as_re[i], as_im = Q.as_im[i];
  const double ap_re = Q.ap_re[i], ap_im = Q.ap_im[i];
  if (!tir) {
    if (R.gen + 1 < P.max_gen) {
      const double cs_re = as_re * rt[4] - as_im * rt[5];
      const double cs_im = as_re * rt[5] + as_im * rt[4];
      const double cp_re = ap_re * rt[6] - ap_im * rt[7];
      const double cp_im = ap_re * rt[7] + ap_im * rt[6];
      const double amax = fmax(hypot(cs_re, cs_im), hypot(cp_re, cp_im));
      if (P.amp_min > 0.0 && amax < P.amp_min) {
        C.bump(S_SUPP_AMP);
      } else {
        C.bump(S_SPAWNED);
        const uint64_t c = wave_append(&P.q->tail);
        if (c >= (uint64_t)P.capacity) {
          C.bump(S_FIN);  // no record slot: reported via stats.needed
        } else {
          const double eta = n1 / n2;
          const double f = eta * ci - ct;
          const uint64_t key = Q.key[i];
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
          if ((int)__lane_id() == __ffsll((unsigned long long)m) - 1) *WQ.tail = t + np;
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
  // the parent continues as the reflected ray
  const double rs_re = as_re * rt[0] - as_im * rt[1];
  const double rs_im = as_re * rt[1] + as_im * rt[0];
  const double rp_re = ap_re * rt[2] - ap_im * rt[3];
  const double rp_im = ap_re * rt[3] + ap_im * rt[2];
  Q.as_re[i] = rs_re;
  Q.as_im[i] = rs_im;
  Q.ap_re[i] = rp_re;
  Q.ap_im[i] = rp_im;
  const double c2 = 2.0 * ci;
  set_direction<MODEL, FIELD>(P, R, fma(c2, nin[0], u[0]), fma(c2, nin[1], u[1]),
                              fma(c2, nin[2], u[2]));
  if (P.amp_min > 0.0 && fmax(hypot(rs_re, rs_im), hypot(rp_re, rp_im)) < P.amp_min)
    return RT_ST_AMP;
  return 0;
}

// ---------------------------------------------------------------------------
// Persistent trace kernel.
// Step-size factor of the controller: min(5, 0.9 err^(-1/5)) after an
// accepted trial (exactly 5 below kErrCon), max(0.1, 0.9 err^(-1/4)) after a
// rejected one.  One Newton-refined power serves both cases.
__device__ __forceinline__ double step_factor(double err, bool accepted) {
  if (accepted && err < kErrCon) return kGrowMax;
  const float l = __builtin_amdgcn_logf((float)err);
  const float k = accepted ? -0.2f : -0.25f;
  double y = (double)__builtin_amdgcn_exp2f(l * k);
  // Newton on y^-K = err: y <- y ((K + 1) - err y^K) / K
  const double K = accepted ? 5.0 : 4.0, iK = accepted ? 0.2 : 0.25;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const double y2 = y * y;
    const double yk = accepted ? y2 * y2 * y : y2 * y2;
    y = y * fma(-err, yk, K + 1.0) * iK;
  }
  const double f = kSafety * y;
  return accepted ? f : fmax(kShrinkMin, f);
}

template <int MODEL, int FIELD>
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
  __shared__ double s_a[256], s_Ga[256], s_b[256], s_Gb[256], s_hp[256], s_hn[256];
  __shared__ int32_t s_k[256], s_meta[256];
  __syncthreads();

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
  //  * Primaries (record slots [0, n_primary)) are handed out in slot order,
  //    one fetch_add on q->head per wave refill.
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
  }
  bool prim_done = false;  // wave-uniform: no primaries left to claim
  int32_t ticket = -1;     // overflow ticket: -1 none, -2 exhausted, else entry
  uint32_t sleeps = 0;
  const Pool& Q = P.pool;

  for (;;) {
    // ---- boundary events located in the previous iteration ----
    if (mode == 2) {
      mode = 0;
      int32_t fin = boundary_event<MODEL, FIELD>(P, R, s_k[tid], lc, R.y, s_hn[tid], C, WQ);
      if (!fin) fin = pretrial_status(P, R);
      if (fin) {
        write_record(P, R, fin, C);
        R.slot = -1;
      }
    }
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
            if (Q.status[ti] == RT_ST_QUEUED) {
              load_ray<MODEL, FIELD>(P, (int32_t)ti, R, C);
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
      // nothing to step: publish finished counts, stop once no work can come
      if (lane == 0) {
        const unsigned long long f = C.c[S_FIN];
        if (f) {
          C.c[S_FIN] = 0;
          __hip_atomic_fetch_add(&P.q->finished, (uint64_t)f, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
        }
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
    if (R.slot < 0) continue;

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
      const double hn = clamp_h(P, ht * step_factor(err, accept));
      if (!finite) {
        C.bump(S_NONFINITE);
        fin = RT_ST_NONFINITE;
      } else if (!accept) {
        R.n_rej++;
        C.bump(S_REJ);
        R.h = hn;
      } else {
        R.n_acc++;
        C.bump(S_ACC);
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
          if (G0 <= 0.0) {
            s_meta[tid] = 1;  // pass 0, no iterations, last side 0
            located = true;
            sig = 0.0;
#pragma unroll
            for (int i = 0; i < 7; ++i) y5[i] = R.y[i];
          } else {
            s_a[tid] = 0.0;
            s_Ga[tid] = G0;
            s_b[tid] = ht;
            s_Gb[tid] = G1;
            s_meta[tid] = 1;
            lc = ht - G1 * ht / (G1 - G0);
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
        if (H0 <= 0.0) {
          sig = 0.0;
#pragma unroll
          for (int i = 0; i < 7; ++i) y5[i] = R.y[i];
          continue;
        }
        s_k[tid] = k;
        s_a[tid] = 0.0;
        s_Ga[tid] = H0;
        s_b[tid] = sig;
        s_Gb[tid] = H1;
        s_meta[tid] = (pass << 16) | 1;
        lc = sig - H1 * sig / (H1 - H0);
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

  // ---- per-wave statistics into the launch's rt_stats ----
  if (lane == 0) {
    unsigned long long* s64 = reinterpret_cast<unsigned long long*>(P.stats);
    for (int i = 0; i < S_FIN; ++i) {
      if (i == S_NEEDED || i == S_INVALID || C.c[i] == 0) continue;
      if (i == S_MAXGEN) atomicMax(&s64[i], C.c[i]);
      else atomicAdd(&s64[i], C.c[i]);
    }
  }
}

// Persistent trace kernels.  The stratified variants are held to three
// waves per SIMD (168 VGPRs): latency of the FP64 dependency chains is hidden
// by occupancy, and they fit without spilling.
template <int MODEL>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
trace_strat_kernel(KParams P) {
  trace_body<MODEL, 0>(P);
}
template <int MODEL>
__global__ void __launch_bounds__(256) trace_grid_kernel(KParams P) {
  trace_body<MODEL, 1>(P);
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
  }
}

// Records the launch needed = primaries + every secondary reserved.
__global__ void finish_kernel(KParams P) {
  if (threadIdx.x == 0) P.stats->needed = (int64_t)P.q->tail;
}

// FP32 grid -> float4 nodes (n, Dx, Dy, Dz): D is the central difference of
// the neighbours, or twice the one-sided difference at an edge, so that
// grad n = D / (2 spacing) everywhere.  The FP32 differences are exact for
// values within a factor of two of each other (Sterbenz).
__global__ void grid_prep_kernel(const float* __restrict__ n, float4* __restrict__ out, int nx,
                                 int ny, int nz) {
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
  out[id] = make_float4(c, dx, dy, dz);
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
    const double g = r[0] * B.nrm[0] + r[1] * B.nrm[1] + r[2] * B.nrm[2] - B.d;
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

template <int MODEL, int FIELD>
void* trace_kernel_ptr() {
  return FIELD ? reinterpret_cast<void*>(&trace_grid_kernel<MODEL>)
               : reinterpret_cast<void*>(&trace_strat_kernel<MODEL>);
}

template <int MODEL, int FIELD>
int max_blocks_per_cu(int block) {
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

template <int MODEL, int FIELD>
hipError_t launch_trace(const KParams& P, int grid, int block, hipStream_t s) {
  if constexpr (FIELD == 1)
    hipLaunchKernelGGL((trace_grid_kernel<MODEL>), dim3(grid), dim3(block), 0, s, P);
  else
    hipLaunchKernelGGL((trace_strat_kernel<MODEL>), dim3(grid), dim3(block), 0, s, P);
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

extern "C" rt_status raytrace_launch(const rt_field* field, const rt_boundaries* bnd,
                                     const rt_sources* src, const rt_directions* dirs, double tol,
                                     const rt_step_limits* L, rt_outputs* out, void* workspace,
                                     size_t workspace_bytes, void* stream,
                                     const rt_tuning* tuning) {
  using namespace rt;
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
  const int refill = tuning && tuning->refill_threshold ? tuning->refill_threshold : 16;
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
  }
  int nb = 0;
  for (int i = 0; i < bnd->n_planes; ++i) {
    const rt_plane& p = bnd->planes[i];
    KBnd& b = P.bnd[nb++];
    const double len = sqrt(p.normal[0] * p.normal[0] + p.normal[1] * p.normal[1] +
                            p.normal[2] * p.normal[2]);
    for (int a = 0; a < 3; ++a) b.nrm[a] = p.normal[a] / len;
    b.d = p.point[0] * b.nrm[0] + p.point[1] * b.nrm[1] + p.point[2] * b.nrm[2];
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
  P.pool = Pool{out->x,     out->y,     out->z,     out->ux,    out->uy,    out->uz,
                out->s,     out->t,     out->as_re, out->as_im, out->ap_re, out->ap_im,
                out->h,     out->key,   out->parent, out->gen,  out->status, out->n_acc,
                out->n_rej, out->n_ev,  out->region, out->side};
  P.capacity = out->capacity;
  P.n_primary = dirs->n;
  P.q = static_cast<QueueCounters*>(workspace);
  P.gq = reinterpret_cast<int32_t*>(static_cast<char*>(workspace) + 4096);
  const size_t gq_bytes = ((size_t)out->capacity * 4 + 4095) / 4096 * 4096;
  P.stats = out->stats;
  const bool grid = field_uses_grid(field);
  if (grid) {
    const rt_grid& g = field->grid;
    P.nodes = static_cast<char*>(workspace) + 4096 + gq_bytes;
    P.gnx = g.nx;
    P.gny = g.ny;
    P.gnz = g.nz;
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

  hipLaunchKernelGGL(reset_kernel, dim3(1), dim3(64), 0, s, P);
  HIP_TRY(hipGetLastError());
  if (grid) {
    const int64_t total = (int64_t)field->grid.nx * field->grid.ny * field->grid.nz;
    hipLaunchKernelGGL(grid_prep_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                       field->grid.n, static_cast<float4*>(const_cast<void*>(P.nodes)),
                       field->grid.nx, field->grid.ny, field->grid.nz);
    HIP_TRY(hipGetLastError());
  }
  if (out->capacity > 0) {
    hipLaunchKernelGGL(init_kernel, dim3((unsigned)((out->capacity + 255) / 256)), dim3(256), 0,
                       s, P, src->xyz, src->n, dirs->xyz, dirs->src, P.h_init);
    HIP_TRY(hipGetLastError());
  }

  // persistent grid: every CU filled to its occupancy, fewer blocks for
  // small launches
  int bpc = 0;
  if (L->model == RT_MODEL_PAPER)
    bpc = grid ? max_blocks_per_cu<RT_MODEL_PAPER, 1>(block) : max_blocks_per_cu<RT_MODEL_PAPER, 0>(block);
  else
    bpc = grid ? max_blocks_per_cu<RT_MODEL_EXACT, 1>(block) : max_blocks_per_cu<RT_MODEL_EXACT, 0>(block);
  if (tuning && tuning->blocks_per_cu > 0) bpc = std::min(bpc, (int)tuning->blocks_per_cu);
  int64_t nblk = (int64_t)g_dev.n_cu * bpc;
  const int64_t by_rays = std::max<int64_t>(1, (dirs->n + block - 1) / block);
  nblk = std::max<int64_t>(1, std::min(nblk, by_rays));

  if (tuning && tuning->ev_trace_begin)
    HIP_TRY(hipEventRecord(static_cast<hipEvent_t>(tuning->ev_trace_begin), s));
  hipError_t e;
  if (L->model == RT_MODEL_PAPER)
    e = grid ? launch_trace<RT_MODEL_PAPER, 1>(P, (int)nblk, block, s)
             : launch_trace<RT_MODEL_PAPER, 0>(P, (int)nblk, block, s);
  else
    e = grid ? launch_trace<RT_MODEL_EXACT, 1>(P, (int)nblk, block, s)
             : launch_trace<RT_MODEL_EXACT, 0>(P, (int)nblk, block, s);
  HIP_TRY(e);
  if (tuning && tuning->ev_trace_end)
    HIP_TRY(hipEventRecord(static_cast<hipEvent_t>(tuning->ev_trace_end), s));
  hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(64), 0, s, P);
  HIP_TRY(hipGetLastError());
  return RT_OK;
}
