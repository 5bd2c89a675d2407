// Device building blocks shared by the trace and the solve kernels:
// Cash-Karp trial steps in stratified, general analytic and gridded media
// (first-order and Nystrom forms), the step-size
// controller, boundary functions and crossing selection, Fresnel
// coefficients, per-wave statistics rows.  FP64 throughout; gfx950.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>

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

__device__ constexpr double ck_b(int j) {
  return j == 0 ? kB1 : j == 2 ? kB3 : j == 3 ? kB4 : j == 5 ? kB6 : 0.0;
}
__device__ constexpr double ck_e(int j) {
  return j == 0 ? kE1 : j == 2 ? kE3 : j == 3 ? kE4 : j == 4 ? kE5 : j == 5 ? kE6 : 0.0;
}
// Products of the tableau for the Nystrom form of a step of r'' = f(r):
// nodes c_s = sum_j a_sj, (A^2)_si = sum_j a_sj a_ji, (bA)_i, (eA)_i.
__device__ constexpr double ck_c(int s) {
  double c = 0.0;
  for (int j = 0; j < s; ++j) c += ck_a(s, j);
  return c;
}
__device__ constexpr double ck_aa(int s, int i) {
  double v = 0.0;
  for (int j = i + 1; j < s; ++j) v += ck_a(s, j) * ck_a(j, i);
  return v;
}
__device__ constexpr double ck_ba(int i) {
  double v = 0.0;
  for (int j = i + 1; j < 6; ++j) v += ck_b(j) * ck_a(j, i);
  return v;
}
__device__ constexpr double ck_ea(int i) {
  double v = 0.0;
  for (int j = i + 1; j < 6; ++j) v += ck_e(j) * ck_a(j, i);
  return v;
}

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

// a * b + c as one three-operand FP64 FMA (v_fma_f64) whatever registers
// hold c.  Written out because the compiler otherwise picks the
// two-operand form, whose addend is also its destination, and copies a
// loop-held coefficient into it before every term of a polynomial.
__device__ __forceinline__ double fma3(double a, double b, double c) {
  double r;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}

// e^x for |x| <= 0.25: Taylor polynomial to degree 11 (truncation below
// 2^-52 relative), Horner form.
__device__ __forceinline__ double exp_small(double x) {
  double p = 1.0 / 39916800.0;
  p = fma3(p, x, 1.0 / 3628800.0);
  p = fma3(p, x, 1.0 / 362880.0);
  p = fma3(p, x, 1.0 / 40320.0);
  p = fma3(p, x, 1.0 / 5040.0);
  p = fma3(p, x, 1.0 / 720.0);
  p = fma3(p, x, 1.0 / 120.0);
  p = fma3(p, x, 1.0 / 24.0);
  p = fma3(p, x, 1.0 / 6.0);
  p = fma(p, x, 0.5);
  p = fma(p, x, 1.0);
  return fma(p, x, 1.0);
}

// e^x for any x: Cody and Waite's reduction by ln 2 and a Taylor polynomial.
// x = k ln2 + r with k = rint(x / ln2) and |r| <= ln2 / 2; ln2 = L1 + L2,
// L1 holding 42 significant bits, so that k L1 is exact for |k| < 2^11 and
// x - k L1 is rounded once; e^r by its Taylor polynomial of degree 13
// (remainder below 2^-56 relative), then scaled by 2^k.  x is first clamped
// to [-746, 709], beyond which e^x is below the smallest subnormal or
// overflows.
__device__ __forceinline__ double exp_rr(double x) {
  constexpr double kL1 = 0x1.62e42fefa38p-1, kL2 = 5.497923018708371e-14;
  x = fmin(fmax(x, -746.0), 709.0);
  const double k = __builtin_rint(x * 1.4426950408889634);
  double r = fma(-k, kL1, x);
  r = fma(-k, kL2, r);
  double p = fma(r, 1.0 / 6227020800.0, 1.0 / 479001600.0);
  p = fma3(p, r, 1.0 / 39916800.0);
  p = fma3(p, r, 1.0 / 3628800.0);
  p = fma3(p, r, 1.0 / 362880.0);
  p = fma3(p, r, 1.0 / 40320.0);
  p = fma3(p, r, 1.0 / 5040.0);
  p = fma3(p, r, 1.0 / 720.0);
  p = fma3(p, r, 1.0 / 120.0);
  p = fma3(p, r, 1.0 / 24.0);
  p = fma3(p, r, 1.0 / 6.0);
  p = fma(p, r, 0.5);
  p = fma(p, r, 1.0);
  p = fma(p, r, 1.0);
  return __builtin_amdgcn_ldexp(p, (int)k);
}

// Medium of one ray, kept in registers: n(z) = a + b z - dn exp(-z/z0).
struct Medium {
  double a, b, dn, inv_z0, dn_inv_z0;
  int use_grid, reg;
};

// Media and boundary tables indexed per lane (by a ray's medium or by the
// boundary it is searching): copied into LDS at kernel start.  Loops over all
// boundaries use the uniform copy in the kernel arguments instead.
__shared__ KRegion s_reg[RT_MAX_REGIONS];
__shared__ KBnd s_bnd[kMaxBnd];

__device__ __forceinline__ Medium medium_of(const KParams& P, int r) {
  (void)P;
  const KRegion& R = s_reg[r];
  return Medium{R.a, R.b, R.dn, R.inv_z0, R.dn_inv_z0, R.use_grid, r};
}

__device__ __forceinline__ void strat_field(const Medium& M, double z, double& n, double& gz) {
  double e = 0.0;
  if (M.dn != 0.0) e = exp(-z * M.inv_z0);
  n = fma(M.b, z, M.a) - M.dn * e;
  gz = fma(M.dn_inv_z0, e, M.b);
}

// Same at the step's start z, where E = exp(-z/z0) is known.
__device__ __forceinline__ void strat_field_at(const Medium& M, double z, double E, double& n,
                                               double& gz) {
  const double e = M.dn != 0.0 ? E : 0.0;
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

// 1/k! for k = 0..13.
__device__ constexpr double inv_fact(int k) {
  double f = 1.0;
  for (int i = 2; i <= k; ++i) f *= (double)i;
  return 1.0 / f;
}
// e^x by its Taylor polynomial of degree D in Horner form.  Its remainder,
// at most |x|^(D+1) / (D+1)! e^|x|, is below 2^-53 of e^x for
// |x| <= taylor_max(D): the largest such |x|, rounded down.
template <int D>
__device__ __forceinline__ double exp_taylor(double x) {
  double p = inv_fact(D);
#pragma unroll
  for (int k = D - 1; k >= 3; --k) p = fma3(p, x, inv_fact(k));
  p = fma(p, x, 0.5);
  p = fma(p, x, 1.0);
  return fma(p, x, 1.0);
}
__device__ constexpr double taylor_max(int D) {
  return D <= 7 ? 0.0377 : D == 8 ? 0.0689 : D == 9 ? 0.1123 : D == 10 ? 0.1687 : 0.2380;
}
// Taylor degree at stage s (1..5) of a trial: stage s lies about c_s h
// from the step's start (nodes c = 1/5, 3/10, 3/5, 1, 7/8), so for steps up
// to a sixth of z0 the early stages need fewer terms.
__device__ constexpr int stage_degree(int s) {
  return s == 1 ? 7 : s == 2 ? 8 : s == 3 ? 9 : 10;
}

// strat_field_rel at stage S without a branch: slow is raised when the
// exponent is outside the Taylor range of the stage (or NaN); the caller
// then recomputes the step with strat_field_rel.  The step's start z0 enters
// through A0 = a + b z0, and dnE0 = dn E0 and gE0 = (dn / z0) E0 are the
// step's factors of exp(-dz / z0) in n and dn/dz.  Media with dn = 0 have
// inv_z0 = 0 and both factors 0.
template <int S>
__device__ __forceinline__ void strat_field_stage_fast(const Medium& M, double A0, double dz,
                                                       double dnE0, double gE0, double& n,
                                                       double& gz, bool& slow) {
  constexpr int D = stage_degree(S);
  const double x = -dz * M.inv_z0;
  slow = slow || !(fabs(x) <= taylor_max(D));
  const double p = exp_taylor<D>(x);
  n = fma(-dnE0, p, fma(M.b, dz, A0));
  gz = fma(gE0, p, M.b);
}
__device__ __forceinline__ void strat_field_fast_at(int st, const Medium& M, double A0, double dz,
                                                    double dnE0, double gE0, double& n,
                                                    double& gz, bool& slow) {
  switch (st) {
    case 1: strat_field_stage_fast<1>(M, A0, dz, dnE0, gE0, n, gz, slow); break;
    case 2: strat_field_stage_fast<2>(M, A0, dz, dnE0, gE0, n, gz, slow); break;
    case 3: strat_field_stage_fast<3>(M, A0, dz, dnE0, gE0, n, gz, slow); break;
    case 4: strat_field_stage_fast<4>(M, A0, dz, dnE0, gE0, n, gz, slow); break;
    default: strat_field_stage_fast<5>(M, A0, dz, dnE0, gE0, n, gz, slow); break;
  }
}

// Trilinear n and gradient from float4 nodes (n, Dx, Dy, Dz); positions
// outside the grid are clamped onto it; grad n = D / (2 spacing).  In two
// parts, so that a caller can issue the eight corner loads of one
// evaluation before it blends those of another: grid_fetch (cell, fractions
// and the corner loads), grid_blend (weights and sums).
struct GridFetch {
  float4 c[8];
  double t[3];
};

// Node (i, j, k) of the prepared grid: float4 nodes stored in bricks of
// 2 x 2 x 2 nodes, one 128-byte cache line each, bricks x fastest; within a
// brick the node's x, y, z parities select its float4.  A cell's eight
// corners then lie in one to eight lines (3.4 on average) instead of four
// or more with rows of nodes.
__host__ __device__ __forceinline__ size_t node_index(int i, int j, int k, int bx, int by) {
  const size_t brick = ((size_t)(k >> 1) * by + (size_t)(j >> 1)) * bx + (size_t)(i >> 1);
  return brick * 8 + (size_t)((i & 1) | ((j & 1) << 1) | ((k & 1) << 2));
}

__device__ __forceinline__ void grid_fetch(const KParams& P, double x, double y, double z,
                                           GridFetch& F) {
  const float4* __restrict__ nodes = static_cast<const float4*>(P.nodes);
  double f[3] = {(x - P.gorg[0]) * P.ginv[0], (y - P.gorg[1]) * P.ginv[1],
                 (z - P.gorg[2]) * P.ginv[2]};
  int i0[3];
  const int dims[3] = {P.gnx, P.gny, P.gnz};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double v = fmin(fmax(f[a], 0.0), P.gmax[a]);
    int i = (int)floor(v);
    i = min(i, dims[a] - 2);
    i0[a] = i;
    F.t[a] = v - (double)i;
  }
  // per axis, the byte offsets of the cell's two node planes (32 bits:
  // the node array is under 4 GiB)
  const char* base = static_cast<const char*>(P.nodes);
  const uint32_t sy = (uint32_t)P.gbx * 128u, sz = sy * (uint32_t)P.gby;
  uint32_t ox[2], oy[2], oz[2];
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const uint32_t i = (uint32_t)(i0[0] + e), j = (uint32_t)(i0[1] + e), k = (uint32_t)(i0[2] + e);
    ox[e] = ((i >> 1) << 7) | ((i & 1u) << 4);
    oy[e] = (j >> 1) * sy + ((j & 1u) << 5);
    oz[e] = (k >> 1) * sz + ((k & 1u) << 6);
  }
#pragma unroll
  for (int q = 0; q < 8; ++q)
    F.c[q] = *reinterpret_cast<const float4*>(base + (ox[q & 1] + oy[(q >> 1) & 1] +
                                                      oz[(q >> 2) & 1]));
}

__device__ __forceinline__ void grid_blend(const KParams& P, const GridFetch& F, double& n,
                                           double g[3]) {
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    double w = ((q & 1) ? F.t[0] : 1.0 - F.t[0]) * ((q & 2) ? F.t[1] : 1.0 - F.t[1]) *
               ((q & 4) ? F.t[2] : 1.0 - F.t[2]);
    acc[0] = fma(w, (double)F.c[q].x, acc[0]);
    acc[1] = fma(w, (double)F.c[q].y, acc[1]);
    acc[2] = fma(w, (double)F.c[q].z, acc[2]);
    acc[3] = fma(w, (double)F.c[q].w, acc[3]);
  }
  n = acc[0];
  g[0] = acc[1] * P.ghalf[0];
  g[1] = acc[2] * P.ghalf[1];
  g[2] = acc[3] * P.ghalf[2];
}

__device__ __forceinline__ void grid_field(const KParams& P, double x, double y, double z,
                                           double& n, double g[3]) {
  GridFetch F;
  grid_fetch(P, x, y, z, F);
  grid_blend(P, F, n, g);
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

// FAST (paper model): stages without branches (strat_field_stage_fast);
// *slow_out tells whether a stage left its Taylor range, in which case the
// caller repeats the step with FAST = false.
template <int MODEL, bool FAST = false>
__device__ __forceinline__ void trial_strat(const Medium& M, const double y[7], double h,
                                            double inv_tol, double y5[7], double& err,
                                            bool* slow_out = nullptr) {
  const double E0 = FAST ? exp_rr(-y[2] * M.inv_z0) : (M.dn != 0.0 ? exp(-y[2] * M.inv_z0) : 0.0);
  const double dnE0 = M.dn * E0, gE0 = M.dn_inv_z0 * E0, A0 = fma(M.b, y[2], M.a);
  bool slow = false;
  if constexpr (MODEL == RT_MODEL_PAPER) {
    // w = unit velocity, renormalised after every accepted step (|w| = 1).
    // z'' = (dn/dz)/n depends on z alone: the Nystrom form of the step, as
    // in trial_3d, keeps only the w_z derivatives.
    double kw[6];
    double tsum = 0.0;  // sum_j b_j n_j / c0
#pragma unroll
    for (int st = 0; st < 6; ++st) {
      double n, gz;
      if (st == 0) {
        strat_field_at(M, y[2], E0, n, gz);
      } else {
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i + 1 < st; ++i) acc = fma(ck_aa(st, i), kw[i], acc);
        const double dz = h * fma(h, acc, ck_c(st) * y[5]);
        if constexpr (FAST) strat_field_fast_at(st, M, A0, dz, dnE0, gE0, n, gz, slow);
        else strat_field_rel(M, y[2], dz, E0, n, gz);
      }
      kw[st] = gz * rcp_nr(n);
      if (st == 0) tsum = kB1 * n;
      if (st == 2) tsum = fma(kB3, n, tsum);
      if (st == 3) tsum = fma(kB4, n, tsum);
      if (st == 5) tsum = fma(kB6, n, tsum);
    }
    double ba = 0.0, ea = 0.0;
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      ba = fma(ck_ba(i), kw[i], ba);
      ea = fma(ck_ea(i), kw[i], ea);
    }
    y5[0] = fma(h, y[3], y[0]);
    y5[1] = fma(h, y[4], y[1]);
    y5[2] = fma(h, fma(h, ba, y[5]), y[2]);
    y5[3] = y[3];
    y5[4] = y[4];
    y5[5] = fma(h, b_sum(kw), y[5]);
    y5[6] = fma(h * kInvC0, tsum, y[6]);
    err = fmax(fabs(h * ea), fabs(h * e_sum(kw))) * inv_tol;
    if (slow_out) *slow_out = slow;
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
      if (st == 0) strat_field_at(M, y[2], E0, n, gz);
      else strat_field_rel(M, y[2], dz, E0, n, gz);
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

// General 3-D gradient: gridded media, or analytic media stratified along
// their axis (ax, from LDS), plus the Gaussian anomalies of the medium's
// region (uniform loop over the kernel arguments).
template <int MODEL>
__device__ __forceinline__ void field3(const KParams& P, const Medium& M, double x, double y,
                                       double z, double& n, double g[3]) {
  if (M.use_grid) {
    grid_field(P, x, y, z, n, g);
  } else {
    const double* ax = s_reg[M.reg].ax;
    const double zeta = fma(ax[0], x, fma(ax[1], y, ax[2] * z));
    double gs;
    strat_field(M, zeta, n, gs);
    g[0] = gs * ax[0];
    g[1] = gs * ax[1];
    g[2] = gs * ax[2];
  }
  for (int j = 0; j < P.n_anom; ++j) {
    const KAnom& A = P.anom[j];
    if (A.region != M.reg) continue;
    const double dx = x - A.c[0], dy = y - A.c[1], dz = z - A.c[2];
    const double q = fma(dx, dx, fma(dy, dy, dz * dz));
    const double v = A.amp * exp(-q * A.k);
    const double f = -2.0 * A.k * v;  // grad = -2 k v (r - c)
    n += v;
    g[0] = fma(f, dx, g[0]);
    g[1] = fma(f, dy, g[1]);
    g[2] = fma(f, dz, g[2]);
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

// Paper-model trial in a gridded medium without anomalies (trial_3d's
// Nystrom form, same arithmetic): stage s's position needs the derivatives
// of stages 0 .. s-2 only ((A^2)_s,s-1 = 0), so the corner loads of stage
// s + 1 are issued before stage s is blended, and two stages' gathers are
// in flight at a time.
__device__ __forceinline__ void trial_grid_paper(const KParams& P, const double y[7], double h,
                                                 double inv_tol, double y5[7], double& err) {
  double kw[3][6];
  double tsum = 0.0;
  GridFetch F[2];
  grid_fetch(P, y[0], y[1], y[2], F[0]);
  {
    const double c1h = ck_c(1) * h;
    grid_fetch(P, fma(c1h, y[3], y[0]), fma(c1h, y[4], y[1]), fma(c1h, y[5], y[2]), F[1]);
  }
#pragma unroll
  for (int st = 0; st < 6; ++st) {
    double n, g[3];
    grid_blend(P, F[st & 1], n, g);
    const double in = rcp_nr(n);
#pragma unroll
    for (int c = 0; c < 3; ++c) kw[c][st] = g[c] * in;
    if (st == 0) tsum = kB1 * n;
    if (st == 2) tsum = fma(kB3, n, tsum);
    if (st == 3) tsum = fma(kB4, n, tsum);
    if (st == 5) tsum = fma(kB6, n, tsum);
    const int nx = st + 2;  // the stage whose loads go out now
    if (nx < 6) {
      double rs[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i + 1 < nx; ++i) acc = fma(ck_aa(nx, i), kw[c][i], acc);
        rs[c] = fma(h, fma(h, acc, ck_c(nx) * y[3 + c]), y[c]);
      }
      grid_fetch(P, rs[0], rs[1], rs[2], F[st & 1]);
    }
  }
  double dr[3], dw[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double ba = 0.0, ea = 0.0;
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      ba = fma(ck_ba(i), kw[c][i], ba);
      ea = fma(ck_ea(i), kw[c][i], ea);
    }
    y5[c] = fma(h, fma(h, ba, y[3 + c]), y[c]);
    y5[3 + c] = fma(h, b_sum(kw[c]), y[3 + c]);
    dr[c] = h * ea;
    dw[c] = e_sum(kw[c]);
  }
  y5[6] = fma(h * kInvC0, tsum, y[6]);
  const double dr_h = sqrt(fma(dr[0], dr[0], fma(dr[1], dr[1], dr[2] * dr[2])));
  const double dw_h = sqrt(fma(dw[0], dw[0], fma(dw[1], dw[1], dw[2] * dw[2])));
  const double iw0 = rsqrt_nr(fma(y[3], y[3], fma(y[4], y[4], y[5] * y[5])));
  err = fmax(dr_h, h * dw_h * iw0) * inv_tol;
}

template <int MODEL>
__device__ __forceinline__ void trial_3d(const KParams& P, const Medium& M, const double y[7],
                                         double h, double inv_tol, double y5[7], double& err) {
  if constexpr (MODEL == RT_MODEL_PAPER) {
    // w' = grad n / n depends on r alone, so the same Cash-Karp step takes
    // its Nystrom form (equal in exact arithmetic): stage positions
    // r_s = r0 + h c_s w0 + h^2 sum_i (A^2)_si kw_i, output
    // r5 = r0 + h w0 + h^2 sum_i (bA)_i kw_i, position error / h
    // = h sum_i (eA)_i kw_i (the e_j sum to zero).  Only the w-derivatives
    // kw are kept: half the stage registers of the first-order form.
    double kw[3][6];
    double tsum = 0.0;
#pragma unroll
    for (int st = 0; st < 6; ++st) {
      double rs[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if (st == 0) {
          rs[c] = y[c];
        } else {
          double acc = 0.0;
#pragma unroll
          for (int i = 0; i + 1 < st; ++i) acc = fma(ck_aa(st, i), kw[c][i], acc);
          rs[c] = fma(h, fma(h, acc, ck_c(st) * y[3 + c]), y[c]);
        }
      }
      double n, g[3];
      field3<MODEL>(P, M, rs[0], rs[1], rs[2], n, g);
      const double in = rcp_nr(n);
#pragma unroll
      for (int c = 0; c < 3; ++c) kw[c][st] = g[c] * in;
      if (st == 0) tsum = kB1 * n;
      if (st == 2) tsum = fma(kB3, n, tsum);
      if (st == 3) tsum = fma(kB4, n, tsum);
      if (st == 5) tsum = fma(kB6, n, tsum);
    }
    double dr[3], dw[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      double ba = 0.0, ea = 0.0;
#pragma unroll
      for (int i = 0; i < 5; ++i) {
        ba = fma(ck_ba(i), kw[c][i], ba);
        ea = fma(ck_ea(i), kw[c][i], ea);
      }
      y5[c] = fma(h, fma(h, ba, y[3 + c]), y[c]);
      y5[3 + c] = fma(h, b_sum(kw[c]), y[3 + c]);
      dr[c] = h * ea;
      dw[c] = e_sum(kw[c]);
    }
    y5[6] = fma(h * kInvC0, tsum, y[6]);
    const double dr_h = sqrt(fma(dr[0], dr[0], fma(dr[1], dr[1], dr[2] * dr[2])));
    const double dw_h = sqrt(fma(dw[0], dw[0], fma(dw[1], dw[1], dw[2] * dw[2])));
    const double iw0 = rsqrt_nr(fma(y[3], y[3], fma(y[4], y[4], y[5] * y[5])));
    err = fmax(dr_h, h * dw_h * iw0) * inv_tol;
    return;
  }
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
// Crossing search (Illinois false position) limits: it stops when the
// bracket on the step parameter is narrower than kLocWRel times the step, or
// when |g| <= kLocGTol, which is 0: only an exact zero, since at grazing
// incidence a small |g| leaves the crossing undetermined along the ray.
constexpr double kLocGTol = 0.0, kLocWRel = 1e-12;
constexpr int kLocMaxIt = 60, kLocMaxPass = 8, kMaxEvents = 255;
// A step starts on a boundary when G0 <= 2^-33 m (~1.2e-10 m, about the
// search tolerance), tested as G0 * 2^33 <= 1 with immediate operands only
// (a 64-bit constant would occupy scalar registers across the step loop).
__device__ __forceinline__ bool on_boundary(double G0) {
  return __builtin_amdgcn_ldexp(G0, 33) <= 1.0;
}

__device__ __forceinline__ double clamp_h(const KParams& P, double h) {
  return fmin(fmax(h, P.h_min), P.h_max);
}

// Value of a boundary surface's function g at y (positive on its
// region_pos side): a plane's signed distance, a sphere's distance from its
// centre minus the radius, a paraboloid's depth difference.
__device__ __forceinline__ double bnd_value(const KBnd& B, const double* y) {
  if (B.shape == SH_SPHERE) {
    const double dx = y[0] - B.nrm[0], dy = y[1] - B.nrm[1], dz = y[2] - B.nrm[2];
    return sqrt(fma(dx, dx, fma(dy, dy, dz * dz))) - B.d;
  }
  if (B.shape == SH_PARABOLOID) {
    const double dx = y[0] - B.nrm[0], dy = y[1] - B.nrm[1];
    return y[2] - B.nrm[2] - B.d * fma(dx, dx, dy * dy);
  }
  return fma(y[2], B.nrm[2], fma(y[1], B.nrm[1], y[0] * B.nrm[0])) - B.d;
}

// Unit normal of a boundary at y, pointing to its g > 0 side.
__device__ __forceinline__ void bnd_normal(const KBnd& B, const double* y, double n[3]) {
  if (B.shape == SH_PLANE) {
    n[0] = B.nrm[0];
    n[1] = B.nrm[1];
    n[2] = B.nrm[2];
    return;
  }
  if (B.shape == SH_SPHERE) {
    n[0] = y[0] - B.nrm[0];
    n[1] = y[1] - B.nrm[1];
    n[2] = y[2] - B.nrm[2];
  } else {
    n[0] = -2.0 * B.d * (y[0] - B.nrm[0]);
    n[1] = -2.0 * B.d * (y[1] - B.nrm[1]);
    n[2] = 1.0;
  }
  const double il = rsqrt_nr(fma(n[0], n[0], fma(n[1], n[1], n[2] * n[2])));
  n[0] *= il;
  n[1] *= il;
  n[2] *= il;
}

// Put a located point onto the boundary: along the normal (plane),
// radially (sphere), vertically (paraboloid, whose g is a depth difference).
__device__ __forceinline__ void bnd_snap(const KBnd& B, double* y) {
  if (B.shape == SH_SPHERE) {
    const double dx = y[0] - B.nrm[0], dy = y[1] - B.nrm[1], dz = y[2] - B.nrm[2];
    const double f = B.d * rsqrt_nr(fma(dx, dx, fma(dy, dy, dz * dz)));
    y[0] = fma(f, dx, B.nrm[0]);
    y[1] = fma(f, dy, B.nrm[1]);
    y[2] = fma(f, dz, B.nrm[2]);
  } else if (B.shape == SH_PARABOLOID) {
    y[2] -= bnd_value(B, y);
  } else {
    const double g = bnd_value(B, y);
    y[0] -= g * B.nrm[0];
    y[1] -= g * B.nrm[1];
    y[2] -= g * B.nrm[2];
  }
}

// Boundary function with the ray's side sign applied: > 0 before crossing.
__device__ __forceinline__ double bnd_G(const KParams& P, const KBnd& B, int k, uint32_t side,
                                        const double y[7]) {
  if (B.kind == B_TIME) return (P.t_max - y[6]) * 299792458.0;
  const double g = bnd_value(B, y);
  return ((side >> k) & 1u) ? g : -g;
}

// Departure rate of a ray standing on boundary k: the cosine between its
// direction and the normal pointing into its own side (> 0 when it leaves
// the boundary; -1 for the travel-time limit, which a ray only approaches).
__device__ __forceinline__ double bnd_rate(const KBnd& B, int k, uint32_t side,
                                           const double y[7]) {
  if (B.kind == B_TIME) return -1.0;
  double n0 = B.nrm[0], n1 = B.nrm[1], n2 = B.nrm[2];
  if (B.shape == SH_SPHERE) {
    n0 = y[0] - n0;
    n1 = y[1] - n1;
    n2 = y[2] - n2;
  } else if (B.shape == SH_PARABOLOID) {
    n0 = -2.0 * B.d * (y[0] - n0);
    n1 = -2.0 * B.d * (y[1] - n1);
    n2 = 1.0;
  }
  const double nn = fma(n0, n0, fma(n1, n1, n2 * n2));
  const double uu = fma(y[3], y[3], fma(y[4], y[4], y[5] * y[5]));
  const double c = fma(y[5], n2, fma(y[4], n1, y[3] * n0)) * rsqrt_nr(nn * uu);
  return ((side >> k) & 1u) ? c : -c;
}

// Start value of the return search of a ray leaving boundary k: rate * len,
// the distance from the boundary a straight departure would gain over the
// step; inside a sphere, where a straight line leaving the wall at cosine
// rate meets it again after the chord 2 R rate, the value that puts the
// first false-position iterate at that chord when it lies inside the step
// (exact for a straight ray, as in a void of constant index).
__device__ __forceinline__ double departure_start(const KBnd& B, int k, uint32_t side,
                                                  double rate, double len, double G1) {
  if (B.shape == SH_SPHERE && !((side >> k) & 1u)) {
    const double chord = 2.0 * B.d * rate;
    if (chord < len) return -G1 * chord / (len - chord);
  }
  return rate * len;
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

// Per-wave statistics rows in LDS.  bump() adds the number of lanes
// calling it (one LDS atomic by the first of them), so it may be used
// inside divergent code.
struct Counters {
  unsigned long long* c;  // this wave's row
  __device__ __forceinline__ void bump(int i) const {
    const uint64_t m = __ballot(1);
    if ((int)__lane_id() == __ffsll((unsigned long long)m) - 1)
      atomicAdd(&c[i], (unsigned long long)__popcll(m));
  }
  __device__ __forceinline__ void max(int i, unsigned long long v) const {
    atomicMax(&c[i], v);
  }
};

__device__ __forceinline__ uint64_t lanemask_lt() {
  return __lanemask_lt();
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

template <int MODEL, int FIELD>
__device__ __forceinline__ void trial(const KParams& P, const Ray& R, double h, double y5[7],
                                      double& err) {
  if constexpr (FIELD == 1) {
    const Medium M = medium_of(P, R.region);
    if (MODEL == RT_MODEL_PAPER && M.use_grid && P.n_anom == 0)
      trial_grid_paper(P, R.y, h, P.inv_tol, y5, err);
    else
      trial_3d<MODEL>(P, M, R.y, h, P.inv_tol, y5, err);
  } else {
    if constexpr (MODEL == RT_MODEL_PAPER) {
      // the branch-free form first (one basic block, so the stages' code can
      // interleave); a lane whose stages left their Taylor ranges repeats
      // the step with the general exponential
      const Medium M = medium_of(P, R.region);
      bool slow = false;
      trial_strat<MODEL, true>(M, R.y, h, P.inv_tol, y5, err, &slow);
      if (__builtin_expect(slow, 0)) trial_strat<MODEL>(M, R.y, h, P.inv_tol, y5, err);
    } else {
      trial_strat<MODEL>(medium_of(P, R.region), R.y, h, P.inv_tol, y5, err);
    }
  }
}

// ---------------------------------------------------------------------------
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

}  // namespace rt
