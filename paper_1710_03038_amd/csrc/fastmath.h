// Single-precision elementary functions for the bounded arguments of the
// sweep kernel (|x| < 8*pi), written for gfx950 VALU throughput.
//
// sin/cos: Cody-Waite reduction by pi/2 with a two-part constant
// (W. J. Cody and W. Waite, Software Manual for the Elementary Functions,
// 1980), then the Taylor polynomials of sin (to r^9) and cos (to r^8) on
// |r| <= pi/4, whose truncation errors (< 2.5e-8 relative) are below FP32
// rounding.  atan: for t in [0, 1], atan(t) = t * P(t^2) with P of degree 8,
// fitted for minimum relative error by fit_atan.py next to this file (least
// squares on Chebyshev nodes with Lawson reweighting); the float32
// coefficients give at most 2.0e-8 relative error evaluated in float64 and
// about 1.2e-7 evaluated in FP32; atan2 follows by octant symmetry.
// exp: the hardware base-2 exponential; sin_hw: the hardware sine.
#pragma once

#include <hip/hip_runtime.h>

namespace mpr {
namespace fm {

constexpr float kTwoOverPi = 0.636619772367581343f;
constexpr float kPio2Hi = 1.57079637050628662f;     // float(pi/2)
constexpr float kPio2Lo = -4.37113900018624283e-8f;  // pi/2 - kPio2Hi
constexpr float kPi = 3.14159274101257324f;           // float(pi)
constexpr float kLog2e = 1.44269504088896341f;

__device__ __forceinline__ float sin_poly(float r, float r2) {
  const float p = fmaf(fmaf(fmaf(2.75573192e-06f, r2, -1.98412698e-04f), r2, 8.33333333e-03f), r2, -1.66666667e-01f);
  return fmaf(r * r2, p, r);
}
__device__ __forceinline__ float cos_poly(float r2) {
  const float p = fmaf(fmaf(fmaf(2.48015873e-05f, r2, -1.38888889e-03f), r2, 4.16666667e-02f), r2, -0.5f);
  return fmaf(r2, p, 1.0f);
}

// x = k*pi/2 + r with |r| <= pi/4 (for |x| well below 2^20).
__device__ __forceinline__ float reduce(float x, int &quadrant) {
  const float k = __builtin_rintf(x * kTwoOverPi);
  float r = fmaf(-k, kPio2Hi, x);
  r = fmaf(-k, kPio2Lo, r);
  quadrant = (int)k & 3;
  return r;
}

__device__ __forceinline__ void sincos(float x, float *s, float *c) {
  int q;
  const float r = reduce(x, q);
  const float r2 = r * r;
  const float sp = sin_poly(r, r2), cp = cos_poly(r2);
  float sv = (q & 1) ? cp : sp;
  float cv = (q & 1) ? sp : cp;
  sv = (q & 2) ? -sv : sv;
  cv = ((q + 1) & 2) ? -cv : cv;
  *s = sv;
  *c = cv;
}

// sin and cos of x in [0, pi] (q*phi with q <= 1/2): r = x - pi/2 in
// [-pi/2, pi/2], sin x = cos r and cos x = -sin r, with the Taylor
// polynomials of sin r to r^13 and cos r to r^12 (truncation below 1e-8).
__device__ __forceinline__ void sincos_0pi(float x, float *s, float *c) {
  float r = x - kPio2Hi;
  r = r - kPio2Lo;
  const float r2 = r * r;
  float ps = fmaf(fmaf(fmaf(-1.60590438e-10f, r2, 2.50521084e-08f), r2, -2.75573192e-06f), r2, 1.98412698e-04f);
  ps = fmaf(fmaf(ps, r2, -8.33333333e-03f), r2, 1.66666667e-01f);
  const float sr = fmaf(-r * r2, ps, r);  // sin r = r - r^3/6 + ...
  float pc = fmaf(fmaf(fmaf(2.08767570e-09f, r2, -2.75573192e-07f), r2, 2.48015873e-05f), r2, -1.38888889e-03f);
  pc = fmaf(fmaf(pc, r2, 4.16666667e-02f), r2, -0.5f);
  const float cr = fmaf(pc, r2, 1.0f);
  *s = cr;
  *c = -sr;
}

__device__ __forceinline__ float sin(float x) {
  int q;
  const float r = reduce(x, q);
  const float r2 = r * r;
  const float sp = sin_poly(r, r2), cp = cos_poly(r2);  // both, then select: no divergent branch
  const float v = (q & 1) ? cp : sp;
  return (q & 2) ? -v : v;
}

// atan2(y, x) for (x, y) != (0, 0).
__device__ __forceinline__ float atan2(float y, float x) {
  const float ax = fabsf(x), ay = fabsf(y);
  const float mx = fmaxf(ax, ay), mn = fminf(ax, ay);
  const float t = mn * __builtin_amdgcn_rcpf(mx);
  const float s = t * t;
  float p = 2.92068860e-03f;
  p = fmaf(p, s, -1.63679142e-02f);
  p = fmaf(p, s, 4.32118364e-02f);
  p = fmaf(p, s, -7.55221248e-02f);
  p = fmaf(p, s, 1.06660038e-01f);
  p = fmaf(p, s, -1.42110556e-01f);
  p = fmaf(p, s, 1.99937731e-01f);
  p = fmaf(p, s, -3.33331525e-01f);
  p = fmaf(p, s, 1.0f);
  float r = t * p;
  r = (ay > ax) ? kPio2Hi - r : r;
  r = (x < 0.0f) ? kPi - r : r;
  return copysignf(r, y);
}

// sin through the hardware unit, which takes its argument in revolutions;
// about 1e-6 relative error (measured on gfx950), used where only a
// Metropolis decision depends on the value.
__device__ __forceinline__ float sin_hw(float x) { return __builtin_amdgcn_sinf(x * 0.159154943091895336f); }

__device__ __forceinline__ float exp(float x) { return __builtin_amdgcn_exp2f(x * kLog2e); }

__device__ __forceinline__ float sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

}  // namespace fm
}  // namespace mpr
