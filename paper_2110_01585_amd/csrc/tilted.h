// Device-side moments of the tilted distribution of one pixel difference u
// (Sec. III-C, Eq. (marginal_tilted_un)) for the l1-TV factor exp(-lambda |u|)
// (Eq. (L1_TV)), and the site update that follows from the Gehre-Jin pair
// projection and Eq. (update_qk_x).
//
// Precision: FP32.  In the far tails of the truncated Gaussian components the
// direct formula for the variance cancels catastrophically; there K and r come
// from Laplace's continued fraction of the Mills ratio, whose evaluation only
// adds positive terms.  The expressions are arranged so that the quantities the site update
// needs -- rho = 1 - S_bar/s and delta = m_bar - m -- never come out of a
// difference of nearly equal numbers:
//
//   the tilted density is a mixture of  N(m - lambda s, s) on u > 0  and
//   N(m + lambda s, s) on u < 0, with weights proportional to erfcx(z+) and
//   erfcx(z-), z+- = (lambda s -+ m) / (sigma sqrt 2).  For a component with its
//   cut x = sqrt2 z standard deviations beyond its mean, r = sqrt(2/pi)/erfcx(z)
//   (inverse Mills ratio) and K = r - x give the mean sigma K beyond the cut and
//   the variance s (1 - r K).  Hence
//     rho   = p+ r+ K+ + p- r- K- - p+ p- (K+ + K-)^2,
//     delta = sigma (p+ r+ - p- r-) - lambda s (p+ - p-),
//     E|u|  = sigma (p+ K+ + p- K-).
#pragma once

#include <hip/hip_runtime.h>

#include "ep_tv_internal.h"

namespace eptv {

__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }

struct Tilt {
  float rho;    // 1 - S_bar / s
  float delta;  // m_bar - m
  float eabs;   // E|u| under the tilted distribution
};

// (K, r) of a component whose cut lies x >= kTailX standard deviations beyond
// its mean, by the bottom-up continued fraction K = 1/(x + L),
// L = 2/(x + 3/(x + ...)).  Every step adds positive numbers, so the
// recurrence is stable in FP32 (relative error ~ depth * eps) and, unlike the
// direct formula, never subtracts nearly equal quantities.
__device__ __forceinline__ void tail_cf(float x, float& K, float& r) {
  float t = 0.0f;
#pragma unroll
  for (int n = kTailDepth; n >= 2; --n) t = (float)n * frcp(x + t);
  K = frcp(x + t);
  r = x + K;
}

__device__ __forceinline__ Tilt laplace_tilt(float m, float s, float lam) {
  const float kSqrt2 = 1.41421356237309515f;
  const float kInvSqrt2 = 0.707106781186547573f;
  const float kSqrt2OverPi = 0.797884560802865406f;
  const float sig = __builtin_amdgcn_sqrtf(s);
  const float ls = lam * s;
  const float k = kInvSqrt2 * frcp(sig);
  const float zp = (ls - m) * k;
  const float zm = (ls + m) * k;
  const float exp_ = erfcxf(fabsf(zp));
  const float exm = erfcxf(fabsf(zm));
  // At most one of z+, z- is negative (their sum is sqrt2 lambda sigma >= 0).
  // For z < 0, erfcx(z) = e^{z^2} erfc(z) with erfc(z) = 2 - e^{-z^2} erfcx(|z|);
  // both weights are rescaled by e^{-z^2} so nothing overflows.
  const float zneg = fminf(fminf(zp, zm), 0.0f);
  const float g = __expf(-zneg * zneg);
  float wp, wm, rp, rm;
  if (zp < 0.0f) {
    wp = 2.0f - g * exp_;
    wm = exm * g;
    rp = kSqrt2OverPi * g * frcp(wp);
    rm = kSqrt2OverPi * frcp(exm);
  } else if (zm < 0.0f) {
    wm = 2.0f - g * exm;
    wp = exp_ * g;
    rm = kSqrt2OverPi * g * frcp(wm);
    rp = kSqrt2OverPi * frcp(exp_);
  } else {
    wp = exp_;
    wm = exm;
    rp = kSqrt2OverPi * frcp(exp_);
    rm = kSqrt2OverPi * frcp(exm);
  }
  const float inv = frcp(wp + wm);
  const float pp = wp * inv;
  const float pm = wm * inv;
  const float xp = kSqrt2 * zp;
  const float xm = kSqrt2 * zm;
  float Kp = rp - xp;
  float Km = rm - xm;
  if (xp >= kTailX || xm >= kTailX) {
    if (xp >= kTailX) tail_cf(xp, Kp, rp);
    if (xm >= kTailX) tail_cf(xm, Km, rm);
  }
  Tilt T;
  const float Ks = Kp + Km;
  T.rho = pp * rp * Kp + pm * rm * Km - pp * pm * Ks * Ks;
  T.delta = sig * (pp * rp - pm * rm) - ls * (pp - pm);
  T.eabs = sig * (pp * Kp + pm * Km);
  return T;
}

}  // namespace eptv
