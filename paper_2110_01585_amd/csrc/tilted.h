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
// its mean, from Laplace's continued fraction K = 1/(x + L),
// L = 2/(x + 3/(x + 4/(x + ...))), truncated at depth kTailDepth.  L is
// evaluated forwards as a ratio A/B of the fraction's convergents, scaled by
// x^-j so that they stay O(1): with u = 1/x,
//   A_j = A_{j-1} + (j+1) u^2 A_{j-2},  B_j = B_{j-1} + (j+1) u^2 B_{j-2},
//   A_0 = 0, B_0 = 1, A_1 = 2u, B_1 = 1.
// Every term is positive (no cancellation, as in the bottom-up evaluation) and
// the whole tail costs two reciprocals.
__device__ __forceinline__ void tail_cf(float x, float& K, float& r) {
  const float u = frcp(x);
  const float u2 = u * u;
  float A2 = 0.0f, B2 = 1.0f, A1 = 2.0f * u, B1 = 1.0f;
#pragma unroll
  for (int j = 2; j < kTailDepth; ++j) {
    const float a = (float)(j + 1) * u2;
    const float A0 = A1 + a * A2, B0 = B1 + a * B2;
    A2 = A1; B2 = B1; A1 = A0; B1 = B0;
  }
  K = frcp(x + A1 * frcp(B1));
  r = x + K;
}

// Contraction into fused multiply-adds is switched off here: fma(a, b, c d)
// is not symmetric under exchanging the two components, and with it the moments
// of -m would not be exactly the mirror image of those of m.
__device__ __forceinline__ Tilt laplace_tilt(float m, float s, float lam) {
#pragma clang fp contract(off)
  const float kSqrt2 = 1.41421356237309515f;
  const float kInvSqrt2 = 0.707106781186547573f;
  const float kSqrt2OverPi = 0.797884560802865406f;
  const float sig = __builtin_amdgcn_sqrtf(s);
  const float ls = lam * s;
  const float k = kInvSqrt2 * frcp(sig);
  const float zp = (ls - m) * k;
  const float zm = (ls + m) * k;
  const float xp = kSqrt2 * zp;
  const float xm = kSqrt2 * zm;
  // A component in the far tail takes K, r and its weight erfcx(z) = sqrt(2/pi)/r
  // from the continued fraction; the others call erfcx.
  const bool tp = xp >= kTailX, tm = xm >= kTailX;
  float Kpt = 0.0f, rpt = 1.0f, Kmt = 0.0f, rmt = 1.0f;
  float exp_, exm;
  if (tp) {
    tail_cf(xp, Kpt, rpt);
    exp_ = kSqrt2OverPi * frcp(rpt);
  } else {
    exp_ = erfcxf(fabsf(zp));
  }
  if (tm) {
    tail_cf(xm, Kmt, rmt);
    exm = kSqrt2OverPi * frcp(rmt);
  } else {
    exm = erfcxf(fabsf(zm));
  }
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
  float Kp = rp - xp;
  float Km = rm - xm;
  if (tp) { Kp = Kpt; rp = rpt; }
  if (tm) { Km = Kmt; rm = rmt; }
  Tilt T;
  const float Ks = Kp + Km;
  T.rho = pp * rp * Kp + pm * rm * Km - pp * pm * Ks * Ks;
  T.delta = sig * (pp * rp - pm * rm) - ls * (pp - pm);
  T.eabs = sig * (pp * Kp + pm * Km);
  return T;
}

}  // namespace eptv
