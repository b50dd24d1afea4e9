// Device-side moments of the tilted distribution of one pixel difference u
// (Sec. III-C, Eq. (marginal_tilted_un)) for the l1-TV factor exp(-lambda |u|)
// (Eq. (L1_TV)), and the site update that follows from the Gehre-Jin pair
// projection and Eq. (update_qk_x).
//
// Precision: FP32, with no branch on the argument.  For a truncated Gaussian
// component whose cut lies x >= 0 standard deviations beyond its mean, every
// moment follows from K(x) = r(x) - x, r = sqrt(2/pi) / erfcx(x / sqrt2) the
// inverse Mills ratio: the mean lies sigma K beyond the cut and the variance is
// s (1 - r K).  K comes from one polynomial (below) valid on the whole half line,
// and r = x + K only adds positive numbers, so nothing cancels in the far tail:
//
//   the tilted density is a mixture of  N(m - lambda s, s) on u > 0  and
//   N(m + lambda s, s) on u < 0, with weights proportional to erfcx(z+) and
//   erfcx(z-), z+- = (lambda s -+ m) / (sigma sqrt 2).  Hence
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
  float dels;   // delta / s
  float eabs;   // E|u| under the tilted distribution
  float omr;    // S_bar / s = 1 - rho, formed without the subtraction (mixture factors)
};

// K(x) = t G(s) with z = x / sqrt2, t = 2 / (2 + z), s = 2 t - 1: G is a
// degree-12 polynomial in s fitted for minimum maximum relative error against K
// at 50 digits (fit_mills.py in this directory writes the table); the fit error
// is 3e-8, the FP32 Horner evaluation at an exact t stays within 1.2e-7 of K,
// and the whole evaluation in FP32 from x (rounded z and t included) within
// 2.3e-7, for every x >= 0, the x -> inf limit K ~ 1/x included.
constexpr float kMillsPoly[13] = {
    5.913686752e-01f,
    2.712919712e-01f,
    -1.626213081e-02f,
    -6.369908899e-02f,
    1.618392300e-03f,
    1.930276118e-02f,
    -1.965504140e-03f,
    -6.114535499e-03f,
    1.438202569e-03f,
    1.636359608e-03f,
    -5.852500326e-04f,
    -2.518910915e-04f,
    1.065924080e-04f};

// (K, r) at a cut x = sqrt2 z >= 0 standard deviations beyond the mean.
__device__ __forceinline__ void mills(float z, float x, float& K, float& r) {
  const float t = 2.0f * frcp(2.0f + z);
  const float s = 2.0f * t - 1.0f;
  float G = kMillsPoly[12];
#pragma unroll
  for (int k = 11; k >= 0; --k) G = __builtin_fmaf(G, s, kMillsPoly[k]);
  K = t * G;
  r = x + K;
}

// Contraction into fused multiply-adds is switched off here: fma(a, b, c d)
// is not symmetric under exchanging the two components, and with it the moments
// of -m would not be exactly the mirror image of those of m.  The fused
// multiply-adds written out below take operands that are each either unchanged
// or negated by the exchange (fma(-a, b, -c) = -fma(a, b, c) in
// round-to-nearest), so the mirror stays exact.
__device__ __forceinline__ Tilt laplace_tilt(float m, float s, float lam) {
#pragma clang fp contract(off)
  const float kSqrt2 = 1.41421356237309515f;
  const float kInvSqrt2 = 0.707106781186547573f;
  const float kSqrt2OverPi = 0.797884560802865406f;
  const float rs = __builtin_amdgcn_rsqf(s);   // 1 / sigma
  const float sig = s * rs;
  const float ls = lam * s;
  const float k = kInvSqrt2 * rs;
  const float zp = (ls - m) * k;
  const float zm = (ls + m) * k;
  const float xp = kSqrt2 * zp;
  const float xm = kSqrt2 * zm;
  // Both components evaluated at |z|: exact for a component with z >= 0.
  float Kp1, rp1, Km1, rm1;
  mills(fabsf(zp), fabsf(xp), Kp1, rp1);
  mills(fabsf(zm), fabsf(xm), Km1, rm1);
  // At most one of z+, z- is negative (their sum is sqrt2 lambda sigma >= 0).
  // For z < 0, erfcx(z) = e^{z^2} erfc(z) with erfc(z) = 2 - e^{-z^2} erfcx(|z|);
  // both weights are rescaled by g = e^{-z^2} so nothing overflows: the negative
  // component weighs wn = 2 - g erfcx(|z|) and has r = sqrt(2/pi) g / wn, the
  // other one weighs g sqrt(2/pi) / r.  Only the ratio of the weights matters,
  // so they are scaled by the positive components' r (no reciprocal when both
  // z are non-negative: weights r-, r+).
  const bool sp = zp < 0.0f, sm = zm < 0.0f;
  const float zneg = fminf(fminf(zp, zm), 0.0f);
  const float g = __expf(-zneg * zneg);
  const float gc = g * kSqrt2OverPi;
  const float wn = __builtin_fmaf(-g, kSqrt2OverPi * frcp(sp ? rp1 : rm1), 2.0f);
  const float rn = gc * frcp(wn);
  const float Wp = sp ? wn * rm1 : (sm ? gc : rm1);
  const float Wm = sm ? wn * rp1 : (sp ? gc : rp1);
  const float inv = frcp(Wp + Wm);
  const float pp = Wp * inv;
  const float pm = Wm * inv;
  const float rp = sp ? rn : rp1;
  const float rm = sm ? rn : rm1;
  const float Kp = sp ? rn - xp : Kp1;
  const float Km = sm ? rn - xm : Km1;
  Tilt T;
  const float Ks = Kp + Km;
  T.rho = __builtin_fmaf(-(pp * pm * Ks), Ks, pp * rp * Kp + pm * rm * Km);
  T.delta = __builtin_fmaf(sig, pp * rp - pm * rm, -(ls * (pp - pm)));
  T.dels = T.delta * (rs * rs);
  T.eabs = sig * (pp * Kp + pm * Km);
  T.omr = 0.f;   // not used for this factor
  return T;
}

// Tilted moments for a two-component Gaussian-mixture factor
// phi(u) = a1 N(u; 0, v1) + a2 N(u; 0, v2): MoG2-TV (Eq. (MoG2_TV_prior)) and
// BG-TV (Eq. (BG_TV), v2 = 0 for the point mass).  Each product with the cavity
// N(u; m, s) is N(m; 0, t_k) N(u; mu_k, sigma_k^2), t_k = s + v_k, with
// mu_k - m = -m s / t_k and sigma_k^2 = s v_k / t_k; the weights follow from
// log(w2 / w1) = log(a2 / a1) + log(t1 / t2) / 2 - m^2 (v1 - v2) / (2 t1 t2),
// in which no two large numbers are subtracted.  With i_k = 1 / t_k:
//   delta = m_bar - m = -m s (w1 i1 + w2 i2),
//   rho = 1 - S_bar / s = s (w1 i1 + w2 i2) - w1 w2 m^2 s (i2 - i1)^2,
//   S_bar / s = w1 v1 i1 + w2 v2 i2 + w1 w2 m^2 s (i2 - i1)^2,
// the last term being the spread of the component means (law of total
// variance).  S_bar / s is a sum of non-negative terms; the site update takes
// it where it needs 1 - rho (a point mass or a narrow component can make rho
// come within rounding of 1).  Only m^2 and m times an even function of m enter, so the moments
// of -m mirror those of m exactly.  E|u| is not formed: it serves only the
// EM of the l1 factor.
struct MixFactor {
  float dla;   // log(a2 / a1)
  float dv;    // v1 - v2
  float v1, v2;
};

__device__ __forceinline__ Tilt mixture_tilt(float m, float s, const MixFactor& F) {
  const float t1 = s + F.v1, t2 = s + F.v2;
  const float i1 = frcp(t1), i2 = frcp(t2);
  const float m2 = m * m;
  const float di = F.dv * i1 * i2;                       // i2 - i1
  const float d = F.dla + 0.5f * __logf(t1 * i2) - 0.5f * m2 * di;
  const float g = __expf(-fabsf(d));
  const float whi = frcp(1.0f + g), wlo = g * whi;
  const float w1 = d > 0.f ? wlo : whi;
  const float w2 = d > 0.f ? whi : wlo;
  const float wi = w1 * i1 + w2 * i2;
  Tilt T;
  const float spread = (w1 * w2) * (m2 * s) * (di * di);
  T.delta = -(m * (s * wi));
  T.dels = -(m * wi);
  T.rho = s * wi - spread;
  T.omr = w1 * (F.v1 * i1) + w2 * (F.v2 * i2) + spread;
  T.eabs = 0.f;
  return T;
}

// The factor kinds as types, so the sweep is compiled once per kind.
// den(T, s, c_own, c_other) is s - rho c_own = c_other + (1 - rho) c_own, the
// denominator of the site precision rho / (s - rho c_own) of Eq. (update_qk_x).
struct L1Factor {
  float lam;
  __device__ __forceinline__ Tilt tilt(float m, float s) const { return laplace_tilt(m, s, lam); }
  __device__ __forceinline__ float den(const Tilt& T, float s, float c_own, float) const {
    return __builtin_fmaf(-T.rho, c_own, s);
  }
};
// The l1 factor with the EM sum of option 2 of Sec. IV in place of option 3:
// eabs is E|u| under Q(u_n) = N(m_bar, S_bar), the Gaussian with the tilted
// moments (a folded-normal mean), instead of the tilted E|u| itself.
struct L1FactorQu {
  float lam;
  __device__ __forceinline__ Tilt tilt(float m, float s) const {
    Tilt T = laplace_tilt(m, s, lam);
    const float mb = fabsf(m + T.delta);
    const float Sb = fmaxf(s * (1.0f - T.rho), 0.0f);
    const float sd = __builtin_amdgcn_sqrtf(Sb);
    const float kSqrt2OverPi = 0.797884560802865406f;
    T.eabs = Sb > 0.0f ? sd * kSqrt2OverPi * __expf(-0.5f * mb * mb / Sb) +
                             mb * erff(mb * 0.707106781186547573f / sd)
                       : mb;
    return T;
  }
  __device__ __forceinline__ float den(const Tilt& T, float s, float c_own, float) const {
    return __builtin_fmaf(-T.rho, c_own, s);
  }
};
struct MixtureFactor {
  MixFactor f;
  __device__ __forceinline__ Tilt tilt(float m, float s) const { return mixture_tilt(m, s, f); }
  __device__ __forceinline__ float den(const Tilt& T, float, float c_own, float c_other) const {
    return __builtin_fmaf(T.omr, c_own, c_other);
  }
};

}  // namespace eptv
