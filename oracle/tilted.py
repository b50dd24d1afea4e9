"""Moments of the 1-D tilted distribution of one pixel difference u (FP64).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Sec. III-C, Eq. (marginal_tilted_un): for an edge (i, j) of colour class k the
tilted marginal of u = x_i - x_j is

    P_k(u) ~ N(u; m, s) * phi(u; theta),   m = m_i - m_j,  s = c_i + c_j,

where (m_p, c_p) are the cavity mean and variance of pixel p.  The paper omits
the prior-specific expressions; they are derived here.

l1-TV (Eq. (L1_TV)), phi(u) = exp(-lambda |u|).  Completing the square on each
half line gives a two-component mixture of truncated Gaussians,

    u > 0:  N(u; m - lambda s, s) restricted to u > 0,
    u < 0:  N(u; m + lambda s, s) restricted to u < 0,

with weights proportional to erfcx(z+) and erfcx(z-), where
z+ = (lambda s - m) / (sigma sqrt 2), z- = (lambda s + m) / (sigma sqrt 2),
sigma = sqrt(s) (the common factor exp(-m^2 / 2s) / 2 cancels).  For one
component, let x be the distance of the truncation point u = 0 from that
component's mean in units of sigma (x = sqrt2 z).  With the inverse Mills ratio
r = sqrt(2/pi) / erfcx(z) and K = r - x,

    mean distance from 0 = sigma K,   variance = s (1 - r K).

For x >= 3 the variance formula cancels catastrophically, so K and the
variance are taken from Laplace's continued fraction of the Mills ratio,
1/r = 1/(x + K), K = 1/(x + L), L = 2/(x + 3/(x + 4/(x + ...))), which gives
variance = s K (L - K) with no subtraction of nearly equal numbers.

l2 check prior, phi(u) = exp(-beta u^2 / 2) (the MoG2-TV prior of Eq.
(MoG2_TV_prior) with s1 = s2 = 1/beta, up to a constant): the tilted density is
Gaussian with precision 1/s + beta.

Gaussian-mixture priors, phi(u) = sum_k a_k N(u; 0, v_k): MoG2-TV (Eq.
(MoG2_TV_prior)), a = (omega, 1 - omega), v = (s1^2, s2^2); BG-TV (Eq. (BG_TV)),
a = (omega, 1 - omega), v = (s^2, 0), the point mass delta(u) being the v -> 0
limit of N(u; 0, v).  Each product N(u; m, s) N(u; 0, v_k) is the Gaussian
N(m; 0, s + v_k) N(u; mu_k, sigma_k^2) with sigma_k^2 = s v_k / (s + v_k) and
mu_k = m v_k / (s + v_k), so the tilted distribution is the mixture of those
Gaussians with weights w_k proportional to a_k N(m; 0, s + v_k): its mean is
sum_k w_k mu_k and its variance sum_k w_k sigma_k^2 + sum_k w_k (mu_k - mean)^2.

Parity pins: tests/test_oracle_tilted.py checks every branch against adaptive
quadrature and mpmath at 50 digits, plus the lambda -> 0, m = 0 and Laplace
limits.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erfc, erfcx, expit

SQRT2 = math.sqrt(2.0)
SQRT_2_OVER_PI = math.sqrt(2.0 / math.pi)
TAIL_X = 3.0          # switch to the continued fraction at x >= TAIL_X
TAIL_DEPTH = 100      # continued-fraction depth (converged to < 1e-15 for x >= 3)


def log_erfcx(z):
    """log erfcx(z) for any real z.  For z < 0, erfcx(z) = exp(z^2) erfc(z) with
    erfc(z) in (1, 2], so the log stays finite where erfcx overflows."""
    z = np.asarray(z, dtype=np.float64)
    out = np.empty_like(z)
    pos = z >= 0.0
    out[pos] = np.log(erfcx(z[pos]))
    zn = z[~pos]
    out[~pos] = zn * zn + np.log(erfc(zn))
    return out


def _tail_cf(x, depth=TAIL_DEPTH):
    """(K, L) of Laplace's continued fraction at x > 0, evaluated bottom-up."""
    t = np.zeros_like(x)
    for n in range(depth, 1, -1):
        t = n / (x + t)
    L = t
    K = 1.0 / (x + L)
    return K, L


def truncated_component(x):
    """For a Gaussian truncated at x standard deviations above its mean (kept
    side beyond the cut), return (K, W): the mean distance beyond the cut in
    units of sigma, and the variance in units of s."""
    x = np.asarray(x, dtype=np.float64)
    K = np.empty_like(x)
    W = np.empty_like(x)
    tail = x >= TAIL_X
    xd = x[~tail]
    r = SQRT_2_OVER_PI * np.exp(-log_erfcx(xd / SQRT2))
    K[~tail] = r - xd
    W[~tail] = 1.0 - r * (r - xd)
    if np.any(tail):
        Kt, Lt = _tail_cf(x[tail])
        K[tail] = Kt
        W[tail] = Kt * (Lt - Kt)
    return K, W


def laplace_tilted(m, s, lam):
    """Mean, variance and E|u| of P(u) ~ N(u; m, s) exp(-lam |u|).

    m, s broadcast; s > 0, lam >= 0.  Returns (m_bar, S_bar, E_abs)."""
    m = np.asarray(m, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    m, s = np.broadcast_arrays(m, s)
    lam = np.broadcast_to(np.asarray(lam, dtype=np.float64), m.shape)
    sig = np.sqrt(s)
    zp = (lam * s - m) / (sig * SQRT2)
    zm = (lam * s + m) / (sig * SQRT2)
    # mixture weights p+ = erfcx(z+) / (erfcx(z+) + erfcx(z-)), in the log domain
    pp = expit(log_erfcx(zp) - log_erfcx(zm))
    pm = expit(log_erfcx(zm) - log_erfcx(zp))
    Kp, Wp = truncated_component(SQRT2 * zp)
    Km, Wm = truncated_component(SQRT2 * zm)
    Ep = sig * Kp            # positive component mean
    Em = -sig * Km           # negative component mean
    Vp = s * Wp
    Vm = s * Wm
    m_bar = pp * Ep + pm * Em
    S_bar = pp * Vp + pm * Vm + pp * pm * (Ep - Em) ** 2
    E_abs = pp * Ep - pm * Em
    return m_bar, S_bar, E_abs


def gauss_tilted(m, s, beta):
    """Mean and variance of P(u) ~ N(u; m, s) exp(-beta u^2 / 2); E|u| of it."""
    m = np.asarray(m, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    prec = 1.0 / s + beta
    v = 1.0 / prec
    mu = v * (m / s)
    sd = np.sqrt(v)
    # E|u| of N(mu, v): sd sqrt(2/pi) exp(-mu^2/2v) + mu (1 - 2 Phi(-mu/sd))
    e_abs = sd * SQRT_2_OVER_PI * np.exp(-mu * mu / (2.0 * v)) + mu * (1.0 - erfc(mu / (sd * SQRT2)))
    return mu, v, e_abs


def mixture_tilted(m, s, a, v):
    """Mean, variance and E|u| of P(u) ~ N(u; m, s) sum_k a[k] N(u; 0, v[k]),
    a[k] >= 0, v[k] >= 0 (v[k] = 0: a point mass at 0)."""
    m = np.asarray(m, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    comps = []
    for ak, vk in zip(a, v):
        t = s + vk
        with np.errstate(divide="ignore"):
            logw = np.log(ak) - 0.5 * np.log(2.0 * math.pi * t) - m * m / (2.0 * t)
        comps.append((logw, s * vk / t, m * vk / t))
    top = np.max([c[0] for c in comps], axis=0)
    ws = [np.exp(c[0] - top) for c in comps]
    tot = np.sum(ws, axis=0)
    ws = [w / tot for w in ws]
    mean = np.sum([w * c[2] for w, c in zip(ws, comps)], axis=0)
    var = np.sum([w * (c[1] + (c[2] - mean) ** 2) for w, c in zip(ws, comps)], axis=0)
    e_abs = 0.0
    for w, (_, vk, mk) in zip(ws, comps):
        sd = np.sqrt(vk)
        with np.errstate(divide="ignore", invalid="ignore"):
            fold = np.where(sd > 0.0, sd * SQRT_2_OVER_PI * np.exp(-mk * mk / (2.0 * np.where(vk > 0, vk, 1.0)))
                            + mk * (1.0 - erfc(mk / (np.where(sd > 0, sd, 1.0) * SQRT2))), np.abs(mk))
        e_abs = e_abs + w * fold
    return mean, var, e_abs


def mog2_tilted(m, s, theta):
    """MoG2-TV (Eq. (MoG2_TV_prior)), theta = (omega, s1^2, s2^2)."""
    omega, v1, v2 = theta
    return mixture_tilted(m, s, (omega, 1.0 - omega), (v1, v2))


def bg_tilted(m, s, theta):
    """BG-TV (Eq. (BG_TV)), theta = (omega, s^2)."""
    omega, v = theta
    return mixture_tilted(m, s, (omega, 1.0 - omega), (v, 0.0))


def folded_normal_mean(m, var):
    """E|d| for d ~ N(m, var): m erf(m / sqrt(2 var)) + sqrt(2 var / pi) exp(-m^2 / (2 var))."""
    m = np.asarray(m, np.float64)
    var = np.asarray(var, np.float64)
    sd = np.sqrt(var)
    erf = np.vectorize(math.erf, otypes=[np.float64])
    return m * erf(m / (sd * math.sqrt(2.0))) + sd * math.sqrt(2.0 / math.pi) * np.exp(-m * m / (2 * var))


def tilted(prior, m, s, theta):
    if prior == "l1":
        return laplace_tilted(m, s, theta)
    if prior == "l2":
        return gauss_tilted(m, s, theta)
    if prior == "mog2":
        return mog2_tilted(m, s, theta)
    if prior == "bg":
        return bg_tilted(m, s, theta)
    raise ValueError(f"unknown prior {prior!r}")
