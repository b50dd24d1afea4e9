"""Pins for oracle/tilted.py: Laplace x Gaussian tilted moments.

The reference values come from the definition of the tilted density
P(u) ~ N(u; m, s) exp(-lambda |u|) (Sec. III-C, Eq. (marginal_tilted_un) with
the l1-TV factor of Eq. (L1_TV)), integrated numerically: scipy adaptive
quadrature split at the kink u = 0 and at the component modes, and mpmath at
50 digits.  None of them shares a formula with the closed form under test.
"""
import math

import mpmath as mp
import numpy as np
import pytest
from scipy import integrate

from oracle import tilted as T


def _quad_moments(m, s, lam):
    """Moments of P(u) by scipy.integrate.quad, each half line separately."""
    sig = math.sqrt(s)
    # log-density up to a constant, shifted by its maximum for stability
    def logf(u):
        return -(u - m) ** 2 / (2 * s) - lam * abs(u)
    lo_mode = m + lam * s          # mode of the negative component if < 0
    hi_mode = m - lam * s
    cands = [logf(0.0)]
    if hi_mode > 0:
        cands.append(logf(hi_mode))
    if lo_mode < 0:
        cands.append(logf(lo_mode))
    shift = max(cands)
    res = []
    for k in range(3):
        tot = 0.0
        for a, b, mode in ((-np.inf, 0.0, lo_mode), (0.0, np.inf, hi_mode)):
            pts = []
            f = (lambda u, k=k: (u ** k) * math.exp(logf(u) - shift))
            # split finite ranges around the mode to help quad
            if a == -np.inf:
                c = min(mode, 0.0) - 40 * sig
                v1, _ = integrate.quad(f, c, 0.0, limit=400, epsabs=0, epsrel=1e-13,
                                       points=[p for p in (mode,) if c < p < 0.0] or None)
                v2, _ = integrate.quad(f, -np.inf, c, limit=200, epsabs=0, epsrel=1e-13)
            else:
                c = max(mode, 0.0) + 40 * sig
                v1, _ = integrate.quad(f, 0.0, c, limit=400, epsabs=0, epsrel=1e-13,
                                       points=[p for p in (mode,) if 0.0 < p < c] or None)
                v2, _ = integrate.quad(f, c, np.inf, limit=200, epsabs=0, epsrel=1e-13)
            tot += v1 + v2
        res.append(tot)
    z0, z1, z2 = res
    mean = z1 / z0
    var = z2 / z0 - mean * mean
    # E|u|
    def fa(u):
        return abs(u) * math.exp(logf(u) - shift)
    ea = 0.0
    for a, b, mode in ((-np.inf, 0.0, lo_mode), (0.0, np.inf, hi_mode)):
        ea += integrate.quad(fa, a, b, limit=400, epsabs=0, epsrel=1e-13)[0]
    return mean, var, ea / z0


def _mp_moments(m, s, lam, dps=50):
    """Same moments with mpmath at `dps` digits; variance by central moment."""
    with mp.workdps(dps):
        m = mp.mpf(m); s = mp.mpf(s); lam = mp.mpf(lam)
        logf = lambda u: -(u - m) ** 2 / (2 * s) - lam * abs(u)
        lo_mode = m + lam * s
        hi_mode = m - lam * s
        shift = max(logf(mp.mpf(0)), logf(hi_mode) if hi_mode > 0 else -mp.inf,
                    logf(lo_mode) if lo_mode < 0 else -mp.inf)
        f = lambda u: mp.exp(logf(u) - shift)
        sig = mp.sqrt(s)
        negpts = [-mp.inf] + ([lo_mode] if lo_mode < 0 else []) + [mp.mpf(0)]
        pospts = [mp.mpf(0)] + ([hi_mode] if hi_mode > 0 else []) + [mp.inf]
        Z = mp.quad(f, negpts) + mp.quad(f, pospts)
        M1 = (mp.quad(lambda u: u * f(u), negpts) + mp.quad(lambda u: u * f(u), pospts)) / Z
        V = (mp.quad(lambda u: (u - M1) ** 2 * f(u), negpts)
             + mp.quad(lambda u: (u - M1) ** 2 * f(u), pospts)) / Z
        EA = (mp.quad(lambda u: -u * f(u), negpts) + mp.quad(lambda u: u * f(u), pospts)) / Z
        return float(M1), float(V), float(EA)


GRID = [(mr, ls) for mr in (-60.0, -20.0, -5.0, -1.3, -0.2, 0.0, 0.4, 2.0, 7.5, 30.0, 60.0)
        for ls in (1e-3, 0.05, 0.7, 2.5, 9.0, 40.0, 1e3)]


@pytest.mark.parametrize("m_over_sig,lam_sig", GRID)
def test_laplace_tilted_vs_quad(m_over_sig, lam_sig):
    s = 0.37 ** 2
    sig = math.sqrt(s)
    m = m_over_sig * sig
    lam = lam_sig / sig
    mb, Sb, Ea = T.laplace_tilted(np.array([m]), np.array([s]), lam)
    qm, qv, qa = _quad_moments(m, s, lam)
    # relative to the natural scales of each quantity
    assert abs(mb[0] - qm) <= 1e-10 * max(sig, abs(qm)), (mb[0], qm)
    assert abs(Sb[0] - qv) <= 1e-10 * qv * max(1.0, (qm * qm) / qv * 1e-3) + 1e-14 * s, (Sb[0], qv)
    assert abs(Ea[0] - qa) <= 1e-10 * max(sig, qa), (Ea[0], qa)


MP_POINTS = [(0.0, 0.7), (1.1, 0.05), (-3.0, 4.0), (12.0, 1.0), (0.5, 30.0), (-45.0, 2.0),
             (2.0, 300.0), (0.0, 1e-3), (8.0, 8.0), (-0.3, 6.5)]


@pytest.mark.parametrize("m_over_sig,lam_sig", MP_POINTS)
def test_laplace_tilted_vs_mpmath(m_over_sig, lam_sig):
    s = 2.3
    sig = math.sqrt(s)
    m = m_over_sig * sig
    lam = lam_sig / sig
    mb, Sb, Ea = T.laplace_tilted(np.array([m]), np.array([s]), lam)
    rm, rv, ra = _mp_moments(m, s, lam)
    assert abs(mb[0] - rm) <= 1e-12 * max(sig, abs(rm))
    assert abs(Sb[0] / rv - 1.0) <= 1e-10
    assert abs(Ea[0] - ra) <= 1e-12 * max(sig, ra)


@pytest.mark.parametrize("x", [3.0, 3.5, 5.0, 10.0, 50.0, 1000.0, 1e5])
def test_tail_branch_vs_mpmath(x):
    """Truncated standard normal beyond x: mean distance K and variance W."""
    K, W = T.truncated_component(np.array([x]))
    with mp.workdps(60):
        X = mp.mpf(x)
        Q = mp.erfc(X / mp.sqrt(2)) / 2
        phi = mp.exp(-X * X / 2) / mp.sqrt(2 * mp.pi)
        r = phi / Q
        Kt = r - X
        Wt = 1 - r * (r - X)
    assert abs(K[0] / float(Kt) - 1) <= 1e-14
    assert abs(W[0] / float(Wt) - 1) <= 1e-13


@pytest.mark.parametrize("x", [-30.0, -4.0, -1.0, 0.0, 0.5, 2.0, 2.99])
def test_direct_branch_vs_mpmath(x):
    K, W = T.truncated_component(np.array([x]))
    with mp.workdps(60):
        X = mp.mpf(x)
        Q = mp.erfc(X / mp.sqrt(2)) / 2
        phi = mp.exp(-X * X / 2) / mp.sqrt(2 * mp.pi)
        r = phi / Q
        Kt = r - X
        Wt = 1 - r * (r - X)
    assert abs(K[0] - float(Kt)) <= 1e-13 * max(1.0, abs(float(Kt)))
    assert abs(W[0] / float(Wt) - 1) <= 1e-12


def test_limits():
    # lambda -> 0: the tilted distribution is the cavity Gaussian N(m, s)
    m = np.array([-1.0, 0.0, 0.3, 2.0]); s = np.array([0.5, 0.2, 1.0, 0.1])
    mb, Sb, _ = T.laplace_tilted(m, s, 0.0)
    assert np.allclose(mb, m, rtol=0, atol=1e-14)
    assert np.allclose(Sb, s, rtol=1e-13)
    # m = 0: symmetric, zero mean
    mb, Sb, Ea = T.laplace_tilted(np.zeros(3), np.array([0.1, 1.0, 10.0]), 3.0)
    assert np.all(np.abs(mb) <= 1e-15)
    # s -> infinity with m = 0: Laplace(lambda): variance 2/lambda^2, E|u| = 1/lambda
    lam = 2.0
    mb, Sb, Ea = T.laplace_tilted(np.array([0.0]), np.array([1e12]), lam)
    assert abs(Sb[0] / (2 / lam ** 2) - 1) < 1e-5
    assert abs(Ea[0] * lam - 1) < 1e-5
    # odd symmetry in m
    mb1, Sb1, Ea1 = T.laplace_tilted(np.array([0.7]), np.array([0.3]), 1.5)
    mb2, Sb2, Ea2 = T.laplace_tilted(np.array([-0.7]), np.array([0.3]), 1.5)
    assert mb1[0] == -mb2[0] and Sb1[0] == Sb2[0] and Ea1[0] == Ea2[0]


def test_variance_reduction_log_concave():
    """A log-concave tilt never increases the variance: S_bar <= s (so the TV
    site precision is never negative in exact arithmetic)."""
    rng = np.random.default_rng(5)
    m = rng.normal(0, 3, 2000); s = rng.uniform(0.01, 4, 2000); lam = rng.uniform(0, 20, 2000)
    _, Sb, _ = T.laplace_tilted(m, s, lam)
    assert np.all(Sb <= s * (1 + 1e-12))


def test_gauss_tilted_is_product_of_gaussians():
    m, s, beta = 0.8, 0.25, 3.0
    mu, v, ea = T.gauss_tilted(np.array([m]), np.array([s]), beta)
    # product of N(u; m, s) and N(u; 0, 1/beta): precision-weighted
    assert abs(v[0] - 1 / (1 / s + beta)) < 1e-15
    assert abs(mu[0] - (m / s) / (1 / s + beta)) < 1e-15
    # E|u| against quadrature
    f = lambda u: abs(u) * math.exp(-(u - mu[0]) ** 2 / (2 * v[0])) / math.sqrt(2 * math.pi * v[0])
    q = integrate.quad(f, -np.inf, 0)[0] + integrate.quad(f, 0, np.inf)[0]
    assert abs(ea[0] - q) < 1e-12


# ---- Gaussian-mixture priors: MoG2-TV (Eq. (MoG2_TV_prior)) and BG-TV (Eq. (BG_TV)) ----

def _mix_quad(m, s, a, v):
    """Mean and variance of N(u; m, s) sum_k a_k N(u; 0, v_k) by adaptive
    quadrature (all v_k > 0), with break points at 0 and the component means."""
    def dens(u):
        g = math.exp(-(u - m) ** 2 / (2 * s)) / math.sqrt(2 * math.pi * s)
        return g * sum(ak * math.exp(-u * u / (2 * vk)) / math.sqrt(2 * math.pi * vk) for ak, vk in zip(a, v))
    sd = math.sqrt(s)
    lo, hi = min(m, 0.0) - 40 * sd, max(m, 0.0) + 40 * sd
    pts = sorted({0.0, m} | {m * vk / (s + vk) for vk in v})
    z = integrate.quad(dens, lo, hi, points=pts, epsabs=0, epsrel=1e-13, limit=400)[0]
    m1 = integrate.quad(lambda u: u * dens(u), lo, hi, points=pts, epsabs=0, epsrel=1e-13, limit=400)[0] / z
    m2 = integrate.quad(lambda u: (u - m1) ** 2 * dens(u), lo, hi, points=pts, epsabs=0, epsrel=1e-13,
                        limit=400)[0] / z
    return m1, m2


@pytest.mark.parametrize("seed", range(8))
def test_mog2_tilted_vs_quad(seed):
    rng = np.random.default_rng(100 + seed)
    s = float(10 ** rng.uniform(-3, 0))
    omega = float(rng.uniform(0.05, 0.95))
    v1 = float(10 ** rng.uniform(-1, 1))          # large gradients (object boundaries)
    v2 = float(10 ** rng.uniform(-4, -2))         # small gradients (flat regions)
    for m in (0.0, 0.3 * math.sqrt(s), -2.0 * math.sqrt(s), 5.0 * math.sqrt(s), 0.7):
        mean, var, _ = T.mog2_tilted(np.array([m]), np.array([s]), (omega, v1, v2))
        qm, qv = _mix_quad(m, s, (omega, 1 - omega), (v1, v2))
        scale = math.sqrt(s)
        assert abs(mean[0] - qm) <= 1e-9 * scale, (m, mean[0], qm)
        assert abs(var[0] / qv - 1) <= 1e-8, (m, var[0], qv)


def test_bg_tilted_is_the_limit_of_mog2():
    """The point mass of BG-TV is the s2 -> 0 limit of the MoG2-TV component."""
    rng = np.random.default_rng(7)
    m = rng.normal(size=50) * 0.5
    s = 10 ** rng.uniform(-3, -1, 50)
    for omega, v in ((0.3, 0.5), (0.9, 2.0), (0.02, 0.1)):
        b = T.bg_tilted(m, s, (omega, v))
        g = T.mog2_tilted(m, s, (omega, v, 1e-13))
        assert np.max(np.abs(b[0] - g[0]) / np.sqrt(s)) <= 1e-5
        assert np.max(np.abs(b[1] - g[1]) / s) <= 1e-5


def test_mixture_special_cases():
    m = np.array([-1.3, -0.2, 0.0, 0.4, 2.5])
    s = np.array([0.04, 0.5, 0.1, 0.01, 0.3])
    # one component, or two equal ones: the Gaussian (l2) prior with beta = 1 / v
    for theta in ((1.0, 0.7, 0.01), (0.35, 0.7, 0.7)):
        mean, var, eabs = T.mog2_tilted(m, s, theta)
        gm, gv, ge = T.gauss_tilted(m, s, 1.0 / 0.7)
        assert np.allclose(mean, gm, rtol=1e-13, atol=1e-15) and np.allclose(var, gv, rtol=1e-13)
        assert np.allclose(eabs, ge, rtol=1e-12)
    # even priors: the moments of -m mirror those of m
    for f, theta in ((T.mog2_tilted, (0.3, 1.0, 0.001)), (T.bg_tilted, (0.3, 1.0))):
        a = f(m, s, theta)
        b = f(-m, s, theta)
        assert np.array_equal(a[0], -b[0]) and np.array_equal(a[1], b[1])
    # BG with (almost) all prior mass on the point mass: u is pinned to 0 (the
    # Gaussian part still gains weight where m is many sigma from 0, so omega
    # must be far below the likelihood ratio exp(-m^2 / 2s) of these draws)
    mean, var, _ = T.bg_tilted(m, s, (1e-30, 1.0))
    assert np.max(np.abs(mean)) <= 1e-9 and np.max(var) <= 1e-9
