"""Fit the polynomial behind the device tilted moments (kMillsPoly in tilted.h).

For one Gaussian component whose truncation point lies x >= 0 standard
deviations beyond its mean, the tilted moments need the inverse Mills ratio
r(x) = sqrt(2/pi) / erfcx(x / sqrt2) and K(x) = r(x) - x, the mean distance of
the truncated component from the cut in units of sigma.  K is positive, equals
sqrt(2/pi) at x = 0 and behaves like 1/x for large x.  With

    z = x / sqrt2,   t = 2 / (2 + z) in (0, 1],   s = 2 t - 1 in (-1, 1],

K = t * G(s) with G smooth on [-1, 1] (G(-1) = 1 / (2 sqrt2), the x -> inf
limit).  The device evaluates G by Horner's rule in FP32 and then forms
r = x + K and erfcx = sqrt(2/pi) / r, which only adds positive numbers, so one
branch-free evaluation covers the whole half line, far tail included.

This script computes K from its definition with mpmath at 50 significant digits,
fits G by a polynomial of degree DEG in s that minimises the maximum relative
error (Lawson's iteration on weighted least squares, Chebyshev basis), rounds
the coefficients to float32 and reports the error of the FP32 Horner
evaluation.  Run from the repository root:

    python paper_2110_01585_amd/csrc/fit_mills.py

It prints the coefficient table as C++ (lowest degree first).
"""
from __future__ import annotations

import mpmath as mp
import numpy as np
from numpy.polynomial import chebyshev as C

DEG = 12
mp.mp.dps = 50


def k_exact(t):
    """K at the point t = 2 / (2 + z) (t in (0, 1]), 50 digits."""
    t = mp.mpf(t)
    z = 2 / t - 2
    x = mp.sqrt(2) * z
    erfcx = mp.exp(z * z) * mp.erfc(z)
    return mp.sqrt(2 / mp.pi) / erfcx - x


def g_exact(t):
    if t == 0.0:
        return 1 / (2 * mp.sqrt(2))
    return k_exact(t) / mp.mpf(t)


def sample(n_uniform, n_cheb):
    tu = np.linspace(0.0, 1.0, n_uniform)
    tc = (1 + np.cos(np.pi * (np.arange(n_cheb) + 0.5) / n_cheb)) / 2
    # the tail end t -> 0 (x -> inf) gets its own geometric grid
    tg = np.geomspace(1e-9, 1e-2, 400)
    return np.unique(np.concatenate([tu, tc, tg]))


def fit(t, g, deg=DEG, iters=40):
    s = 2 * t - 1
    w = 1.0 / g
    for _ in range(iters):
        V = C.chebvander(s, deg) * w[:, None]
        c, *_ = np.linalg.lstsq(V, g * w, rcond=None)
        e = np.abs(C.chebval(s, c) / g - 1)
        w = w * np.maximum(e / e.max(), 1e-3) ** 0.5
        w /= w.max()
    return C.cheb2poly(c)


def horner32(coef, t):
    c32 = coef.astype(np.float32)
    t32 = t.astype(np.float32)
    s32 = np.float32(2) * t32 - np.float32(1)
    acc = np.zeros_like(s32)
    for k in range(len(c32) - 1, -1, -1):
        acc = (acc * s32 + c32[k]).astype(np.float32)
    return acc.astype(np.float64)


def main():
    t = sample(2001, 2000)
    g = np.array([float(g_exact(v)) for v in t])
    coef = fit(t, g)
    tt = sample(6001, 3001)
    gg = np.array([float(g_exact(v)) for v in tt])
    e64 = np.max(np.abs(np.polyval(coef[::-1], 2 * tt - 1) / gg - 1))
    e32 = np.max(np.abs(horner32(coef, tt) / gg - 1))
    print(f"// degree {DEG}: max relative error {e64:.2e} (exact arithmetic), "
          f"{e32:.2e} (FP32 Horner, float32 coefficients)")
    body = ",\n".join(f"    {float(np.float32(v)):.9e}f" for v in coef)
    print(f"constexpr float kMillsPoly[{DEG + 1}] = {{\n{body}}};")


if __name__ == "__main__":
    main()
