"""Exact posterior marginals of tiny denoising problems by grid integration.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Sec. II-C, Eq. (exact_posterior_distribution): for H = I and the l1-TV prior,

    f(x | y) ~ prod_p N(y_p; x_p, xi) * prod_{(i,j) in V} exp(-lambda |x_i - x_j|),

with V the 4-neighbour edges inside the image (free boundary).  For an image
with 3 rows, the states of one column (x_0c, x_1c, x_2c) live on a G^3 grid and
the column-to-column coupling factorises over rows, so forward-backward message
passing over the columns gives every pixel marginal exactly up to the grid
error; the grid is uniform on y_min - 8 sqrt(xi) .. y_max + 8 sqrt(xi).  The
kink of |.| makes the midpoint rule second order, so two grids G and 2G are
combined by Richardson extrapolation of the moments.

This checks how close EP is to the exact posterior (approximation quality),
not parity: EP is an approximation.
"""
from __future__ import annotations

import numpy as np


def _moments_on_grid(y, xi, lam, G):
    rows, cols = y.shape
    if rows != 3:
        raise ValueError("brute force supports images with exactly 3 rows")
    sd = np.sqrt(xi)
    lo = float(y.min()) - 8.0 * sd
    hi = float(y.max()) + 8.0 * sd
    h = (hi - lo) / G
    g = lo + h * (np.arange(G) + 0.5)                      # midpoints
    phi = np.exp(-lam * np.abs(g[:, None] - g[None, :]))   # pair factor on the grid

    def column_potential(c):
        lik = [np.exp(-0.5 * (y[r, c] - g) ** 2 / xi) for r in range(3)]
        pot = (lik[0][:, None, None] * lik[1][None, :, None] * lik[2][None, None, :])
        pot = pot * phi[:, :, None] * phi[None, :, :]      # vertical edges (0,1), (1,2)
        return pot

    def couple(msg):
        # sum_{a,b,c} msg(a,b,c) phi(a,a') phi(b,b') phi(c,c')
        out = np.tensordot(msg, phi, axes=([0], [0]))       # (b, c, a')
        out = np.tensordot(out, phi, axes=([0], [0]))       # (c, a', b')
        out = np.tensordot(out, phi, axes=([0], [0]))       # (a', b', c')
        return out

    pots = [column_potential(c) for c in range(cols)]
    alpha = [None] * cols
    a = pots[0]
    alpha[0] = a / a.sum()
    for c in range(1, cols):
        a = pots[c] * couple(alpha[c - 1])
        alpha[c] = a / a.sum()
    beta = [None] * cols
    beta[cols - 1] = np.ones((G, G, G))
    for c in range(cols - 2, -1, -1):
        b = couple(pots[c + 1] * beta[c + 1])
        beta[c] = b / b.sum()
    mean = np.zeros((3, cols))
    var = np.zeros((3, cols))
    for c in range(cols):
        joint = alpha[c] * beta[c]
        joint = joint / joint.sum()
        margs = [joint.sum(axis=(1, 2)), joint.sum(axis=(0, 2)), joint.sum(axis=(0, 1))]
        for r in range(3):
            m1 = float(np.dot(margs[r], g))
            m2 = float(np.dot(margs[r], g * g))
            mean[r, c] = m1
            var[r, c] = m2 - m1 * m1
    return mean, var


def posterior_marginals(y, xi, lam, G=96):
    """Exact posterior means and variances (3 x W image), Richardson-combined
    from grids of G and 2G points per pixel."""
    m1, v1 = _moments_on_grid(np.asarray(y, dtype=np.float64), xi, lam, G)
    m2, v2 = _moments_on_grid(np.asarray(y, dtype=np.float64), xi, lam, 2 * G)
    return (4.0 * m2 - m1) / 3.0, (4.0 * v2 - v1) / 3.0
