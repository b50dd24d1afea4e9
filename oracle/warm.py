"""Oracle of the warm-start initialisation of the EP sites (test infrastructure
only).

Given a predicted posterior mean mu_hat and variance v_hat per pixel (from the
learned network, or any other source), the sites are set so that the global
approximation of Eq. (Q_x_final) equals N(mu_hat, diag v_hat) exactly:

  * identity operator: q_{x,0} is exact and constant, so it keeps its value
    (1/xi, y/xi); the remaining precision R = 1/v_hat - 1/xi (at least
    c_p * 1e-8) and the remaining eta are split equally over the c_p colour
    classes that cover the pixel;
  * other operators: precision 1/v_hat and eta mu_hat/v_hat are split equally
    over q_{x,0} and the covering classes (n_p = 1 + c_p sites).

Uncovered classes keep (0, 0).  lambda_0 is the EM update with option 1 of the
paper's approximations of a_0 (Sec. IV-B): a_x = sum over all pairs of
E_Q |x_i - x_j| under Q(x) = N(mu_hat, diag v_hat), i.e. a folded-normal mean
with variance v_i + v_j, and lambda_0 = N / a_x.  Non-finite or non-positive
predictions are rejected (the caller then starts cold).
"""
from __future__ import annotations

import math

import numpy as np

from . import ep
from . import operators as ops
from . import tilted as tilted_mod


folded_normal_mean = tilted_mod.folded_normal_mean
a_x = ep.a_x


def lambda_option1(pb: ep.EPProblem, mu, v, scale=1.0, power=1.0):
    """scale * (N / a_x)^power; scale = power = 1 is option 1 as is."""
    a = a_x(pb, mu, v)
    return scale * (pb.N / a) ** power if a > 0.0 else pb.lam0


def init_warm(pb: ep.EPProblem, mu_hat, v_hat, set_lambda=True, scale=1.0, power=1.0):
    """EPState with the warm sites, or None when the prediction is unusable."""
    mu = np.asarray(mu_hat, np.float64).ravel()
    v = np.asarray(v_hat, np.float64).ravel()
    if not (np.all(np.isfinite(mu)) and np.all(np.isfinite(v)) and np.all(v > 0)):
        return None
    N = pb.N
    tau = np.zeros((5, N))
    eta = np.zeros((5, N))
    cov = pb.covered                      # (4, N) bool
    c = cov.sum(axis=0).astype(np.float64)
    prec = 1.0 / v
    if pb.op.kind == ops.IDENTITY:
        y = np.asarray(pb.y, np.float64).ravel()
        w = 1.0 / pb.xi if pb.noise_prec is None else pb.noise_prec
        tau[0] = w
        eta[0] = y * w
        rest_tau = np.maximum(prec - w, c * ep.SITE_INIT_PREC)
        rest_eta = mu * (w + rest_tau) - y * w
        share = np.where(c > 0, 1.0 / np.maximum(c, 1.0), 0.0)
        for k in range(4):
            tau[k + 1] = np.where(cov[k], rest_tau * share, 0.0)
            eta[k + 1] = np.where(cov[k], rest_eta * share, 0.0)
    else:
        n = 1.0 + c
        tau[0] = prec / n
        eta[0] = mu * prec / n
        for k in range(4):
            tau[k + 1] = np.where(cov[k], prec / n, 0.0)
            eta[k + 1] = np.where(cov[k], mu * prec / n, 0.0)
    lam = lambda_option1(pb, mu, v, scale, power) if set_lambda else pb.lam0
    return ep.EPState(tau=tau, eta=eta, lam=lam, warm=True)
