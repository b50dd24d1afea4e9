"""Variance estimators of the likelihood site (diag Cov_{P_0}, Sec. III-C, Eq.
(tilted_P_1)) and the divergence rule.

The spectral estimator replaces the cavity precision by its mean, which is exact
at constant cavity (pinned in tests/test_oracle_ops.py).  On small images with a
sparse transform mask the cavity spans many decades (flat TV sites at 1e-8
next to sharp ones), the estimator then assigns the likelihood factor far more
precision than it has where the mask leaves the flat pixels unobserved, and EP
runs away: the tilted mean grows without bound.  The exact diagonal solves the
same problem.  These tests fix that diagnosis on the CPU."""
import numpy as np
import pytest

import synthetic as syn
from oracle import ep


def _runaway_case(kind="hcs"):
    h = w = 4
    rng = syn.rng_for(90, h * 1000 + w)
    if kind == "hcs":
        return syn.make_hadamard_cs(h, w, 3, 0.01, 0.3, rng, sweeps=10, em=False, lam0=10.0)
    return syn.make_cs(h, w, 3, 0.01, 0.3, syn.rng_for(95, 3 * 100 + 44), sweeps=10, em=False,
                       lam0=10.0)


def test_spectral_estimator_runs_away_on_a_sparse_4x4_mask():
    p = _runaway_case()
    pb = ep.problem_from_synthetic(p, estimator="spectral")
    mu, v, st, info = ep.solve(pb, 60, False)
    assert info["diverged"] and info["sweeps"] <= 10
    # the runaway pixels are the ones whose TV cavity stayed flat
    tau_c = st.tau[1:].sum(axis=0)
    assert tau_c.min() < 1e-7 and tau_c.max() > 10.0


def test_exact_estimator_solves_the_same_problem():
    p = _runaway_case()
    pb = ep.problem_from_synthetic(p, estimator="exact")
    mu, v, st, info = ep.solve(pb, 2000, False, tol=1e-10)
    assert info["converged"] and not info["diverged"]
    hty = pb.hty
    assert np.abs(mu).max() <= 3 * (hty.max() - hty.min())
    assert np.all(v > 0) and np.all(np.isfinite(v))


def test_divergence_rule_stays_quiet_on_converging_runs():
    """The workload families (deconvolution, DFT and Walsh-Hadamard CS) at small
    size: no false alarm from cold, including the first, least regularised
    likelihood solves."""
    for p in (syn.config1(size=64, sweeps=40), syn.config2(size=64, sweeps=40),
              syn.make_hadamard_cs(64, 64, 6, 0.01, 0.3, syn.rng_for(91, 0), sweeps=40)):
        mu, v, st, info = ep.solve(ep.problem_from_synthetic(p), 40, True)
        assert not info["diverged"]
