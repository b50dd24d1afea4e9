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


# ---------------------------------------------------------------------------
# RBMC estimator (Rao-Blackwellised Monte Carlo, perturbation-optimisation samples)
# ---------------------------------------------------------------------------
from oracle import operators as ops  # noqa: E402


def _op(kind, h=6, w=8, seed=0):
    rng = np.random.default_rng(seed)
    if kind == "blur":
        return ops.Operator(ops.BLUR, (h, w), taps=syn.gaussian_taps(1.3, 5))
    mask = syn.dft_mask(h, w, 0.4, rng)
    return ops.Operator(ops.DFT if kind == "dft" else ops.HADAMARD, (h, w), mask=mask)


def _cavity(h, w, seed=1):
    """A cavity precision spanning several decades, like a TV cavity after a few
    sweeps (flat pixels next to sharp ones)."""
    rng = np.random.default_rng(seed)
    return 10.0 ** rng.uniform(-3, 2.5, size=(h, w))


@pytest.mark.parametrize("kind", ["blur", "dft", "hadamard"])
def test_diag_of_hth_is_the_mean_eigenvalue(kind):
    op = _op(kind, 8, 8)
    assert np.allclose(np.diag(op.dense_HtH()), op.diag_HtH(), rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("kind", ["blur", "dft", "hadamard"])
def test_rbmc_with_a_spanning_design_is_exact(kind):
    """With the white noise replaced by a scaled orthonormal basis of the joint
    (observation, pixel) noise space, the sample second moment of z is exactly
    Q, so the estimator returns the exact diagonal of Q^{-1} (dense inverse):
    any dropped term, wrong scale of either noise part (sqrt(xi), sqrt(tau_c))
    or wrong sign shows up here."""
    h, w = 4, 8
    op = _op(kind, h, w)
    xi = 0.05
    tau_c = _cavity(h, w)
    n = h * w
    obs_dims = 2 * n if kind == "dft" else n     # real and imaginary parts
    ns = obs_dims + n
    e1 = np.zeros((ns, h, w), dtype=complex if kind == "dft" else float)
    e2 = np.zeros((ns, h, w))
    scale = np.sqrt(ns)
    for s in range(ns):
        if s < obs_dims:
            k, part = (s // 2, s % 2) if kind == "dft" else (s, 0)
            e1[s].flat[k] = scale * (1j if part else 1.0)
        else:
            e2[s].flat[s - obs_dims] = scale
    v = ops.rbmc_variance(op, xi, tau_c, ops.RBMCSamples(e1, e2))
    v_ex = ops.tilted_variance(op, xi, tau_c, "exact")
    assert np.allclose(v, v_ex, rtol=1e-9, atol=0)


def test_rbmc_is_exact_for_identity_and_bounded_below():
    """H = I: Q is diagonal, every off-diagonal sum vanishes, and the estimate
    is 1 / Q_ii for any noise; in general v_i >= 1 / Q_ii."""
    h, w = 5, 7
    tau_c = _cavity(h, w)
    rng = np.random.default_rng(3)
    e1, e2 = rng.standard_normal((4, h, w)), rng.standard_normal((4, h, w))
    op = ops.Operator(ops.BLUR, (h, w), taps=np.pad(np.ones((1, 1)), 1))   # the identity as a blur
    v = ops.rbmc_variance(op, 0.1, tau_c, ops.RBMCSamples(e1, e2))
    assert np.allclose(v, 1.0 / (1.0 / 0.1 + tau_c), rtol=1e-12)
    op = _op("blur", h, w)
    v = ops.rbmc_variance(op, 0.1, tau_c, ops.RBMCSamples(e1, e2))
    assert np.all(v >= 1.0 / (op.diag_HtH() / 0.1 + tau_c) * (1 - 1e-12))


@pytest.mark.parametrize("kind", ["blur", "dft", "hadamard"])
def test_rbmc_converges_to_the_exact_diagonal(kind):
    """Random white noise: the estimate is unbiased, and with 1500 samples
    every pixel lies within 5 standard errors (estimated from the samples
    themselves) of the exact diagonal."""
    h, w = 4, 8
    op = _op(kind, h, w, seed=4)
    xi = 0.05
    tau_c = _cavity(h, w, seed=5)
    rng = np.random.default_rng(6)
    ns = 1500
    e2 = rng.standard_normal((ns, h, w))
    if kind == "dft":
        e1 = rng.standard_normal((ns, h, w)) + 1j * rng.standard_normal((ns, h, w))
    else:
        e1 = rng.standard_normal((ns, h, w))
    qd = op.diag_HtH() / xi + tau_c
    # per-sample terms, for the standard error (the same arithmetic as the estimator)
    terms = []
    for s in range(ns):
        z = op.Ht(e1[s]) / np.sqrt(xi) + np.sqrt(tau_c) * e2[s]
        x, _ = ops.solve_tilted_mean(op, xi, tau_c, z)
        off = op.HtH(x) / xi + tau_c * x - qd * x
        terms.append(off * off / (qd * qd))
    terms = np.asarray(terms)
    se = terms.std(axis=0, ddof=1) / np.sqrt(ns)
    v = ops.rbmc_variance(op, xi, tau_c, ops.RBMCSamples(e1, e2))
    v_ex = ops.tilted_variance(op, xi, tau_c, "exact")
    assert np.allclose(v, 1.0 / qd + terms.mean(axis=0), rtol=1e-9)
    assert np.all(np.abs(v - v_ex) <= 5 * se + 1e-12 * v_ex)


def test_rbmc_ep_solves_the_runaway_case():
    """The 4 x 4 case where the spectral estimator runs away: EP with the RBMC
    estimator (16 samples, fixed for the run) converges, inside the data range,
    close to EP with the exact diagonal."""
    p = _runaway_case()
    rng = np.random.default_rng(11)
    noise = (rng.standard_normal((16, 4, 4)), rng.standard_normal((16, 4, 4)))
    pb = ep.problem_from_synthetic(p, estimator="rbmc", rbmc_noise=noise)
    mu, v, st, info = ep.solve(pb, 3000, False, tol=1e-10)
    assert info["converged"] and not info["diverged"]
    pe = ep.problem_from_synthetic(p, estimator="exact")
    mu_e, v_e, _, info_e = ep.solve(pe, 3000, False, tol=1e-10)
    rng_e = mu_e.max() - mu_e.min()
    assert np.max(np.abs(mu - mu_e)) <= 0.1 * rng_e
    assert np.all(v > 0)
