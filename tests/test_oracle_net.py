"""Pins of the warm-start oracles (oracle/net.py, oracle/warm.py) against things
other than themselves: a library correlation routine, torch's bfloat16
conversion, finite differences, adjoint identities, Adam's closed form under a
constant gradient, normalisation invariance, quadrature of the folded normal,
and exact reconstruction of the predicted marginals by the warm sites."""
import math

import numpy as np
import pytest
from scipy import integrate, signal

import synthetic as syn
from oracle import ep as oep
from oracle import net
from oracle import warm

SMALL = (1, 3, 4, 2)


def test_param_count():
    assert net.param_count() == 9 * 32 + 32 + 4 * (9 * 32 * 32 + 32) + 9 * 32 * 2 + 2 == 37890


def test_bf16_round_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=5000) * 10.0 ** rng.integers(-30, 30, 5000),
                        np.float32([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -1.0 - 2 ** -8, 0.0, -0.0,
                                    3.0e38, 1e-39, 65504.0])]).astype(np.float32)
    ref = torch.tensor(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(net.bf16_round(x), ref)


def test_conv_matches_scipy_correlate():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(2, 7, 9, 3))
    w = rng.normal(size=(3, 3, 3, 4))
    b = rng.normal(size=4)
    out = net.conv3x3(x, w, b)
    for n in range(2):
        for o in range(4):
            ref = b[o] + sum(signal.correlate(x[n, :, :, i], w[:, :, i, o], mode="same")
                             for i in range(3))
            assert np.allclose(out[n, :, :, o], ref, rtol=1e-12, atol=1e-12)


def test_conv_adjoints():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(2, 6, 5, 3))
    w = rng.normal(size=(3, 3, 3, 4))
    g = rng.normal(size=(2, 6, 5, 4))
    lhs = np.sum(net.conv3x3(x, w) * g)
    assert np.isclose(lhs, np.sum(x * net.conv3x3_input_grad(g, w)), rtol=1e-12)
    assert np.isclose(lhs, np.sum(w * net.conv3x3_weight_grad(x, g)), rtol=1e-12)


def _small_problem(seed=3):
    rng = np.random.default_rng(seed)
    y = rng.normal(size=(2, 6, 7)) * 0.3 + 0.5
    mu = y + 0.05 * rng.normal(size=y.shape)
    v = np.exp(rng.normal(size=y.shape) * 0.3) * 2e-4
    theta = net.init_params(rng, SMALL)
    for k in range(len(theta)):            # non-zero biases so every term is exercised
        pass
    layers = net.unpack(theta, SMALL)
    for _, b in layers:
        b[:] = rng.normal(size=b.shape) * 0.1
    return y, mu, v, theta


def _loss(theta, y, mu, v, xi):
    o, cache = net.forward(theta, y, False, SMALL)
    return net.loss(o, net.targets(mu, v, cache, xi))


def test_backward_matches_finite_differences():
    y, mu, v, theta = _small_problem()
    xi = 1e-4
    o, cache = net.forward(theta, y, False, SMALL)
    g = net.backward(theta, o, net.targets(mu, v, cache, xi), cache, SMALL)
    rng = np.random.default_rng(4)
    idx = rng.choice(theta.size, size=60, replace=False)
    h = 1e-6
    for k in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        fd = (_loss(tp, y, mu, v, xi) - _loss(tm, y, mu, v, xi)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(fd)), (k, fd, g[k])


def test_output_invariant_to_affine_rescaling_of_y():
    y, _, _, theta = _small_problem(5)
    o1, c1 = net.forward(theta, y, False, SMALL)
    o2, c2 = net.forward(theta, 3.5 * y - 2.0, False, SMALL)
    assert np.allclose(o1, o2, rtol=1e-10, atol=1e-10)
    mu1, _ = net.outputs(o1, c1, 1e-4)
    mu2, _ = net.outputs(o2, c2, 1e-4)
    assert np.allclose(mu2, 3.5 * mu1 - 2.0, rtol=1e-10, atol=1e-10)


def test_bf16_mode_is_close_to_exact():
    y, mu, v, theta = _small_problem(6)
    o64, _ = net.forward(theta, y, False, SMALL)
    o16, _ = net.forward(theta, y, True, SMALL)
    assert np.max(np.abs(o16 - o64)) <= 3e-2 * np.max(np.abs(o64))
    assert not np.array_equal(o16, o64)


def test_adam_constant_gradient_closed_form():
    """With a constant gradient g the bias-corrected moments are g and g^2 at
    every step, so each step moves theta by -lr g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    th = np.array([1.0, 2.0, 3.0, 4.0])
    opt = net.Adam(4)
    lr = 1e-2
    x = th.copy()
    for _ in range(7):
        x = opt.step(x, g, lr)
    assert np.allclose(x, th - 7 * lr * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("m,var", [(0.0, 1.0), (0.7, 0.2), (-3.0, 0.5), (1e-3, 4.0)])
def test_folded_normal_mean_quadrature(m, var):
    f = lambda d: abs(d) * math.exp(-(d - m) ** 2 / (2 * var)) / math.sqrt(2 * math.pi * var)
    ref = integrate.quad(f, -np.inf, 0)[0] + integrate.quad(f, 0, np.inf)[0]
    assert abs(warm.folded_normal_mean(m, var) - ref) <= 1e-10


@pytest.mark.parametrize("kind", ["blur", "identity", "dft"])
def test_warm_sites_reproduce_prediction(kind):
    rng = syn.rng_for(60, 0)
    if kind == "blur":
        p = syn.make_deconv(12, 10, 3, 0.02, 1.0, rng, ksize=5)
    elif kind == "dft":
        p = syn.make_cs(8, 16, 3, 0.02, 0.4, rng)
    else:
        p = syn.make_denoise(12, 10, 3, 0.1, rng, mode="paint")
    pb = oep.problem_from_synthetic(p)
    mu_hat = p.x_true + 0.01 * rng.standard_normal(p.shape)
    v_hat = np.full(p.shape, 0.5 * p.xi) * np.exp(0.1 * rng.standard_normal(p.shape))
    st = warm.init_warm(pb, mu_hat, v_hat)
    mu, v = oep.marginals(st)
    assert np.allclose(mu.reshape(p.shape), mu_hat, rtol=1e-12, atol=1e-12)
    assert np.allclose(v.reshape(p.shape), v_hat, rtol=1e-12)
    assert np.all(st.tau >= 0) and st.warm
    for k in range(4):                      # uncovered classes stay flat
        assert np.all(st.tau[k + 1][~pb.covered[k]] == 0)


def test_warm_rejects_bad_prediction():
    p = syn.make_denoise(6, 6, 2, 0.1, syn.rng_for(60, 1), mode="paint")
    pb = oep.problem_from_synthetic(p)
    v = np.full(p.shape, 1e-3)
    mu = np.zeros(p.shape)
    assert warm.init_warm(pb, mu, -v) is None
    mu[2, 3] = np.nan
    assert warm.init_warm(pb, mu, v) is None


def test_lambda_option1_constant_image():
    """Constant mean, variance v everywhere: every pair difference is N(0, 2v),
    E|d| = 2 sqrt(v / pi), so lambda_0 = N / (E 2 sqrt(v / pi))."""
    p = syn.make_denoise(9, 7, 2, 0.1, syn.rng_for(60, 2), mode="paint")
    pb = oep.problem_from_synthetic(p)
    v = 3e-3
    lam = warm.lambda_option1(pb, np.full(p.shape, 0.4), np.full(p.shape, v))
    E = 9 * 6 + 8 * 7
    assert np.isclose(lam, 63 / (E * 2 * math.sqrt(v / math.pi)), rtol=1e-12)


def test_warm_start_at_fixed_point_is_near_stationary():
    """At fixed lambda, warm-starting the oracle from its own converged
    marginals must converge in fewer sweeps than a cold start (the equal
    split is not the fixed point's split, so it is not instantaneous)."""
    p = syn.make_deconv(24, 24, 4, 0.02, 1.5, syn.rng_for(60, 3), lam0=5.0)
    pb = oep.problem_from_synthetic(p)
    mu, v, st, info = oep.solve(pb, 600, False, tol=1e-6)
    assert info["converged"]
    st_w = warm.init_warm(pb, mu, v, set_lambda=False)
    mu_w, v_w, _, info_w = oep.solve(pb, 600, False, tol=1e-6, state=st_w)
    assert info_w["converged"] and info_w["sweeps"] < info["sweeps"]
    yr = p.y.max() - p.y.min()
    assert np.max(np.abs(mu_w - mu)) <= 1e-4 * yr
