"""Pins for the EM options of Sec. IV (approximations of a_0 in lambda = N / a_0)
and for the non-i.i.d. noise of the denoising problem (Sec. III-C).

* option 1 (a_x under Q(x)): Monte Carlo over samples of the diagonal Gaussian
  Q(x) itself, summed over every 4-neighbour edge (an independent enumeration
  of the edges), within 5 standard errors;
* option 2 (a_u under Q(u)): on a single edge EP is exact, so after one
  undamped update Q(u) is the Gaussian with the exact posterior moments of
  u = x_1 - x_2, obtained here by quadrature; a_u is its folded-normal mean;
* the three options on one EP state differ the way the paper describes:
  Q(x)'s diagonal covariance ignores neighbour correlation, so a_x exceeds the
  tilted a_bar_u on a smooth image, and the EM fixed point of each option
  satisfies lambda = N / a_0(lambda);
* non-i.i.d. noise: the l2-TV fixed point (any EP fixed point has the exact
  posterior mean) solves (W + beta L) mu = W y with W = diag(1 / xi_i), solved
  densely here; a constant map reproduces the i.i.d. run exactly."""
import math

import numpy as np
import pytest
from scipy import integrate

import synthetic as syn
from oracle import ep
from oracle import operators as ops
from oracle.tilted import folded_normal_mean


def _edges(h, w):
    out = []
    for r in range(h):
        for c in range(w):
            if c + 1 < w:
                out.append((r * w + c, r * w + c + 1))
            if r + 1 < h:
                out.append((r * w + c, (r + 1) * w + c))
    return out


def test_option1_is_the_expected_tv_under_q():
    h, w = 6, 7
    rng = np.random.default_rng(1)
    y = syn.piecewise_image(h, w, 3, rng) + 0.1 * rng.normal(size=(h, w))
    pb = ep.EPProblem(y, ops.Operator(ops.IDENTITY, (h, w)), 0.01, 6.0, em_diagnostics=True)
    mu, v, st, _ = ep.solve(pb, 7, em=False)
    ns = 200000
    xs = mu.ravel()[None, :] + np.sqrt(v.ravel())[None, :] * rng.standard_normal((ns, h * w))
    tv = np.zeros(ns)
    for i, j in _edges(h, w):
        tv += np.abs(xs[:, i] - xs[:, j])
    se = tv.std(ddof=1) / math.sqrt(ns)
    assert abs(st.a_x - tv.mean()) <= 5 * se


def test_option2_on_a_single_edge_uses_the_exact_moments_of_u():
    y = np.array([[0.35, -0.2]])
    xi, lam = 0.03, 5.0
    pb = ep.EPProblem(y, ops.Operator(ops.IDENTITY, (1, 2)), xi, lam, damping=1.0,
                      em_diagnostics=True)
    mu, v, st, _ = ep.solve(pb, 1, em=False)
    # exact posterior of u = x1 - x2: N(u; y1 - y2, 2 xi) exp(-lam |u|)
    d = y[0, 0] - y[0, 1]
    f = lambda u: math.exp(-(u - d) ** 2 / (4 * xi) - lam * abs(u))
    opts = dict(epsabs=0, epsrel=1e-12, points=[0.0])
    Z = integrate.quad(f, -3, 3, **opts)[0]
    m1 = integrate.quad(lambda u: u * f(u), -3, 3, **opts)[0] / Z
    m2 = integrate.quad(lambda u: u * u * f(u), -3, 3, **opts)[0] / Z
    e_abs = integrate.quad(lambda u: abs(u) * f(u), -3, 3, **opts)[0] / Z
    assert abs(st.a_u - float(folded_normal_mean(m1, m2 - m1 * m1))) <= 1e-9
    assert abs(st.a_bar - e_abs) <= 1e-9           # option 3: the tilted E|u| itself


@pytest.mark.parametrize("option", [1, 2, 3])
def test_em_fixed_point_of_each_option(option):
    h, w = 8, 8
    rng = np.random.default_rng(2)
    y = syn.piecewise_image(h, w, 3, rng) + 0.1 * rng.normal(size=(h, w))
    pb = ep.EPProblem(y, ops.Operator(ops.IDENTITY, (h, w)), 0.01, 1.0, em_option=option,
                      em_diagnostics=True)
    mu, v, st, info = ep.solve(pb, 5000, em=True, tol=1e-12)
    assert info["converged"]
    a0 = {1: st.a_x, 2: st.a_u, 3: st.a_bar}[option]
    assert abs(pb.N / a0 / st.lam - 1) <= 1e-9
    # the diagonal Q(x) ignores the positive correlation of neighbours, so its
    # expected TV is the largest, and option 1 gives the smallest lambda
    assert st.a_x > st.a_bar


def _laplacian(h, w):
    n = h * w
    L = np.zeros((n, n))
    for a, b in _edges(h, w):
        L[a, a] += 1; L[b, b] += 1; L[a, b] -= 1; L[b, a] -= 1
    return L


def test_non_iid_noise_l2_fixed_point_is_the_dense_posterior_mean():
    h, w = 7, 6
    rng = np.random.default_rng(3)
    x = syn.piecewise_image(h, w, 3, rng)
    nv = 10.0 ** rng.uniform(-3, -1, size=(h, w))
    y = x + np.sqrt(nv) * rng.normal(size=(h, w))
    beta = 25.0
    pb = ep.EPProblem(y, ops.Operator(ops.IDENTITY, (h, w)), float(nv.mean()), beta, damping=0.5,
                      prior="l2", noise_var_map=nv)
    mu, v, st, info = ep.solve(pb, 4000, em=False, tol=1e-14)
    W = np.diag(1.0 / nv.ravel())
    mu_ref = np.linalg.solve(W + beta * _laplacian(h, w), W @ y.ravel()).reshape(h, w)
    assert np.max(np.abs(mu - mu_ref)) <= 1e-9 * (mu_ref.max() - mu_ref.min())


def test_constant_noise_map_is_the_iid_problem():
    p = syn.make_denoise(9, 11, 3, 0.1, np.random.default_rng(4), lam0=7.0, em=True)
    a = ep.solve(ep.problem_from_synthetic(p), 25, True)
    pb = ep.problem_from_synthetic(p)
    pb2 = ep.EPProblem(p.y, pb.op, p.xi, p.lam0, damping=p.damping,
                       noise_var_map=np.full(p.shape, p.xi))
    b = ep.solve(pb2, 25, True)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
