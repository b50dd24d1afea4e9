"""Pins for oracle/ep.py: EP with TV priors, Algorithms 1 and 2.

Each pin is fixed by something other than the oracle itself:

* colour classes: rebuilt here from the 4-neighbour definition (Fig. 1);
* l2-TV (Gaussian pair factor) fixed point: any EP fixed point has the exact
  posterior mean, which solves (H^T H / xi + beta L) mu = H^T y / xi with L the
  graph Laplacian -- built here by explicit neighbour loops and solved densely;
* a single edge (1 x 2 image, H = I): the tilted distribution is the exact
  posterior, so one undamped update gives the exact marginals (2-D quadrature);
* EM on a single edge: the EP-EM fixed point is a stationary point of the
  marginal likelihood f(y | lambda) of Sec. IV (1-D quadrature + optimiser),
  which fixes lambda = N / a_bar_u with N the number of pixels;
* symmetry invariants (sign flip, 180 degree rotation, transpose with the
  matching block order).
"""
import math

import numpy as np
import pytest
from scipy import integrate, optimize

import synthetic as syn
from oracle import ep
from oracle import operators as ops


def _edges_reference(h, w, periodic):
    """All 4-neighbour edges as a set of frozensets of flat indices."""
    E = set()
    for r in range(h):
        for c in range(w):
            p = r * w + c
            if c + 1 < w:
                E.add(frozenset((p, r * w + c + 1)))
            elif periodic:
                E.add(frozenset((p, r * w)))
            if r + 1 < h:
                E.add(frozenset((p, (r + 1) * w + c)))
            elif periodic:
                E.add(frozenset((p, c)))
    return E


@pytest.mark.parametrize("h,w,bnd", [(5, 7, "free"), (4, 6, "periodic"), (1, 2, "free"),
                                     (6, 1, "free"), (8, 8, "periodic"), (3, 3, "free")])
def test_colour_classes_partition_edges(h, w, bnd):
    classes = ep.colour_classes(h, w, bnd)
    seen = []
    for k, (i, j) in enumerate(classes):
        pix = np.concatenate([i, j])
        assert len(set(pix.tolist())) == pix.size, "a pixel appears twice in one class"
        for a, b in zip(i, j):
            ra, ca = divmod(int(a), w)
            rb, cb = divmod(int(b), w)
            if k < 2:   # horizontal, left pixel column parity = k
                assert ra == rb and ca % 2 == k and cb == (ca + 1) % w
            else:       # vertical, top pixel row parity = k - 2
                assert ca == cb and ra % 2 == k - 2 and rb == (ra + 1) % h
        seen += [frozenset((int(a), int(b))) for a, b in zip(i, j)]
    assert len(seen) == len(set(seen))
    assert set(seen) == _edges_reference(h, w, bnd == "periodic")


def _laplacian(h, w, periodic):
    n = h * w
    L = np.zeros((n, n))
    for e in _edges_reference(h, w, periodic):
        a, b = tuple(e)
        L[a, a] += 1; L[b, b] += 1; L[a, b] -= 1; L[b, a] -= 1
    return L


@pytest.mark.parametrize("kind,bnd", [(ops.IDENTITY, "free"), (ops.IDENTITY, "periodic"),
                                      (ops.BLUR, "free"), (ops.BLUR, "periodic"),
                                      (ops.DFT, "free"), (ops.DFT, "periodic")])
def test_l2_fixed_point_is_dense_posterior_mean(kind, bnd):
    h = w = 8
    rng = np.random.default_rng(11)
    x = syn.piecewise_image(h, w, 4, rng)
    xi = 0.01
    if kind == ops.IDENTITY:
        op = ops.Operator(kind, (h, w))
        y = x + 0.1 * rng.normal(size=(h, w))
    elif kind == ops.BLUR:
        op = ops.Operator(kind, (h, w), taps=syn.gaussian_taps(1.0, 5))
        y = op.H(x) + 0.1 * rng.normal(size=(h, w))
    else:
        op = ops.Operator(kind, (h, w), mask=syn.dft_mask(h, w, 0.4, rng))
        y = op.H(x) + 0.07 * (rng.normal(size=(h, w)) + 1j * rng.normal(size=(h, w))) * op.mask
    beta = 30.0
    pb = ep.EPProblem(y, op, xi, beta, damping=0.5, prior="l2", boundary=bnd)
    mu, v, st, info = ep.solve(pb, 4000, em=False, tol=1e-14)
    A = op.dense_HtH() / xi + beta * _laplacian(h, w, bnd == "periodic")
    mu_ref = np.linalg.solve(A, op.Hty(y).ravel() / xi).reshape(h, w)
    scale = mu_ref.max() - mu_ref.min()
    assert np.max(np.abs(mu - mu_ref)) <= 1e-9 * scale
    assert st.clamp_count == 0


def test_single_edge_update_is_exact_posterior():
    y = np.array([[0.3, -0.45]])
    xi, lam = 0.04, 6.0
    pb = ep.EPProblem(y, ops.Operator(ops.IDENTITY, (1, 2)), xi, lam, damping=1.0)
    mu, v, st, _ = ep.solve(pb, 1, em=False)

    def post(x1, x2):
        return math.exp(-((x1 - y[0, 0]) ** 2 + (x2 - y[0, 1]) ** 2) / (2 * xi)
                        - lam * abs(x1 - x2))
    lo, hi = -2.5, 2.5
    opts = dict(epsabs=0, epsrel=1e-12)
    Z = integrate.dblquad(lambda b, a: post(a, b), lo, hi, lo, hi, **opts)[0]
    m1 = integrate.dblquad(lambda b, a: a * post(a, b), lo, hi, lo, hi, **opts)[0] / Z
    m2 = integrate.dblquad(lambda b, a: b * post(a, b), lo, hi, lo, hi, **opts)[0] / Z
    s1 = integrate.dblquad(lambda b, a: (a - m1) ** 2 * post(a, b), lo, hi, lo, hi, **opts)[0] / Z
    s2 = integrate.dblquad(lambda b, a: (b - m2) ** 2 * post(a, b), lo, hi, lo, hi, **opts)[0] / Z
    assert abs(mu[0, 0] - m1) < 1e-8 and abs(mu[0, 1] - m2) < 1e-8
    assert abs(v[0, 0] / s1 - 1) < 1e-7 and abs(v[0, 1] / s2 - 1) < 1e-7


def test_single_edge_update_is_exact_posterior_mog2():
    """The same single-edge exactness for the MoG2-TV prior (Eq. (MoG2_TV_prior)):
    the posterior is a mixture of two 2-D Gaussians, integrated numerically.
    Exact as long as the tilted variance of u stays below the cavity variance
    (rho > 0, here 0.63); beyond that the site precision would be negative and
    the clamp of Sec. III-C applies instead."""
    y = np.array([[0.2, -0.1]])
    xi = 0.04
    theta = (0.3, 0.5, 0.01)
    pb = ep.EPProblem(y, ops.Operator(ops.IDENTITY, (1, 2)), xi, theta, damping=1.0, prior="mog2")
    mu, v, st, _ = ep.solve(pb, 1, em=False)
    om, v1, v2 = theta

    def post(x1, x2):
        u = x1 - x2
        phi = om * math.exp(-u * u / (2 * v1)) / math.sqrt(v1) + (1 - om) * math.exp(-u * u / (2 * v2)) / math.sqrt(v2)
        return math.exp(-((x1 - y[0, 0]) ** 2 + (x2 - y[0, 1]) ** 2) / (2 * xi)) * phi
    lo, hi = -2.5, 2.5
    opts = dict(epsabs=0, epsrel=1e-12)
    Z = integrate.dblquad(lambda b, a: post(a, b), lo, hi, lo, hi, **opts)[0]
    m1 = integrate.dblquad(lambda b, a: a * post(a, b), lo, hi, lo, hi, **opts)[0] / Z
    m2 = integrate.dblquad(lambda b, a: b * post(a, b), lo, hi, lo, hi, **opts)[0] / Z
    s1 = integrate.dblquad(lambda b, a: (a - m1) ** 2 * post(a, b), lo, hi, lo, hi, **opts)[0] / Z
    s2 = integrate.dblquad(lambda b, a: (b - m2) ** 2 * post(a, b), lo, hi, lo, hi, **opts)[0] / Z
    assert abs(mu[0, 0] - m1) < 1e-8 and abs(mu[0, 1] - m2) < 1e-8
    assert abs(v[0, 0] / s1 - 1) < 1e-7 and abs(v[0, 1] / s2 - 1) < 1e-7


def test_mixture_prior_with_equal_components_is_l2():
    """MoG2-TV with s1 = s2 is the Gaussian (l2) pair factor: the whole EP run,
    through the mixture code path, gives the l2 run's result."""
    h = w = 8
    rng = np.random.default_rng(3)
    y = syn.piecewise_image(h, w, 4, rng) + 0.1 * rng.normal(size=(h, w))
    op = ops.Operator(ops.IDENTITY, (h, w))
    beta = 30.0
    a = ep.solve(ep.EPProblem(y, op, 0.01, beta, damping=0.5, prior="l2"), 30, em=False)
    b = ep.solve(ep.EPProblem(y, op, 0.01, (0.4, 1 / beta, 1 / beta), damping=0.5, prior="mog2"), 30, em=False)
    assert np.allclose(a[0], b[0], rtol=0, atol=1e-12) and np.allclose(a[1], b[1], rtol=1e-12)


def test_em_fixed_point_is_marginal_likelihood_stationary_point():
    """Single edge: EP is exact, so fast EP-EM converges to a local maximiser of
    log f(y | lambda) = N log(lambda) + log int N(u; y1 - y2, 2 xi) e^{-lambda |u|} du
    + const, with N = 2 pixels (Sec. IV, C(lambda) ~ lambda^-N)."""
    y = np.array([[0.6, -0.4]])
    xi = 0.01
    d = y[0, 0] - y[0, 1]
    pb = ep.EPProblem(y, ops.Operator(ops.IDENTITY, (1, 2)), xi, 3.0, damping=1.0)
    mu, v, st, info = ep.solve(pb, 500, em=True, tol=1e-13)
    lam_ep = st.lam

    def neg_loglik(loglam):
        lam = math.exp(loglam)
        f = lambda u: math.exp(-(u - d) ** 2 / (4 * xi) - lam * abs(u))
        Z = integrate.quad(f, -np.inf, 0, epsabs=0, epsrel=1e-13)[0] + \
            integrate.quad(f, 0, np.inf, epsabs=0, epsrel=1e-13, points=None)[0]
        return -(2 * loglam + math.log(Z))
    res = optimize.minimize_scalar(neg_loglik, bracket=(math.log(0.5), math.log(3.0), math.log(8.0)),
                                   tol=1e-12)
    lam_ml = math.exp(res.x)
    assert abs(lam_ep / lam_ml - 1) < 1e-6, (lam_ep, lam_ml)


def _small_problem(kind, h=8, w=10, seed=3):
    rng = np.random.default_rng(seed)
    x = syn.piecewise_image(h, w, 4, rng)
    if kind == ops.IDENTITY:
        op = ops.Operator(kind, (h, w))
        y = x + 0.1 * rng.normal(size=(h, w))
    else:
        op = ops.Operator(kind, (h, w), taps=syn.gaussian_taps(1.2, 5))
        y = op.H(x) + 0.05 * rng.normal(size=(h, w))
    return y, op


@pytest.mark.parametrize("kind", [ops.IDENTITY, ops.BLUR])
def test_sign_flip_invariance(kind):
    y, op = _small_problem(kind)
    a = ep.solve(ep.EPProblem(y, op, 0.01, 4.0), 30, em=True)
    b = ep.solve(ep.EPProblem(-y, op, 0.01, 4.0), 30, em=True)
    assert np.allclose(a[0], -b[0], rtol=0, atol=1e-12)
    assert np.allclose(a[1], b[1], rtol=1e-11)


@pytest.mark.parametrize("kind", [ops.IDENTITY, ops.BLUR])
def test_rotation_invariance(kind):
    y, op = _small_problem(kind)
    if kind == ops.BLUR:
        op_r = ops.Operator(kind, op.shape, taps=op.taps[::-1, ::-1])
    else:
        op_r = op
    a = ep.solve(ep.EPProblem(y, op, 0.01, 4.0), 30, em=True)
    b = ep.solve(ep.EPProblem(y[::-1, ::-1].copy(), op_r, 0.01, 4.0), 30, em=True)
    assert np.allclose(a[0], b[0][::-1, ::-1], rtol=0, atol=1e-11)
    assert np.allclose(a[1], b[1][::-1, ::-1], rtol=1e-10)


def test_transpose_with_block_order():
    y, op = _small_problem(ops.IDENTITY, 8, 10)
    a = ep.solve(ep.EPProblem(y, op, 0.01, 4.0, order=(1, 2, 3, 4)), 25, em=True)
    b = ep.solve(ep.EPProblem(y.T.copy(), ops.Operator(ops.IDENTITY, (10, 8)), 0.01, 4.0,
                              order=(3, 4, 1, 2)), 25, em=True)
    assert np.allclose(a[0], b[0].T, rtol=0, atol=1e-12)
    assert np.allclose(a[1], b[1].T, rtol=1e-11)


def test_likelihood_site_is_noop_for_identity():
    y, op = _small_problem(ops.IDENTITY)
    pb = ep.EPProblem(y, op, 0.02, 4.0, damping=1.0)
    st = ep.init_cold(pb)
    for k in (1, 2, 3, 4):
        ep.tv_block_update(pb, st, k)
    tau0, eta0 = st.tau[0].copy(), st.eta[0].copy()
    ep.likelihood_site_update(pb, st)
    assert np.allclose(st.tau[0], tau0, rtol=1e-12)
    assert np.allclose(st.eta[0], eta0, rtol=1e-10, atol=1e-10)


def test_uncovered_sites_stay_flat_and_l1_never_clamps_negative():
    y, op = _small_problem(ops.IDENTITY, 5, 7)
    pb = ep.EPProblem(y, op, 0.01, 8.0)
    mu, v, st, _ = ep.solve(pb, 20, em=False)
    for k in range(4):
        unc = ~pb.covered[k]
        assert np.all(st.tau[k + 1, unc] == 0) and np.all(st.eta[k + 1, unc] == 0)
        assert np.all(st.tau[k + 1, ~unc] > 0)
    # global = sum of sites
    assert np.allclose(1 / v.ravel(), st.tau.sum(0))


def test_em_fixed_point_identity():
    """At convergence of fast EP-EM, lambda = N / a_bar_u of the last sweep."""
    y, op = _small_problem(ops.IDENTITY, 10, 10)
    pb = ep.EPProblem(y, op, 0.01, 1.0)
    mu, v, st, info = ep.solve(pb, 3000, em=True, tol=1e-12)
    assert info["converged"]
    a_bar = sum(ep.tv_block_update(pb, st, k) for k in (1, 2, 3, 4))
    assert abs(pb.N / a_bar / st.lam - 1) < 1e-9


def test_hadamard_full_mask_equals_denoising_of_back_projection():
    """With every Walsh coefficient kept, H is orthonormal (H^T H = I) and the
    EP problem is denoising of H^T y with the same noise: the Hadamard path of
    the oracle (CG solve, spectral variance) must give the identity path's
    result."""
    p = syn.make_hadamard_cs(16, 16, 3, 0.05, 1.0, np.random.default_rng(18), lam0=8.0,
                             sweeps=12, em=False)
    assert p.mask.all()
    pb = ep.problem_from_synthetic(p)
    mu_h, v_h, _, _ = ep.solve(pb, 12, False)
    q = syn.make_denoise(16, 16, 3, 0.05, np.random.default_rng(0), lam0=8.0, sweeps=12, em=False)
    q.y = ops.Operator(ops.HADAMARD, p.shape, mask=p.mask).Ht(p.y)
    q.xi = p.xi
    pd = ep.problem_from_synthetic(q)
    mu_d, v_d, _, _ = ep.solve(pd, 12, False)
    assert np.allclose(mu_h, mu_d, rtol=0, atol=1e-9)
    assert np.allclose(v_h, v_d, rtol=1e-8, atol=0)


def _order_case(kind, n):
    rng = syn.rng_for(7, n)
    if kind == "blur":
        return syn.make_deconv(n, n, 4, 0.01, 2.0, rng, lam0=10.0)
    return syn.make_cs(n, n, 4, 0.005, 0.25, rng, lam0=10.0)


@pytest.mark.parametrize("kind,n,em", [("blur", 8, False), ("blur", 16, False), ("blur", 8, True),
                                       ("dft", 8, False), ("dft", 16, False)])
def test_first_sweep_order_reaches_the_same_fixed_point(kind, n, em):
    """Reading of the first sweep of a cold start: the oracle lets the initial
    likelihood factor (mean y, variance xi) stand in for the first likelihood
    update and runs the first CG in sweep 2; Algorithm 1's loop body taken
    literally runs the likelihood update at t = 1 as well.  Both orders must
    converge (FP64, tol 1e-12) to the same EP fixed point, so the reading
    changes the trajectory of a fixed number of sweeps, not the answer."""
    p = _order_case(kind, n)
    runs = []
    for literal in (False, True):
        pb = ep.problem_from_synthetic(p)
        pb.first_sweep_likelihood = literal
        mu, v, st, info = ep.solve(pb, 3000, em, tol=1e-12, record=True)
        assert info["converged"] and not info["diverged"]
        # the literal order really solves for E in sweep 1
        assert (st.history[0]["cg"] > 0) == literal
        runs.append((mu, v, info))
    (mu_a, v_a, ia), (mu_b, v_b, ib) = runs
    scale = mu_a.max() - mu_a.min()
    assert np.max(np.abs(mu_a - mu_b)) <= 1e-9 * scale
    assert np.max(np.abs(v_a / v_b - 1)) <= 1e-9
    if em:
        assert abs(ia["lam"] / ib["lam"] - 1) <= 1e-9


def test_convergence_rule_reference_marginal():
    """The convergence rule's change is the one the colour-class updates make:
    a sweep that updates the likelihood site records the marginal right after
    that update, and the recorded history's dmu is measured from it; a sweep
    that does not (identity operator, first cold sweep) measures from the
    previous sweep's end.  Checked by recomputing both from the states."""
    rng = syn.rng_for(95, 0)
    p = syn.make_deconv(16, 12, 3, 0.05, 1.0, rng, lam0=2.0, sweeps=3, em=False)
    pb = ep.problem_from_synthetic(p)
    st = ep.init_cold(pb)
    yrange = float(pb.y.max() - pb.y.min())
    mu0, _ = ep.marginals(st)
    ep.sweep(pb, st, 1, False)                 # first cold sweep: no likelihood update
    assert st.mid is None
    mu1, _ = ep.marginals(st)
    ep.sweep(pb, st, 2, False)
    assert st.mid is not None
    mid_mu, _ = st.mid
    mu2, _ = ep.marginals(st)
    assert not np.allclose(mid_mu, mu1)         # the likelihood update moved the marginal
    # solve() from the same start reports the same two changes
    _, _, st2, info = ep.solve(ep.problem_from_synthetic(p), 2, False, tol=0.0, record=True)
    h = st2.history
    assert math.isclose(h[0]["dmu"], float(np.max(np.abs(mu1 - mu0))) / yrange, rel_tol=1e-12)
    assert math.isclose(h[1]["dmu"], float(np.max(np.abs(mu2 - mid_mu))) / yrange, rel_tol=1e-12)
    # an identity operator never records one
    q = syn.make_denoise(10, 9, 3, 0.1, syn.rng_for(95, 1), lam0=3.0, sweeps=2, em=False)
    sq = ep.init_cold(ep.problem_from_synthetic(q))
    ep.sweep(ep.problem_from_synthetic(q), sq, 2, False)
    assert sq.mid is None
