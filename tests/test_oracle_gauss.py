"""Pins for the Gaussian i.i.d. compressive-sensing operator of the oracle and
its Woodbury moments (Sec. II-A case (iii), Sec. III-C, Sec. V):

* H and H^T are adjoint, H^T H = H^T(H(.));
* the Woodbury mean and diagonal equal a dense solve and the diagonal of the
  dense inverse of H^T H / xi + diag(tau_c), with tau_c spanning eleven decades
  (flat TV cavities at the 1e-8 floor next to sharp ones), where the
  subtraction 1/d - |z|^2/d^2 is the delicate part;
* EP with an l2 (Gaussian) pair factor reaches the exact posterior mean, the
  dense solve of (H^T H / xi + beta L) mu = H^T y / xi."""
import numpy as np
import pytest

import synthetic as syn
from oracle import ep
from oracle import operators as ops


def _gauss(h=6, w=8, frac=0.3, seed=0):
    rng = np.random.default_rng(seed)
    p = syn.make_gauss_cs(h, w, 3, 0.05, frac, rng, lam0=6.0)
    return p, ops.Operator(ops.GAUSS, (h, w), sense=p.sense)


def test_adjoint_and_normal_operator():
    p, op = _gauss()
    rng = np.random.default_rng(1)
    x = rng.normal(size=op.shape)
    v = rng.normal(size=p.sense.shape[0])
    assert abs(np.dot(op.H(x), v) - np.sum(x * op.Ht(v))) <= 1e-12 * np.abs(x).sum() * np.abs(v).sum()
    assert np.allclose(op.HtH(x), op.Ht(op.H(x)), rtol=1e-14, atol=0)
    assert p.sense.dtype == np.float64 and np.array_equal(p.sense.astype(np.float32).astype(np.float64),
                                                          p.sense)


@pytest.mark.parametrize("frac,seed", [(0.3, 2), (0.1, 3), (0.9, 4)])
def test_woodbury_equals_dense_inverse(frac, seed):
    """Reference: the dense inverse in 40-digit arithmetic (mpmath); A has a
    condition number near 1e12 here, beyond what an FP64 dense inverse resolves.
    The Woodbury form itself loses digits in FP64 as S = xi I + H D^-1 H^T
    grows ill-conditioned (up to 1.4e-6 relative at M / N = 0.9 with d down to
    1e-8), so the bound is 1e-5: a wrong term or scale is off by orders of
    magnitude more."""
    import mpmath as mp
    p, op = _gauss(5, 6, frac=frac, seed=seed)
    rng = np.random.default_rng(seed + 10)
    xi = 1e-4
    tau_c = 10.0 ** rng.uniform(-8, 3, size=op.shape)
    b = rng.normal(size=op.shape) * 100
    E, v = ops.woodbury_moments(op, xi, tau_c, b)
    mp.mp.dps = 40
    H = mp.matrix(p.sense.tolist())
    A = (H.T * H) / mp.mpf(xi) + mp.diag([mp.mpf(float(t)) for t in tau_c.ravel()])
    Ainv = mp.inverse(A)
    n = op.shape[0] * op.shape[1]
    v_ref = np.array([float(Ainv[i, i]) for i in range(n)])
    E_ref = np.array([float(x) for x in Ainv * mp.matrix(b.ravel().tolist())]).reshape(op.shape)
    assert np.allclose(v.ravel(), v_ref, rtol=1e-5, atol=0)
    assert np.max(np.abs(E - E_ref)) <= 1e-6 * np.max(np.abs(E_ref))
    assert np.allclose(ops.tilted_variance(op, xi, tau_c), v, rtol=0, atol=0)


def test_l2_fixed_point_is_dense_posterior_mean_gauss():
    h, w = 6, 7
    p, op = _gauss(h, w, 0.4, seed=5)
    xi, beta = p.xi, 20.0
    pb = ep.EPProblem(p.y, op, xi, beta, damping=0.5, prior="l2")
    mu, v, st, info = ep.solve(pb, 4000, em=False, tol=1e-14)
    L = np.zeros((h * w, h * w))
    for r in range(h):
        for c in range(w):
            for (r2, c2) in ((r, c + 1), (r + 1, c)):
                if r2 < h and c2 < w:
                    a, b2 = r * w + c, r2 * w + c2
                    L[a, a] += 1; L[b2, b2] += 1; L[a, b2] -= 1; L[b2, a] -= 1
    A = op.dense_HtH() / xi + beta * L
    mu_ref = np.linalg.solve(A, op.Ht(p.y).ravel() / xi).reshape(h, w)
    assert np.max(np.abs(mu - mu_ref)) <= 1e-9 * (mu_ref.max() - mu_ref.min())


def test_l1_gauss_cs_runs_and_is_sign_symmetric():
    p, op = _gauss(8, 8, 0.3, seed=6)
    a = ep.solve(ep.problem_from_synthetic(p), 20, True)
    q = syn.make_gauss_cs(8, 8, 3, 0.05, 0.3, np.random.default_rng(6), lam0=6.0)
    q.y = -p.y
    b = ep.solve(ep.problem_from_synthetic(q), 20, True)
    assert not a[3]["diverged"]
    assert np.allclose(a[0], -b[0], rtol=0, atol=1e-11) and np.allclose(a[1], b[1], rtol=1e-10)
