"""The MoG2-TV (Eq. (MoG2_TV_prior)) and BG-TV (Eq. (BG_TV)) pixel-difference
factors on the GPU against the FP64 oracle:

* the device tilted moments (Sec. III-C) over cavity variances 1e-6..1 and
  |m| / sigma 1e-4..1e2 of either sign, for both mixtures; the l1 factor through
  the general entry point is bit-identical to the l1 entry point;
* the moments of -m mirror those of m exactly;
* whole EP runs at fixed hyperparameters: 64^2 denoising with each mixture and
  64^2 deconvolution with MoG2 (circulant-preconditioned CG), to the parity
  bar of the l1 runs.  BG-TV is compared after 10 sweeps: its EP iteration is
  not log-concave and amplifies rounding, so that the oracle run on an
  observation perturbed by 1e-7 (relative) already moves by 5e-6 in variance
  after 10 sweeps but by 0.1 after 30 (MoG2-TV: 1.4e-6 at 30);
* EM (defined for the l1 factor only) and contexts mixing factor kinds are
  rejected.

Tolerances: rho absolute 2e-5 (1e-5 relative beyond |rho| = 1, where the
mixture's two components are far apart and rho is a large negative number),
delta 2e-5 sigma.  The FP32 evaluation rounds the log weight d (a sum of three
terms of moderate size) and the two reciprocals; measured maxima are printed."""
import numpy as np
import pytest

import synthetic as syn
from oracle import ep as oep
from oracle import tilted as OT
from tests.gpu_util import MEAN_TOL, VAR_TOL, f32_problem, mean_err, observation_tensor, var_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2110_01585_amd import (Context, EPTVError, ProblemSpec, ep_tv_tilted_moments,  # noqa: E402
                                  ep_tv_tilted_moments_prior, spec_from_synthetic)
from paper_2110_01585_amd import _native as N  # noqa: E402

MOG2 = (0.1, 0.25, 1e-3)     # omega, s1^2 (object boundaries), s2^2 (flat regions)
BG = (0.5, 0.25)             # omega, s^2


def _draws(seed, n=100_000):
    rng = np.random.default_rng(seed)
    s = 10.0 ** rng.uniform(-6, 0, n)
    m = np.sqrt(s) * rng.choice([1.0, -1.0], n) * 10.0 ** rng.uniform(-4, 2, n)
    return m.astype(np.float32), s.astype(np.float32)


def _gpu_moments(prior, theta, m, s):
    rho, de, ea = ep_tv_tilted_moments_prior(prior, theta, torch.tensor(m, device="cuda"),
                                             torch.tensor(s, device="cuda"))
    torch.cuda.synchronize()
    return rho.cpu().numpy().astype(np.float64), de.cpu().numpy().astype(np.float64), ea.cpu().numpy()


@pytest.mark.parametrize("prior,theta,fn", [(N.PRIOR_MOG2, MOG2, OT.mog2_tilted), (N.PRIOR_BG, BG, OT.bg_tilted)])
def test_mixture_moments_against_oracle(prior, theta, fn):
    m, s = _draws(1 + prior)
    rho, de, ea = _gpu_moments(prior, theta, m, s)
    m64, s64 = m.astype(np.float64), s.astype(np.float64)
    mb, Sb, _ = fn(m64, s64, theta)
    rho_o = 1.0 - Sb / s64
    e_rho = np.max(np.abs(rho - rho_o) / np.maximum(1.0, np.abs(rho_o)))
    e_de = np.max(np.abs(de - (mb - m64)) / np.sqrt(s64))
    print(f"prior {prior}: rho err {e_rho:.2e}, delta err {e_de:.2e} sigma, rho range "
          f"{rho_o.min():.3g}..{rho_o.max():.3g}")
    assert np.all(np.isfinite(rho)) and np.all(np.isfinite(de)) and np.all(ea == 0.0)
    assert e_rho <= 2e-5
    assert e_de <= 2e-5


def test_general_entry_point_l1_is_the_l1_entry_point():
    m, s = _draws(9, 20_000)
    a = ep_tv_tilted_moments(torch.tensor(m, device="cuda"), torch.tensor(s, device="cuda"), 7.5)
    b = ep_tv_tilted_moments_prior(N.PRIOR_L1, (7.5,), torch.tensor(m, device="cuda"),
                                   torch.tensor(s, device="cuda"))
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert torch.equal(x, y)


@pytest.mark.parametrize("prior,theta", [(N.PRIOR_MOG2, MOG2), (N.PRIOR_BG, BG)])
def test_mixture_mirror_symmetry_is_exact(prior, theta):
    m, s = _draws(20 + prior, 30_000)
    r1, d1, _ = _gpu_moments(prior, theta, m, s)
    r2, d2, _ = _gpu_moments(prior, theta, -m, s)
    assert np.array_equal(r1, r2) and np.array_equal(d1, -d2)


def _spec(p, prior, theta):
    sp = spec_from_synthetic(p)
    sp.prior = prior
    sp.prior_omega = theta[0]
    sp.prior_s1sq = theta[1]
    sp.prior_s2sq = theta[2] if len(theta) > 2 else 0.0
    return sp


def _run(p, prior, theta, sweeps):
    ctx = Context([_spec(p, prior, theta)])
    ctx.ep_tv_set_observation([observation_tensor(p, torch)])
    ctx.ep_tv_set_option(N.OPT_GRAPH, 1)
    ctx.ep_tv_init_cold()
    ctx.ep_tv_run(sweeps, False)
    mus, vs = ctx.marginals()
    st = ctx.ep_tv_get_stats()[0]
    torch.cuda.synchronize()
    out = mus[0].cpu().numpy().astype(np.float64), vs[0].cpu().numpy().astype(np.float64), st
    ctx.close()
    return out


@pytest.mark.parametrize("case", ["denoise-mog2", "denoise-bg", "deconv-mog2"])
def test_mixture_ep_against_oracle(case):
    kind, name = case.split("-")
    prior, theta, oprior = ((N.PRIOR_MOG2, MOG2, "mog2") if name == "mog2" else (N.PRIOR_BG, BG, "bg"))
    if kind == "denoise":
        sweeps = 10 if name == "bg" else 30
        p = syn.config0(size=64, sweeps=sweeps)
    else:
        p = syn.config1(size=64, sweeps=40)
        sweeps = 40
    mu, v, st = _run(p, prior, theta, sweeps)
    pb = oep.problem_from_synthetic(f32_problem(p), prior=oprior, lam=theta)
    mu_o, v_o, _, _ = oep.solve(pb, sweeps, em=False)
    e_mu, e_v = mean_err(mu, mu_o), var_err(v, v_o)
    print(f"{case}: mean err {e_mu:.2e}, var err {e_v:.2e}, clamps {st['clamps']}")
    assert e_mu <= MEAN_TOL and e_v <= VAR_TOL


def test_em_and_mixed_kinds_are_rejected():
    p = syn.config0(size=32, sweeps=5)
    ctx = Context([_spec(p, N.PRIOR_MOG2, MOG2)])
    ctx.ep_tv_set_observation([observation_tensor(p, torch)])
    ctx.ep_tv_init_cold()
    with pytest.raises(EPTVError):
        ctx.ep_tv_run(2, True)
    with pytest.raises(EPTVError):
        ctx.ep_tv_em_step(1)
    ctx.ep_tv_run(2, False)
    ctx.close()
    with pytest.raises(EPTVError):
        Context([_spec(p, N.PRIOR_MOG2, MOG2), ProblemSpec(32, 32)])
