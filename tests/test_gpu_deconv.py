"""GPU parity of the deconvolution path (periodic blur: likelihood site by CG with
the spectral variance estimator, then the colour-class sweep, EM) against the
FP64 oracle, through the C ABI."""
import numpy as np
import pytest

import synthetic as syn
from oracle import ep as oep
from tests.gpu_util import MEAN_TOL, VAR_TOL, f32_problem, mean_err, observation_tensor, var_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2110_01585_amd import Context, spec_from_synthetic  # noqa: E402


def _gpu(problems, sweeps, em, lam0=None):
    ctx = Context([spec_from_synthetic(p, lam0=lam0) for p in problems])
    ctx.ep_tv_set_observation([observation_tensor(p, torch) for p in problems])
    ctx.ep_tv_run(sweeps, em)
    mus, vs = ctx.marginals()
    st = ctx.ep_tv_get_stats()
    torch.cuda.synchronize()
    out = [(m.cpu().numpy().astype(np.float64), v.cpu().numpy().astype(np.float64)) for m, v in zip(mus, vs)]
    ctx.close()
    return out, st


def _check(p, sweeps, em, lam_tol=2e-4):
    (res,), st = _gpu([p], sweeps, em)
    pb = oep.problem_from_synthetic(f32_problem(p))
    mu_o, v_o, ost, info = oep.solve(pb, sweeps, em)
    e_mu, e_v = mean_err(res[0], mu_o), var_err(res[1], v_o)
    print(f"{p.name} {p.shape} sweeps={sweeps}: mean err {e_mu:.2e} var err {e_v:.2e} "
          f"lambda gpu {st[0]['lambda']:.6g} oracle {info['lam']:.6g} cg_last {st[0]['cg_last']} "
          f"cg_total {st[0]['cg_total']} (oracle last {ost.cg_iters})")
    assert e_mu <= MEAN_TOL and e_v <= VAR_TOL
    if em:
        assert abs(st[0]["lambda"] / info["lam"] - 1) <= lam_tol
    return st


@pytest.mark.parametrize("size,sweeps", [(64, 40), (96, 60)])
def test_deconv_square(size, sweeps):
    p = syn.config1(size=size, sweeps=sweeps)
    _check(p, sweeps, True)


def test_deconv_config1_reduced_200_sweeps():
    """The deconvolution workload's operator, noise and schedule at 128^2."""
    p = syn.config1(size=128, sweeps=200)
    st = _check(p, 200, True)
    assert st[0]["sweeps"] == 200


@pytest.mark.parametrize("h,w", [(50, 77), (33, 130), (70, 9)])
def test_deconv_ragged(h, w):
    rng = syn.rng_for(70, h * 1000 + w)
    p = syn.make_deconv(h, w, 6, 0.02, 1.5, rng, lam0=2.0, sweeps=30, em=True)
    _check(p, 30, True)


def test_deconv_periodic_boundary():
    rng = syn.rng_for(71, 0)
    p = syn.make_deconv(64, 96, 8, 0.02, 1.3, rng, lam0=3.0, sweeps=30, em=True)
    p.boundary = "periodic"
    _check(p, 30, True)


def test_deconv_non_separable_taps():
    """General (rank > 1) taps take the two-pass H then H^T path."""
    rng = syn.rng_for(72, 0)
    p = syn.make_deconv(48, 40, 5, 0.02, 1.0, rng, lam0=2.0, sweeps=25, em=True)
    taps = np.abs(rng.normal(size=(5, 3))) + 0.1
    taps[1, 2] += 1.0
    taps /= taps.sum()
    p.taps = taps
    p.y = syn._circular_blur_fft(p.x_true, taps) + 0.02 * rng.standard_normal(p.shape)
    _check(p, 25, True)


def test_deconv_fixed_lambda_and_wide_taps():
    rng = syn.rng_for(73, 0)
    p = syn.make_deconv(80, 72, 6, 0.03, 3.0, rng, lam0=20.0, sweeps=30, em=False, ksize=15)
    _check(p, 30, False)


def test_mixed_batch_denoise_and_deconv():
    ps = [syn.make_deconv(64, 64, 5, 0.02, 2.0, syn.rng_for(74, 0), sweeps=20, em=True),
          syn.make_denoise(40, 90, 6, 0.05, syn.rng_for(74, 1), mode="paint", lam0=2.0, sweeps=20,
                           em=True),
          syn.make_deconv(45, 33, 4, 0.05, 1.2, syn.rng_for(74, 2), sweeps=20, em=True)]
    outs, st = _gpu(ps, 20, True)
    for p, (mu, v), s in zip(ps, outs, st):
        mu_o, v_o, _, info = oep.solve(oep.problem_from_synthetic(f32_problem(p)), 20, True)
        assert mean_err(mu, mu_o) <= MEAN_TOL and var_err(v, v_o) <= VAR_TOL, p.name
        assert abs(s["lambda"] / info["lam"] - 1) <= 2e-4
