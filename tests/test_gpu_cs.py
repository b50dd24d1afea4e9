"""GPU parity of the compressive-sensing path (masked orthonormal 2-D DFT, the
hand-written FFT, CG, spectral variance) against the FP64 oracle."""
import numpy as np
import pytest

import synthetic as syn
from oracle import ep as oep
from tests.gpu_util import MEAN_TOL, VAR_TOL, f32_problem, mean_err, observation_tensor, var_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2110_01585_amd import Context, spec_from_synthetic  # noqa: E402


def _check(p, sweeps, em):
    ctx = Context([spec_from_synthetic(p)])
    ctx.ep_tv_set_observation([observation_tensor(p, torch)])
    ctx.ep_tv_run(sweeps, em)
    mus, vs = ctx.marginals()
    st = ctx.ep_tv_get_stats()[0]
    torch.cuda.synchronize()
    mu, v = mus[0].cpu().numpy().astype(np.float64), vs[0].cpu().numpy().astype(np.float64)
    ctx.close()
    pb = oep.problem_from_synthetic(f32_problem(p))
    mu_o, v_o, ost, info = oep.solve(pb, sweeps, em)
    e_mu, e_v = mean_err(mu, mu_o), var_err(v, v_o)
    print(f"{p.name} {p.shape} sweeps={sweeps}: mean err {e_mu:.2e} var err {e_v:.2e} lambda gpu "
          f"{st['lambda']:.6g} oracle {info['lam']:.6g} cg_last {st['cg_last']} cg_total "
          f"{st['cg_total']} (oracle last {ost.cg_iters})")
    assert e_mu <= MEAN_TOL and e_v <= VAR_TOL
    if em:
        assert abs(st["lambda"] / info["lam"] - 1) <= 2e-4
    return st


@pytest.mark.parametrize("h,w,sweeps", [(16, 16, 20), (32, 64, 30), (64, 32, 30), (128, 128, 40)])
def test_cs_small(h, w, sweeps):
    rng = syn.rng_for(80, h * 1000 + w)
    p = syn.make_cs(h, w, max(3, h * w // 2000), 0.01, 0.3, rng, sweeps=sweeps, em=True)
    _check(p, sweeps, True)


def test_cs_config2_reduced():
    """The CS workload's mask density, noise and schedule at 128^2 (300 sweeps)."""
    p = syn.config2(size=128, sweeps=300)
    _check(p, 300, True)


def test_cs_fixed_lambda():
    rng = syn.rng_for(81, 0)
    p = syn.make_cs(64, 64, 6, 0.02, 0.25, rng, lam0=40.0, sweeps=25, em=False)
    _check(p, 25, False)
