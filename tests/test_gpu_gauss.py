"""GPU parity of Gaussian i.i.d. compressive sensing (a dense sensing matrix,
Sec. II-A case (iii), Sec. V): the likelihood site's Woodbury moments in FP64 on
the matrix cores (GEMM, blocked Cholesky, blocked triangular solve) against
the FP64 oracle's Woodbury moments (scipy Cholesky and triangular solve)."""
import numpy as np
import pytest

import synthetic as syn
from oracle import ep as oep
from tests.gpu_util import MEAN_TOL, VAR_TOL, f32_problem, mean_err, observation_tensor, var_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2110_01585_amd import Context, spec_from_synthetic  # noqa: E402
from paper_2110_01585_amd import _native as N  # noqa: E402


def _check(p, sweeps, em, timing=False):
    h, w = p.shape
    print(f"case gauss-cs {h}x{w} M={p.sense.shape[0]} sweeps={sweeps} em={em}", flush=True)
    ctx = Context([spec_from_synthetic(p)])
    ctx.ep_tv_set_observation([observation_tensor(p, torch)])
    if timing:
        ctx.ep_tv_set_timing(True)
    ctx.ep_tv_run(sweeps, em)
    (mu,), (v,) = ctx.marginals()
    st = ctx.ep_tv_get_stats()[0]
    tm = ctx.ep_tv_get_timing() if timing else None
    torch.cuda.synchronize()
    ctx.close()
    pb = oep.problem_from_synthetic(f32_problem(p))
    mu_o, v_o, ost, info = oep.solve(pb, sweeps, em)
    mu, v = mu.cpu().numpy().astype(np.float64), v.cpu().numpy().astype(np.float64)
    e_mu, e_v = mean_err(mu, mu_o), var_err(v, v_o)
    print(f"  mean err {e_mu:.2e} var err {e_v:.2e} lambda gpu {st['lambda']:.6g} oracle "
          f"{info['lam']:.6g} status {st['status']}", flush=True)
    if tm:
        print(f"  dgemm {tm['dgemm_ms']:.2f} ms / {tm['dgemm_launches']} launches, "
              f"{tm['dgemm_flops'] / max(tm['dgemm_ms'], 1e-9) / 1e9:.1f} TFLOP/s", flush=True)
    assert not info["diverged"]
    assert e_mu <= MEAN_TOL and e_v <= VAR_TOL
    if em:
        assert abs(st["lambda"] / info["lam"] - 1) <= 2e-4


@pytest.mark.parametrize("h,w,frac,sweeps,em", [(16, 16, 0.3, 15, False), (32, 32, 0.3, 20, True),
                                                (24, 40, 0.3, 15, True), (20, 20, 0.7, 12, True),
                                                (8, 12, 0.5, 10, True)])
def test_gauss_cs_matches_oracle(h, w, frac, sweeps, em):
    rng = syn.rng_for(89, h * 100 + w)
    p = syn.make_gauss_cs(h, w, max(3, h * w // 300), 0.01, frac, rng, lam0=1.0 if em else 10.0)
    _check(p, sweeps, em)


def test_gauss_cs_64x64_paper_ratio():
    """M / N = 0.3 and noise variance 1e-4 as in the paper's CS experiment, at
    64^2 (M = 1229, twenty Cholesky blocks, the last one partial)."""
    p = syn.make_gauss_cs(64, 64, 12, 0.01, 0.3, syn.rng_for(89, 1), lam0=1.0)
    _check(p, 8, True, timing=True)
