"""What the trained warm-start network gains over plain EP-EM: on a held-out
deconvolution instance of the training family (9 x 9 Gaussian blur sigma_b = 2,
noise sigma = 0.01, seed not used in training), EP started from the network's
prediction reaches the convergence rule in fewer sweeps and less wall time than
the cold start, and both results agree with a cold run at a 100x tighter
tolerance to the parity tolerances."""
import time

import numpy as np
import pytest

import synthetic as syn
from tests.gpu_util import MEAN_TOL, VAR_TOL

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2110_01585_amd import Context, Net, load_weights, spec_from_synthetic  # noqa: E402
from paper_2110_01585_amd import _native as N  # noqa: E402

TOL = 1e-5


def _solve(ctx, shape, tol, max_sweeps):
    mu = torch.empty(*shape, device="cuda")
    var = torch.empty(*shape, device="cuda")
    rc, st = ctx.ep_tv_solve(max_sweeps, tol, True, [mu], [var])
    return mu, var, st[0]


@pytest.mark.parametrize("size,seed", [(512, 1), (1024, 2)])
def test_warm_start_gain(size, seed):
    params, meta = load_weights()
    p = syn.config4_test(seed=seed, size=size)
    y = torch.tensor(p.y, dtype=torch.float32, device="cuda")
    ctx = Context([spec_from_synthetic(p)])
    ctx.ep_tv_set_observation([y])
    net = Net(params, max_batch=1, max_h=size, max_w=size)
    mh, vh = net.infer(y, p.xi)                 # warm-up
    ctx.ep_tv_solve(3, 0.0, True)               # warm-up of the EP kernels
    # cold
    ctx.ep_tv_init_cold()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mu_c, v_c, st_c = _solve(ctx, p.shape, TOL, 2000)
    torch.cuda.synchronize()
    t_cold = time.perf_counter() - t0
    # warm: inference + site initialisation + EP, all inside the timed region
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mh, vh = net.infer(y, p.xi)
    rc = ctx.ep_tv_init_warm([mh], [vh], meta["lambda_scale"], meta.get("lambda_power", 1.0))
    mu_w, v_w, st_w = _solve(ctx, p.shape, TOL, 2000)
    torch.cuda.synchronize()
    t_warm = time.perf_counter() - t0
    # reference: cold at a 100x tighter tolerance
    ctx.ep_tv_init_cold()
    mu_r, v_r, st_r = _solve(ctx, p.shape, TOL / 100, 1500)
    torch.cuda.synchronize()
    rng = float(mu_r.max() - mu_r.min())
    errs = {}
    for tag, m_, v_ in (("cold", mu_c, v_c), ("warm", mu_w, v_w)):
        errs[tag] = (float((m_ - mu_r).abs().max()) / rng, float((v_ / v_r - 1).abs().max()))
    print(f"{size}^2: cold {st_c['sweeps']} sweeps {t_cold:.3f} s | warm {st_w['sweeps']} sweeps "
          f"{t_warm:.3f} s | tight {st_r['sweeps']} sweeps (converged {st_r['converged']}) | errs {errs}")
    ctx.close()
    net.close()
    assert rc == N.EP_TV_OK
    assert st_c["converged"] and st_w["converged"]
    assert st_w["sweeps"] < st_c["sweeps"]
    assert t_warm < t_cold
    for tag in ("cold", "warm"):
        assert errs[tag][0] <= MEAN_TOL and errs[tag][1] <= VAR_TOL, tag
