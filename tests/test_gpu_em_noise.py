"""GPU parity of the EM options of Sec. IV (a_0 approximated by option 1, a_x
under Q(x), or option 2, a_u under Q(u), besides the default option 3) and of
denoising with non-i.i.d. noise (one variance per pixel; Sec. III-C) against
the FP64 oracle."""
import numpy as np
import pytest

import synthetic as syn
from oracle import ep as oep
from oracle import warm as owarm
from tests.gpu_util import MEAN_TOL, VAR_TOL, f32, f32_problem, mean_err, observation_tensor, var_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2110_01585_amd import Context, EPTVError, ProblemSpec, spec_from_synthetic  # noqa: E402
from paper_2110_01585_amd import _native as N  # noqa: E402


@pytest.mark.parametrize("kind,option", [("denoise", 1), ("denoise", 2), ("deconv", 1),
                                         ("deconv", 2), ("denoise_periodic", 1)])
def test_em_options_match_oracle(kind, option):
    if kind.startswith("denoise"):
        p = syn.make_denoise(48, 64, 6, 0.1, syn.rng_for(88, option), lam0=1.0, em=True)
        if kind.endswith("periodic"):
            p.boundary = "periodic"
    else:
        p = syn.make_deconv(32, 32, 4, 0.01, 1.5, syn.rng_for(88, 10 + option), em=True)
    sweeps = 30
    print(f"case em option {option} {kind} {p.shape}", flush=True)
    ctx = Context([spec_from_synthetic(p)])
    ctx.ep_tv_set_observation([observation_tensor(p, torch)])
    ctx.ep_tv_set_option(N.OPT_EM_OPTION, option)
    assert ctx.ep_tv_get_option(N.OPT_EM_OPTION) == option
    ctx.ep_tv_run(sweeps, True)
    (mu,), (v,) = ctx.marginals()
    lam = ctx.ep_tv_get_stats()[0]["lambda"]
    torch.cuda.synchronize()
    ctx.close()
    pb = oep.problem_from_synthetic(f32_problem(p), em_option=option)
    mu_o, v_o, st, info = oep.solve(pb, sweeps, True)
    mu, v = mu.cpu().numpy().astype(np.float64), v.cpu().numpy().astype(np.float64)
    e_mu, e_v = mean_err(mu, mu_o), var_err(v, v_o)
    print(f"  mean err {e_mu:.2e} var err {e_v:.2e} lambda gpu {lam:.6g} oracle {info['lam']:.6g}",
          flush=True)
    assert e_mu <= MEAN_TOL and e_v <= VAR_TOL
    assert abs(lam / info["lam"] - 1) <= 2e-4


def _noisy(h, w, seed):
    rng = np.random.default_rng(seed)
    x = syn.piecewise_image(h, w, 5, rng)
    nv = (10.0 ** rng.uniform(-2.5, -1.0, size=(h, w))).astype(np.float32).astype(np.float64)
    y = f32(x + np.sqrt(nv) * rng.normal(size=(h, w)))
    return y, nv


@pytest.mark.parametrize("em,graph", [(False, False), (True, False), (True, True)])
def test_non_iid_noise_denoising_matches_oracle(em, graph):
    h, w = 50, 70
    y, nv = _noisy(h, w, 5)
    lam0 = 1.0 if em else 8.0
    print(f"case non-iid noise em={em} graph={graph}", flush=True)
    ctx = Context([ProblemSpec(h, w, N.OP_IDENTITY, N.BND_FREE, float(nv.mean()), lam0, 0.5,
                               noise_map=True)])
    ctx.ep_tv_set_observation([torch.tensor(y, dtype=torch.float32, device="cuda")])
    with pytest.raises(EPTVError) as e:
        ctx.ep_tv_run(1, em)
    assert e.value.code == N.EP_TV_E_STATE
    ctx.ep_tv_set_noise_variance([torch.tensor(nv, dtype=torch.float32, device="cuda")])
    if graph:
        ctx.ep_tv_set_option(N.OPT_GRAPH, 1)
    ctx.ep_tv_run(25, em)
    (mu,), (v,) = ctx.marginals()
    lam = ctx.ep_tv_get_stats()[0]["lambda"]
    torch.cuda.synchronize()
    ctx.close()
    pb = oep.EPProblem(y, oep.ops.Operator(oep.ops.IDENTITY, (h, w)), float(nv.mean()), lam0,
                       damping=0.5, noise_var_map=nv)
    mu_o, v_o, st, info = oep.solve(pb, 25, em)
    e_mu = mean_err(mu.cpu().numpy().astype(np.float64), mu_o)
    e_v = var_err(v.cpu().numpy().astype(np.float64), v_o)
    print(f"  mean err {e_mu:.2e} var err {e_v:.2e} lambda gpu {lam:.6g} oracle {info['lam']:.6g}",
          flush=True)
    assert e_mu <= MEAN_TOL and e_v <= VAR_TOL
    if em:
        assert abs(lam / info["lam"] - 1) <= 2e-4


def test_non_iid_noise_warm_start_sites():
    """The warm start keeps the exact likelihood factor (1 / xi_i, y_i / xi_i)."""
    h, w = 20, 30
    y, nv = _noisy(h, w, 6)
    rng = np.random.default_rng(7)
    mu_hat = f32(y + 0.01 * rng.normal(size=(h, w)))
    v_hat = f32(nv * rng.uniform(0.2, 0.6, size=(h, w)))
    ctx = Context([ProblemSpec(h, w, N.OP_IDENTITY, N.BND_FREE, float(nv.mean()), 3.0, 0.5,
                               noise_map=True)])
    ctx.ep_tv_set_observation([torch.tensor(y, dtype=torch.float32, device="cuda")])
    ctx.ep_tv_set_noise_variance([torch.tensor(nv, dtype=torch.float32, device="cuda")])
    ctx.ep_tv_init_warm([torch.tensor(mu_hat, dtype=torch.float32, device="cuda")],
                        [torch.tensor(v_hat, dtype=torch.float32, device="cuda")], 0.0, 1.0)
    sites = torch.empty(10 * h * w, device="cuda")
    ctx.ep_tv_get_sites([sites])
    torch.cuda.synchronize()
    ctx.close()
    s = sites.cpu().numpy().astype(np.float64).reshape(10, h * w)
    pb = oep.EPProblem(y, oep.ops.Operator(oep.ops.IDENTITY, (h, w)), float(nv.mean()), 3.0,
                       noise_var_map=nv)
    st = owarm.init_warm(pb, mu_hat, v_hat, set_lambda=False)
    tau_tot = st.tau.sum(0)
    for k in range(5):
        assert np.max(np.abs(s[2 * k] - st.tau[k]) / tau_tot) <= 1e-6
        assert np.max(np.abs(s[2 * k + 1] - st.eta[k]) / (np.abs(st.eta.sum(0)) + tau_tot)) <= 1e-6
