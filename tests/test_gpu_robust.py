"""GPU behaviour at the edges of the method: the smallest transform images,
runaways the divergence rule must flag on both sides, frozen instances, the
automatic cold restart of a failed warm start, and non-finite input.

EP has no convergence guarantee.  On small images with a sparse transform mask
the spectral variance estimator lets EP run away (tests/test_oracle_estimators.py
pins that on the CPU); the device must then report EP_TV_E_DIVERGED at the
same sweep as the oracle, not return finite, meaningless means."""
import numpy as np
import pytest

import synthetic as syn
from oracle import ep as oep
from tests.gpu_util import MEAN_TOL, VAR_TOL, f32_problem, mean_err, observation_tensor, var_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2110_01585_amd import Context, EPTVError, spec_from_synthetic  # noqa: E402
from paper_2110_01585_amd import _native as N  # noqa: E402


def _gpu(p, sweeps, em, precond=N.PRECOND_AUTO):
    ctx = Context([spec_from_synthetic(p, cg_precond=precond)])
    ctx.ep_tv_set_observation([observation_tensor(p, torch)])
    ctx.ep_tv_run(sweeps, em)
    mus, vs = ctx.marginals()
    st = ctx.ep_tv_get_stats()[0]
    torch.cuda.synchronize()
    out = mus[0].cpu().numpy().astype(np.float64), vs[0].cpu().numpy().astype(np.float64), st
    ctx.close()
    return out


def _parity(p, sweeps, em, precond=N.PRECOND_AUTO):
    print(f"case {p.name} {p.shape} sweeps={sweeps} em={em} precond={precond}", flush=True)
    mu, v, st = _gpu(p, sweeps, em, precond)
    mu_o, v_o, ost, info = oep.solve(oep.problem_from_synthetic(f32_problem(p)), sweeps, em)
    assert not info["diverged"]
    e_mu, e_v = mean_err(mu, mu_o), var_err(v, v_o)
    print(f"  mean err {e_mu:.2e} var err {e_v:.2e} lambda gpu {st['lambda']:.6g} oracle "
          f"{info['lam']:.6g} cg_last {st['cg_last']} (oracle {ost.cg_iters})", flush=True)
    assert st["status"] in (N.EP_TV_OK, N.EP_TV_W_NOT_CONVERGED)
    assert e_mu <= MEAN_TOL and e_v <= VAR_TOL
    if em:
        assert abs(st["lambda"] / info["lam"] - 1) <= 2e-4


@pytest.mark.parametrize("kind,seed,em", [("hcs", 2, False), ("hcs", 3, True), ("cs", 2, False),
                                          ("cs", 3, True)])
def test_4x4_transform_images(kind, seed, em):
    """The smallest transform images (one 4 x 4 Walsh or DFT block) on seeds the
    oracle solves without running away."""
    mk = syn.make_hadamard_cs if kind == "hcs" else syn.make_cs
    p = mk(4, 4, 3, 0.01, 0.3, syn.rng_for(96, seed), sweeps=20, em=em, lam0=1.0 if em else 10.0)
    _parity(p, 20, em)


@pytest.mark.parametrize("seed", [0, 2])
def test_8x8_hadamard_jacobi_fixed_lambda(seed):
    p = syn.make_hadamard_cs(8, 8, 3, 0.01, 0.3, syn.rng_for(97, seed), sweeps=25, em=False, lam0=10.0)
    _parity(p, 25, False, precond=N.PRECOND_JACOBI)


@pytest.mark.parametrize("kind", ["hcs", "cs"])
def test_runaway_is_flagged_like_the_oracle(kind):
    """The 4 x 4 cases the spectral estimator cannot solve: both sides stop at
    the same sweep with the divergence status."""
    if kind == "hcs":
        p = syn.make_hadamard_cs(4, 4, 3, 0.01, 0.3, syn.rng_for(90, 4004), sweeps=10, em=False,
                                 lam0=10.0)
    else:
        p = syn.make_cs(4, 4, 3, 0.01, 0.3, syn.rng_for(96, 0), sweeps=10, em=False, lam0=10.0)
    info = oep.solve(oep.problem_from_synthetic(f32_problem(p)), 60, False)[3]
    assert info["diverged"]
    print(f"case runaway {kind}: oracle diverged at sweep {info['sweeps']}", flush=True)
    ctx = Context([spec_from_synthetic(p)])
    ctx.ep_tv_set_observation([observation_tensor(p, torch)])
    mu = torch.empty(4, 4, device="cuda")
    with pytest.raises(EPTVError) as e:
        ctx.ep_tv_solve(60, 1e-6, False, [mu], None)
    assert e.value.code == N.EP_TV_E_DIVERGED
    st = ctx.ep_tv_get_stats()[0]
    ctx.close()
    assert st["status"] == N.EP_TV_E_DIVERGED
    assert st["sweeps"] == info["sweeps"]


@pytest.mark.parametrize("graph", [False, True])
def test_solve_returns_the_state_of_its_last_sweep(graph):
    """A batch where instances converge at different sweeps: every instance's
    marginals after ep_tv_solve equal those of a fresh context run for exactly
    that instance's sweep count (frozen instances carry their sites through
    the later sweeps, whatever their parity)."""
    ps = [syn.make_denoise(40 + 7 * i, 50 - 5 * i, 6, 0.1, syn.rng_for(98, i), lam0=6.0 + i, em=True)
          for i in range(3)]
    ps.append(syn.make_deconv(32, 32, 5, 0.02, 1.5, syn.rng_for(98, 7), em=True))
    ctx = Context([spec_from_synthetic(p) for p in ps])
    ctx.ep_tv_set_observation([observation_tensor(p, torch) for p in ps])
    if graph:
        ctx.ep_tv_set_option(N.OPT_GRAPH, 1)
    mus = [torch.empty(p.shape, device="cuda") for p in ps]
    vs = [torch.empty(p.shape, device="cuda") for p in ps]
    rc, st = ctx.ep_tv_solve(400, 1e-5, True, mus, vs)
    ctx.close()
    sweeps = [s["sweeps"] for s in st]
    print(f"case frozen graph={graph}: sweeps {sweeps}", flush=True)
    assert all(s["converged"] for s in st) and len(set(sweeps)) > 1
    for p, s, m, v in zip(ps, sweeps, mus, vs):
        ref = Context([spec_from_synthetic(p)])
        ref.ep_tv_set_observation([observation_tensor(p, torch)])
        ref.ep_tv_run(s, True)
        (m_r,), (v_r,) = ref.marginals()
        torch.cuda.synchronize()
        ref.close()
        assert torch.equal(m, m_r) and torch.equal(v, v_r)


def test_failed_warm_start_restarts_cold():
    """Sites restored with a NaN (a warm start): the solve detects the
    non-finite state, re-initialises the instance cold, converges, reports the
    fallback, and ends exactly where a cold solve ends."""
    p = syn.make_deconv(48, 48, 6, 0.01, 2.0, syn.rng_for(99, 0), em=True)
    y = observation_tensor(p, torch)
    tol, cap = 1e-5, 600
    ref = Context([spec_from_synthetic(p)])
    ref.ep_tv_set_observation([y])
    mu_c = torch.empty(p.shape, device="cuda")
    rc_c, st_c = ref.ep_tv_solve(cap, tol, True, [mu_c], None)
    sites = torch.empty(10 * 48 * 48, device="cuda")
    ref.ep_tv_get_sites([sites])
    torch.cuda.synchronize()
    ref.close()
    assert rc_c == N.EP_TV_OK
    bad = sites.clone()
    bad[2 * 48 * 48 + 100] = float("nan")      # eta_1 at one pixel
    ctx = Context([spec_from_synthetic(p)])
    ctx.ep_tv_set_observation([y])
    ctx.ep_tv_set_sites([bad])
    mu_w = torch.empty(p.shape, device="cuda")
    rc, st = ctx.ep_tv_solve(cap + 8, tol, True, [mu_w], None)
    ctx.close()
    print(f"case warm restart: rc {rc} status {st[0]['status']} sweeps {st[0]['sweeps']} "
          f"(cold {st_c[0]['sweeps']})", flush=True)
    assert rc == N.EP_TV_W_WARM_FALLBACK and st[0]["status"] == N.EP_TV_W_WARM_FALLBACK
    assert st[0]["cold_restarts"] == 1 and st[0]["converged"]
    assert st[0]["sweeps"] == st_c[0]["sweeps"]
    assert torch.equal(mu_w, mu_c)


@pytest.mark.parametrize("kind", ["denoise", "deconv"])
def test_nan_in_observation_is_reported(kind):
    if kind == "denoise":
        p = syn.make_denoise(32, 32, 4, 0.1, syn.rng_for(99, 1), lam0=5.0, em=False)
    else:
        p = syn.make_deconv(32, 32, 4, 0.01, 2.0, syn.rng_for(99, 2), em=True)
    y = observation_tensor(p, torch)
    y[5, 7] = float("nan")
    ctx = Context([spec_from_synthetic(p)])
    ctx.ep_tv_set_observation([y])
    with pytest.raises(EPTVError) as e:
        ctx.ep_tv_solve(40, 1e-5, kind == "deconv", None, None)
    st = ctx.ep_tv_get_stats()[0]
    ctx.close()
    print(f"case nan-in-y {kind}: status {st['status']} after {st['sweeps']} sweeps", flush=True)
    assert e.value.code == N.EP_TV_E_NONFINITE and st["status"] == N.EP_TV_E_NONFINITE
