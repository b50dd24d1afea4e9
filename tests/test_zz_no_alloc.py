"""ep_tv_denoise_noalloc (no allocation: buffers in the library's static device
array) against the workspace entry points it is a variant of
(ep_tv_create + ep_tv_set_observation + ep_tv_run + ep_tv_marginals), on two
calls in a row, the second with a smaller image, to the parity bar (means 1e-4
of the range, variances 1e-3 relative)."""
import numpy as np
import pytest

import synthetic as syn
from tests.gpu_util import MEAN_TOL, VAR_TOL, mean_err, observation_tensor, var_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2110_01585_amd import Context, EPTVError, ProblemSpec, ep_tv_denoise_noalloc  # noqa: E402
from paper_2110_01585_amd import _native as N  # noqa: E402


def _context_result(p, sweeps, em, bnd):
    h, w = p.shape
    ctx = Context([ProblemSpec(h, w, N.OP_IDENTITY, bnd, float(p.xi), float(p.lam0), float(p.damping))])
    ctx.ep_tv_set_observation([observation_tensor(p, torch)])
    ctx.ep_tv_run(sweeps, em)
    (mu,), (v,) = ctx.marginals()
    torch.cuda.synchronize()
    ctx.close()
    return mu, v


def test_noalloc_matches_workspace_path_on_two_calls():
    cases = [(syn.make_denoise(400, 300, 20, 0.1, syn.rng_for(60, 0), lam0=4.0), 30, True, N.BND_FREE),
             (syn.make_denoise(200, 150, 8, 0.05, syn.rng_for(60, 1), lam0=12.0), 20, False,
              N.BND_PERIODIC)]
    for p, sweeps, em, bnd in cases:
        h, w = p.shape
        print(f"case noalloc {h}x{w} sweeps={sweeps} em={em} boundary={bnd}", flush=True)
        y = observation_tensor(p, torch)
        mu = torch.full((h, w), float("nan"), device="cuda")
        v = torch.full((h, w), float("nan"), device="cuda")
        ep_tv_denoise_noalloc(y, p.xi, p.lam0, p.damping, sweeps, em, mu, v, boundary=bnd)
        mu_r, v_r = _context_result(p, sweeps, em, bnd)
        torch.cuda.synchronize()
        a, b = mu.cpu().numpy().astype(np.float64), mu_r.cpu().numpy().astype(np.float64)
        e_mu, e_v = mean_err(a, b), var_err(v.cpu().numpy().astype(np.float64),
                                            v_r.cpu().numpy().astype(np.float64))
        print(f"  mean err {e_mu:.2e} var err {e_v:.2e} bit-equal "
              f"{bool(torch.equal(mu, mu_r) and torch.equal(v, v_r))}", flush=True)
        assert e_mu <= MEAN_TOL and e_v <= VAR_TOL


def test_noalloc_rejects_sizes_beyond_its_array():
    y = torch.zeros(513, 8, device="cuda")
    mu, v = torch.empty_like(y), torch.empty_like(y)
    with pytest.raises(EPTVError) as e:
        ep_tv_denoise_noalloc(y, 0.01, 5.0, 0.5, 3, False, mu, v)
    assert e.value.code == N.EP_TV_E_ARG
