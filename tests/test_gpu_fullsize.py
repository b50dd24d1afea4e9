"""Full-size checks of the GPU path in the configuration the benchmark uses
(graph launches).  Properties that hold at any size, exactly:

* negating the observation negates every mean and leaves every variance
  unchanged (all EP updates and the linear likelihood-site solve are odd in y;
  IEEE arithmetic is symmetric under sign changes), bit for bit, for the
  512^2 deconvolution and the 1024^2 compressive-sensing workloads;
* for denoising at fixed lambda with even sizes, rotating the observation by
  180 degrees rotates the result bit for bit (the rotation maps each colour
  class onto itself with the roles of the two pixels of a pair swapped, and
  the pair update is symmetric under that swap);
* stored FP64-oracle references of the full 512^2 deconvolution (200 sweeps)
  and 1024^2 compressive-sensing (300 sweeps) runs, written by
  tests/golden/make_golden.py, at sampled pixels."""
import json
import os

import numpy as np
import pytest

import synthetic as syn
from tests.gpu_util import MEAN_TOL, VAR_TOL, observation_tensor

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2110_01585_amd import Context, spec_from_synthetic  # noqa: E402
from paper_2110_01585_amd import _native as N  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _solve(p, y_tensor, sweeps, em, graph=True):
    ctx = Context([spec_from_synthetic(p)])
    ctx.ep_tv_set_option(N.OPT_GRAPH, 1 if graph else 0)
    ctx.ep_tv_set_observation([y_tensor])
    ctx.ep_tv_run(sweeps, em)
    mus, vs = ctx.marginals()
    st = ctx.ep_tv_get_stats()[0]
    torch.cuda.synchronize()
    out = mus[0].cpu().numpy(), vs[0].cpu().numpy(), st
    ctx.close()
    return out


@pytest.mark.parametrize("which,sweeps", [("deconv512", 40), ("cs1024", 30)])
def test_sign_flip_is_exact(which, sweeps):
    p = syn.config1() if which == "deconv512" else syn.config2()
    y = observation_tensor(p, torch)
    m1, v1, s1 = _solve(p, y, sweeps, True)
    m2, v2, s2 = _solve(p, -y, sweeps, True)
    assert np.array_equal(m1, -m2) and np.array_equal(v1, v2)
    assert s1["lambda"] == s2["lambda"]


def test_rotation_is_exact_for_denoising():
    rng = syn.rng_for(97, 0)
    p = syn.make_denoise(1024, 512, 200, 0.1, rng, mode="paint", lam0=8.0, sweeps=30, em=False)
    y = torch.tensor(p.y, dtype=torch.float32, device="cuda")
    m1, v1, _ = _solve(p, y, 30, False)
    m2, v2, _ = _solve(p, torch.flip(y, dims=(0, 1)).contiguous(), 30, False)
    assert np.array_equal(m1, m2[::-1, ::-1]) and np.array_equal(v1, v2[::-1, ::-1])


@pytest.mark.parametrize("which", ["deconv512", "cs1024"])
def test_full_size_against_stored_oracle(which):
    path = os.path.join(GOLDEN, f"{which}.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} has not been generated")
    ref = json.load(open(path))
    p = syn.config1() if which == "deconv512" else syn.config2()
    assert list(p.shape) == ref["shape"] and p.sweeps == ref["sweeps"]
    m, v, st = _solve(p, observation_tensor(p, torch), p.sweeps, p.em)
    idx = np.array(ref["pixels"])
    mg = m[idx[:, 0], idx[:, 1]].astype(np.float64)
    vg = v[idx[:, 0], idx[:, 1]].astype(np.float64)
    e_mu = np.max(np.abs(mg - np.array(ref["mu"]))) / ref["mu_range"]
    e_v = np.max(np.abs(vg / np.array(ref["var"]) - 1))
    print(f"{which}: sampled mean err {e_mu:.2e}, var err {e_v:.2e}, lambda gpu {st['lambda']:.8g} "
          f"oracle {ref['lambda']:.8g}")
    assert e_mu <= MEAN_TOL and e_v <= VAR_TOL
    assert abs(st["lambda"] / ref["lambda"] - 1) <= 2e-4
