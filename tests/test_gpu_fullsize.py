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
  tests/golden/make_golden.py, at sampled pixels;
* one sweep of the 2048^2 deconvolution checked step by step against the
  oracle's update functions fed the GPU's state before each step."""
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


def test_deconv2048_one_sweep_step_by_step(monkeypatch):
    """The 2048^2 deconvolution in the benchmark's launch configuration (graph
    replay, autotuned tile height), at full size: after 30 sweeps from cold with
    EM, one more sweep at the current lambda (no EM) is checked step by step in
    FP64 against the oracle's own update functions, each fed the GPU's state
    before that step:

    * the cavity of the likelihood site (tau_c, eta_c) is the sum of the four
      TV sites before the sweep, and b = H^T y / xi + eta_c (Eq. (tilted_P_1));
    * the CG iterate E solves (H^T H / xi + diag tau_c) E = b: its true
      residual, computed in FP64, stays within the CG's target 1e-8 plus
      (2 + n) 2^-24 (|H|^2_max / xi + tau_c,max) ||E|| / ||b||, the residual of
      E rounded to float32 and the gap that n float32 iterations can open
      between the true and the recursively updated residual (about one
      u ||A|| ||E|| per iteration);
    * the likelihood site after the sweep equals the oracle's update
      (Eq. (update_q0_x), spectral variance, clamp, damping) from that E;
    * every colour class's TV sites after the sweep equal the oracle's block
      update (Sec. III-C) at 200,000 sampled factors per class, from the sites
      of the classes before it (after the sweep) and after it (before).

    Sites are compared relative to the pixel's total precision (eta: plus its
    |total eta|), at the parity bar of the means, 1e-4."""
    import types
    import oracle.ep as oep
    from oracle import operators as oops
    from tests.gpu_util import f32_problem

    p = syn.config4_test(seed=0, size=2048)
    H, W = p.shape
    ctx = Context([spec_from_synthetic(p)])
    ctx.ep_tv_set_observation([observation_tensor(p, torch)])
    ctx.ep_tv_set_option(N.OPT_GRAPH, 1)
    ctx.ep_tv_autotune(3)
    ctx.ep_tv_init_cold()
    ctx.ep_tv_run(30, True)
    pre_d = torch.empty(10, H, W, device="cuda")
    ctx.ep_tv_get_sites([pre_d])
    lam = ctx.ep_tv_get_stats()[0]["lambda"]
    ctx.ep_tv_run(1, False)
    n_it = ctx.ep_tv_get_stats()[0]["cg_last"]
    post_d = torch.empty(10, H, W, device="cuda")
    lik_d = torch.empty(10, H, W, device="cuda")
    ctx.ep_tv_get_sites([post_d])
    ctx.ep_tv_get_lik_planes(0, lik_d)
    torch.cuda.synchronize()
    pre = pre_d.cpu().numpy().astype(np.float64).reshape(5, 2, H * W)
    post = post_d.cpu().numpy().astype(np.float64).reshape(5, 2, H * W)
    lik = lik_d.cpu().numpy().astype(np.float64)
    del pre_d, post_d, lik_d
    ctx.close()

    pb = oep.problem_from_synthetic(f32_problem(p))
    E, tau_c, eta_c, b = lik[0], lik[1], lik[2], lik[3]

    # cavity of the likelihood site and the right-hand side
    tc_ref = pre[1:, 0].sum(axis=0).reshape(H, W)
    ec_ref = pre[1:, 1].sum(axis=0).reshape(H, W)
    e_tc = np.max(np.abs(tau_c - tc_ref) / tc_ref)
    e_ec = np.max(np.abs(eta_c - ec_ref) / (np.abs(pre[1:, 1]).sum(axis=0).reshape(H, W) + tc_ref))
    b_ref = pb.hty / pb.xi + eta_c
    e_b = np.max(np.abs(b - b_ref)) / np.max(np.abs(b_ref))
    # the CG solves its system
    res = pb.op.HtH(E) / pb.xi + tau_c * E - b
    rel_res = np.linalg.norm(res) / np.linalg.norm(b)
    bound = 1e-8 + (2 + n_it) * 2.0 ** -24 * (np.max(pb.op.spectrum()) / pb.xi + np.max(tau_c)) \
        * np.linalg.norm(E) / np.linalg.norm(b)

    # likelihood-site update from the GPU's E
    st = oep.EPState(tau=pre[:, 0].copy(), eta=pre[:, 1].copy(), lam=lam)
    monkeypatch.setattr(oops, "solve_tilted_mean", lambda *a, **k: (E, 0))
    oep.likelihood_site_update(pb, st)
    tau_tot = post[:, 0].sum(axis=0)
    eta_scale = np.abs(post[:, 1].sum(axis=0)) + tau_tot
    e_s0 = max(np.max(np.abs(post[0, 0] - st.tau[0]) / tau_tot),
               np.max(np.abs(post[0, 1] - st.eta[0]) / eta_scale))

    # the four colour classes, each from the GPU's sites before it
    rng = np.random.default_rng(2048)
    e_tv = []
    for k in (1, 2, 3, 4):
        i_all, j_all = pb.edges[k - 1]
        pick = rng.choice(i_all.size, 200_000, replace=False)
        sub = types.SimpleNamespace(edges=[(np.zeros(0, int), np.zeros(0, int))] * 4,
                                    prior=pb.prior, damping=pb.damping,
                                    em_option=pb.em_option, em_diagnostics=False)
        sub.edges[k - 1] = (i_all[pick], j_all[pick])
        tau = np.concatenate([post[:k, 0], pre[k:, 0]])
        eta = np.concatenate([post[:k, 1], pre[k:, 1]])
        stk = oep.EPState(tau=tau, eta=eta, lam=lam)
        oep.tv_block_update(sub, stk, k)
        px = np.concatenate([i_all[pick], j_all[pick]])
        e_tv.append(max(np.max(np.abs(post[k, 0, px] - stk.tau[k, px]) / tau_tot[px]),
                        np.max(np.abs(post[k, 1, px] - stk.eta[k, px]) / eta_scale[px])))
    print(f"2048^2 sweep: cavity {e_tc:.1e}/{e_ec:.1e}, b {e_b:.1e}, CG residual {rel_res:.2e} "
          f"(bound {bound:.2e}, {n_it} iterations), q0 {e_s0:.1e}, TV classes " + " ".join(f"{e:.1e}" for e in e_tv))
    assert e_tc <= 1e-6 and e_ec <= 1e-6
    assert e_b <= 1e-5
    assert rel_res <= bound
    assert e_s0 <= MEAN_TOL
    assert max(e_tv) <= MEAN_TOL
