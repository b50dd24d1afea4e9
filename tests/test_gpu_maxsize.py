"""The largest accepted image, 16384 x 16384 (about 19 GiB of workspace),
denoised at fixed lambda (no EM) in the bench's launch configuration (graph
replay, autotuned tile height), checked at sampled pixels against the oracle
run on crops.

With the likelihood site exact and constant (H = I) and lambda fixed, one sweep
couples a pixel only with pixels a few columns or rows away (V1 then V2 along a
row, V3 then V4 along a column), so after t sweeps a pixel's marginal depends
only on the observation within 4t + 4 pixels of it (each colour class moves
information by at most one pixel per class, two classes per direction).  A crop
of that radius, with even offsets so the colour classes of the crop are those of
the image, therefore reproduces the full image's result at its centre exactly
in exact arithmetic; where the crop touches the image border it has the image's
free boundary.  The oracle (FP64) runs the crop; the GPU (FP32) runs the whole
image; the sampled means and variances must agree to the parity bar."""
import numpy as np
import pytest

import oracle.ep as oep
from oracle import operators as oops
from tests.gpu_util import MEAN_TOL, VAR_TOL

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2110_01585_amd import Context, ProblemSpec  # noqa: E402
from paper_2110_01585_amd import _native as N  # noqa: E402

SIZE = 16384
SWEEPS = 6
XI = 0.01
LAM = 8.0


def _observation(seed=11):
    """Seeded piecewise-constant image (random axis-aligned blocks) plus noise,
    generated on the device in float32."""
    g = torch.Generator(device="cuda").manual_seed(seed)
    coarse = torch.rand(SIZE // 32, SIZE // 32, generator=g, device="cuda")
    img = coarse.repeat_interleave(32, 0).repeat_interleave(32, 1)
    img += 0.5 * (torch.rand(SIZE // 8, SIZE // 8, generator=g, device="cuda")
                  .repeat_interleave(8, 0).repeat_interleave(8, 1) > 0.8)
    return (img + 0.1 * torch.randn(SIZE, SIZE, generator=g, device="cuda")).contiguous()


def test_denoise_at_the_largest_size_matches_oracle_crops():
    y = _observation()
    spec = ProblemSpec(SIZE, SIZE, noise_var=XI, lambda0=LAM, damping=0.5)
    ctx = Context([spec])
    ctx.ep_tv_set_observation([y])
    ctx.ep_tv_set_option(N.OPT_GRAPH, 1)
    ctx.ep_tv_autotune(2)
    ctx.ep_tv_init_cold()
    ctx.ep_tv_run(SWEEPS, False)
    mus, vs = ctx.marginals()
    torch.cuda.synchronize()
    R = 4 * SWEEPS + 4
    rng = np.random.default_rng(5)
    pts = [(0, 0), (0, SIZE - 1), (SIZE - 1, 0), (SIZE - 1, SIZE - 1), (SIZE // 2, 0),
           (0, SIZE // 2 + 1), (SIZE - 1, 12345), (7777, SIZE - 1)]
    pts += [tuple(int(v) for v in rng.integers(0, SIZE, 2)) for _ in range(8)]
    worst_m = worst_v = 0.0
    for (r, c) in pts:
        r0 = max(0, (r - R) // 2 * 2)
        c0 = max(0, (c - R) // 2 * 2)
        r1 = min(SIZE, r + R + 1)
        c1 = min(SIZE, c + R + 1)
        crop = y[r0:r1, c0:c1].cpu().numpy().astype(np.float64)
        op = oops.Operator(oops.IDENTITY, crop.shape)
        pb = oep.EPProblem(crop, op, XI, LAM, damping=0.5)
        st = oep.init_cold(pb)
        for t in range(1, SWEEPS + 1):
            oep.sweep(pb, st, t, False)
        mu_o, v_o = oep.marginals(st)
        k = (r - r0) * (c1 - c0) + (c - c0)
        mg = float(mus[0][r, c])
        vg = float(vs[0][r, c])
        rng_c = float(crop.max() - crop.min())
        worst_m = max(worst_m, abs(mg - mu_o[k]) / rng_c)
        worst_v = max(worst_v, abs(vg / v_o[k] - 1))
    ctx.close()
    print(f"{SIZE}^2 denoising, {SWEEPS} sweeps, {len(pts)} sampled pixels: "
          f"mean err {worst_m:.2e}, var err {worst_v:.2e}")
    assert worst_m <= MEAN_TOL and worst_v <= VAR_TOL
