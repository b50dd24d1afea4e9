"""Write the stored oracle references for the full-size parity tests.

    python tests/golden/make_golden.py [deconv512|cs1024|all]

Each reference runs the FP64 oracle (oracle/ only) on the full-size seeded
workload -- the 512^2 deconvolution (9 x 9 Gaussian blur sigma_b = 2, sigma =
0.01, EM from lambda = 1, 200 sweeps) and the 1024^2 compressive-sensing
workload (25 % DFT mask, sigma = 0.005, EM, 300 sweeps) -- with the
observation and taps rounded to float32 exactly as the GPU receives them, and
stores the final lambda and the marginal means and variances at a fixed set of
sampled pixels (corners, borders, a seeded uniform sample) as JSON.  No value
comes from the GPU path.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synthetic as syn  # noqa: E402
from oracle import ep as oep  # noqa: E402


def f32_problem(p):
    import copy
    q = copy.copy(p)
    q.y = (p.y.real.astype(np.float32).astype(np.float64) +
           1j * p.y.imag.astype(np.float32).astype(np.float64)) if p.op == "dft" else \
        p.y.astype(np.float32).astype(np.float64)
    if p.taps is not None:
        q.taps = p.taps.astype(np.float32).astype(np.float64)
    return q


def sample_pixels(h, w, n=400, seed=12345):
    rng = np.random.default_rng(seed)
    pts = {(0, 0), (0, w - 1), (h - 1, 0), (h - 1, w - 1), (0, w // 2), (h // 2, 0), (h - 1, w // 2),
           (h // 2, w - 1), (h // 2, w // 2)}
    while len(pts) < n:
        pts.add((int(rng.integers(0, h)), int(rng.integers(0, w))))
    return sorted(pts)


def make(name):
    if name == "deconv512":
        p = syn.config1()
    elif name == "cs1024":
        p = syn.config2()
    else:
        raise SystemExit(f"unknown reference {name}")
    t0 = time.time()
    pb = oep.problem_from_synthetic(f32_problem(p))
    mu, v, st, info = oep.solve(pb, p.sweeps, p.em)
    h, w = p.shape
    pts = sample_pixels(h, w)
    out = {"workload": name, "shape": [h, w], "sweeps": p.sweeps, "em": p.em,
           "lambda": info["lam"], "clamp_count": info["clamp_count"],
           "mu_range": float(mu.max() - mu.min()),
           "pixels": [[r, c] for r, c in pts],
           "mu": [float(mu[r, c]) for r, c in pts], "var": [float(v[r, c]) for r, c in pts],
           "oracle_seconds": round(time.time() - t0, 1),
           "source": "tests/golden/make_golden.py (oracle/ep.py, FP64)"}
    with open(os.path.join(HERE, f"{name}.json"), "w") as f:
        json.dump(out, f)
    print(f"{name}: lambda {info['lam']:.8g}, {out['oracle_seconds']} s", flush=True)


if __name__ == "__main__":
    names = ["deconv512", "cs1024"] if len(sys.argv) < 2 or sys.argv[1] == "all" else sys.argv[1:]
    for n in names:
        make(n)
