"""The polynomial behind the device tilted moments (kMillsPoly in
paper_2110_01585_amd/csrc/tilted.h) against its definition.

K(x) = r(x) - x, r = sqrt(2/pi) / erfcx(x / sqrt2), the mean distance of a
truncated standard Gaussian beyond its cut x >= 0 (Sec. III-C moments of the
tilted distribution).  Checked here, on the CPU:
* the table in tilted.h is exactly what fit_mills.py produces;
* its evaluation in FP32 from x, K = t G(2t - 1), t = 2 / (2 + x / sqrt2) (z, t
  and every Horner step rounded to float32), is within 3e-7 relative (about
  4 ulp; 2.2e-7 measured) of K computed at 50 digits from the definition, over
  the whole half line (x from 0 to 1e7);
* the two limits: K(0) = sqrt(2/pi) and x K(x) -> 1 as x -> inf."""
import os
import re
import sys

import mpmath as mp
import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2110_01585_amd", "csrc")


def _table():
    src = open(os.path.join(CSRC, "tilted.h")).read()
    body = src[src.index("kMillsPoly[13] = {"):]
    body = body[:body.index("};")]
    vals = re.findall(r"([-+]?[0-9.]+e[-+][0-9]+)f", body)
    assert len(vals) == 13
    return np.array([float(v) for v in vals], dtype=np.float32)


def _k_exact(x):
    mp.mp.dps = 50
    x = mp.mpf(x)
    z = x / mp.sqrt(2)
    return mp.sqrt(2 / mp.pi) / (mp.exp(z * z) * mp.erfc(z)) - x


def _k_fp32(c, x):
    x = np.float32(x)
    z = x * np.float32(1 / np.sqrt(2))
    t = np.float32(2) / (np.float32(2) + z)
    s = np.float32(2) * t - np.float32(1)
    g = c[12]
    for k in range(11, -1, -1):
        g = np.float32(g * s + c[k])
    return float(np.float32(t * g))


def test_table_matches_generator():
    sys.path.insert(0, CSRC)
    try:
        import fit_mills
    finally:
        sys.path.pop(0)
    t = fit_mills.sample(2001, 2000)
    g = np.array([float(fit_mills.g_exact(v)) for v in t])
    coef = fit_mills.fit(t, g).astype(np.float32)
    assert np.array_equal(coef, _table())


def test_fp32_evaluation_against_definition():
    c = _table()
    xs = np.concatenate([np.linspace(0.0, 10.0, 401), np.geomspace(10.0, 1e7, 200)])
    worst = 0.0
    for x in xs:
        ref = float(_k_exact(x))
        worst = max(worst, abs(_k_fp32(c, x) / ref - 1.0))
    assert worst <= 3e-7, worst


def test_limits():
    c = _table()
    assert abs(_k_fp32(c, 0.0) / np.sqrt(2 / np.pi) - 1) <= 3e-7
    for x in (1e4, 1e6):
        assert abs(x * _k_fp32(c, x) - 1.0) <= 2e-7 + 1.0 / x ** 2
