"""Pins for oracle/operators.py and the synthetic observation model."""
import numpy as np
import pytest

import synthetic as syn
from oracle import operators as ops


def _rand_op(kind, h=12, w=10, seed=0):
    rng = np.random.default_rng(seed)
    if kind == ops.BLUR:
        taps = rng.random((5, 3))
        return ops.Operator(kind, (h, w), taps=taps / taps.sum())
    if kind == ops.DFT:
        return ops.Operator(kind, (h, w), mask=syn.dft_mask(h, w, 0.3, rng))
    return ops.Operator(kind, (h, w))


def test_blur_impulse_response_orientation():
    """H e_(0,0) puts tap k[a, b] at pixel (a - kh//2, b - kw//2) mod size:
    a periodic convolution, not a correlation."""
    taps = np.arange(15, dtype=float).reshape(5, 3) + 1.0
    op = ops.Operator(ops.BLUR, (9, 8), taps=taps)
    e = np.zeros((9, 8)); e[0, 0] = 1.0
    out = op.H(e)
    for a in range(5):
        for b in range(3):
            assert out[(a - 2) % 9, (b - 1) % 8] == taps[a, b]
    assert np.count_nonzero(out) == 15


def test_blur_delta_is_identity():
    taps = np.zeros((9, 9)); taps[4, 4] = 1.0
    op = ops.Operator(ops.BLUR, (7, 11), taps=taps)
    x = np.random.default_rng(1).normal(size=(7, 11))
    assert np.array_equal(op.H(x), x)
    assert np.allclose(op.spectrum(), 1.0, atol=1e-14)


@pytest.mark.parametrize("kind", [ops.BLUR, ops.DFT])
def test_adjoint(kind):
    op = _rand_op(kind)
    rng = np.random.default_rng(2)
    x = rng.normal(size=op.shape)
    if kind == ops.DFT:
        v = rng.normal(size=op.shape) + 1j * rng.normal(size=op.shape)
        lhs = np.real(np.vdot(v, op.H(x)))       # <Hx, v> as a real inner product
    else:
        v = rng.normal(size=op.shape)
        lhs = float(np.sum(op.H(x) * v))
    rhs = float(np.sum(x * op.Ht(v)))
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))


@pytest.mark.parametrize("kind", [ops.BLUR, ops.DFT])
def test_hth_fft_equals_definition(kind):
    op = _rand_op(kind, 16, 14, seed=3)
    x = np.random.default_rng(4).normal(size=op.shape)
    assert np.allclose(op.HtH(x), op.Ht(op.H(x)), rtol=0, atol=1e-12)


@pytest.mark.parametrize("kind", [ops.BLUR, ops.DFT])
def test_spectrum_is_eigenvalues(kind):
    op = _rand_op(kind, 6, 8, seed=5)
    A = op.dense_HtH()
    assert np.allclose(A, A.T, atol=1e-13)
    ev = np.sort(np.linalg.eigvalsh(A))
    assert np.allclose(ev, np.sort(op.spectrum().ravel()), atol=1e-12)


@pytest.mark.parametrize("kind", [ops.BLUR, ops.DFT])
def test_spectral_estimator_exact_for_constant_cavity(kind):
    op = _rand_op(kind, 16, 16, seed=6)
    tau_c = np.full(op.shape, 3.7)
    v_spec = ops.tilted_variance(op, 0.05, tau_c, "spectral")
    v_ex = ops.tilted_variance(op, 0.05, tau_c, "exact")
    assert np.allclose(v_spec, v_ex, rtol=1e-12, atol=0)


def test_spectral_estimator_identity_gives_exact_site():
    """For H = I the likelihood-site precision from the spectral rule is 1/xi."""
    taps = np.zeros((3, 3)); taps[1, 1] = 1.0
    op = ops.Operator(ops.BLUR, (8, 6), taps=taps)
    tau_c = np.random.default_rng(7).uniform(1, 9, (8, 6))
    V = ops.tilted_variance(op, 0.02, tau_c, "spectral")
    assert np.allclose(1.0 / V - tau_c, 1.0 / 0.02, rtol=1e-12)


@pytest.mark.parametrize("kind", [ops.BLUR, ops.DFT])
def test_cg_solves_tilted_mean(kind):
    op = _rand_op(kind, 10, 12, seed=8)
    rng = np.random.default_rng(9)
    tau_c = rng.uniform(0.5, 50, op.shape)
    b = rng.normal(size=op.shape)
    E, it = ops.solve_tilted_mean(op, 0.01, tau_c, b)
    A = op.dense_HtH() / 0.01 + np.diag(tau_c.ravel())
    Ed = np.linalg.solve(A, b.ravel()).reshape(op.shape)
    assert np.allclose(E, Ed, rtol=0, atol=1e-10 * np.abs(Ed).max())


def test_synthetic_observation_matches_operator_definition():
    """The generator's y - H x_true is white noise of the stated level, with H
    the oracle's definition-form convolution (so both agree on orientation)."""
    p = syn.make_deconv(64, 64, 8, 0.05, 1.7, syn.rng_for(9), mode="paint")
    taps = p.taps.copy()
    taps[0, 1] += 0.3          # make the kernel asymmetric so orientation matters
    taps /= taps.sum()
    rng = syn.rng_for(9)
    x = syn.piecewise_image(64, 64, 8, rng, mode="paint")
    noise_free = syn._circular_blur_fft(x, taps)
    op = ops.Operator(ops.BLUR, (64, 64), taps=taps)
    assert np.allclose(op.H(x), noise_free, atol=1e-12)
    r = p.y - ops.Operator(ops.BLUR, (64, 64), taps=p.taps).H(p.x_true)
    assert abs(np.std(r) / 0.05 - 1) < 0.05


def test_synthetic_cs_mask_and_noise():
    p = syn.config2(size=64, sweeps=1)
    assert p.mask[0, 0] == 1
    assert abs(p.mask.sum() - round(0.25 * 64 * 64)) <= 1
    X = np.fft.fft2(p.x_true, norm="ortho")
    r = (p.y - X)[p.mask.astype(bool)]
    assert np.all(p.y[~p.mask.astype(bool)] == 0)
    # CN(0, sigma^2): each of Re, Im has variance sigma^2 / 2 = xi
    assert abs(np.var(r.real) / p.xi - 1) < 0.1 and abs(np.var(r.imag) / p.xi - 1) < 0.1


# ---------------- the Paley-ordered Walsh-Hadamard operator ----------------

def _had_op(h=8, w=16, frac=0.3, seed=11):
    rng = np.random.default_rng(seed)
    return ops.Operator(ops.HADAMARD, (h, w), mask=syn.dft_mask(h, w, frac, rng))


def _sign_changes(row):
    return int(np.count_nonzero(row[1:] != row[:-1]))


def test_walsh_paley_sign_changes_follow_gray_code():
    """Paley ordering: the Walsh function of Paley index k changes sign g^{-1}(k)
    times on [0, 1), with g the binary reflected Gray code (the sequency index
    s satisfies k = s xor (s >> 1)); rows are orthogonal and row 0 is constant."""
    n = 32
    W = ops.walsh_paley(n)
    for s in range(n):
        k = s ^ (s >> 1)
        assert _sign_changes(W[k]) == s, (k, s)
    assert np.array_equal(W @ W.T, n * np.eye(n))
    assert np.all(W[0] == 1.0)
    # the first Rademacher function: + on the first half, - on the second
    assert np.array_equal(W[1], np.r_[np.ones(n // 2), -np.ones(n // 2)])


def test_walsh_paley_is_bit_reversed_sylvester():
    """Row k of the Paley-ordered matrix is row bitreverse(k) of the natural
    (Sylvester) Hadamard matrix of the library."""
    from scipy.linalg import hadamard
    for n in (2, 8, 64):
        m = int(np.log2(n))
        rev = [int(format(k, f"0{m}b")[::-1], 2) if m else 0 for k in range(n)]
        assert np.array_equal(ops.walsh_paley(n), hadamard(n)[rev].astype(float))


def test_hadamard_adjoint_and_full_mask_identity():
    op = _had_op()
    rng = np.random.default_rng(12)
    x, v = rng.normal(size=op.shape), rng.normal(size=op.shape)
    lhs, rhs = float(np.sum(op.H(x) * v)), float(np.sum(x * op.Ht(v)))
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))
    full = ops.Operator(ops.HADAMARD, op.shape, mask=np.ones(op.shape))
    assert np.allclose(full.Ht(full.H(x)), x, atol=1e-13)     # orthonormal
    # a single kept coefficient (u, v): H^T H x is the projection on w_u w_v^T / sqrt(N)
    m = np.zeros(op.shape); m[3, 5] = 1
    one = ops.Operator(ops.HADAMARD, op.shape, mask=m)
    b = np.outer(ops.walsh_paley(8)[3], ops.walsh_paley(16)[5]) / np.sqrt(128)
    assert np.allclose(one.HtH(x), b * np.sum(b * x), atol=1e-13)


def test_hadamard_mask_is_spectrum():
    op = _had_op(4, 8, seed=13)
    A = op.dense_HtH()
    assert np.allclose(A, A.T, atol=1e-13)
    assert np.allclose(np.sort(np.linalg.eigvalsh(A)), np.sort(op.spectrum().ravel()), atol=1e-12)
    # unit-norm Walsh functions: the diagonal of H^T H is the kept fraction
    assert np.allclose(np.diag(A), op.mask.mean(), atol=1e-13)


def test_hadamard_spectral_estimator_exact_for_constant_cavity():
    op = _had_op(16, 16, seed=14)
    tau_c = np.full(op.shape, 2.3)
    v_spec = ops.tilted_variance(op, 0.05, tau_c, "spectral")
    v_ex = ops.tilted_variance(op, 0.05, tau_c, "exact")
    assert np.allclose(v_spec, v_ex, rtol=1e-12, atol=0)


def test_hadamard_cg_solves_tilted_mean():
    op = _had_op(8, 16, seed=15)
    rng = np.random.default_rng(16)
    tau_c = rng.uniform(0.5, 50, op.shape)
    b = rng.normal(size=op.shape)
    E, it = ops.solve_tilted_mean(op, 0.01, tau_c, b)
    A = op.dense_HtH() / 0.01 + np.diag(tau_c.ravel())
    Ed = np.linalg.solve(A, b.ravel()).reshape(op.shape)
    assert np.allclose(E, Ed, rtol=0, atol=1e-10 * np.abs(Ed).max())
    assert it < 60


def test_synthetic_hadamard_observation_matches_operator_definition():
    p = syn.make_hadamard_cs(16, 32, 3, 0.0, 0.3, np.random.default_rng(17))
    op = ops.Operator(ops.HADAMARD, p.shape, mask=p.mask)
    assert np.allclose(p.y, op.H(p.x_true), atol=1e-12)
    assert p.mask[0, 0] == 1 and abs(p.mask.mean() - 0.3) < 0.01
