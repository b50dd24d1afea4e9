"""Degradation operators H, H^T, H^T H and the likelihood-site variance (FP64).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Sec. II-A, Eq. (1): y = H x + n, n ~ N(0, xi I).  Three operators:

* identity (denoising, case (i));
* periodic 2-D convolution with centred taps k of odd size (deconvolution,
  case (ii)): (H x)(r, c) = sum_{a,b} k(a, b) x(r - a + kh//2, c - b + kw//2),
  indices modulo the image size;  H^T is the matching correlation;
* masked orthonormal 2-D DFT (compressive sensing, case (iii) replaced by a
  Fourier sensing matrix): observations are the masked complex coefficients of
  F x.  Treating (Re, Im) of each kept coefficient as two real observations of
  variance xi gives H^T H x = Re(F^H P F x) and H^T y = Re(F^H P y);
* dense Gaussian i.i.d. sensing matrix (compressive sensing, case (iii) with
  the paper's random matrix, Sec. V): H is given (M x N, acting on the image
  flattened row-major); H^T H is neither diagonal nor circulant, so the
  likelihood site's mean and variances come from the Woodbury identity the
  paper names for low-rank H^T H (M < N): with D = diag(tau_c) and
  S = xi I_M + H D^{-1} H^T = L L^T (Cholesky), Z = L^{-1} H,
      (H^T H / xi + D)^{-1} = D^{-1} - D^{-1} Z^T Z D^{-1},
  so v_i = 1/d_i - |z_i|^2 / d_i^2 (z_i column i of Z) and
  E = D^{-1} (b - Z^T (Z D^{-1} b));
* subsampled Paley-ordered 2-D Walsh-Hadamard transform (compressive sensing,
  case (iii) with the paper's Hadamard sensing matrix, Sec. II-A and the CS
  experiment of Sec. V): observations are the kept coefficients
  (W x)(u, v) = sum_{r,c} w_u(r) w_v(c) x(r, c) / sqrt(h w), where w_k is the
  k-th Walsh function in Paley order, the product of the Rademacher functions
  selected by the binary digits of k.  W is real and orthonormal, so
  H^T H = W^T P W is diagonal in the Walsh basis with the mask as eigenvalues.

The blur H and H^T are written as sums of shifted copies (their definition);
H^T H and its spectrum use the FFT (a library primitive), and tests check the
two forms against each other.

Eq. (tilted_P_1) needs diag((H^T H / xi + diag(tau_c))^{-1}).  The paper notes
it is exact when H^T H is diagonal and otherwise names Monte Carlo estimators
(RBMC).  Two estimators are provided:

* "exact":    the dense inverse (tiny images only);
* "spectral": replace the cavity precision by its mean d (a scalar), where the
              inverse is circulant and its diagonal is the constant
              c = mean_w 1 / (|H(w)|^2 / xi + d); the site precision is then the
              constant gamma = 1/c - d, and the tilted variance at pixel p is
              1 / (gamma + tau_c[p]).  Exact when tau_c is constant.  For the
              Walsh-Hadamard operator the same holds with the Walsh basis in
              place of the Fourier basis (every Walsh function has squared
              entries 1 / N, like every Fourier mode).
* "rbmc":     the simple Rao-Blackwellised Monte Carlo estimator the paper names
              (Siden, Lindgren, Bolin, Villani 2018).  With Q the precision
              H^T H / xi + diag(tau_c), Var(x_i) = 1/Q_ii + Var(E[x_i | x_-i]) and
              E[x_i | x_-i] = -(sum_{j != i} Q_ij x_j) / Q_ii, so
                v_i = 1/Q_ii + (1/Q_ii^2) (1/Ns) sum_s (sum_{j != i} Q_ij x_j^(s))^2,
              x^(s) ~ N(0, Q^{-1}) drawn by perturbation-optimisation: solve
              Q x^(s) = z^(s) with z^(s) = H^T e1^(s) / sqrt(xi) + sqrt(tau_c) e2^(s)
              ~ N(0, Q), e1^(s) white in observation space (complex for the DFT:
              real and imaginary parts each N(0, 1)), e2^(s) white in pixel
              space.  The white noise is an input (the caller draws it); each
              sample costs one CG solve.  Unbiased for any Ns, v_i >= 1/Q_ii.
"""
from __future__ import annotations

import numpy as np

IDENTITY = "identity"
BLUR = "blur"
DFT = "dft"
HADAMARD = "hadamard"
GAUSS = "gauss"


def walsh_paley(n):
    """n x n matrix of the Walsh functions in Paley order sampled at t = j / n
    (n a power of two), from their definition: w_k = prod_i r_{i+1}^{k_i} with
    k_i the binary digits of k and r_{i+1}(t) = sign(sin(2^{i+1} pi t)) the
    Rademacher functions, which at t = j / n is -1 exactly when binary digit
    i + 1 after the point of t, bit (m - 1 - i) of j, is one (n = 2^m)."""
    m = int(round(np.log2(n)))
    if 1 << m != n:
        raise ValueError("Walsh matrix size must be a power of two")
    j = np.arange(n)
    out = np.ones((n, n))
    for k in range(n):
        for i in range(m):
            if (k >> i) & 1:
                rad = np.where((j >> (m - 1 - i)) & 1, -1.0, 1.0)
                out[k] *= rad
    return out


class Operator:
    def __init__(self, kind, shape, taps=None, mask=None, sense=None):
        self.kind = kind
        self.shape = tuple(shape)
        self.sense = None if sense is None else np.asarray(sense, dtype=np.float64)
        if kind == GAUSS and (self.sense is None or self.sense.shape[1] != self.shape[0] * self.shape[1]):
            raise ValueError("the Gaussian operator needs an M x (h w) sensing matrix")
        self.taps = None if taps is None else np.asarray(taps, dtype=np.float64)
        self.mask = None if mask is None else np.asarray(mask).astype(bool)
        if kind == BLUR:
            kh, kw = self.taps.shape
            if kh % 2 == 0 or kw % 2 == 0:
                raise ValueError("blur taps must have odd sizes")
        if kind in (DFT, HADAMARD) and self.mask.shape != self.shape:
            raise ValueError("mask shape mismatch")
        self._spec = None
        if kind == HADAMARD:
            self._wr = walsh_paley(self.shape[0])
            self._wc = walsh_paley(self.shape[1])
            self._norm = 1.0 / np.sqrt(self.shape[0] * self.shape[1])

    def walsh(self, x):
        """Orthonormal 2-D Walsh transform (Paley order) of an image."""
        return self._wr @ x @ self._wc.T * self._norm

    def walsh_t(self, v):
        """Its transpose (and inverse)."""
        return self._wr.T @ v @ self._wc * self._norm

    # ---------------- definition forms ----------------
    def H(self, x):
        """Forward operator on a real image.  DFT: returns the complex masked
        spectrum (h, w) with zeros off the mask."""
        if self.kind == IDENTITY:
            return x.copy()
        if self.kind == GAUSS:
            return self.sense @ np.asarray(x, np.float64).ravel()
        if self.kind == BLUR:
            kh, kw = self.taps.shape
            out = np.zeros_like(x)
            for a in range(kh):
                for b in range(kw):
                    out += self.taps[a, b] * np.roll(x, (a - kh // 2, b - kw // 2), axis=(0, 1))
            return out
        if self.kind == HADAMARD:
            return np.where(self.mask, self.walsh(x), 0.0)
        X = np.fft.fft2(x, norm="ortho")
        return np.where(self.mask, X, 0.0)

    def Ht(self, v):
        """Adjoint: real image."""
        if self.kind == IDENTITY:
            return np.asarray(v, dtype=np.float64).copy()
        if self.kind == GAUSS:
            return (self.sense.T @ np.asarray(v, np.float64)).reshape(self.shape)
        if self.kind == BLUR:
            kh, kw = self.taps.shape
            out = np.zeros_like(v)
            for a in range(kh):
                for b in range(kw):
                    out += self.taps[a, b] * np.roll(v, (-(a - kh // 2), -(b - kw // 2)), axis=(0, 1))
            return out
        V = np.where(self.mask, v, 0.0)
        if self.kind == HADAMARD:
            return self.walsh_t(np.real(V))
        return np.real(np.fft.ifft2(V, norm="ortho"))

    # ---------------- spectral forms ----------------
    def spectrum(self):
        """Eigenvalues |H(w)|^2 of the circulant H^T H, shape (h, w); for the
        Walsh-Hadamard operator the eigenvalues in the Walsh basis (the mask)."""
        if self._spec is not None:
            return self._spec
        h, w = self.shape
        if self.kind == IDENTITY:
            spec = np.ones((h, w))
        elif self.kind == BLUR:
            kh, kw = self.taps.shape
            pad = np.zeros((h, w))
            for a in range(kh):
                for b in range(kw):
                    pad[(a - kh // 2) % h, (b - kw // 2) % w] += self.taps[a, b]
            spec = np.abs(np.fft.fft2(pad)) ** 2
        elif self.kind == HADAMARD:
            spec = self.mask.astype(np.float64)
        else:
            m = self.mask.astype(np.float64)
            # P(-w): index (-r mod h, -c mod w)
            m_neg = np.roll(m[::-1, ::-1], (1, 1), axis=(0, 1))
            spec = 0.5 * (m + m_neg)
        self._spec = spec
        return spec

    def HtH(self, x):
        """H^T H x through the spectrum (FFT); tests pin it to Ht(H(x))."""
        if self.kind == IDENTITY:
            return x.copy()
        if self.kind in (HADAMARD, GAUSS):
            return self.Ht(self.H(x))
        return np.real(np.fft.ifft2(np.fft.fft2(x) * self.spectrum()))

    def diag_basis_apply(self, v, d):
        """U^T diag(d) U v for the unitary U that diagonalises H^T H (the DFT,
        or the Walsh transform): the preconditioner of the mean solve."""
        if self.kind == HADAMARD:
            return self.walsh_t(d * self.walsh(v))
        return np.real(np.fft.ifft2(np.fft.fft2(v) * d))

    def Hty(self, y):
        return self.Ht(y)

    def diag_HtH(self):
        """Diagonal of H^T H, the same at every pixel for these operators: the
        mean eigenvalue (every basis function of the diagonalising transform has
        squared entries 1 / N; for the blur it equals the sum of squared taps)."""
        return float(np.mean(self.spectrum()))

    def dense_HtH(self):
        """Explicit N x N matrix of H^T H (tiny images only)."""
        h, w = self.shape
        n = h * w
        A = np.zeros((n, n))
        e = np.zeros((h, w))
        for p in range(n):
            e.flat[p] = 1.0
            A[:, p] = self.Ht(self.H(e)).ravel()
            e.flat[p] = 0.0
        return A


def woodbury_moments(op: Operator, xi, tau_c, b):
    """Mean (H^T H / xi + D)^{-1} b and the diagonal of (H^T H / xi + D)^{-1},
    D = diag(tau_c), by the Woodbury identity (see the module header); the
    Cholesky factor and the triangular solve are library routines."""
    from scipy.linalg import cholesky, solve_triangular
    H = op.sense
    d = np.asarray(tau_c, np.float64).ravel()
    S = xi * np.eye(H.shape[0]) + (H / d) @ H.T
    L = cholesky(S, lower=True)
    Z = solve_triangular(L, H, lower=True)
    v = 1.0 / d - (Z * Z).sum(axis=0) / (d * d)
    bv = np.asarray(b, np.float64).ravel()
    E = (bv - Z.T @ (Z @ (bv / d))) / d
    return E.reshape(op.shape), v.reshape(op.shape)


def solve_tilted_mean(op: Operator, xi, tau_c, b, x0=None, rtol=1e-12, maxiter=5000):
    """E = (H^T H / xi + diag(tau_c))^{-1} b by preconditioned conjugate
    gradients (the paper's suggestion for the mean of Eq. (tilted_P_1)).

    The preconditioner is (H^T H / xi + mean(tau_c) I)^{-1}, diagonal in the
    basis that diagonalises H^T H (circulant for the blur and the DFT, Walsh
    for the Hadamard operator); it changes the iteration count, not the
    solution.  Returns (E, iterations)."""
    h, w = op.shape
    if op.kind == IDENTITY:
        return b / (1.0 / xi + tau_c), 0
    if op.kind == GAUSS:
        return woodbury_moments(op, xi, tau_c, b)[0], 0
    spec = op.spectrum()
    dbar = float(np.mean(tau_c))
    pre = 1.0 / (spec / xi + dbar)

    def A(v):
        return op.HtH(v) / xi + tau_c * v

    def M(v):
        return op.diag_basis_apply(v, pre)

    x = np.zeros((h, w)) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - A(x)
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return np.zeros((h, w)), 0
    z = M(r)
    p = z.copy()
    rz = float(np.vdot(r, z))
    it = 0
    while np.linalg.norm(r) > rtol * bn and it < maxiter:
        q = A(p)
        alpha = rz / float(np.vdot(p, q))
        x += alpha * p
        r -= alpha * q
        z = M(r)
        rz_new = float(np.vdot(r, z))
        p = z + (rz_new / rz) * p
        rz = rz_new
        it += 1
    return x, it


class RBMCSamples:
    """White-noise inputs of the RBMC estimator and the per-sample solutions of
    the last call (the CG starting points of the next one; they change the
    iteration counts, not the estimate).  e1: (Ns, h, w), complex for the DFT
    operator; e2: (Ns, h, w)."""

    def __init__(self, e1, e2):
        self.e1 = np.asarray(e1)
        self.e2 = np.asarray(e2, dtype=np.float64)
        if self.e1.shape != self.e2.shape:
            raise ValueError("e1 and e2 must hold Ns images each")
        self.ns = self.e2.shape[0]
        self.x = [None] * self.ns
        self.cg_iters = 0


def rbmc_variance(op: Operator, xi, tau_c, samples: RBMCSamples, rtol=1e-12):
    """Diagonal of Q^{-1}, Q = H^T H / xi + diag(tau_c), by the RBMC estimator
    (see the module header)."""
    qd = op.diag_HtH() / xi + tau_c
    acc = np.zeros_like(tau_c, dtype=np.float64)
    samples.cg_iters = 0
    for s in range(samples.ns):
        z = op.Ht(samples.e1[s]) / np.sqrt(xi) + np.sqrt(tau_c) * samples.e2[s]
        x, it = solve_tilted_mean(op, xi, tau_c, z, x0=samples.x[s], rtol=rtol)
        samples.x[s] = x
        samples.cg_iters += it
        off = op.HtH(x) / xi + tau_c * x - qd * x          # sum_{j != i} Q_ij x_j
        acc += off * off
    return 1.0 / qd + acc / samples.ns / (qd * qd)


def tilted_variance(op: Operator, xi, tau_c, estimator="spectral", rbmc: RBMCSamples = None):
    """Diagonal of (H^T H / xi + diag(tau_c))^{-1}."""
    if op.kind == IDENTITY:
        return 1.0 / (1.0 / xi + tau_c)
    if estimator == "rbmc":
        if rbmc is None:
            raise ValueError("the RBMC estimator needs its white-noise samples")
        return rbmc_variance(op, xi, tau_c, rbmc)
    if op.kind == GAUSS or estimator == "woodbury":
        # exact; the right-hand side does not enter the diagonal
        return woodbury_moments(op, xi, tau_c, np.zeros(op.shape))[1]
    if estimator == "exact":
        A = op.dense_HtH() / xi + np.diag(tau_c.ravel())
        return np.diag(np.linalg.inv(A)).reshape(op.shape).copy()
    if estimator == "spectral":
        d = float(np.mean(tau_c))
        c = float(np.mean(1.0 / (op.spectrum() / xi + d)))
        gamma = 1.0 / c - d
        return 1.0 / (gamma + tau_c)
    raise ValueError(f"unknown estimator {estimator!r}")
