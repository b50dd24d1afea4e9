"""Seeded synthetic workloads for TV-prior image restoration.

This module only draws inputs: ground-truth piecewise-constant images, noise,
Gaussian blur taps, subsampled-DFT masks and the noisy observations they
produce.  It holds none of the EP method's arithmetic and is shared by the
FP64 oracle (``oracle/``) and by the GPU path's tests and benchmark, which
must see bit-identical inputs.

Observation model (paper, Sec. II-A, Eq. (1)): y = H x + n with i.i.d.
Gaussian noise of variance xi.  Three degradation operators are drawn:

* identity (denoising),
* periodic 2-D convolution with a centred, normalised Gaussian kernel
  (deconvolution),
* a seeded subset of the orthonormal 2-D DFT coefficients, always keeping
  the DC coefficient (compressive sensing).  Noise on the kept coefficients
  is circular complex Gaussian CN(0, sigma^2), which is equivalent to real
  observations of Re and Im with variance xi = sigma^2 / 2 each.

The images stand in for the paper's test images (Cameraman, Flinstones,
Mandrill, Shepp-Logan; Sec. V), which are not used: they are random
axis-aligned rectangles and disks with intensities U[0, 1].
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

OP_IDENTITY = "identity"
OP_BLUR = "blur"
OP_DFT = "dft"
OP_HADAMARD = "hadamard"
OP_GAUSS = "gauss"


def rng_for(config: int, instance: int = 0) -> np.random.Generator:
    """PCG64 stream for (workload config, instance): seed = 1000*config + instance."""
    return np.random.Generator(np.random.PCG64(1000 * config + instance))


def piecewise_image(h: int, w: int, n_shapes: int, rng: np.random.Generator,
                    mode: str = "paint", disk_fraction: float = 0.5) -> np.ndarray:
    """Random piecewise-constant image.

    mode="sum":   rectangles are added on top of each other (values may exceed 1).
    mode="paint": shapes overwrite what lies under them, background 0; a shape
                  is a disk with probability ``disk_fraction``, else a rectangle.
    Rectangle sides are U{ceil(S/16) .. ceil(S/4)} with S = min(h, w), top-left
    corner uniform in the image, clipped at the border.  Disk radii are
    U[S/32, S/8] with a uniform centre.  Intensities are U[0, 1].
    """
    s = min(h, w)
    img = np.zeros((h, w), dtype=np.float64)
    lo, hi = max(1, math.ceil(s / 16)), max(1, math.ceil(s / 4))
    for _ in range(n_shapes):
        is_disk = (mode == "paint") and (rng.random() < disk_fraction)
        val = rng.random()
        if is_disk:
            r0 = rng.random() * h
            c0 = rng.random() * w
            rad = rng.uniform(s / 32.0, s / 8.0)
            ra, rb = max(0, int(math.floor(r0 - rad)) - 1), min(h, int(math.ceil(r0 + rad)) + 1)
            ca, cb = max(0, int(math.floor(c0 - rad)) - 1), min(w, int(math.ceil(c0 + rad)) + 1)
            rr, cc = np.mgrid[ra:rb, ca:cb]
            m = (rr + 0.5 - r0) ** 2 + (cc + 0.5 - c0) ** 2 <= rad * rad
            if mode == "sum":
                img[ra:rb, ca:cb][m] += val
            else:
                img[ra:rb, ca:cb][m] = val
        else:
            hh = int(rng.integers(lo, hi + 1))
            ww = int(rng.integers(lo, hi + 1))
            r0 = int(rng.integers(0, h))
            c0 = int(rng.integers(0, w))
            sl = (slice(r0, min(h, r0 + hh)), slice(c0, min(w, c0 + ww)))
            if mode == "sum":
                img[sl] += val
            else:
                img[sl] = val
    return img


def window_image(h: int, w: int, scale: int, rng: np.random.Generator,
                 density: float = 60.0 / (512 * 512), disk_fraction: float = 0.5) -> np.ndarray:
    """An h x w window of a large painted canvas whose shapes are sized for an
    S x S image, S = ``scale`` (rectangle sides U{ceil(S/16) .. ceil(S/4)}, disk
    radii U[S/32, S/8]), with ``density`` shapes per canvas pixel.  Shape anchors
    are uniform over the window grown by the largest shape extent on every side,
    so every shape that can overlap the window is drawn; only the overlap is
    painted (in drawing order, background 0)."""
    s = scale
    lo, hi = max(1, math.ceil(s / 16)), max(1, math.ceil(s / 4))
    ext = hi
    n = int(round(density * (h + 2 * ext) * (w + 2 * ext)))
    img = np.zeros((h, w), dtype=np.float64)
    for _ in range(n):
        is_disk = rng.random() < disk_fraction
        val = rng.random()
        if is_disk:
            r0 = rng.uniform(-ext, h + ext)
            c0 = rng.uniform(-ext, w + ext)
            rad = rng.uniform(s / 32.0, s / 8.0)
            ra, rb = max(0, int(math.floor(r0 - rad)) - 1), min(h, int(math.ceil(r0 + rad)) + 1)
            ca, cb = max(0, int(math.floor(c0 - rad)) - 1), min(w, int(math.ceil(c0 + rad)) + 1)
            if ra >= rb or ca >= cb:
                continue
            rr, cc = np.mgrid[ra:rb, ca:cb]
            m = (rr + 0.5 - r0) ** 2 + (cc + 0.5 - c0) ** 2 <= rad * rad
            img[ra:rb, ca:cb][m] = val
        else:
            hh = int(rng.integers(lo, hi + 1))
            ww = int(rng.integers(lo, hi + 1))
            r0 = int(rng.integers(-ext, h + ext))
            c0 = int(rng.integers(-ext, w + ext))
            ra, rb = max(0, r0), min(h, r0 + hh)
            ca, cb = max(0, c0), min(w, c0 + ww)
            if ra < rb and ca < cb:
                img[ra:rb, ca:cb] = val
    return img


def gaussian_taps(sigma_b: float, size: int = 9) -> np.ndarray:
    """Centred size x size Gaussian kernel exp(-(a^2+b^2)/(2 sigma_b^2)), sum 1."""
    a = np.arange(size) - size // 2
    k1 = np.exp(-(a.astype(np.float64) ** 2) / (2.0 * sigma_b * sigma_b))
    k = np.outer(k1, k1)
    return k / k.sum()


def _circular_blur_fft(x: np.ndarray, taps: np.ndarray) -> np.ndarray:
    """Periodic convolution (k * x)(r, c) = sum_ab k(a, b) x(r - a, c - b) via FFT."""
    h, w = x.shape
    kh, kw = taps.shape
    pad = np.zeros((h, w), dtype=np.float64)
    for a in range(kh):
        for b in range(kw):
            pad[(a - kh // 2) % h, (b - kw // 2) % w] += taps[a, b]
    return np.real(np.fft.ifft2(np.fft.fft2(x) * np.fft.fft2(pad)))


def dft_mask(h: int, w: int, frac: float, rng: np.random.Generator) -> np.ndarray:
    """uint8 mask keeping round(frac*h*w) DFT coefficients, uniform without
    replacement, with the DC coefficient (0, 0) always kept."""
    n = h * w
    k = int(round(frac * n))
    idx = rng.choice(n, size=k, replace=False)
    m = np.zeros(n, dtype=np.uint8)
    m[idx] = 1
    m[0] = 1
    return m.reshape(h, w)


def _bitrev(n: int) -> np.ndarray:
    m = int(round(math.log2(n)))
    j = np.arange(n)
    out = np.zeros(n, dtype=np.int64)
    for b in range(m):
        out |= ((j >> b) & 1) << (m - 1 - b)
    return out


def walsh_paley_2d(x: np.ndarray) -> np.ndarray:
    """Orthonormal 2-D Walsh transform in Paley order (observation model of the
    Hadamard CS workload): a fast Walsh-Hadamard butterfly along each axis in
    natural (Sylvester) order, whose row k is Paley row bitreverse(k)."""
    h, w = x.shape
    v = np.asarray(x, dtype=np.float64).copy()
    for axis, n in ((0, h), (1, w)):
        v = np.moveaxis(v, axis, 0)
        s = 1
        while s < n:
            v = v.reshape(n // (2 * s), 2, s, -1)
            a, b = v[:, 0].copy(), v[:, 1].copy()
            v[:, 0], v[:, 1] = a + b, a - b
            v = v.reshape(n, -1)
            s *= 2
        v = v.reshape((n,) + tuple(np.delete(np.array(x.shape), axis)))
        v = np.moveaxis(v, 0, axis)
    return v[np.ix_(_bitrev(h), _bitrev(w))] / math.sqrt(h * w)


@dataclass
class Problem:
    """One restoration instance: what a caller hands to a solver."""
    name: str
    x_true: np.ndarray
    y: np.ndarray                     # real (h, w); complex (h, w) for OP_DFT (0 off-mask);
                                      # (M,) for OP_GAUSS
    op: str
    xi: float                         # noise variance per real observation
    lam0: float                       # initial (or fixed) lambda
    damping: float                    # weight on the new site value
    sweeps: int
    em: bool
    taps: Optional[np.ndarray] = None
    mask: Optional[np.ndarray] = None
    boundary: str = "free"
    meta: dict = field(default_factory=dict)
    sense: Optional[np.ndarray] = None   # OP_GAUSS: M x N sensing matrix (float32 values)

    @property
    def shape(self):
        return self.x_true.shape


def make_denoise(h, w, n_shapes, sigma, rng, mode="sum", lam0=10.0, damping=0.5,
                 sweeps=100, em=False, name="denoise"):
    x = piecewise_image(h, w, n_shapes, rng, mode=mode)
    y = x + sigma * rng.standard_normal((h, w))
    return Problem(name, x, y, OP_IDENTITY, sigma * sigma, lam0, damping, sweeps, em,
                   meta={"sigma": sigma})


def make_deconv(h, w, n_shapes, sigma, sigma_b, rng, mode="paint", lam0=1.0,
                damping=0.5, sweeps=200, em=True, name="deconv", ksize=9):
    x = piecewise_image(h, w, n_shapes, rng, mode=mode)
    taps = gaussian_taps(sigma_b, ksize)
    y = _circular_blur_fft(x, taps) + sigma * rng.standard_normal((h, w))
    return Problem(name, x, y, OP_BLUR, sigma * sigma, lam0, damping, sweeps, em,
                   taps=taps, meta={"sigma": sigma, "sigma_b": sigma_b})


def make_cs(h, w, n_shapes, sigma, frac, rng, mode="paint", lam0=1.0, damping=0.5,
            sweeps=300, em=True, name="cs"):
    x = piecewise_image(h, w, n_shapes, rng, mode=mode)
    mask = dft_mask(h, w, frac, rng)
    X = np.fft.fft2(x, norm="ortho")
    noise = (sigma / math.sqrt(2.0)) * (rng.standard_normal((h, w))
                                        + 1j * rng.standard_normal((h, w)))
    Y = np.where(mask.astype(bool), X + noise, 0.0 + 0.0j)
    return Problem(name, x, Y, OP_DFT, sigma * sigma / 2.0, lam0, damping, sweeps, em,
                   mask=mask, meta={"sigma": sigma, "frac": frac})


def make_hadamard_cs(h, w, n_shapes, sigma, frac, rng, mode="paint", lam0=1.0, damping=0.5,
                     sweeps=300, em=True, name="hcs"):
    """Hadamard CS: a uniform random subset of round(frac h w) Paley-ordered
    Walsh coefficients (the constant function (0, 0) always kept), real noise
    of standard deviation sigma on each."""
    x = piecewise_image(h, w, n_shapes, rng, mode=mode)
    mask = dft_mask(h, w, frac, rng)
    Y = walsh_paley_2d(x) + sigma * rng.standard_normal((h, w))
    Y = np.where(mask.astype(bool), Y, 0.0)
    return Problem(name, x, Y, OP_HADAMARD, sigma * sigma, lam0, damping, sweeps, em,
                   mask=mask, meta={"sigma": sigma, "frac": frac})


def make_gauss_cs(h, w, n_shapes, sigma, frac, rng, mode="paint", lam0=1.0, damping=0.5,
                  sweeps=100, em=True, name="gcs"):
    """Compressive sensing with a Gaussian i.i.d. sensing matrix (Sec. II-A case
    (iii), the CS experiment of Sec. V): M = round(frac h w) rows with entries
    N(0, 1/M), rounded to float32; y = H vec(x) + noise of standard deviation
    sigma (x row-major)."""
    x = piecewise_image(h, w, n_shapes, rng, mode=mode)
    n = h * w
    m = max(1, int(round(frac * n)))
    H = (rng.standard_normal((m, n)) / math.sqrt(m)).astype(np.float32).astype(np.float64)
    y = H @ x.ravel() + sigma * rng.standard_normal(m)
    return Problem(name, x, y, OP_GAUSS, sigma * sigma, lam0, damping, sweeps, em, sense=H,
                   meta={"sigma": sigma, "frac": frac})


# --------------------------------------------------------------------------
# The five workloads (sizes can be overridden for small parity cases).
# --------------------------------------------------------------------------

def config0(size: int = 128, sweeps: int = 100) -> Problem:
    """Denoising, sum of 20 rectangles, sigma = 0.1, lambda = 10 fixed, 100 sweeps."""
    return make_denoise(size, size, 20, 0.1, rng_for(0), mode="sum", lam0=10.0,
                        damping=0.5, sweeps=sweeps, em=False, name=f"denoise{size}")


def config1(size: int = 512, sweeps: int = 200) -> Problem:
    """Deconvolution, 60 painted shapes, 9x9 Gaussian blur sigma_b = 2 (periodic),
    sigma = 0.01, EM from lambda = 1, 200 sweeps."""
    n = max(3, round(60 * size * size / (512 * 512)))
    return make_deconv(size, size, n, 0.01, 2.0, rng_for(1), lam0=1.0, damping=0.5,
                       sweeps=sweeps, em=True, name=f"deconv{size}")


def config2(size: int = 1024, sweeps: int = 300) -> Problem:
    """CS, 150 painted shapes, 25 % DFT mask with DC, CN noise sigma = 0.005, EM, 300 sweeps."""
    n = max(3, round(150 * size * size / (1024 * 1024)))
    return make_cs(size, size, n, 0.005, 0.25, rng_for(2), lam0=1.0, damping=0.5,
                   sweeps=sweeps, em=True, name=f"cs{size}")


def config3_instance(i: int, max_sweeps: int = 200, size_lo: int = 64,
                     size_hi: int = 1024) -> Problem:
    """Instance i of the batched mix (its own seed, independent of the others)."""
    rng = rng_for(3, i)
    s = int(round(math.exp(rng.uniform(math.log(size_lo), math.log(size_hi)))))
    shapes = max(3, round(60 * s * s / (512 * 512)))
    sigma = rng.uniform(0.01, 0.1)
    if rng.random() < 0.5:
        return make_denoise(s, s, shapes, sigma, rng, mode="paint", lam0=1.0,
                            sweeps=max_sweeps, em=True, name=f"b{i}_denoise{s}")
    sb = rng.uniform(1.0, 3.0)
    return make_deconv(s, s, shapes, sigma, sb, rng, lam0=1.0, sweeps=max_sweeps,
                       em=True, name=f"b{i}_deconv{s}")


def config3_instances(n_instances: int = 256, max_sweeps: int = 200,
                      size_lo: int = 64, size_hi: int = 1024):
    """Batched mix: sizes round(exp(U[ln lo, ln hi])), 50/50 denoise/deconv,
    sigma_b ~ U[1, 3], sigma ~ U[0.01, 0.1], EM from lambda = 1 per instance."""
    return [config3_instance(i, max_sweeps, size_lo, size_hi) for i in range(n_instances)]


def config4_train(index: int, size: int = 256) -> Problem:
    """Warm-start training instance: 256^2 deconvolution, config-1 operator and noise."""
    rng = rng_for(4, 100000 + index)
    shapes = max(3, round(60 * size * size / (512 * 512)))
    return make_deconv(size, size, shapes, 0.01, 2.0, rng, lam0=1.0, sweeps=200,
                       em=True, name=f"train{index}")


def config4_train_mixed(index: int, size: int = 256) -> Problem:
    """Warm-start training instance across image scales: instance i is a
    size x size window of a canvas whose shapes are sized for an S x S image,
    S = size * 2^(i mod 4) (256^2 windows of 256^2 ... 2048^2 scale images), so
    that the training pixels cover the statistics of the large test image.
    i mod 4 == 0 is exactly config4_train(i).  Operator and noise as the
    deconvolution workload: 9 x 9 Gaussian blur sigma_b = 2, sigma = 0.01."""
    k = index % 4
    if k == 0:
        return config4_train(index, size)
    rng = rng_for(4, 200000 + index)
    x = window_image(size, size, size << k, rng)
    taps = gaussian_taps(2.0, 9)
    y = _circular_blur_fft(x, taps) + 0.01 * rng.standard_normal((size, size))
    return Problem(name=f"trainmix{index}", x_true=x, y=y, op=OP_BLUR, xi=0.01 ** 2, lam0=1.0,
                   damping=0.5, sweeps=200, em=True, taps=taps, boundary="free",
                   meta={"sigma": 0.01, "sigma_b": 2.0, "scale": size << k})


def config4_test(seed: int = 0, size: int = 2048) -> Problem:
    """Warm-start test instance: 2048^2 deconvolution (sigma_b = 2, sigma = 0.01)."""
    rng = rng_for(4, seed)
    shapes = max(3, round(60 * size * size / (512 * 512)))
    return make_deconv(size, size, shapes, 0.01, 2.0, rng, lam0=1.0, sweeps=400,
                       em=True, name=f"test{size}_{seed}")
