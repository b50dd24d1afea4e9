"""Oracle of the learned warm start (test infrastructure only; shares no code
with the HIP path).

A 6-layer 3x3 convolutional network maps a normalised observation to a
normalised posterior mean and log variance; its output initialises the EP
sites (`oracle.warm`).  Everything here is plain NumPy in float64, written from
the definitions:

  * cross-correlation with 3x3 taps, zero padding, stride 1;
  * ReLU after layers 1..5, none after layer 6 (channels 1 -> 32 -> 32 -> 32
    -> 32 -> 32 -> 2);
  * input  x0 = (y - m) / s, with m, s the mean and population standard
    deviation of the image (s floored at 1e-6);
  * output mu_hat = m + s * o[..., 0],  v_hat = xi * exp(o[..., 1]);
  * loss   L = mean over pixels (and images) of
           (o0 - (mu - m)/s)^2 + (o1 - log(v / xi))^2;
  * backward by the chain rule; Adam (Kingma & Ba, 2015, Algorithm 1) with
    bias correction on float32-like master weights.

Storage precision.  The GPU network keeps weights, activations and the
back-propagated activation gradients in bfloat16 and accumulates in float32.
With ``bf16=True`` the oracle rounds the same quantities to bfloat16 (round to
nearest, ties to even) at the same points, so that the comparison measures
accumulation order only; with ``bf16=False`` it is the exact float64 network
(this is the mode pinned by finite differences).

Parameters are one flat float64 vector in the canonical order
  W1[3][3][1][32], b1[32], (W_l[3][3][32][32], b_l[32]) for l = 2..5,
  W6[3][3][32][2], b6[2]
(tap row a, tap column b, input channel, output channel), 37,890 numbers.
Tap (a, b) multiplies the input pixel at (r + a - 1, c + b - 1).
"""
from __future__ import annotations

import numpy as np

CHANNELS = (1, 32, 32, 32, 32, 32, 2)
S_FLOOR = 1e-6


def layer_shapes(ch=CHANNELS):
    return [((3, 3, ch[i], ch[i + 1]), (ch[i + 1],)) for i in range(len(ch) - 1)]


def param_count(ch=CHANNELS):
    return sum(int(np.prod(w)) + b[0] for w, b in layer_shapes(ch))


def unpack(theta, ch=CHANNELS):
    """Flat vector -> list of (W, b) views."""
    out, o = [], 0
    for ws, bs in layer_shapes(ch):
        n = int(np.prod(ws))
        out.append((theta[o:o + n].reshape(ws), theta[o + n:o + n + bs[0]]))
        o += n + bs[0]
    assert o == theta.size
    return out


def pack(layers):
    return np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in layers])


def init_params(rng, ch=CHANNELS):
    """He-normal weights (std sqrt(2 / (9 cin))), zero biases."""
    parts = []
    for (ws, bs) in layer_shapes(ch):
        std = np.sqrt(2.0 / (9 * ws[2]))
        parts += [rng.normal(0.0, std, size=ws).ravel(), np.zeros(bs)]
    return np.concatenate(parts)


def bf16_round(x):
    """Round float values to the nearest bfloat16 (ties to even), returned as
    float64.  bfloat16 keeps the 8 high bits of the float32 significand."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    r = np.where(np.isnan(f), u | 0x400000, r)          # keep NaNs NaN
    return (r.astype(np.uint32)).view(np.float32).astype(np.float64)


def conv3x3(x, w, b=None):
    """out[n, r, c, o] = b[o] + sum_{a, bb, i} x[n, r + a - 1, c + bb - 1, i] w[a, bb, i, o]
    with x = 0 outside the image.  x: (N, H, W, Cin), w: (3, 3, Cin, Cout)."""
    n, h, wd, _ = x.shape
    xp = np.zeros((n, h + 2, wd + 2, x.shape[3]))
    xp[:, 1:h + 1, 1:wd + 1] = x
    out = np.zeros((n, h, wd, w.shape[3]))
    for a in range(3):
        for bb in range(3):
            out += xp[:, a:a + h, bb:bb + wd, :] @ w[a, bb]
    if b is not None:
        out += b
    return out


def conv3x3_input_grad(g, w):
    """Adjoint of conv3x3 in x: dx[n, p, i] = sum_{a, bb, o} g[n, p - (a-1, bb-1), o] w[a, bb, i, o]."""
    n, h, wd, _ = g.shape
    gp = np.zeros((n, h + 2, wd + 2, g.shape[3]))
    gp[:, 1:h + 1, 1:wd + 1] = g
    dx = np.zeros((n, h, wd, w.shape[2]))
    for a in range(3):
        for bb in range(3):
            # x pixel q receives g at q - (a - 1, bb - 1): rows q + 1 - a of the padded g
            dx += gp[:, 2 - a:2 - a + h, 2 - bb:2 - bb + wd, :] @ w[a, bb].T
    return dx


def conv3x3_weight_grad(x, g):
    """dw[a, bb, i, o] = sum_{n, p} x[n, p + (a-1, bb-1), i] g[n, p, o] (x zero-padded)."""
    n, h, wd, cin = x.shape
    xp = np.zeros((n, h + 2, wd + 2, cin))
    xp[:, 1:h + 1, 1:wd + 1] = x
    dw = np.zeros((3, 3, cin, g.shape[3]))
    gf = g.reshape(-1, g.shape[3])
    for a in range(3):
        for bb in range(3):
            dw[a, bb] = xp[:, a:a + h, bb:bb + wd, :].reshape(-1, cin).T @ gf
    return dw


def normalise(y):
    """Per-image mean and population standard deviation (floored)."""
    y = np.asarray(y, dtype=np.float64)
    m = y.mean(axis=(1, 2))
    s = np.maximum(y.std(axis=(1, 2)), S_FLOOR)
    return m, s


def forward(theta, y, bf16=False, ch=CHANNELS, ms=None):
    """y: (N, H, W).  Returns (o, cache) with o: (N, H, W, 2).  ms = (m, s)
    arrays replace the image statistics (to evaluate a crop of a larger image:
    an output pixel depends on the input within 6 pixels)."""
    y = np.asarray(y, dtype=np.float64)
    m, s = normalise(y) if ms is None else (np.asarray(ms[0], np.float64), np.asarray(ms[1], np.float64))
    x0 = ((y - m[:, None, None]) / s[:, None, None])
    if bf16:
        x0 = np.asarray(x0, np.float32).astype(np.float64)   # the GPU forms x0 in float32
    x0 = x0[..., None]
    layers = unpack(theta, ch)
    rw = (lambda w: bf16_round(w)) if bf16 else (lambda w: w)
    ra = (lambda a: bf16_round(a)) if bf16 else (lambda a: a)
    acts = [x0]
    a = x0
    for li, (w, b) in enumerate(layers):
        z = conv3x3(a, rw(w), b)
        if li < len(layers) - 1:
            a = ra(np.maximum(z, 0.0))
            acts.append(a)
        else:
            o = z
    return o, {"m": m, "s": s, "acts": acts, "bf16": bf16}


def outputs(o, cache, xi):
    """(mu_hat, v_hat) from the network output."""
    m, s = cache["m"], cache["s"]
    mu = m[:, None, None] + s[:, None, None] * o[..., 0]
    v = xi * np.exp(o[..., 1])
    return mu, v


def targets(mu, v, cache, xi):
    m, s = cache["m"], cache["s"]
    t0 = (np.asarray(mu, np.float64) - m[:, None, None]) / s[:, None, None]
    t1 = np.log(np.asarray(v, np.float64) / xi)
    return np.stack([t0, t1], axis=-1)


def loss(o, t):
    n = o.shape[0] * o.shape[1] * o.shape[2]
    return float(np.sum((o - t) ** 2) / n)


def backward(theta, o, t, cache, ch=CHANNELS):
    """Gradient of `loss` with respect to theta (flat, canonical order)."""
    bf16 = cache["bf16"]
    layers = unpack(theta, ch)
    rw = (lambda w: bf16_round(w)) if bf16 else (lambda w: w)
    rg = (lambda g: bf16_round(g)) if bf16 else (lambda g: g)
    n = o.shape[0] * o.shape[1] * o.shape[2]
    g = 2.0 * (o - t) / n                    # dL/dz of the last layer (kept in float32 on the GPU)
    if bf16:
        g = np.asarray(g, np.float32).astype(np.float64)
    acts = cache["acts"]
    grads = [None] * len(layers)
    for li in range(len(layers) - 1, -1, -1):
        w, _ = layers[li]
        a_in = acts[li]
        grads[li] = (conv3x3_weight_grad(a_in, g), g.sum(axis=(0, 1, 2)))
        if li > 0:
            g = rg(conv3x3_input_grad(g, rw(w)) * (a_in > 0))
    return pack(grads)


def loss_and_grad(theta, y, mu, v, xi, bf16=False):
    o, cache = forward(theta, y, bf16)
    t = targets(mu, v, cache, xi)
    return loss(o, t), backward(theta, o, t, cache), o


class Adam:
    """Adam with bias correction (Kingma & Ba, 2015, Algorithm 1)."""

    def __init__(self, n, beta1=0.9, beta2=0.999, eps=1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.b1, self.b2, self.eps = beta1, beta2, eps

    def step(self, theta, g, lr):
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * g
        self.v = self.b2 * self.v + (1 - self.b2) * g * g
        mh = self.m / (1 - self.b1 ** self.t)
        vh = self.v / (1 - self.b2 ** self.t)
        return theta - lr * mh / (np.sqrt(vh) + self.eps)
