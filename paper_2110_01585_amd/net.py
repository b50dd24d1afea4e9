"""Thin binding of the learned warm start (include/ep_tv_net.h).

Net owns the float32 parameter tensor and the workspace (torch device memory)
and forwards every call to libeptv.so.  Weight files are plain little-endian
float32 arrays with a JSON side file (parameter count, training set, the
lambda_0 calibration factor); loading them executes nothing.
"""
from __future__ import annotations

import ctypes
import json
import os
from typing import Optional

import numpy as np

from . import _native as N
from .api import EPTVError

PKG = os.path.dirname(os.path.abspath(__file__))
WEIGHTS_DIR = os.path.join(PKG, "weights")
DEFAULT_WEIGHTS = os.path.join(WEIGHTS_DIR, "warmstart_deconv_sb2_s001")


def param_count() -> int:
    return int(N.lib().ep_tv_net_param_count())


def init_params(seed: int = 0) -> np.ndarray:
    """He-normal weights (std sqrt(2 / (9 cin))), zero biases, canonical order."""
    rng = np.random.default_rng(seed)
    ch = (1, 32, 32, 32, 32, 32, 2)
    parts = []
    for i in range(6):
        n = 9 * ch[i] * ch[i + 1]
        parts += [rng.normal(0.0, np.sqrt(2.0 / (9 * ch[i])), size=n), np.zeros(ch[i + 1])]
    return np.concatenate(parts).astype(np.float32)


def save_weights(path: str, params: np.ndarray, meta: dict):
    params = np.asarray(params, dtype="<f4")
    params.tofile(path + ".f32")
    with open(path + ".json", "w") as f:
        json.dump(dict(meta, param_count=int(params.size)), f, indent=1, sort_keys=True)


def load_weights(path: str = DEFAULT_WEIGHTS):
    with open(path + ".json") as f:
        meta = json.load(f)
    params = np.fromfile(path + ".f32", dtype="<f4")
    if params.size != meta["param_count"]:
        raise ValueError(f"{path}.f32 holds {params.size} values, expected {meta['param_count']}")
    return params.astype(np.float32), meta


class Net:
    def __init__(self, params: Optional[np.ndarray] = None, max_batch=1, max_h=256, max_w=256,
                 device="cuda", stream=None):
        import torch
        self.torch = torch
        n = param_count()
        p = init_params(0) if params is None else np.asarray(params, np.float32)
        if p.size != n:
            raise ValueError(f"expected {n} parameters")
        self.params = torch.tensor(p, device=device)
        nb = ctypes.c_size_t(0)
        rc = N.lib().ep_tv_net_workspace_bytes(max_batch, max_h, max_w, ctypes.byref(nb))
        if rc:
            raise EPTVError(rc, "ep_tv_net_workspace_bytes")
        self.workspace = torch.empty(nb.value + 256, dtype=torch.uint8, device=device)
        aligned = (self.workspace.data_ptr() + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p(None)
        rc = N.lib().ep_tv_net_create(ctypes.c_void_p(self.params.data_ptr()), ctypes.c_void_p(aligned),
                                      nb.value, max_batch, max_h, max_w,
                                      ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if rc:
            raise EPTVError(rc, "ep_tv_net_create")
        self.handle = h

    def _check(self, rc, what):
        if rc != 0:
            msg = N.lib().ep_tv_net_last_error(self.handle)
            raise EPTVError(rc, f"{what}: {msg.decode() if msg else ''}")

    def set_params(self, params):
        self.params.copy_(self.torch.as_tensor(np.asarray(params, np.float32)))
        self._check(N.lib().ep_tv_net_sync(self.handle), "sync")

    def infer(self, y, noise_var, mu_out=None, var_out=None):
        """y: (batch, h, w) or (h, w) float32 CUDA tensor."""
        t = self.torch
        y3 = y if y.dim() == 3 else y.unsqueeze(0)
        b, h, w = y3.shape
        mu = mu_out if mu_out is not None else t.empty_like(y)
        var = var_out if var_out is not None else t.empty_like(y)
        self._check(N.lib().ep_tv_net_infer(self.handle, ctypes.c_void_p(y3.data_ptr()), b, h, w,
                                            float(noise_var), ctypes.c_void_p(mu.data_ptr()),
                                            ctypes.c_void_p(var.data_ptr())), "infer")
        return mu, var

    def loss_grad(self, y, mu_t, var_t, noise_var, want_grad=True, want_loss=True):
        t = self.torch
        b, h, w = y.shape
        g = t.empty_like(self.params) if want_grad else None
        loss = ctypes.c_double(0.0)
        self._check(N.lib().ep_tv_net_loss_grad(
            self.handle, ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(mu_t.data_ptr()),
            ctypes.c_void_p(var_t.data_ptr()), b, h, w, float(noise_var),
            ctypes.c_void_p(g.data_ptr()) if g is not None else None,
            ctypes.byref(loss) if want_loss else None), "loss_grad")
        return (loss.value if want_loss else None), g

    def adam_step(self, lr):
        self._check(N.lib().ep_tv_net_adam_step(self.handle, float(lr)), "adam_step")

    def train_step(self, y, mu_t, var_t, noise_var, lr, want_loss=False):
        b, h, w = y.shape
        loss = ctypes.c_double(0.0)
        self._check(N.lib().ep_tv_net_train_step(
            self.handle, ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(mu_t.data_ptr()),
            ctypes.c_void_p(var_t.data_ptr()), b, h, w, float(noise_var), float(lr),
            ctypes.byref(loss) if want_loss else None), "train_step")
        return loss.value if want_loss else None

    def adam_count(self) -> int:
        return int(N.lib().ep_tv_net_adam_count(self.handle))

    def close(self):
        if getattr(self, "handle", None):
            N.lib().ep_tv_net_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
