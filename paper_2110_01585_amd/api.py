"""Thin Python binding of the C ABI (argument marshalling only).

Every function here forwards to the entry point of the same name in
libeptv.so; torch supplies device memory (the workspace and the caller's
image tensors) and the current HIP stream.  No EP arithmetic runs in Python.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

from . import _native as N


class EPTVError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{N.STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


@dataclass
class ProblemSpec:
    """Host description of one instance (mirrors ep_tv_problem)."""
    height: int
    width: int
    op: int = N.OP_IDENTITY
    boundary: int = N.BND_FREE
    noise_var: float = 0.01
    lambda0: float = 1.0
    damping: float = 0.5
    taps: Optional[np.ndarray] = None
    mask: Optional[np.ndarray] = None
    cg_tol: float = 0.0          # 0 = library default
    cg_max_iters: int = 0        # 0 = library default
    cg_precond: int = N.PRECOND_AUTO
    cg_reduce: float = 0.0       # 0 = every solve to cg_tol
    prior: int = N.PRIOR_L1      # N.PRIOR_*; the mixtures take the three fields below
    prior_omega: float = 1.0
    prior_s1sq: float = 1.0
    prior_s2sq: float = 1.0
    var_estimator: int = N.VAR_SPECTRAL
    rbmc_samples: int = 0
    noise_map: bool = False      # per-pixel noise variances (identity operator)
    sense: Optional[np.ndarray] = None   # Gaussian CS: M x (H W) sensing matrix


_OPS = {"identity": N.OP_IDENTITY, "blur": N.OP_BLUR_PERIODIC, "dft": N.OP_DFT_MASK,
        "hadamard": N.OP_HADAMARD_MASK, "gauss": N.OP_GAUSS_CS}
_BNDS = {"free": N.BND_FREE, "periodic": N.BND_PERIODIC}


def spec_from_synthetic(p, lam0=None, damping=None, cg_tol=0.0, cg_max_iters=0,
                        cg_precond=N.PRECOND_AUTO, cg_reduce=0.0, rbmc_samples=0) -> ProblemSpec:
    """ProblemSpec of a synthetic.Problem (same fields, C enums); rbmc_samples > 0
    selects the RBMC variance estimator with that many samples."""
    h, w = p.shape
    return ProblemSpec(h, w, _OPS[p.op], _BNDS[p.boundary], float(p.xi),
                       float(p.lam0 if lam0 is None else lam0),
                       float(p.damping if damping is None else damping),
                       taps=None if p.taps is None else np.asarray(p.taps, np.float32),
                       mask=None if p.mask is None else np.asarray(p.mask, np.uint8),
                       cg_tol=cg_tol, cg_max_iters=cg_max_iters, cg_precond=cg_precond,
                       cg_reduce=cg_reduce,
                       var_estimator=N.VAR_RBMC if rbmc_samples else N.VAR_SPECTRAL,
                       rbmc_samples=int(rbmc_samples),
                       sense=None if getattr(p, "sense", None) is None
                       else np.asarray(p.sense, np.float32))


def _problems(specs: Sequence[ProblemSpec]):
    arr = (N.EpTvProblem * len(specs))()
    keep = []
    for i, s in enumerate(specs):
        a = arr[i]
        a.height, a.width, a.op, a.boundary = s.height, s.width, s.op, s.boundary
        a.noise_var, a.lambda0, a.damping = s.noise_var, s.lambda0, s.damping
        a.cg_tol, a.cg_max_iters, a.cg_precond = s.cg_tol, s.cg_max_iters, s.cg_precond
        a.cg_reduce = s.cg_reduce
        a.prior, a.prior_omega, a.prior_s1sq, a.prior_s2sq = s.prior, s.prior_omega, s.prior_s1sq, s.prior_s2sq
        a.var_estimator, a.rbmc_samples = s.var_estimator, s.rbmc_samples
        a.noise_map = 1 if s.noise_map else 0
        if s.sense is not None:
            hm = np.ascontiguousarray(s.sense, dtype=np.float32)
            keep.append(hm)
            a.sense_matrix = hm.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
            a.sense_rows = hm.shape[0]
        if s.taps is not None:
            t = np.ascontiguousarray(s.taps, dtype=np.float32)
            keep.append(t)
            a.blur_taps = t.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
            a.blur_h, a.blur_w = t.shape
        if s.mask is not None:
            m = np.ascontiguousarray(s.mask, dtype=np.uint8)
            keep.append(m)
            a.dft_mask = m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    return arr, keep


def _ptrs(tensors):
    arr = (ctypes.c_void_p * len(tensors))()
    for i, t in enumerate(tensors):
        arr[i] = None if t is None else t.data_ptr()
    return arr


def ep_tv_version() -> str:
    return N.lib().ep_tv_version().decode()


def ep_tv_workspace_bytes(specs: Sequence[ProblemSpec]) -> int:
    arr, _keep = _problems(specs)
    out = ctypes.c_size_t(0)
    rc = N.lib().ep_tv_workspace_bytes(arr, len(specs), ctypes.byref(out))
    if rc != 0:
        raise EPTVError(rc, "invalid problem description")
    return int(out.value)


def ep_tv_tilted_moments_prior(prior, theta, m, s, stream=None):
    """rho, delta and E|u| (0 for the mixtures) of N(u; m, s) phi(u) for the factor
    kind `prior` (N.PRIOR_*) with hyperparameters theta ({lambda}, {omega, s1^2,
    s2^2} or {omega, s^2}).  m, s: contiguous float32 CUDA tensors."""
    import torch
    n = m.numel()
    rho = torch.empty_like(m); de = torch.empty_like(m); ea = torch.empty_like(m)
    th = (ctypes.c_double * 3)(*([float(t) for t in theta] + [0.0] * (3 - len(theta))))
    st = stream if stream is not None else torch.cuda.current_stream()
    rc = N.lib().ep_tv_tilted_moments_prior(int(prior), th, n, m.data_ptr(), s.data_ptr(), rho.data_ptr(),
                                            de.data_ptr(), ea.data_ptr(), st.cuda_stream)
    if rc != 0:
        raise EPTVError(rc, "ep_tv_tilted_moments_prior failed")
    return rho, de, ea


def ep_tv_tilted_moments(m, s, lam, stream=None):
    """rho = 1 - Var/s, delta = E[u] - m, E|u| of N(u; m, s) exp(-lam |u|) on the GPU.
    m, s: contiguous float32 CUDA tensors of equal length."""
    import torch
    n = m.numel()
    rho = torch.empty_like(m); de = torch.empty_like(m); ea = torch.empty_like(m)
    st = stream if stream is not None else torch.cuda.current_stream()
    rc = N.lib().ep_tv_tilted_moments(n, m.data_ptr(), s.data_ptr(), float(lam), rho.data_ptr(),
                                      de.data_ptr(), ea.data_ptr(), st.cuda_stream)
    if rc != 0:
        raise EPTVError(rc, "ep_tv_tilted_moments failed")
    return rho, de, ea


def ep_tv_denoise_noalloc(y, noise_var, lam, damping, n_sweeps, em, mean, var,
                          boundary=N.BND_FREE, stream=None):
    """Forward to ep_tv_denoise_noalloc (no allocation inside the library):
    y, mean, var are contiguous float32 device tensors of one H x W image."""
    import torch
    for t in (y, mean, var):
        if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
            raise ValueError("expected contiguous float32 CUDA tensors")
    h, w = y.shape
    if mean.shape != y.shape or var.shape != y.shape:
        raise ValueError("mean and var must have the shape of y")
    s = stream if stream is not None else torch.cuda.current_stream(y.device)
    rc = N.lib().ep_tv_denoise_noalloc(int(h), int(w), int(boundary), float(noise_var), float(lam),
                                       float(damping), int(n_sweeps), int(bool(em)), y.data_ptr(),
                                       mean.data_ptr(), var.data_ptr(),
                                       ctypes.c_void_p(s.cuda_stream))
    if rc != 0:
        raise EPTVError(rc, "ep_tv_denoise_noalloc failed (sizes above 512, or invalid arguments)")
    return rc


class Context:
    """Owns a libeptv context and the torch workspace tensor backing it."""

    def __init__(self, specs: Sequence[ProblemSpec], device="cuda", stream=None):
        import torch
        self.torch = torch
        self.specs = list(specs)
        self.n = len(self.specs)
        nbytes = ep_tv_workspace_bytes(self.specs)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        self._ws_ptr = aligned
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        arr, keep = _problems(self.specs)
        h = ctypes.c_void_p(None)
        rc = N.lib().ep_tv_create(arr, self.n, ctypes.c_void_p(aligned), nbytes,
                                  ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if rc != 0:
            raise EPTVError(rc, "ep_tv_create failed (invalid arguments or workspace)")
        self.handle = h
        self._y = None

    # -- helpers --
    def _check(self, rc, what, ok=(0,)):
        if rc not in ok:
            msg = N.lib().ep_tv_last_error(self.handle)
            raise EPTVError(rc, f"{what}: {msg.decode() if msg else ''}")
        return rc

    def _dev(self, t, shape):
        torch = self.torch
        if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
            raise ValueError("expected a contiguous float32 CUDA tensor")
        if t.numel() != int(np.prod(shape)):
            raise ValueError(f"expected {shape}, got {tuple(t.shape)}")
        return t

    # -- entry points --
    def ep_tv_set_observation(self, ys):
        def shape(s):
            if s.op == N.OP_DFT_MASK:
                return (s.height, s.width, 2)
            if s.op == N.OP_GAUSS_CS:
                return (s.sense.shape[0],)
            return (s.height, s.width)
        ys = [self._dev(y, shape(s)) for y, s in zip(ys, self.specs)]
        self._y = ys
        return self._check(N.lib().ep_tv_set_observation(self.handle, _ptrs(ys)), "set_observation")

    def ep_tv_set_rbmc_noise(self, noises):
        """noises: per instance a contiguous float32 device tensor of
        rbmc_samples * (K + H*W) values (layout in include/ep_tv.h), or None."""
        for t, s in zip(noises, self.specs):
            if t is None or s.rbmc_samples == 0 or s.op == N.OP_IDENTITY:
                continue
            k = s.height * s.width * (2 if s.op == N.OP_DFT_MASK else 1)
            self._dev(t, (s.rbmc_samples * (k + s.height * s.width),))
        return self._check(N.lib().ep_tv_set_rbmc_noise(self.handle, _ptrs(noises)), "set_rbmc_noise")

    def ep_tv_set_noise_variance(self, variances):
        """variances: per instance a contiguous (H, W) float32 device tensor, or None
        for instances without a noise map."""
        vs = [None if v is None else self._dev(v, (s.height, s.width))
              for v, s in zip(variances, self.specs)]
        self._noise = vs
        return self._check(N.lib().ep_tv_set_noise_variance(self.handle, _ptrs(vs)),
                           "set_noise_variance")

    def ep_tv_init_cold(self):
        return self._check(N.lib().ep_tv_init_cold(self.handle), "init_cold")

    def ep_tv_run(self, n_sweeps: int, em: bool):
        return self._check(N.lib().ep_tv_run(self.handle, int(n_sweeps), int(bool(em))), "run")

    def ep_tv_em_step(self, n_ep_sweeps: int = 1, want_lambda=True):
        out = (ctypes.c_double * self.n)() if want_lambda else None
        self._check(N.lib().ep_tv_em_step(self.handle, int(n_ep_sweeps), out), "em_step")
        return list(out) if want_lambda else None

    def ep_tv_solve(self, max_sweeps: int, tol: float, em: bool, means=None, variances=None):
        st = (N.EpTvStats * self.n)()
        mp = _ptrs(means) if means is not None else None
        vp = _ptrs(variances) if variances is not None else None
        rc = N.lib().ep_tv_solve(self.handle, int(max_sweeps), float(tol), int(bool(em)), mp, vp, st)
        self._check(rc, "solve", ok=(0, 1, 2))
        return rc, [self._stats_dict(s) for s in st]

    def ep_tv_marginals(self, means=None, variances=None):
        mp = _ptrs(means) if means is not None else None
        vp = _ptrs(variances) if variances is not None else None
        return self._check(N.lib().ep_tv_marginals(self.handle, mp, vp), "marginals")

    def ep_tv_get_sites(self, outs):
        return self._check(N.lib().ep_tv_get_sites(self.handle, _ptrs(outs)), "get_sites")

    def ep_tv_set_sites(self, ins, lambdas=None):
        lam = (ctypes.c_double * self.n)(*lambdas) if lambdas is not None else None
        return self._check(N.lib().ep_tv_set_sites(self.handle, _ptrs(ins), lam), "set_sites")

    def ep_tv_get_stats(self):
        st = (N.EpTvStats * self.n)()
        self._check(N.lib().ep_tv_get_stats(self.handle, st), "get_stats")
        return [self._stats_dict(s) for s in st]

    def ep_tv_get_lik_planes(self, instance: int, out):
        return self._check(N.lib().ep_tv_get_lik_planes(self.handle, int(instance), out.data_ptr()),
                           "get_lik_planes")

    def ep_tv_set_timing(self, enable: bool):
        return self._check(N.lib().ep_tv_set_timing(self.handle, int(bool(enable))), "set_timing")

    def ep_tv_get_timing(self):
        t = N.EpTvTiming()
        self._check(N.lib().ep_tv_get_timing(self.handle, ctypes.byref(t)), "get_timing")
        return {name: getattr(t, name) for name, _ in N.EpTvTiming._fields_}

    def ep_tv_init_warm(self, mu_hats, var_hats, lambda_scale: float = 1.0,
                        lambda_power: float = 1.0) -> int:
        """Returns the status (EP_TV_OK or EP_TV_W_WARM_FALLBACK)."""
        rc = N.lib().ep_tv_init_warm(self.handle, _ptrs(mu_hats), _ptrs(var_hats), float(lambda_scale),
                                     float(lambda_power))
        return self._check(rc, "init_warm", ok=(0, N.EP_TV_W_WARM_FALLBACK))

    def ep_tv_set_option(self, option: int, value: int):
        return self._check(N.lib().ep_tv_set_option(self.handle, int(option), int(value)), "set_option")

    def ep_tv_get_option(self, option: int) -> int:
        v = ctypes.c_int64(0)
        self._check(N.lib().ep_tv_get_option(self.handle, int(option), ctypes.byref(v)), "get_option")
        return int(v.value)

    def ep_tv_autotune(self, repeats: int = 5):
        r = N.EpTvTuneResult()
        self._check(N.lib().ep_tv_autotune(self.handle, int(repeats), ctypes.byref(r)), "autotune")
        return {"tile_rows": r.tile_rows, "best_ms": r.best_ms, "default_ms": r.default_ms,
                "candidates": {int(r.rows[i]): float(r.ms[i]) for i in range(r.candidates)}}

    @staticmethod
    def _stats_dict(s):
        return {"sweeps": s.sweeps_done, "cg_last": s.cg_iters_last, "cg_total": s.cg_iters_total,
                "clamps": s.clamp_count, "status": s.status, "converged": bool(s.converged),
                "lambda": s.lambda_, "a_bar_u": s.a_bar_u, "dmu": s.max_dmu_rel,
                "dv": s.max_dv_rel, "elapsed_ms": s.elapsed_ms, "gamma": s.lik_precision,
                "dbar": s.cavity_precision_mean, "cg_rel_residual": s.cg_rel_residual,
                "cold_restarts": s.cold_restarts}

    # -- conveniences built only from the entry points above --
    def marginals(self):
        torch = self.torch
        mus = [torch.empty(s.height, s.width, device=self.workspace.device) for s in self.specs]
        vs = [torch.empty(s.height, s.width, device=self.workspace.device) for s in self.specs]
        self.ep_tv_marginals(mus, vs)
        return mus, vs

    def close(self):
        if getattr(self, "handle", None):
            N.lib().ep_tv_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
