"""Shared helpers of the GPU parity tests (not collected by pytest)."""
import numpy as np

MEAN_TOL = 1e-4   # max |mu - mu_oracle| / (max mu_oracle - min mu_oracle)
VAR_TOL = 1e-3    # max |v / v_oracle - 1|


def f32(a):
    """Round an input to float32 and back, so both sides see the same numbers."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def mean_err(mu, mu_ref):
    rng = float(mu_ref.max() - mu_ref.min()) or 1.0
    return float(np.max(np.abs(mu - mu_ref))) / rng


def var_err(v, v_ref):
    return float(np.max(np.abs(v / v_ref - 1.0)))


def to_dev(a, torch, device="cuda"):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float32), device=device)


def observation_tensor(p, torch, device="cuda"):
    """Device observation in the layout ep_tv_set_observation expects."""
    if p.op == "dft":
        y = np.stack([p.y.real, p.y.imag], axis=-1)
        return to_dev(y, torch, device)
    return to_dev(p.y, torch, device)


def f32_problem(p):
    """Copy of a synthetic.Problem whose observation is float32-rounded."""
    import copy
    q = copy.copy(p)
    if p.op == "dft":
        q.y = f32(p.y.real) + 1j * f32(p.y.imag)
    else:
        q.y = f32(p.y)
    if p.taps is not None:
        q.taps = f32(p.taps)
    return q
