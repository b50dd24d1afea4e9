"""CPU checks of the C-ABI library: it loads, exports every symbol that the
headers under include/ declare, and validates descriptors on the host."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2110_01585_amd import _native as N
from paper_2110_01585_amd import ProblemSpec, ep_tv_workspace_bytes, EPTVError

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in sorted(os.listdir(os.path.join(ROOT, "include")))
           if h.endswith(".h")]


def _declared():
    names = set()
    for h in HEADERS:
        with open(h) as f:
            src = re.sub(r"/\*.*?\*/", "", f.read(), flags=re.S)
        names |= set(re.findall(r"\b(ep_tv_[a-z_0-9]+)\s*\(", src))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    lib = N.lib()
    declared = _declared()
    assert len(declared) >= 30
    for name in declared:
        assert hasattr(lib, name), name
        assert name in N.SIGNATURES, f"binding lacks {name}"
    out = subprocess.run(["nm", "-D", "--defined-only", N.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (ep_tv_\w+)", out))
    assert set(declared) <= exported


def test_version():
    assert N.lib().ep_tv_version().decode().startswith("eptv-gfx950")


def test_workspace_bytes_and_validation():
    ok = ProblemSpec(128, 128, noise_var=0.01, lambda0=10.0, damping=0.5)
    b1 = ep_tv_workspace_bytes([ok])
    b2 = ep_tv_workspace_bytes([ok, ProblemSpec(300, 17)])
    assert b1 >= 128 * 128 * (5 * 8 + 4) and b2 > b1
    # the mixture factors: BG ignores s2^2
    ep_tv_workspace_bytes([ProblemSpec(9, 9, prior=N.PRIOR_BG, prior_omega=0.2, prior_s1sq=0.3, prior_s2sq=0.0)])
    ep_tv_workspace_bytes([ProblemSpec(9, 9, prior=N.PRIOR_MOG2, prior_omega=1.0, prior_s1sq=0.3, prior_s2sq=1e-3)])
    # the Walsh-Hadamard operator: power-of-two sizes in [4, 4096] with a mask
    hb = ep_tv_workspace_bytes([ProblemSpec(64, 32, op=N.OP_HADAMARD_MASK, mask=np.ones((64, 32), np.uint8))])
    assert hb >= 64 * 32 * (5 * 8 + 4 + 2 * 4)
    # the largest accepted sizes (16384 on a side) size without error
    big = ep_tv_workspace_bytes([ProblemSpec(16384, 3), ProblemSpec(2, 16384)])
    assert big >= (16384 * 3 + 2 * 16384) * (5 * 8)
    # the RBMC estimator: Ns planes of noise, H^T e1 and sample solutions on top
    blur = dict(op=N.OP_BLUR_PERIODIC, taps=np.ones((3, 3), np.float32) / 9)
    b_spec = ep_tv_workspace_bytes([ProblemSpec(64, 64, **blur)])
    b_rbmc = ep_tv_workspace_bytes([ProblemSpec(64, 64, var_estimator=N.VAR_RBMC, rbmc_samples=4, **blur)])
    assert b_rbmc >= b_spec + 64 * 65 * 4 * (3 * 4 + 2)
    for bad_rbmc in (ProblemSpec(8, 8, var_estimator=N.VAR_RBMC, rbmc_samples=0, **blur),
                     ProblemSpec(8, 8, var_estimator=N.VAR_RBMC, rbmc_samples=65, **blur),
                     ProblemSpec(8, 8, var_estimator=2, **blur)):
        with pytest.raises(EPTVError):
            ep_tv_workspace_bytes([bad_rbmc])
    # the smallest transform images (one 4 x 4 block) are accepted
    for op in (N.OP_HADAMARD_MASK, N.OP_DFT_MASK):
        assert ep_tv_workspace_bytes([ProblemSpec(4, 4, op=op, mask=np.ones((4, 4), np.uint8))]) > 0
    bad = [ProblemSpec(0, 5), ProblemSpec(5, 5, noise_var=0.0), ProblemSpec(5, 5, lambda0=-1),
           ProblemSpec(5, 5, damping=0.0), ProblemSpec(5, 5, damping=1.5),
           ProblemSpec(5, 6, boundary=N.BND_PERIODIC),
           ProblemSpec(8, 8, op=N.OP_BLUR_PERIODIC, taps=np.ones((4, 3), np.float32)),
           ProblemSpec(8, 8, op=N.OP_BLUR_PERIODIC),
           ProblemSpec(12, 8, op=N.OP_DFT_MASK, mask=np.ones((12, 8), np.uint8)),
           ProblemSpec(8, 8, op=7), ProblemSpec(5, 5, cg_reduce=1.0), ProblemSpec(5, 5, cg_reduce=-0.1),
           ProblemSpec(16385, 4), ProblemSpec(4, 16385), ProblemSpec(5, 5, prior=7),
           ProblemSpec(5, 5, prior=N.PRIOR_MOG2, prior_omega=0.0),
           ProblemSpec(5, 5, prior=N.PRIOR_MOG2, prior_omega=1.5),
           ProblemSpec(5, 5, prior=N.PRIOR_MOG2, prior_s2sq=0.0),
           ProblemSpec(5, 5, prior=N.PRIOR_BG, prior_s1sq=-1.0),
           ProblemSpec(16, 16, op=N.OP_HADAMARD_MASK),
           ProblemSpec(12, 16, op=N.OP_HADAMARD_MASK, mask=np.ones((12, 16), np.uint8)),
           ProblemSpec(8192, 4, op=N.OP_HADAMARD_MASK, mask=np.ones((8192, 4), np.uint8)),
           ProblemSpec(8, 8, op=4)]
    for s in bad:
        with pytest.raises(EPTVError):
            ep_tv_workspace_bytes([s])


def test_null_arguments_are_rejected():
    lib = N.lib()
    out = ctypes.c_size_t(0)
    assert lib.ep_tv_workspace_bytes(None, 1, ctypes.byref(out)) == N.EP_TV_E_ARG
    one = (N.EpTvProblem * 1)()
    assert lib.ep_tv_workspace_bytes(one, 0, ctypes.byref(out)) == N.EP_TV_E_ARG   # empty batch
    assert lib.ep_tv_workspace_bytes(one, -1, ctypes.byref(out)) == N.EP_TV_E_ARG
    h = ctypes.c_void_p(None)
    arr = (N.EpTvProblem * 1)()
    assert lib.ep_tv_create(arr, 1, None, 0, None, ctypes.byref(h)) == N.EP_TV_E_ARG
    assert lib.ep_tv_run(None, 1, 0) == N.EP_TV_E_ARG
    assert lib.ep_tv_solve(None, 1, 0.0, 0, None, None, None) == N.EP_TV_E_ARG
    assert lib.ep_tv_last_error(None) == b"null context"
    lib.ep_tv_destroy(None)


def test_net_host_validation():
    lib = N.lib()
    assert lib.ep_tv_net_param_count() == 37890
    nb = ctypes.c_size_t(0)
    assert lib.ep_tv_net_workspace_bytes(16, 256, 256, ctypes.byref(nb)) == 0
    assert nb.value > 16 * 256 * 256 * 64 * 7
    for bad in [(0, 8, 8), (1, 0, 8), (1, 8, 0), (1, 20000, 8)]:
        assert lib.ep_tv_net_workspace_bytes(*bad, ctypes.byref(nb)) == N.EP_TV_E_ARG
    h = ctypes.c_void_p(None)
    assert lib.ep_tv_net_create(None, None, 0, 1, 8, 8, None, ctypes.byref(h)) == N.EP_TV_E_ARG
    assert lib.ep_tv_net_adam_count(None) == -1
    assert lib.ep_tv_init_warm(None, None, None, 1.0, 1.0) == N.EP_TV_E_ARG
