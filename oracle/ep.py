"""Plain FP64 EP for TV priors: Algorithm 1 and the fast EP-EM of Algorithm 2.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

State (Sec. III-A): five Gaussian approximating factors q_{x,k}, k = 0..4, with
diagonal covariances, stored as natural parameters per pixel,
tau_k = 1 / Sigma_{x,k} and eta_k = mu_{x,k} / Sigma_{x,k}.  The global
approximation is their product (Eq. (Q_x_final)): tau = sum_k tau_k,
eta = sum_k eta_k, mu_x = eta / tau, v_x = 1 / tau.

Colour classes (Sec. II-B, Fig. 1, Eq. (prior1)), pixel (r, c), row-major,
0-based, i = left/top pixel of the edge, j = right/bottom pixel:
  V1: (r, c)-(r, c+1), c even;   V2: (r, c)-(r, c+1), c odd;
  V3: (r, c)-(r+1, c), r even;   V4: (r, c)-(r+1, c), r odd.
FREE boundary keeps only edges inside the image; PERIODIC (even sizes) adds the
wrap edges (r, W-1)-(r, 0) to V2 and (H-1, c)-(0, c) to V4.  A pixel that no
edge of V_k touches keeps the flat site (tau_k, eta_k) = (0, 0).

One sweep t (where the paper is silent, the reading taken is stated at the step):
  1. likelihood site (Eqs. (tilted_P_1), (update_q0_x)), skipped for H = I,
     where it is exact and constant, and in sweep 1 of a cold start, where the
     initial q_{x,0} of the initialisation line stands in for it
     (``first_sweep_likelihood=True`` runs it at t = 1 as well, Algorithm 1's
     loop body taken literally; both orders reach the same fixed point);
  2. for k in the block order (default 1, 2, 3, 4): every edge of V_k in
     parallel -- cavity, tilted moments of u (Eq. (marginal_tilted_un)),
     Gehre-Jin projection back to (x_i, x_j), site update (Eq. (update_qk_x)),
     negative-variance clamp, damping;
  3. EM (Algorithm 2): lambda <- N / a_0 with N the number of pixels and a_0
     one of the three approximations of Sec. IV (em_option):
       3 (default, Eq. (3rd_alternative_a0)): a_bar_u = sum over all edges of
         the sweep of the tilted E|u_n| at the lambda used in the sweep;
       2 (Eq. (eq:au)): a_u = sum over the edges of E|u_n| under Q(u_n), the
         Gaussian with the tilted mean and variance of u_n (the moments that
         update Q(u_k));
       1 (Eq. (eq:ax)): a_x = sum over the edges of E|x_i - x_j| under the
         global Q(x) after the sweep (x_i - x_j ~ N(mu_i - mu_j, v_i + v_j)).
     All three are folded-normal or tilted means in closed form; the unused
     ones are kept as diagnostics (EPState.a_x, a_u, a_bar).

Parity pins: tests/test_oracle_ep.py (l2-TV fixed point = dense posterior mean,
exact single-edge posterior, EM fixed point = marginal-likelihood maximiser on a
single edge, symmetry invariants, colour-class structure) and
tests/test_oracle_brute.py (3x3 brute-force posterior marginals, the transfer
pass against a direct sum over the joint grid), tests/test_oracle_estimators.py
(the divergence rule; runaway of the spectral estimator on sparse masks).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

from . import operators as ops
from .tilted import folded_normal_mean, tilted

SITE_INIT_PREC = 1e-8     # 1 / 1e8: initial TV-site variance 1e8
PREC_FLOOR = 1e-8         # clamp: site variance negative or above 1e8 -> 1e8
# Divergence rule (the paper gives none; EP is not guaranteed to converge): a run
# is declared diverged once the mean of the global approximation right after a
# likelihood-site update exceeds DIVERGE_FACTOR times the scale of the
# pixel-space observation (the larger of its range and its largest magnitude)
# at some pixel (converging runs stay within about twice that scale, from
# cold on).  The tilted mean E itself is no indicator: where the cavity is
# flat and the operator leaves a direction unobserved it is huge but carries a
# vanishing precision.
DIVERGE_FACTOR = 1e3


def colour_classes(h: int, w: int, boundary: str = "free"):
    """Edge lists (i, j) of flat pixel indices for V1..V4 (index 0..3)."""
    if boundary not in ("free", "periodic"):
        raise ValueError(boundary)
    if boundary == "periodic" and (h % 2 or w % 2):
        raise ValueError("periodic boundary needs even image sizes")
    idx = np.arange(h * w).reshape(h, w)
    out = []
    for parity in (0, 1):              # horizontal: V1 (c even), V2 (c odd)
        i_list, j_list = [], []
        for c in range(parity, w, 2):
            if c + 1 < w:
                i_list.append(idx[:, c]); j_list.append(idx[:, c + 1])
            elif boundary == "periodic":
                i_list.append(idx[:, c]); j_list.append(idx[:, 0])
        out.append((np.concatenate(i_list) if i_list else np.zeros(0, int),
                    np.concatenate(j_list) if j_list else np.zeros(0, int)))
    for parity in (0, 1):              # vertical: V3 (r even), V4 (r odd)
        i_list, j_list = [], []
        for r in range(parity, h, 2):
            if r + 1 < h:
                i_list.append(idx[r, :]); j_list.append(idx[r + 1, :])
            elif boundary == "periodic":
                i_list.append(idx[r, :]); j_list.append(idx[0, :])
        out.append((np.concatenate(i_list) if i_list else np.zeros(0, int),
                    np.concatenate(j_list) if j_list else np.zeros(0, int)))
    return out


@dataclass
class EPState:
    tau: np.ndarray                 # (5, N)
    eta: np.ndarray                 # (5, N)
    lam: float                      # l1: lambda; l2: beta
    E: Optional[np.ndarray] = None  # last tilted mean of the likelihood site (CG warm start)
    clamp_count: int = 0
    cg_iters: int = 0
    history: list = field(default_factory=list)
    warm: bool = False              # sites carry information already: no skipped q0 update
    lik_mu_absmax: float = 0.0      # max |mu| of the global approximation after the last q0 update
    rbmc: Optional[ops.RBMCSamples] = None   # RBMC inputs and per-sample CG starts
    a_bar: float = 0.0              # last sweep's a_0, option 3 (tilted E|u|)
    a_u: float = 0.0                # option 2 (E|u| under Q(u)), when computed
    a_x: float = 0.0                # option 1 (E|x_i - x_j| under Q(x)), when computed
    # marginal (mu, v) right after this sweep's likelihood-site update, or None
    # when the sweep did not update that site (the convergence rule's reference)
    mid: Optional[tuple] = None


class EPProblem:
    """Everything Algorithm 1 takes as input (y, H, xi, theta) plus the readings'
    knobs: damping, boundary, block order, prior, variance estimator."""

    def __init__(self, y, op: ops.Operator, xi, lam, damping=0.5, prior="l1",
                 boundary="free", order: Sequence[int] = (1, 2, 3, 4),
                 estimator="spectral", cg_rtol=1e-12, first_sweep_likelihood=False,
                 rbmc_noise=None, em_option=3, em_diagnostics=False, noise_var_map=None):
        self.op = op
        self.h, self.w = op.shape
        self.N = self.h * self.w
        self.xi = float(xi)
        # l1: lambda; l2: beta; mog2: (omega, s1^2, s2^2); bg: (omega, s^2)
        self.lam0 = tuple(float(t) for t in lam) if prior in ("mog2", "bg") else float(lam)
        self.damping = float(damping)
        self.prior = prior
        self.boundary = boundary
        self.order = tuple(order)
        self.estimator = estimator
        self.cg_rtol = cg_rtol
        self.first_sweep_likelihood = bool(first_sweep_likelihood)
        # RBMC estimator: (e1, e2) white noise, Ns images each (operators.RBMCSamples)
        self.rbmc_noise = rbmc_noise
        if estimator == "rbmc" and rbmc_noise is None:
            raise ValueError("the RBMC estimator needs white-noise samples (rbmc_noise)")
        if em_option not in (1, 2, 3):
            raise ValueError("em_option must be 1, 2 or 3")
        self.em_option = em_option
        self.em_diagnostics = bool(em_diagnostics)   # compute all three a_0 every sweep
        # non-i.i.d. noise (Sec. III-C, after Eq. (tilted_P_1)): a per-pixel noise
        # variance for denoising, where the likelihood factor stays exact: q_{x,0}
        # = N(y, diag(xi_i)) and it is never updated
        self.noise_prec = None
        if noise_var_map is not None:
            if op.kind != ops.IDENTITY:
                raise ValueError("per-pixel noise variances are supported for denoising")
            nv = np.asarray(noise_var_map, np.float64)
            if nv.shape != op.shape or not np.all(nv > 0):
                raise ValueError("noise_var_map must hold one positive variance per pixel")
            self.noise_prec = (1.0 / nv).ravel()
        self.y = y
        self.hty = op.Hty(y)
        self.edges = colour_classes(self.h, self.w, boundary)
        self.covered = np.zeros((4, self.N), dtype=bool)
        for k in range(4):
            i, j = self.edges[k]
            self.covered[k, i] = True
            self.covered[k, j] = True


def problem_from_synthetic(p, prior="l1", estimator="spectral", boundary=None, order=(1, 2, 3, 4),
                           lam=None, damping=None, rbmc_noise=None, em_option=3):
    """Build an EPProblem from a synthetic.Problem."""
    op = ops.Operator(p.op, p.shape, taps=p.taps, mask=p.mask, sense=getattr(p, "sense", None))
    return EPProblem(p.y, op, p.xi, p.lam0 if lam is None else lam,
                     damping=p.damping if damping is None else damping, prior=prior,
                     boundary=p.boundary if boundary is None else boundary, order=order,
                     estimator=estimator, rbmc_noise=rbmc_noise, em_option=em_option)


def init_cold(pb: EPProblem) -> EPState:
    """Initialisation line of Algorithm 1: q_{x,0} = N(y, xi I) when y lives in
    pixel space (denoising, deconvolution); for the masked DFT and Walsh-Hadamard
    operators, whose y are transform coefficients, the pixel-space
    back-projection H^T y takes its place.
    TV sites get variance 1e8 where covered."""
    N = pb.N
    tau = np.zeros((5, N))
    eta = np.zeros((5, N))
    prec0 = 1.0 / pb.xi if pb.noise_prec is None else pb.noise_prec
    tau[0] = prec0
    y0 = pb.hty if pb.op.kind in (ops.DFT, ops.HADAMARD, ops.GAUSS) else np.asarray(pb.y, dtype=np.float64)
    eta[0] = y0.ravel() * prec0
    for k in range(4):
        tau[k + 1, pb.covered[k]] = SITE_INIT_PREC
    return EPState(tau=tau, eta=eta, lam=pb.lam0)


def marginals(st: EPState):
    """Eq. (Q_x_final): global precision/mean from the sum of all five sites."""
    tau = st.tau.sum(axis=0)
    eta = st.eta.sum(axis=0)
    return eta / tau, 1.0 / tau


def cavity(st: EPState, k: int):
    """Natural parameters of Q^{\\k} = Q / q_{x,k}: leave-one-out sums (Sec. III-B)."""
    others = [l for l in range(5) if l != k]
    return st.tau[others].sum(axis=0), st.eta[others].sum(axis=0)


def likelihood_site_update(pb: EPProblem, st: EPState):
    """Update q_{x,0} (Eqs. (tilted_P_1) and (update_q0_x)), clamp, damp."""
    tau_c, eta_c = cavity(st, 0)
    shape = (pb.h, pb.w)
    b = (pb.hty / pb.xi) + eta_c.reshape(shape)
    x0 = st.E
    if x0 is None:
        x0 = marginals(st)[0].reshape(shape)
    E, it = ops.solve_tilted_mean(pb.op, pb.xi, tau_c.reshape(shape), b, x0=x0, rtol=pb.cg_rtol)
    st.E = E
    st.cg_iters = it
    if pb.estimator == "rbmc" and st.rbmc is None:
        st.rbmc = ops.RBMCSamples(*pb.rbmc_noise)
    V = ops.tilted_variance(pb.op, pb.xi, tau_c.reshape(shape), pb.estimator, st.rbmc).ravel()
    E = E.ravel()
    tau_new = 1.0 / V - tau_c
    clamp = tau_new < PREC_FLOOR
    st.clamp_count += int(clamp.sum())
    tau_new = np.where(clamp, PREC_FLOOR, tau_new)
    eta_new = (tau_new + tau_c) * E - eta_c
    a = pb.damping
    st.tau[0] = a * tau_new + (1.0 - a) * st.tau[0]
    st.eta[0] = a * eta_new + (1.0 - a) * st.eta[0]
    st.lik_mu_absmax = float(np.max(np.abs((st.eta[0] + eta_c) / (st.tau[0] + tau_c))))


def tv_block_update(pb: EPProblem, st: EPState, k: int) -> float:
    """Update q_{x,k} for every edge of V_k in parallel (k = 1..4).
    Returns the sum over the block's edges of the tilted E|u_n|."""
    i, j = pb.edges[k - 1]
    if i.size == 0:
        return 0.0
    tau_c, eta_c = cavity(st, k)
    ci = 1.0 / tau_c[i]
    cj = 1.0 / tau_c[j]
    mi = eta_c[i] * ci
    mj = eta_c[j] * cj
    m = mi - mj
    s = ci + cj
    m_bar, S_bar, e_abs = tilted(pb.prior, m, s, st.lam)
    if pb.em_option == 2 or pb.em_diagnostics:
        st.a_u += float(folded_normal_mean(m_bar, S_bar).sum())
    # Gehre-Jin projection of the tilted moments of u back to (x_i, x_j)
    Ei = mi + (m_bar - m) / s * ci
    Ej = mj - (m_bar - m) / s * cj
    Vi = ci + (S_bar - s) / (s * s) * ci * ci
    Vj = cj + (S_bar - s) / (s * s) * cj * cj
    a = pb.damping
    for idx, Ep, Vp, cp in ((i, Ei, Vi, ci), (j, Ej, Vj, cj)):
        tau_new = 1.0 / Vp - 1.0 / cp
        clamp = tau_new < PREC_FLOOR
        st.clamp_count += int(clamp.sum())
        tau_new = np.where(clamp, PREC_FLOOR, tau_new)
        eta_new = (tau_new + 1.0 / cp) * Ep - eta_c[idx]
        st.tau[k, idx] = a * tau_new + (1.0 - a) * st.tau[k, idx]
        st.eta[k, idx] = a * eta_new + (1.0 - a) * st.eta[k, idx]
    return float(e_abs.sum())


def a_x(pb: EPProblem, mu, v):
    """Option 1 of Sec. IV: sum over all edges of E|x_i - x_j| under N(mu, diag v)."""
    mu = np.asarray(mu, np.float64).ravel()
    v = np.asarray(v, np.float64).ravel()
    tot = 0.0
    for k in range(4):
        i, j = pb.edges[k]
        tot += float(folded_normal_mean(mu[i] - mu[j], v[i] + v[j]).sum())
    return tot


def sweep(pb: EPProblem, st: EPState, t: int, em: bool) -> float:
    """Sweep t (1-based).  Returns a_bar_u (option 3) of the sweep."""
    st.mid = None
    if pb.op.kind != ops.IDENTITY and (t > 1 or st.warm or pb.first_sweep_likelihood):
        likelihood_site_update(pb, st)
        st.mid = marginals(st)
    a_bar = 0.0
    st.a_u = 0.0
    for k in pb.order:
        a_bar += tv_block_update(pb, st, k)
    st.a_bar = a_bar
    if pb.em_option == 1 or pb.em_diagnostics:
        st.a_x = a_x(pb, *marginals(st))
    if em:
        if pb.prior != "l1":
            raise ValueError("EM is defined for the l1-TV prior only")
        a0 = {1: st.a_x, 2: st.a_u, 3: a_bar}[pb.em_option]
        if a0 > 0.0:                 # an image without edges has nothing to re-estimate
            st.lam = pb.N / a0
    return a_bar


def solve(pb: EPProblem, sweeps: int, em: bool, tol: Optional[float] = None,
          state: Optional[EPState] = None, record=False):
    """Run up to ``sweeps`` sweeps.  With ``tol`` set, stop at the first sweep
    whose changes satisfy the convergence rule (the paper runs EP "until
    convergence" without a formula; this is the reading both implementations
    apply):
        max|mu_t - mu'_t| <= tol * (max y - min y),
        max|v_t / v'_t - 1| <= 10 tol,
        |lambda_t / lambda_{t-1} - 1| <= tol (EM only),
    where (mu'_t, v'_t) is the marginal right after sweep t's likelihood-site
    update, or the previous sweep's final marginal when sweep t did not update
    that site (identity operator, first cold sweep): the change of the
    colour-class updates of the sweep.  (The likelihood site's own change is
    left out: it carries the linear solve's error from sweep to sweep, which
    an FP32 solver's tolerance cannot push below this threshold at large
    sizes; a drifting likelihood site still moves the colour-class sites in
    the next sweep.)  Stops as well, with info["diverged"], once the
    divergence rule holds (DIVERGE_FACTOR).  Returns (mu, v, state, info)."""
    st = init_cold(pb) if state is None else state
    yr = np.asarray(pb.hty if pb.op.kind in (ops.DFT, ops.HADAMARD, ops.GAUSS) else pb.y,
                    dtype=np.float64)
    yrange = float(yr.max() - yr.min()) or 1.0
    yscale = max(float(yr.max() - yr.min()), float(np.abs(yr).max()))
    mu_prev, v_prev = marginals(st)
    done = 0
    converged = False
    diverged = False
    for t in range(1, sweeps + 1):
        lam_prev = st.lam
        a_bar = sweep(pb, st, t, em)
        done = t
        if st.lik_mu_absmax > DIVERGE_FACTOR * yscale:
            diverged = True
            break
        mu, v = marginals(st)
        mu_ref, v_ref = st.mid if st.mid is not None else (mu_prev, v_prev)
        dmu = float(np.max(np.abs(mu - mu_ref))) / yrange
        dv = float(np.max(np.abs(v / v_ref - 1.0)))
        dl = abs(st.lam / lam_prev - 1.0) if em else 0.0   # lambda moves under EM only
        if record:
            st.history.append({"t": t, "lam": st.lam, "a_bar": a_bar, "dmu": dmu, "dv": dv,
                               "cg": st.cg_iters})
        mu_prev, v_prev = mu, v
        if tol is not None and dmu <= tol and dv <= 10 * tol and (not em or dl <= tol):
            converged = True
            break
    mu, v = marginals(st)
    info = {"sweeps": done, "lam": st.lam, "converged": converged, "clamp_count": st.clamp_count,
            "diverged": diverged}
    return mu.reshape(pb.h, pb.w), v.reshape(pb.h, pb.w), st, info
