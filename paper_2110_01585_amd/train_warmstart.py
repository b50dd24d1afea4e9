"""Train the warm-start network on EP solutions that the EP solver itself produces.

    python -m paper_2110_01585_amd.train_warmstart [--n-train 10000] [--epochs 8]
        [--out paper_2110_01585_amd/weights/warmstart_deconv_sb2_s001]

1. Training set: seeded 256 x 256 deconvolution instances (9 x 9 Gaussian blur,
   sigma_b = 2, periodic; noise sigma = 0.01; piecewise-constant images drawn
   as windows of 256^2 .. 2048^2-scale images, synthetic.config4_train_mixed), each
   solved to convergence by the batched GPU EP-EM solver (graph launches, Jacobi
   CG) from a cold start.  Targets: the converged marginal means and variances.
2. Training: the network's own GPU kernels (bfloat16 MFMA forward / backward,
   Adam), batches of 16 images, cosine learning-rate decay.
3. Calibration of lambda_0: option 1 (lambda_1 = N / a_x under the prediction)
   is biased low because it treats the pixels as independent, by a factor that
   drifts with the image scale; lambda_0 = kappa * lambda_1^rho is fitted to the
   converged lambda* of training instances (least squares in log space) and
   stored as `lambda_scale` = kappa, `lambda_power` = rho.
4. Held-out check: sweeps to convergence, warm versus cold.

Everything runs on the GPU except the image generation (NumPy, a process pool).
Progress lines go to stderr; the weights are written as <out>.f32 + <out>.json.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synthetic as syn  # noqa: E402


def log(msg):
    print(f"[train {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def _gen(i, size):
    p = syn.config4_train_mixed(i, size=size)
    return p.y.astype(np.float32), p.taps, p.xi, p.boundary, p.meta.get("scale", size)


def generate(ids, size, workers):
    with ProcessPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(_gen, ids, [size] * len(ids), chunksize=16))


def solve_batch(torch, probs, y_dev, mu_out, v_out, max_sweeps, tol, warm=None, lam_scale=1.0,
                lam_power=1.0):
    """Solve a batch of instances (list of synthetic.Problem-like specs) on the GPU."""
    from paper_2110_01585_amd import Context, spec_from_synthetic
    from paper_2110_01585_amd import _native as N
    ctx = Context([spec_from_synthetic(p, cg_precond=N.PRECOND_JACOBI) for p in probs])
    ctx.ep_tv_set_option(N.OPT_GRAPH, 1)
    ctx.ep_tv_set_observation(list(y_dev))
    if warm is not None:
        ctx.ep_tv_init_warm(warm[0], warm[1], lam_scale, lam_power)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, st = ctx.ep_tv_solve(max_sweeps, tol, True, list(mu_out), list(v_out))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.close()
    return st, dt


class _Spec:
    """The fields spec_from_synthetic reads, for a generated instance."""

    def __init__(self, y, taps, xi, size, boundary, scale):
        self.shape = (size, size)
        self.op = "blur"
        self.boundary = boundary
        self.scale = scale
        self.xi = xi
        self.lam0 = 1.0
        self.damping = 0.5
        self.taps = taps
        self.mask = None
        self.y = y


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n-train", type=int, default=10000)
    ap.add_argument("--n-val", type=int, default=64)
    ap.add_argument("--size", type=int, default=256)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--gen-batch", type=int, default=256)
    ap.add_argument("--max-sweeps", type=int, default=400)
    ap.add_argument("--tol", type=float, default=1e-5)
    ap.add_argument("--workers", type=int, default=8)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=os.path.join(ROOT, "paper_2110_01585_amd", "weights",
                                                  "warmstart_deconv_sb2_s001"))
    args = ap.parse_args(argv)

    S = args.size
    n_all = args.n_train + args.n_val
    t_start = time.perf_counter()
    # ---- 1. data: generate every image on the host first (worker processes are
    # forked before this process touches the GPU), then solve with the batched
    # EP solver
    gen = generate(list(range(n_all)), S, args.workers)
    specs = [_Spec(y, taps, xi, S, bnd, sc) for (y, taps, xi, bnd, sc) in gen]
    log(f"generated {n_all} images of {S}x{S} in {time.perf_counter() - t_start:.1f} s")

    import torch
    from paper_2110_01585_amd import Context, Net, spec_from_synthetic
    from paper_2110_01585_amd.net import init_params, save_weights
    from paper_2110_01585_amd import _native as N

    dev = torch.device("cuda:0")
    Y = torch.empty(n_all, S, S, device=dev)
    MU = torch.empty(n_all, S, S, device=dev)
    V = torch.empty(n_all, S, S, device=dev)
    for k, sp in enumerate(specs):
        Y[k].copy_(torch.from_numpy(sp.y))
    lam_star = np.zeros(n_all)
    sweeps = np.zeros(n_all, dtype=int)
    conv = np.zeros(n_all, dtype=bool)
    gb = args.gen_batch
    for b0 in range(0, n_all, gb):
        ids = list(range(b0, min(n_all, b0 + gb)))
        st, dt = solve_batch(torch, specs[b0:b0 + len(ids)], [Y[k] for k in ids], [MU[k] for k in ids],
                             [V[k] for k in ids], args.max_sweeps, args.tol)
        for k, s in zip(ids, st):
            lam_star[k], sweeps[k], conv[k] = s["lambda"], s["sweeps"], s["converged"]
        log(f"EP solutions {ids[-1] + 1}/{n_all}: batch of {len(ids)} in {dt:.2f} s, "
            f"converged {int(conv[ids].sum())}/{len(ids)}, mean sweeps {sweeps[ids].mean():.1f}")
    xi = specs[0].xi
    log(f"data ready in {time.perf_counter() - t_start:.1f} s; lambda* median {np.median(lam_star):.4g}")

    # ---- 2. training
    ntr = args.n_train
    net = Net(init_params(args.seed), max_batch=args.batch, max_h=S, max_w=S, device=dev)
    rng = np.random.default_rng(args.seed)
    steps_per_epoch = ntr // args.batch
    total = steps_per_epoch * args.epochs
    step = 0
    t_tr = time.perf_counter()
    hist = []
    for ep in range(args.epochs):
        perm = torch.tensor(rng.permutation(ntr), device=dev)
        run = 0.0
        nrun = 0
        for s_i in range(steps_per_epoch):
            idx = perm[s_i * args.batch:(s_i + 1) * args.batch]
            yb, mb, vb = Y[idx].contiguous(), MU[idx].contiguous(), V[idx].contiguous()
            lr = 1e-5 + 0.5 * (args.lr - 1e-5) * (1 + math.cos(math.pi * step / total))
            want = (s_i % 50 == 0)
            loss = net.train_step(yb, mb, vb, xi, lr, want_loss=want)
            if want:
                run += loss
                nrun += 1
            step += 1
        hist.append(run / max(nrun, 1))
        log(f"epoch {ep + 1}/{args.epochs}: sampled mean loss {hist[-1]:.5f} "
            f"({time.perf_counter() - t_tr:.1f} s)")
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t_tr
    # validation loss
    val = list(range(ntr, n_all))
    vl = []
    for b0 in range(0, len(val), args.batch):
        idx = torch.tensor(val[b0:b0 + args.batch], device=dev)
        l, _ = net.loss_grad(Y[idx].contiguous(), MU[idx].contiguous(), V[idx].contiguous(), xi,
                             want_grad=False)
        vl.append(l)
    val_loss = float(np.mean(vl))
    log(f"training done in {train_s:.1f} s ({total} steps); validation loss {val_loss:.5f}")

    # ---- 3. lambda_0 calibration on training instances
    cal = list(range(min(512, ntr)))
    mu_h = torch.empty(len(cal), S, S, device=dev)
    v_h = torch.empty(len(cal), S, S, device=dev)
    for b0 in range(0, len(cal), args.batch):
        sl = slice(b0, min(len(cal), b0 + args.batch))
        net.infer(Y[cal[sl.start]:cal[sl.stop - 1] + 1].contiguous(), xi, mu_h[sl], v_h[sl])
    ctx = Context([spec_from_synthetic(specs[k], cg_precond=N.PRECOND_JACOBI) for k in cal])
    ctx.ep_tv_set_observation([Y[k] for k in cal])
    ctx.ep_tv_init_warm([mu_h[i] for i in range(len(cal))], [v_h[i] for i in range(len(cal))], 1.0, 1.0)
    lam1 = np.array([s["lambda"] for s in ctx.ep_tv_get_stats()])
    ctx.close()
    ratio = lam_star[cal] / lam1
    # lambda_0 = kappa * lambda_1^rho, least squares in log space
    A = np.stack([np.ones(len(cal)), np.log(lam1)], axis=1)
    coef, *_ = np.linalg.lstsq(A, np.log(lam_star[cal]), rcond=None)
    lam_scale, lam_power = float(np.exp(coef[0])), float(coef[1])
    resid = np.log(lam_star[cal]) - A @ coef
    log(f"lambda calibration: ratio lambda*/lambda1 median {np.median(ratio):.4f} "
        f"(IQR {np.percentile(ratio, 25):.4f}..{np.percentile(ratio, 75):.4f}); fit "
        f"lambda0 = {lam_scale:.4f} lambda1^{lam_power:.4f}, log residual std {resid.std():.4f}")
    scales = np.array([specs[k].scale for k in cal])
    by_scale = {}
    for sc in sorted(set(scales.tolist())):
        m = scales == sc
        by_scale[int(sc)] = {"ratio_median": float(np.median(ratio[m])),
                             "lambda_star_median": float(np.median(lam_star[cal][m]))}
    log(f"  by image scale: {by_scale}")

    # ---- 4. held-out: warm versus cold sweeps
    vk = val
    mu_v = torch.empty(len(vk), S, S, device=dev)
    v_v = torch.empty(len(vk), S, S, device=dev)
    for b0 in range(0, len(vk), args.batch):
        sl = slice(b0, min(len(vk), b0 + args.batch))
        net.infer(Y[vk[sl.start]:vk[sl.stop - 1] + 1].contiguous(), xi, mu_v[sl], v_v[sl])
    out_mu = torch.empty(len(vk), S, S, device=dev)
    out_v = torch.empty(len(vk), S, S, device=dev)
    st_c, dt_c = solve_batch(torch, [specs[k] for k in vk], [Y[k] for k in vk], list(out_mu), list(out_v),
                             args.max_sweeps, args.tol)
    st_w, dt_w = solve_batch(torch, [specs[k] for k in vk], [Y[k] for k in vk], list(out_mu), list(out_v),
                             args.max_sweeps, args.tol,
                             warm=([mu_v[i] for i in range(len(vk))], [v_v[i] for i in range(len(vk))]),
                             lam_scale=lam_scale, lam_power=lam_power)
    sc = np.array([s["sweeps"] for s in st_c])
    sw = np.array([s["sweeps"] for s in st_w])
    log(f"held-out {len(vk)}: cold mean sweeps {sc.mean():.1f} ({dt_c:.2f} s), "
        f"warm {sw.mean():.1f} ({dt_w:.2f} s)")

    params = net.params.cpu().numpy()
    meta = {"architecture": "3x3 conv x6, channels 1-32-32-32-32-32-2, ReLU, zero padding",
            "train_instances": ntr, "size": S, "generator": "synthetic.config4_train_mixed",
            "operator": "blur sigma_b=2 9x9 periodic, free TV boundary", "noise_sigma": 0.01,
            "epochs": args.epochs, "batch": args.batch, "lr": args.lr, "steps": total,
            "train_seconds": round(train_s, 1), "epoch_loss": [round(h, 6) for h in hist],
            "val_loss": val_loss, "lambda_scale": lam_scale, "lambda_power": lam_power,
            "lambda_fit_log_residual_std": float(resid.std()),
            "lambda_ratio_iqr": [float(np.percentile(ratio, 25)), float(np.percentile(ratio, 75))],
            "lambda_by_scale": by_scale,
            "ep_targets": {"tol": args.tol, "max_sweeps": args.max_sweeps,
                           "converged_fraction": float(conv.mean()), "mean_sweeps": float(sweeps.mean())},
            "heldout": {"n": len(vk), "cold_mean_sweeps": float(sc.mean()),
                        "warm_mean_sweeps": float(sw.mean()), "cold_s": dt_c, "warm_s": dt_w}}
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    save_weights(args.out, params, meta)
    log(f"wrote {args.out}.f32 / .json; total {time.perf_counter() - t_start:.1f} s")
    print(json.dumps(meta))
    net.close()


if __name__ == "__main__":
    main()
