"""Benchmark: EP factor-updates/s on one MI355X, plus seconds to convergence.

A step is one EP-EM sweep of the whole hot path over one image: the
likelihood-site update (CG solve with H^T H applications, spectral variance,
damped site update) for non-identity operators, the fused sweep over the four
colour classes (cavity, tilted moments, site update, damping, clamp), and the
EM update of lambda.  value = factor updates (edges per sweep x sweeps) per
second of wall time over the K timed sweeps, inputs already resident on the GPU.

Workloads (synthetic, seeded; generators in synthetic.py):
  deconv2048  2048^2 deconvolution, 9x9 Gaussian blur sigma_b = 2 (periodic),
              sigma = 0.01, EM from lambda = 1, damping 0.5     [default]
              (--launch graph [default]: each sweep replayed as a hipGraph;
              --launch stream: every kernel launched on the stream)
  denoise128  128^2 denoising, sigma = 0.1, lambda = 10 fixed, damping 0.5
  denoise4096 4096^2 denoising, sigma = 0.1, EM (an HBM-resident probe of the sweep)
  hcs2048     2048^2 Hadamard compressive sensing: 30 % of the Paley-ordered Walsh
              coefficients, sigma = 0.01, EM from lambda = 1 (hcs128: the paper's
              128^2 size)
  batch256    256 instances, square sizes log-uniform in [64, 1024], 50/50 denoising /
              deconvolution, per-instance EM; graph launches, autotuned tile height,
              Jacobi CG (about 40M pixels in one context)

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
SWEEP_BYTES_PER_PX = 72        # 5 sites (tau, eta) read + 4 written, float32
HTH_BYTES_PER_PX = 20          # z, p_in, tau_c read; p_out, q written (float32)
WHT_BYTES_PER_PX = 24          # the same, plus the mask (float32)
PMC_FILE = os.path.join(ROOT, "profiles", "pmc_traffic.json")


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` on `workload` from the committed rocprofv3
    counter summary, or None when there is none for this workload or a source
    file the kernel is built from changed since the counters were taken."""
    import hashlib
    try:
        with open(PMC_FILE) as f:
            rec = json.load(f).get(kernel)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("workload") != workload:
        return None
    h = hashlib.sha256()
    for src in rec["sources"]:
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != rec["sources_sha256"]:
        return None
    return rec["traffic_bytes_per_launch"]


def roofline_entry(kernel, bytes_per_launch, avg_s, workload):
    achieved = bytes_per_launch / avg_s / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(kernel, workload),
            "kernel": kernel, "bytes_per_launch": bytes_per_launch,
            "avg_launch_us": round(avg_s * 1e6, 2)}


def copy_probe(nbytes=1 << 30, reps=5):
    """A plain device-to-device copy of known size (for scaling the HBM byte
    counters of rocprofv3)."""
    import torch
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": nbytes, "copy_probe_bytes_written": nbytes,
                      "repetitions": reps}), flush=True)


def make_workload(name):
    import synthetic as syn
    if name == "batch256":
        return syn.config3_instances(), True
    if name == "deconv2048":
        return syn.config4_test(seed=0, size=2048), True
    if name == "denoise128":
        return syn.config0(), False
    if name == "denoise4096":
        rng = syn.rng_for(5, 0)
        return syn.make_denoise(4096, 4096, 960, 0.1, rng, mode="paint", lam0=1.0, sweeps=50,
                                em=True, name="denoise4096"), True
    if name in ("hcs2048", "hcs128"):
        size = 2048 if name == "hcs2048" else 128
        n = max(3, round(150 * size * size / 1024 ** 2))
        return syn.make_hadamard_cs(size, size, n, 0.01, 0.3, syn.rng_for(6, size), lam0=1.0,
                                    sweeps=300, em=True, name=name), True
    raise SystemExit(f"unknown workload {name}")


def edges(h, w):
    return h * (w - 1) + (h - 1) * w


def cpu_sample(name, size):
    """A smaller instance of the same workload family for the oracle timing."""
    import synthetic as syn
    if name == "deconv2048":
        return syn.config1(size=size, sweeps=1), True
    if name == "denoise4096":
        return syn.make_denoise(size, size, max(3, round(960 * size * size / 4096 ** 2)), 0.1,
                                syn.rng_for(5, 1), mode="paint", lam0=1.0, sweeps=1, em=True), True
    if name.startswith("hcs"):
        return syn.make_hadamard_cs(size, size, max(3, round(150 * size * size / 1024 ** 2)), 0.01,
                                    0.3, syn.rng_for(6, 1), lam0=1.0, sweeps=1, em=True), True
    return syn.config0(), False


def cpu_baseline(name, size, sweeps):
    """The FP64 oracle, as it stands, on a bounded sample of the workload: the
    first `sweeps` sweeps (cold start, so including the first, most expensive
    likelihood-site solve) of a size x size instance of the same generator,
    operator and noise, single-threaded."""
    from threadpoolctl import threadpool_limits
    from oracle import ep as oep
    p, em = cpu_sample(name, size)
    with threadpool_limits(limits=1):
        pb = oep.problem_from_synthetic(p)
        t0 = time.perf_counter()
        oep.solve(pb, sweeps, em)
        dt = time.perf_counter() - t0
    h, w = p.shape
    return {"value": edges(h, w) * sweeps / dt, "unit": "factor-updates/s", "cores": 1,
            "kind": "oracle", "sample": f"first {sweeps} sweeps (cold start) of a {h}x{w} instance "
                                        f"of the same workload family, {dt:.1f} s, numpy FP64, "
                                        f"one thread"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="deconv2048")
    ap.add_argument("--tol", type=float, default=5e-6)
    ap.add_argument("--max-sweeps", type=int, default=2000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-warm", action="store_true")
    ap.add_argument("--cg-reduce", type=float, default=1e-2,
                    help="also time the solves with this opt-in CG residual reduction (0: skip)")
    ap.add_argument("--launch", choices=("graph", "stream"), default="graph",
                    help="single-image workloads: replay each sweep's launches as a hipGraph, "
                         "or launch them one by one on the stream")
    ap.add_argument("--cpu-sweeps", type=int, default=4)
    ap.add_argument("--cpu-size", type=int, default=256)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device copy (counter scaling for rocprofv3)")
    args = ap.parse_args()
    if args.copy_probe:
        return copy_probe()
    if args.gpus != 1:
        print("bench.py measures one GPU only: there is no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2110_01585_amd import Context, spec_from_synthetic
    from paper_2110_01585_amd import _native

    p, em = make_workload(args.workload)
    if isinstance(p, list):
        return bench_batch(args, p, em)
    h, w = p.shape
    print(f"[bench] workload {args.workload} {h}x{w} op={p.op} em={em}", file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    ctx = Context([spec_from_synthetic(p)], device=dev)
    y = torch.tensor(p.y, dtype=torch.float32, device=dev).contiguous()
    ctx.ep_tv_set_observation([y])
    ctx.ep_tv_set_option(_native.OPT_GRAPH, 1 if args.launch == "graph" else 0)
    ctx.ep_tv_run(args.warmup, em)
    # tile height of the sweep chosen by the autotuner (times the sweep kernel
    # only and leaves the EP state unchanged)
    tune = ctx.ep_tv_autotune(5)
    print(f"[bench] autotune: {tune}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()

    # timed region: K sweeps from a cold start
    ctx.ep_tv_init_cold()
    ctx.ep_tv_set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.ep_tv_run(args.steps, em)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tm = ctx.ep_tv_get_timing()
    ctx.ep_tv_set_timing(False)
    st = ctx.ep_tv_get_stats()[0]
    dt = t1 - t0
    if args.launch == "graph":
        # kernel events are not recorded inside replayed graphs: the per-kernel
        # durations come from the same sweeps launched on the stream
        ctx.ep_tv_set_option(_native.OPT_GRAPH, 0)
        ctx.ep_tv_init_cold()
        ctx.ep_tv_set_timing(True)
        ctx.ep_tv_run(args.steps, em)
        tm = ctx.ep_tv_get_timing()
        ctx.ep_tv_set_timing(False)
        ctx.ep_tv_set_option(_native.OPT_GRAPH, 1)
        torch.cuda.synchronize()
    E = edges(h, w)
    value = E * args.steps / dt
    print(f"[bench] {args.steps} sweeps in {dt*1e3:.1f} ms; sweep kernel {tm['sweep_ms']:.2f} ms / "
          f"{tm['sweep_launches']}, likelihood {tm['lik_ms']:.2f} ms / {tm['lik_updates']}",
          file=sys.stderr, flush=True)

    # rooflines (algorithmic bytes per launch / average launch time from HIP
    # events on the context's stream): the TV sweep (every site read once, the
    # TV sites written once) and, for deconvolution, the H^T H kernel of the CG;
    # `roofline` is the one with the larger total time
    sweep_avg_s = tm["sweep_ms"] / max(tm["sweep_launches"], 1) / 1e3
    roof_sweep = roofline_entry("k_tv_sweep", SWEEP_BYTES_PER_PX * h * w, sweep_avg_s, args.workload)
    roofline = roof_sweep
    roof_apply = None
    if p.op == "blur" and tm["apply_launches"] > 0:
        apply_avg_s = tm["apply_ms"] / tm["apply_launches"] / 1e3
        roof_apply = roofline_entry("k_hth_sep", HTH_BYTES_PER_PX * h * w, apply_avg_s, args.workload)
        if tm["apply_ms"] > tm["sweep_ms"]:
            roofline = roof_apply
    if p.op == "hadamard" and tm["apply_launches"] > 0:
        # the whole product (transform passes, mask, post-op and p.q partials)
        # against its algorithmic bytes
        apply_avg_s = tm["apply_ms"] / tm["apply_launches"] / 1e3
        roof_apply = roofline_entry("wht_product", WHT_BYTES_PER_PX * h * w, apply_avg_s, args.workload)
        if tm["apply_ms"] > tm["sweep_ms"]:
            roofline = roof_apply

    # seconds to converged from a cold start (y resident on the GPU)
    conv = None
    if args.max_sweeps > 0:
        conv = converge(ctx, args, em, p, y, dev, torch)
    ctx.close()

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] timing the oracle on the host", file=sys.stderr, flush=True)
        cpu = cpu_baseline(args.workload, args.cpu_size, args.cpu_sweeps)
    return emit(args, p, em, h, w, value, dt, roofline, cpu, conv, tm, roof_sweep, tune, roof_apply)


def bench_batch(args, ps, em):
    """Many instances in one context: graph launches, autotuned tiles."""
    import torch
    from paper_2110_01585_amd import Context, spec_from_synthetic
    from paper_2110_01585_amd import _native as N
    dev = torch.device("cuda:0")
    E = sum(edges(*p.shape) for p in ps)
    npx = sum(p.shape[0] * p.shape[1] for p in ps)
    print(f"[bench] workload {args.workload}: {len(ps)} instances, {npx / 1e6:.2f} M pixels, "
          f"{E / 1e6:.2f} M edges per sweep", file=sys.stderr, flush=True)
    ctx = Context([spec_from_synthetic(p, cg_precond=N.PRECOND_JACOBI) for p in ps], device=dev)
    ctx.ep_tv_set_observation([torch.tensor(p.y, dtype=torch.float32, device=dev) for p in ps])
    tune = ctx.ep_tv_autotune(5)
    print(f"[bench] autotune: {tune}", file=sys.stderr, flush=True)
    # direct-launch pass with kernel timing for the sweep roofline
    ctx.ep_tv_set_timing(True)
    ctx.ep_tv_run(max(args.warmup, 3), em)
    tm = ctx.ep_tv_get_timing()
    ctx.ep_tv_set_timing(False)
    ctx.ep_tv_set_option(N.OPT_GRAPH, 1)
    ctx.ep_tv_run(2, em)                       # captures the graphs
    ctx.ep_tv_init_cold()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.ep_tv_run(args.steps, em)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    value = E * args.steps / dt
    print(f"[bench] {args.steps} sweeps in {dt * 1e3:.1f} ms", file=sys.stderr, flush=True)
    sweep_avg_s = tm["sweep_ms"] / max(tm["sweep_launches"], 1) / 1e3
    roofline = roofline_entry("k_tv_sweep", SWEEP_BYTES_PER_PX * npx, sweep_avg_s, args.workload)
    conv = None
    if args.max_sweeps > 0:
        ctx.ep_tv_init_cold()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        rc, st = ctx.ep_tv_solve(min(args.max_sweeps, 200), args.tol, em, None, None)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        sw = [s["sweeps"] for s in st]
        upd = sum(edges(*p.shape) * s for p, s in zip(ps, sw))
        conv = {"s_to_all_converged_cold": round(t3 - t2, 4), "tol": args.tol,
                "converged": int(sum(s["converged"] for s in st)), "instances": len(ps),
                "sweeps_max": max(sw), "sweeps_mean": round(sum(sw) / len(sw), 1),
                "factor_updates_per_s_to_converged": upd / (t3 - t2)}
        print(f"[bench] solve: {conv}", file=sys.stderr, flush=True)
    ctx.close()
    line = {
        "metric": "EP factor-updates/s, batched denoising+deconvolution, 1 GPU",
        "value": value, "unit": "factor-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3 / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.workload, "instances": len(ps), "pixels": npx,
                   "edges_per_sweep": E, "launch": "hipGraph", "tile_rows": tune["tile_rows"],
                   "cg_precond": "jacobi"},
        "roofline": roofline, "cpu_baseline": None, "convergence": conv, "autotune": tune,
        "timing_ms": {"sweep": tm["sweep_ms"], "likelihood": tm["lik_ms"]},
    }
    print(json.dumps(line), flush=True)


def converge(ctx, args, em, p, y, dev, torch):
    """Seconds to converged (y resident on the GPU -> converged marginals on the
    GPU), cold start versus the learned warm start (network inference, warm site
    initialisation, then EP-EM to the same convergence rule).  Both results are
    checked against a cold run at a 100x tighter tolerance."""
    h, w = p.shape
    ctx.ep_tv_init_cold()
    torch.cuda.synchronize()
    mu = torch.empty(h, w, device=dev)
    var = torch.empty(h, w, device=dev)
    t2 = time.perf_counter()
    rc, stats = ctx.ep_tv_solve(args.max_sweeps, args.tol, em, [mu], [var])
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    conv = {"s_to_converged_cold": round(t3 - t2, 4), "sweeps_cold": stats[0]["sweeps"],
            "converged_cold": stats[0]["converged"], "tol": args.tol,
            "lambda_cold": stats[0]["lambda"]}
    print(f"[bench] cold solve: {conv}", file=sys.stderr, flush=True)
    if args.no_warm or p.op != "blur":
        return conv
    from paper_2110_01585_amd import Net, load_weights
    try:
        params, meta = load_weights()
    except FileNotFoundError:
        print("[bench] no trained warm-start weights in the package", file=sys.stderr, flush=True)
        return conv
    net = Net(params, max_batch=1, max_h=h, max_w=w, device=dev)
    mu_w = torch.empty(h, w, device=dev)
    var_w = torch.empty(h, w, device=dev)
    mu_hat = torch.empty(h, w, device=dev)
    var_hat = torch.empty(h, w, device=dev)
    net.infer(y, p.xi, mu_hat, var_hat)          # warm-up (code objects, caches)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t4 = time.perf_counter()
    e0.record()
    net.infer(y, p.xi, mu_hat, var_hat)
    e1.record()
    wrc = ctx.ep_tv_init_warm([mu_hat], [var_hat], meta["lambda_scale"], meta.get("lambda_power", 1.0))
    rc, st_w = ctx.ep_tv_solve(args.max_sweeps, args.tol, em, [mu_w], [var_w])
    torch.cuda.synchronize()
    t5 = time.perf_counter()
    ctx.ep_tv_init_warm([mu_hat], [var_hat], meta["lambda_scale"], meta.get("lambda_power", 1.0))  # untimed
    conv["lambda0_warm"] = ctx.ep_tv_get_stats()[0]["lambda"]
    conv.update({"s_to_converged_warm": round(t5 - t4, 4), "sweeps_warm": st_w[0]["sweeps"],
                 "converged_warm": st_w[0]["converged"], "lambda_warm": st_w[0]["lambda"],
                 "warm_status": wrc, "net_infer_ms": round(e0.elapsed_time(e1), 3),
                 "speedup_warm_vs_cold": round((t3 - t2) / (t5 - t4), 3),
                 "lambda_scale": meta["lambda_scale"]})
    net.close()
    # reference: cold start at a 100x tighter tolerance
    ctx.ep_tv_init_cold()
    mu_r = torch.empty(h, w, device=dev)
    var_r = torch.empty(h, w, device=dev)
    rc, st_r = ctx.ep_tv_solve(min(4 * args.max_sweeps, 1500), args.tol / 100, em, [mu_r], [var_r])
    torch.cuda.synchronize()
    rng = float(mu_r.max() - mu_r.min())
    for tag, m_, v_ in (("cold", mu, var), ("warm", mu_w, var_w)):
        conv[f"mean_err_{tag}_vs_tight"] = float((m_ - mu_r).abs().max()) / rng
        conv[f"var_err_{tag}_vs_tight"] = float((v_ / var_r - 1).abs().max())
    conv["tight_sweeps"] = st_r[0]["sweeps"]
    conv["tight_converged"] = st_r[0]["converged"]
    print(f"[bench] warm solve: {conv}", file=sys.stderr, flush=True)
    if args.cg_reduce > 0.0:
        conv["inexact"] = inexact_solves(args, em, p, y, dev, torch,
                                         net_in=(mu_hat, var_hat, meta, conv["net_infer_ms"]),
                                         ref=(mu_r, var_r, rng))
    return conv


def inexact_solves(args, em, p, y, dev, torch, net_in, ref):
    """The same cold and warm solves with the opt-in inexact likelihood solves
    (each CG also stops once its residual has fallen by cg_reduce), checked
    against the same tight reference.  Not part of the headline numbers."""
    from paper_2110_01585_amd import Context, spec_from_synthetic
    from paper_2110_01585_amd import _native as N
    h, w = p.shape
    mu_hat, var_hat, meta, infer_ms = net_in
    mu_r, var_r, rng = ref
    ctx = Context([spec_from_synthetic(p, cg_reduce=args.cg_reduce)], device=dev)
    ctx.ep_tv_set_observation([y])
    ctx.ep_tv_set_option(N.OPT_GRAPH, 1 if args.launch == "graph" else 0)
    ctx.ep_tv_run(3, em)                        # captures the graphs
    out = {"cg_reduce": args.cg_reduce}
    mu = torch.empty(h, w, device=dev)
    var = torch.empty(h, w, device=dev)
    for tag in ("cold", "warm"):
        if tag == "cold":
            ctx.ep_tv_init_cold()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        else:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.ep_tv_init_warm([mu_hat], [var_hat], meta["lambda_scale"], meta.get("lambda_power", 1.0))
        rc, st = ctx.ep_tv_solve(args.max_sweeps, args.tol, em, [mu], [var])
        torch.cuda.synchronize()
        # the warm time includes the network inference, as the default one does
        extra = infer_ms / 1e3 if tag == "warm" else 0.0
        out[f"s_to_converged_{tag}"] = round(time.perf_counter() - t0 + extra, 4)
        out[f"sweeps_{tag}"] = st[0]["sweeps"]
        out[f"cg_iters_{tag}"] = st[0]["cg_total"]
        out[f"converged_{tag}"] = st[0]["converged"]
        out[f"mean_err_{tag}_vs_tight"] = float((mu - mu_r).abs().max()) / rng
        out[f"var_err_{tag}_vs_tight"] = float((var / var_r - 1).abs().max())
    ctx.close()
    print(f"[bench] inexact solves: {out}", file=sys.stderr, flush=True)
    return out


def emit(args, p, em, h, w, value, dt, roofline, cpu, conv, tm, roof_sweep, tune, roof_apply=None):
    E = edges(h, w)
    line = {
        "metric": "EP factor-updates/s + s to converged 2048^2 deconv, warm-start vs plain, 1 GPU",
        "value": value, "unit": "factor-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3 / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.workload, "height": h, "width": w, "op": p.op, "em": em,
                   "edges_per_sweep": E, "damping": p.damping, "xi": p.xi,
                   "tile_rows": tune["tile_rows"], "launch": args.launch},
        "kernel_timing": ("HIP events on the context's stream over the timed sweeps"
                          if args.launch == "stream" else
                          "HIP events on the context's stream over the same sweeps launched on "
                          "the stream right after the timed graph replays (events are not "
                          "recorded inside a replayed graph)"),
        "roofline": roofline, "roofline_sweep": roof_sweep, "roofline_apply": roof_apply,
        "cpu_baseline": cpu, "convergence": conv,
        "timing_ms": {"sweep": tm["sweep_ms"], "likelihood": tm["lik_ms"],
                      "cg_products": tm["apply_ms"], "cg_products_launches": tm["apply_launches"],
                      "cg_preconditioner": tm["precond_ms"],
                      "cg_preconditioner_launches": tm["precond_launches"]},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
