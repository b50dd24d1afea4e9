"""Benchmark: EP factor-updates/s and seconds to converged on one MI355X.

One EP sweep is the whole hot path over one image: the likelihood-site update
(CG solve with H^T H applications, spectral variance, damped site update) for
non-identity operators, the fused sweep over the four colour classes (cavity,
tilted moments, site update, damping, clamp), the EM update of lambda and the
convergence rule.

Steps (the definition is printed in the JSON line as "step"):
  deconv2048 [default]  a step is one cold-start solve to convergence (tol 5e-6,
              at most --max-sweeps sweeps) of the 2048^2 deconvolution, y
              resident on the GPU: initialisation, every sweep, the gather of
              the marginals.  value = factor updates (edges x sweeps, summed
              over the K timed solves) / wall time of the K solves, so it does
              not depend on K; ms_per_step = seconds to converged (cold).
  batch256    a step is one sweep over all 256 instances from cold (graph replay).
  denoise*, hcs*  a step is one sweep; for hcs (whose solve does not converge in
              2000 sweeps) the K timed sweeps follow --cold-phase untimed sweeps
              from cold.

Workloads (synthetic, seeded; generators in synthetic.py):
  deconv2048  2048^2 deconvolution, 9x9 Gaussian blur sigma_b = 2 (periodic),
              sigma = 0.01, EM from lambda = 1, damping 0.5
  denoise128  128^2 denoising, sigma = 0.1, lambda = 10 fixed
  denoise4096 4096^2 denoising, sigma = 0.1, EM (the sweep on an HBM-resident state)
  hcs2048     2048^2 Hadamard compressive sensing: 30 % of the Paley-ordered Walsh
              coefficients, sigma = 0.01, EM from lambda = 1 (hcs128: 128^2)
  batch256    256 instances, square sizes log-uniform in [64, 1024], 50/50 denoising /
              deconvolution, per-instance EM; Jacobi CG (about 40M pixels)
  gcs128      128^2 compressive sensing with a Gaussian i.i.d. sensing matrix, M / N = 0.3,
              sigma = 0.01, EM (the paper's CS setting): Woodbury moments in FP64 on the
              matrix cores (roofline against the FP64 MFMA peak)
  rbmc512     512^2 deconvolution with the RBMC variance estimator (8 samples)
  net2048     the warm-start network: a step is one inference on the 2048^2
              deconvolution observation; also times training steps (forward,
              backward, Adam) on batches of 16 x 256^2 synthetic targets

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
       python bench.py --stream-probe   (the TV sweep's plane accesses with no arithmetic:
                                         the rate its access pattern reaches on the device)
       python bench.py --copy-probe     (a plain 1 GiB copy: rate, and the byte counters' scale)
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_MFMA_PEAK_TFLOPS = 78.6
# algorithmic bytes per pixel and launch (float32): what the kernel must read
# and write at least once
BYTES_PER_PX = {
    "k_tv_sweep": 72,     # 5 sites (tau, eta) read + 4 written
    "k_hth_sep": 20,      # z, p_in, tau_c read; p_out, q written
    "wht_product": 24,    # the same, plus the mask
    "rf_fwd": 28,         # x, p, r, q read, x, r written, half spectrum (8 B/px) written
    "rf_filt": 8,         # half spectrum read and written (4 + 4 B per real pixel)
    "rf_inv": 12,         # half spectrum read, z written
}
CG_ITER_BYTES_PER_PX = 20 + 28 + 8 + 12
KERNEL_SYMBOL = {"k_tv_sweep": "eptv::k_tv_sweep", "k_hth_sep": "eptv::k_hth_sep<8, 1>",
                 "rf_fwd": "eptv::k_rfft<L, 0> (RF_FWD)", "rf_filt": "eptv::k_rfft<L, 1> (RF_FILT)",
                 "rf_inv": "eptv::k_rfft<L, 2> (RF_INV)", "wht_product": "k_wht_low + k_wht_high passes"}
PMC_FILE = os.path.join(ROOT, "profiles", "pmc_traffic.json")
GOLDEN_DECONV512 = os.path.join(ROOT, "tests", "golden", "deconv512.json")


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` on `workload` from the committed rocprofv3
    counter summary, or None when there is none for this workload or a source
    file the kernel is built from changed since the counters were taken."""
    import hashlib
    try:
        with open(PMC_FILE) as f:
            rec = json.load(f).get(f"{kernel}@{workload}")
    except (OSError, ValueError):
        return None
    if not rec:
        return None
    h = hashlib.sha256()
    for src in rec["sources"]:
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != rec["sources_sha256"]:
        return None
    return rec["traffic_bytes_per_launch"]


def roofline_entry(kernel, npx, total_ms, launches, workload):
    bytes_per_launch = BYTES_PER_PX[kernel] * npx
    avg_s = total_ms / max(launches, 1) / 1e3
    achieved = bytes_per_launch / avg_s / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(kernel, workload),
            "kernel": kernel, "symbol": KERNEL_SYMBOL[kernel],
            "bytes_per_launch": bytes_per_launch, "bytes_per_px": BYTES_PER_PX[kernel],
            "avg_launch_us": round(avg_s * 1e6, 2), "launches": launches,
            "total_ms": round(total_ms, 3)}


def kernel_rooflines(tm, npx, workload, op):
    """Roofline entry of every timed kernel with an algorithmic byte count, and
    the one with the largest total time (the step's dominant kernel)."""
    cand = {"k_tv_sweep": (tm["sweep_ms"], tm["sweep_launches"])}
    if op == "blur":
        cand["k_hth_sep"] = (tm["apply_ms"], tm["apply_launches"])
    if op == "hadamard":
        cand["wht_product"] = (tm["apply_ms"], tm["apply_launches"])
    for k in ("rf_fwd", "rf_filt", "rf_inv"):
        if tm[f"{k}_launches"] > 0:
            cand[k] = (tm[f"{k}_ms"], tm[f"{k}_launches"])
    entries = {k: roofline_entry(k, npx, ms, n, workload) for k, (ms, n) in cand.items() if n > 0}
    if tm.get("dgemm_launches", 0) > 0:
        # the FP64 GEMMs of the Woodbury moments, against the FP64 matrix-core peak
        t_s = tm["dgemm_ms"] / 1e3
        ach = tm["dgemm_flops"] / t_s / 1e12
        entries["dgemm_f64"] = {"bound": "mfma", "achieved": round(ach, 2),
                                "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                                "frac": round(ach / FP64_MFMA_PEAK_TFLOPS, 4), "traffic": None,
                                "kernel": "dgemm_f64",
                                "symbol": "eptv::k_dgemm_nt (v_mfma_f64_16x16x4f64)",
                                "flops": tm["dgemm_flops"], "launches": tm["dgemm_launches"],
                                "avg_launch_us": round(tm["dgemm_ms"] * 1e3 / tm["dgemm_launches"], 2),
                                "total_ms": round(tm["dgemm_ms"], 3)}
    dominant = max(entries, key=lambda k: entries[k]["total_ms"])
    return entries[dominant], entries


def copy_probe(nbytes=1 << 30, reps=9):
    """A plain device-to-device copy of known size (for scaling the HBM byte
    counters of rocprofv3)."""
    import torch
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    ev[0].record()
    for i in range(reps):
        dst.copy_(src)
        ev[i + 1].record()
    torch.cuda.synchronize()
    # the copy's own rate: the practical ceiling of a pure streaming kernel
    # (one read, one write per element) next to the 8 TB/s peak
    ms = sorted(ev[i].elapsed_time(ev[i + 1]) for i in range(1, reps))
    med = ms[len(ms) // 2] if ms else float("nan")
    print(json.dumps({"copy_probe_bytes_read": nbytes, "copy_probe_bytes_written": nbytes,
                      "repetitions": reps, "median_ms": round(med, 4),
                      "gbps": round(2 * nbytes / (med * 1e-3) / 1e9, 1)}), flush=True)


def stream_probe(h=4096, w=4096, reps=15):
    """The sweep's access pattern (five float2 site planes read, four written,
    h x w pixels each, 1.2 GB at 4096^2) with no arithmetic, timed with HIP
    events on the probe's stream: the rate this pattern reaches on the device,
    i.e. the practical ceiling for the sweep's fraction of the 8 TB/s peak."""
    import ctypes

    import torch
    from paper_2110_01585_amd.build import PROBE_LIB
    if not os.path.exists(PROBE_LIB):
        raise RuntimeError(f"{PROBE_LIB} is not built; run __graft_entry__.build() first")
    lib = ctypes.CDLL(PROBE_LIB)
    lib.eptv_stream_probe.restype = ctypes.c_int
    lib.eptv_stream_probe.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p),
                                      ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_void_p]
    planes = [torch.zeros(h, w, 2, dtype=torch.float32, device="cuda") for _ in range(9)]
    ins = (ctypes.c_void_p * 5)(*[t.data_ptr() for t in planes[:5]])
    outs = (ctypes.c_void_p * 4)(*[t.data_ptr() for t in planes[5:]])
    stream = torch.cuda.current_stream()
    nbytes = 9 * h * w * 8
    res = {"pattern": "5 float2 planes read, 4 written (the TV sweep's), no arithmetic",
           "height": h, "width": w, "bytes_per_launch": nbytes}
    for name, mode, rows in (("flat", 0, 0), ("march12", 1, 12), ("march48", 1, 48)):
        def launch():
            rc = lib.eptv_stream_probe(ins, outs, h, w, mode, rows, ctypes.c_void_p(stream.cuda_stream))
            if rc != 0:
                raise RuntimeError(f"eptv_stream_probe failed ({rc})")
        for _ in range(3):
            launch()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * reps)]
        for i in range(reps):
            ev[2 * i].record(stream)
            launch()
            ev[2 * i + 1].record(stream)
        torch.cuda.synchronize()
        us = sorted(ev[2 * i].elapsed_time(ev[2 * i + 1]) * 1e3 for i in range(reps))[reps // 2]
        gbs = nbytes / (us * 1e-6) / 1e9
        res[name] = {"us": round(us, 2), "gbps": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}
    print(json.dumps(res), flush=True)


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
    if name == "gcs128":
        return syn.make_gauss_cs(128, 128, 12, 0.01, 0.3, syn.rng_for(7, 0), lam0=1.0, sweeps=100,
                                 em=True, name="gcs128"), True
    if name == "rbmc512":
        p = syn.config1(size=512, sweeps=200)
        p.name = "rbmc512"
        return p, True
    if name in ("hcs2048", "hcs128"):
        size = 2048 if name == "hcs2048" else 128
        n = max(3, round(150 * size * size / 1024 ** 2))
        return syn.make_hadamard_cs(size, size, n, 0.01, 0.3, syn.rng_for(6, size), lam0=1.0,
                                    sweeps=300, em=True, name=name), True
    raise SystemExit(f"unknown workload {name}")


def edges(h, w):
    return h * (w - 1) + (h - 1) * w


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


# --------------------------------------------------------------------------
# CPU baselines: the FP64 oracle as it stands, on bounded samples
# --------------------------------------------------------------------------

def cpu_baseline_fullsize(p, em, cg_iters_per_sweep, cg_probe_iters=4):
    """The oracle's cost of one sweep of this very workload at full size,
    extrapolated: one sweep of the four colour blocks (+ EM) timed at full
    size (a band of rows scaled by the edge count would understate it: numpy
    runs 4.5x slower per edge on the full 2048^2 arrays than on 512-row bands),
    the likelihood update's fixed part (cavity, right-hand side, spectral
    variance, site formulas) timed at full size, and its CG timed for a few
    iterations at full size and scaled to the GPU path's mean CG iterations
    per sweep.  One thread."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import ep as oep
    from oracle import operators as oops
    h, w = p.shape
    with threadpool_limits(limits=1):
        pb = oep.problem_from_synthetic(p)
        st = oep.init_cold(pb)
        t0 = time.perf_counter()
        a_bar = 0.0
        for k in pb.order:
            a_bar += oep.tv_block_update(pb, st, k)
        if em and a_bar > 0:
            st.lam = pb.N / a_bar
        t_tv = time.perf_counter() - t0
        lik = {"t_lik_fixed_s": 0.0, "t_cg_iter_s": 0.0}
        t_lik = 0.0
        if pb.op.kind != oops.IDENTITY:
            shape = (h, w)
            t1 = time.perf_counter()
            tau_c, eta_c = oep.cavity(st, 0)
            b = pb.hty / pb.xi + eta_c.reshape(shape)
            V = oops.tilted_variance(pb.op, pb.xi, tau_c.reshape(shape), pb.estimator).ravel()
            E = oep.marginals(st)[0]
            tau_new = np.maximum(1.0 / V - tau_c, oep.PREC_FLOOR)
            eta_new = (tau_new + tau_c) * E - eta_c
            t_fixed = time.perf_counter() - t1
            t2 = time.perf_counter()
            oops.solve_tilted_mean(pb.op, pb.xi, tau_c.reshape(shape), b, x0=E.reshape(shape),
                                   rtol=1e-30, maxiter=cg_probe_iters)
            t_cg = (time.perf_counter() - t2) / cg_probe_iters
            t_lik = t_fixed + cg_iters_per_sweep * t_cg
            lik = {"t_lik_fixed_s": round(t_fixed, 3), "t_cg_iter_s": round(t_cg, 3),
                   "cg_iters_per_sweep": round(cg_iters_per_sweep, 2)}
            del eta_new
    t_sweep = t_tv + t_lik
    return {"value": edges(h, w) / t_sweep, "unit": "factor-updates/s", "cores": 1, "kind": "oracle",
            "sample": (f"extrapolated per sweep at the workload's own size {h}x{w}: the oracle's four "
                       f"colour blocks + EM timed once ({t_tv:.2f} s), its likelihood update's fixed "
                       f"part timed once and its CG timed over {cg_probe_iters} iterations at full "
                       f"size, scaled to the GPU path's mean CG iterations per sweep; numpy FP64, one "
                       f"thread"),
            "seconds_per_sweep": round(t_sweep, 3), "t_tv_sweep_s": round(t_tv, 3), **lik,
            "cpu_model": cpu_model()}


def _oracle_worker(args):
    import numpy as np  # noqa: F401
    from threadpoolctl import threadpool_limits
    from oracle import ep as oep
    import synthetic as syn
    idx, sweeps = args
    p = syn.config3_instance(idx)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        oep.solve(oep.problem_from_synthetic(p), sweeps, True)
        dt = time.perf_counter() - t0
    return edges(*p.shape) * sweeps, dt


def cpu_baseline_pool(ps, stride=8, sweeps=2):
    """The oracle over a process pool on all host cores (capped at 16, the
    CPU share of one GPU): the first `sweeps` sweeps from cold of every
    `stride`-th instance of the batch, one thread per process."""
    import multiprocessing as mp
    n_proc = max(1, min(16, os.cpu_count() or 1))
    jobs = [(i, sweeps) for i in range(0, len(ps), stride)]
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(n_proc) as pool:
        res = pool.map(_oracle_worker, jobs, chunksize=1)
    wall = time.perf_counter() - t0
    upd = sum(r[0] for r in res)
    return {"value": upd / wall, "unit": "factor-updates/s", "cores": n_proc, "kind": "oracle",
            "sample": (f"first {sweeps} sweeps (cold start) of every {stride}th instance of the batch "
                       f"({len(jobs)} instances), numpy FP64, a pool of {n_proc} single-threaded "
                       f"processes; wall {wall:.1f} s including process start"),
            "cpu_count": os.cpu_count(), "cpu_model": cpu_model()}


# CPU samples of the secondary workloads (side, sweeps), each about 10-30 s of
# oracle work on one core and with at least two likelihood-site updates where
# there is a likelihood site (the first sweep from cold has none): 1024^2
# denoising (the oracle's per-sweep rate there is within 10 % of its rate at
# 4096^2, where two sweeps take two minutes), a 1024^2 Hadamard instance (the
# oracle's dense Walsh products grow as the cube of the side), an 80^2 Gaussian
# CS instance (the dense Woodbury solve grows as the cube of the pixel count),
# a 128^2 RBMC instance (8 CG solves per sweep)
CPU_SAMPLE = {"denoise4096": (1024, 3), "hcs2048": (1024, 3), "gcs128": (80, 3),
              "rbmc512": (128, 3)}


def cpu_baseline_sample(name, size, sweeps):
    """The oracle on the first sweeps of a smaller instance of the same family
    (secondary workloads)."""
    from threadpoolctl import threadpool_limits
    from oracle import ep as oep
    import synthetic as syn
    if name == "denoise4096":
        p, em = syn.make_denoise(size, size, max(3, round(960 * size * size / 4096 ** 2)), 0.1,
                                 syn.rng_for(5, 1), mode="paint", lam0=1.0, sweeps=1, em=True), True
    elif name.startswith("hcs"):
        p, em = syn.make_hadamard_cs(size, size, max(3, round(150 * size * size / 1024 ** 2)), 0.01,
                                     0.3, syn.rng_for(6, 1), lam0=1.0, sweeps=1, em=True), True
    elif name == "gcs128":
        p, em = syn.make_gauss_cs(size, size, max(3, round(12 * size * size / 128 ** 2)), 0.01, 0.3,
                                  syn.rng_for(7, 1), lam0=1.0), True
    elif name == "rbmc512":
        size = min(size, 128)
        p, em = syn.config1(size=size, sweeps=1), True
    else:
        p, em = syn.config0(), False
    rbmc = None
    if name == "rbmc512":
        import numpy as np
        rng = np.random.default_rng(1)
        rbmc = (rng.standard_normal((RBMC_SAMPLES,) + p.shape), rng.standard_normal((RBMC_SAMPLES,) + p.shape))
    with threadpool_limits(limits=1):
        pb = oep.problem_from_synthetic(p, estimator="rbmc" if rbmc else "spectral", rbmc_noise=rbmc)
        t0 = time.perf_counter()
        oep.solve(pb, sweeps, em)
        dt = time.perf_counter() - t0
    h, w = p.shape
    return {"value": edges(h, w) * sweeps / dt, "unit": "factor-updates/s", "cores": 1,
            "kind": "oracle", "sample": f"first {sweeps} sweeps (cold start) of a {h}x{w} instance "
                                        f"of the same workload family, {dt:.1f} s, numpy FP64, one "
                                        f"thread", "cpu_model": cpu_model()}


# --------------------------------------------------------------------------
# GPU
# --------------------------------------------------------------------------

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="deconv2048")
    ap.add_argument("--tol", type=float, default=5e-6)
    ap.add_argument("--max-sweeps", type=int, default=2000)
    ap.add_argument("--cold-phase", type=int, default=100,
                    help="hcs workloads: untimed sweeps from cold before the timed ones")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-warm", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the long reference run and the oracle comparison")
    ap.add_argument("--cg-reduce", type=float, default=0.0,
                    help="also time one cold and one warm solve with this opt-in CG residual "
                         "reduction (0: skip)")
    ap.add_argument("--persistent", type=int, choices=(0, 1), default=0,
                    help="launch the TV sweep as one resident grid looping over the tile blocks")
    ap.add_argument("--launch", choices=("graph", "stream"), default="graph",
                    help="replay each sweep's launches as a hipGraph, or launch them one by one")
    ap.add_argument("--cpu-sweeps", type=int, default=None,
                    help="secondary workloads: oracle sweeps of the CPU sample (default per workload)")
    ap.add_argument("--cpu-size", type=int, default=None,
                    help="secondary workloads: side of the CPU sample (default per workload)")
    ap.add_argument("--stream-probe", action="store_true",
                    help="only run the streaming probe: the TV sweep's plane accesses without "
                         "arithmetic (its practical HBM ceiling)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device copy (counter scaling for rocprofv3)")
    args = ap.parse_args()
    if args.copy_probe:
        return copy_probe()
    if args.stream_probe:
        return stream_probe()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path, so run it "
              "with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.workload == "net2048":
        return bench_net(args)
    p, em = make_workload(args.workload)
    if isinstance(p, list):
        return bench_batch(args, p, em)
    if args.workload == "deconv2048":
        return bench_solves(args, p, em)
    return bench_sweeps(args, p, em)


RBMC_SAMPLES = 8
BF16_MFMA_PEAK_TFLOPS = 2500.0
# the warm-start network: 3x3 convolutions 1 -> 32, four 32 -> 32, 32 -> 2
NET_FLOP_PER_PX = 2 * 9 * (1 * 32 + 4 * 32 * 32 + 32 * 2)
# bytes each step must move per pixel (input read, output written): the statistics
# pass over the observation, then per layer: the float
# observation in, BF16 activations of 32 channels (64 B) between layers, two
# float outputs
NET_BYTES_PER_PX = 4 + (4 + 64) + 4 * (64 + 64) + (64 + 8)


def bench_net(args):
    """The warm-start network on its own: inference at 2048^2 (a step), and
    training steps (forward, backward through all six layers, Adam) on batches
    of 16 x 256^2, both timed with HIP events on the network's stream."""
    import numpy as np
    import torch
    from paper_2110_01585_amd.net import Net, load_weights
    dev = torch.device("cuda:0")
    p, _ = make_workload("deconv2048")
    h, w = p.shape
    params, _ = load_weights()
    net = Net(params, max_batch=1, max_h=h, max_w=w, device=dev)
    y = torch.tensor(p.y, dtype=torch.float32, device=dev)
    mu = torch.empty_like(y)
    var = torch.empty_like(y)
    st = net.stream
    for _ in range(max(args.warmup, 1)):
        net.infer(y, p.xi, mu, var)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(st)
    for _ in range(args.steps):
        net.infer(y, p.xi, mu, var)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    net.close()
    npx = h * w
    flops = NET_FLOP_PER_PX * npx
    nbytes = NET_BYTES_PER_PX * npx
    # training at the size the network was trained at
    b, th, tw = 16, 256, 256
    tnet = Net(params, max_batch=b, max_h=th, max_w=tw, device=dev)
    g = torch.Generator(device="cpu").manual_seed(7)
    ty = torch.rand((b, th, tw), generator=g).to(dev)
    tmu = (ty + 0.01 * torch.randn((b, th, tw), generator=g).to(dev)).contiguous()
    tvar = torch.full((b, th, tw), 2e-5, device=dev)
    for _ in range(max(args.warmup, 1)):
        tnet.train_step(ty, tmu, tvar, 1e-4, 1e-4)
    torch.cuda.synchronize()
    e0.record(tnet.stream)
    for _ in range(args.steps):
        tnet.train_step(ty, tmu, tvar, 1e-4, 1e-4)
    e1.record(tnet.stream)
    torch.cuda.synchronize()
    tms = e0.elapsed_time(e1) / args.steps
    tnet.close()
    tflops = 3 * NET_FLOP_PER_PX * b * th * tw   # forward, input gradient, weight gradient
    line = {
        "metric": "warm-start network inferences/s, 2048^2, 1 GPU",
        "value": 1e3 / ms, "unit": "inferences/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "step": "one inference of the 6-layer 3x3 conv net on the 2048^2 deconvolution "
                "observation (statistics, six BF16-MFMA convolution layers, output map)",
        "config": {"workload": "net2048", "height": h, "width": w, "channels": 32, "layers": 6},
        "roofline": {"bound": "hbm", "achieved": round(nbytes / ms / 1e6, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(nbytes / ms / 1e6 / HBM_PEAK_GBS, 4),
                     "traffic": None, "kernel": "whole inference",
                     "bytes_per_px": NET_BYTES_PER_PX},
        "mfma": {"achieved_tflops": round(flops / ms / 1e9, 2), "peak_tflops": BF16_MFMA_PEAK_TFLOPS,
                 "frac": round(flops / ms / 1e9 / BF16_MFMA_PEAK_TFLOPS, 4),
                 "flop_per_px": NET_FLOP_PER_PX},
        "training": {"batch": [b, th, tw], "ms_per_step": round(tms, 3),
                     "achieved_tflops": round(tflops / tms / 1e9, 2),
                     "frac_bf16_peak": round(tflops / tms / 1e9 / BF16_MFMA_PEAK_TFLOPS, 4)},
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def _ctx(p, dev, graph, **kw):
    import numpy as np
    import torch
    from paper_2110_01585_amd import Context, spec_from_synthetic
    from paper_2110_01585_amd import _native as N
    rbmc = p.name == "rbmc512"
    if rbmc:
        kw["rbmc_samples"] = RBMC_SAMPLES
    ctx = Context([spec_from_synthetic(p, **kw)], device=dev)
    yh = np.stack([p.y.real, p.y.imag], -1) if p.op == "dft" else p.y
    y = torch.tensor(yh, dtype=torch.float32, device=dev).contiguous()
    ctx.ep_tv_set_observation([y])
    if rbmc:
        # the estimator's white noise (e1 in pixel space for the blur, then e2), seeded
        h, w = p.shape
        g = torch.Generator(device="cpu").manual_seed(12345)
        noise = torch.randn(RBMC_SAMPLES * 2 * h * w, generator=g).to(dev)
        ctx.ep_tv_set_rbmc_noise([noise])
    ctx.ep_tv_set_option(N.OPT_GRAPH, 1 if graph else 0)
    return ctx, y


def timing_pass_solve(ctx, args, em, N):
    """One cold solve launched kernel by kernel with HIP events around every
    launch (events are not recorded inside replayed graphs)."""
    ctx.ep_tv_set_option(N.OPT_GRAPH, 0)
    ctx.ep_tv_init_cold()
    ctx.ep_tv_set_timing(True)
    rc, st = ctx.ep_tv_solve(args.max_sweeps, args.tol, em, None, None)
    tm = ctx.ep_tv_get_timing()
    ctx.ep_tv_set_timing(False)
    ctx.ep_tv_set_option(N.OPT_GRAPH, 1 if args.launch == "graph" else 0)
    return tm, st[0]


def bench_solves(args, p, em):
    """Headline: K cold-start solves to convergence of the 2048^2 deconvolution."""
    import torch
    from paper_2110_01585_amd import _native as N
    h, w = p.shape
    E = edges(h, w)
    dev = torch.device("cuda:0")
    print(f"[bench] workload {args.workload} {h}x{w} op={p.op} em={em}", file=sys.stderr, flush=True)
    ctx, y = _ctx(p, dev, args.launch == "graph")
    ctx.ep_tv_set_option(N.OPT_PERSISTENT, args.persistent)
    ctx.ep_tv_run(3, em)                      # code objects, graph capture
    tune = ctx.ep_tv_autotune(5)              # sweep tile height (state unchanged)
    print(f"[bench] autotune: {tune}", file=sys.stderr, flush=True)
    mu = torch.empty(h, w, device=dev)
    var = torch.empty(h, w, device=dev)

    def cold_solve():
        ctx.ep_tv_init_cold()
        rc, st = ctx.ep_tv_solve(args.max_sweeps, args.tol, em, [mu], [var])
        return rc, st[0]

    for _ in range(args.warmup):
        cold_solve()
    torch.cuda.synchronize()
    sweeps, cg, times = [], [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        rc, st = cold_solve()
        times.append(time.perf_counter() - ts)
        sweeps.append(st["sweeps"])
        cg.append(st["cg_total"])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    value = E * sum(sweeps) / dt
    conv = {"s_to_converged_cold": round(dt / args.steps, 4),
            "s_to_converged_cold_min": round(min(times), 4),
            "sweeps_cold": sweeps[-1], "converged_cold": st["converged"], "status_cold": rc,
            "cg_iters_cold": cg[-1], "tol": args.tol, "lambda_cold": st["lambda"]}
    print(f"[bench] {args.steps} cold solves in {dt:.3f} s: {conv}", file=sys.stderr, flush=True)
    mu_c, var_c = mu.clone(), var.clone()

    # kernel timing pass and rooflines
    tm, st_t = timing_pass_solve(ctx, args, em, N)
    roof, kernels = kernel_rooflines(tm, h * w, args.workload, p.op)
    iters = max(tm["precond_launches"], 1)
    t_iter = (tm["apply_ms"] + tm["precond_ms"]) / iters / 1e3
    cg_iter = {"bytes_per_px": CG_ITER_BYTES_PER_PX, "avg_us": round(t_iter * 1e6, 2),
               "achieved": round(CG_ITER_BYTES_PER_PX * h * w / t_iter / 1e9, 1),
               "frac": round(CG_ITER_BYTES_PER_PX * h * w / t_iter / 1e9 / HBM_PEAK_GBS, 4),
               "iterations": tm["precond_launches"],
               "note": "H^T H product + RF_FWD + RF_FILT + RF_INV per CG iteration (finishing "
                       "kernel excluded)"}
    print(f"[bench] kernel timing ({st_t['sweeps']} sweeps): {tm}", file=sys.stderr, flush=True)

    if not args.no_warm:
        warm_solves(ctx, args, em, p, y, dev, torch, conv, mu, var)
    mu_w, var_w = mu.clone(), var.clone()
    if not args.no_accuracy:
        accuracy(ctx, args, em, p, dev, torch, conv, (mu_c, var_c), (mu_w, var_w))
    if args.cg_reduce > 0.0:
        conv["inexact"] = inexact_solves(args, em, p, y, dev, torch)
    ctx.close()

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] timing the oracle on the host", file=sys.stderr, flush=True)
        cpu = cpu_baseline_fullsize(p, em, sum(cg) / max(sum(sweeps), 1))
    line = {
        "metric": "EP factor-updates/s + s to converged 2048^2 deconv, warm-start vs plain, 1 GPU",
        "value": value, "unit": "factor-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3 / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "step": ("one cold-start EP-EM solve to convergence (tol %g) of the 2048^2 "
                 "deconvolution, y resident on the GPU; value = edges x sweeps summed over the "
                 "timed solves / their wall time; ms_per_step = seconds to converged" % args.tol),
        "config": {"workload": args.workload, "height": h, "width": w, "op": p.op, "em": em,
                   "edges_per_sweep": E, "damping": p.damping, "xi": p.xi,
                   "tile_rows": tune["tile_rows"], "launch": args.launch},
        "kernel_timing": ("HIP events on the context's stream around every launch of one more "
                          "cold solve launched kernel by kernel right after the timed solves "
                          "(events are not recorded inside replayed graphs)"),
        "roofline": roof, "roofline_kernels": kernels, "cg_iteration": cg_iter,
        "cpu_baseline": cpu, "convergence": conv,
        "timing_ms": {k: round(v, 3) if isinstance(v, float) else v for k, v in tm.items()},
    }
    print(json.dumps(line), flush=True)


def warm_solves(ctx, args, em, p, y, dev, torch, conv, mu, var):
    """Seconds to converged from the learned warm start: network inference,
    warm site initialisation, EP-EM to the same rule, min(K, 5) timed runs."""
    from paper_2110_01585_amd import Net, load_weights
    h, w = p.shape
    try:
        params, meta = load_weights()
    except FileNotFoundError:
        print("[bench] no trained warm-start weights in the package", file=sys.stderr, flush=True)
        return
    net = Net(params, max_batch=1, max_h=h, max_w=w, device=dev)
    mu_hat = torch.empty(h, w, device=dev)
    var_hat = torch.empty(h, w, device=dev)
    scale, power = meta["lambda_scale"], meta.get("lambda_power", 1.0)
    net.infer(y, p.xi, mu_hat, var_hat)          # code objects, caches
    ctx.ep_tv_init_warm([mu_hat], [var_hat], scale, power)
    ctx.ep_tv_solve(args.max_sweeps, args.tol, em, [mu], [var])
    torch.cuda.synchronize()
    n = max(1, min(args.steps, 5))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    for _ in range(n):
        e0.record()
        net.infer(y, p.xi, mu_hat, var_hat)
        e1.record()
        wrc = ctx.ep_tv_init_warm([mu_hat], [var_hat], scale, power)
        rc, st = ctx.ep_tv_solve(args.max_sweeps, args.tol, em, [mu], [var])
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / n
    conv.update({"s_to_converged_warm": round(dt, 4), "sweeps_warm": st[0]["sweeps"],
                 "converged_warm": st[0]["converged"], "status_warm": rc,
                 "cg_iters_warm": st[0]["cg_total"], "lambda_warm": st[0]["lambda"],
                 "warm_init_status": wrc, "net_infer_ms": round(e0.elapsed_time(e1), 3),
                 "speedup_warm_vs_cold": round(conv["s_to_converged_cold"] / dt, 3),
                 "lambda_scale": scale, "lambda_power": power})
    ctx.ep_tv_init_warm([mu_hat], [var_hat], scale, power)
    conv["lambda0_warm"] = ctx.ep_tv_get_stats()[0]["lambda"]
    net.close()
    print(f"[bench] warm solves: {conv}", file=sys.stderr, flush=True)


def accuracy(ctx, args, em, p, dev, torch, conv, cold, warm, ref_sweeps=3000):
    """Both results against the end of a 3000-sweep cold run (10x the sweeps
    to converge; the FP32 path's change per sweep settles at about 2.9e-6 of
    the range, so tolerances below 2.5e-6 are never met and a run to a 100x
    tighter tolerance does not end), with the last sweep's change reported, and
    the same GPU path against the FP64 oracle on the 512^2 member of the
    workload family (stored oracle run, tests/golden/deconv512.json: 200
    sweeps, 400 sampled pixels)."""
    import numpy as np
    h, w = p.shape
    ctx.ep_tv_init_cold()
    mu_r = torch.empty(h, w, device=dev)
    var_r = torch.empty(h, w, device=dev)
    # a tolerance no sweep meets: exactly ref_sweeps sweeps, with the deltas recorded
    rc, st_r = ctx.ep_tv_solve(ref_sweeps, 1e-12, em, [mu_r], [var_r])
    torch.cuda.synchronize()
    rng = float(mu_r.max() - mu_r.min())
    conv["reference"] = {"sweeps": st_r[0]["sweeps"], "last_dmu_range_rel": st_r[0]["dmu"],
                         "last_dv_rel": st_r[0]["dv"], "lambda": st_r[0]["lambda"]}
    for tag, (m_, v_) in (("cold", cold), ("warm", warm)):
        conv[f"mean_err_{tag}_vs_reference"] = float((m_ - mu_r).abs().max()) / rng
        conv[f"var_err_{tag}_vs_reference"] = float((v_ / var_r - 1).abs().max())
    # the FP32 path against the FP64 oracle at 512^2
    import synthetic as syn
    from paper_2110_01585_amd import _native as N
    with open(GOLDEN_DECONV512) as f:
        g = json.load(f)
    q = syn.config1()
    c2, _ = _ctx(q, dev, True)
    c2.ep_tv_run(g["sweeps"], True)
    (m5,), (v5,) = c2.marginals()
    lam5 = c2.ep_tv_get_stats()[0]["lambda"]
    torch.cuda.synchronize()
    c2.close()
    idx = np.asarray(g["pixels"])
    m5 = m5.cpu().numpy().astype(np.float64)[idx[:, 0], idx[:, 1]]
    v5 = v5.cpu().numpy().astype(np.float64)[idx[:, 0], idx[:, 1]]
    conv["oracle_check"] = {
        "workload": "deconv512 (200 sweeps from cold, EM), graph launches",
        "mean_err_range_rel": float(np.max(np.abs(m5 - np.asarray(g["mu"]))) / g["mu_range"]),
        "var_err_rel": float(np.max(np.abs(v5 / np.asarray(g["var"]) - 1))),
        "lambda_rel": abs(lam5 / g["lambda"] - 1), "pixels": len(idx)}
    print(f"[bench] accuracy: {conv}", file=sys.stderr, flush=True)


def inexact_solves(args, em, p, y, dev, torch):
    """One cold solve with the opt-in inexact likelihood solves (each CG also
    stops once its residual has fallen by cg_reduce); not part of the headline."""
    from paper_2110_01585_amd import Context, spec_from_synthetic
    from paper_2110_01585_amd import _native as N
    ctx = Context([spec_from_synthetic(p, cg_reduce=args.cg_reduce)], device=dev)
    ctx.ep_tv_set_observation([y])
    ctx.ep_tv_set_option(N.OPT_GRAPH, 1 if args.launch == "graph" else 0)
    ctx.ep_tv_run(3, em)
    ctx.ep_tv_init_cold()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, st = ctx.ep_tv_solve(args.max_sweeps, args.tol, em, None, None)
    torch.cuda.synchronize()
    out = {"cg_reduce": args.cg_reduce, "s_to_converged_cold": round(time.perf_counter() - t0, 4),
           "sweeps_cold": st[0]["sweeps"], "cg_iters_cold": st[0]["cg_total"]}
    ctx.close()
    return out


def bench_sweeps(args, p, em):
    """Secondary single-image workloads: a step is one sweep."""
    import torch
    from paper_2110_01585_amd import _native as N
    h, w = p.shape
    E = edges(h, w)
    dev = torch.device("cuda:0")
    print(f"[bench] workload {args.workload} {h}x{w} op={p.op} em={em}", file=sys.stderr, flush=True)
    ctx, y = _ctx(p, dev, args.launch == "graph")
    ctx.ep_tv_set_option(N.OPT_PERSISTENT, args.persistent)
    ctx.ep_tv_run(max(args.warmup, 2), em)
    tune = ctx.ep_tv_autotune(5)
    print(f"[bench] autotune: {tune}", file=sys.stderr, flush=True)
    cold_phase = args.cold_phase if p.op == "hadamard" else (20 if p.name == "rbmc512" else 0)

    def prime():
        ctx.ep_tv_init_cold()
        if cold_phase:
            ctx.ep_tv_run(cold_phase, em)
        ctx.ep_tv_run(args.warmup, em)

    prime()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.ep_tv_run(args.steps, em)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    value = E * args.steps / dt
    # the same sweeps launched one by one with HIP events
    ctx.ep_tv_set_option(N.OPT_GRAPH, 0)
    prime()
    ctx.ep_tv_set_timing(True)
    ctx.ep_tv_run(args.steps, em)
    tm = ctx.ep_tv_get_timing()
    ctx.ep_tv_set_timing(False)
    ctx.close()
    roof, kernels = kernel_rooflines(tm, h * w, args.workload, p.op)
    cpu = None
    if not args.no_cpu_baseline:
        size, sweeps = CPU_SAMPLE.get(args.workload, (256, 4))
        cpu = cpu_baseline_sample(args.workload, args.cpu_size or size, args.cpu_sweeps or sweeps)
    line = {
        "metric": f"EP factor-updates/s, {args.workload}, 1 GPU",
        "value": value, "unit": "factor-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3 / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "step": ("one EP sweep" + (f" after {cold_phase} untimed sweeps from cold" if cold_phase
                                   else " (the sweeps after the warm-up ones)")),
        "config": {"workload": args.workload, "height": h, "width": w, "op": p.op, "em": em,
                   "edges_per_sweep": E, "tile_rows": tune["tile_rows"], "launch": args.launch},
        "kernel_timing": "HIP events on the context's stream around every launch of the same "
                         "number of sweeps launched kernel by kernel",
        "roofline": roof, "roofline_kernels": kernels, "cpu_baseline": cpu,
        "timing_ms": {k: round(v, 3) if isinstance(v, float) else v for k, v in tm.items()},
    }
    print(json.dumps(line), flush=True)


def bench_batch(args, ps, em):
    """Many instances in one context: graph launches, autotuned tiles; a step is
    one sweep over all instances."""
    import torch
    from paper_2110_01585_amd import Context, spec_from_synthetic
    from paper_2110_01585_amd import _native as N
    dev = torch.device("cuda:0")
    E = sum(edges(*p.shape) for p in ps)
    npx = sum(p.shape[0] * p.shape[1] for p in ps)
    print(f"[bench] workload {args.workload}: {len(ps)} instances, {npx / 1e6:.2f} M pixels, "
          f"{E / 1e6:.2f} M edges per sweep", file=sys.stderr, flush=True)
    ctx = Context([spec_from_synthetic(p, cg_precond=N.PRECOND_JACOBI) for p in ps], device=dev)
    ctx.ep_tv_set_option(N.OPT_PERSISTENT, args.persistent)
    ctx.ep_tv_set_observation([torch.tensor(p.y, dtype=torch.float32, device=dev) for p in ps])
    tune = ctx.ep_tv_autotune(5)
    print(f"[bench] autotune: {tune}", file=sys.stderr, flush=True)
    ctx.ep_tv_set_timing(True)
    ctx.ep_tv_run(max(args.warmup, 3), em)
    tm = ctx.ep_tv_get_timing()
    ctx.ep_tv_set_timing(False)
    ctx.ep_tv_set_option(N.OPT_GRAPH, 1)
    ctx.ep_tv_run(2, em)                       # captures the graphs
    ctx.ep_tv_init_cold()
    ctx.ep_tv_run(args.warmup, em)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.ep_tv_run(args.steps, em)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    value = E * args.steps / dt
    print(f"[bench] {args.steps} sweeps in {dt * 1e3:.1f} ms", file=sys.stderr, flush=True)
    roof = roofline_entry("k_tv_sweep", npx, tm["sweep_ms"], tm["sweep_launches"], args.workload)
    conv = None
    if args.max_sweeps > 0:
        ctx.ep_tv_init_cold()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        rc, st = ctx.ep_tv_solve(min(args.max_sweeps, 1000), args.tol, em, None, None)
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
    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] timing the oracle on a process pool", file=sys.stderr, flush=True)
        cpu = cpu_baseline_pool(ps)
    line = {
        "metric": "EP factor-updates/s, batched denoising+deconvolution, 1 GPU",
        "value": value, "unit": "factor-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3 / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "step": "one EP sweep over all instances (graph replay), after the warm-up sweeps from cold",
        "config": {"workload": args.workload, "instances": len(ps), "pixels": npx,
                   "edges_per_sweep": E, "launch": "hipGraph", "tile_rows": tune["tile_rows"],
                   "cg_precond": "jacobi"},
        "roofline": roof, "cpu_baseline": cpu, "convergence": conv, "autotune": tune,
        "timing_ms": {"sweep": tm["sweep_ms"], "likelihood": tm["lik_ms"]},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
