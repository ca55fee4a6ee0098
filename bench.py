"""Throughput of the randomized von Neumann entropy estimator on one MI355X.

A step is one complete estimate (trace check, power method, interval and
coefficients, the m recurrence products with fused epilogues, reductions) of
one synthetic density matrix already resident in HBM.  The default workload
is the dense one: n = 8192, p_i ~ exp(-i/1000), random orthogonal U,
Chebyshev degree 50, 256 Gaussian probes, 20 power iterations.

Printed: one JSON line with estimates/s, a roofline entry for the dominant
kernel (the dense R.V step; HIP events recorded by the library on its stream
around each launch) and the CPU oracle timed on a bounded sample of the same
estimate, which also checks the sampled per-probe values of the GPU run.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAKS = {  # MI355X published peaks
    "f64": ("mfma", 78.6, "TFLOP/s"),
    "f32": ("mfma", 157.3, "TFLOP/s"),
    "bf16x3": ("mfma", 2500.0, "TFLOP/s"),
    "hbm": ("hbm", 8000.0, "GB/s"),
}

WORKLOADS = {
    "dense8192": dict(n=8192, tau=1000.0, method="chebyshev", m=50, s=256, dist="gaussian", t=20),
    "dense8192_taylor": dict(n=8192, tau=1000.0, method="taylor", m=50, s=256, dist="gaussian", t=20),
    "dense512": dict(n=512, spectrum="inverse", method="chebyshev", m=30, s=50, dist="rademacher", t=20),
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_dense(cfg, seed):
    import workloads as W

    n = cfg["n"]
    p = W.spectrum_inverse(n) if cfg.get("spectrum") == "inverse" else W.spectrum_exp(n, cfg["tau"])
    return W.dense_density(p, seed), p


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="dense8192", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="f64", choices=["f64", "f32", "bf16x3"])
    ap.add_argument("--cpu-probes", type=int, default=0, help="oracle sample size (0 = host threads)")
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (the estimator shards "
              "over probes with one all-reduce of the moment partials; see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1801_01072_amd as ent
    import workloads as W

    cfg = WORKLOADS[args.workload]
    n, m, s, t = cfg["n"], cfg["m"], cfg["s"], cfg["t"]
    mseed, pseed = W.MATRIX_SEED + 2, W.PROBE_SEED + 2
    t0 = time.time()
    R, p = make_dense(cfg, mseed)
    log(f"generated R n={n} in {time.time() - t0:.1f}s")
    H_exact = float(-np.sum(p[p > 0] * np.log(p[p > 0])))
    Rd = torch.from_numpy(R).to("cuda:0")
    torch.cuda.synchronize()
    kw = dict(probe_dist=cfg["dist"], precision=args.precision, power_iters=t)

    for _ in range(args.warmup):
        ent.entropy_estimate(Rd, cfg["method"], m, s, pseed, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = ent.entropy_estimate(Rd, cfg["method"], m, s, pseed, **kw)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps
    log(f"timed {args.steps} estimates: {ms_per_step:.3f} ms/estimate, H^={res.entropy:.12f}")

    # per-launch durations of the dominant kernel from HIP events on its stream
    ent.timing_enable(True)
    step_ms, power_ms, total_ms, launches = [], [], [], 0
    for _ in range(max(3, min(args.steps, 10))):
        ent.entropy_estimate(Rd, cfg["method"], m, s, pseed, **kw)
        tm = ent.last_timing()
        step_ms.append(tm["steps_ms"] / tm["step_launches"])
        power_ms.append(tm["power_ms"])
        total_ms.append(tm["total_ms"])
        launches = tm["step_launches"]
    ent.timing_enable(False)
    avg_step_ms = float(np.mean(step_ms))
    flop_per_launch = 2.0 * n * n * s
    bound, peak, unit = PEAKS[args.precision]
    achieved = flop_per_launch / (avg_step_ms * 1e-3) / 1e12
    log(f"step kernel avg {avg_step_ms:.4f} ms over {launches} launches -> {achieved:.2f} TFLOP/s; "
        f"power {np.mean(power_ms):.3f} ms; total {np.mean(total_ms):.3f} ms")

    # accuracy of sampled probes and the CPU oracle baseline on the same estimate
    gpu_res, per, _ = ent.entropy_estimate_detail(Rd, cfg["method"], m, s, pseed, **kw)
    cpu = None
    max_rel = None
    if not args.no_cpu:
        import oracle

        threads = oracle.max_threads()
        nsamp = args.cpu_probes or min(threads, s)
        probes = list(np.linspace(0, s - 1, nsamp).astype(int))
        meth = oracle.CHEBYSHEV if cfg["method"] == "chebyshev" else oracle.TAYLOR
        dist = 1 if cfg["dist"] == "gaussian" else 0
        tc = time.perf_counter()
        ref = oracle.estimate(R, meth, m, s, pseed, t=t, dist=dist, probes=probes)
        cpu_s = time.perf_counter() - tc
        # the sample ran the power method once plus nsamp of the s probes
        tp = time.perf_counter()
        oracle.power_method(R, t, 1, pseed)
        power_s = time.perf_counter() - tp
        per_probe_s = max(cpu_s - power_s, 1e-9)
        waves = int(np.ceil(s / nsamp))
        est_s = power_s + waves * per_probe_s
        scale = np.mean(np.abs(ref.per_probe))
        max_rel = float(np.max(np.abs(per[probes] - ref.per_probe)) / scale)
        log(f"oracle: {nsamp} probes + power method in {cpu_s:.2f}s on {threads} threads; "
            f"sampled per-probe rel err {max_rel:.2e}")
        cpu = {"value": 1.0 / est_s, "unit": "estimates/s", "cores": threads, "kind": "oracle",
               "sample": f"power method + {nsamp} of {s} probes of the same estimate, "
                         f"extrapolated to {s} probes ({waves} rounds of {nsamp})"}

    out = {
        "metric": "entropy estimates/s at <=1e-3 rel err",
        "value": 1e3 / ms_per_step,
        "unit": "estimates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": f"dense density matrix n={n}, p_i ~ exp(-i/{cfg.get('tau')}), "
                               f"{cfg['method']} m={m}, s={s} {cfg['dist']} probes, t={t}",
                   "n": n, "degree": m, "probes": s, "method": cfg["method"],
                   "precision": args.precision, "parallelism": "single GPU"},
        "roofline": {"bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
                     "frac": achieved / peak, "traffic": None,
                     "kernel": "dense_step_kernel", "avg_launch_ms": avg_step_ms,
                     "flop_per_launch": flop_per_launch},
        "cpu_baseline": cpu,
        "accuracy": {"entropy": gpu_res.entropy, "std_err": gpu_res.std_err, "exact_H": H_exact,
                     "rel_err_vs_exact": abs(gpu_res.entropy - H_exact) / H_exact,
                     "sampled_per_probe_rel_err_vs_oracle": max_rel},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
