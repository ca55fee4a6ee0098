"""Throughput of the randomized von Neumann entropy estimator on one MI355X.

A step is one complete estimate -- trace check, power method (20
iterations), interval and coefficients, the m recurrence products with their
epilogues, reductions -- of one synthetic density matrix already resident in
HBM.  Default workload: dense n = 8192, p_i ~ exp(-i/1000), random orthogonal
eigenvectors, Chebyshev degree 50, 256 Gaussian probes, in the paper's
arithmetic (FP64; its experiments run in double precision).  The same
estimate in FP32 and in BF16x3 (three bf16 products, FP32 accumulation) is
timed beside it, with its speedup over FP64 and its error.

Printed: one JSON line with estimates/s, a roofline entry for the dominant
kernel (its launches timed by HIP events the library records on its own
stream) and the CPU oracle timed on a bounded sample of the same estimate.
The same oracle sample checks the GPU's per-probe values of every form: a
headline whose sampled per-probe error exceeds 1e-3 relative is printed with
value null and the script exits non-zero.
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

# MI355X published peaks
MFMA_PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16x3": 2500.0}
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "dense8192": dict(kind="dense", n=8192, spectrum=("exp", 1000.0), method="chebyshev", m=50,
                      s=256, dist="gaussian", t=20),
    "dense8192_taylor": dict(kind="dense", n=8192, spectrum=("exp", 1000.0), method="taylor",
                             m=50, s=256, dist="gaussian", t=20),
    "dense512": dict(kind="dense", n=512, spectrum=("inverse",), method="chebyshev", m=30, s=50,
                     dist="rademacher", t=20),
    "csr1e7": dict(kind="csr", n=10_000_000, hb=8, method="chebyshev", m=40, s=64,
                   dist="rademacher", t=20),
    "csr1e5": dict(kind="csr", n=100_000, hb=8, method="chebyshev", m=40, s=64,
                   dist="rademacher", t=20),
    # the paper's largest experiment at full size: the 10^8 x 10^8 tridiagonal
    # (-1, 2, -1)/2n, m = 10, s = 100, c = 1; exact H from the closed-form spectrum
    "poisson1e8": dict(kind="csr", matrix="poisson", n=100_000_000, method="chebyshev", m=10, s=100,
                       dist="rademacher", t=20, c=1.0, cpu_probes=4),
    "batch1024": dict(kind="batch", count=1024, n_lo=64, n_hi=2048, method="chebyshev", m=40,
                      s=64, dist="rademacher", t=20),
    "batch64": dict(kind="batch", count=64, n_lo=64, n_hi=2048, method="chebyshev", m=40,
                    s=64, dist="rademacher", t=20),
    "learned4096": dict(kind="learned", count=512, n=4096, m=40, s=64, dist="rademacher", t=20),
    "rp65536": dict(kind="rp", n=65536, k=64, s=128, tau=8.0),
    "rp65536_srht": dict(kind="rp", n=65536, k=64, s=128, tau=8.0, sketch="srht"),
    # the input-sparsity sketch needs s ~ k^2: rank 8, s = 2 k^2 (widths above
    # 128 run the s x s eigenproblem out of LDS, ~0.2 s at s = 256)
    "rp65536_count": dict(kind="rp", n=65536, k=8, s=128, tau=2.0, sketch="count"),
    # Hermitian (complex) density matrix of the paper's Hermitian experiment size
    "herm5000": dict(kind="herm", n=5000, spectrum=("exp", 600.0), method="chebyshev", m=50,
                     s=256, dist="gaussian", t=20),
    # plain device-to-device copy of 1 GiB: the achievable HBM rate, and the
    # reference that scales the hardware byte counters of the other kernels
    "copy1g": dict(kind="copy", nbytes=1 << 30),
}


KERNEL_SOURCES = {
    "bf16x3_gemm_kernel": "kernels_bf16.hip",
    "batch_bf16x3_step_kernel": "kernels_bf16.hip",
    "batch_bf16x3_persistent_kernel": "kernels_bf16.hip",
    "dense_step_kernel": "kernels_dense.hip",
    "dense_step_split_kernel": "kernels_dense.hip",
    "batch_dense_step_kernel": "kernels_dense.hip",
    "batch_dense_persistent_kernel": "kernels_dense.hip",
    "csr_step_kernel": "kernels_csr.hip",
    "band_step_kernel": "kernels_band.hip",
    "band_pair_kernel": "kernels_band.hip",
    "tri_step_kernel": "kernels_tri.hip",
    "tri_fused_kernel": "tri_fused_impl.hpp",
}


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` on `workload` from the committed
    hardware-counter summary (profiles/<kernel>__<workload>__traffic.md),
    or None when there is none or the kernel's source changed since."""
    import hashlib

    path = os.path.join(ROOT, "profiles", f"{kernel}__{workload}__traffic.md")
    src = os.path.join(ROOT, "paper_1801_01072_amd", "csrc", KERNEL_SOURCES.get(kernel, ""))
    if not os.path.exists(path) or not os.path.isfile(src):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            fields[k.strip()] = v.strip().strip("`")
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if fields.get("source_sha256") != digest or "hbm_bytes_per_launch" not in fields:
        return None
    return float(fields["hbm_bytes_per_launch"])


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def describe(cfg, precision, store):
    if cfg["kind"] == "herm":
        sp = cfg["spectrum"]
        return (f"Hermitian (complex) density matrix n={cfg['n']}, p_i ~ exp(-i/{sp[1]:g}), Haar-random "
                f"unitary U, {store} storage; {cfg['method']} m={cfg['m']}, s={cfg['s']} {cfg['dist']} "
                f"probes, u = 6 p~1 from t={cfg['t']} power iterations on the real 2n x 2n form, {precision}")
    if cfg["kind"] == "dense":
        sp = cfg["spectrum"]
        spec = "p_i ~ 1/i" if sp[0] == "inverse" else f"p_i ~ exp(-i/{sp[1]:g})"
        return (f"dense density matrix n={cfg['n']}, {spec}, random orthogonal U; {cfg['method']} "
                f"m={cfg['m']}, s={cfg['s']} {cfg['dist']} probes, t={cfg['t']}, {precision}")
    if cfg.get("matrix") == "poisson":
        return (f"tridiagonal CSR density matrix (-1, 2, -1)/2n, n={cfg['n']:.0e}, {store} values; "
                f"{cfg['method']} m={cfg['m']}, s={cfg['s']} {cfg['dist']} probes, t={cfg['t']}, "
                f"u = {cfg.get('c', 6.0):g} p~1, {precision}")
    return (f"banded CSR density matrix n={cfg['n']:.0e}, R = B B^T / tr with B half-bandwidth "
            f"{cfg['hb']}, {store} values; {cfg['method']} m={cfg['m']}, s={cfg['s']} "
            f"{cfg['dist']} probes, t={cfg['t']}, {precision}")


def csr_step_bytes(n, nnz, s, m, vbytes, method):
    """Algorithmic HBM bytes of the m product steps: the CSR arrays, the probe
    sign bits and the V blocks each step must read and write once."""
    csr = (vbytes + 4) * nnz + 8 * (n + 1)
    signs = n * s / 8
    blk = n * s * vbytes
    tot = 0.0
    steps = m if method == "chebyshev" else m + 1
    for k in range(steps):
        reads_vk = k > 0                                   # V_0 is the sign block
        reads_vm1 = method == "chebyshev" and k > 1        # V_{k-1} for k = 1 is the sign block
        writes = method == "chebyshev" or k < steps - 1
        tot += csr + signs + blk * (reads_vk + reads_vm1 + writes)
    return tot, steps


def tri_step_bytes(n, s, m, vbytes, method):
    """Algorithmic HBM bytes of the m product steps of the tridiagonal kernel:
    three values (stored as four) per row, the probe sign bits and the V
    blocks each step must read and write once."""
    diag = 4 * vbytes * n
    signs = n * s / 8
    blk = n * s * vbytes
    tot = 0.0
    steps = m if method == "chebyshev" else m + 1
    for k in range(steps):
        reads_vk = k > 0
        reads_vm1 = method == "chebyshev" and k > 1
        writes = method == "chebyshev" or k < steps - 1
        tot += diag + signs + blk * (reads_vk + reads_vm1 + writes)
    return tot, steps


def fuse_split(steps, nf):
    """The engine's split of the recurrence steps into launches of at most nf
    steps, as even as possible, longer launches first."""
    nl = -(-steps // nf)
    return [steps // nl + (1 if i < steps % nl else 0) for i in range(nl)]


def tri_fused_bytes(n, s, m, vbytes, method, nf):
    """Algorithmic HBM bytes of the multi-step tridiagonal launches (up to nf
    steps per pass): the diagonals and sign bits once per pass, V_k and
    V_{k-1} read once, the last two steps' blocks written once (a one-step
    launch excluded).  Returns (bytes, launches)."""
    diag = 4 * vbytes * n
    signs = n * s / 8
    blk = n * s * vbytes
    steps = m if method == "chebyshev" else m + 1
    tot, launches, k = 0.0, 0, 0
    for ln in fuse_split(steps, nf):
        if ln >= 2:
            reads = (k > 0) + (method == "chebyshev" and k > 1)
            writes = 1 + (method == "chebyshev" or k + ln - 1 < steps - 1)
            tot += diag + signs + blk * (reads + writes)
            launches += 1
        k += ln
    return tot, launches


def band_pair_bytes(n, hp, s, m, vbytes, method):
    """Algorithmic HBM bytes of the two-step banded launches (steps k, k + 1
    in one pass): the slabs and sign bits once per pass, V_k and V_{k-1}
    read once, V_{k+1} and V_{k+2} written once.  Returns (bytes of the pair
    launches, number of pair launches); an odd last step runs alone and is
    not included."""
    slabs = ((n + 15) // 16) * 16 * (16 + 2 * hp) * vbytes
    signs = n * s / 8
    blk = n * s * vbytes
    steps = m if method == "chebyshev" else m + 1
    tot, pairs = 0.0, 0
    for k in range(0, steps - 1, 2):
        reads = (k > 0) + (method == "chebyshev" and k > 1)
        writes = 1 + (method == "chebyshev" or k + 1 < steps - 1)
        tot += slabs + signs + blk * (reads + writes)
        pairs += 1
    return tot, pairs


def band_step_bytes(n, hp, s, m, vbytes, method):
    """Algorithmic HBM bytes of the m product steps of the banded kernel: the
    16-row slabs (16 + 2 hp values per row, zeros of the band included), the
    probe sign bits and the V blocks each step must read and write once."""
    slabs = ((n + 15) // 16) * 16 * (16 + 2 * hp) * vbytes
    signs = n * s / 8
    blk = n * s * vbytes
    tot = 0.0
    steps = m if method == "chebyshev" else m + 1
    for k in range(steps):
        reads_vk = k > 0
        reads_vm1 = method == "chebyshev" and k > 1
        writes = method == "chebyshev" or k < steps - 1
        tot += slabs + signs + blk * (reads_vk + reads_vm1 + writes)
    return tot, steps


def bench_batch(args, cfg):
    """Many dense matrices of uneven n in one hipGraph launch (one step = one batch)."""
    import torch

    import paper_1801_01072_amd as ent
    import workloads as W

    precision = args.precision or "f32"
    count, m, s, t = cfg["count"], cfg["m"], cfg["s"], cfg["t"]
    mseed, pseed = W.MATRIX_SEED + 4, W.PROBE_SEED + 4
    t0 = time.time()
    ns, ks = W.batch_shapes(count, mseed, cfg["n_lo"], cfg["n_hi"])
    spectra = W.batch_spectra(ns, ks, mseed)
    mats = []
    for i, p in enumerate(spectra):
        mats.append(W.dense_density_torch(p, mseed * 7 + i, device="cuda:0", dtype=torch.float32))
        if (i + 1) % 128 == 0:
            torch.cuda.synchronize()
            log(f"generated {i + 1}/{count} matrices ({time.time() - t0:.1f} s)")
    torch.cuda.synchronize()
    sum_n2 = float(np.sum(ns.astype(np.float64) ** 2))
    log(f"generated {count} matrices (sum n^2 = {sum_n2:.3e}) in {time.time() - t0:.1f}s")
    flags = ent.FLAG_AUTOTUNE | (ent.FLAG_BATCH_STEPWISE if getattr(args, "batch_stepwise", False) else 0)
    g = ent.Graph(mats, cfg["method"], m, s, pseed, precision=precision, probe_dist=cfg["dist"],
                  power_iters=t, flags=flags)
    log(f"graph ready: tile rows {g.tile_rows}, step schedule window {g.window_bytes >> 20} MB "
        f"(0: one launch per step), workspace {g.workspace_bytes / 1e9:.2f} GB")
    for _ in range(args.warmup):
        g.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = g.launch()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps
    log(f"timed {args.steps} batch launches: {ms_per_step:.2f} ms per batch of {count}")
    tms = [g.time_eager()[1] for _ in range(3)]
    avg_step_ms = float(np.mean([x["steps_ms"] / x["step_launches"] for x in tms]))
    phases = {k: float(np.mean([x[k] for x in tms])) for k in ("total_ms", "power_ms", "steps_ms", "epilogue_ms", "other_ms")}
    flop = 2.0 * sum_n2 * s
    achieved = flop / (avg_step_ms * 1e-3) / 1e12
    peak = MFMA_PEAK_TFLOPS[precision]
    nsteps = m if cfg["method"] == "chebyshev" else m + 1
    persistent = g.window_bytes > 0
    bf = precision == "bf16x3"
    if persistent:
        # one launch runs every recurrence step of every matrix
        kernel = "batch_bf16x3_persistent_kernel" if bf else "batch_dense_persistent_kernel"
        launch_ms, flop_launch = avg_step_ms * nsteps, flop * nsteps
    else:
        kernel = "batch_bf16x3_step_kernel" if bf else "batch_dense_step_kernel"
        launch_ms, flop_launch = avg_step_ms, flop
    log(f"{kernel}: {launch_ms:.3f} ms/launch, {avg_step_ms:.3f} ms per recurrence step -> "
        f"{achieved:.1f} TFLOP/s; phases {phases}")
    cpu = None
    H_exact = [float(-np.sum(p[p > 0] * np.log(p[p > 0]))) for p in spectra]
    import oracle

    per = g.per_probe()
    # the accuracy gate: 4 matrices spread over the sizes (1, the smallest,
    # under --no-cpu), all probes, against the FP64 oracle
    if args.no_cpu:
        idx = [int(np.argmin(ns))]
    else:
        idx = [int(i) for i in np.argsort(ns)[np.linspace(0, count - 1, 4).astype(int)]]
    tc = time.perf_counter()
    errs = []
    for b in idx:
        Rh = mats[b].double().cpu().numpy()
        ref = oracle.estimate(Rh, 1 if cfg["method"] == "chebyshev" else 0, m, s, pseed + b, t=t,
                              dist=0 if cfg["dist"] == "rademacher" else 1)
        errs.append(float(np.max(np.abs(per[b] - ref.per_probe)) / np.mean(np.abs(ref.per_probe))))
    cpu_s = time.perf_counter() - tc
    samp_n2 = float(np.sum(ns[idx].astype(np.float64) ** 2))
    max_rel = max(errs)
    if not args.no_cpu:
        cpu = {"value": count / (cpu_s * sum_n2 / samp_n2), "unit": "estimates/s",
               "cores": oracle.max_threads(), "kind": "oracle",
               "sample": f"{len(idx)} of {count} matrices (all {s} probes), {cpu_s:.1f} s, "
                         f"extrapolated by sum n^2"}
    log(f"oracle sample: {cpu_s:.1f}s, per-probe rel err vs fp64 oracle {max_rel:.2e}")
    meets = max_rel <= ACC_BAR
    rel_exact = float(np.median([abs(r.entropy - h) / h for r, h in zip(res, H_exact) if h > 0]))
    out = {
        "metric": "entropy estimates/s at <=1e-3 rel err",
        "value": (count * 1e3 / ms_per_step) if meets else None,
        "unit": "estimates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": precision,
        "data": "synthetic",
        "config": {"workload": f"batch of {count} dense density matrices, n ~ U[{cfg['n_lo']},{cfg['n_hi']}], "
                               f"rank ~ U[n/8,n], Dirichlet(0.5) spectra; {cfg['method']} m={m}, s={s} "
                               f"{cfg['dist']} probes, t={t}; one hipGraph launch per batch",
                   "count": count, "sum_n2": sum_n2, "precision": precision,
                   "tile_rows": g.tile_rows, "schedule_window_bytes": g.window_bytes,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak,
                     "traffic": measured_traffic(kernel, args.workload + ("" if precision == "f32" else "_" + precision)),
                     "kernel": kernel,
                     "avg_launch_ms": launch_ms, "algorithmic_flop_per_launch": flop_launch,
                     "ms_per_recurrence_step": avg_step_ms, "launches_per_batch": 1 if persistent else nsteps},
        "cpu_baseline": cpu,
        "phases_ms": phases,
        "accuracy": {"sampled_matrices": len(idx),
                     "sampled_per_probe_max_rel_err_vs_fp64_oracle": max_rel,
                     "bar": ACC_BAR, "meets_bar": meets,
                     "median_rel_err_vs_exact": rel_exact},
    }
    g.destroy()
    print(json.dumps(out), flush=True)
    if not meets:
        sys.exit(3)


def truncation_report(spectra, auto, plain, m_plain, L, m_max=400):
    """Truncation error of the polynomial each run used, from the known
    spectrum: |sum_i p(lambda_i) - H| / H with p the Chebyshev expansion of
    x ln x on the run's [lo, u] at its degree (the probe-free part of the
    estimate).  Reports how often the selector's runs and the plain runs meet
    the selector's training target, and the smallest fixed plain degree on
    [0, u] that meets it on as many matrices (the plain schedule at matched
    accuracy)."""
    import torch

    bar = L.TARGET_ERR
    e_auto, e_plain, curves = [], [], []
    for p, ra, rp in zip(spectra, auto, plain):
        p = np.asarray(p, dtype=np.float64)
        H = float(-np.sum(p[p > 0] * np.log(p[p > 0])))

        def moments(lo, u, deg):
            t = (2.0 * p - (u + lo)) / (u - lo)
            out = np.empty(deg + 1)
            tkm1, tk = np.ones_like(t), t.copy()
            out[0] = p.size
            if deg >= 1:
                out[1] = tk.sum()
            for k in range(2, deg + 1):
                tkm1, tk = tk, 2.0 * t * tk - tkm1
                out[k] = tk.sum()
            return out

        def coeffs(lo, u, deg):
            uu = torch.tensor([u], dtype=torch.float64)
            if lo > 0:
                return L.cutoff_coeffs(lo / u, uu, deg)[0].numpy()
            return L.lemma3_coeffs(uu, deg)[0].numpy()

        if ra.method == 2:  # Algorithm 3: no polynomial
            e_auto.append(abs(ra.entropy - H) / H)
        else:
            e_auto.append(abs(-coeffs(ra.lo, ra.u, ra.degree) @ moments(ra.lo, ra.u, ra.degree) - H) / H)
        c = coeffs(0.0, rp.u, m_max)
        curve = np.abs(-np.cumsum(c * moments(0.0, rp.u, m_max)) - H) / H
        e_plain.append(curve[m_plain])
        curves.append(curve)
    e_auto, e_plain, curves = np.array(e_auto), np.array(e_plain), np.array(curves)
    need = int(np.sum(e_auto <= bar))
    meets = (curves <= bar).sum(axis=0)
    ok = np.nonzero(meets >= need)[0]
    m_eq = int(ok[0]) if ok.size else None
    return {"bar": bar, "auto_meets_bar": float(np.mean(e_auto <= bar)),
            "plain_meets_bar": float(np.mean(e_plain <= bar)),
            "median_auto": float(np.median(e_auto)), "median_plain": float(np.median(e_plain)),
            "plain_degree_matching_auto": m_eq,
            "plain_products_matching_auto": (m_eq * len(spectra)) if m_eq is not None else None}


def bench_learned(args, cfg):
    """The learned selector (method "auto") on held-out dense n = 4096 density
    matrices of the training families, against the plain schedule (Chebyshev
    on [0, u], degree m) with the same probes.  One step = one pass over the
    held-out set."""
    import torch

    import paper_1801_01072_amd as ent
    import workloads as W
    from paper_1801_01072_amd import learned as L

    precision = args.precision or "f32"
    count = args.count or cfg["count"]
    n, m, s, t = cfg["n"], cfg["m"], cfg["s"], cfg["t"]
    mseed, pseed = W.MATRIX_SEED + 5, W.PROBE_SEED + 5
    ent.selector_load(L.load())
    rng = np.random.default_rng(mseed + 10**6)          # disjoint from the training seeds
    t0 = time.time()
    spectra, fams, mats = [], [], []
    for i in range(count):
        p, fam = L.sample_spectrum(rng, n)
        spectra.append(p)
        fams.append(fam)
        mats.append(W.dense_density_torch(p, mseed * 7 + i, device="cuda:0", dtype=torch.float32,
                                          rng_device="cuda:0"))
        if (i + 1) % 64 == 0:
            torch.cuda.synchronize()
            log(f"generated {i + 1}/{count} held-out matrices ({time.time() - t0:.1f} s)")
    torch.cuda.synchronize()
    H = np.array([float(-np.sum(p[p > 0] * np.log(p[p > 0]))) for p in spectra])
    kw = dict(probe_dist=cfg["dist"], precision=precision, power_iters=t)

    def one_pass(method, degree=m):
        return [ent.entropy_estimate(R, method, degree, s, pseed + i, **kw) for i, R in enumerate(mats)]

    for _ in range(args.warmup):
        one_pass("auto")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        auto = one_pass("auto")
    torch.cuda.synchronize()
    ms_auto = 1e3 * (time.perf_counter() - t0) / args.steps
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plain = one_pass("chebyshev")
    torch.cuda.synchronize()
    ms_plain = 1e3 * (time.perf_counter() - t0) / args.steps
    err_auto = np.array([abs(r.entropy - h) / h for r, h in zip(auto, H)])
    err_plain = np.array([abs(r.entropy - h) / h for r, h in zip(plain, H)])
    prod_auto = int(sum(r.products for r in auto))
    prod_plain = int(sum(r.products for r in plain))
    fb = float(np.mean([r.fell_back for r in auto]))
    log(f"auto {ms_auto:.1f} ms/pass ({prod_auto} products, fallback {100 * fb:.1f}%), plain "
        f"{ms_plain:.1f} ms/pass ({prod_plain} products); median rel err vs exact: auto "
        f"{np.median(err_auto):.2e}, plain {np.median(err_plain):.2e}")
    trunc = truncation_report(spectra, auto, plain, m, L)
    log(f"truncation (polynomial trace vs exact, bar {L.TARGET_ERR:g}): auto meets it on "
        f"{trunc['auto_meets_bar']:.3f}, plain m={m} on {trunc['plain_meets_bar']:.3f}; plain needs "
        f"m={trunc['plain_degree_matching_auto']} to meet it as often ({trunc['plain_products_matching_auto']} "
        f"products vs {prod_auto})")
    m_eq = trunc["plain_degree_matching_auto"]
    if m_eq is not None:
        one_pass("chebyshev", m_eq)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        one_pass("chebyshev", m_eq)
        torch.cuda.synchronize()
        trunc["plain_matching_estimates_per_s"] = count / (time.perf_counter() - t0)
        log(f"plain at m={m_eq}: {trunc['plain_matching_estimates_per_s']:.1f} estimates/s "
            f"(auto {count * 1e3 / ms_auto:.1f})")

    # dominant kernel: the recurrence product of the main pass
    ent.timing_enable(True)
    tms = []
    for i in range(min(count, 16)):
        ent.entropy_estimate(mats[i], "chebyshev", m, s, pseed + i, **kw)
        tms.append(ent.last_timing())
    ent.timing_enable(False)
    avg_step_ms = float(np.mean([x["steps_ms"] / x["step_launches"] for x in tms]))
    split = int(tms[-1]["epilogue_launches"]) > 0
    avg_epi_ms = float(np.mean([x["epilogue_ms"] / max(x["epilogue_launches"], 1) for x in tms]))
    step_kernel = "dense_step_split_kernel" if split else "dense_step_kernel"
    flop = 2.0 * n * n * s
    achieved = flop / (avg_step_ms * 1e-3) / 1e12
    peak = MFMA_PEAK_TFLOPS[precision]

    cpu = None
    import oracle

    # the accuracy gate (one matrix under --no-cpu) and the CPU baseline
    idx = [0] if (args.no_cpu or count == 1) else [0, count // 2]
    tc = time.perf_counter()
    errs = []
    for i in idx:
        r = auto[i]
        per = ent.entropy_estimate_detail(mats[i], "auto", m, s, pseed + i, **kw)[1]
        Rh = mats[i].double().cpu().numpy()
        ref = oracle.estimate(Rh, oracle.CHEBYSHEV, r.degree, s, pseed + i, t=t, dist=0,
                              lo=r.lo, u_override=r.u)
        errs.append(float(np.max(np.abs(per - ref.per_probe)) / np.mean(np.abs(ref.per_probe))))
    cpu_s = time.perf_counter() - tc
    max_rel = max(errs)
    if not args.no_cpu:
        cpu = {"value": len(idx) / cpu_s, "unit": "estimates/s", "cores": oracle.max_threads(),
               "kind": "oracle",
               "sample": f"{len(idx)} of {count} held-out matrices at the selector's (m, lo, u), all "
                         f"{s} probes, {cpu_s:.1f} s"}
    log(f"oracle sample: {cpu_s:.1f}s, per-probe rel err vs fp64 oracle {max_rel:.2e}")
    meets = max_rel <= ACC_BAR
    out = {
        "metric": "entropy estimates/s at <=1e-3 rel err",
        "value": (count * 1e3 / ms_auto) if meets else None,
        "unit": "estimates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_auto,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": precision,
        "data": "synthetic",
        "config": {"workload": f"learned degree/cutoff selector on {count} held-out dense density "
                               f"matrices n={n} (power-law / exponential / Dirichlet spectra), "
                               f"s={s} {cfg['dist']} probes, fallback Chebyshev m={m} on [0,u]",
                   "count": count, "n": n, "precision": precision, "parallelism": "single GPU"},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": None, "kernel": step_kernel,
                     "avg_launch_ms": avg_step_ms, "algorithmic_flop_per_launch": flop,
                     "epilogue_avg_launch_ms": avg_epi_ms if split else None},
        "cpu_baseline": cpu,
        "learned_vs_plain": {
            "plain_estimates_per_s": count * 1e3 / ms_plain,
            "products_auto": prod_auto, "products_plain": prod_plain,
            "fallback_rate": fb,
            "routed_to_randproj": int(sum(r.method == ent.RANDPROJ for r in auto)),
            "truncation": trunc,
            "median_rel_err_vs_exact_auto": float(np.median(err_auto)),
            "median_rel_err_vs_exact_plain": float(np.median(err_plain)),
            "mean_rel_err_vs_exact_auto": float(np.mean(err_auto)),
            "mean_rel_err_vs_exact_plain": float(np.mean(err_plain)),
            "per_family_mean_rel_err_auto": [float(np.mean(err_auto[np.array(fams) == f])) for f in range(3)],
            "per_family_mean_rel_err_plain": [float(np.mean(err_plain[np.array(fams) == f])) for f in range(3)],
        },
        "accuracy": {"sampled_matrices": len(idx),
                     "sampled_per_probe_max_rel_err_vs_fp64_oracle": max_rel,
                     "bar": ACC_BAR, "meets_bar": meets},
    }
    print(json.dumps(out), flush=True)
    if not meets:
        sys.exit(3)


def bench_rp(args, cfg):
    """Algorithm 3 on a rank-k dense density matrix, n = 65536 (17.2 GB in
    FP32): sketch R Pi (s columns; Gaussian, subsampled randomized Hadamard or
    input-sparsity), Gram, Jacobi eigenvalues."""
    import torch

    import paper_1801_01072_amd as ent
    import workloads as W

    precision = args.precision or "f32"
    n, k, s = cfg["n"], cfg["k"], cfg["s"]
    mseed, pseed = W.MATRIX_SEED + 5, W.PROBE_SEED + 5
    t0 = time.time()
    pk = W.spectrum_exp(k, cfg["tau"])
    R = W.low_rank_density_torch(pk, n, mseed, device="cuda:0", dtype=torch.float32)
    torch.cuda.synchronize()
    H = float(-np.sum(pk * np.log(pk)))
    log(f"generated rank-{k} R, n={n}, in {time.time() - t0:.1f}s")
    sketch = cfg.get("sketch", "gaussian")
    kw = dict(precision=precision, rank_k=k, sketch_width=s, sketch=sketch)
    for _ in range(args.warmup):
        ent.entropy_estimate(R, "randproj", 1, 1, pseed, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = ent.entropy_estimate(R, "randproj", 1, 1, pseed, **kw)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / args.steps
    ent.timing_enable(True)
    tms = []
    for _ in range(3):
        ent.entropy_estimate(R, "randproj", 1, 1, pseed, **kw)
        tms.append(ent.last_timing())
    ent.timing_enable(False)
    avg_ms = float(np.mean([x["steps_ms"] / max(x["step_launches"], 1) for x in tms]))
    phases = {kk: float(np.mean([x[kk] for x in tms])) for kk in ("total_ms", "steps_ms", "epilogue_ms", "other_ms")}
    if sketch == "count":
        # one pass over R (FP32) plus the s x n FP64 output and the bucket lists
        nbytes = 4.0 * n * n + 8.0 * s * (-(-n // 64) * 64) + 4.0 * n + 8.0 * (s + 1)
        achieved = nbytes / (avg_ms * 1e-3) / 1e9
        kernel = "cs_apply_kernel"
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": kernel,
                "avg_launch_ms": avg_ms, "algorithmic_bytes_per_launch": nbytes}
        log(f"{kernel}: {avg_ms:.3f} ms -> {achieved:.1f} GB/s; H^={res.entropy:.8f}, exact {H:.8f}")
    else:
        flop = 2.0 * n * n * s
        achieved = flop / (avg_ms * 1e-3) / 1e12
        peak = MFMA_PEAK_TFLOPS[precision]
        kernel = "bf16x3_gemm_kernel" if precision == "bf16x3" else "dense_step_kernel"
        roof = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                "frac": achieved / peak, "traffic": None, "kernel": kernel,
                "avg_launch_ms": avg_ms, "algorithmic_flop_per_launch": flop}
        log(f"{kernel}: {avg_ms:.3f} ms -> {achieved:.1f} TFLOP/s; H^={res.entropy:.8f}, exact {H:.8f}")
    del R
    torch.cuda.empty_cache()
    # second spectrum family of the same shape: Dirichlet(0.5) over the k slots
    pd = W.spectrum_dirichlet(k, k, 0.5, np.random.default_rng(mseed))
    Rd = W.low_rank_density_torch(pd, n, mseed + 1, device="cuda:0", dtype=torch.float32)
    res_d = ent.entropy_estimate(Rd, "randproj", 1, 1, pseed, **kw)
    pdp = pd[pd > 0]
    H_d = float(-np.sum(pdp * np.log(pdp)))
    del Rd
    torch.cuda.empty_cache()
    cpu = None
    if not args.no_cpu:
        import oracle

        ns = 8192
        Rs = W.low_rank_density_torch(pk, ns, mseed, device="cpu", dtype=torch.float64).numpy()
        tc = time.perf_counter()
        h_s, _ = oracle.rp_entropy(Rs, s, k, pseed, kind={"gaussian": 0, "srht": 1, "count": 2}[sketch])
        cpu_s = time.perf_counter() - tc
        scale = (n / ns) ** 2
        cpu = {"value": 1.0 / (cpu_s * scale), "unit": "estimates/s", "cores": 1, "kind": "oracle",
               "sample": f"the same estimate at n={ns} ({cpu_s:.1f} s, single-threaded oracle), "
                         f"extrapolated by n^2 (the sketch product dominates)"}
        log(f"oracle at n={ns}: {cpu_s:.1f}s (H^={h_s:.8f})")
    out = {
        "metric": "entropy estimates/s at <=1e-3 rel err",
        "value": 1e3 / ms,
        "unit": "estimates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": precision,
        "data": "synthetic",
        "config": {"workload": f"random projection (Algorithm 3): dense rank-{k} density matrix "
                               f"n={n}, p ~ exp(-i/{cfg['tau']:g}), {sketch} sketch width {s}",
                   "n": n, "rank_k": k, "sketch_width": s, "sketch": sketch, "precision": precision,
                   "parallelism": "single GPU"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "phases_ms": phases,
        "accuracy": {"entropy": res.entropy, "exact_H": H, "rel_err_vs_exact": (res.entropy - H) / H,
                     "dirichlet_entropy": res_d.entropy, "dirichlet_exact_H": H_d,
                     "dirichlet_rel_err_vs_exact": (res_d.entropy - H_d) / H_d},
    }
    print(json.dumps(out), flush=True)


def bench_copy(args, cfg):
    import torch

    nb = cfg["nbytes"]
    src = torch.ones(nb // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(args.warmup):
        dst.copy_(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        dst.copy_(src)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / args.steps
    gbs = 2 * nb / (ms * 1e-3) / 1e9
    print(json.dumps({"metric": "device copy GB/s (read + write)", "value": gbs, "unit": "GB/s",
                      "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
                      "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                      "dtype": "f32", "data": "synthetic",
                      "config": {"workload": f"device copy of {nb} bytes", "bytes": nb},
                      "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS,
                                   "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS, "traffic": None},
                      "cpu_baseline": None}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="dense8192", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default=None, choices=["f64", "f32", "bf16x3"])
    ap.add_argument("--store", default=None, choices=["f64", "f32"])
    ap.add_argument("--cpu-probes", type=int, default=0, help="oracle sample size (0 = host threads)")
    ap.add_argument("--no-cpu", action="store_true",
                    help="no CPU baseline (the accuracy gate still checks 2 sampled probes)")
    ap.add_argument("--no-compare", action="store_true",
                    help="dense workloads: time only the headline precision")
    ap.add_argument("--csr-general", action="store_true",
                    help="CSR workloads: the general CSR step kernel even for banded R")
    ap.add_argument("--count", type=int, default=0, help="matrices in the learned4096 workload")
    ap.add_argument("--batch-stepwise", action="store_true",
                    help="batch workloads: one grouped launch per recurrence step instead of the "
                         "persistent schedule")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (the estimator "
              "would shard over probes with one all-reduce of the moment partials)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1801_01072_amd as ent
    import workloads as W

    cfg = WORKLOADS[args.workload]
    if cfg["kind"] == "batch":
        return bench_batch(args, cfg)
    if cfg["kind"] == "learned":
        return bench_learned(args, cfg)
    if cfg["kind"] == "rp":
        return bench_rp(args, cfg)
    if cfg["kind"] == "copy":
        return bench_copy(args, cfg)
    return bench_single(args, cfg)


# accuracy bar of the metric: per-probe values within 1e-3 relative of the
# FP64 oracle on the sampled probes
ACC_BAR = 1e-3


def time_estimates(ent, Rd, cfg, pseed, kw, steps, warmup):
    """Warm-up, then `steps` timed estimates bracketed by device synchronisations;
    returns (ms per estimate, last result)."""
    import torch

    m, s = cfg["m"], cfg["s"]
    for _ in range(warmup):
        ent.entropy_estimate(Rd, cfg["method"], m, s, pseed, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        res = ent.entropy_estimate(Rd, cfg["method"], m, s, pseed, **kw)
    torch.cuda.synchronize()
    return 1e3 * (time.perf_counter() - t0) / steps, res


def kernel_timing(ent, Rd, cfg, pseed, kw, reps):
    """Per-launch durations of the recurrence product kernel from the HIP events
    the library records on its own stream (phase timing)."""
    ent.timing_enable(True)
    tms = []
    for _ in range(reps):
        ent.entropy_estimate(Rd, cfg["method"], cfg["m"], cfg["s"], pseed, **kw)
        tms.append(ent.last_timing())
    ent.timing_enable(False)
    avg_step_ms = float(np.mean([x["steps_ms"] / x["step_launches"] for x in tms]))
    avg_epi_ms = float(np.mean([x["epilogue_ms"] / max(x["epilogue_launches"], 1) for x in tms]))
    phases = {k: float(np.mean([x[k] for x in tms])) for k in ("total_ms", "power_ms", "steps_ms",
                                                               "epilogue_ms", "other_ms")}
    return avg_step_ms, avg_epi_ms, phases, tms[-1]


def bench_single(args, cfg):
    """One density matrix: dense (real or Hermitian) or CSR.  Dense workloads
    time the paper's arithmetic (FP64) for the headline and, unless a precision
    is forced, the same estimate in FP32 and BF16x3 beside it."""
    import torch

    import paper_1801_01072_amd as ent
    import workloads as W

    herm = cfg["kind"] == "herm"
    dense = cfg["kind"] in ("dense", "herm")
    precision = args.precision or ("f64" if dense else "f32")
    compare = [] if (args.precision or not dense or args.no_compare) else ["f32", "bf16x3"]
    if herm:
        store = "c64" if args.store == "f32" else "c128"
    else:
        store = args.store or ("f64" if dense else ("f32" if precision != "f64" else "f64"))
    n, m, s, t = cfg["n"], cfg["m"], cfg["s"], cfg["t"]
    mseed, pseed = W.MATRIX_SEED + 2, W.PROBE_SEED + 2
    t0 = time.time()
    H_exact = None
    if herm:
        p = W.spectrum_exp(n, cfg["spectrum"][1])
        cdt = torch.complex64 if store == "c64" else torch.complex128
        try:
            Rd = W.hermitian_density_torch(p, mseed, device="cuda:0", dtype=cdt)
        except RuntimeError as e:  # a device QR this torch build lacks: build it on the host
            log(f"device QR unavailable ({str(e)[:60]}); building R on the host")
            Rd = torch.from_numpy(W.hermitian_density(p, mseed)).to("cuda:0").to(cdt)
        H_exact = float(-np.sum(p * np.log(p)))
        host_R = None
    elif dense:
        sp = cfg["spectrum"]
        p = W.spectrum_inverse(n) if sp[0] == "inverse" else W.spectrum_exp(n, sp[1])
        R = W.dense_density(p, mseed)
        if store == "f32":
            R = R.astype(np.float32)
        H_exact = float(-np.sum(p[p > 0] * np.log(p[p > 0])))
        Rd = torch.from_numpy(R).to("cuda:0")
        host_R = R
    elif cfg.get("matrix") == "poisson":
        Rd = W.poisson_csr_torch(n, device="cuda:0", dtype=torch.float64 if store == "f64" else torch.float32)
        lam = W.poisson_eigenvalues(n)
        H_exact = float(-np.sum(lam * np.log(lam)))
        del lam
        host_R = None
    else:
        csr = W.banded_density_csr(n, cfg["hb"], seed=mseed, dtype=np.float64 if store == "f64" else np.float32)
        Rd = tuple(torch.from_numpy(a).to("cuda:0") for a in csr[:3]) + (n,)
        host_R = csr
    torch.cuda.synchronize()
    log(f"generated R ({args.workload}, {store}) in {time.time() - t0:.1f}s")
    base_kw = dict(probe_dist=cfg["dist"], power_iters=t, u_factor=cfg.get("c", 6.0))
    if herm:
        base_kw["flags"] = ent.FLAG_COMPLEX_POWER
    if getattr(args, "csr_general", False):
        base_kw["flags"] = base_kw.get("flags", 0) | ent.FLAG_CSR_GENERAL
    kw = dict(base_kw, precision=precision)

    ms_per_step, res = time_estimates(ent, Rd, cfg, pseed, kw, args.steps, args.warmup)
    log(f"timed {args.steps} estimates ({precision}): {ms_per_step:.3f} ms/estimate, H^={res.entropy:.12f}")
    avg_step_ms, avg_epi_ms, phases, last_t = kernel_timing(ent, Rd, cfg, pseed, kw, max(3, min(args.steps, 10)))
    launches = last_t["step_launches"]
    if dense:
        # FP32/FP64: the split-K form runs when the tile grid is small (its
        # product kernel, with the split reduction in a separate epilogue)
        split = precision != "bf16x3" and int(last_t["epilogue_launches"]) > 0
        kernel = ("bf16x3_gemm_kernel" if precision == "bf16x3" else
                  ("dense_step_split_kernel" if split else "dense_step_kernel"))
        # a complex n x n by n x s product is 8 n^2 s real flops (the real 2n x 2n form)
        flop = (8.0 if herm else 2.0) * n * n * s
        achieved = flop / (avg_step_ms * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": MFMA_PEAK_TFLOPS[precision],
                "unit": "TFLOP/s", "frac": achieved / MFMA_PEAK_TFLOPS[precision],
                "traffic": measured_traffic(kernel, args.workload + ("" if precision == "bf16x3" else "_" + precision)),
                "kernel": kernel, "avg_launch_ms": avg_step_ms, "algorithmic_flop_per_launch": flop}
        if precision == "bf16x3":
            roof["executed_tflops"] = 3 * achieved
        if precision == "bf16x3" or split:
            roof["epilogue_avg_launch_ms"] = avg_epi_ms
        log(f"{kernel}: {avg_step_ms:.4f} ms/launch over {launches} launches -> {achieved:.2f} TFLOP/s")
    else:
        nnz = int(Rd[0][-1]) if host_R is None else int(host_R[0][-1])
        vb = 8 if precision == "f64" else 4
        hp = int(last_t["csr_band"])
        if hp == 1 and int(last_t["steps_fused"]) >= 2:
            # tridiagonal input, several steps per launch
            kernel = "tri_fused_kernel"
            tot_bytes, steps = tri_fused_bytes(n, s, m, vb, cfg["method"], int(last_t["steps_fused"]))
        elif hp == 1:
            # tridiagonal input: the three-row stencil kernel
            kernel = "tri_step_kernel"
            tot_bytes, steps = tri_step_bytes(n, s, m, vb, cfg["method"])
        elif hp > 0 and int(last_t["steps_fused"]) == 2:
            # banded input, two steps per launch
            kernel = "band_pair_kernel"
            tot_bytes, steps = band_pair_bytes(n, hp, s, m, vb, cfg["method"])
        elif hp > 0:
            # banded input: the step ran on the 16-row slabs
            kernel = "band_step_kernel"
            tot_bytes, steps = band_step_bytes(n, hp, s, m, vb, cfg["method"])
        else:
            kernel = "csr_step_kernel"
            tot_bytes, steps = csr_step_bytes(n, nnz, s, m, vb, cfg["method"])
        per_launch = tot_bytes / steps
        achieved = per_launch / (avg_step_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS,
                "traffic": measured_traffic(kernel, args.workload + ("" if precision == "f32" else "_" + precision)),
                "kernel": kernel, "band_half_width": hp,
                "avg_launch_ms": avg_step_ms, "algorithmic_bytes_per_launch": per_launch}
        log(f"{kernel}: {avg_step_ms:.4f} ms/launch -> {achieved:.1f} GB/s")
    log(f"phases (ms): {phases}")
    gpu_res, per, _ = ent.entropy_estimate_detail(Rd, cfg["method"], m, s, pseed, **kw)

    # the other precision forms of the same estimate (same matrix, probes, seed)
    forms = {}
    for prec in compare:
        kwp = dict(base_kw, precision=prec)
        ms_p, _ = time_estimates(ent, Rd, cfg, pseed, kwp, args.steps, args.warmup)
        st_ms, epi_ms, ph, _ = kernel_timing(ent, Rd, cfg, pseed, kwp, 3)
        r_p, per_p, _ = ent.entropy_estimate_detail(Rd, cfg["method"], m, s, pseed, **kwp)
        k_p = ("bf16x3_gemm_kernel" if prec == "bf16x3" else
               ("dense_step_split_kernel" if epi_ms > 0 else "dense_step_kernel"))
        flop = (8.0 if herm else 2.0) * n * n * s
        ach = flop / (st_ms * 1e-3) / 1e12
        forms[prec] = {"value": 1e3 / ms_p, "unit": "estimates/s", "ms_per_step": ms_p,
                       "speedup_vs_f64": ms_per_step / ms_p if precision == "f64" else None,
                       "entropy": r_p.entropy,
                       "rel_err_vs_exact": abs(r_p.entropy - H_exact) / H_exact if H_exact else None,
                       "kernel": k_p, "avg_launch_ms": st_ms, "achieved_tflops": ach,
                       "frac": ach / MFMA_PEAK_TFLOPS[prec],
                       "traffic": measured_traffic(k_p, args.workload + ("" if prec == "bf16x3" else "_" + prec)),
                       "epilogue_avg_launch_ms": epi_ms if epi_ms > 0 else None,
                       "phases_ms": ph, "_per_probe": per_p}
        log(f"{prec}: {ms_p:.3f} ms/estimate ({1e3 / ms_p:.2f} est/s, {ms_per_step / ms_p:.2f}x the "
            f"{precision} path); {k_p} {st_ms:.4f} ms/launch -> {ach:.1f} TFLOP/s")

    # the FP64 oracle on sampled probes of the same estimate: the accuracy gate
    # of every form, and (unless --no-cpu) the CPU baseline
    import oracle

    threads = oracle.max_threads()
    nsamp = 2 if args.no_cpu else min(args.cpu_probes or cfg.get("cpu_probes") or threads, s)
    if host_R is None and not herm:
        host_R = tuple(a.cpu().numpy() for a in Rd[:3]) + (n,)
    probes = [int(x) for x in np.linspace(0, s - 1, nsamp).astype(int)]
    meth = oracle.CHEBYSHEV if cfg["method"] == "chebyshev" else oracle.TAYLOR
    dist = 1 if cfg["dist"] == "gaussian" else 0
    if herm:
        host_R = Rd.cpu().numpy()
        tc = time.perf_counter()
        ref = oracle.zestimate(host_R, meth, m, s, pseed, t=t, dist=dist, u_override=0.0, probes=probes)
        cpu_s = time.perf_counter() - tc
        tp = time.perf_counter()
        oracle.zpower_method(host_R, t, 1, pseed)
        power_s = time.perf_counter() - tp
    else:
        tc = time.perf_counter()
        ref = oracle.estimate(host_R, meth, m, s, pseed, t=t, dist=dist, probes=probes, c=cfg.get("c", 6.0))
        cpu_s = time.perf_counter() - tc
        tp = time.perf_counter()
        oracle.power_method(host_R, t, 1, pseed)
        power_s = time.perf_counter() - tp
    scale = np.mean(np.abs(ref.per_probe))
    max_rel = float(np.max(np.abs(per[probes] - ref.per_probe)) / scale)
    log(f"oracle: power method + {nsamp} probes in {cpu_s:.2f}s on {threads} threads; "
        f"sampled per-probe rel err ({precision}) {max_rel:.2e}")
    for prec, f in forms.items():
        pp = f.pop("_per_probe")
        f["sampled_per_probe_max_rel_err_vs_fp64_oracle"] = float(np.max(np.abs(pp[probes] - ref.per_probe)) / scale)
        f["meets_bar"] = f["sampled_per_probe_max_rel_err_vs_fp64_oracle"] <= ACC_BAR
        log(f"{prec}: sampled per-probe rel err {f['sampled_per_probe_max_rel_err_vs_fp64_oracle']:.2e}")
    cpu = None
    if not args.no_cpu:
        per_round = max(cpu_s - power_s, 1e-9)
        rounds = int(np.ceil(s / nsamp))
        est_s = power_s + rounds * per_round
        cpu = {"value": 1.0 / est_s, "unit": "estimates/s", "cores": min(threads, nsamp), "kind": "oracle",
               "sample": f"power method + {nsamp} of {s} probes of the same estimate "
                         f"({cpu_s:.1f} s), extrapolated to {s} probes ({rounds} rounds of {nsamp})"}
    meets = max_rel <= ACC_BAR
    if not meets:
        log(f"accuracy bar missed: sampled per-probe error {max_rel:.3e} > {ACC_BAR:g}; no value reported")

    out = {
        "metric": "entropy estimates/s at <=1e-3 rel err",
        "value": (1e3 / ms_per_step) if meets else None,
        "unit": "estimates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": precision,
        "data": "synthetic",
        "config": {"workload": describe(cfg, precision, store), "n": n, "degree": m, "probes": s,
                   "method": cfg["method"], "precision": precision, "storage": store,
                   "parallelism": "single GPU"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "phases_ms": phases,
        "accuracy": {"entropy": gpu_res.entropy, "std_err": gpu_res.std_err, "exact_H": H_exact,
                     "rel_err_vs_exact": (abs(gpu_res.entropy - H_exact) / H_exact) if H_exact else None,
                     "sampled_probes": len(probes),
                     "sampled_per_probe_max_rel_err_vs_fp64_oracle": max_rel,
                     "bar": ACC_BAR, "meets_bar": meets},
    }
    if forms:
        out["precision_forms"] = forms
    print(json.dumps(out), flush=True)
    if not meets:
        sys.exit(3)


if __name__ == "__main__":
    main()
