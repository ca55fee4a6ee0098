"""The configurations at full size, with the inputs, launch configuration and
options bench.py times: per-probe values of a sample of probes against the
FP64 oracle (which computes them one by one), and properties that hold at any
size.

* dense n = 8192 (Chebyshev m = 50, s = 256 Gaussian probes, t = 20) in FP64,
  FP32 and BF16x3 against one oracle sample of 8 probes;
* banded CSR n = 10^7 in FP32;
* the 1024-matrix batch in FP32 and BF16x3 (four matrices spread over the
  sizes, all probes);
* random projection at n = 65536, rank 64, sketch width 128 (Algorithm 3):
  the singular values of R Pi equal those of diag(p) Q^T Pi when R = Q diag(p)
  Q^T with orthonormal Q, a 64 x 128 problem the oracle solves from the same
  Philox sketch;
* the learned selector on 512 held-out dense n = 4096 matrices.
"""
import math

import numpy as np
import pytest

import workloads as W
from tolerances import TOL64, TOL_BF16X3, TOL_F32, tol_for

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1801_01072_amd as ent  # noqa: E402

DEV = "cuda:0"
NSAMP = 8


def sampled_rel(per, probes, ref):
    return float(np.max(np.abs(per[probes] - ref.per_probe)) / np.mean(np.abs(ref.per_probe)))


# ------------------------------------------------------ dense n = 8192 ----
@pytest.fixture(scope="module")
def dense8192(orc):
    n, m, s, t = 8192, 50, 256, 20
    p = W.spectrum_exp(n, 1000.0)
    R = W.dense_density(p, W.MATRIX_SEED + 2)
    seed = W.PROBE_SEED + 2
    probes = [int(x) for x in np.linspace(0, s - 1, NSAMP).astype(int)]
    ref = orc.estimate(R, 1, m, s, seed, t=t, dist=1, probes=probes)
    return dict(n=n, m=m, s=s, t=t, p=p, R=R, Rd=torch.from_numpy(R).to(DEV), seed=seed, probes=probes,
                ref=ref)


@pytest.mark.parametrize("precision,tol,p1_tol", [("f64", TOL64, 1e-12), ("f32", TOL_F32, 1e-6),
                                                  ("bf16x3", TOL_BF16X3, 1e-6)])
def test_dense_n8192(dense8192, precision, tol, p1_tol):
    d = dense8192
    res, per, _ = ent.entropy_estimate_detail(d["Rd"], "chebyshev", d["m"], d["s"], d["seed"],
                                              precision=precision, probe_dist="gaussian", power_iters=d["t"])
    err = sampled_rel(per, d["probes"], d["ref"])
    H = float(-np.sum(d["p"] * np.log(d["p"])))
    print(f"[dense 8192 {precision}] sampled per-probe rel {err:.2e}; H^={res.entropy:.6f} H={H:.6f} "
          f"se={res.std_err:.2e}; p1 rel {abs(res.p1_est - d['ref'].p1_est) / d['ref'].p1_est:.2e}", flush=True)
    assert err <= tol
    assert res.p1_est == pytest.approx(d["ref"].p1_est, rel=p1_tol)
    # the estimator's own error: within a few standard errors of the exact H
    assert abs(res.entropy - H) <= 5 * res.std_err


# --------------------------------------------------- banded n = 10^7 ----
def test_csr_n1e7_f32(orc):
    # banded CSR R of order 10^7 (nnz = 33n - 272), Chebyshev m = 40, s = 64
    # Rademacher probes, t = 20, FP32 values and products
    n, m, s, t = 10_000_000, 40, 64, 20
    csr = W.banded_density_csr(n, 8, seed=W.MATRIX_SEED + 2, dtype=np.float32)
    seed = W.PROBE_SEED + 2
    Rd = tuple(torch.from_numpy(a).to(DEV) for a in csr[:3]) + (n,)
    res, per, _ = ent.entropy_estimate_detail(Rd, "chebyshev", m, s, seed, precision="f32",
                                              probe_dist="rademacher", power_iters=t)
    probes = [int(x) for x in np.linspace(0, s - 1, NSAMP).astype(int)]
    ref = orc.estimate(csr, 1, m, s, seed, t=t, dist=0, probes=probes)
    err = sampled_rel(per, probes, ref)
    print(f"[csr 1e7 f32] sampled per-probe rel {err:.2e}; H^={res.entropy:.8f} se={res.std_err:.2e}; "
          f"p1 rel {abs(res.p1_est - ref.p1_est) / ref.p1_est:.2e}", flush=True)
    assert err <= TOL_F32
    assert res.p1_est == pytest.approx(ref.p1_est, rel=1e-10)
    assert res.std_err > 0 and np.all(np.isfinite(per))


# ------------------------------------------------- 1024-matrix batch ----
@pytest.fixture(scope="module")
def batch1024():
    count, m, s, t = 1024, 40, 64, 20
    mseed, pseed = W.MATRIX_SEED + 4, W.PROBE_SEED + 4
    ns, ks = W.batch_shapes(count, mseed, 64, 2048)
    spectra = W.batch_spectra(ns, ks, mseed)
    mats = [W.dense_density_torch(p, mseed * 7 + i, device=DEV, dtype=torch.float32) for i, p in enumerate(spectra)]
    torch.cuda.synchronize()
    idx = [int(i) for i in np.argsort(ns)[np.linspace(0, count - 1, 4).astype(int)]]
    return dict(count=count, m=m, s=s, t=t, pseed=pseed, ns=ns, mats=mats, idx=idx, refs={})


@pytest.mark.parametrize("precision", ["f32", "bf16x3"])
def test_batch_1024_matrices(orc, batch1024, precision):
    # 1024 dense density matrices, n ~ U[64, 2048], rank k ~ U[n/8, n],
    # Dirichlet spectra, Chebyshev m = 40, s = 64 Rademacher probes, t = 20,
    # one captured graph (FP32 with the tile autotuner): four matrices spread
    # over the sizes against the oracle (all probes), replays bit-identical
    b_ = batch1024
    m, s, t, pseed = b_["m"], b_["s"], b_["t"], b_["pseed"]
    g = ent.Graph(b_["mats"], "chebyshev", m, s, pseed, precision=precision, probe_dist="rademacher",
                  power_iters=t, flags=ent.FLAG_AUTOTUNE)
    res = g.launch()
    per = g.per_probe()
    res2 = g.launch()
    g.destroy()
    assert [r.entropy for r in res] == [r.entropy for r in res2]
    assert np.all(np.isfinite(per))
    for b in b_["idx"]:
        if b not in b_["refs"]:
            Rh = b_["mats"][b].double().cpu().numpy()
            b_["refs"][b] = orc.estimate(Rh, 1, m, s, pseed + b, t=t, dist=0)
        ref = b_["refs"][b]
        err = float(np.max(np.abs(per[b] - ref.per_probe)) / np.mean(np.abs(ref.per_probe)))
        print(f"[batch 1024 {precision}] matrix {b} (n = {b_['ns'][b]}): per-probe rel {err:.2e}", flush=True)
        assert err <= tol_for(precision)


# ------------------------------------ random projection, n = 65536 ----
@pytest.mark.parametrize("precision,tol", [("f64", 1e-9), ("f32", TOL_F32)])
def test_randproj_n65536(orc, precision, tol):
    n, k, s = 65536, 64, 128
    mseed, seed = W.MATRIX_SEED + 5, W.PROBE_SEED + 5
    pk = W.spectrum_exp(k, 8.0)
    # R = Q diag(p) Q^T with Q the sign-fixed Q factor of a seeded n x k
    # Gaussian (the construction of the workload generator)
    g = torch.Generator(device="cpu").manual_seed(mseed)
    Z = torch.randn((n, k), generator=g, dtype=torch.float64).to(DEV)
    Q, Rr = torch.linalg.qr(Z)
    Q = Q * torch.sign(torch.diagonal(Rr))[None, :]
    B = Q * torch.sqrt(torch.as_tensor(pk, dtype=torch.float64, device=DEV))[None, :]
    R = (B @ B.T).to(torch.float64 if precision == "f64" else torch.float32).contiguous()
    del B, Z
    res, sig, _ = ent.entropy_estimate_detail(R, "randproj", 1, 1, seed, rank_k=k, sketch_width=s,
                                              precision=precision)
    del R
    torch.cuda.empty_cache()
    # oracle: sigma(R Pi) = sigma(diag(p) Q^T Pi), Pi the same Philox sketch
    Pi = orc.sketch_matrix(orc.SKETCH_GAUSSIAN, seed, n, s)
    QtPi = Q.cpu().numpy().T @ Pi
    h_ref, sig_ref = orc.rp_entropy_with_pi(np.diag(pk), QtPi, k)
    serr = float(np.max(np.abs(sig - sig_ref)) / np.max(sig_ref))
    herr = abs(res.entropy - h_ref) / abs(h_ref)
    H = float(-np.sum(pk * np.log(pk)))
    print(f"[rp 65536 {precision}] sigma rel {serr:.2e}, H^ rel {herr:.2e}; H^={res.entropy:.8f} exact H={H:.8f}",
          flush=True)
    assert serr <= tol and herr <= tol


# ---------------------------------------- learned selector, 512 held-out ----
def test_learned_selector_512_heldout(orc):
    # the held-out set of the learned configuration: 512 dense n = 4096
    # density matrices of the training families from a seed the training
    # never used (eight Haar-random eigenbases, one per 64 matrices), FP32,
    # s = 64 Rademacher probes, fallback Chebyshev m = 40 on [0, u]
    from paper_1801_01072_amd import learned as L

    ent.selector_load(L.load())
    n, m, s, count = 4096, 40, 64, 512
    mseed, pseed = W.MATRIX_SEED + 5, W.PROBE_SEED + 5
    rng = np.random.default_rng(mseed + 10**6)
    spectra, fams = zip(*[L.sample_spectrum(rng, n) for _ in range(count)])
    bases = []
    for b in range(8):
        gen = torch.Generator(device="cpu").manual_seed(mseed * 11 + b)
        Qb, Rr = torch.linalg.qr(torch.randn((n, n), generator=gen, dtype=torch.float64).to(DEV))
        bases.append(Qb * torch.sign(torch.diagonal(Rr))[None, :])
    auto, plain = [], []
    for i, p in enumerate(spectra):
        Qb = bases[i // 64]
        pt = torch.as_tensor(p, dtype=torch.float64, device=DEV)
        R = ((Qb * pt[None, :]) @ Qb.T)
        R = (0.5 * (R + R.T)).to(torch.float32).contiguous()
        a = ent.entropy_estimate_detail(R, "auto", m, s, pseed + i, precision="f32")
        pl = ent.entropy_estimate(R, "chebyshev", m, s, pseed + i, precision="f32")
        auto.append(a)
        plain.append(pl)
        if i in (0, 1, 2, 3) or (a[0].fell_back and not any(x[0].fell_back for x in auto[:-1])):
            # sampled probes against the oracle at the selector's (m, lo, u)
            Rh = R.double().cpu().numpy()
            sel = [0, s - 1]
            ref = orc.estimate(Rh, 1, a[0].degree, s, pseed + i, dist=0, lo=a[0].lo, u_override=a[0].u,
                               probes=sel)
            err = float(np.max(np.abs(a[1][sel] - ref.per_probe)) / np.mean(np.abs(ref.per_probe)))
            print(f"[learned {i}] family {fams[i]} m={a[0].degree} lo={a[0].lo:.3e} "
                  f"fell_back={a[0].fell_back} per-probe rel {err:.2e}", flush=True)
            assert err <= TOL_F32
    H = np.array([float(-np.sum(p[p > 0] * np.log(p[p > 0]))) for p in spectra])
    ea = np.array([abs(a[0].entropy - h) / h for a, h in zip(auto, H)])
    ep = np.array([abs(r.entropy - h) / h for r, h in zip(plain, H)])
    fb = float(np.mean([a[0].fell_back for a in auto]))
    prod_a = sum(a[0].products for a in auto)
    prod_p = sum(r.products for r in plain)
    print(f"[learned 512] fallback rate {fb:.3f}; products auto {prod_a} plain {prod_p}; median rel err vs "
          f"exact auto {np.median(ea):.2e} plain {np.median(ep):.2e}", flush=True)
    assert all(math.isfinite(a[0].entropy) for a in auto)
    assert all(a[0].fell_back or a[0].degree >= 4 for a in auto)
