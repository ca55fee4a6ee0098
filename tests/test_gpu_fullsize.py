"""The benchmark's headline configurations at full size, with the inputs,
launch configuration and options bench.py times: per-probe values of a
sample of probes against the FP64 oracle (which computes them one by one),
and properties that hold at any size."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1801_01072_amd as ent  # noqa: E402

DEV = "cuda:0"
NSAMP = 8


def sampled_rel(per, probes, ref):
    return float(np.max(np.abs(per[probes] - ref.per_probe)) / np.mean(np.abs(ref.per_probe)))


def test_dense_n8192_bf16x3(orc):
    # n = 8192, p_i ~ exp(-i/1000), Chebyshev m = 50, s = 256 Gaussian probes,
    # t = 20, BF16x3 products of an FP64-stored R
    n, m, s, t = 8192, 50, 256, 20
    p = W.spectrum_exp(n, 1000.0)
    R = W.dense_density(p, W.MATRIX_SEED + 2)
    seed = W.PROBE_SEED + 2
    res, per, _ = ent.entropy_estimate_detail(torch.from_numpy(R).to(DEV), "chebyshev", m, s, seed,
                                              precision="bf16x3", probe_dist="gaussian", power_iters=t)
    probes = [int(x) for x in np.linspace(0, s - 1, NSAMP).astype(int)]
    ref = orc.estimate(R, 1, m, s, seed, t=t, dist=1, probes=probes)
    err = sampled_rel(per, probes, ref)
    H = float(-np.sum(p * np.log(p)))
    print(f"[dense 8192 bf16x3] sampled per-probe rel {err:.2e}; H^={res.entropy:.6f} H={H:.6f} "
          f"se={res.std_err:.2e}; p1 rel {abs(res.p1_est - ref.p1_est) / ref.p1_est:.2e}", flush=True)
    assert err <= 1e-3
    assert res.p1_est == pytest.approx(ref.p1_est, rel=1e-6)
    # the estimator's own error: within a few standard errors of the exact H
    assert abs(res.entropy - H) <= 5 * res.std_err


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
    assert err <= 1e-3
    assert res.p1_est == pytest.approx(ref.p1_est, rel=1e-10)
    assert res.std_err > 0 and np.all(np.isfinite(per))


def test_batch_1024_matrices_f32(orc):
    # 1024 dense density matrices, n ~ U[64, 2048], rank k ~ U[n/8, n],
    # Dirichlet spectra, Chebyshev m = 40, s = 64 Rademacher probes, t = 20,
    # FP32, one captured graph with the tile autotuner: four matrices spread
    # over the sizes against the oracle (all probes), replays bit-identical
    count, m, s, t = 1024, 40, 64, 20
    mseed, pseed = W.MATRIX_SEED + 4, W.PROBE_SEED + 4
    ns, ks = W.batch_shapes(count, mseed, 64, 2048)
    spectra = W.batch_spectra(ns, ks, mseed)
    mats = [W.dense_density_torch(p, mseed * 7 + i, device=DEV, dtype=torch.float32) for i, p in enumerate(spectra)]
    torch.cuda.synchronize()
    g = ent.Graph(mats, "chebyshev", m, s, pseed, precision="f32", probe_dist="rademacher", power_iters=t,
                  flags=ent.FLAG_AUTOTUNE)
    res = g.launch()
    per = g.per_probe()
    res2 = g.launch()
    assert [r.entropy for r in res] == [r.entropy for r in res2]
    assert np.all(np.isfinite(per))
    idx = [int(i) for i in np.argsort(ns)[np.linspace(0, count - 1, 4).astype(int)]]
    for b in idx:
        Rh = mats[b].double().cpu().numpy()
        ref = orc.estimate(Rh, 1, m, s, pseed + b, t=t, dist=0)
        err = float(np.max(np.abs(per[b] - ref.per_probe)) / np.mean(np.abs(ref.per_probe)))
        print(f"[batch 1024] matrix {b} (n = {ns[b]}): per-probe rel {err:.2e}", flush=True)
        assert err <= 1e-3
