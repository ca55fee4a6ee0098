"""Random-projection estimator (Algorithm 3) on the GPU against the FP64
oracle with the same Gaussian sketch (Philox stream 2)."""
import numpy as np
import pytest

import workloads as W
from tolerances import tol_for

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1801_01072_amd as ent  # noqa: E402

DEV = "cuda:0"


def low_rank(n, k, seed, tau=3.0):
    p = np.zeros(n)
    p[:k] = W.spectrum_exp(k, tau)
    return W.dense_density(p, seed), p


@pytest.mark.parametrize("n,k,s", [(600, 10, 64), (257, 7, 33), (1000, 40, 128), (130, 5, 5), (300, 12, 200),
                                   (400, 30, 256)])
def test_randproj_fp64_parity(orc, n, k, s):
    R, p = low_rank(n, k, 40 + n)
    seed = 3
    res, sig, _ = ent.entropy_estimate_detail(torch.from_numpy(R).to(DEV), "randproj", 1, 1, seed,
                                              rank_k=k, sketch_width=s, precision="f64")
    h_ref, sig_ref = orc.rp_entropy(R, s, k, seed)
    print(f"[rp f64 n={n} k={k} s={s}] H gpu={res.entropy:.14f} oracle={h_ref:.14f}", flush=True)
    assert res.entropy == pytest.approx(h_ref, rel=1e-10)
    # sigma = sqrt(lambda): an FP64 eigenvalue error ~ eps * lambda_max gives the
    # small singular values an absolute error ~ 1e-11 sigma_max
    assert np.allclose(sig, sig_ref, rtol=1e-9, atol=1e-10 * sig_ref.max())


@pytest.mark.parametrize("precision", ["f32", "bf16x3"])
def test_randproj_reduced_precision(orc, precision):
    n, k, s = 1024, 16, 64
    R, p = low_rank(n, k, 7)
    res, sig, _ = ent.entropy_estimate_detail(torch.from_numpy(R).to(DEV), "randproj", 1, 1, 5,
                                              rank_k=k, sketch_width=s, precision=precision)
    h_ref, sig_ref = orc.rp_entropy(R, s, k, 5)
    rel = abs(res.entropy - h_ref) / h_ref
    serr = float(np.max(np.abs(sig - sig_ref)) / np.max(sig_ref))
    print(f"[rp {precision}] H gpu={res.entropy:.10f} oracle={h_ref:.10f} rel={rel:.2e} sigma={serr:.2e}",
          flush=True)
    assert rel <= tol_for(precision) and serr <= tol_for(precision)


def test_randproj_orthonormal_limit_and_errors():
    # with s >= n every singular value of R Pi ~ p (Gaussian Pi), so H^ ~ H
    n, k = 64, 4
    R, p = low_rank(n, k, 9, tau=1.5)
    H = float(-np.sum(p[:k] * np.log(p[:k])))
    res = ent.entropy_estimate(torch.from_numpy(R).to(DEV), "randproj", 1, 1, 1, rank_k=k,
                               sketch_width=256, precision="f64")
    assert abs(res.entropy - H) / H < 0.1
    with pytest.raises(ent.EntropyError):
        ent.entropy_estimate(torch.from_numpy(R).to(DEV), "randproj", 1, 1, 1, rank_k=10, sketch_width=5)
    with pytest.raises(ent.EntropyError):
        ent.entropy_estimate(torch.from_numpy(R).to(DEV), "randproj", 1, 1, 1, rank_k=2, sketch_width=300)


KINDS = {"srht": 1, "count": 2}


@pytest.mark.parametrize("sketch", ["srht", "count"])
@pytest.mark.parametrize("n,k,s", [(600, 10, 64), (257, 7, 33), (1000, 8, 128), (1, 1, 3)])
def test_structured_sketch_fp64_parity(orc, sketch, n, k, s):
    R, p = low_rank(n, k, 50 + n) if n > 1 else (np.ones((1, 1)), np.ones(1))
    seed = 4
    res, sig, _ = ent.entropy_estimate_detail(torch.from_numpy(R).to(DEV), "randproj", 1, 1, seed,
                                              rank_k=k, sketch_width=s, precision="f64", sketch=sketch)
    h_ref, sig_ref = orc.rp_entropy(R, s, k, seed, kind=KINDS[sketch])
    print(f"[rp {sketch} f64 n={n} k={k} s={s}] H gpu={res.entropy:.14f} oracle={h_ref:.14f}", flush=True)
    assert res.entropy == pytest.approx(h_ref, rel=1e-10, abs=1e-14)
    assert np.allclose(sig, sig_ref, rtol=1e-9, atol=1e-10 * max(sig_ref.max(), 1e-300))


def test_count_sketch_f32_storage_and_exact_recovery(orc):
    # FP32 storage: the same stored values summed in FP64 on both sides
    n, k, s = 700, 6, 64
    R, p = low_rank(n, k, 3)
    R32 = R.astype(np.float32)
    res, sig, _ = ent.entropy_estimate_detail(torch.from_numpy(R32).to(DEV), "randproj", 1, 1, 8,
                                              rank_k=k, sketch_width=s, sketch="count")
    h_ref, sig_ref = orc.rp_entropy(R32, s, k, 8, kind=2)
    assert res.entropy == pytest.approx(h_ref, rel=1e-9)
    # diag(p) on rows that fall into distinct buckets: R Pi has orthogonal rows, exact spectrum
    n, s, seed = 300, 64, 2
    rows, used = [], set()
    for j in range(n):
        b = orc.sketch_bucket(seed, j, s)
        if b not in used:
            used.add(b)
            rows.append(j)
        if len(rows) == 5:
            break
    q = np.array([0.4, 0.25, 0.2, 0.1, 0.05])
    D = np.zeros((n, n))
    D[rows, rows] = q
    res = ent.entropy_estimate(torch.from_numpy(D).to(DEV), "randproj", 1, 1, seed, rank_k=5, sketch_width=s,
                               sketch="count")
    assert res.entropy == pytest.approx(float(-np.sum(q * np.log(q))), rel=1e-13)


@pytest.mark.parametrize("precision", ["f32", "bf16x3"])
def test_srht_reduced_precision(orc, precision):
    n, k, s = 1024, 16, 64
    R, p = low_rank(n, k, 17)
    res = ent.entropy_estimate(torch.from_numpy(R).to(DEV), "randproj", 1, 1, 6, rank_k=k, sketch_width=s,
                               precision=precision, sketch="srht")
    h_ref, _ = orc.rp_entropy(R, s, k, 6, kind=1)
    rel = abs(res.entropy - h_ref) / h_ref
    print(f"[rp srht {precision}] rel={rel:.2e}", flush=True)
    assert rel <= tol_for(precision)


def test_count_sketch_at_n8192(orc):
    n, k, s = 8192, 4, 32
    pk = W.spectrum_exp(k, 2.0)
    R = W.low_rank_density_torch(pk, n, 9, device=DEV, dtype=torch.float64)
    res, sig, _ = ent.entropy_estimate_detail(R, "randproj", 1, 1, 3, rank_k=k, sketch_width=s,
                                              precision="f64", sketch="count")
    h_ref, sig_ref = orc.rp_entropy(R.cpu().numpy(), s, k, 3, kind=2)
    assert res.entropy == pytest.approx(h_ref, rel=1e-10)
    assert np.allclose(sig, sig_ref, rtol=1e-9)


def test_unknown_sketch_rejected():
    R, _ = low_rank(64, 4, 1)
    with pytest.raises(ent.EntropyError):
        ent.entropy_estimate(torch.from_numpy(R).to(DEV), "randproj", 1, 1, 1, rank_k=4, sketch_width=8, sketch=7)
