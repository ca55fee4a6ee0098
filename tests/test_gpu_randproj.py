"""Random-projection estimator (Algorithm 3) on the GPU against the FP64
oracle with the same Gaussian sketch (Philox stream 2)."""
import numpy as np
import pytest

import workloads as W

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


@pytest.mark.parametrize("n,k,s", [(600, 10, 64), (257, 7, 33), (1000, 40, 128), (130, 5, 5)])
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
    print(f"[rp {precision}] H gpu={res.entropy:.10f} oracle={h_ref:.10f} rel={rel:.2e}", flush=True)
    assert rel <= 1e-3


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
