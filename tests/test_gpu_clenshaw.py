"""The Clenshaw schedule (Algorithm 5, Appendix B) on the GPU: the backward
recurrence y_k = alpha_k g + 2X y_{k+1} - y_{k+2} against the oracle, whose
Chebyshev estimator is itself Clenshaw's vector recurrence, and against the
library's forward recurrence (the same estimate up to rounding)."""
import numpy as np
import pytest

import workloads as W
from tolerances import TOL_F32, tol_for

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1801_01072_amd as ent  # noqa: E402

DEV = "cuda:0"
CL = ent.FLAG_CLENSHAW


def rel(a, b):
    return np.max(np.abs(a - b)) / np.mean(np.abs(b))


@pytest.mark.parametrize("m", [1, 2, 3, 15])
def test_dense_fp64_against_oracle_and_forward(orc, m):
    n, s, seed = 300, 20, 4
    R = W.dense_density(W.spectrum_exp(n, 30.0), 8)
    Rt = torch.from_numpy(R).to(DEV)
    res, per, mom = ent.entropy_estimate_detail(Rt, "chebyshev", m, s, seed, flags=CL)
    ref = orc.estimate(R, 1, m, s, seed)
    fwd, per_f, _ = ent.entropy_estimate_detail(Rt, "chebyshev", m, s, seed)
    print(f"[clenshaw f64 m={m}] per-probe vs oracle {rel(per, ref.per_probe):.2e}, vs forward "
          f"{rel(per, per_f):.2e}", flush=True)
    assert rel(per, ref.per_probe) <= 1e-10
    assert rel(per, per_f) <= 1e-10
    # y_m = alpha_m g: its dots are alpha_m g^T g
    alpha = orc.cheb_coeffs(res.u, m)
    gg = np.array([float(g @ g) for g in (orc.probe_vector(seed, 0, 0, n, j) for j in range(s))])
    assert np.allclose(mom[m], alpha[m] * gg, rtol=1e-12)


def test_csr_fp64_and_cutoff(orc):
    n, m, s, seed = 5000, 20, 64, 6
    csr = W.banded_density_csr(n, 4, seed=3)
    dev = tuple(torch.from_numpy(a).to(DEV) for a in csr[:3]) + (n,)
    res, per, _ = ent.entropy_estimate_detail(dev, "chebyshev", m, s, seed, flags=CL)
    ref = orc.estimate(csr, 1, m, s, seed)
    assert rel(per, ref.per_probe) <= 1e-10
    lo = 0.05 * res.u
    res2, per2, _ = ent.entropy_estimate_detail(dev, "chebyshev", m, s, seed, flags=CL, cutoff=lo)
    ref2 = orc.estimate(csr, 1, m, s, seed, lo=lo)
    print(f"[clenshaw csr] per-probe {rel(per, ref.per_probe):.2e}, cutoff {rel(per2, ref2.per_probe):.2e}",
          flush=True)
    assert rel(per2, ref2.per_probe) <= 1e-10


@pytest.mark.parametrize("prec", ["f32", "bf16x3"])
def test_reduced_precision(orc, prec):
    n, m, s, seed = 1024, 30, 64, 2
    R = W.dense_density(W.spectrum_exp(n, 100.0), 5)
    res, per, _ = ent.entropy_estimate_detail(torch.from_numpy(R).to(DEV), "chebyshev", m, s, seed, flags=CL,
                                              precision=prec, probe_dist="gaussian")
    ref = orc.estimate(R, 1, m, s, seed, dist=1)
    print(f"[clenshaw {prec}] per-probe {rel(per, ref.per_probe):.2e}", flush=True)
    assert rel(per, ref.per_probe) <= tol_for(prec)


def test_csr_fp32(orc):
    n, m, s, seed = 20000, 25, 64, 9
    csr = W.banded_density_csr(n, 8, seed=4, dtype=np.float32)
    dev = tuple(torch.from_numpy(a).to(DEV) for a in csr[:3]) + (n,)
    res, per, _ = ent.entropy_estimate_detail(dev, "chebyshev", m, s, seed, flags=CL, precision="f32")
    ref = orc.estimate(csr, 1, m, s, seed, probes=[0, 31, 63])
    assert rel(per[[0, 31, 63]], ref.per_probe) <= TOL_F32


def test_hermitian(orc):
    n, m, s, seed = 150, 12, 16, 3
    R = W.hermitian_density(W.spectrum_exp(n, 20.0), 6)
    res, per, _ = ent.entropy_estimate_detail(torch.from_numpy(R).to(DEV), "chebyshev", m, s, seed, flags=CL,
                                              probe_dist="gaussian")
    ref = orc.zestimate(R, 1, m, s, seed, dist=1, u_override=1.0)
    assert rel(per, ref.per_probe) <= 1e-10
