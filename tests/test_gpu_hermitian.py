"""Hermitian density matrices (Section 4, Algorithms 1c / 2c) through the
C-ABI against the oracle's complex-arithmetic estimators.  The library runs
them on the real 2n x 2n form with probes [g; 0]; the oracle works on R in
complex arithmetic, so the two share neither code nor method."""
import numpy as np
import pytest

import workloads as W
from tolerances import TOL_BF16X3, TOL_F32

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1801_01072_amd as ent  # noqa: E402

DEV = "cuda:0"
DISTS = {"rademacher": 0, "gaussian": 1}


def herm(n, seed, tau=None, dtype=np.complex128):
    p = W.spectrum_exp(n, tau or n / 8)
    return W.hermitian_density(p, seed, dtype=dtype), p


def rel_per_probe(a, b):
    return np.max(np.abs(a - b)) / np.mean(np.abs(b))


@pytest.mark.parametrize("dist", ["gaussian", "rademacher"])
@pytest.mark.parametrize("method", ["chebyshev", "taylor"])
def test_fp64_parity(orc, method, dist):
    n, m, s, seed = 200, 12, 24, 7          # 2n = 400: several tiles and a ragged tail
    R, _ = herm(n, 31)
    Rt = torch.from_numpy(R).to(DEV)
    res, per, mom = ent.entropy_estimate_detail(Rt, method, m, s, seed, probe_dist=dist)
    meth = 1 if method == "chebyshev" else 0
    ref = orc.zestimate(R, meth, m, s, seed, dist=DISTS[dist], u_override=1.0)
    err = rel_per_probe(per, ref.per_probe)
    print(f"[herm f64 {method} {dist}] H gpu={res.entropy:.12f} oracle={ref.entropy:.12f} per-probe={err:.2e}",
          flush=True)
    assert res.u == 1.0 and res.p1_est == 0.0
    assert err <= 1e-10
    assert res.entropy == pytest.approx(ref.entropy, rel=1e-10)
    if method == "chebyshev":
        for j in (0, 5, s - 1):
            g = orc.probe_vector(seed, DISTS[dist], 0, n, j)
            d = orc.zcheb_moments_forward(R, 0.0, 1.0, m, g)
            assert np.max(np.abs(mom[:, j] - d)) <= 1e-10 * float(g @ g)


@pytest.mark.parametrize("prec,storage,tol", [("f32", np.complex64, TOL_F32), ("bf16x3", np.complex128, TOL_BF16X3),
                                              ("f64", np.complex64, 1e-10)])
def test_reduced_precision_and_storage(orc, prec, storage, tol):
    n, m, s, seed = 300, 15, 16, 3
    R, _ = herm(n, 12, dtype=storage)
    res, per, _ = ent.entropy_estimate_detail(torch.from_numpy(R).to(DEV), "chebyshev", m, s, seed,
                                              precision=prec, probe_dist="gaussian")
    ref = orc.zestimate(R, 1, m, s, seed, dist=1, u_override=1.0)   # widened exactly from the stored values
    err = rel_per_probe(per, ref.per_probe)
    print(f"[herm {prec} {np.dtype(storage).name}] per-probe={err:.2e}", flush=True)
    assert err <= tol


def test_power_method_option(orc):
    n, m, s, seed = 160, 10, 8, 5
    R, p = herm(n, 3, tau=6.0)
    Rt = torch.from_numpy(R).to(DEV)
    res = ent.entropy_estimate(Rt, "chebyshev", m, s, seed, flags=ent.FLAG_COMPLEX_POWER, probe_dist="gaussian")
    p1 = orc.zpower_method(R, t=20, q=1, seed=seed)
    assert res.p1_est == pytest.approx(p1, rel=1e-12)
    assert res.u == pytest.approx(min(1.0, 6.0 * p1), rel=1e-12)
    ref = orc.zestimate(R, 1, m, s, seed, dist=1, u_override=0.0)
    assert res.entropy == pytest.approx(ref.entropy, rel=1e-10)
    # the stand-alone entry point runs the same iteration
    assert ent.power_method(Rt, t=20, q=1, seed=seed) == pytest.approx(p1, rel=1e-12)
    assert ent.power_method(Rt, t=300, q=1, seed=seed) == pytest.approx(p.max(), rel=1e-9)


def test_real_matrix_as_complex_matches_real_path():
    n, m, s, seed = 256, 20, 16, 9
    R = W.dense_density(W.spectrum_exp(n, 20.0), 44)
    real = ent.entropy_estimate_detail(torch.from_numpy(R).to(DEV), "chebyshev", m, s, seed, u_fixed=1.0)
    cplx = ent.entropy_estimate_detail(torch.from_numpy(R.astype(np.complex128)).to(DEV), "chebyshev", m, s,
                                       seed)
    assert rel_per_probe(cplx[1], real[1]) <= 1e-12
    assert np.max(np.abs(cplx[2] - real[2])) <= 1e-11 * n


def test_estimate_close_to_exact_entropy():
    n, m, s = 512, 60, 128
    p = W.spectrum_exp(n, 40.0)
    R = W.hermitian_density(p, 77)
    H = float(-np.sum(p * np.log(p)))
    for method, deg in (("chebyshev", m), ("taylor", 4 * m)):
        res = ent.entropy_estimate(torch.from_numpy(R).to(DEV), method, deg, s, 1, probe_dist="gaussian")
        print(f"[herm accuracy {method}] H={H:.6f} est={res.entropy:.6f} se={res.std_err:.2e}", flush=True)
        assert abs(res.entropy - H) <= 4 * res.std_err + 0.02 * H


def test_trace_check_and_padding_strides(orc):
    n = 70
    R, _ = herm(n, 5)
    bad = torch.from_numpy(2.0 * R).to(DEV)
    with pytest.raises(ent.EntropyError) as e:
        ent.entropy_estimate(bad, "chebyshev", 5, 4, 1)
    assert e.value.status == ent.ENOTDENSITY
    # a view with leading dimension > n
    big = torch.zeros((n, n + 9), dtype=torch.complex128)
    big[:, :n] = torch.from_numpy(R)
    view = big.to(DEV)[:, :n]
    res, per, _ = ent.entropy_estimate_detail(view, "taylor", 6, 5, 2, probe_dist="gaussian")
    ref = orc.zestimate(R, 0, 6, 5, 2, dist=1, u_override=1.0)
    assert rel_per_probe(per, ref.per_probe) <= 1e-10


def test_sampled_probes_at_n2048_bf16x3(orc):
    n, m, s, seed = 2048, 10, 64, 11
    p = W.spectrum_exp(n, n / 10)
    R = W.hermitian_density(p, 5)
    res, per, _ = ent.entropy_estimate_detail(torch.from_numpy(R).to(DEV), "chebyshev", m, s, seed,
                                              precision="bf16x3", probe_dist="gaussian")
    sel = [0, 17, 63]
    ref = orc.zestimate(R, 1, m, s, seed, dist=1, u_override=1.0, probes=sel)
    err = np.max(np.abs(per[sel] - ref.per_probe)) / np.mean(np.abs(ref.per_probe))
    print(f"[herm n=2048 bf16x3] sampled per-probe rel err {err:.2e}", flush=True)
    assert err <= TOL_BF16X3


def test_release_while_estimating_from_another_thread():
    # a Hermitian estimate holds its real-form buffer while it takes the
    # workspace; releasing both from another thread must neither deadlock
    # nor disturb the estimates
    import threading

    n, m, s, seed = 300, 10, 16, 5
    R, _ = herm(n, 41)
    Rt = torch.from_numpy(R).to(DEV)
    ref = ent.entropy_estimate(Rt, "chebyshev", m, s, seed).entropy
    out, errs = [], []

    def worker():
        try:
            for _ in range(6):
                out.append(ent.entropy_estimate(Rt, "chebyshev", m, s, seed).entropy)
        except Exception as e:  # pragma: no cover
            errs.append(e)

    def releaser():
        try:
            for _ in range(30):
                ent.release_workspace()
        except Exception as e:  # pragma: no cover
            errs.append(e)

    th = [threading.Thread(target=worker, daemon=True), threading.Thread(target=releaser, daemon=True)]
    for t in th:
        t.start()
    for t in th:
        t.join(timeout=60)
    assert not any(t.is_alive() for t in th), "estimate and release did not both finish"
    assert not errs, errs
    assert out == [ref] * 6
