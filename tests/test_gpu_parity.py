"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle on
the same seeded inputs, probe by probe.

FP64 bar: per-probe values and the estimate within 1e-10 relative, moments
within 1e-10 of ||g||^2, p~1 within 1e-12 relative.  FP32 / BF16x3 bar:
TOL_F32 / TOL_BF16X3 per probe (tests/tolerances.py; measured errors are printed).
"""
import math

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
TOL64 = 1e-10


def to_dev(R):
    return torch.from_numpy(np.ascontiguousarray(R)).to(DEV)


def csr_to_dev(csr):
    rp, ci, val, n = csr
    return (torch.from_numpy(rp).to(DEV), torch.from_numpy(ci).to(DEV), torch.from_numpy(val).to(DEV), n)


def check_fp64(gpu, per, mom, ref, orc, R, method, m, s, seed, dist, lo=0.0, u_fixed=0.0, label=""):
    # relative to the mean |h_j|; a state with H = 0 (pure) is held to 1e-12 absolute
    scale = max(np.mean(np.abs(ref.per_probe)), 1e-2)
    err = np.max(np.abs(per - ref.per_probe)) / scale
    print(f"[{label}] H gpu={gpu.entropy:.15f} oracle={ref.entropy:.15f} per-probe rel err={err:.2e}", flush=True)
    assert err <= TOL64
    assert abs(gpu.entropy - ref.entropy) <= TOL64 * abs(ref.entropy) + 1e-12
    assert gpu.u == pytest.approx(ref.u, rel=1e-12)
    if not u_fixed:
        assert gpu.p1_est == pytest.approx(ref.p1_est, rel=1e-12)
    assert gpu.std_err == pytest.approx(ref.std_err, rel=1e-8, abs=1e-14)
    # moments of a few probes against the oracle's forward recurrence (Chebyshev)
    if method == "chebyshev" and mom is not None:
        n = R.n if hasattr(R, "n") else (R[3] if isinstance(R, tuple) else R.shape[0])
        for j in sorted({0, s // 2, s - 1}):
            g = orc.probe_vector(seed, dist, 0, n, j)
            dref = orc.cheb_moments_forward(R, lo, ref.u, m, g)
            assert np.max(np.abs(mom[:, j] - dref)) <= TOL64 * float(g @ g)


@pytest.mark.parametrize("method", ["chebyshev", "taylor"])
@pytest.mark.parametrize("dist", ["rademacher", "gaussian"])
def test_dense_fp64_small_config(orc, method, dist):
    # n = 512, p_i ~ 1/i, degree 30, 50 probes, t = 20 (the small dense workload)
    n, m, s, seed = 512, 30, 50, W.PROBE_SEED + 1
    R = W.dense_density(W.spectrum_inverse(n), W.MATRIX_SEED + 1)
    d = 0 if dist == "rademacher" else 1
    gpu, per, mom = ent.entropy_estimate_detail(to_dev(R), method, m, s, seed, probe_dist=dist)
    ref = orc.estimate(R, 0 if method == "taylor" else 1, m, s, seed, dist=d)
    check_fp64(gpu, per, mom, ref, orc, R, method, m, s, seed, d, label=f"512 {method} {dist}")


@pytest.mark.parametrize("n,s,m", [(1, 1, 1), (5, 3, 2), (63, 17, 5), (200, 37, 7), (257, 129, 9),
                                   (300, 300, 4)])
@pytest.mark.parametrize("method", ["chebyshev", "taylor"])
def test_dense_fp64_ragged_shapes(orc, n, s, m, method):
    R = W.dense_density(W.spectrum_exp(n, max(n / 5.0, 1.0)), 100 + n)
    seed = 3 + n
    gpu, per, mom = ent.entropy_estimate_detail(to_dev(R), method, m, s, seed, probe_dist="gaussian")
    ref = orc.estimate(R, 0 if method == "taylor" else 1, m, s, seed, dist=1)
    check_fp64(gpu, per, mom, ref, orc, R, method, m, s, seed, 1, label=f"ragged {n}x{s} m={m} {method}")


def test_dense_fp64_interval_options(orc):
    n, m, s, seed = 130, 16, 20, 11
    R = W.dense_density(W.spectrum_exp(n, 30.0), 77)
    # fixed u (no power method) and a lower cutoff (interpolant on [lo, u])
    gpu, per, mom = ent.entropy_estimate_detail(to_dev(R), "chebyshev", m, s, seed, u_fixed=0.5, cutoff=1e-4)
    ref = orc.estimate(R, 1, m, s, seed, u_override=0.5, lo=1e-4)
    check_fp64(gpu, per, mom, ref, orc, R, "chebyshev", m, s, seed, 0, lo=1e-4, u_fixed=0.5, label="cutoff")
    # u factor c = 1 and several power trials
    gpu, per, _ = ent.entropy_estimate_detail(to_dev(R), "taylor", m, s, seed, u_factor=1.0, power_trials=3)
    ref = orc.estimate(R, 0, m, s, seed, c=1.0, q=3)
    check_fp64(gpu, per, None, ref, orc, R, "taylor", m, s, seed, 0, label="c=1 q=3")


def test_dense_storage_fp32_and_strided(orc):
    n, m, s, seed = 200, 10, 33, 5
    R = W.dense_density(W.spectrum_inverse(n), 8).astype(np.float32)
    # FP32 storage, FP64 compute: the oracle widens the same bytes
    gpu, per, _ = ent.entropy_estimate_detail(to_dev(R), "chebyshev", m, s, seed)
    ref = orc.estimate(R, 1, m, s, seed)
    check_fp64(gpu, per, None, ref, orc, R, "chebyshev", m, s, seed, 0, label="fp32 storage")
    # odd leading dimension (a column slice of a wider buffer)
    big = np.zeros((n, n + 3), dtype=np.float64)
    big[:, 1:n + 1] = R.astype(np.float64)
    Bd = to_dev(big)
    view = Bd[:, 1:n + 1]
    # (FP32-rounded entries: the trace is 1 only to ~1e-9, so widen the check)
    gpu2, per2, _ = ent.entropy_estimate_detail(view, "chebyshev", m, s, seed, trace_tol=1e-6)
    ref2 = orc.estimate(R.astype(np.float64), 1, m, s, seed)
    check_fp64(gpu2, per2, None, ref2, orc, R.astype(np.float64), "chebyshev", m, s, seed, 0, label="strided")


@pytest.mark.parametrize("method", ["chebyshev", "taylor"])
def test_dense_fp32_compute(orc, method):
    n, m, s, seed = 512, 30, 50, 9
    R = W.dense_density(W.spectrum_inverse(n), W.MATRIX_SEED + 1)
    gpu, per, _ = ent.entropy_estimate_detail(to_dev(R), method, m, s, seed, precision="f32")
    ref = orc.estimate(R, 0 if method == "taylor" else 1, m, s, seed)
    rel = abs(gpu.entropy - ref.entropy) / abs(ref.entropy)
    perr = np.max(np.abs(per - ref.per_probe)) / np.mean(np.abs(ref.per_probe))
    print(f"[f32 {method}] H gpu={gpu.entropy:.10f} oracle={ref.entropy:.10f} rel err={rel:.2e} "
          f"per-probe={perr:.2e}", flush=True)
    assert rel <= TOL_F32 and perr <= TOL_F32


@pytest.mark.parametrize("n,s", [(2048, 8), (3000, 20)])
def test_dense_split_k(orc, n, s):
    # few row tiles: the product runs over 8 column ranges (the last one of
    # n = 3000 ends inside a 32-column chunk) and the split epilogue sums
    # them; FP64 to the oracle, forward (Chebyshev, Taylor) and Clenshaw
    R = W.dense_density(W.spectrum_exp(n, n / 6.0), 300 + n)
    m, seed = 6, 4
    for method, flags in (("chebyshev", 0), ("taylor", 0), ("chebyshev", ent.FLAG_CLENSHAW)):
        gpu, per, mom = ent.entropy_estimate_detail(to_dev(R), method, m, s, seed, flags=flags)
        ref = orc.estimate(R, 0 if method == "taylor" else 1, m, s, seed)
        err = np.max(np.abs(per - ref.per_probe)) / np.mean(np.abs(ref.per_probe))
        print(f"[split-K n={n} s={s} {method} flags={flags}] per-probe rel {err:.2e}", flush=True)
        assert err <= 1e-10
    gpu, per, _ = ent.entropy_estimate_detail(to_dev(R), "chebyshev", m, s, seed, precision="f32")
    ref = orc.estimate(R, 1, m, s, seed)
    assert np.max(np.abs(per - ref.per_probe)) / np.mean(np.abs(ref.per_probe)) <= TOL_F32


def test_special_states(orc):
    n = 96
    # pure state: Taylor gives exactly ln(1) + 0 (u = 1)
    Rp = W.pure_state(n, 4)
    gpu = ent.entropy_estimate(to_dev(Rp), "taylor", 20, 8, 1)
    assert gpu.u == 1.0 and abs(gpu.entropy) < 1e-12
    # maximally mixed: p~1 = 1/n exactly; Chebyshev equals -n f_m(1/n)
    Rm = W.maximally_mixed(n)
    gpu = ent.entropy_estimate(to_dev(Rm), "chebyshev", 20, 8, 1)
    ref = orc.estimate(Rm, 1, 20, 8, 1)
    assert gpu.p1_est == pytest.approx(1.0 / n, rel=1e-14)
    assert gpu.entropy == pytest.approx(ref.entropy, rel=1e-12)
    assert abs(gpu.entropy - math.log(n)) <= n * gpu.u / (2 * 20 * 20)


def test_trace_check_and_numeric_errors():
    n = 64
    R = W.maximally_mixed(n) * 2.0
    with pytest.raises(ent.EntropyError) as e:
        ent.entropy_estimate(to_dev(R), "chebyshev", 10, 4, 0)
    assert e.value.status == ent.ENOTDENSITY
    gpu = ent.entropy_estimate(to_dev(R), "chebyshev", 10, 4, 0, flags=ent.FLAG_SKIP_TRACE_CHECK)
    assert math.isfinite(gpu.entropy)
    Z = np.zeros((n, n))
    with pytest.raises(ent.EntropyError) as e:
        ent.entropy_estimate(to_dev(Z), "chebyshev", 10, 4, 0, flags=ent.FLAG_SKIP_TRACE_CHECK)
    assert e.value.status == ent.ENUMERIC


def test_power_method_and_coefficients(orc):
    n = 300
    p = W.spectrum_exp(n, 50.0)
    R = W.dense_density(p, 31)
    for q in (1, 4):
        v = ent.power_method(to_dev(R), 20, q, 17)
        assert v == pytest.approx(orc.power_method(R, 20, q, 17), rel=1e-12)
        assert v <= p[0] * (1 + 1e-12)
    for lo in (0.0, 1e-3):
        a = ent.chebyshev_coeffs(lo, 0.3, 40)
        b = orc.cheb_interp_coeffs(lo, 0.3, 40, orc.cutoff_nodes(40)) if lo > 0 else orc.cheb_coeffs(0.3, 40)
        # small coefficients of the projection come out of a 1024-term cancelling
        # sum: compare at 1e-13 relative to u (libm vs device cos/log)
        assert np.max(np.abs(a - b)) <= 1e-13 * 0.3


def test_determinism_bitwise():
    n, m, s = 257, 20, 70
    R = to_dev(W.dense_density(W.spectrum_inverse(n), 5))
    a = ent.entropy_estimate_detail(R, "chebyshev", m, s, 3, probe_dist="gaussian")
    b = ent.entropy_estimate_detail(R, "chebyshev", m, s, 3, probe_dist="gaussian")
    assert a[0].entropy == b[0].entropy
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


# ------------------------------------------------------------------ CSR ------
@pytest.mark.parametrize("method", ["chebyshev", "taylor"])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_csr_banded_parity(orc, method, dtype):
    # banded R = B B^T / tr, half-bandwidth 16, the sparse workload at n = 10^5
    n, m, s, seed = 100_000, 40, 64, W.PROBE_SEED + 3
    csr = W.banded_density_csr(n, 8, seed=W.MATRIX_SEED + 3, dtype=dtype)
    prec = "f64" if dtype == np.float64 else "f32"
    gpu, per, mom = ent.entropy_estimate_detail(csr_to_dev(csr), method, m, s, seed, precision=prec)
    ref = orc.estimate(csr, 0 if method == "taylor" else 1, m, s, seed)
    if dtype == np.float64:
        check_fp64(gpu, per, mom, ref, orc, csr, method, m, s, seed, 0, label=f"csr 1e5 {method}")
    else:
        rel = abs(gpu.entropy - ref.entropy) / abs(ref.entropy)
        perr = np.max(np.abs(per - ref.per_probe)) / np.mean(np.abs(ref.per_probe))
        print(f"[csr f32 {method}] H gpu={gpu.entropy:.10f} oracle={ref.entropy:.10f} rel={rel:.2e} per-probe={perr:.2e}", flush=True)
        assert rel <= TOL_F32 and perr <= TOL_F32


@pytest.mark.parametrize("n,s", [(1, 1), (7, 3), (1000, 65), (4097, 130)])
def test_csr_ragged(orc, n, s):
    csr = W.banded_density_csr(n, 3, seed=n)
    m, seed = 9, 2
    for dist in ("rademacher", "gaussian"):
        d = 0 if dist == "rademacher" else 1
        gpu, per, mom = ent.entropy_estimate_detail(csr_to_dev(csr), "chebyshev", m, s, seed, probe_dist=dist)
        ref = orc.estimate(csr, 1, m, s, seed, dist=d)
        check_fp64(gpu, per, mom, ref, orc, csr, "chebyshev", m, s, seed, d, label=f"csr {n} {s} {dist}")


def test_csr_wide_windows_fall_back(orc):
    # scattered columns: most chunks' column windows exceed the LDS window
    # buffer, so the step gathers those chunks' V_k rows from global memory
    import scipy.sparse as sp

    n, m, s, seed = 3000, 12, 32, 6
    rng = np.random.default_rng(8)
    B = sp.random(n, n, density=4.0 / n, random_state=rng, format="csr") + sp.eye(n, format="csr")
    Rs = (B @ B.T).tocsr()
    Rs = Rs / Rs.diagonal().sum()
    Rs.sort_indices()
    csr = (Rs.indptr.astype(np.int64), Rs.indices.astype(np.int32), Rs.data.astype(np.float64))
    for method in ("chebyshev", "taylor"):
        gpu, per, mom = ent.entropy_estimate_detail(csr_to_dev(csr + (n,)), method, m, s, seed)
        ref = orc.estimate(csr + (n,), 0 if method == "taylor" else 1, m, s, seed)
        check_fp64(gpu, per, mom, ref, orc, csr + (n,), method, m, s, seed, 0, label=f"csr wide {method}")


def test_csr_long_rows(orc):
    # ~100 entries per row: several rounds of the step's gather loop per row
    # (it loads 40 entries of a row at a time), with ragged row lengths
    import scipy.sparse as sp

    n, m, s, seed = 2000, 10, 64, 3
    rng = np.random.default_rng(12)
    B = sp.random(n, n, density=10.0 / n, random_state=rng, format="csr") + sp.eye(n, format="csr")
    Rs = (B @ B.T).tocsr()
    Rs = Rs / Rs.diagonal().sum()
    Rs.sort_indices()
    assert np.diff(Rs.indptr).mean() > 60
    csr = (Rs.indptr.astype(np.int64), Rs.indices.astype(np.int32), Rs.data.astype(np.float64), n)
    for method in ("chebyshev", "taylor"):
        gpu, per, mom = ent.entropy_estimate_detail(csr_to_dev(csr), method, m, s, seed)
        ref = orc.estimate(csr, 0 if method == "taylor" else 1, m, s, seed)
        check_fp64(gpu, per, mom, ref, orc, csr, method, m, s, seed, 0, label=f"csr long rows {method}")


def test_csr_poisson_closed_form():
    # tridiagonal experiment: exact H from lambda_i = (4/2n) sin^2(i pi/(2n+2))
    n = 100_000
    csr = W.poisson_csr_fast(n)
    lam = W.poisson_eigenvalues(n)
    H = float(-np.sum(lam * np.log(lam)))
    gpu = ent.entropy_estimate(csr_to_dev(csr), "chebyshev", 40, 64, 5, u_factor=1.0)
    rel = abs(gpu.entropy - H) / H
    print(f"[poisson 1e5] H exact={H:.10f} gpu={gpu.entropy:.10f} rel={rel:.2e} se={gpu.std_err:.2e}", flush=True)
    # truncation (NTE) + sampling; the paper reports < 0.5% for m = 5, s = 50 at n = 5000
    assert rel < 5e-3


def test_poisson_1e7_paper_configuration(orc):
    # the paper's tridiagonal experiment settings (m = 10, s = 100, c = 1) at n = 10^7,
    # built on the device; exact H from the closed-form spectrum
    n, m, s, seed = 10_000_000, 10, 100, 12
    Rd = W.poisson_csr_torch(n, device=DEV, dtype=torch.float32)
    lam = W.poisson_eigenvalues(n)
    H = float(-np.sum(lam * np.log(lam)))
    res, per, _ = ent.entropy_estimate_detail(Rd, "chebyshev", m, s, seed, precision="f32", u_factor=1.0)
    rel = abs(res.entropy - H) / H
    print(f"[poisson 1e7 m=10 s=100] H exact={H:.8f} gpu={res.entropy:.8f} rel={rel:.2e} se={res.std_err:.2e}",
          flush=True)
    assert rel < 2e-3
    # sampled probes against the oracle on the same (host) matrix
    host = tuple(a.cpu().numpy() for a in Rd[:3]) + (n,)
    sel = [0, 99]
    ref = orc.estimate(host, 1, m, s, seed, t=20, dist=0, c=1.0, probes=sel)
    err = np.max(np.abs(per[sel] - ref.per_probe)) / np.mean(np.abs(ref.per_probe))
    print(f"[poisson 1e7] sampled per-probe rel err vs oracle {err:.2e}", flush=True)
    assert err <= TOL_F32


# --------------------------------------------------------------- BF16x3 ------
@pytest.mark.parametrize("method", ["chebyshev", "taylor"])
@pytest.mark.parametrize("dist", ["rademacher", "gaussian"])
def test_dense_bf16x3_small_config(orc, method, dist):
    n, m, s, seed = 512, 30, 50, W.PROBE_SEED + 1
    R = W.dense_density(W.spectrum_inverse(n), W.MATRIX_SEED + 1)
    d = 0 if dist == "rademacher" else 1
    gpu, per, mom = ent.entropy_estimate_detail(to_dev(R), method, m, s, seed, probe_dist=dist,
                                                precision="bf16x3")
    ref = orc.estimate(R, 0 if method == "taylor" else 1, m, s, seed, dist=d)
    rel = abs(gpu.entropy - ref.entropy) / abs(ref.entropy)
    perr = np.max(np.abs(per - ref.per_probe)) / np.mean(np.abs(ref.per_probe))
    print(f"[bf16x3 512 {method} {dist}] H gpu={gpu.entropy:.12f} oracle={ref.entropy:.12f} "
          f"rel={rel:.2e} per-probe={perr:.2e}", flush=True)
    # the power method reads the bf16 hi/lo split of R (about 2^-17 relative per
    # entry) and accumulates in FP64
    assert gpu.p1_est == pytest.approx(ref.p1_est, rel=1e-6)
    assert rel <= TOL_BF16X3 and perr <= TOL_BF16X3


@pytest.mark.parametrize("n,s,m", [(1, 1, 1), (100, 5, 3), (200, 37, 7), (300, 300, 6), (700, 129, 12)])
def test_dense_bf16x3_ragged(orc, n, s, m):
    R = W.dense_density(W.spectrum_exp(n, max(n / 5.0, 1.0)), 100 + n)
    seed = 3 + n
    for method in ("chebyshev", "taylor"):
        gpu, per, mom = ent.entropy_estimate_detail(to_dev(R), method, m, s, seed, probe_dist="gaussian",
                                                    precision="bf16x3")
        ref = orc.estimate(R, 0 if method == "taylor" else 1, m, s, seed, dist=1)
        # n = 1 (a pure state): h_j is about 0 and its bf16x3 error is a
        # fraction of ||g||^2, so the scale has a floor of 1
        scale = max(np.mean(np.abs(ref.per_probe)), 1.0)
        perr = np.max(np.abs(per - ref.per_probe)) / scale
        print(f"[bf16x3 {n}x{s} m={m} {method}] rel per-probe err={perr:.2e}", flush=True)
        assert perr <= TOL_BF16X3
        if method == "chebyshev":
            # moments of a matrix with spectrum in [-1, 1] stay within ||g||^2
            g2 = mom[0]
            assert np.all(np.abs(mom) <= g2[None, :] * (1 + 1e-3) + 1e-6)


def test_bf16x3_fp32_storage_and_determinism(orc):
    n, m, s, seed = 384, 20, 64, 4
    R = W.dense_density(W.spectrum_inverse(n), 9).astype(np.float32)
    a = ent.entropy_estimate_detail(to_dev(R), "chebyshev", m, s, seed, precision="bf16x3")
    b = ent.entropy_estimate_detail(to_dev(R), "chebyshev", m, s, seed, precision="bf16x3")
    assert np.array_equal(a[1], b[1])
    ref = orc.estimate(R, 1, m, s, seed)
    assert np.max(np.abs(a[1] - ref.per_probe)) / np.mean(np.abs(ref.per_probe)) <= TOL_BF16X3


def _hip_runtime():
    # the HIP runtime this process already uses (the library's calls go to it)
    import ctypes

    paths = {l.split()[-1] for l in open("/proc/self/maps") if "libamdhip64" in l}
    assert len(paths) == 1, paths
    return ctypes.CDLL(paths.pop())


def test_oversized_descriptor_rejected():
    # a descriptor larger than its device allocation is refused on the host,
    # before any kernel runs; each case is handed to the library only after
    # the same runtime query confirms that the library's check will refuse it
    # (host arrays are copied in instead: tests/test_gpu_boundary.py)
    import ctypes

    hip = _hip_runtime()
    res = ent.EntResult()
    R = torch.eye(1024, dtype=torch.float64, device=DEV) / 1024.0
    base, size = ctypes.c_void_p(), ctypes.c_size_t()
    if hip.hipMemGetAddressRange(ctypes.byref(base), ctypes.byref(size), ctypes.c_void_p(R.data_ptr())) != 0:
        pytest.skip("the runtime reports no allocation range")  # pragma: no cover
    avail = base.value + size.value - R.data_ptr()
    nbig = int(np.sqrt(avail / 8)) + 2
    assert ((nbig - 1) * nbig + nbig) * 8 > avail
    M = ent.EntMatrix(nbig, ent.DENSE, ent.STORE_F64, nbig, 0, R.data_ptr(), None, None)
    assert ent._lib.ent_entropy_estimate(ctypes.byref(M), 1, 10, 8, 0, None, ctypes.byref(res)) == ent.EINVAL
    assert "exceed its allocation" in ent.last_error()
    assert ent._lib.ent_power_method(ctypes.byref(M), 5, 1, 0, None, ctypes.byref(ctypes.c_double())) == ent.EINVAL
    # CSR: col_idx shorter than nnz
    rp = torch.tensor([0, 1, 2], dtype=torch.int64, device=DEV)
    ci = torch.tensor([0, 1], dtype=torch.int32, device=DEV)
    va = torch.tensor([0.5, 0.5], dtype=torch.float64, device=DEV)
    if hip.hipMemGetAddressRange(ctypes.byref(base), ctypes.byref(size), ctypes.c_void_p(ci.data_ptr())) != 0:
        pytest.skip("the runtime reports no allocation range")  # pragma: no cover
    big_nnz = (base.value + size.value - ci.data_ptr()) // 4 + 1
    M = ent.EntMatrix(2, ent.CSR, ent.STORE_F64, 0, big_nnz, va.data_ptr(), rp.data_ptr(), ci.data_ptr())
    assert ent._lib.ent_entropy_estimate(ctypes.byref(M), 1, 10, 8, 0, None, ctypes.byref(res)) == ent.EINVAL
    # the same arrays with their true sizes are accepted
    M = ent.EntMatrix(2, ent.CSR, ent.STORE_F64, 0, 2, va.data_ptr(), rp.data_ptr(), ci.data_ptr())
    assert ent._lib.ent_entropy_estimate(ctypes.byref(M), 1, 10, 8, 0, None, ctypes.byref(res)) == ent.OK


def test_csr_structure_rejected(orc):
    # malformed CSR input is refused by the device-side structure check
    # before any step reads it (n is not a multiple of 64, so even a column
    # index of n would stay inside the padded buffers)
    n = 100
    rp, ci, val, _ = W.banded_density_csr(n, 3, seed=5)
    ci = ci.astype(np.int32)

    def run(rp_, ci_, val_, nnz=None):
        M = ent.csr_matrix(torch.from_numpy(rp_).to(DEV), torch.from_numpy(ci_).to(DEV),
                           torch.from_numpy(val_).to(DEV), n)
        if nnz is not None:
            M.nnz = nnz
        return ent.entropy_estimate(M, "chebyshev", 8, 8, 1)

    good = run(rp, ci, val)
    bad = []
    c = ci.copy(); c[len(c) // 2] = n; bad.append((rp, c, val, None))
    c = ci.copy(); c[7] = -1; bad.append((rp, c, val, None))
    r = rp.copy(); r[10], r[11] = r[11], r[10]; bad.append((r, ci, val, None))
    r = rp.copy(); r[0] = 1; bad.append((r, ci, val, None))
    bad.append((rp, ci, val, len(ci) - 1))
    for k, (r_, c_, v_, nnz) in enumerate(bad):
        with pytest.raises(ent.EntropyError) as e:
            run(r_, c_, v_, nnz)
        assert e.value.status == ent.EINVAL, k
        assert "CSR structure" in str(e.value), k
    # column indices not 16-byte aligned (scalar path of the check): same result
    ci_off = torch.zeros(len(ci) + 1, dtype=torch.int32, device=DEV)
    ci_off[1:] = torch.from_numpy(ci).to(DEV)
    M = ent.csr_matrix(torch.from_numpy(rp).to(DEV), ci_off[1:], torch.from_numpy(val).to(DEV), n)
    assert ent.entropy_estimate(M, "chebyshev", 8, 8, 1).entropy == good.entropy
