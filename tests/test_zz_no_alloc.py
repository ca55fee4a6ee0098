"""The entry point that allocates no device memory: its results against the
allocating entry point's on the same inputs (FP64 to 1e-10 relative per
probe -- the same kernels, so in practice identical), on two calls in a row
with the second smaller, and its refusal of requests beyond its fixed
scratch."""
import ctypes

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1801_01072_amd as ent  # noqa: E402

DEV = "cuda:0"


def compare(R, method, m, s, seed, tol, **kw):
    a, pa, ma = ent.entropy_estimate_noalloc(R, method, m, s, seed, **kw)
    b, pb, mb = ent.entropy_estimate_detail(R, method, m, s, seed, **kw)
    scale = max(np.mean(np.abs(pb)), 1e-2)
    err = float(np.max(np.abs(pa - pb)) / scale)
    merr = float(np.max(np.abs(ma - mb)))
    print(f"[noalloc {method} m={m} s={s} {kw}] H={a.entropy:.15f} vs {b.entropy:.15f} "
          f"per-probe err={err:.2e} moments err={merr:.2e}", flush=True)
    assert err <= tol
    assert abs(a.entropy - b.entropy) <= tol * abs(b.entropy) + 1e-14
    assert (a.degree, a.probes, a.method) == (b.degree, b.probes, b.method)
    assert a.u == b.u and a.p1_est == b.p1_est
    return a


@pytest.mark.parametrize("method", ["chebyshev", "taylor"])
def test_noalloc_matches_allocating_entry_point_twice(method):
    # first call: n = 700, s = 96; second call smaller: n = 130, s = 20
    R1 = torch.from_numpy(W.dense_density(W.spectrum_exp(700, 90.0), 5)).to(DEV)
    R2 = torch.from_numpy(W.dense_density(W.spectrum_inverse(130), 6)).to(DEV)
    compare(R1, method, 24, 96, 11, 1e-10, probe_dist="gaussian")
    compare(R2, method, 9, 20, 12, 1e-10)


def test_noalloc_other_forms():
    R = torch.from_numpy(W.dense_density(W.spectrum_exp(300, 40.0), 8)).to(DEV)
    compare(R, "chebyshev", 16, 40, 3, 1e-6, precision="f32")
    compare(R, "chebyshev", 16, 40, 3, 1e-6, precision="bf16x3")
    compare(R, "chebyshev", 16, 40, 3, 1e-10, flags=ent.FLAG_CLENSHAW)
    csr = W.banded_density_csr(5000, 8, seed=4)
    Rc = tuple(torch.from_numpy(a).to(DEV) for a in csr[:3]) + (5000,)
    compare(Rc, "chebyshev", 12, 64, 2, 1e-10)
    compare(Rc, "taylor", 6, 10, 2, 1e-10, flags=ent.FLAG_CSR_GENERAL)


def test_noalloc_refusals_leave_output_untouched():
    lib = ent._lib
    res = ent.EntResult()
    res.entropy = 7.0
    o = ent.options()
    # beyond the fixed scratch: dense n = 8192 FP64 with 1024 probes (~200 MB of V blocks)
    big = torch.zeros((8192, 8192), dtype=torch.float64, device=DEV)
    big.diagonal().fill_(1.0 / 8192)
    M = ent.as_matrix(big)
    st = lib.ent_entropy_estimate_noalloc(ctypes.byref(M), ent.CHEBYSHEV, 10, 1024, 1, ctypes.byref(o),
                                          ctypes.byref(res), None, None)
    assert st == ent.ENOMEM and "fixed scratch" in ent.last_error()
    assert res.entropy == 7.0
    del big
    # host arrays, random projection, learned selector
    Rh = torch.from_numpy(W.dense_density(W.spectrum_inverse(16), 1))
    Mh = ent.as_matrix(Rh)
    assert lib.ent_entropy_estimate_noalloc(ctypes.byref(Mh), ent.CHEBYSHEV, 4, 4, 1, ctypes.byref(o),
                                            ctypes.byref(res), None, None) == ent.EINVAL
    Md = ent.as_matrix(Rh.to(DEV))
    for meth in (ent.RANDPROJ, ent.AUTO):
        assert lib.ent_entropy_estimate_noalloc(ctypes.byref(Md), meth, 4, 4, 1, ctypes.byref(o),
                                                ctypes.byref(res), None, None) == ent.EUNSUPPORTED
    assert res.entropy == 7.0
    # the entry point still works after the refusals
    a, _, _ = ent.entropy_estimate_noalloc(Rh.to(DEV), "chebyshev", 6, 8, 1)
    assert np.isfinite(a.entropy)
