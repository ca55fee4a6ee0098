"""GPU parity of the banded CSR kernels (a CSR R whose entries all lie within
16 of the diagonal runs as 16-row MFMA slabs when they are no larger than the
CSR arrays, or always with FLAG_CSR_BANDED): which kernel ran, per-probe
values against the FP64 oracle for every padded band width, precision,
schedule and probe distribution, ragged sizes, duplicate entries, and
agreement with the general CSR kernel on the same input."""
import numpy as np
import pytest

import workloads as W
from tolerances import TOL_F32

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1801_01072_amd as ent  # noqa: E402

DEV = "cuda:0"
TOL64 = 1e-10
TOL32 = TOL_F32


def csr_to_dev(csr):
    rp, ci, val, n = csr
    return (torch.from_numpy(rp).to(DEV), torch.from_numpy(ci).to(DEV), torch.from_numpy(val).to(DEV), n)


def run(csr, method, m, s, seed, **kw):
    ent.timing_enable(True)
    try:
        res, per, mom = ent.entropy_estimate_detail(csr_to_dev(csr), method, m, s, seed, **kw)
        band = ent.last_timing()["csr_band"]
    finally:
        ent.timing_enable(False)
    return res, per, mom, band


def per_probe_rel(per, ref):
    return float(np.max(np.abs(per - ref.per_probe)) / max(np.mean(np.abs(ref.per_probe)), 1e-2))


# half-bandwidth of B -> of R = B B^T (2 hb), and the padded width served
@pytest.mark.parametrize("hb,hp", [(1, 4), (2, 4), (3, 8), (4, 8), (5, 16), (8, 16)])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_band_widths(orc, hb, hp, dtype):
    n, m, s, seed = 5003, 20, 64, 41 + hb
    csr = W.banded_density_csr(n, hb, seed=100 + hb, dtype=dtype)
    prec = "f64" if dtype == np.float64 else "f32"
    res, per, _, band = run(csr, "chebyshev", m, s, seed, precision=prec, flags=ent.FLAG_CSR_BANDED)
    ref = orc.estimate(csr, 1, m, s, seed)
    err = per_probe_rel(per, ref)
    print(f"[band hb={hb} {prec}] kernel band {band}; H gpu={res.entropy:.12f} oracle={ref.entropy:.12f} "
          f"per-probe rel {err:.2e}", flush=True)
    assert band == hp
    assert err <= (TOL64 if dtype == np.float64 else TOL32)
    if dtype == np.float64:
        assert abs(res.entropy - ref.entropy) <= TOL64 * abs(ref.entropy)


@pytest.mark.parametrize("method,flags", [("chebyshev", 0), ("taylor", 0), ("chebyshev", ent.FLAG_CLENSHAW)])
@pytest.mark.parametrize("dist", ["rademacher", "gaussian"])
def test_band_schedules_and_probes(orc, method, flags, dist):
    n, m, s, seed = 20_000, 30, 96, 17
    csr = W.banded_density_csr(n, 8, seed=7)
    d = 0 if dist == "rademacher" else 1
    res, per, mom, band = run(csr, method, m, s, seed, probe_dist=dist, flags=flags | ent.FLAG_CSR_BANDED)
    ref = orc.estimate(csr, 0 if method == "taylor" else 1, m, s, seed, dist=d)
    err = per_probe_rel(per, ref)
    print(f"[band {method} flags={flags} {dist}] H gpu={res.entropy:.14f} oracle={ref.entropy:.14f} "
          f"per-probe rel {err:.2e}", flush=True)
    assert band == 16
    assert err <= TOL64
    assert res.std_err == pytest.approx(ref.std_err, rel=1e-8)
    if method == "chebyshev" and not flags:
        for j in (0, s // 2, s - 1):
            g = orc.probe_vector(seed, d, 0, n, j)
            dref = orc.cheb_moments_forward(csr, 0.0, ref.u, m, g)
            assert np.max(np.abs(mom[:, j] - dref)) <= TOL64 * float(g @ g)


@pytest.mark.parametrize("n,s", [(1, 1), (5, 3), (16, 64), (17, 65), (1000, 50), (4111, 130)])
def test_band_ragged(orc, n, s):
    # n below one 16-row block, exactly one, one plus a row; probe counts
    # below, at and above one 64-probe chunk
    csr = W.banded_density_csr(n, 4, seed=n + 3)
    m, seed = 11, 5
    res, per, _, band = run(csr, "chebyshev", m, s, seed, flags=ent.FLAG_CSR_BANDED)
    ref = orc.estimate(csr, 1, m, s, seed)
    err = per_probe_rel(per, ref)
    print(f"[band ragged n={n} s={s}] kernel band {band}; per-probe rel {err:.2e}", flush=True)
    assert band == (4 if n <= 5 else 8)
    assert err <= TOL64


def test_band_duplicates_and_empty_rows(orc):
    # duplicate (row, col) entries are summed; a zero row contributes nothing
    n, m, s, seed = 3000, 15, 64, 9
    rp, ci, val, _ = W.banded_density_csr(n, 2, seed=11)
    rows = np.repeat(np.arange(n), np.diff(rp))
    # split every diagonal entry into two halves stored twice
    diag = ci == rows
    val2 = np.concatenate([np.where(diag, val / 2, val), val[diag] / 2])
    ci2 = np.concatenate([ci, ci[diag]])
    rows2 = np.concatenate([rows, rows[diag]])
    order = np.argsort(rows2, kind="stable")
    ci2, val2, rows2 = ci2[order], val2[order], rows2[order]
    rp2 = np.zeros(n + 1, np.int64)
    np.add.at(rp2, rows2 + 1, 1)
    rp2 = np.cumsum(rp2)
    dup = (rp2, ci2.astype(np.int32), val2, n)
    res, per, _, band = run(dup, "chebyshev", m, s, seed, flags=ent.FLAG_CSR_BANDED)
    ref = orc.estimate((rp, ci, val, n), 1, m, s, seed)
    assert band == 4
    assert per_probe_rel(per, ref) <= TOL64
    # a matrix with empty rows (rank deficient, still unit trace)
    keep = (rows % 7) != 3
    ce = ((ci % 7) != 3) & keep
    rp3 = np.zeros(n + 1, np.int64)
    np.add.at(rp3, rows[ce] + 1, 1)
    rp3 = np.cumsum(rp3)
    v3 = val[ce] / val[ce][ci[ce] == rows[ce]].sum()
    z = (rp3, ci[ce].astype(np.int32), v3, n)
    res, per, _, band = run(z, "chebyshev", m, s, seed, flags=ent.FLAG_CSR_BANDED)
    ref = orc.estimate(z, 1, m, s, seed)
    assert band == 4
    assert per_probe_rel(per, ref) <= TOL64


def test_band_pack_unstaged_blocks(orc):
    # every entry stored 20 times (value / 20): 16-row blocks of 1600 entries,
    # more than the pack kernel stages in LDS, so it reads them from global
    # memory; the sums are the original matrix
    n, m, s, seed = 2000, 12, 64, 5
    rp, ci, val, _ = W.banded_density_csr(n, 2, seed=13)
    rep = 20
    rp2 = rp * rep
    ci2 = np.repeat(ci, rep).astype(np.int32)
    val2 = np.repeat(val / rep, rep)
    assert (rp2[16] - rp2[0]) > 1024
    res, per, _, band = run((rp2, ci2, val2, n), "chebyshev", m, s, seed, flags=ent.FLAG_CSR_BANDED)
    ref = orc.estimate((rp, ci, val, n), 1, m, s, seed)
    print(f"[band unstaged] per-probe rel {per_probe_rel(per, ref):.2e}", flush=True)
    assert band == 4
    assert per_probe_rel(per, ref) <= TOL64


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_band_matches_general_kernel(orc, dtype):
    n, m, s, seed = 30_000, 25, 64, 23
    csr = W.banded_density_csr(n, 8, seed=29, dtype=dtype)
    prec = "f64" if dtype == np.float64 else "f32"
    a = run(csr, "chebyshev", m, s, seed, precision=prec)
    b = run(csr, "chebyshev", m, s, seed, precision=prec, flags=ent.FLAG_CSR_GENERAL)
    assert a[3] == 16 and b[3] == 0
    tol = TOL64 if dtype == np.float64 else TOL_F32
    rel = float(np.max(np.abs(a[1] - b[1])) / np.mean(np.abs(b[1])))
    print(f"[band vs general {prec}] per-probe rel {rel:.2e}", flush=True)
    assert rel <= tol
    # repeated runs are bit-identical
    c = run(csr, "chebyshev", m, s, seed, precision=prec)
    assert np.array_equal(a[1], c[1])


def test_wider_band_runs_general_kernel(orc):
    # half-bandwidth 18 (> 16): the general CSR kernel
    n, m, s, seed = 4000, 12, 64, 3
    csr = W.banded_density_csr(n, 9, seed=31)
    res, per, _, band = run(csr, "chebyshev", m, s, seed)
    ref = orc.estimate(csr, 1, m, s, seed)
    assert band == 0
    assert per_probe_rel(per, ref) <= TOL64
    # asking for the banded kernels does not change that
    res2, per2, _, band2 = run(csr, "chebyshev", m, s, seed, flags=ent.FLAG_CSR_BANDED)
    assert band2 == 0
    assert np.array_equal(per, per2)


def test_default_kernel_choice_by_bytes(orc):
    # half-bandwidth 16 with 33 entries per row: slabs of 48 values per row
    # are smaller than the CSR arrays (FP32: 192 against 272 bytes), so the
    # banded kernels run by default; a tridiagonal R (3 entries per row) runs
    # the tridiagonal kernel, the general kernels or the slabs when asked
    n, m, s, seed = 20_000, 12, 64, 4
    csr = W.banded_density_csr(n, 8, seed=5, dtype=np.float32)
    assert run(csr, "chebyshev", m, s, seed, precision="f32")[3] == 16
    tri = W.poisson_csr_fast(n)
    res, per, _, band = run(tri, "chebyshev", m, s, seed)
    assert band == 1
    res1, per1, _, band1 = run(tri, "chebyshev", m, s, seed, flags=ent.FLAG_CSR_GENERAL)
    assert band1 == 0
    res2, per2, _, band2 = run(tri, "chebyshev", m, s, seed, flags=ent.FLAG_CSR_BANDED)
    assert band2 == 4
    ref = orc.estimate(tri, 1, m, s, seed)
    for p in (per, per1, per2):
        assert per_probe_rel(p, ref) <= TOL64


@pytest.mark.parametrize("method,flags", [("chebyshev", 0), ("taylor", 0), ("chebyshev", ent.FLAG_CLENSHAW)])
@pytest.mark.parametrize("dist", ["rademacher", "gaussian"])
def test_band_fp32_schedules_and_probes(orc, method, flags, dist):
    # FP32 values and products: stored Gaussian probe block or sign bits, every
    # schedule, three 64-probe chunks with a ragged last one
    n, m, s, seed = 12_345, 25, 150, 31
    csr = W.banded_density_csr(n, 8, seed=13, dtype=np.float32)
    d = 0 if dist == "rademacher" else 1
    res, per, _, band = run(csr, method, m, s, seed, precision="f32", probe_dist=dist,
                            flags=flags | ent.FLAG_CSR_BANDED)
    ref = orc.estimate(csr, 0 if method == "taylor" else 1, m, s, seed, dist=d)
    err = per_probe_rel(per, ref)
    rel = abs(res.entropy - ref.entropy) / abs(ref.entropy)
    print(f"[band f32 {method} flags={flags} {dist}] H gpu={res.entropy:.10f} oracle={ref.entropy:.10f} "
          f"rel {rel:.2e} per-probe rel {err:.2e}", flush=True)
    assert band == 16
    assert err <= TOL32 and rel <= TOL32


@pytest.mark.parametrize("n,s,m", [(1, 1, 3), (5, 3, 4), (16, 64, 5), (17, 65, 6), (1000, 50, 7), (4111, 130, 8)])
def test_band_two_step_launches(orc, monkeypatch, n, s, m):
    """FP32 banded R runs two recurrence steps per launch (the last step of
    an odd count alone): per-probe values against the FP64 oracle and against
    one launch per step (ENT_BAND_PAIRS=0), for every schedule, with sizes
    below, at and past one 16-row block and one 64-probe chunk, and odd and
    even step counts."""
    csr = W.banded_density_csr(n, 4, seed=n + 5, dtype=np.float32)
    seed = 3
    for method, flags in (("chebyshev", 0), ("taylor", 0), ("chebyshev", ent.FLAG_CLENSHAW)):
        for dist in ("rademacher", "gaussian"):
            kw = dict(precision="f32", probe_dist=dist, flags=flags | ent.FLAG_CSR_BANDED)
            ent.timing_enable(True)
            try:
                res, per, mom = ent.entropy_estimate_detail(csr_to_dev(csr), method, m, s, seed, **kw)
                t = ent.last_timing()
                monkeypatch.setenv("ENT_BAND_PAIRS", "0")
                res1, per1, mom1 = ent.entropy_estimate_detail(csr_to_dev(csr), method, m, s, seed, **kw)
                t1 = ent.last_timing()
                monkeypatch.delenv("ENT_BAND_PAIRS")
            finally:
                ent.timing_enable(False)
            ref = orc.estimate(csr, 0 if method == "taylor" else 1, m, s, seed, dist=0 if dist == "rademacher" else 1)
            e2, e1 = per_probe_rel(per, ref), per_probe_rel(per1, ref)
            print(f"[band pairs n={n} s={s} m={m} {method} flags={flags} {dist}] fused {t['steps_fused']} "
                  f"launches {t['step_launches']}; per-probe rel {e2:.2e} (one step per launch {e1:.2e})",
                  flush=True)
            assert t["csr_band"] == (4 if n <= 5 else 8) and t["steps_fused"] == 2 and t1["steps_fused"] == 1
            assert e2 <= TOL32 and e1 <= TOL32
            assert np.max(np.abs(mom - mom1)) <= TOL32 * max(1.0, float(np.max(np.abs(mom1))))


@pytest.mark.parametrize("hb,hp", [(1, 4), (3, 8), (8, 16)])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("n", [7, 33, 1000, 5003])
def test_band_power_fused(orc, monkeypatch, hb, hp, dtype, n):
    """After the first product, the power method's products on a banded R
    run up to ten per launch (ENT_POWER_FUSE; each product one 16-row block
    behind the one before, the middle products scaled by the previous Rayleigh
    quotient): p~1 against the oracle's power method and against one product
    per launch, for iteration counts that split evenly and unevenly, one and
    two trials, every padded band width, ranges of one block and of many."""
    csr = W.banded_density_csr(n, hb, seed=300 + hb, dtype=dtype)
    prec = "f64" if dtype == np.float64 else "f32"
    seed = 7
    for t, q in ((2, 1), (5, 2), (20, 1), (23, 2)):
        kw = dict(precision=prec, power_iters=t, power_trials=q, flags=ent.FLAG_CSR_BANDED)
        ref = orc.estimate(csr, 1, 4, 8, seed, t=t, q=q)
        ent.timing_enable(True)
        try:
            res, _, _ = ent.entropy_estimate_detail(csr_to_dev(csr), "chebyshev", 4, 8, seed, **kw)
            tl = ent.last_timing()
            monkeypatch.setenv("ENT_POWER_FUSE", "1")
            res1, _, _ = ent.entropy_estimate_detail(csr_to_dev(csr), "chebyshev", 4, 8, seed, **kw)
            tl1 = ent.last_timing()
        finally:
            monkeypatch.delenv("ENT_POWER_FUSE", raising=False)
            ent.timing_enable(False)
        print(f"[band power {prec} hb={hb} n={n} t={t} q={q}] p1 {res.p1_est:.15e} oracle {ref.p1_est:.15e} "
              f"one per launch {res1.p1_est:.15e}; launches {tl['power_launches']} / {tl1['power_launches']}",
              flush=True)
        h = min(2 * hb, n - 1)  # the half-bandwidth R = B B^T reaches at this n
        assert tl["csr_band"] == (4 if h <= 4 else (8 if h <= 8 else 16)) and (n < 17 or tl["csr_band"] == hp)
        assert tl["power_launches"] == q * (1 + -(-t // 10)) and tl1["power_launches"] == q * (t + 1)
        assert abs(res.p1_est - ref.p1_est) <= 1e-12 * ref.p1_est
        assert abs(res.p1_est - res1.p1_est) <= 1e-12 * res1.p1_est
