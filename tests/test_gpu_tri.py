"""GPU parity of the tridiagonal step kernel (a CSR R whose entries all lie
within one of the diagonal, such as the Poisson matrix of Section 6): which
kernel ran, per-probe values against the FP64 oracle for both precisions,
every schedule and probe distribution, ragged sizes and probe counts,
duplicate and missing entries, and agreement with the general CSR kernel on
the same input."""
import numpy as np
import pytest

import workloads as W
from tolerances import TOL64, TOL_F32

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1801_01072_amd as ent  # noqa: E402

DEV = "cuda:0"


def csr_to_dev(csr):
    rp, ci, val, n = csr
    return (torch.from_numpy(rp).to(DEV), torch.from_numpy(ci).to(DEV), torch.from_numpy(val).to(DEV), n)


def run(csr, method, m, s, seed, **kw):
    ent.timing_enable(True)
    try:
        res, per, mom = ent.entropy_estimate_detail(csr_to_dev(csr), method, m, s, seed, **kw)
        kern = ent.last_timing()["csr_band"]
    finally:
        ent.timing_enable(False)
    return res, per, mom, kern


def rel(per, ref):
    return float(np.max(np.abs(per - ref.per_probe)) / max(np.mean(np.abs(ref.per_probe)), 1e-2))


def random_tridiagonal(n, seed, dtype=np.float64):
    """R = B B^T / tr with B lower bidiagonal is pentadiagonal; a symmetric
    positive tridiagonal R instead: diagonally dominant, random off-diagonal."""
    rng = np.random.default_rng(seed)
    off = rng.uniform(-1.0, 1.0, size=max(n - 1, 0))
    diag = np.abs(np.concatenate([[0.0], off])) + np.abs(np.concatenate([off, [0.0]])) + rng.uniform(0.1, 1.0, n)
    tr = diag.sum()
    rows, cols, vals = [], [], []
    for i in range(n):
        for j, v in ((i - 1, off[i - 1] if i > 0 else 0.0), (i, diag[i]), (i + 1, off[i] if i < n - 1 else 0.0)):
            if 0 <= j < n:
                rows.append(i)
                cols.append(j)
                vals.append(v / tr)
    rp = np.zeros(n + 1, np.int64)
    np.add.at(rp, np.array(rows) + 1, 1)
    return np.cumsum(rp), np.array(cols, np.int32), np.array(vals, dtype), n


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("method,flags", [("chebyshev", 0), ("taylor", 0), ("chebyshev", ent.FLAG_CLENSHAW)])
@pytest.mark.parametrize("dist", ["rademacher", "gaussian"])
def test_tri_schedules_probes_precisions(orc, dtype, method, flags, dist):
    n, m, s, seed = 30_001, 25, 96, 13
    csr = random_tridiagonal(n, 3, dtype)
    prec = "f64" if dtype == np.float64 else "f32"
    d = 0 if dist == "rademacher" else 1
    res, per, mom, kern = run(csr, method, m, s, seed, probe_dist=dist, precision=prec, flags=flags)
    ref = orc.estimate(csr, 0 if method == "taylor" else 1, m, s, seed, dist=d)
    err = rel(per, ref)
    print(f"[tri {prec} {method} flags={flags} {dist}] kernel {kern}; H gpu={res.entropy:.12f} "
          f"oracle={ref.entropy:.12f} per-probe rel {err:.2e}", flush=True)
    assert kern == 1
    assert err <= (TOL64 if dtype == np.float64 else TOL_F32)
    if dtype == np.float64:
        assert abs(res.entropy - ref.entropy) <= TOL64 * abs(ref.entropy)
        if method == "chebyshev" and not flags:
            for j in (0, s - 1):
                g = orc.probe_vector(seed, d, 0, n, j)
                dref = orc.cheb_moments_forward(csr, 0.0, ref.u, m, g)
                assert np.max(np.abs(mom[:, j] - dref)) <= TOL64 * float(g @ g)


@pytest.mark.parametrize("n,s", [(1, 1), (2, 3), (3, 64), (5, 65), (33, 100), (1000, 130), (4097, 50), (999, 256), (1000, 300)])
def test_tri_ragged(orc, n, s):
    # n of one, two or a few rows (streams with no rows, with one row, with
    # an odd count); probe counts for each stream width (16 lanes up to 64
    # probes, 32 up to 128, 64 up to 256, then 64-probe passes over rows of
    # 64-multiple length), at and past each width's edge
    csr = W.poisson_csr(n) if n > 1 else (np.array([0, 1], np.int64), np.array([0], np.int32), np.ones(1), 1)
    m, seed = 9, 7
    for dist in ("rademacher", "gaussian"):
        d = 0 if dist == "rademacher" else 1
        res, per, _, kern = run(csr, "chebyshev", m, s, seed, probe_dist=dist)
        ref = orc.estimate(csr, 1, m, s, seed, dist=d)
        err = rel(per, ref)
        print(f"[tri ragged n={n} s={s} {dist}] kernel {kern}; per-probe rel {err:.2e}", flush=True)
        assert kern == 1
        assert err <= TOL64


def test_tri_duplicates_missing_entries_and_general_agreement(orc):
    # rows with no coupling to their neighbours (a block-diagonal tridiagonal
    # R), duplicate diagonal entries (summed; within the 3n entries that make
    # a tridiagonal candidate) and an all-diagonal R run the tridiagonal
    # kernel; the general CSR kernel agrees on each
    n, m, s, seed = 5000, 15, 64, 21
    rp, ci, val, _ = random_tridiagonal(n, 9)
    rows = np.repeat(np.arange(n), np.diff(rp))
    # cut the coupling between rows 99 and 100, 199 and 200, ...
    keep = ~((np.abs(ci - rows) == 1) & ((np.minimum(ci, rows) % 100) == 99))
    ci, val, rows = ci[keep], val[keep], rows[keep]

    def build(r, c, v):
        order = np.argsort(r, kind="stable")
        ptr = np.zeros(n + 1, np.int64)
        np.add.at(ptr, r[order] + 1, 1)
        return np.cumsum(ptr), c[order].astype(np.int32), v[order], n

    cut = build(rows, ci, val)
    # the diagonal entry of every 100th row stored as two halves
    twice = (ci == rows) & (rows % 100 == 0)
    dup = build(np.concatenate([rows, rows[twice]]), np.concatenate([ci, ci[twice]]),
                np.concatenate([np.where(twice, val / 2, val), val[twice] / 2]))
    assert dup[0][-1] <= 3 * n
    p = np.random.default_rng(2).uniform(0.5, 1.5, n)
    p /= p.sum()
    dg = (np.arange(n + 1, dtype=np.int64), np.arange(n, dtype=np.int32), p, n)
    for name, csr, base in (("cut", cut, cut), ("duplicates", dup, cut), ("diagonal", dg, dg)):
        res, per, _, kern = run(csr, "chebyshev", m, s, seed)
        res_g, per_g, _, kern_g = run(csr, "chebyshev", m, s, seed, flags=ent.FLAG_CSR_GENERAL)
        ref = orc.estimate(base, 1, m, s, seed)
        print(f"[tri {name}] kernel {kern} / {kern_g}; per-probe rel {rel(per, ref):.2e} "
              f"(general {rel(per_g, ref):.2e})", flush=True)
        assert kern == 1 and kern_g == 0
        assert rel(per, ref) <= TOL64 and rel(per_g, ref) <= TOL64


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("n,s,m", [(1, 1, 3), (2, 3, 4), (7, 64, 5), (33, 100, 6), (4097, 130, 7),
                                   (1000, 100, 10)])
def test_tri_fused_launches(orc, monkeypatch, dtype, n, s, m):
    """A tridiagonal R runs several recurrence steps per launch
    (ENT_TRI_FUSE = 1..10, the steps split as evenly as possible, a launch of
    one step on the single-step kernel): per-probe values against the FP64
    oracle and moments against one launch per step, for every schedule and
    probe kind, streams with no rows, one row and a few."""
    csr = W.poisson_csr(n, dtype) if n > 1 else (np.array([0, 1], np.int64), np.array([0], np.int32),
                                                 np.ones(1, dtype), 1)
    prec = "f64" if dtype == np.float64 else "f32"
    tol = TOL64 if dtype == np.float64 else TOL_F32
    seed = 5

    def first_launch(nsteps, nf):
        nl = -(-nsteps // nf)
        return nsteps // nl + (1 if nsteps % nl else 0)

    for method, flags in (("chebyshev", 0), ("taylor", 0), ("chebyshev", ent.FLAG_CLENSHAW)):
        nsteps = m if (method == "chebyshev" and not flags) else m + 1
        ref = orc.estimate(csr, 0 if method == "taylor" else 1, m, s, seed, dist=0)
        for dist in ("rademacher", "gaussian"):
            kw = dict(precision=prec, probe_dist=dist, flags=flags)
            if dist == "gaussian":
                ref = orc.estimate(csr, 0 if method == "taylor" else 1, m, s, seed, dist=1)
            out = {}
            ent.timing_enable(True)
            try:
                for nf in (1, 2, 3, 5, 10):
                    monkeypatch.setenv("ENT_TRI_FUSE", str(nf))
                    res, per, mom = ent.entropy_estimate_detail(csr_to_dev(csr), method, m, s, seed, **kw)
                    out[nf] = (per, mom, ent.last_timing())
            finally:
                monkeypatch.delenv("ENT_TRI_FUSE")
                ent.timing_enable(False)
            mom1 = out[1][1]
            for nf, (per, mom, t) in out.items():
                e = rel(per, ref)
                print(f"[tri fused {prec} n={n} s={s} m={m} {method} flags={flags} {dist} nf={nf}] "
                      f"fused {t['steps_fused']} launches {t['step_launches']}; per-probe rel {e:.2e}", flush=True)
                want = 1 if nf == 1 else first_launch(nsteps, nf)
                assert t["csr_band"] == 1 and t["steps_fused"] == want
                assert e <= tol
                assert np.max(np.abs(mom - mom1)) <= tol * max(1.0, float(np.max(np.abs(mom1))))


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("n", [1, 2, 7, 63, 64, 65, 130, 4097])
def test_tri_power_fused(orc, monkeypatch, dtype, n):
    """After the first product, the power method's products on a tridiagonal
    R run up to ten per launch (ENT_POWER_FUSE; the middle products
    scaled by the previous Rayleigh quotient, not normalised): p~1 against
    the oracle's power method and against one product per launch, for
    iteration counts that split evenly and unevenly, one and two trials,
    tiles that the rows fill, overrun and leave nearly empty."""
    csr = random_tridiagonal(n, 11, dtype)
    prec = "f64" if dtype == np.float64 else "f32"
    seed = 3
    for t, q in ((1, 1), (2, 1), (5, 2), (20, 1), (23, 2)):
        kw = dict(precision=prec, power_iters=t, power_trials=q)
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
        nl = -(-t // 10) if t >= 2 else t
        print(f"[tri power {prec} n={n} t={t} q={q}] p1 {res.p1_est:.15e} oracle {ref.p1_est:.15e} "
              f"one per launch {res1.p1_est:.15e}; launches {tl['power_launches']} / {tl1['power_launches']}",
              flush=True)
        assert tl["csr_band"] == 1
        assert tl["power_launches"] == q * (1 + nl) and tl1["power_launches"] == q * (t + 1)
        assert abs(res.p1_est - ref.p1_est) <= 1e-12 * ref.p1_est
        assert abs(res.p1_est - res1.p1_est) <= 1e-12 * res1.p1_est


def test_tri_csr_structure_rejected():
    """Malformed short-row CSR input (at most three entries per row: the
    one-pass row check that also measures the half-bandwidth) is refused
    before any kernel reads it: a column index of n or -1, row pointers out of
    order, a first row pointer of 1, an nnz that row_ptr does not end at.  The
    well-formed matrix goes through the tridiagonal kernel."""
    n = 100
    rp, ci, val, _ = W.poisson_csr(n, np.float64)
    ci = ci.astype(np.int32)

    def attempt(rp_, ci_, val_, nnz=None):
        M = ent.csr_matrix(torch.from_numpy(rp_).to(DEV), torch.from_numpy(ci_).to(DEV),
                           torch.from_numpy(val_).to(DEV), n)
        if nnz is not None:
            M.nnz = nnz
        return ent.entropy_estimate(M, "chebyshev", 8, 8, 1)

    _, _, _, kern = run((rp, ci, val, n), "chebyshev", 8, 8, 1)
    assert kern == 1
    bad = []
    c = ci.copy(); c[len(c) // 2] = n; bad.append((rp, c, val, None))
    c = ci.copy(); c[7] = -1; bad.append((rp, c, val, None))
    r = rp.copy(); r[10], r[11] = r[11], r[10]; bad.append((r, ci, val, None))
    r = rp.copy(); r[0] = 1; bad.append((r, ci, val, None))
    bad.append((rp, ci, val, len(ci) - 1))
    for k, (r_, c_, v_, nnz) in enumerate(bad):
        with pytest.raises(ent.EntropyError) as e:
            attempt(r_, c_, v_, nnz)
        print(f"[tri structure {k}] {e.value}", flush=True)
        assert e.value.status == ent.EINVAL, k
        assert "CSR structure" in str(e.value), k
