"""Pins for the oracle's estimators (Algorithms 1, 2, 4 and Lemmas 1, 2, 5)
against closed forms, invariants and brute force."""
import itertools
import math

import numpy as np
import pytest
from numpy.polynomial import chebyshev as C

import workloads as W


def shannon(p):
    p = p[p > 0]
    return float(-np.sum(p * np.log(p)))


# ---------------------------------------------------------------- matvec ----
def test_matvec_dense_and_csr_against_numpy(orc):
    rng = np.random.default_rng(1)
    A = rng.standard_normal((37, 37))
    x = rng.standard_normal(37)
    assert np.allclose(orc.matvec(A, x), A @ x, rtol=1e-14, atol=1e-14)
    A32 = A.astype(np.float32)
    assert np.allclose(orc.matvec(A32, x), A32.astype(np.float64) @ x, rtol=1e-14, atol=1e-13)
    csr = W.banded_density_csr(50, 3, seed=2)
    D = W.csr_to_dense(csr)
    x = rng.standard_normal(50)
    assert np.allclose(orc.matvec(csr, x), D @ x, rtol=1e-13, atol=1e-18)


def test_banded_generator_structure():
    n, hb = 300, 8
    csr = W.banded_density_csr(n, hb, seed=4)
    rp, ci, val, _ = csr
    assert rp[-1] == 33 * n - 272
    D = W.csr_to_dense(csr)
    assert np.array_equal(D, D.T)
    assert abs(np.trace(D) - 1.0) < 1e-13
    assert np.linalg.eigvalsh(D).min() > -1e-15


# ---------------------------------------------------------- power method ----
def test_power_method_maximally_mixed(orc):
    n = 64
    assert orc.power_method(W.maximally_mixed(n), t=20, q=1, seed=3) == pytest.approx(1.0 / n, rel=1e-14)


def test_power_method_diagonal_closed_form(orc):
    # x0 in {+-1}^n, R = diag(p): RQ(x_t) = sum p^(2t+1) / sum p^(2t)
    p = W.spectrum_inverse(30)
    for t in (1, 3, 20):
        want = np.sum(p ** (2 * t + 1)) / np.sum(p ** (2 * t))
        assert orc.power_method(np.diag(p), t=t, q=1, seed=9) == pytest.approx(want, rel=1e-13)


def test_power_method_rayleigh_bound_and_lemma5(orc):
    n = 120
    p = W.spectrum_exp(n, 30.0)
    R = W.dense_density(p, 11)
    for seed in range(5):
        est = orc.power_method(R, t=20, q=2, seed=seed)
        assert est <= p[0] * (1 + 1e-12)          # Rayleigh quotient never exceeds p_1
        assert est >= p[0] / 6.0                  # Lemma 5, holds with high probability


# ---------------------------------------------------------------- Taylor ----
def taylor_diag_closed_form(p, u, m):
    k = np.arange(1, m + 1)
    return math.log(1.0 / u) + float(np.sum(p[:, None] * (1 - p[:, None] / u) ** k[None, :] / k[None, :]))


def test_taylor_diagonal_rademacher_is_deterministic(orc):
    p = W.spectrum_inverse(50)
    u, m = 1.0, 25
    est = orc.estimate(np.diag(p), 0, m, 8, seed=1, u_override=u)
    assert np.allclose(est.per_probe, taylor_diag_closed_form(p, u, m), rtol=1e-13)


def test_taylor_maximally_mixed_c6(orc):
    n, m = 40, 30
    est = orc.estimate(W.maximally_mixed(n), 0, m, 4, seed=2, c=6.0)
    assert est.p1_est == pytest.approx(1.0 / n, rel=1e-14)
    want = math.log(n / 6.0) + sum((5.0 / 6.0) ** k / k for k in range(1, m + 1))
    assert est.entropy == pytest.approx(want, rel=1e-12)


def test_taylor_pure_state_is_zero(orc):
    R = W.pure_state(32, 5)
    est = orc.estimate(R, 0, 20, 6, seed=3, c=6.0)
    assert est.u == 1.0
    assert abs(est.entropy) < 1e-12


def test_taylor_series_converges_to_entropy(orc):
    # Lemma 2: on a positive definite R the full series equals H; truncation
    # error after m terms is at most (1 - l/u)^m H (proof of Theorem 1)
    p = np.linspace(1.0, 3.0, 25)
    p /= p.sum()
    u = 1.05 * p.max()
    H = shannon(p)
    for m in (5, 50, 400):
        est = orc.estimate(np.diag(p), 0, m, 2, seed=0, u_override=u)
        assert abs(est.entropy - H) <= (1 - p.min() / u) ** m * H * (1 + 1e-9) + 1e-14
    assert est.entropy == pytest.approx(H, rel=1e-12)


def test_taylor_literal_equals_dense_algebra(orc):
    n, m = 30, 12
    R = W.dense_density(W.spectrum_inverse(n), 6)
    u = 0.7
    g = orc.probe_vector(4, 1, 0, n, 2)
    Cm = np.eye(n) - R / u
    want = sum(g @ R @ np.linalg.matrix_power(Cm, k) @ g / k for k in range(1, m + 1))
    assert orc.taylor_quadform(R, u, m, g) == pytest.approx(want, rel=1e-12)


# ------------------------------------------------------------- Chebyshev ----
def test_chebyshev_diagonal_rademacher(orc):
    p = W.spectrum_exp(64, 10.0)
    m = 30
    est = orc.estimate(np.diag(p), 1, m, 5, seed=7, c=6.0)
    u = est.u
    want = -np.sum(C.chebval(2 * p / u - 1, orc.cheb_coeffs(u, m)))
    assert np.allclose(est.per_probe, want, rtol=1e-13)
    # NTE bound of the proof of Theorem 2: |H - tr(-f_m(R))| <= n u / (2 m^2)
    assert abs(want - shannon(p)) <= len(p) * u / (2 * m * m)


def test_chebyshev_zero_eigenvalues_add_exact_bias(orc):
    # each zero eigenvalue contributes -f_m(0) = u / (2 m (m+1))
    p = np.zeros(20)
    p[:5] = [0.4, 0.3, 0.15, 0.1, 0.05]
    m, u = 10, 1.0
    est_full = orc.estimate(np.diag(p), 1, m, 1, seed=1, u_override=u)
    est_nz = orc.estimate(np.diag(p[:5]), 1, m, 1, seed=1, u_override=u)
    assert est_full.entropy - est_nz.entropy == pytest.approx(15 * u / (2 * m * (m + 1)), rel=1e-12)


def test_chebyshev_maximally_mixed_and_pure(orc):
    n, m = 48, 20
    est = orc.estimate(W.maximally_mixed(n), 1, m, 3, seed=4, c=6.0)
    u = 6.0 / n
    want = -n * C.chebval(2 * (1.0 / n) / u - 1, orc.cheb_coeffs(u, m))
    assert est.entropy == pytest.approx(want, rel=1e-12)
    assert abs(est.entropy - math.log(n)) <= n * u / (2 * m * m)


@pytest.mark.parametrize("method", [0, 1])
def test_hutchinson_unbiased_by_enumeration(orc, method):
    # Lemma 1 with Rademacher vectors: the average of g^T A g over all 2^n sign
    # vectors is exactly tr(A).  Here A is the Taylor or Chebyshev polynomial
    # in R, whose trace follows from the known spectrum.
    n, m = 10, 8
    p = W.spectrum_inverse(n)
    R = W.dense_density(p, 12)
    u = 1.3 * p[0]
    if method == 1:
        a = orc.cheb_coeffs(u, m)
        tr = float(np.sum(C.chebval(2 * p / u - 1, a)))
    else:
        k = np.arange(1, m + 1)
        tr = float(np.sum(p[:, None] * (1 - p[:, None] / u) ** k / k))
    acc = 0.0
    for signs in itertools.product((1.0, -1.0), repeat=n):
        g = np.array(signs)
        acc += (orc.cheb_quadform(R, a, 0.0, u, g) if method == 1 else orc.taylor_quadform(R, u, m, g))
    assert acc / 2 ** n == pytest.approx(tr, rel=1e-12)


def test_gaussian_probes_sample_mean_within_error(orc):
    # Lemma 1 with Gaussian probes: mean over many probes within a few standard errors
    n, m = 50, 20
    p = W.spectrum_exp(n, 8.0)
    R = W.dense_density(p, 13)
    est = orc.estimate(R, 1, m, 400, seed=21, dist=1, c=6.0)
    u = est.u
    tr = -float(np.sum(C.chebval(2 * p / u - 1, orc.cheb_coeffs(u, m))))
    assert abs(est.entropy - tr) < 5 * est.std_err


def test_probe_subset_matches_full_run_and_thread_count(orc):
    n = 40
    R = W.dense_density(W.spectrum_inverse(n), 14)
    full = orc.estimate(R, 1, 15, 12, seed=5, dist=1)
    sub = orc.estimate(R, 1, 15, 12, seed=5, dist=1, probes=[3, 7, 11])
    assert np.array_equal(sub.per_probe, full.per_probe[[3, 7, 11]])
    assert full.entropy == pytest.approx(np.mean(full.per_probe), rel=1e-15)
    se = np.std(full.per_probe, ddof=1) / math.sqrt(12)
    assert full.std_err == pytest.approx(se, rel=1e-12)


def test_estimators_accept_fp32_storage(orc):
    n = 32
    R = W.dense_density(W.spectrum_inverse(n), 15)
    R32 = R.astype(np.float32)
    a = orc.estimate(R32, 1, 10, 4, seed=1)
    b = orc.estimate(R32.astype(np.float64), 1, 10, 4, seed=1)
    assert a.entropy == b.entropy
