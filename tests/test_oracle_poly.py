"""Pins for the oracle's Chebyshev machinery (Lemma 3, Appendix B) against the
mathematics: a numerical Chebyshev projection of x ln x, the trigonometric
definition of T_w, numpy's Chebyshev-series evaluator, and the tight
truncation bound at x = 0."""
import math

import numpy as np
import pytest
from numpy.polynomial import chebyshev as C


def h(x):
    x = np.asarray(x, dtype=np.float64)
    return np.where(x > 0, x * np.log(np.where(x > 0, x, 1.0)), 0.0)


@pytest.mark.parametrize("u", [1.0, 0.37, 6.0 / 8192])
def test_closed_form_coefficients_match_projection(orc, u):
    # alpha_w = (2/pi) int_0^pi h(u (1 + cos th)/2) cos(w th) dth  (alpha_0 halved),
    # evaluated by Gauss-Chebyshev quadrature with many nodes.
    m, N = 30, 1 << 16
    th = math.pi * (np.arange(N) + 0.5) / N
    hx = h(0.5 * u * (1.0 + np.cos(th)))
    proj = np.array([2.0 / N * np.sum(hx * np.cos(w * th)) for w in range(m + 1)])
    proj[0] *= 0.5
    alpha = orc.cheb_coeffs(u, m)
    assert np.max(np.abs(alpha - proj)) < 1e-13 * u


def test_coefficient_values_spelled_out(orc):
    u = 0.5
    a = orc.cheb_coeffs(u, 4)
    assert a[0] == pytest.approx(u / 2 * (math.log(u / 4) + 1), rel=1e-15)
    assert a[1] == pytest.approx(u / 4 * (2 * math.log(u / 4) + 3), rel=1e-15)
    assert a[2] == pytest.approx(u / 6, rel=1e-15)        # (+1) u / (8 - 2)
    assert a[3] == pytest.approx(-u / 24, rel=1e-15)      # (-1) u / (27 - 3)
    assert a[4] == pytest.approx(u / 60, rel=1e-15)       # (+1) u / (64 - 4)


@pytest.mark.parametrize("m", [5, 30, 50])
def test_value_at_zero_and_tight_bound(orc, m):
    # f_m(0) = sum_w (-1)^w alpha_w = -u / (2 m (m+1)): the Lemma 3 bound is attained at x = 0
    u = 0.8
    a = orc.cheb_coeffs(u, m)
    f0 = orc.cheb_eval_scalar(a, 0.0, u, 0.0)
    assert f0 == pytest.approx(-u / (2 * m * (m + 1)), rel=1e-12)
    xs = np.linspace(0.0, u, 2001)
    err = np.array([abs(x * math.log(x) - orc.cheb_eval_scalar(a, 0.0, u, x)) if x > 0
                    else abs(orc.cheb_eval_scalar(a, 0.0, u, x)) for x in xs])
    assert err.max() <= u / (2 * m * (m + 1)) * (1 + 1e-9)
    assert err.argmax() == 0


def test_scalar_clenshaw_matches_trig_definition(orc):
    # T_w(x) = cos(w arccos(2x/u - 1)) (Section 3) and numpy's series evaluator
    u, m = 0.6, 25
    rng = np.random.default_rng(0)
    alpha = rng.standard_normal(m + 1)
    for x in rng.uniform(0, u, 50):
        t = 2 * x / u - 1
        trig = sum(alpha[w] * math.cos(w * math.acos(t)) for w in range(m + 1))
        assert orc.cheb_eval_scalar(alpha, 0.0, u, x) == pytest.approx(trig, abs=1e-12)
        assert orc.cheb_eval_scalar(alpha, 0.0, u, x) == pytest.approx(C.chebval(t, alpha), abs=1e-12)


def test_scalar_clenshaw_general_interval(orc):
    lo, u, m = 0.1, 0.9, 12
    alpha = np.arange(1.0, m + 2)
    for x in np.linspace(lo, u, 7):
        t = (2 * x - (u + lo)) / (u - lo)
        assert orc.cheb_eval_scalar(alpha, lo, u, x) == pytest.approx(C.chebval(t, alpha), rel=1e-13)


def test_quadform_on_diagonal_with_signs_is_exact_trace(orc):
    # With g in {+-1}^n and R = diag(p): g^T f(R) g = sum_i f(p_i)
    import workloads as W

    p = W.spectrum_exp(40, 7.0)
    u, m = 1.2 * p[0], 20
    a = orc.cheb_coeffs(u, m)
    g = orc.probe_vector(5, 0, 0, 40, 3)
    want = np.sum(C.chebval(2 * p / u - 1, a))
    got = orc.cheb_quadform(np.diag(p), a, 0.0, u, g)
    assert got == pytest.approx(want, rel=1e-13)
    # same through CSR storage
    got_csr = orc.cheb_quadform(W.diag_csr(p), a, 0.0, u, g)
    assert got_csr == pytest.approx(want, rel=1e-13)


def test_clenshaw_equals_forward_recurrence(orc):
    import workloads as W

    n, m = 60, 30
    R = W.dense_density(W.spectrum_inverse(n), 3)
    u = 0.9
    a = orc.cheb_coeffs(u, m)
    g = orc.probe_vector(8, 1, 0, n, 0)
    d = orc.cheb_moments_forward(R, 0.0, u, m, g)
    assert d[0] == pytest.approx(g @ g, rel=1e-15)
    # moments of a matrix with spectrum in [-1, 1] are bounded by ||g||^2
    assert np.all(np.abs(d) <= (g @ g) * (1 + 1e-12))
    assert float(a @ d) == pytest.approx(orc.cheb_quadform(R, a, 0.0, u, g), rel=1e-12)


def test_interp_coefficients(orc):
    # exact interpolation at the N = m+1 Chebyshev nodes of [lo, u]
    lo, u, m = 1e-3, 0.05, 16
    c = orc.cheb_interp_coeffs(lo, u, m)
    N = m + 1
    th = math.pi * (np.arange(N) + 0.5) / N
    x = 0.5 * (u + lo) + 0.5 * (u - lo) * np.cos(th)
    assert np.allclose(C.chebval(np.cos(th), c), x * np.log(x), rtol=0, atol=1e-15)
    # lo = 0 with many nodes reproduces the closed form of Lemma 3
    cc = orc.cheb_interp_coeffs(0.0, u, m, 1 << 15)
    assert np.max(np.abs(cc - orc.cheb_coeffs(u, m))) < 1e-12 * u


def test_cutoff_coefficients_are_nested_projection(orc):
    # the estimator's lower-cutoff coefficients do not depend on the degree
    lo, u = 2e-3, 0.4
    a20 = orc.cheb_interp_coeffs(lo, u, 20, orc.cutoff_nodes(20))
    a50 = orc.cheb_interp_coeffs(lo, u, 50, orc.cutoff_nodes(50))
    assert np.array_equal(a20, a50[:21])
    # and converge geometrically (x ln x is analytic on [lo, u] for lo > 0)
    assert abs(a50[50]) < 1e-6 * abs(a50[1])
    # truncation error on [lo, u] is bounded by the tail of the series (|T_w| <= 1)
    a200 = orc.cheb_interp_coeffs(lo, u, 200, orc.cutoff_nodes(200))
    tail = float(np.sum(np.abs(a200[51:])))
    xs = np.linspace(lo, u, 500)
    err = max(abs(orc.cheb_eval_scalar(a50, lo, u, x) - x * math.log(x)) for x in xs)
    assert err <= 1.01 * tail + 1e-15
