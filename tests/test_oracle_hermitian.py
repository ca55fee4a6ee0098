"""Pins for the oracle's Hermitian estimators (Section 4, Algorithms 1c / 2c)
against the mathematics: real matrices given as complex reduce to the pinned
real oracle; with the canonical basis as probes, sum_i e_i^T Re[f_m(R)] e_i is
the trace of f_m(R), i.e. f_m summed over the eigenvalues, for a genuinely
complex R; the complex power method reaches lambda_max; Clenshaw and the
forward recurrence agree."""
import math

import numpy as np
import pytest

import workloads as W


def phased(R_real, seed):
    """D R D^H with a random diagonal unitary D: complex entries, same spectrum."""
    rng = np.random.default_rng(seed)
    ph = np.exp(1j * rng.uniform(0, 2 * np.pi, R_real.shape[0]))
    return (ph[:, None] * R_real) * ph.conj()[None, :]


@pytest.mark.parametrize("method", [0, 1])
def test_real_input_as_complex_matches_real_oracle(orc, method):
    n, m, s, seed = 40, 9, 6, 3
    p = W.spectrum_exp(n, 6.0)
    R = W.dense_density(p, 21)
    for dist in (0, 1):
        ref = orc.estimate(R, method, m, s, seed, dist=dist, u_override=0.7)
        z = orc.zestimate(R.astype(np.complex128), method, m, s, seed, dist=dist, u_override=0.7)
        assert np.max(np.abs(z.per_probe - ref.per_probe)) <= 1e-13 * np.max(np.abs(ref.per_probe))


def test_basis_probe_traces_equal_eigenvalue_sums(orc):
    n, m, u = 24, 12, 1.0
    p = W.spectrum_power(n, 1.0)
    R = W.hermitian_density(p, 5)
    assert np.max(np.abs(R.imag)) > 1e-3          # genuinely complex
    lam = np.linalg.eigvalsh(R)
    alpha = orc.cheb_coeffs(u, m)
    tr_cheb = sum(orc.zcheb_quadform(R, alpha, 0.0, u, np.eye(n)[i]) for i in range(n))
    want = sum(orc.cheb_eval_scalar(alpha, 0.0, u, x) for x in lam)
    assert tr_cheb == pytest.approx(want, rel=1e-12, abs=1e-14)
    # Taylor (Algorithm 1c, u = 1): sum_k sum_i lambda_i (1 - lambda_i)^k / k
    tr_tay = sum(orc.ztaylor_quadform(R, u, m, np.eye(n)[i]) for i in range(n))
    want_t = sum(x * (1 - x) ** k / k for x in lam for k in range(1, m + 1))
    assert tr_tay == pytest.approx(want_t, rel=1e-12)


def test_phases_change_quadratic_forms_but_not_traces(orc):
    # a dropped imaginary part would leave the per-probe value of the phased
    # matrix equal to the real one; the trace (basis probes) must not move
    n, m = 20, 8
    R0 = W.dense_density(W.spectrum_exp(n, 5.0), 4)
    R1 = phased(R0, 9)
    alpha = orc.cheb_coeffs(1.0, m)
    g = orc.probe_vector(7, 1, 0, n, 0)
    q0 = orc.cheb_quadform(R0, alpha, 0.0, 1.0, g)
    q1 = orc.zcheb_quadform(R1, alpha, 0.0, 1.0, g)
    # the phased form is g^T Re[D f(R0) D^H] g: check it against that product
    lam, V = np.linalg.eigh(R0)
    fl = np.array([orc.cheb_eval_scalar(alpha, 0.0, 1.0, x) for x in lam])
    FR0 = (V * fl[None, :]) @ V.T
    rng = np.random.default_rng(9)
    d = np.exp(1j * rng.uniform(0, 2 * np.pi, n))
    want = float(g @ np.real((d[:, None] * FR0) * d.conj()[None, :]) @ g)
    assert q1 == pytest.approx(want, rel=1e-11)
    assert abs(q1 - q0) > 1e-6 * abs(q0)
    tr0 = sum(orc.cheb_quadform(R0, alpha, 0.0, 1.0, np.eye(n)[i]) for i in range(n))
    tr1 = sum(orc.zcheb_quadform(R1, alpha, 0.0, 1.0, np.eye(n)[i]) for i in range(n))
    assert tr1 == pytest.approx(tr0, rel=1e-12)


def test_forward_moments_match_clenshaw(orc):
    n, m, lo, u = 30, 15, 0.0, 1.0
    R = W.hermitian_density(W.spectrum_exp(n, 4.0), 8)
    g = orc.probe_vector(3, 1, 0, n, 2)
    alpha = orc.cheb_coeffs(u, m)
    d = orc.zcheb_moments_forward(R, lo, u, m, g)
    assert d[0] == pytest.approx(float(g @ g), rel=1e-15)
    # sum_k alpha_k d_k = g^T Re[f_m(R)] g
    assert float(alpha @ d) == pytest.approx(orc.zcheb_quadform(R, alpha, lo, u, g), rel=1e-12)
    # against an explicit T_k(X) from the eigen-decomposition
    lam, V = np.linalg.eigh(R)
    t = np.clip(2 * lam / u - 1, -1, 1)
    for k in (0, 1, 2, 7, m):
        Tk = (V * np.cos(k * np.arccos(t))[None, :]) @ V.conj().T
        assert d[k] == pytest.approx(float(g @ np.real(Tk) @ g), rel=1e-11, abs=1e-12)


def test_complex_power_method_reaches_lambda_max(orc):
    n = 50
    p = W.spectrum_exp(n, 3.0)
    R = W.hermitian_density(p, 13)
    lam = np.linalg.eigvalsh(R)
    p1 = orc.zpower_method(R, t=300, q=1, seed=4)
    assert p1 == pytest.approx(lam[-1], rel=1e-12)
    # Rayleigh quotients never exceed lambda_max
    for t in (1, 5, 20):
        assert orc.zpower_method(R, t=t, q=2, seed=4) <= lam[-1] * (1 + 1e-14)


def test_estimate_is_close_to_exact_entropy(orc):
    # Algorithm 2c with u = 1 at a degree whose truncation error is small for this spectrum
    n, m, s = 64, 60, 200
    p = W.spectrum_exp(n, 10.0)
    R = W.hermitian_density(p, 17)
    H = float(-np.sum(p * np.log(p)))
    est = orc.zestimate(R, 1, m, s, 5)
    assert est.u == 1.0
    assert abs(est.entropy - H) <= 4 * est.std_err + 0.01 * H


def test_complex64_storage_widens_exactly(orc):
    n, m, s = 16, 6, 3
    R = W.hermitian_density(W.spectrum_exp(n, 3.0), 2, dtype=np.complex64)
    a = orc.zestimate(R, 1, m, s, 1)
    b = orc.zestimate(R.astype(np.complex128), 1, m, s, 1)
    assert np.array_equal(a.per_probe, b.per_probe)
