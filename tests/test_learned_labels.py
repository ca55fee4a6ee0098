"""The selector's training labels against the FP64 oracle.

A label (ln m*, log10(lo*/u)) claims that the polynomial trace -sum_i f_m(p_i)
with the Chebyshev approximation of x ln x on [lo*, u] (closed form of
Lemma 3 for lo* = 0, the lower-cutoff projection otherwise) is within the
target relative error of the exact entropy at m = m*, and, for lo* = 0, that
no smaller degree >= 4 is.  Both claims are re-checked here with the
oracle's coefficients and its Clenshaw evaluation of g^T f(R) g on diag(p)
with a sign probe, which equals sum_i f(p_i) exactly."""
import math

import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")

from paper_1801_01072_amd import learned as L  # noqa: E402


def poly_trace(orc, p, lo, u, m):
    if lo > 0:
        a = orc.cheb_interp_coeffs(lo, u, m, orc.cutoff_nodes(m))
    else:
        a = orc.cheb_coeffs(u, m)
    g = np.ones(len(p))
    return -orc.cheb_quadform(W.diag_csr(p), a, lo, u, g)


def test_labels_match_oracle_polynomial_traces(orc):
    rng = np.random.default_rng(11)
    specs = [L.sample_spectrum(rng, int(n))[0] for n in rng.integers(96, 200, size=12)]
    nmax = max(len(p) for p in specs)
    P = np.zeros((len(specs), nmax))
    mask = np.zeros_like(P)
    for r, p in enumerate(specs):
        P[r, :len(p)] = p
        mask[r, :len(p)] = 1
    feats, labels, H, u = L.batch_features_labels(P, mask, seed=3)
    labels = labels.double().numpy()
    H, u = H.numpy(), u.numpy()
    checked_cutoff = 0
    for r, p in enumerate(specs):
        Hx = float(-np.sum(p[p > 0] * np.log(p[p > 0])))
        assert H[r] == pytest.approx(Hx, rel=1e-12)
        m = int(round(math.exp(labels[r, 0])))
        z = labels[r, 1]
        if m >= L.M_MAX:
            continue
        lo = 0.0 if z <= L.ZERO_CODE + 1e-3 else u[r] * 10.0 ** z
        assert lo <= p[p > 0].min() * (1 + 1e-12)       # the cutoff never cuts the spectrum
        est = poly_trace(orc, p, lo, u[r], m)
        assert abs(est - Hx) <= L.TARGET_ERR * Hx * (1 + 1e-6), (r, m, lo)
        if lo == 0.0 and m > 4:
            prev = poly_trace(orc, p, 0.0, u[r], m - 1)
            assert abs(prev - Hx) > L.TARGET_ERR * Hx * (1 - 1e-6)
        checked_cutoff += lo > 0
        assert np.all(np.isfinite(feats[r].numpy()))
    assert checked_cutoff >= 1


def test_features_of_flat_spectrum():
    # I/n: every normalised moment is T_k(2/(n u) - 1) exactly, whatever the probes
    n = 64
    P = np.full((1, n), 1.0 / n)
    feats, _, H, u = L.batch_features_labels(P, np.ones_like(P), seed=0)
    f = feats[0].double().numpy()
    uu = float(u[0])
    assert uu == pytest.approx(min(1.0, 6.0 / n), rel=1e-12)
    t = 2.0 / (n * uu) - 1.0
    for k in range(1, 13):
        assert f[2 + k] == pytest.approx(math.cos(k * math.acos(t)), abs=1e-6)
    assert f[0] == pytest.approx(math.log(n) / 10, rel=1e-6)
    assert float(H[0]) == pytest.approx(math.log(n), rel=1e-14)
