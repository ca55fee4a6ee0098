"""Pin of the maximum over q power-method trials (Algorithm 4, Appendix A).

With R = U diag(p) U^T (U known) and start vector x_j of trial j, t products
give x_t proportional to R^t x_j, so the Rayleigh quotient of trial j is
    r_j = sum_i c_i^2 p_i^(2t+1) / sum_i c_i^2 p_i^(2t),   c = U^T x_j,
whatever normalisation is applied between products.  Algorithm 4 returns the
maximum of r_j over the q trials.  The cases below are chosen so that the
trials' quotients differ and the maximum is neither the first nor the last
trial: an oracle that returns the first, the last, the mean or the minimum
trial fails them.  Start vectors are the stream-1 Rademacher vectors of the
probe generator (pinned separately by the Philox known-answer vectors).
"""
import numpy as np
import pytest

import workloads as W


def trial_quotients_real(orc, U, p, t, q, seed):
    out = []
    for j in range(q):
        x = orc.probe_vector(seed, 0, 1, len(p), j)
        c = U.T @ x
        out.append(float(np.sum(c * c * p ** (2 * t + 1)) / np.sum(c * c * p ** (2 * t))))
    return np.array(out)


def _interior_max_seed(quot_fn, seeds):
    """First seed whose trial quotients are distinct with the maximum strictly
    inside the trial range."""
    for seed in seeds:
        r = quot_fn(seed)
        j = int(np.argmax(r))
        spread = (r.max() - r.min()) / r.max()
        if 0 < j < len(r) - 1 and spread > 1e-3:
            return seed, r
    raise AssertionError("no seed with an interior maximum")


@pytest.mark.parametrize("t,q", [(1, 4), (2, 5), (3, 6)])
def test_real_power_method_is_max_over_trials(orc, t, q):
    n = 48
    p = W.spectrum_exp(n, 4.0)                       # p_1 / p_2 = e^(1/4): slow convergence
    rng = np.random.default_rng(777)
    U = W.random_orthogonal(n, rng)
    R = (U * p[None, :]) @ U.T
    seed, r = _interior_max_seed(lambda sd: trial_quotients_real(orc, U, p, t, q, sd), range(40))
    got = orc.power_method(R, t=t, q=q, seed=seed)
    assert got == pytest.approx(r.max(), rel=1e-12)
    # the maximum differs from the first and last trial, the mean and the minimum
    for wrong in (r[0], r[-1], r.mean(), r.min()):
        assert abs(got - wrong) > 1e-6 * r.max()
    # each trial alone (q = 1 with the trial's own start vector is trial 0 only)
    assert orc.power_method(R, t=t, q=1, seed=seed) == pytest.approx(r[0], rel=1e-12)


def trial_quotients_complex(orc, U, p, t, q, seed):
    n = len(p)
    out = []
    for j in range(q):
        s = orc.probe_vector(seed, 0, 1, 2 * n, j)
        x = s[:n] + 1j * s[n:]
        c = U.conj().T @ x
        a = np.abs(c) ** 2
        out.append(float(np.sum(a * p ** (2 * t + 1)) / np.sum(a * p ** (2 * t))))
    return np.array(out)


@pytest.mark.parametrize("t,q", [(1, 4), (2, 5)])
def test_complex_power_method_is_max_over_trials(orc, t, q):
    n = 40
    p = W.spectrum_exp(n, 4.0)
    rng = np.random.default_rng(991)
    U = W.random_unitary(n, rng)
    R = (U * p[None, :]) @ U.conj().T
    R = 0.5 * (R + R.conj().T)
    assert np.max(np.abs(R.imag)) > 1e-3           # genuinely complex
    seed, r = _interior_max_seed(lambda sd: trial_quotients_complex(orc, U, p, t, q, sd), range(40))
    got = orc.zpower_method(R, t=t, q=q, seed=seed)
    assert got == pytest.approx(r.max(), rel=1e-11)
    for wrong in (r[0], r[-1], r.mean(), r.min()):
        assert abs(got - wrong) > 1e-6 * r.max()
