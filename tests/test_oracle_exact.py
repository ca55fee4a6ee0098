"""Pins for the oracle's exact entropy (eqn. (1)), Jacobi eigensolver, random
projection (Algorithm 3) and the FP64 MLP."""
import math

import numpy as np
import pytest

import workloads as W


def shannon(p):
    p = p[p > 0]
    return float(-np.sum(p * np.log(p)))


def test_jacobi_against_known_spectrum_and_numpy(orc):
    n = 80
    p = W.spectrum_exp(n, 20.0)
    R = W.dense_density(p, 21)
    e, V, sweeps = orc.jacobi_eigen(R, vectors=True)
    assert np.max(np.abs(np.sort(e)[::-1] - p)) < 1e-15
    assert np.max(np.abs(np.sort(e) - np.linalg.eigvalsh(R))) < 1e-15
    assert np.max(np.abs(R @ V - V * e[None, :])) < 1e-13 * np.abs(R).max()
    assert np.max(np.abs(V.T @ V - np.eye(n))) < 1e-13
    assert sweeps < 20


def test_exact_entropy_invariants(orc):
    n = 40
    assert abs(orc.exact_entropy(W.pure_state(n, 1))) < 1e-12
    assert orc.exact_entropy(W.maximally_mixed(n)) == pytest.approx(math.log(n), rel=1e-14)
    p = W.spectrum_inverse(n)
    assert orc.exact_entropy(np.diag(p)) == pytest.approx(shannon(p), rel=1e-14)
    R = W.dense_density(p, 3)
    assert orc.exact_entropy(R) == pytest.approx(shannon(p), rel=1e-12)
    # rank-deficient: zero eigenvalues contribute nothing
    q = np.zeros(n)
    q[:7] = W.spectrum_inverse(7)
    assert orc.exact_entropy(W.dense_density(q, 4)) == pytest.approx(shannon(q), rel=1e-12)


def test_poisson_spectrum_closed_form(orc):
    # tridiagonal experiment (Section 6): lambda_i = (4/2n) sin^2(i pi/(2n+2))
    n = 150
    csr = W.poisson_csr(n)
    lam = W.poisson_eigenvalues(n)
    assert abs(lam.sum() - 1.0) < 1e-14
    e = orc.jacobi_eigen(W.csr_to_dense(csr))
    assert np.max(np.abs(np.sort(e) - np.sort(lam))) < 1e-13 * lam.max()
    assert orc.exact_entropy(csr) == pytest.approx(shannon(lam), rel=1e-13)
    fast = W.poisson_csr_fast(n)
    for a, b in zip(fast[:3], csr[:3]):
        assert np.array_equal(a, b)


def test_poisson_entropy_values():
    # closed-form entropies of the normalised tridiagonal matrix at the paper's sizes
    for n, want in ((5000, 8.210417630846004), (100000, 11.206076508473785)):
        assert shannon(W.poisson_eigenvalues(n)) == pytest.approx(want, rel=1e-12)


def test_rp_with_orthonormal_sketch_recovers_spectrum(orc):
    # Algorithm 3: if Pi has orthonormal columns spanning the range of R, the
    # singular values of R Pi are exactly the nonzero p_i
    n, k = 60, 6
    p = np.zeros(n)
    p[:k] = W.spectrum_inverse(k)
    rng = np.random.default_rng(5)
    U = W.random_orthogonal(n, rng)
    R = (U * p) @ U.T
    R = 0.5 * (R + R.T)
    h, sig = orc.rp_entropy_with_pi(R, U[:, :10], k)
    assert np.allclose(sig, p[:k], rtol=1e-12, atol=1e-15)
    assert h == pytest.approx(shannon(p), rel=1e-12)
    Q = W.random_orthogonal(n, rng)   # any orthogonal n x n sketch
    h2, _ = orc.rp_entropy_with_pi(R, Q, k)
    assert h2 == pytest.approx(shannon(p), rel=1e-11)


def test_rp_gaussian_sketch_theorem3_sanity(orc):
    n, k = 200, 5
    p = np.zeros(n)
    p[:k] = W.spectrum_exp(k, 2.0)
    R = W.dense_density(p, 6)
    h, sig = orc.rp_entropy(R, s=150, k=k, seed=3)
    H = shannon(p)
    # Theorem 3 with a generous eps; a sanity check, not a gate on the bound
    eps = 0.5
    assert abs(h - H) <= math.sqrt(eps) * H + math.sqrt(1.5) * eps
    assert np.all(np.abs(sig ** 2 - p[:k] ** 2) <= eps * p[:k] ** 2)


def test_mlp_gradient_finite_differences(orc):
    rng = np.random.default_rng(0)
    npar = orc.mlp_nparams()
    assert npar == 64 * 16 + 64 + 64 * 64 + 64 + 2 * 64 + 2
    P = rng.standard_normal(npar) * 0.3
    X = rng.standard_normal((7, 16))
    T = rng.standard_normal((7, 2))
    loss, g = orc.mlp_loss_grad(P, X, T)
    Y = orc.mlp_forward(P, X)
    assert loss == pytest.approx(np.mean(np.sum((Y - T) ** 2, axis=1)), rel=1e-14)
    idx = rng.choice(npar, 60, replace=False)
    hstep = 1e-6
    for i in idx:
        Pp, Pm = P.copy(), P.copy()
        Pp[i] += hstep
        Pm[i] -= hstep
        fd = (orc.mlp_loss_grad(Pp, X, T)[0] - orc.mlp_loss_grad(Pm, X, T)[0]) / (2 * hstep)
        assert fd == pytest.approx(g[i], rel=1e-6, abs=2e-8)  # FD rounding ~ eps*loss/h


def test_mlp_forward_closed_forms(orc):
    # special parameter choices whose outputs follow from the network's
    # definition (16 -> 64 -> 64 -> 2, ReLU after the two hidden layers) with
    # no matrix product: a transposed weight block, a misplaced bias or a
    # wrong activation changes them
    IN, H, OUT = 16, 64, 2
    rng = np.random.default_rng(5)
    X = rng.standard_normal((9, IN))

    def pack(W1, b1, W2, b2, W3, b3):
        return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3.ravel(), b3])

    # all weights zero: the output is the last bias for every input
    b3 = np.array([0.25, -1.5])
    P = pack(np.zeros((H, IN)), rng.standard_normal(H), np.zeros((H, H)), rng.standard_normal(H),
             np.zeros((OUT, H)), b3)
    assert np.array_equal(orc.mlp_forward(P, X), np.tile(b3, (9, 1)))

    # W1 copies input (o mod 16) into hidden unit o with weight w_o; W2 is a
    # permutation (unit o reads unit perm[o]); W3 weights c; biases zero:
    # y_r = sum_o c[r, o] * relu(w_perm[o] * x[perm[o] mod 16])
    w = rng.uniform(0.5, 2.0, H)
    W1 = np.zeros((H, IN))
    W1[np.arange(H), np.arange(H) % IN] = w
    perm = rng.permutation(H)
    W2 = np.zeros((H, H))
    W2[np.arange(H), perm] = 1.0
    C = rng.standard_normal((OUT, H))
    P = pack(W1, np.zeros(H), W2, np.zeros(H), C, np.zeros(OUT))
    Y = orc.mlp_forward(P, X)
    for r in range(X.shape[0]):
        for k in range(OUT):
            expect = sum(C[k, o] * max(w[perm[o]] * X[r, perm[o] % IN], 0.0) for o in range(H))
            assert Y[r, k] == pytest.approx(expect, rel=1e-13, abs=1e-13)
    # the hidden biases enter before the ReLU: a bias of -inf-like size
    # switches every unit off
    P = pack(W1, np.full(H, -1e3), W2, np.zeros(H), C, np.zeros(OUT))
    assert np.array_equal(orc.mlp_forward(P, X), np.zeros((9, OUT)))
