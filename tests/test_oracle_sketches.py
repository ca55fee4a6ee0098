"""Pins for the oracle's sketch constructions of Algorithm 3 (Section 5.2):
the subsampled randomized Hadamard transform against scipy's Sylvester
Hadamard matrix, the input-sparsity transform's structure, E[Pi Pi^T] = I on
the diagonal exactly, exact recovery when a sketch is an isometry on the range
of R, and the accuracy the embedding lemmas predict for a rank-k R."""
import math

import numpy as np
import pytest
from scipy.linalg import hadamard

import workloads as W


@pytest.mark.parametrize("n", [1, 7, 64, 100])
def test_srht_matches_sylvester_hadamard(orc, n):
    s, seed = 12, 31
    N = orc.hadamard_order(n)
    assert N >= n and N & (N - 1) == 0 and (N == 1 or N // 2 < n)
    Pi = orc.sketch_matrix(orc.SKETCH_SRHT, seed, n, s)
    H = hadamard(N)                                          # entries +-1, H_ji = (-1)^popcount(j & i)
    cols = [orc.srht_column(seed, t, N) for t in range(s)]
    D = np.array([orc.sketch_sign(seed, j) for j in range(n)])
    want = D[:, None] * H[:n][:, cols] / math.sqrt(s)
    assert np.array_equal(Pi, want)
    assert all(0 <= c < N for c in cols)


def test_diagonal_of_pi_pi_t_is_one(orc):
    n, s = 50, 16
    for kind in (orc.SKETCH_SRHT, orc.SKETCH_COUNT):
        Pi = orc.sketch_matrix(kind, 4, n, s)
        assert np.allclose(np.sum(Pi * Pi, axis=1), 1.0, rtol=0, atol=1e-15)


def test_count_sketch_structure(orc):
    n, s, seed = 4000, 37, 9
    Pi = orc.sketch_matrix(orc.SKETCH_COUNT, seed, n, s)
    nz = Pi != 0
    assert np.all(nz.sum(axis=1) == 1)
    assert set(np.unique(Pi[nz])) <= {-1.0, 1.0}
    buckets = np.argmax(nz, axis=1)
    assert all(buckets[j] == orc.sketch_bucket(seed, j, s) for j in range(0, n, 97))
    counts = np.bincount(buckets, minlength=s)
    chi2 = float(np.sum((counts - n / s) ** 2 / (n / s)))
    assert chi2 < 2.5 * s                                   # roughly uniform buckets
    signs = Pi[nz]
    assert abs(signs.mean()) < 4 / math.sqrt(n)


def test_count_sketch_is_exact_on_distinct_buckets(orc):
    # R = diag(p) on k coordinates that fall into distinct buckets: R Pi has
    # orthogonal rows p_a D e_h, so its singular values are exactly p
    n, s, k, seed = 300, 64, 5, 2
    rows, used = [], set()
    for j in range(n):
        b = orc.sketch_bucket(seed, j, s)
        if b not in used:
            used.add(b)
            rows.append(j)
        if len(rows) == k:
            break
    p = np.array([0.4, 0.25, 0.2, 0.1, 0.05])
    R = np.zeros((n, n))
    R[rows, rows] = p
    h, sig = orc.rp_entropy(R, s, k, seed, kind=orc.SKETCH_COUNT)
    assert np.allclose(np.sort(sig)[::-1], np.sort(p)[::-1], rtol=1e-13)
    assert h == pytest.approx(float(-np.sum(p * np.log(p))), rel=1e-13)


def test_full_hadamard_is_an_isometry(orc):
    # sampling every column once (S = I) gives Pi = D H, orthogonal: exact spectrum
    n, k = 32, 6
    p = W.spectrum_exp(k, 2.0)
    R = W.dense_density(np.concatenate([p, np.zeros(n - k)]), 3)
    D = np.array([orc.sketch_sign(7, j) for j in range(n)])
    Pi = D[:, None] * hadamard(n) / math.sqrt(n)
    h, sig = orc.rp_entropy_with_pi(R, Pi, k)
    assert np.allclose(sig, np.sort(p)[::-1], rtol=1e-12)


@pytest.mark.parametrize("kind", [1, 2])
def test_rank_k_accuracy(orc, kind):
    # the embedding lemmas: s large against k (and k^2 for the input-sparsity
    # transform) gives |p_i^2 - p~_i^2| <= eps p_i^2 with high probability
    n, k, s = 256, 4, 256
    p = np.array([0.4, 0.3, 0.2, 0.1])
    R = W.dense_density(np.concatenate([p, np.zeros(n - k)]), 11)
    H = float(-np.sum(p * np.log(p)))
    h, sig = orc.rp_entropy(R, s, k, 5, kind=kind)
    assert np.max(np.abs(sig ** 2 - p ** 2) / p ** 2) < 0.5
    assert abs(h - H) / H < 0.1
