"""Pins for the oracle's random numbers: Philox4x32-10 known answers and the
probe mapping (Rademacher signs, Box-Muller Gaussians)."""
import math
import os

import numpy as np
import pytest
from scipy import stats

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat_rows():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        w = [int(x, 16) for x in line.replace("->", " ").split()]
        rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,expect", _kat_rows())
def test_philox_known_answers(orc, ctr, key, expect):
    assert orc.philox4x32_10(ctr, key) == expect


def test_rademacher_is_bit_of_philox_word(orc):
    # probe j of row i is bit (j & 31) of word (j >> 5) & 3 of the block j >> 7
    seed, i = 0x1234_5678_9ABC_DEF0, 77
    for j in (0, 1, 31, 32, 63, 64, 127, 128, 200):
        ctr = [i, j >> 7, 0, 0]
        key = [seed & 0xFFFFFFFF, seed >> 32]
        w = orc.philox4x32_10(ctr, key)[(j >> 5) & 3]
        want = -1.0 if (w >> (j & 31)) & 1 else 1.0
        assert orc.probe_value(seed, 0, 0, i, j) == want


def test_rademacher_balance(orc):
    g = orc.probe_block(3, 0, 0, 512, 64)
    assert set(np.unique(g)) <= {-1.0, 1.0}
    k = int((g > 0).sum())
    N = g.size
    # two-sided binomial test at a very small level
    assert abs(k - N / 2) < 6 * math.sqrt(N / 4)
    # distinct probes and distinct streams are not copies of each other
    assert not np.array_equal(g[:, 0], g[:, 1])
    h = orc.probe_block(3, 0, 1, 512, 2)
    assert not np.array_equal(g[:, :2], h)


def test_gaussian_box_muller_definition(orc):
    seed, i, j = 99, 5, 6
    w = orc.philox4x32_10([i, j >> 1, 0, 0], [seed, 0])
    a = ((w[1] << 32) | w[0]) >> 11
    b = ((w[3] << 32) | w[2]) >> 11
    u1 = (a + 1) * 2.0 ** -53
    u2 = b * 2.0 ** -53
    r = math.sqrt(-2.0 * math.log(u1))
    assert orc.probe_value(seed, 1, 0, i, j) == pytest.approx(r * math.cos(2 * math.pi * u2), rel=1e-15)
    assert orc.probe_value(seed, 1, 0, i, j + 1) == pytest.approx(r * math.sin(2 * math.pi * u2), rel=1e-15)


def test_gaussian_distribution(orc):
    g = orc.probe_block(11, 1, 0, 4000, 8).ravel()
    assert abs(g.mean()) < 5 / math.sqrt(g.size)
    assert abs(g.var() - 1.0) < 5 * math.sqrt(2.0 / g.size)
    assert stats.kstest(g, "norm").pvalue > 1e-4


def test_large_row_index_uses_high_counter_word(orc):
    seed = 7
    i = (1 << 32) + 5
    w = orc.philox4x32_10([5, 0, 0, 1], [seed, 0])
    assert orc.probe_value(seed, 0, 0, i, 3) == (-1.0 if (w[0] >> 3) & 1 else 1.0)
