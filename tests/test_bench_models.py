"""The byte models behind bench.py's roofline figures (algorithmic HBM bytes
per launch of the sparse step kernels) and the split of the recurrence into
multi-step launches, against closed forms written out by hand for the
workloads' shapes: Chebyshev's m steps pass V 3m - 3 times one step per
launch (V_k from step 1, V_{k-1} from step 2, every step writes), Taylor's
m + 1 steps 2m times (no V_{k-1} term, the last step writes nothing), and a
multi-step launch reads V_k and V_{k-1} once and writes two blocks."""
import bench as B


def test_fuse_split():
    assert B.fuse_split(10, 10) == [10]
    assert B.fuse_split(10, 4) == [4, 3, 3]
    assert B.fuse_split(11, 10) == [6, 5]
    assert B.fuse_split(3, 2) == [2, 1]
    assert B.fuse_split(1, 10) == [1]
    for steps in range(1, 64):
        for nf in range(1, 11):
            sz = B.fuse_split(steps, nf)
            assert sum(sz) == steps and max(sz) <= nf and max(sz) - min(sz) <= 1
            assert sz == sorted(sz, reverse=True) and len(sz) == -(-steps // nf)


def test_tridiagonal_models_poisson():
    n, s, m = 10**8, 100, 10
    diag, signs, blk = 4 * 4 * n, n * s / 8, 4 * n * s
    one, steps = B.tri_step_bytes(n, s, m, 4, "chebyshev")
    assert steps == m and one == m * (diag + signs) + (3 * m - 3) * blk
    tay, tsteps = B.tri_step_bytes(n, s, m, 4, "taylor")
    assert tsteps == m + 1 and tay == (m + 1) * (diag + signs) + 2 * m * blk
    # all ten steps in one launch from the sign bits: two blocks written
    tot, launches = B.tri_fused_bytes(n, s, m, 4, "chebyshev", 10)
    assert launches == 1 and tot == diag + signs + 2 * blk
    # launches of 4, 3 and 3 steps (k = 0, 4, 7): the later two read V_k and V_{k-1}
    tot4, l4 = B.tri_fused_bytes(n, s, m, 4, "chebyshev", 4)
    assert l4 == 3 and tot4 == 3 * (diag + signs) + (2 + 4 + 4) * blk
    # FP64 doubles every stored value, not the sign bits
    t64, _ = B.tri_fused_bytes(n, s, m, 8, "chebyshev", 10)
    assert t64 == 2 * diag + signs + 4 * blk
    # Taylor, m + 1 = 11 steps in launches of 6 and 5: the last launch's last step is not written
    tt, lt = B.tri_fused_bytes(n, s, m, 4, "taylor", 10)
    assert lt == 2 and tt == 2 * (diag + signs) + (2 + (1 + 1)) * blk


def test_banded_models_csr1e7():
    n, hp, s, m = 10**7, 16, 64, 40
    slabs = ((n + 15) // 16) * 16 * (16 + 2 * hp) * 4
    signs, blk = n * s / 8, 4 * n * s
    one, steps = B.band_step_bytes(n, hp, s, m, 4, "chebyshev")
    assert steps == m and one == m * (slabs + signs) + (3 * m - 3) * blk
    pair, pairs = B.band_pair_bytes(n, hp, s, m, 4, "chebyshev")
    # 20 launches: the first writes two blocks, the others read two and write two
    assert pairs == 20 and pair == 20 * (slabs + signs) + (2 + 19 * 4) * blk
    # per recurrence step the pairs move about 37% fewer algorithmic bytes
    # (the counters show 26% fewer: the kernel reads each slab twice, once
    # per 32-probe chunk)
    assert 0.60 < (pair / (2 * pairs)) / (one / steps) < 0.66


def test_general_csr_model():
    n, nnz, s, m = 1000, 7000, 64, 8
    csr = (4 + 4) * nnz + 8 * (n + 1)
    one, steps = B.csr_step_bytes(n, nnz, s, m, 4, "chebyshev")
    assert steps == m and one == m * (csr + n * s / 8) + (3 * m - 3) * 4 * n * s
