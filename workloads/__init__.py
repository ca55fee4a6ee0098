"""Seeded synthetic inputs: density matrices and their known spectra.

This module builds inputs only.  It holds none of the estimators' arithmetic
(no traces, polynomials, power iterations or entropies); both the CPU oracle
and the GPU library are fed from here.  Shapes and value distributions follow
the paper's workloads (Section 6): dense random density matrices
R = U diag(p) U^T with a random orthogonal U, banded/tridiagonal matrices
normalised to unit trace, and low-rank matrices with decaying spectra.  The
paper's QETLAB matrices are not available; these seeded generators stand in
for them.
"""
from __future__ import annotations

import math

import numpy as np

# Fixed seeds of the benchmark workloads: matrix seed, probe seed.
MATRIX_SEED = 18010720
PROBE_SEED = 1801


# --------------------------------------------------------------------------
# Spectra (eigenvalues p_i, non-increasing, summing to one)
# --------------------------------------------------------------------------
def spectrum_inverse(n: int) -> np.ndarray:
    """p_i proportional to 1/i, i = 1..n."""
    p = 1.0 / np.arange(1, n + 1, dtype=np.float64)
    return p / p.sum()


def spectrum_exp(n: int, tau: float) -> np.ndarray:
    """p_i proportional to exp(-i/tau), i = 1..n."""
    p = np.exp(-np.arange(1, n + 1, dtype=np.float64) / tau)
    return p / p.sum()


def spectrum_power(n: int, a: float) -> np.ndarray:
    """p_i proportional to i^-a."""
    p = np.arange(1, n + 1, dtype=np.float64) ** (-a)
    return p / p.sum()


def spectrum_dirichlet(n: int, k: int, alpha: float, rng: np.random.Generator) -> np.ndarray:
    """Dirichlet(alpha) weights over k slots (normalised Gamma draws), zeros elsewhere."""
    g = rng.gamma(alpha, 1.0, size=k)
    while g.sum() <= 0.0:
        g = rng.gamma(alpha, 1.0, size=k)
    p = np.zeros(n, dtype=np.float64)
    p[:k] = np.sort(g / g.sum())[::-1]
    return p


def spectrum_linear_topk(n: int, k: int) -> np.ndarray:
    """Top-k linearly decaying weights, the rest equal (the paper's fourth dataset shape)."""
    top = np.linspace(2.0, 1.0, k) if k > 0 else np.zeros(0)
    p = np.concatenate([top * 10.0, np.full(n - k, top[-1] if k > 0 else 1.0)])
    return p / p.sum()


# --------------------------------------------------------------------------
# Dense density matrices
# --------------------------------------------------------------------------
def random_orthogonal(n: int, rng: np.random.Generator) -> np.ndarray:
    """Q factor of a Gaussian matrix with the sign of diag(R) fixed (Haar measure)."""
    Z = rng.standard_normal((n, n))
    Q, Rr = np.linalg.qr(Z)
    Q *= np.sign(np.diag(Rr))[None, :]
    return Q


def dense_density(p: np.ndarray, seed: int, dtype=np.float64) -> np.ndarray:
    """R = U diag(p) U^T, symmetrised entry by entry so that R == R^T exactly."""
    rng = np.random.default_rng(seed)
    n = len(p)
    U = random_orthogonal(n, rng)
    R = (U * p[None, :]) @ U.T
    R = 0.5 * (R + R.T)
    return np.ascontiguousarray(R.astype(dtype))


def dense_density_torch(p: np.ndarray, seed: int, device: str = "cuda", dtype=None,
                        rng_device: str = "cpu"):
    """Same construction on a torch device (fast input preparation for large n).

    Returns a contiguous torch tensor; the orthogonal factor comes from torch's
    QR of a seeded Gaussian matrix, drawn by torch's generator on `rng_device`.
    """
    import torch

    dtype = dtype or torch.float64
    g = torch.Generator(device=rng_device).manual_seed(seed)
    n = len(p)
    Z = torch.randn((n, n), generator=g, dtype=torch.float64, device=rng_device).to(device)
    Q, Rr = torch.linalg.qr(Z)
    Q = Q * torch.sign(torch.diagonal(Rr))[None, :]
    pt = torch.as_tensor(p, dtype=torch.float64, device=device)
    R = (Q * pt[None, :]) @ Q.T
    R = 0.5 * (R + R.T)
    return R.to(dtype).contiguous()


def low_rank_density_torch(pk: np.ndarray, n: int, seed: int, device: str = "cuda", dtype=None):
    """R = B B^T with B = Q diag(sqrt(pk)), Q (n x k) the sign-fixed Q factor of
    a seeded Gaussian n x k matrix: rank k = len(pk), spectrum pk (plus n - k
    zeros).  Only the n x n result is materialised, in `dtype`."""
    import torch

    dtype = dtype or torch.float64
    g = torch.Generator(device="cpu").manual_seed(seed)
    k = len(pk)
    Z = torch.randn((n, k), generator=g, dtype=torch.float64).to(device)
    Q, Rr = torch.linalg.qr(Z)
    Q = Q * torch.sign(torch.diagonal(Rr))[None, :]
    B = (Q * torch.sqrt(torch.as_tensor(pk, dtype=torch.float64, device=device))[None, :]).to(dtype)
    return (B @ B.T).contiguous()


def random_unitary(n: int, rng: np.random.Generator) -> np.ndarray:
    """Q factor of a complex Gaussian matrix with diag(R) made real positive
    (Haar measure on U(n))."""
    Z = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2.0)
    Q, Rr = np.linalg.qr(Z)
    d = np.diagonal(Rr)
    return Q * (d / np.abs(d))[None, :]


def hermitian_density(p: np.ndarray, seed: int, dtype=np.complex128) -> np.ndarray:
    """R = U diag(p) U^H with Haar-random unitary U, made Hermitian entry by
    entry (R == R^H exactly).  Stand-in for the random complex density
    matrices of the paper's Hermitian experiment."""
    rng = np.random.default_rng(seed)
    n = len(p)
    U = random_unitary(n, rng)
    R = (U * p[None, :]) @ U.conj().T
    R = 0.5 * (R + R.conj().T)
    return np.ascontiguousarray(R.astype(dtype))


def hermitian_density_torch(p: np.ndarray, seed: int, device: str = "cuda", dtype=None,
                            rng_device: str = "cpu"):
    """hermitian_density on a torch device (torch's QR of a seeded complex
    Gaussian matrix drawn on `rng_device`)."""
    import torch

    dtype = dtype or torch.complex128
    g = torch.Generator(device=rng_device).manual_seed(seed)
    n = len(p)
    Z = torch.complex(torch.randn((n, n), generator=g, dtype=torch.float64, device=rng_device),
                      torch.randn((n, n), generator=g, dtype=torch.float64, device=rng_device))
    Q, Rr = torch.linalg.qr(Z.to(device))
    d = torch.diagonal(Rr)
    Q = Q * (d / d.abs())[None, :]
    pt = torch.as_tensor(p, dtype=torch.float64, device=device).to(torch.complex128)
    R = (Q * pt[None, :]) @ Q.conj().T
    R = 0.5 * (R + R.conj().T)
    return R.to(dtype).contiguous()


def maximally_mixed(n: int) -> np.ndarray:
    return np.eye(n, dtype=np.float64) / n


def pure_state(n: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    psi = rng.standard_normal(n)
    psi /= np.linalg.norm(psi)
    R = np.outer(psi, psi)
    return 0.5 * (R + R.T)


# --------------------------------------------------------------------------
# Sparse (CSR) density matrices
# --------------------------------------------------------------------------
def banded_density_csr(n: int, half_bw: int = 8, seed: int = MATRIX_SEED, dtype=np.float64):
    """R = B B^T / tr(B B^T) with B square banded (|i-j| <= half_bw), B_ij ~ N(0,1).

    R has half-bandwidth 2*half_bw and nnz = (4 hb + 1) n - 2 sum_{d=1}^{2hb} d.
    Returns (row_ptr int64[n+1], col_idx int32[nnz], values, n).
    """
    rng = np.random.default_rng(seed)
    hb = half_bw
    idx = np.arange(n, dtype=np.int64)
    # b[a + hb][i] = B[i, i + a]  (zero where i + a falls outside [0, n))
    b = rng.standard_normal((2 * hb + 1, n))
    for a in range(-hb, hb + 1):
        bad = (idx + a < 0) | (idx + a >= n)
        b[a + hb][bad] = 0.0
    tr = float(np.sum(b * b))
    D = 2 * hb
    width = 2 * D + 1
    vals = np.zeros((n, width), dtype=np.float64)
    for d in range(-D, D + 1):
        col = vals[:, d + D]
        lo_i = max(0, -d)
        hi_i = min(n, n - d)
        if hi_i <= lo_i:
            continue
        ii = np.arange(lo_i, hi_i)
        acc = np.zeros(hi_i - lo_i)
        for a in range(-hb, hb + 1):
            a2 = a - d
            if a2 < -hb or a2 > hb:
                continue
            acc += b[a + hb][ii] * b[a2 + hb][ii + d]
        col[lo_i:hi_i] = acc
    vals /= tr
    cols = idx[:, None] + np.arange(-D, D + 1)[None, :]
    mask = (cols >= 0) & (cols < n)
    counts = mask.sum(axis=1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    col_idx = cols[mask].astype(np.int32)
    values = vals[mask].astype(dtype)
    return row_ptr, col_idx, values, n


def poisson_csr(n: int, dtype=np.float64):
    """Tridiagonal (-1, 2, -1) divided by its trace 2n (the paper's third dataset)."""
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    cols = np.empty(3 * n - 2, dtype=np.int32)
    vals = np.empty(3 * n - 2, dtype=np.float64)
    e = 0
    for i in range(n):
        for j, v in ((i - 1, -1.0), (i, 2.0), (i + 1, -1.0)):
            if 0 <= j < n:
                cols[e] = j
                vals[e] = v / (2.0 * n)
                e += 1
        row_ptr[i + 1] = e
    return row_ptr, cols, vals.astype(dtype), n


def poisson_csr_fast(n: int, dtype=np.float64):
    """Vectorised poisson_csr for large n (identical output)."""
    idx = np.arange(n, dtype=np.int64)
    cols = np.stack([idx - 1, idx, idx + 1], axis=1)
    v = np.array([-1.0, 2.0, -1.0]) / (2.0 * n)
    vals = np.broadcast_to(v, (n, 3))
    mask = (cols >= 0) & (cols < n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(mask.sum(axis=1), out=row_ptr[1:])
    return row_ptr, cols[mask].astype(np.int32), vals[mask].astype(dtype), n


def poisson_csr_torch(n: int, device: str = "cuda", dtype=None):
    """poisson_csr_fast built on a torch device (row_ptr int64, col_idx int32,
    values), for n up to the 10^8 of the paper's largest experiment."""
    import torch

    dtype = dtype or torch.float32
    idx = torch.arange(n, dtype=torch.int64, device=device)
    cols = torch.stack([idx - 1, idx, idx + 1], dim=1)
    mask = (cols >= 0) & (cols < n)
    row_ptr = torch.zeros(n + 1, dtype=torch.int64, device=device)
    torch.cumsum(mask.sum(dim=1), dim=0, out=row_ptr[1:])
    v = torch.tensor([-1.0, 2.0, -1.0], dtype=torch.float64, device=device) / (2.0 * n)
    vals = v.to(dtype).expand(n, 3)[mask].contiguous()
    col_idx = cols[mask].to(torch.int32).contiguous()
    del cols, mask, idx
    return row_ptr, col_idx, vals, n


def poisson_eigenvalues(n: int) -> np.ndarray:
    """Eigenvalues of the trace-normalised tridiagonal matrix (eqn. for lambda_i, Section 6):
    lambda_i = (4 / 2n) sin^2(i pi / (2n + 2)), i = 1..n."""
    i = np.arange(1, n + 1, dtype=np.float64)
    return (4.0 / (2.0 * n)) * np.sin(i * math.pi / (2.0 * n + 2.0)) ** 2


def csr_to_dense(csr) -> np.ndarray:
    rp, ci, val, n = csr
    A = np.zeros((n, n), dtype=np.float64)
    for i in range(n):
        A[i, ci[rp[i]:rp[i + 1]]] = val[rp[i]:rp[i + 1]]
    return A


def diag_csr(p: np.ndarray):
    n = len(p)
    return (np.arange(n + 1, dtype=np.int64), np.arange(n, dtype=np.int32),
            np.asarray(p, dtype=np.float64), n)


# --------------------------------------------------------------------------
# Batches of uneven density matrices
# --------------------------------------------------------------------------
def batch_shapes(count: int, seed: int, n_lo: int = 64, n_hi: int = 2048):
    """n_i ~ U{n_lo..n_hi}, k_i ~ U{ceil(n_i/8)..n_i}."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(n_lo, n_hi + 1, size=count)
    ks = np.array([rng.integers(int(math.ceil(n / 8)), n + 1) for n in ns])
    return ns, ks


def batch_spectra(ns, ks, seed: int, alpha: float = 0.5):
    rng = np.random.default_rng(seed + 1)
    return [spectrum_dirichlet(int(n), int(k), alpha, rng) for n, k in zip(ns, ks)]
