"""Training data and driver for the learned degree / lower-cutoff selector.

The selector maps 16 features of a cheap sketch of R -- the power method and
a degree-12 Chebyshev moment pass with 16 probes on [0, u] -- to
(ln m*, log10(lo*/u)): the smallest Chebyshev degree, and the largest lower
cutoff, at which the polynomial trace (no sampling) is within 5e-4 of the
exact entropy.  Training spectra are drawn from three families (power law,
exponential, Dirichlet with rank deficiency), and the features are simulated
exactly in distribution from the spectrum alone: for R = U diag(p) U^T with
Haar U, a probe g in the eigenbasis is U^T g, whose direction is uniform on
the sphere, so normalised moments sum_i z_i^2 T_k(t_i) / |z|^2 with Gaussian z
have the law of the library's Rademacher sketch, and the power method's start
vector has the same property.

Array work here is data generation only (torch tensors as bulk arrays, on the
GPU when present); the network is trained by the library's own forward,
backward and Adam kernels (ent_mlp_train_epoch).
"""
from __future__ import annotations

import math
import os

import numpy as np

FEAT_DEGREE = 12
FEAT_PROBES = 16
POWER_ITERS = 20
U_FACTOR = 6.0
TARGET_ERR = 5e-4
M_MAX = 300
ZERO_CODE = -6.0                                      # log10(lo/u) label meaning lo = 0 (decoded below -5.25)
RHO_GRID = 10.0 ** (-np.arange(1, 49) / 4.0)          # lo/u candidates 10^-0.25 .. 10^-12
CUTOFF_NODES = 1024
WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "selector_weights.npz")


# ---------------------------------------------------------------------------
# spectra
# ---------------------------------------------------------------------------
def sample_spectrum(rng: np.random.Generator, n: int):
    """One spectrum of a random family: power law, exponential or Dirichlet."""
    fam = int(rng.integers(0, 3))
    i = np.arange(1, n + 1, dtype=np.float64)
    if fam == 0:
        p = i ** (-rng.uniform(0.5, 2.0))
    elif fam == 1:
        tau = math.exp(rng.uniform(math.log(n / 100.0), math.log(float(n))))
        p = np.exp(-(i - 1.0) / tau)
    else:
        alpha = math.exp(rng.uniform(math.log(0.1), math.log(2.0)))
        k = int(rng.integers(max(1, n // 8), n + 1))
        g = rng.gamma(alpha, 1.0, size=k)
        p = np.zeros(n)
        p[:k] = np.sort(g)[::-1]
        if p.sum() <= 0.0:
            p[0] = 1.0
    p = p / p.sum()
    return p, fam


# ---------------------------------------------------------------------------
# coefficients (same definitions as the library's device code)
# ---------------------------------------------------------------------------
def lemma3_coeffs(u, m: int):
    """Closed-form Chebyshev coefficients of x ln x on [0, u] (Lemma 3), for a
    tensor of u values: shape u.shape + (m + 1,)."""
    import torch

    u = u[..., None]
    w = torch.arange(m + 1, dtype=torch.float64, device=u.device)
    sign = torch.where(w % 2 == 1, -1.0, 1.0)
    denom = torch.where(w >= 2, w ** 3 - w, torch.ones_like(w))
    a = sign * u / denom
    a0 = 0.5 * u[..., 0] * (torch.log(u[..., 0] / 4.0) + 1.0)
    a1 = 0.25 * u[..., 0] * (2.0 * torch.log(u[..., 0] / 4.0) + 3.0)
    return torch.cat([a0[..., None], a1[..., None], a[..., 2:]], dim=-1)


def ylny_projection(rho: float, m: int) -> np.ndarray:
    """Chebyshev coefficients of y ln y on [rho, 1] by the 1024-node rule."""
    N = CUTOFF_NODES
    th = math.pi * (np.arange(N) + 0.5) / N
    y = 0.5 * (1.0 + rho) + 0.5 * (1.0 - rho) * np.cos(th)
    h = y * np.log(y)
    c = np.array([2.0 / N * np.sum(h * np.cos(w * th)) for w in range(m + 1)])
    c[0] *= 0.5
    return c


_YLNY = {}


def cutoff_coeffs(lo_over_u: float, u, m: int):
    """Coefficients of x ln x on [lo, u] with lo = rho u, from those of y ln y on
    [rho, 1]: x ln x = u (y ln y) + u ln(u) y with y = x / u."""
    import torch

    key = (float(lo_over_u), m)
    if key not in _YLNY:
        _YLNY[key] = ylny_projection(lo_over_u, m)
    base = torch.as_tensor(_YLNY[key], dtype=torch.float64, device=u.device)
    lin = torch.zeros(m + 1, dtype=torch.float64, device=u.device)
    lin[0] = 0.5 * (1.0 + lo_over_u)
    lin[1] = 0.5 * (1.0 - lo_over_u)
    u = u[..., None]
    return u * (base + torch.log(u) * lin)


# ---------------------------------------------------------------------------
# features and labels for a batch of spectra (padded, masked)
# ---------------------------------------------------------------------------
def _cheb_moments(t, weights, kmax, torch):
    """sum_i weights_i(...) T_k(t_i) for k = 0..kmax; t: B x n, weights: B x n x J."""
    out = []
    tkm1 = torch.ones_like(t)
    tk = t.clone()
    out.append(torch.einsum("bn,bnj->bj", tkm1, weights))
    if kmax >= 1:
        out.append(torch.einsum("bn,bnj->bj", tk, weights))
    for _ in range(2, kmax + 1):
        tkm1, tk = tk, 2.0 * t * tk - tkm1
        out.append(torch.einsum("bn,bnj->bj", tk, weights))
    return torch.stack(out, dim=1)  # B x (kmax+1) x J


def batch_features_labels(P, mask, seed: int, device="cpu"):
    """Features (B x 16) and labels (B x 2) of padded spectra P (B x n, rows
    sum to one, mask marks the real entries)."""
    import torch

    g = torch.Generator(device="cpu").manual_seed(seed)
    P = torch.as_tensor(P, dtype=torch.float64, device=device)
    mask = torch.as_tensor(mask, dtype=torch.float64, device=device)
    B, n = P.shape
    nvalid = mask.sum(dim=1)
    # power method from a uniformly random direction: RQ = sum w q^(2t+1) / sum w q^(2t) * p1
    x2 = torch.randn((B, n), generator=g, dtype=torch.float64).to(device) ** 2 * mask
    p1 = P.max(dim=1).values
    q = P / p1[:, None]
    e = 2 * POWER_ITERS
    num = (x2 * q ** (e + 1)).sum(dim=1)
    den = (x2 * q ** e).sum(dim=1)
    p1t = p1 * num / den
    u = torch.clamp(U_FACTOR * p1t, max=1.0)
    # sketch moments with normalised Gaussian probes in the eigenbasis
    z2 = torch.randn((B, n, FEAT_PROBES), generator=g, dtype=torch.float64).to(device) ** 2
    z2 = z2 * mask[:, :, None]
    norms = z2.sum(dim=1)                               # B x J
    t = 2.0 * P / u[:, None] - 1.0
    M = _cheb_moments(t, z2, FEAT_DEGREE, torch)        # B x 13 x J
    mu = (M / norms[:, None, :]).mean(dim=2)            # B x 13
    alpha = lemma3_coeffs(u, FEAT_DEGREE)     # B x 13
    h12 = -(alpha[:, :, None] * M).sum(dim=1).mean(dim=1)
    ln_n = torch.log(nvalid)
    feats = torch.cat([(ln_n / 10.0)[:, None], (torch.log(nvalid * p1t) / 10.0)[:, None],
                       (torch.log(u) / 10.0)[:, None], mu[:, 1:13], (h12 / ln_n)[:, None]], dim=1)
    # labels: exact entropy vs the polynomial trace on each candidate interval
    H = -(torch.where(P > 0, P * torch.log(torch.where(P > 0, P, torch.ones_like(P))), torch.zeros_like(P))).sum(dim=1)
    has_zero = ((P <= 0) & (mask > 0)).any(dim=1)
    pmin = torch.where(mask > 0, torch.where(P > 0, P, torch.full_like(P, float("inf"))),
                       torch.full_like(P, float("inf"))).min(dim=1).values
    m0 = _degree_needed(P, mask, u, H, torch.zeros_like(u), torch)
    # the largest feasible cutoffs (rho u <= p_min) for full-rank spectra: the
    # grid point just below p_min / u and the next one down
    ratio = (pmin / u).cpu().numpy()
    hz = has_zero.cpu().numpy()
    ja = np.searchsorted(-RHO_GRID, -ratio, side="left")      # first j with RHO_GRID[j] <= ratio
    usable = (~hz) & (ja < len(RHO_GRID))
    best_m, best_z = m0, torch.full((B,), ZERO_CODE, dtype=torch.float64, device=device)
    if usable.any():
        for jj in (np.minimum(ja, len(RHO_GRID) - 1), np.minimum(ja + 1, len(RHO_GRID) - 1)):
            rho = torch.as_tensor(np.where(usable, RHO_GRID[jj], 0.0), dtype=torch.float64, device=device)
            mr = _degree_needed(P, mask, u, H, rho, torch)
            better = torch.as_tensor(usable, device=device) & (mr < best_m)
            best_m = torch.where(better, mr, best_m)
            best_z = torch.where(better, torch.log10(rho.clamp(min=1e-300)), best_z)
    labels = torch.stack([torch.log(best_m), best_z], dim=1)
    return feats.float(), labels.float(), H, u


def _degree_needed(P, mask, u, H, rho, torch):
    """Per row: the smallest degree m >= 4 whose polynomial trace on
    [rho u, u] is within TARGET_ERR (relative) of H, else M_MAX; rho = 0 rows
    use the closed form of Lemma 3, rho > 0 rows the cutoff projection."""
    lo = rho * u
    tt = (2.0 * P - (u + lo)[:, None]) / (u - lo)[:, None]
    Mw = _cheb_moments(tt, mask[:, :, None], M_MAX, torch)[:, :, 0]      # B x (M_MAX+1)
    c = torch.where((rho > 0)[:, None], cutoff_coeffs_rows(rho, u, M_MAX, torch),
                    lemma3_coeffs(u, M_MAX))
    est = -torch.cumsum(c * Mw, dim=1)
    err = (est - H[:, None]).abs() / H.clamp(min=1e-300)[:, None]
    ok = err <= TARGET_ERR
    ok[:, :4] = False
    return torch.where(ok.any(dim=1), ok.double().argmax(dim=1).double(),
                       torch.full_like(H, float(M_MAX)))


def cutoff_coeffs_rows(rho, u, m: int, torch):
    """cutoff_coeffs for a per-row rho taken from RHO_GRID (rows with rho = 0
    get zeros): shape (B, m + 1)."""
    table = np.zeros((len(RHO_GRID) + 1, m + 1))
    for j, r in enumerate(RHO_GRID):
        key = (float(r), m)
        if key not in _YLNY:
            _YLNY[key] = ylny_projection(float(r), m)
        table[j] = _YLNY[key]
    rr = rho.cpu().numpy()
    idx = np.array([int(np.argmin(np.abs(RHO_GRID - x))) if x > 0 else len(RHO_GRID) for x in rr])
    base = torch.as_tensor(table[idx], dtype=torch.float64, device=u.device)
    lin = torch.zeros((rho.shape[0], m + 1), dtype=torch.float64, device=u.device)
    lin[:, 0] = 0.5 * (1.0 + rho)
    lin[:, 1] = 0.5 * (1.0 - rho)
    uu = u[:, None]
    out = uu * (base + torch.log(uu) * lin)
    return torch.where((rho > 0)[:, None], out, torch.zeros_like(out))


def make_dataset(count: int, n_lo: int, n_hi: int, seed: int, device="cpu", chunk: int = 256):
    """count training samples: features (count x 16) and labels (count x 2) as
    float32 tensors on `device`, plus the family of each sample."""
    import torch

    rng = np.random.default_rng(seed)
    X, T, F = [], [], []
    done = 0
    while done < count:
        b = min(chunk, count - done)
        ns = rng.integers(n_lo, n_hi + 1, size=b)
        nmax = int(ns.max())
        P = np.zeros((b, nmax))
        mask = np.zeros((b, nmax))
        for r in range(b):
            p, fam = sample_spectrum(rng, int(ns[r]))
            P[r, :ns[r]] = p
            mask[r, :ns[r]] = 1.0
            F.append(fam)
        f, l, _, _ = batch_features_labels(P, mask, seed * 7919 + done, device=device)
        X.append(f)
        T.append(l)
        done += b
    return torch.cat(X).to(device), torch.cat(T).to(device), np.array(F)


# ---------------------------------------------------------------------------
# training with the library's kernels
# ---------------------------------------------------------------------------
def init_params(seed: int) -> np.ndarray:
    """He-uniform weights, zero biases, in the library's parameter layout."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_in, fan_out in ((16, 64), (64, 64), (64, 2)):
        lim = math.sqrt(6.0 / fan_in)
        parts.append(rng.uniform(-lim, lim, size=fan_out * fan_in))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32)


def train(X, T, epochs: int = 30, batch: int = 4096, lr: float = 2e-3, seed: int = 0,
          log=None):
    """Minibatch Adam on the GPU by ent_mlp_train_epoch; returns (params, losses)."""
    import torch

    import paper_1801_01072_amd as ent

    params = torch.from_numpy(init_params(seed)).to(X.device)
    state = ent.AdamState(params)
    g = torch.Generator(device="cpu").manual_seed(seed)
    losses = []
    for ep in range(epochs):
        perm = torch.randperm(X.shape[0], generator=g).to(X.device)
        Xs = X[perm].contiguous()
        Ts = T[perm].contiguous()
        lr_ep = lr * (0.5 * (1 + math.cos(math.pi * ep / epochs)))
        losses.append(state.epoch(Xs, Ts, batch, lr_ep))
        if log:
            log(f"epoch {ep}: loss {losses[-1]:.5f}")
    return params, losses


def save(params, path: str = WEIGHTS, **meta):
    np.savez(path, params=np.asarray(params.detach().cpu() if hasattr(params, "detach") else params,
                                     dtype=np.float32), **meta)


def load(path: str = WEIGHTS) -> np.ndarray:
    with np.load(path, allow_pickle=False) as z:
        return np.asarray(z["params"], dtype=np.float32)
