"""The learned selector: hand-written MLP kernels against the FP64 oracle MLP,
GPU training, and ENT_AUTO with its a-posteriori check and fallback."""
import math

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1801_01072_amd as ent  # noqa: E402
from paper_1801_01072_amd import learned as L  # noqa: E402

DEV = "cuda:0"


def test_mlp_forward_and_gradient_match_oracle(orc):
    rng = np.random.default_rng(1)
    npar = ent.mlp_nparams()
    assert npar == orc.mlp_nparams()
    P = (rng.standard_normal(npar) * 0.3).astype(np.float32)
    for B in (1, 31, 100, 257):
        X = rng.standard_normal((B, 16)).astype(np.float32)
        T = rng.standard_normal((B, 2)).astype(np.float32)
        Pd, Xd, Td = (torch.from_numpy(a).to(DEV) for a in (P, X, T))
        Y = ent.mlp_forward(Pd, Xd).cpu().numpy()
        Yo = orc.mlp_forward(P.astype(np.float64), X.astype(np.float64))
        assert np.max(np.abs(Y - Yo)) <= 1e-5 * max(1.0, np.max(np.abs(Yo)))
        g, loss = ent.mlp_grad(Pd, Xd, Td)
        lo, go = orc.mlp_loss_grad(P.astype(np.float64), X.astype(np.float64), T.astype(np.float64))
        g = g.cpu().numpy()
        rel = np.max(np.abs(g - go)) / np.max(np.abs(go))
        print(f"[mlp B={B}] loss gpu={loss:.8f} oracle={lo:.8f} grad rel err={rel:.2e}", flush=True)
        assert loss == pytest.approx(lo, rel=1e-5)
        assert rel <= 1e-4


def test_training_reduces_loss():
    X, T, _ = L.make_dataset(2048, 128, 384, seed=5, device=DEV)
    params, losses = L.train(X, T, epochs=40, batch=256, lr=3e-3, seed=1)
    print(f"[train] loss {losses[0]:.4f} -> {losses[-1]:.4f}", flush=True)
    assert losses[-1] < 0.3 * losses[0]
    assert np.all(np.isfinite(losses))


def _trained_small():
    X, T, _ = L.make_dataset(4096, 128, 512, seed=7, device=DEV)
    params, _ = L.train(X, T, epochs=40, batch=256, lr=3e-3, seed=2)
    return params


def test_auto_estimates_and_features():
    params = _trained_small()
    ent.selector_load(params)
    n = 384
    for name, p in (("exp", W.spectrum_exp(n, 60.0)), ("power", W.spectrum_power(n, 1.0)),
                    ("flat", np.linspace(1.0, 2.0, n) / np.linspace(1.0, 2.0, n).sum())):
        R = torch.from_numpy(W.dense_density(p, 11)).to(DEV)
        H = float(-np.sum(p * np.log(p)))
        f, y = ent.selector_features(R, 3)
        assert np.all(np.isfinite(f)) and np.all(np.isfinite(y))
        assert abs(f[0] - math.log(n) / 10) < 1e-6
        auto = ent.entropy_estimate(R, "auto", 40, 64, 3, probe_dist="gaussian")
        plain = ent.entropy_estimate(R, "chebyshev", 40, 64, 3, probe_dist="gaussian")
        print(f"[auto {name}] H={H:.6f} auto={auto.entropy:.6f} (m={auto.degree}, lo={auto.lo:.3e}, "
              f"fell_back={auto.fell_back}, products={auto.products}) plain={plain.entropy:.6f}",
              flush=True)
        assert math.isfinite(auto.entropy)
        assert abs(auto.entropy - H) / H < 0.05


def test_auto_fallback_is_the_plain_schedule():
    # a network that always predicts degree 4 and lo = 10^-0.25 u fails the
    # check on a spectrum reaching far below lo, and must fall back
    params = np.zeros(ent.mlp_nparams(), dtype=np.float32)
    params[-2] = math.log(4.0)       # b3[0]
    params[-1] = -0.25               # b3[1]
    ent.selector_load(params)
    n = 200
    p = W.spectrum_exp(n, 20.0)
    R = torch.from_numpy(W.dense_density(p, 12)).to(DEV)
    auto = ent.entropy_estimate(R, "auto", 30, 32, 9)
    assert auto.fell_back == 1
    plain = ent.entropy_estimate(R, "chebyshev", 30, 32, 9, u_fixed=auto.u)
    assert auto.entropy == plain.entropy
    assert auto.products == 12 + 5 + 30   # degree 4 with the 25% margin -> 5


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_auto_continues_the_recurrence_before_falling_back(precision):
    """A predicted degree whose partial sums have not converged (spectrum
    inside the interval) is extended on the same recurrence to 1.5x the
    degree: the estimate is the one a direct Chebyshev run at that degree on
    the same interval gives, bit for bit, with 12 + 15 products and no
    fallback.  A network predicting degree 8 (10 with the margin) and
    lo = 10^-1.7 u on p_i ~ exp(-i/100), n = 200 (p_min/u = 0.023): the
    4-step difference is 1.6e-3 at degree 10 and 8.4e-5 at 15."""
    params = np.zeros(ent.mlp_nparams(), dtype=np.float32)
    params[-2] = math.log(8.0)
    params[-1] = -1.2
    ent.selector_load(params)
    p = W.spectrum_exp(200, 100.0)
    R = torch.from_numpy(W.dense_density(p, 12)).to(DEV)
    auto = ent.entropy_estimate(R, "auto", 30, 32, 9, precision=precision)
    print(f"[auto stages {precision}] degree {auto.degree} products {auto.products} fell_back {auto.fell_back} "
          f"lo/u {auto.lo / auto.u:.3e}", flush=True)
    assert auto.fell_back == 0 and auto.degree == 15 and auto.products == 12 + 15
    direct = ent.entropy_estimate(R, "chebyshev", 15, 32, 9, precision=precision, u_fixed=auto.u,
                                  cutoff=auto.lo)
    assert auto.entropy == direct.entropy and auto.std_err == direct.std_err


def test_trained_selector_gain(orc):
    """What the committed network gains over the plain schedule.

    Held-out spectra of the training families (a seed the training never
    used), n = 1024, as diagonal matrices with sign probes: then
    g^T f(R) g = sum_i f(p_i) for every probe, so each estimate is the exact
    polynomial trace and its error vs H is the truncation error alone.  The
    plain schedule (Chebyshev on [0, u], degree 40) meets a 1e-3 relative
    error on about a third of them; the learned degree and cutoff must meet
    it on most, and every result must equal the oracle's polynomial trace at
    the (degree, cutoff, u) the selector chose."""
    ent.selector_load(L.load())
    rng = np.random.default_rng(424242)
    rows = []
    for i in range(24):
        p, fam = L.sample_spectrum(rng, 1024)
        H = float(-np.sum(p[p > 0] * np.log(p[p > 0])))
        R = torch.from_numpy(np.diag(p)).to(DEV)
        auto = ent.entropy_estimate(R, "auto", 40, 8, 100 + i, precision="f64")
        plain = ent.entropy_estimate(R, "chebyshev", 40, 8, 100 + i, precision="f64")
        # the oracle's polynomial trace at the selector's choice
        lo, u, m = auto.lo, auto.u, auto.degree
        a = orc.cheb_interp_coeffs(lo, u, m, orc.cutoff_nodes(m)) if lo > 0 else orc.cheb_coeffs(u, m)
        ref = -orc.cheb_quadform(W.diag_csr(p), a, lo, u, np.ones(len(p)))
        assert auto.entropy == pytest.approx(ref, rel=1e-9, abs=1e-12)
        rows.append((fam, abs(auto.entropy - H) / H, abs(plain.entropy - H) / H, auto.products,
                     plain.products, auto.fell_back, m, lo / u))
    fam, ea, ep, pa, pp, fb, ms, rho = (np.array(c) for c in zip(*rows))
    for r in rows:
        print(f"[gain] family {r[0]}: auto err {r[1]:.2e} (m={r[6]}, lo/u={r[7]:.1e}, products "
              f"{r[3]}, fell_back={r[5]})  plain err {r[2]:.2e} (products {r[4]})", flush=True)
    ok_a, ok_p = float(np.mean(ea <= 1e-3)), float(np.mean(ep <= 1e-3))
    print(f"[gain] within 1e-3: auto {ok_a:.2f}, plain {ok_p:.2f}; median error auto "
          f"{np.median(ea):.2e}, plain {np.median(ep):.2e}; products auto {pa.sum()}, plain "
          f"{pp.sum()}; fallbacks {int(fb.sum())}", flush=True)
    assert ok_a >= 0.75
    assert ok_a >= ok_p + 0.25
    assert np.median(ea) < 0.25 * np.median(ep)


def test_auto_moments_fit_the_callers_table():
    # the selector may pick a degree above the caller's; the moment table the
    # caller passes has (degree + 1) rows and must not be overrun
    ent.selector_load(L.load())
    p = W.spectrum_dirichlet(512, 300, 0.5, np.random.default_rng(3))
    R = torch.from_numpy(np.diag(p)).to(DEV)
    for deg in (4, 9):
        res, per, mom = ent.entropy_estimate_detail(R, "auto", deg, 8, 5, precision="f64")
        assert mom.shape == (deg + 1, 8)
        rows = min(res.degree, deg) + 1
        assert np.all(mom[rows:] == 0.0)
        assert np.all(np.isfinite(mom)) and np.all(np.isfinite(per))
        print(f"[auto moments] caller degree {deg}: selector degree {res.degree}, "
              f"fell_back={res.fell_back}", flush=True)


def test_selector_rejects_bad_params():
    with pytest.raises(ent.EntropyError):
        ent.selector_load(np.zeros(10, dtype=np.float32))


def test_simulated_features_match_library_features():
    """The training features are simulated from the spectrum alone (Gaussian
    directions in the eigenbasis stand for the sketch's probes under a Haar
    U).  On explicit R = U diag(p) U^T with random orthogonal U, the library's
    own sketch features must follow the same law: per feature, the means of
    48 library samples (6 matrices x 8 sketch seeds) and 2048 simulated ones
    agree within 5 standard errors, and the spreads within a factor of 2."""
    n = 512
    ent.selector_load(np.zeros(ent.mlp_nparams(), dtype=np.float32))
    rng = np.random.default_rng(17)
    cases = (("exp", W.spectrum_exp(n, 60.0)), ("power", W.spectrum_power(n, 1.0)),
             ("dirichlet", W.spectrum_dirichlet(n, 256, 0.5, rng)))
    for name, p in cases:
        lib = []
        for u_seed in range(6):
            R = torch.from_numpy(W.dense_density(p, 1000 + u_seed)).to(DEV)
            for s_seed in range(8):
                f, _ = ent.selector_features(R, 77 + 13 * s_seed)
                lib.append(f.astype(np.float64))
        lib = np.array(lib)
        P = np.tile(p, (2048, 1))
        sim, _, _, _ = L.batch_features_labels(P, np.ones_like(P), seed=5, device=DEV)
        sim = sim.cpu().numpy().astype(np.float64)
        for k in range(16):
            a, b = lib[:, k], sim[:, k]
            se = math.sqrt(a.var(ddof=1) / len(a) + b.var(ddof=1) / len(b))
            diff = abs(a.mean() - b.mean())
            print(f"[features {name}] f{k:2d} library {a.mean():+.5f} +- {a.std():.5f}  "
                  f"simulated {b.mean():+.5f} +- {b.std():.5f}  z={diff / max(se, 1e-12):.2f}", flush=True)
            assert diff <= 5.0 * se + 2e-5, (name, k)
            if b.std() > 1e-3:
                assert 0.5 <= a.std() / b.std() <= 2.0, (name, k)


def test_auto_routes_low_rank_to_randproj():
    """With ENT_FLAG_AUTO_RANDPROJ, a numerically low-rank R (sketch rank <=
    128 / 8) goes to Algorithm 3: the result is the random projection's own
    (bit-identical to calling it with width 128, k = 64), with 12 + 1
    products; its error is Algorithm 3's (the singular values of R Pi deviate
    from the eigenvalues by O(sqrt(rank / width)); at most 4.7% in 200
    simulated draws of each case below).  Without the flag nothing is
    routed; a full-rank spectrum is not routed, and a power law whose sketch
    looks low-rank (p_i ~ 1/i) is tried and rejected by the trace the
    singular values hold, costing one product."""
    ent.selector_load(np.zeros(ent.mlp_nparams(), dtype=np.float32))
    n = 1024
    F = ent.FLAG_AUTO_RANDPROJ
    for k, kind in ((8, "flat"), (12, "exp")):
        pk = np.ones(k) / k if kind == "flat" else np.exp(-np.arange(k) / 3.0)
        pk = pk / pk.sum()
        H = float(-np.sum(pk * np.log(pk)))
        R = W.low_rank_density_torch(pk, n, 40 + k, device=DEV)
        auto = ent.entropy_estimate(R, "auto", 40, 64, 5, flags=F)
        rp = ent.entropy_estimate(R, "randproj", 40, 64, 5, sketch_width=128, rank_k=64)
        plain = ent.entropy_estimate(R, "chebyshev", 40, 64, 5)
        print(f"[route rank {k} {kind}] H={H:.6f} auto={auto.entropy:.6f} (method {auto.method}, "
              f"products {auto.products}) plain m=40: {plain.entropy:.6f}", flush=True)
        assert auto.method == ent.RANDPROJ and auto.products == 13 and auto.fell_back == 0
        assert auto.entropy == rp.entropy
        assert abs(auto.entropy - H) / H < 0.06
        off = ent.entropy_estimate(R, "auto", 40, 64, 5)
        assert off.method == ent.AUTO
    full = ent.entropy_estimate(torch.from_numpy(W.dense_density(W.spectrum_exp(n, 60.0), 3)).to(DEV),
                                "auto", 40, 64, 5, flags=F)
    assert full.method == ent.AUTO
    assert full.products == 12 + full.degree if not full.fell_back else full.products > 12 + 40
    power = ent.entropy_estimate(torch.from_numpy(W.dense_density(W.spectrum_power(384, 1.0), 4)).to(DEV),
                                 "auto", 40, 64, 5, flags=F)
    print(f"[route power] method {power.method} products {power.products} degree {power.degree}", flush=True)
    assert power.method == ent.AUTO
    assert power.products == 13 + power.degree if not power.fell_back else power.products > 13 + 40
