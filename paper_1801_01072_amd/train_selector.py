"""Train the learned degree / lower-cutoff selector and write its weights.

    python -m paper_1801_01072_amd.train_selector --count 200000 --out selector_weights.npz

Training spectra (power law, exponential, rank-deficient Dirichlet) and their
simulated sketch features come from `learned.make_dataset`; the network is
trained by the library's own MLP forward/backward and Adam kernels.  A
held-out simulated set (other seed) reports the validation loss and how often
the decoded degree (with the library's 25% margin) reaches the label.
"""
from __future__ import annotations

import argparse
import sys
import time

import numpy as np


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--count", type=int, default=200000)
    ap.add_argument("--val", type=int, default=8192)
    ap.add_argument("--n-lo", type=int, default=256)
    ap.add_argument("--n-hi", type=int, default=4096)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--batch", type=int, default=2048)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--seed", type=int, default=2024)
    ap.add_argument("--chunk", type=int, default=1024)
    ap.add_argument("--out", required=True)
    args = ap.parse_args(argv)

    import torch

    from paper_1801_01072_amd import learned as L

    dev = "cuda:0" if torch.cuda.is_available() else "cpu"

    def log(msg):
        print(msg, flush=True)

    t0 = time.time()
    parts_x, parts_t = [], []
    made = 0
    step = max(args.chunk * 16, args.count // 10)
    while made < args.count:
        b = min(step, args.count - made)
        X, T, _ = L.make_dataset(b, args.n_lo, args.n_hi, seed=args.seed + made, device=dev,
                                 chunk=args.chunk)
        parts_x.append(X)
        parts_t.append(T)
        made += b
        log(f"data {made}/{args.count} ({time.time() - t0:.1f} s)")
    X = torch.cat(parts_x)
    T = torch.cat(parts_t)
    Xv, Tv, Fv = L.make_dataset(args.val, args.n_lo, args.n_hi, seed=args.seed + 10**7, device=dev,
                                chunk=args.chunk)
    t_data = time.time() - t0
    log(f"data done: {X.shape[0]} train, {Xv.shape[0]} validation, {t_data:.1f} s")

    t1 = time.time()
    params, losses = L.train(X, T, epochs=args.epochs, batch=args.batch, lr=args.lr, seed=args.seed,
                             log=log)
    if dev != "cpu":
        torch.cuda.synchronize()
    t_train = time.time() - t1

    import paper_1801_01072_amd as ent

    _, vloss = ent.mlp_grad(params, Xv, Tv)
    Y = ent.mlp_forward(params, Xv).cpu().numpy().astype(np.float64)
    tv = Tv.cpu().numpy().astype(np.float64)
    m_label = np.exp(tv[:, 0])
    m_pred = np.ceil(1.25 * np.exp(Y[:, 0]))
    cover = float(np.mean(m_pred >= np.round(m_label)))
    log(f"train {t_train:.1f} s, final loss {losses[-1]:.5f}, validation loss {vloss:.5f}, "
        f"degree covered on {100 * cover:.1f}% of validation samples, "
        f"mean predicted m {m_pred.mean():.1f} vs label {m_label.mean():.1f}")
    L.save(params, args.out, losses=np.asarray(losses), val_loss=np.float64(vloss),
           cover=np.float64(cover), count=np.int64(args.count), n_lo=np.int64(args.n_lo),
           n_hi=np.int64(args.n_hi), epochs=np.int64(args.epochs), seed=np.int64(args.seed),
           data_seconds=np.float64(t_data), train_seconds=np.float64(t_train))
    log(f"wrote {args.out}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
