"""Writes the stored collocation networks shared by the oracle and the GPU path.

Calls only ``oracle`` and ``workloads``: labels are the oracle's Euler-Maruyama
quantile labels (Algorithm I step 1; eq. 6.2 with 100 substeps, 10^4 paths
per label, empirical quantiles at Phi(x_j)) or, for CIR, its closed-form
noncentral chi-square quantiles; training is the oracle's FP64 Adam with
Glorot initial weights, batch 1024 and learning rate 1e-3 (Numerical Results
section).  The result is rounded to FP32 when written.

    python tests/golden/make_weights.py gbm [--epochs 200]
    python tests/golden/make_weights.py cir [--epochs 200]
    python tests/golden/make_weights.py ou  [--epochs 200]   (4 x 50 Softplus, EM labels)
"""
import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def cir_labels(features: np.ndarray, m: int) -> np.ndarray:
    """Closed-form CIR conditional quantiles at Phi(x_j) (oracle routine)."""
    from concurrent.futures import ThreadPoolExecutor
    x, _ = oracle.gh_nodes(m)
    probs = [oracle.Phi(v) for v in x]

    def one(r):
        Y, dt, kap, ybar, gam = features[r]
        e = np.exp(-kap * dt)
        c = gam * gam * (1 - e) / (4 * kap)
        d = 4 * kap * ybar / (gam * gam)
        return [c * oracle.ncx2_ppf(p, d, Y * e / c) for p in probs]

    with ThreadPoolExecutor(oracle.n_threads()) as ex:
        return np.array(list(ex.map(one, range(len(features)))))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("model", choices=["gbm", "cir", "ou"])
    ap.add_argument("--epochs", type=int, default=200)
    ap.add_argument("--labels", type=int, default=W.N_LABELS)
    args = ap.parse_args()
    t0 = time.time()
    if args.model == "gbm":
        d_in, m, model = 4, 5, oracle.GBM
        lo, hi = W.GBM_DOMAIN_LO, W.GBM_DOMAIN_HI
        feats = W.gbm_features(args.labels)
        labels = oracle.em_labels(model, feats, m, W.LABEL_PATHS, W.LABEL_SUBSTEPS, seed=W.TRAIN_SEED)
        out = os.path.join(HERE, "gbm_mlp_4x64.sl7w")
    elif args.model == "ou":
        d_in, m, model = 5, 5, oracle.OU
        lo, hi = W.OU_DOMAIN_LO, W.OU_DOMAIN_HI
        feats = W.ou_features(args.labels)
        labels = oracle.em_labels(model, feats, m, W.LABEL_PATHS, W.LABEL_SUBSTEPS, seed=W.TRAIN_SEED)
        out = os.path.join(HERE, "ou_mlp_5x50_softplus.sl7w")
    else:
        d_in, m, model = 5, 7, oracle.CIR
        lo, hi = W.CIR_DOMAIN_LO, W.CIR_DOMAIN_HI
        feats = W.cir_features(args.labels)
        labels = cir_labels(feats, m)
        out = os.path.join(HERE, "cir_mlp_5x64.sl7w")
    print(f"labels: {time.time() - t0:.1f} s", flush=True)
    width = W.OU_WIDTH if args.model == "ou" else W.WIDTH
    act = oracle.ACT_SOFTPLUS if args.model == "ou" else oracle.ACT_RELU
    H0 = oracle.glorot_mlp(d_in, width, W.DEPTH, m, model, lo, hi,
                           W.glorot_params(d_in, m, seed=W.TRAIN_SEED, width=width), act=act)
    order = W.minibatch_order(len(feats), args.epochs, seed=W.TRAIN_SEED)
    H, hist = oracle.train(H0, feats, labels, order, batch=W.BATCH, lr=1e-3, log_every=20)
    H = H.with_params(H.params_f32())
    final = float(np.mean(hist[-(len(feats) // W.BATCH):]))
    H.meta = {"trainer": "oracle fp64 adam", "epochs": args.epochs, "labels": len(feats),
              "seed": W.TRAIN_SEED, "batch": W.BATCH, "lr": 1e-3, "final_epoch_loss": final}
    oracle.save_mlp(H, out)
    print(f"wrote {out}: final epoch loss {final:.4e}, {time.time() - t0:.1f} s", flush=True)


if __name__ == "__main__":
    main()
