"""The stored GBM network (C1-C3; 4 -> 4 x 64 ReLU -> 5, trained by the oracle
on Euler-Maruyama quantile labels) against the closed-form lognormal law.

Over one step of length dt the GBM transition is lognormal, so the
conditional collocation values are exactly y_j = Y exp((mu - sigma^2/2) dt +
sigma sqrt(dt) x_j).  What limits the network is measured here:

* the labels' sampling noise: an empirical quantile at p_j = Phi(x_j) of
  n = 10^4 paths has relative standard deviation
  sigma sqrt(dt) sqrt(p_j (1 - p_j) / n) / phi(x_j);
* the labels' bias: Euler-Maruyama with 100 substeps against the exact law,
  from 4 x 10^5 paths at the C1 point;
* the network's own error, per node, over the training domain and at the
  C1 / C2 points, and the per-step bias of E[Y_{i+1} | Y_i] it implies,
  beside Euler's exact per-step mean Y (1 + mu dt).
"""
import os

import numpy as np
from scipy.stats import norm

import oracle
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WEIGHTS = os.path.join(ROOT, "tests", "golden", "gbm_mlp_4x64.sl7w")


def exact_collocation(f, x):
    Y, dt, sig, mu = f.T
    return Y[:, None] * np.exp(((mu - 0.5 * sig * sig) * dt)[:, None]
                               + (sig * np.sqrt(dt))[:, None] * x[None, :])


def label_noise(f, x, n=W.LABEL_PATHS):
    p = norm.cdf(x)
    b = f[:, 2] * np.sqrt(f[:, 1])
    return b[:, None] * np.sqrt(p * (1 - p) / n)[None, :] / norm.pdf(x)[None, :]


def test_network_against_the_lognormal_law_over_its_domain():
    H = oracle.load_mlp(WEIGHTS)
    x, _ = oracle.gh_nodes(H.m)
    f = W.gbm_features(4000, seed=321)
    ex = exact_collocation(f, x)
    rel = (H.forward(f) - ex) / ex
    rms = np.sqrt((rel ** 2).mean(0))
    noise = np.sqrt((label_noise(f, x) ** 2).mean(0))
    print("GBM network vs lognormal law, relative rms per node", rms.round(5),
          "mean", rel.mean(0).round(5), "; one label's sampling noise", noise.round(5))
    # measured: rms [0.0070 0.0030 0.0026 0.0022 0.0045]; the label noise of a
    # single label is [0.0117 0.0030 0.0021 0.0030 0.0117]
    assert np.all(rms <= 0.01)
    assert np.abs(rel).max() <= 0.06
    # the fit does not average the noise of the 2^16 labels away: its error is
    # of the order of one label's noise at the inner nodes
    assert np.all(rms[1:4] >= 0.5 * noise[1:4])


def test_label_bias_is_below_the_networks_error_at_the_c1_point():
    H = oracle.load_mlp(WEIGHTS)
    x, w = oracle.gh_nodes(H.m)
    c = W.CONFIGS["gbm_mlp_2p22x16"]
    dt = c["T"] / c["M"]
    sig, mu = c["theta"]
    f = np.array([[c["Y0"], dt, sig, mu]])
    ex = exact_collocation(f, x)[0]
    lab = oracle.em_labels(W.GBM, f, H.m, 400_000, W.LABEL_SUBSTEPS, seed=3)[0]
    net = H.forward(f)[0]
    sd = label_noise(f, x, n=400_000)[0]
    bias_lab = (lab - ex) / ex
    err_net = (net - ex) / ex
    step_net = w @ net / (c["Y0"] * np.exp(mu * dt)) - 1
    step_euler = (1 + mu * dt) / np.exp(mu * dt) - 1
    print(f"C1 point (dt = {dt}): label bias {bias_lab.round(5)} (+- {sd.round(5)}), network "
          f"error {err_net.round(5)}; per-step mean bias: network {step_net:+.2e}, Euler "
          f"{step_euler:+.2e}")
    # Euler's labels with 100 substeps are within a few sampling SD of the law
    assert np.all(np.abs(bias_lab) <= 4 * sd + 1e-4)
    # the network's per-step bias is far above Euler's exact-mean step: over
    # M = 16 steps it accumulates to the weak error the benchmark reports
    assert abs(step_net) > 10 * abs(step_euler)
    assert np.max(np.abs(err_net)) > 3 * np.max(np.abs(bias_lab))
