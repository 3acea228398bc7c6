"""The stored OU network (the paper's 4 x 50 Softplus shape, trained by the
oracle on Euler-Maruyama labels) against the closed-form OU law (eq. 6.6).

The OU transition over dt is normal with mean Y e^{-lambda dt} +
ybar (1 - e^{-lambda dt}) and variance sigma^2 (1 - e^{-2 lambda dt}) /
(2 lambda), so its conditional collocation values are exactly
mean + sd x_j.  The labels the network was fitted to are empirical quantiles
of 10^4 EM paths, whose sampling error is about 1.5 % of sd; the bounds below
allow a few times that.
"""
import os

import numpy as np

import oracle
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WEIGHTS = os.path.join(ROOT, "tests", "golden", "ou_mlp_5x50_softplus.sl7w")


def exact_collocation(f, m):
    x, _ = oracle.gh_nodes(m)
    Y, dt, ybar, sig, lam = f.T
    e = np.exp(-lam * dt)
    mean = Y * e + ybar * (1 - e)
    sd = sig * np.sqrt((1 - e * e) / (2 * lam))
    return mean[:, None] + sd[:, None] * x[None, :], sd


def test_stored_network_is_the_papers_shape():
    H = oracle.load_mlp(WEIGHTS)
    assert (H.d_in, H.width, H.depth, H.m, H.act, H.model) == (5, 50, 4, 5, oracle.ACT_SOFTPLUS,
                                                               W.OU)
    assert H.meta["epochs"] == 200 and H.meta["labels"] == W.N_LABELS


def test_network_matches_closed_form_collocation_values():
    H = oracle.load_mlp(WEIGHTS)
    f = W.ou_features(2000, seed=123)
    ex, sd = exact_collocation(f, H.m)
    err = np.abs(H.forward(f) - ex)
    rms = np.sqrt((err ** 2).mean())
    print("OU network vs closed form: max", err.max(), "rms", rms)
    assert rms <= 0.01
    assert err.max() <= 0.08
    # no node is biased by more than a fraction of the label noise
    assert np.abs((H.forward(f) - ex).mean(0)).max() <= 3e-3


def test_7l_with_network_tracks_the_exact_law():
    H = oracle.load_mlp(WEIGHTS)
    P = W.OU_PAPER
    pr = oracle.Problem(P["model"], P["theta"], P["Y0"], P["T"], P["M"], P["m"], 0)
    paths = np.arange(20_000)
    ya, _, _ = oracle.simulate(pr, None, P["seed"], paths)
    ym, _, nood = oracle.simulate(pr, H, P["seed"], paths)
    assert nood == 0
    ybar, sig, lam = P["theta"]
    e = np.exp(-lam * P["T"])
    mean_T = P["Y0"] * e + ybar * (1 - e)
    var_T = sig ** 2 * (1 - e * e) / (2 * lam)
    se = ya.std() / np.sqrt(len(ya))
    # the analytic map is the exact law; the network adds its fitting error
    assert abs(ya.mean() - mean_T) <= 4 * se
    assert abs(ym.mean() - mean_T) <= 4 * se + 5e-3
    assert abs(ym.var() / var_T - 1) <= 0.05
    assert np.sqrt(((ym - ya) ** 2).mean()) <= 0.01
