"""Pins for the oracle's online stage (Algorithm I) and its derivatives.

* GBM with the analytic collocation map: Gauss quadrature with m nodes is
  exact for polynomials of degree <= 2m-1 and E[L_j(X)] = w_j, so
  E[Y_T] = Y0 (sum_j w_j e^{a + b x_j})^M and E[Y_T^2] = Y0^2 (sum_j w_j
  e^{2(a + b x_j)})^M in closed form; the Monte Carlo estimates must sit
  within 4 standard errors, and the call price within 4 SE of Black-Scholes.
* OU (eq. 6.5/6.6) with its analytic map: the conditional law is Gaussian,
  so the collocation points are linear in x_j and 7L reproduces the exact
  transition path by path.
* The GBM analytic scheme is homogeneous of degree one in Y0, so the
  pathwise delta equals Y_T / Y0.
* Forward-mode tangents agree with central differences of the oracle.
"""
import math
import os

import numpy as np
import pytest
from scipy.stats import norm

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _c0_problem(orc):
    c = W.CONFIGS["gbm_analytic_1e5x4"]
    return orc.Problem(c["model"], c["theta"], c["Y0"], c["T"], c["M"], c["m"])


def test_gbm_analytic_closed_form_mean_and_second_moment(orc):
    c = W.CONFIGS["gbm_analytic_1e5x4"]
    sig, mu = c["theta"]
    dt = c["T"] / c["M"]
    x, w = orc.gh_nodes(c["m"])
    a, b = (mu - 0.5 * sig ** 2) * dt, sig * math.sqrt(dt)
    m1 = c["Y0"] * np.sum(w * np.exp(a + b * x)) ** c["M"]
    m2 = c["Y0"] ** 2 * np.sum(w * np.exp(2 * (a + b * x))) ** c["M"]
    # quadrature of e^{bX} with 5 nodes: relative error far below 1e-11 here
    assert abs(m1 - math.exp(mu * c["T"])) < 1e-11
    assert abs(m1 - 1.10517091807481) < 1e-13
    YT, _, _ = orc.simulate(_c0_problem(orc), None, c["seed"], np.arange(c["N"]))
    e1 = orc.estimate(YT)
    assert abs(e1["mean"] - m1) < 4 * e1["se"]
    e2 = orc.estimate(YT ** 2)
    assert abs(e2["mean"] - m2) < 4 * e2["se"]
    # call: Black-Scholes with drift mu; the 7L bias is ~1e-7, far below SE
    K, T, Y0 = c["K"], c["T"], c["Y0"]
    d1 = (math.log(Y0 / K) + (mu + 0.5 * sig ** 2) * T) / (sig * math.sqrt(T))
    d2 = d1 - sig * math.sqrt(T)
    bs = Y0 * math.exp(mu * T) * norm.cdf(d1) - K * norm.cdf(d2)
    assert abs(bs - 0.184940777744) < 1e-11
    ec = orc.estimate(np.maximum(YT - K, 0.0))
    assert abs(ec["mean"] - bs) < 4 * ec["se"]


def test_ou_analytic_7l_equals_exact_transition(orc):
    ybar, sig, lamr = 0.5, 0.4, 1.7
    pr = orc.Problem(orc.OU, (ybar, sig, lamr), 0.2, 2.0, 8, 5, instance=1)
    paths = np.arange(500)
    YT, _, _ = orc.simulate(pr, None, 9, paths)
    X = orc.step_normals(9, orc.make_tag(0, 1), paths, pr.M)
    dt = pr.T / pr.M
    e = math.exp(-lamr * dt)
    sd = sig * math.sqrt((1 - math.exp(-2 * lamr * dt)) / (2 * lamr))
    Y = np.full(len(paths), pr.Y0)
    for i in range(pr.M):
        Y = Y * e + ybar * (1 - e) + sd * X[:, i]
    assert np.max(np.abs(YT - Y)) < 1e-13


def test_gbm_analytic_homogeneous_in_y0(orc):
    pr1 = orc.Problem(orc.GBM, (0.3, 0.1), 1.0, 1.0, 4, 5)
    pr2 = orc.Problem(orc.GBM, (0.3, 0.1), 2.0, 1.0, 4, 5)
    paths = np.arange(2000)
    y1, _, _ = orc.simulate(pr1, None, 42, paths)
    y2, _, _ = orc.simulate(pr2, None, 42, paths)
    assert np.max(np.abs(y2 - 2 * y1) / (2 * y1)) < 1e-14
    _, dY = orc.simulate_tangent(pr1, None, 42, paths)
    assert np.max(np.abs(dY[:, 0] - y1) / y1) < 1e-13


def test_gbm_exact_path_close_to_7l(orc):
    """Per path, the 7L analytic scheme tracks the exact lognormal path driven
    by the same normals (the Lagrange remainder is the only difference)."""
    pr = _c0_problem(orc)
    paths = np.arange(20000)
    YT, _, _ = orc.simulate(pr, None, 42, paths)
    X = orc.step_normals(42, orc.make_tag(0, 0), paths, pr.M)
    sig, mu = pr.theta
    dt = pr.T / pr.M
    exact = pr.Y0 * np.exp(np.sum((mu - 0.5 * sig ** 2) * dt + sig * math.sqrt(dt) * X, axis=1))
    rel = np.abs(YT - exact) / exact
    assert np.mean(rel) < 3e-5 and np.max(rel) < 2e-2


def _fd(orc, pr, H, seed, paths, p, h):
    def with_param(delta):
        th = list(pr.theta)
        y0 = pr.Y0
        if p == 0:
            y0 += delta
        else:
            th[p - 1] += delta
        return orc.Problem(pr.model, tuple(th), y0, pr.T, pr.M, pr.m, pr.instance)
    yp, _, _ = orc.simulate(with_param(h), H, seed, paths)
    ym, _, _ = orc.simulate(with_param(-h), H, seed, paths)
    return (yp - ym) / (2 * h)


@pytest.mark.parametrize("model,theta", [(0, (0.3, 0.1)), (1, (0.5, 0.4, 1.7))])
def test_tangents_vs_central_differences_analytic(orc, model, theta):
    pr = orc.Problem(model, theta, 1.0, 1.0, 6, 5)
    paths = np.arange(300)
    _, dY = orc.simulate_tangent(pr, None, 5, paths)
    for p in range(1 + len(theta)):
        fd = _fd(orc, pr, None, 5, paths, p, 1e-6)
        assert np.max(np.abs(dY[:, p] - fd)) < 1e-7 * (1 + np.max(np.abs(fd)))


def test_tangents_vs_central_differences_mlp(orc):
    params = W.glorot_params(4, 5, seed=3)
    H = orc.glorot_mlp(4, 64, 4, 5, orc.GBM, W.GBM_DOMAIN_LO, W.GBM_DOMAIN_HI, params)
    # shift the output bias so the map is near identity in Y, like a trained net
    H.b[-1] = H.b[-1] + 1.0
    pr = orc.Problem(orc.GBM, (0.3, 0.1), 1.0, 1.0, 4, 5)
    paths = np.arange(200)
    _, dY = orc.simulate_tangent(pr, H, 8, paths)
    for p in range(3):
        fd = _fd(orc, pr, H, 8, paths, p, 1e-7)
        # ReLU kinks make a few paths non-differentiable within +-h
        bad = np.abs(dY[:, p] - fd) > 1e-6 * (1 + np.abs(fd))
        assert bad.mean() < 0.02


def test_tangents_vs_central_differences_softplus_ou(orc):
    """The stored OU network (4 x 50 Softplus, smooth): forward-mode tangents
    in (Y0, ybar, sigma, lambda) against central differences on every path."""
    H = orc.load_mlp(os.path.join(ROOT, "tests", "golden", "ou_mlp_5x50_softplus.sl7w"))
    P = W.OU_PAPER
    pr = orc.Problem(P["model"], P["theta"], P["Y0"], P["T"], P["M"], P["m"])
    paths = np.arange(200)
    _, dY = orc.simulate_tangent(pr, H, 8, paths)
    for p in range(4):
        fd = _fd(orc, pr, H, 8, paths, p, 1e-6)
        assert np.max(np.abs(dY[:, p] - fd)) <= 1e-6 * (1 + np.max(np.abs(fd))), p


def test_em_large_step_mean(orc):
    """E[Y_T] under large-step EM for GBM is Y0 (1 + mu dt)^M exactly."""
    pr = orc.Problem(orc.GBM, (0.3, 0.1), 1.0, 1.0, 4, 5)
    YT = orc.em_paths(pr, 42, np.arange(100_000))
    e = orc.estimate(YT)
    assert abs(e["mean"] - 1.025 ** 4) < 4 * e["se"]


def test_estimators(orc):
    v = np.random.default_rng(1).normal(3.0, 2.0, size=10001)
    e = orc.estimate(v)
    assert abs(e["mean"] - math.fsum(v) / len(v)) < 1e-15 * abs(e["mean"])
    assert abs(e["var"] - np.var(v, ddof=1)) < 1e-12 * e["var"]
    assert orc.neumaier_sum([1e16, 1.0, -1e16]) == 1.0
