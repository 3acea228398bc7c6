"""Pins for the oracle's 7L-CDC variant (Numerical Results, the paragraph
after Table 6.1: marginal collocation points from the map over [0, t_i], the
conditional points computed only at them, a global interpolation over them
per path, then the step's interpolation in X).

* Lagrange interpolation through m >= 2 nodes reproduces every function of
  degree < m exactly, and the analytic GBM and OU maps are affine in Y: CDC
  then equals 7L path by path, to rounding.
* The marginal points of the analytic GBM map are the quantiles of the
  lognormal law of Y(t_i) at Phi(x_k) (scipy's lognormal CDF); those of the
  OU map match the empirical quantiles of exact OU paths.
* With m = 2 the global interpolation is the straight line through the two
  marginal points (written out here), and at a marginal point it returns the
  conditional points computed there, bit for bit.
* CIR with the closed-form noncentral chi-square map: the CDC mean of Y_T
  lies within 4 standard errors of the exact CIR mean.
"""
import math
import os

import numpy as np
import pytest
from scipy.stats import lognorm, norm

import workloads as W
from nets import network_with_m_outputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GBM_WEIGHTS = os.path.join(ROOT, "tests", "golden", "gbm_mlp_4x64.sl7w")
OU_WEIGHTS = os.path.join(ROOT, "tests", "golden", "ou_mlp_5x50_softplus.sl7w")


def test_cdc_equals_7l_for_maps_affine_in_y(orc):
    paths = np.arange(20_000)
    c = W.CONFIGS["gbm_analytic_1e5x4"]
    for M in (4, 9):
        pr = orc.Problem(c["model"], c["theta"], c["Y0"], c["T"], M, c["m"])
        a, _, _ = orc.simulate(pr, None, c["seed"], paths)
        b, _, _ = orc.simulate_cdc(pr, None, c["seed"], paths)
        assert np.max(np.abs(a - b) / np.abs(a)) <= 1e-13, M
    P = W.OU_PAPER
    for m in (3, 5, 7):
        pr = orc.Problem(P["model"], P["theta"], P["Y0"], P["T"], P["M"], m)
        a, _, _ = orc.simulate(pr, None, P["seed"], paths)
        b, _, _ = orc.simulate_cdc(pr, None, P["seed"], paths)
        assert np.max(np.abs(a - b) / np.maximum(np.abs(a), 0.5)) <= 1e-13, m


def test_gbm_marginal_points_are_lognormal_quantiles(orc):
    c = W.CONFIGS["gbm_analytic_1e5x4"]
    sig, mu = c["theta"]
    pr = orc.Problem(c["model"], c["theta"], c["Y0"], c["T"], 8, 5)
    s, lams, ykj, _ = orc.cdc_tables(pr, None)
    x, _ = orc.gh_nodes(5)
    for i in range(1, 8):
        t = i * c["T"] / 8
        F = lognorm.cdf(s[i], sig * math.sqrt(t), scale=c["Y0"] * math.exp((mu - sig ** 2 / 2) * t))
        assert np.max(np.abs(F - norm.cdf(x))) <= 1e-12, i
        # barycentric weights of the marginal nodes
        for k in range(5):
            assert lams[i, k] == pytest.approx(1 / np.prod([s[i, k] - s[i, l] for l in range(5) if l != k]),
                                               rel=1e-12)


def test_ou_marginal_points_match_empirical_quantiles(orc):
    P = W.OU_PAPER
    M, n = 4, 200_000
    x, _ = orc.gh_nodes(5)
    s, _, _, _ = orc.cdc_tables(orc.Problem(P["model"], P["theta"], P["Y0"], P["T"], M, 5), None)
    for i in (1, 2, 3):
        # exact OU paths (analytic 7L is the exact transition) over i steps of T/M
        pr = orc.Problem(P["model"], P["theta"], P["Y0"], i * P["T"] / M, i, 5)
        y, _, _ = orc.simulate(pr, None, 1234, np.arange(n))
        p = norm.cdf(x)
        q = np.quantile(y, p)
        f = norm.pdf(x) / y.std()  # density of the (normal) law at its quantiles
        tol = 4 * np.sqrt(p * (1 - p) / n) / f
        assert np.all(np.abs(q - s[i]) <= tol), (i, q, s[i])


def test_global_interpolation_two_points_is_the_line_and_hits_nodes(orc):
    class _NoLib:
        class Mlp:
            @staticmethod
            def load(path):
                return None
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        _, H2 = network_with_m_outputs(_NoLib, 2, os.path.join(d, "m2.sl7w"))
    c = W.CONFIGS["gbm_mlp_2p22x16"]
    pr = orc.Problem(c["model"], c["theta"], c["Y0"], 0.5, 8, 2)
    tables = orc.cdc_tables(pr, H2)
    s, _, ykj, _ = tables
    rng = np.random.default_rng(5)
    for i in range(1, 8):
        for Y in np.concatenate([rng.uniform(s[i, 0] - 0.3, s[i, 1] + 0.3, 20), s[i]]):
            got = orc.cdc_collocation(tables, i, Y)
            line = ykj[i, 0] + (Y - s[i, 0]) * (ykj[i, 1] - ykj[i, 0]) / (s[i, 1] - s[i, 0])
            assert np.allclose(got, line, rtol=1e-13, atol=1e-14), (i, Y)
    # m = 5 network: a path at a marginal point gets that point's conditional row exactly
    Ho = orc.load_mlp(GBM_WEIGHTS)
    pr5 = orc.Problem(c["model"], c["theta"], c["Y0"], 0.5, 8, 5)
    t5 = orc.cdc_tables(pr5, Ho)
    for i in range(1, 8):
        for k in range(5):
            assert np.array_equal(orc.cdc_collocation(t5, i, t5[0][i, k]), t5[2][i, k])
    # step 0 is the map at Y0 itself
    dt = 0.5 / 8
    row = Ho.forward(np.array([[c["Y0"], dt, *c["theta"]]]))[0]
    assert np.array_equal(orc.cdc_collocation(t5, 0, c["Y0"]), row)


def test_cdc_cir_mean_matches_exact_mean(orc):
    for k in (5, 40):
        d = W.cir_instances(256)[k]
        pr = orc.Problem(d["model"], d["theta"], d["Y0"], d["T"], d["M"], 7)
        y, _, _ = orc.simulate_cdc(pr, None, 11, np.arange(200_000))
        kap, ybar, gam = d["theta"]
        e = math.exp(-kap * d["T"])
        exact = d["Y0"] * e + ybar * (1 - e)
        se = y.std() / math.sqrt(len(y))
        assert abs(y.mean() - exact) <= 4 * se, (k, y.mean(), exact, se)


def test_cdc_refuses_coincident_marginal_points(orc):
    c = W.CONFIGS["gbm_analytic_1e5x4"]
    pr = orc.Problem(c["model"], (1e-200, 0.1), c["Y0"], c["T"], 4, 5)
    with pytest.raises(ValueError):
        orc.cdc_tables(pr, None)
