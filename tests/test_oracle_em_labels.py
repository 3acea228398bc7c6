"""Pins for the oracle's Euler-Maruyama labels of the OU and CIR models.

The offline labels (Algorithm I step 1) are empirical quantiles at Phi(x_j)
of many Euler-Maruyama paths (eq. 6.2) with 100 substeps.  The GBM labels are
pinned in ``test_oracle_mlp_labels.py``; here the same pin for the other two
drift/diffusion branches, against laws fixed by the mathematics:

* OU (eq. 6.5).  Euler-Maruyama for a linear SDE with additive noise is
  itself Gaussian: after S substeps of size d from Y, with r = 1 - lambda d,
  the mean is ybar + (Y - ybar) r^S and the variance
  sigma^2 d (1 - r^{2S}) / (1 - r^2).  Labels must sit within 4 sampling
  standard deviations sqrt(p(1-p)/n)/f(q) of that law's quantiles, and that
  law must sit within its own O(d) distance of the exact transition (eq. 6.6).
* CIR.  The exact transition is a scaled noncentral chi-square law
  (c chi'^2(d, Y e^{-kappa dt}/c)); its quantiles come from scipy (a library
  independent of the oracle).  Full truncation keeps the raw state, so below
  the Euler step's scale gamma^2 d the labels may undershoot zero; there the
  pin is an absolute bound of that scale.
A wrong sign or a dropped term in either branch's drift or diffusion moves
the labels by many standard deviations.
"""
import math

import numpy as np
from scipy import stats


def _probs(orc, m):
    x, _ = orc.gh_nodes(m)
    return x, np.array([orc.Phi(v) for v in x])


def _ou_em_law(Y, dt, ybar, sig, lam, S):
    d = dt / S
    r = 1.0 - lam * d
    mean = ybar + (Y - ybar) * r ** S
    var = sig * sig * d * (1.0 - r ** (2 * S)) / (1.0 - r * r)
    return mean, math.sqrt(var)


def test_ou_em_labels_follow_their_gaussian_law(orc):
    feats = np.array([[0.2, 0.25, 0.5, 0.3, 1.0],
                      [-0.8, 0.5, 1.0, 0.5, 2.5],
                      [1.7, 0.05, 0.0, 0.1, 0.5]])
    x, p = _probs(orc, 5)
    S = 100
    errs = {}
    for n in (10_000, 40_000):
        lab = orc.em_labels(orc.OU, feats, 5, n, S, seed=7)
        e = []
        for r, (Y, dt, ybar, sig, lam) in enumerate(feats):
            mean, sd_law = _ou_em_law(Y, dt, ybar, sig, lam, S)
            q = mean + sd_law * x
            f = stats.norm.pdf(q, loc=mean, scale=sd_law)
            sd = np.sqrt(p * (1 - p) / n) / f
            assert np.all(np.abs(lab[r] - q) <= 4 * sd), (n, r, lab[r], q)
            e.append(np.abs(lab[r] - q) / sd)
        errs[n] = float(np.mean(e))
    assert errs[10_000] < 2.0 and errs[40_000] < 2.0, errs


def test_ou_em_law_near_exact_transition():
    """The Euler law above against eq. 6.6 over the same step: the mean and
    standard deviation differ by O(lambda d) relative."""
    for Y, dt, ybar, sig, lam in [(0.2, 0.25, 0.5, 0.3, 1.0), (-0.8, 0.5, 1.0, 0.5, 2.5)]:
        S = 100
        mean, sd = _ou_em_law(Y, dt, ybar, sig, lam, S)
        e = math.exp(-lam * dt)
        mean_x = Y * e + ybar * (1 - e)
        sd_x = sig * math.sqrt((1 - math.exp(-2 * lam * dt)) / (2 * lam))
        d = dt / S
        assert abs(mean - mean_x) <= lam * d * abs(Y - ybar)
        assert abs(sd - sd_x) <= lam * d * sd_x


def _cir_law(Y, dt, kap, ybar, gam):
    e = math.exp(-kap * dt)
    c = gam * gam * (1 - e) / (4 * kap)
    return c, 4 * kap * ybar / (gam * gam), Y * e / c


def test_cir_em_labels_converge_to_noncentral_chi2_quantiles(orc):
    # Three features with 2 kappa ybar > gamma^2 (the law has no mass at 0)
    # and one without (C4's parameter ranges include both).
    feats = np.array([[0.08, 0.5, 1.5, 0.06, 0.3],
                      [0.5, 0.2, 2.0, 0.1, 0.2],
                      [0.02, 0.3, 2.5, 0.03, 0.25],
                      [0.05, 1.0, 0.5, 0.05, 0.45]])
    m = 7
    _, p = _probs(orc, m)
    S = 100
    errs = {}
    for n in (10_000, 40_000):
        lab = orc.em_labels(orc.CIR, feats, m, n, S, seed=7)
        e = []
        for r, (Y, dt, kap, ybar, gam) in enumerate(feats):
            c, d, nc = _cir_law(Y, dt, kap, ybar, gam)
            q = c * stats.ncx2.ppf(p, d, nc)
            f = stats.ncx2.pdf(q / c, d, nc) / c
            sd = np.sqrt(p * (1 - p) / n) / f
            step = gam * gam * dt / S  # the Euler step's scale near zero
            body = q > 10 * step
            assert np.all(np.abs(lab[r][body] - q[body]) <= 4 * sd[body]), (n, r, lab[r], q)
            assert np.all(np.abs(lab[r][~body] - q[~body]) <= 4 * step), (n, r, lab[r], q)
            if 2 * kap * ybar > gam * gam:
                e.append(np.abs(lab[r] - q) / sd)
        errs[n] = float(np.mean(e))
    assert errs[10_000] < 2.0 and errs[40_000] < 2.0, errs
