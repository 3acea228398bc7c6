"""Pins for the oracle's network maths, training step, labels and CIR law.

* Forward and backward passes of H against torch float64 on the CPU (an
  independent library implementation of Linear + ReLU / Softplus and
  autograd), also at the paper's width of 50.
* Adam against torch.optim.Adam.
* Euler-Maruyama labels (eq. 6.2 with tiny steps, empirical quantiles at
  Phi(x_j)) converge to the closed-form GBM conditional quantiles.
* Type-7 quantiles against numpy.quantile.
* Noncentral chi-square CDF/quantile and the incomplete gamma function
  against scipy; the CIR analytic map keeps the exact conditional mean.
"""
import math
import os
import tempfile

import numpy as np
import pytest
import torch
from scipy import special, stats

import workloads as W


def _net(orc, seed=3, d_in=4, m=5, act=0, width=64):
    params = W.glorot_params(d_in, m, seed=seed, width=width)
    lo = W.GBM_DOMAIN_LO if d_in == 4 else W.CIR_DOMAIN_LO
    hi = W.GBM_DOMAIN_HI if d_in == 4 else W.CIR_DOMAIN_HI
    H = orc.glorot_mlp(d_in, width, 4, m, 0, lo, hi, params, act=act)
    rng = np.random.default_rng(seed)
    H.b = [b + rng.normal(scale=0.1, size=b.shape) for b in H.b]
    return H


def _torch_net(H):
    layers = []
    for l, (Wl, bl) in enumerate(zip(H.W, H.b)):
        lin = torch.nn.Linear(Wl.shape[1], Wl.shape[0]).double()
        with torch.no_grad():
            lin.weight.copy_(torch.from_numpy(Wl))
            lin.bias.copy_(torch.from_numpy(bl))
        layers.append(lin)
        if l < H.depth:
            # no linear cut-over: torch's Softplus returns x above its threshold
            layers.append(torch.nn.ReLU() if H.act == 0 else torch.nn.Softplus(threshold=1000.0))
    return torch.nn.Sequential(*layers)


@pytest.mark.parametrize("act", [0, 1])
def test_forward_vs_torch(orc, act):
    H = _net(orc, act=act)
    X = W.gbm_features(257, seed=5)
    ref = _torch_net(H)(torch.from_numpy(X * H.in_scale + H.in_shift)).detach().numpy()
    got_c = H.forward(X)
    got_b, _ = orc.mlp_forward_batch(H, X)
    assert np.max(np.abs(got_c - ref)) < 1e-13
    assert np.max(np.abs(got_b - ref)) < 1e-13


@pytest.mark.parametrize("act,width", [(0, 64), (1, 64), (1, 50)])
def test_backward_vs_torch_autograd(orc, act, width):
    H = _net(orc, act=act, width=width)
    X = W.gbm_features(300, seed=6)
    Y = np.random.default_rng(2).normal(size=(300, 5))
    loss, dW, db = orc.mse_loss_and_grads(H, X, Y)
    net = _torch_net(H)
    out = net(torch.from_numpy(X * H.in_scale + H.in_shift))
    tl = torch.mean((out - torch.from_numpy(Y)) ** 2)
    tl.backward()
    assert abs(loss - tl.item()) < 1e-13 * abs(loss)
    lins = [m for m in net if isinstance(m, torch.nn.Linear)]
    for l, lin in enumerate(lins):
        assert np.max(np.abs(dW[l] - lin.weight.grad.numpy())) < 1e-14
        assert np.max(np.abs(db[l] - lin.bias.grad.numpy())) < 1e-14


def test_adam_vs_torch(orc):
    rng = np.random.default_rng(0)
    p = rng.normal(size=50)
    tp = torch.tensor(p.copy(), requires_grad=True)
    opt = torch.optim.Adam([tp], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    st = orc.AdamState(np.zeros(50), np.zeros(50))
    for _ in range(20):
        g = rng.normal(size=50)
        p = orc.adam_step(p, g, st)
        opt.zero_grad()
        tp.grad = torch.tensor(g)
        opt.step()
    assert np.max(np.abs(p - tp.detach().numpy())) < 1e-14


def test_weight_file_roundtrip(orc):
    H = _net(orc)
    H = H.with_params(H.params_f32())
    H.meta = {"note": "roundtrip"}
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "h.sl7w")
        orc.save_mlp(H, path)
        G = orc.load_mlp(path)
    assert G.meta == {"note": "roundtrip"}
    assert np.array_equal(G.params_f32(), H.params_f32())
    assert np.array_equal(G.in_scale, H.in_scale) and np.array_equal(G.dom_hi, H.dom_hi)


def test_type7_quantiles_vs_numpy(orc):
    import ctypes
    rng = np.random.default_rng(4)
    v = np.sort(rng.normal(size=1001))
    probs = np.array([0.0, 0.00214, 0.1, 0.5, 0.77, 0.99786, 1.0])
    out = np.empty(len(probs))
    orc.lib().orc_type7_quantiles(orc._ptr(v), len(v), len(probs), orc._ptr(probs), orc._ptr(out))
    assert np.max(np.abs(out - np.quantile(v, probs))) < 1e-15


def test_em_labels_converge_to_gbm_quantiles(orc):
    """|label_j - q_j| within 4 sampling standard deviations
    sqrt(p(1-p)/n)/f(q) plus the Euler bias; 4x the paths roughly halves the
    average error."""
    feats = np.array([[1.0, 0.25, 0.3, 0.1], [0.7, 0.5, 0.5, 0.0], [1.4, 0.05, 0.1, 0.2]])
    x, _ = orc.gh_nodes(5)
    p = np.array([orc.Phi(v) for v in x])
    errs = {}
    for n in (10_000, 40_000):
        lab = orc.em_labels(orc.GBM, feats, 5, n, 100, seed=7)
        e = []
        for r, (Y, dt, sig, mu) in enumerate(feats):
            q = Y * np.exp((mu - 0.5 * sig ** 2) * dt + sig * math.sqrt(dt) * x)
            # lognormal density at q
            s = sig * math.sqrt(dt)
            f = stats.lognorm.pdf(q, s, scale=Y * math.exp((mu - 0.5 * sig ** 2) * dt))
            sd = np.sqrt(p * (1 - p) / n) / f
            bias = 1e-3 * Y * sig * math.sqrt(dt)
            assert np.all(np.abs(lab[r] - q) <= 4 * sd + bias), (n, r, lab[r], q)
            e.append(np.abs(lab[r] - q) / sd)
        errs[n] = np.mean(e)
    assert errs[40_000] < 2.0 and errs[10_000] < 2.0


def test_gammainc_and_ncx2_vs_scipy(orc):
    for a, z in [(0.3, 0.01), (0.3, 2.0), (2.5, 1.0), (7.0, 12.0), (40.0, 35.0), (500.0, 520.0)]:
        assert abs(orc.gammainc_lower(a, z) - special.gammainc(a, z)) < 1e-13
    for k, nc in [(0.4, 0.0), (0.4, 3.0), (2.5, 10.0), (8.0, 0.5), (1.2, 400.0)]:
        for pv in [0.00054827, 0.0307, 0.24, 0.5, 0.9, 0.99945]:
            ref = stats.ncx2.ppf(pv, k, nc) if nc > 0 else stats.chi2.ppf(pv, k)
            got = orc.ncx2_ppf(pv, k, nc)
            assert abs(got - ref) <= 1e-9 * max(ref, 1e-12), (k, nc, pv, got, ref)


def test_cir_analytic_map_keeps_conditional_mean(orc):
    """With many collocation nodes the quadrature of the CIR quantile map
    reproduces the exact conditional mean Y e^{-k dt} + ybar (1 - e^{-k dt})."""
    import ctypes
    kap, ybar, gam, Y, dt = 1.5, 0.06, 0.3, 0.08, 0.5
    m = 7
    x, w = orc.gh_nodes(m)
    e = math.exp(-kap * dt)
    c = gam ** 2 * (1 - e) / (4 * kap)
    d = 4 * kap * ybar / gam ** 2
    y = np.array([c * orc.ncx2_ppf(orc.Phi(v), d, Y * e / c) for v in x])
    exact = Y * e + ybar * (1 - e)
    assert abs(np.sum(w * y) - exact) < 2e-3 * exact
