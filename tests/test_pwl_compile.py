"""The exact piecewise-linear form of a ReLU collocation network along Y
(sl7_pwl_compile, host code of the library) against the oracle's forward
pass of the same network.

For a fixed instance (dt, theta) the network's only varying input is Y; a
ReLU network is then continuous and piecewise linear in Y.  The compiled
pieces must reproduce the oracle's FP64 forward pass everywhere (dense grids,
at and next to every breakpoint, far outside the training domain), be
continuous across breakpoints, and account for every slope change that
brute-force sampling finds on a small network.
"""
import ctypes
import os

import numpy as np
import pytest

import oracle
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GBM_W = os.path.join(ROOT, "tests", "golden", "gbm_mlp_4x64.sl7w")
CIR_W = os.path.join(ROOT, "tests", "golden", "cir_mlp_5x64.sl7w")
OU_W = os.path.join(ROOT, "tests", "golden", "ou_mlp_5x50_softplus.sl7w")


@pytest.fixture(scope="module")
def S():
    import paper_2302_05170_amd as S
    return S


def evaluate(pw, Y):
    idx = np.searchsorted(pw["breaks"], Y, side="right")
    return pw["value"][idx] + pw["slope"][idx] * (Y - pw["anchor"][idx])[:, None]


def features(model, Y, dt, theta):
    cols = [Y, np.full_like(Y, dt)] + [np.full_like(Y, t) for t in theta]
    return np.stack(cols, 1)


def probe_points(pw, lo, hi):
    b = pw["breaks"]
    return np.concatenate([np.linspace(lo, hi, 20001), b, b + 1e-9 * np.maximum(1, abs(b)),
                           b - 1e-9 * np.maximum(1, abs(b)), [-1e6, 1e6]])


@pytest.mark.parametrize("case", ["gbm_mlp_2p22x16", "gbm_mlp_2p24x32"])
def test_gbm_network_pieces_match_oracle(S, case):
    c = W.CONFIGS[case]
    H, Ho = S.Mlp.load(GBM_W), oracle.load_mlp(GBM_W)
    pr = S.Problem(c["model"], c["theta"], c["Y0"], c["T"], c["M"], c["m"], 100)
    pw = S.pwl_compile(H, pr)
    P = len(pw["anchor"])
    assert 2 <= P < 2000 and len(pw["breaks"]) == P - 1
    assert np.all(np.diff(pw["breaks"]) > 0)
    Y = probe_points(pw, -5.0, 8.0)
    ref = Ho.forward(features(c["model"], Y, c["T"] / c["M"], c["theta"]))
    err = np.abs(evaluate(pw, Y) - ref) / np.maximum(np.abs(ref), 1e-3)
    print(case, "pieces", P, "max rel err", err.max())
    assert err.max() <= 1e-12


def test_cir_network_pieces_match_oracle(S):
    H, Ho = S.Mlp.load(CIR_W), oracle.load_mlp(CIR_W)
    for d in W.cir_instances(8):
        pr = S.Problem(d["model"], d["theta"], d["Y0"], d["T"], d["M"], d["m"], 100)
        pw = S.pwl_compile(H, pr)
        Y = probe_points(pw, -0.5, 2.0)
        ref = Ho.forward(features(d["model"], Y, d["T"] / d["M"], d["theta"]))
        err = np.abs(evaluate(pw, Y) - ref) / np.maximum(np.abs(ref), 1e-3)
        assert err.max() <= 1e-12, d


def test_pieces_are_continuous(S):
    c = W.CONFIGS["gbm_mlp_2p24x32"]
    pw = S.pwl_compile(S.Mlp.load(GBM_W), S.Problem(c["model"], c["theta"], c["Y0"], c["T"], c["M"],
                                                    c["m"], 100))
    b = pw["breaks"]
    left = pw["value"][:-1] + pw["slope"][:-1] * (b - pw["anchor"][:-1])[:, None]
    right = pw["value"][1:] + pw["slope"][1:] * (b - pw["anchor"][1:])[:, None]
    scale = np.maximum(np.abs(left), 1e-3)
    assert np.max(np.abs(left - right) / scale) <= 1e-12


def test_piece_count_equals_brute_force_slope_changes(S):
    """A small random ReLU network (width 3): every slope change found by
    sampling on a fine grid lies at a compiled breakpoint, and there are no
    more of them than compiled breakpoints."""
    d_in, m, width = 4, 2, 3
    rng = np.random.default_rng(5)
    p = rng.normal(0, 1, size=W.glorot_params(d_in, m, width=width).size).astype(np.float32)
    H = S.Mlp.create(d_in, m, W.GBM, p, [1.0] * 4, [0.0] * 4, W.GBM_DOMAIN_LO, W.GBM_DOMAIN_HI,
                     width=width)
    pr = S.Problem(W.GBM, (0.3, 0.1), 1.0, 1.0, 4, m, 10)
    pw = S.pwl_compile(H, pr)
    # plain numpy forward pass of the same parameters
    Wl, bl, off, n_in = [], [], 0, d_in
    for l in range(5):
        n_out = m if l == 4 else width
        Wl.append(p[off:off + n_out * n_in].astype(np.float64).reshape(n_out, n_in)); off += n_out * n_in
        bl.append(p[off:off + n_out].astype(np.float64)); off += n_out
        n_in = n_out
    Y = np.linspace(-20, 20, 400001)
    h = features(W.GBM, Y, 0.25, (0.3, 0.1))
    for l in range(5):
        h = h @ Wl[l].T + bl[l]
        if l < 4:
            h = np.maximum(h, 0)
    assert np.max(np.abs(evaluate(pw, Y) - h)) <= 1e-9 * max(1.0, np.abs(h).max())
    slope = np.diff(h, axis=0) / np.diff(Y)[:, None]
    changes = np.any(np.abs(np.diff(slope, axis=0)) > 1e-6 * (1 + np.abs(slope[1:])), axis=1)
    # each true breakpoint inside (-20, 20) shows up as one or two adjacent flagged cells
    cells = np.flatnonzero(changes)
    groups = np.split(cells, np.flatnonzero(np.diff(cells) > 1) + 1) if cells.size else []
    inside = pw["breaks"][(pw["breaks"] > -20 + 1e-3) & (pw["breaks"] < 20 - 1e-3)]
    # a breakpoint may not change any output's slope (a unit feeding only
    # switched-off units), so compiled breakpoints can outnumber visible ones
    assert len(groups) <= len(inside)
    for g in groups:
        y_c = Y[g[0] + 1]
        assert np.min(np.abs(inside - y_c)) <= 3 * (Y[1] - Y[0])


def test_limits_and_rejections(S):
    from paper_2302_05170_amd import _lib as L
    c = W.CONFIGS["gbm_mlp_2p24x32"]
    H = S.Mlp.load(GBM_W)
    pr = S.Problem(c["model"], c["theta"], c["Y0"], c["T"], c["M"], c["m"], 100)
    with pytest.raises(S.Sl7Error) as e:
        S.pwl_compile(H, pr, max_pieces=10)
    assert e.value.code == L.SL7_EUNSUPPORTED
    for bad in (0, (1 << 16) + 1):
        with pytest.raises(S.Sl7Error) as e:
            S.pwl_compile(H, pr, max_pieces=bad)
        assert e.value.code == L.SL7_EINVAL
    ou = S.Problem(W.OU, (0.5, 0.3, 1.0), 0.2, 2.0, 8, 5, 100)
    with pytest.raises(S.Sl7Error) as e:
        S.pwl_compile(S.Mlp.load(OU_W), ou)
    assert e.value.code == L.SL7_EUNSUPPORTED
    # the PWL modes need a ReLU network: rejected before any device work
    st = L.Stats()
    rc = L.lib().sl7_simulate(ctypes.byref(ou.c()), S.Mlp.load(OU_W).handle, L.PWL32, 1, None,
                              ctypes.byref(st), None, None)
    assert rc == L.SL7_EUNSUPPORTED
    rc = L.lib().sl7_simulate(ctypes.byref(pr.c()), None, L.PWL64, 1, None, ctypes.byref(st),
                              None, None)
    assert rc == L.SL7_EUNSUPPORTED
