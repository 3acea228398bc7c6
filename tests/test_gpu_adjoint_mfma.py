"""The reverse sweeps with the network on MFMA (sl7_adjoint with a network,
prec "f32" and "bf16x3") against the oracle's forward-mode tangents.

Per path, in the scale of the FP64 tests, err = |df_gpu - df| / (1 +
max |df|) per parameter must be <= TOL: 1e-4 in FP32, which rounds each of
the M steps' Jacobian products (four 64-term layers) at ~1e-7 relative, so
the sensitivities carry ~1e-6; 2e-3 in BF16X3, the per-path bound of the
16-bit modes, whose split products keep ~2^-16 of each term.  A dropped
term, a wrong sign or a transposed weight block moves them by 1e-2 or more.
A path may exceed the bound only at a kink the precision can resolve
differently from FP64: a ReLU pre-activation within KINK of zero somewhere on
its FP64 trajectory, Y_T within KINK of the strike (payoff 1), or a CIR step
within KINK of the clamp (KINK 1e-5 in FP32, 1e-4 in BF16X3); at most 1 % of
the paths are so exempt.  The forward half of each sweep takes the
arithmetic of the simulation kernel of its precision, so f per path equals
the payoff of that kernel's Y_T bit for bit, and the checkpoint interval
changes nothing.
"""
import os

import numpy as np
import pytest
import torch

import oracle
import workloads as W
from nets import network_with_m_outputs

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GBM_WEIGHTS = os.path.join(ROOT, "tests", "golden", "gbm_mlp_4x64.sl7w")
OU_WEIGHTS = os.path.join(ROOT, "tests", "golden", "ou_mlp_5x50_softplus.sl7w")
CIR_WEIGHTS = os.path.join(ROOT, "tests", "golden", "cir_mlp_5x64.sl7w")
TOL = {"f32": 1e-4, "bf16x3": 2e-3}
KINK = {"f32": 1e-5, "bf16x3": 1e-4}
MAX_EXEMPT = 0.01
PRECS = ["f32", "bf16x3"]


@pytest.fixture(scope="module")
def S():
    import paper_2302_05170_amd as S
    assert torch.cuda.is_available()
    return S


def opr_of(pr):
    return oracle.Problem(pr.model, pr.theta, pr.Y0, pr.T, pr.M, pr.m, pr.instance)


def kink_distance(pr, Ho, seed, paths):
    """Per path, the distance of its FP64 trajectory to the nearest kink the
    reverse sweep sees: the smallest |pre-activation| of a ReLU hidden unit
    over all steps, the smallest pre-clamp value of a CIR step and, for the
    call, |Y_T - K|.  The trajectory is rebuilt from the oracle's network
    forward, nodes, barycentric weights and normals; its Y_T is returned to
    be checked against the oracle's own pass."""
    x, _ = oracle.gh_nodes(pr.m)
    lam = oracle.bary_weights(x)
    X = oracle.step_normals(seed, oracle.make_tag(0, pr.instance), paths, pr.M)
    dt = pr.T / pr.M
    Y = np.full(len(paths), float(pr.Y0))
    dist = np.full(len(paths), np.inf)
    for i in range(pr.M):
        feats = np.column_stack([Y, np.full_like(Y, dt)] + [np.full_like(Y, t) for t in pr.theta])
        y, (_, zs) = oracle.mlp_forward_batch(Ho, feats)
        if Ho.act == oracle.ACT_RELU:
            for z in zs[:-1]:
                dist = np.minimum(dist, np.abs(z).min(axis=1))
        t = lam[None, :] / (X[:, i, None] - x[None, :])
        Y = (t * y).sum(1) / t.sum(1)
        if pr.model == W.CIR:
            dist = np.minimum(dist, np.abs(Y))
            Y = np.maximum(Y, 0.0)
    return Y, dist


def check_case(S, pr, H, Ho, seed, payoff, ckpt, prec):
    g, pp = S.adjoint(pr, H, prec=prec, seed=seed, payoff=payoff, ckpt_every=ckpt, per_path=True)
    pp = pp.cpu().numpy()
    paths = np.arange(pr.N)
    YT, dY = oracle.simulate_tangent(opr_of(pr), Ho, seed, paths)
    df = dY if payoff == 0 else dY * (YT > pr.K)[:, None]
    # f per path: the payoff of the simulation kernel's Y_T
    _, yt = S.simulate(pr, H, prec=prec, seed=seed, want_yt=True)
    y32 = yt.cpu().numpy().astype(np.float64)
    f32 = y32 if payoff == 0 else np.maximum(y32 - np.float64(np.float32(pr.K)), 0.0)
    assert np.array_equal(pp[:, 0], f32)
    # sensitivities
    scale = 1 + np.max(np.abs(df), axis=0)
    err = np.max(np.abs(pp[:, 1:] - df) / scale, axis=1)
    Yk, dist = kink_distance(pr, Ho, seed, paths)
    assert np.max(np.abs(Yk - YT) / (1 + np.abs(YT))) <= 1e-12
    if payoff == 1:
        dist = np.minimum(dist, np.abs(YT - pr.K))
    bad = err > TOL[prec]
    exempt = bad & (dist < KINK[prec])
    print(f"{prec} N={pr.N} M={pr.M} m={pr.m} payoff={payoff}: max err {err.max():.2e}, "
          f"median {np.median(err):.2e}, over {TOL[prec]:g}: {bad.sum()} (at kinks: "
          f"{exempt.sum()}), paths near a kink {np.sum(dist < KINK[prec])}", flush=True)
    assert np.all(~bad | exempt), np.flatnonzero(bad & ~exempt)[:10]
    assert exempt.sum() <= MAX_EXEMPT * pr.N
    for q in range(df.shape[1]):
        assert abs(g["grad"][q] - df[:, q].mean()) <= TOL[prec] * scale[q]
    return g, pp


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("payoff", [0, 1])
def test_gbm_network(S, payoff, prec):
    H, Ho = S.Mlp.load(GBM_WEIGHTS), oracle.load_mlp(GBM_WEIGHTS)
    pr = S.Problem(W.GBM, (0.3, 0.1), 1.0, 1.0, 16, 5, 2 ** 14, K=1.0)
    check_case(S, pr, H, Ho, 42, payoff, 4, prec)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("payoff", [0, 1])
def test_cir_network_with_clamp(S, payoff, prec):
    """Five inputs, seven outputs, three parameters and the clamp at zero
    (a clamped step passes no gradient)."""
    Hc, Hco = S.Mlp.load(CIR_WEIGHTS), oracle.load_mlp(CIR_WEIGHTS)
    d = W.cir_instances(4)[2]
    pr = S.Problem(d["model"], d["theta"], d["Y0"], d["T"], d["M"], d["m"], 3000,
                   K=d["theta"][1])
    check_case(S, pr, Hc, Hco, 9, payoff, 3, prec)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("payoff", [0, 1])
def test_ou_softplus_network(S, payoff, prec):
    """The paper's network (4 x 50 Softplus, padded to 64): the reverse step
    recomputes the pre-activations from Y_i for the logistic derivative."""
    H, Ho = S.Mlp.load(OU_WEIGHTS), oracle.load_mlp(OU_WEIGHTS)
    P = W.OU_PAPER
    pr = S.Problem(P["model"], P["theta"], P["Y0"], P["T"], P["M"], P["m"], 5000, K=P["K"])
    check_case(S, pr, H, Ho, P["seed"], payoff, 3, prec)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("m2", [2, 3, 8])
def test_other_node_counts(S, m2, prec, tmp_path):
    H2, Ho2 = network_with_m_outputs(S, m2, str(tmp_path / f"gbm_m{m2}.sl7w"))
    pr = S.Problem(W.GBM, (0.3, 0.1), 1.0, 1.0, 9, m2, 1500, K=1.0)
    check_case(S, pr, H2, Ho2, 23, 1, 4, prec)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("N", [1, 15, 17, 63, 65, 1000])
def test_ragged_path_counts(S, N, prec):
    H, Ho = S.Mlp.load(GBM_WEIGHTS), oracle.load_mlp(GBM_WEIGHTS)
    pr = S.Problem(W.GBM, (0.3, 0.1), 1.0, 1.0, 5, 5, N, K=1.0)
    check_case(S, pr, H, Ho, 3, 1, 2, prec)


@pytest.mark.parametrize("prec", PRECS)
def test_checkpoint_interval_changes_nothing(S, prec):
    """Recomputed segments repeat the forward arithmetic exactly: every
    checkpoint interval gives the same per-path results, bit for bit."""
    H = S.Mlp.load(GBM_WEIGHTS)
    pr = S.Problem(W.GBM, (0.3, 0.1), 1.0, 1.0, 16, 5, 3000, K=1.0)
    g0, p0 = S.adjoint(pr, H, prec=prec, seed=3, payoff=1, ckpt_every=4, per_path=True)
    for k in (1, 3, 7, 16, 32):
        g, p = S.adjoint(pr, H, prec=prec, seed=3, payoff=1, ckpt_every=k, per_path=True)
        assert torch.equal(p, p0) and g == g0, k


@pytest.mark.parametrize("prec", PRECS)
def test_path_indices_beyond_32_bits(S, prec):
    H, Ho = S.Mlp.load(GBM_WEIGHTS), oracle.load_mlp(GBM_WEIGHTS)
    off, N = 2 ** 32 - 500, 1000
    pr = S.Problem(W.GBM, (0.3, 0.1), 1.0, 1.0, 6, 5, N, K=1.0, path_offset=off)
    g, pp = S.adjoint(pr, H, prec=prec, seed=19, payoff=0, ckpt_every=4, per_path=True)
    YT, dY = oracle.simulate_tangent(opr_of(pr), Ho, 19, off + np.arange(N, dtype=np.int64))
    err = np.max(np.abs(pp.cpu().numpy()[:, 1:] - dY) / (1 + np.max(np.abs(dY), axis=0)), axis=1)
    assert np.quantile(err, 0.99) <= TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
def test_full_size_sampled_paths(S, prec):
    """The adjoint workload at full size (N = 2^22, M = 16, checkpoint every
    4; the launch the benchmark times): sampled paths against the oracle's
    tangents under the same rule."""
    c = W.CONFIGS["gbm_adjoint_2p22x16"]
    H, Ho = S.Mlp.load(GBM_WEIGHTS), oracle.load_mlp(GBM_WEIGHTS)
    pr = S.Problem(c["model"], c["theta"], c["Y0"], c["T"], c["M"], c["m"], c["N"], K=c["K"])
    g, pp = S.adjoint(pr, H, prec=prec, seed=c["seed"], payoff=1, ckpt_every=c["ckpt"],
                      per_path=True)
    idx = np.unique(np.concatenate([np.arange(512), np.arange(pr.N - 512, pr.N),
                                    np.linspace(0, pr.N - 1, 2048).astype(np.int64)]))
    pp = pp[torch.from_numpy(idx).cuda()].cpu().numpy()
    YT, dY = oracle.simulate_tangent(opr_of(pr), Ho, c["seed"], idx)
    df = dY * (YT > pr.K)[:, None]
    err = np.max(np.abs(pp[:, 1:] - df) / (1 + np.max(np.abs(df), axis=0)), axis=1)
    _, dist = kink_distance(pr, Ho, c["seed"], idx)
    dist = np.minimum(dist, np.abs(YT - pr.K))
    bad = err > TOL[prec]
    print(f"{prec} full size, {len(idx)} sampled paths: max err {err.max():.2e}, over "
          f"{TOL[prec]:g}: {bad.sum()}, all at kinks: {np.all(dist[bad] < KINK[prec])}")
    assert np.all(dist[bad] < KINK[prec]) and bad.sum() <= MAX_EXEMPT * len(idx)


def test_split_mode_needs_a_network(S):
    from paper_2302_05170_amd import _lib as L
    pr = S.Problem(W.GBM, (0.3, 0.1), 1.0, 1.0, 4, 5, 100, K=1.0)
    with pytest.raises(L.Sl7Error, match="needs a network"):
        S.adjoint(pr, None, prec="bf16x3", seed=1)


@pytest.mark.parametrize("prec", PRECS)
def test_reverse_sweep_only_for_paths_with_nonzero_payoff_derivative(S, prec):
    """The reverse sweep visits only paths with f'(Y_T) != 0.  A strike above
    every Y_T leaves none: value and sensitivities exactly zero, per path
    too.  A strike below every Y_T makes every path active: the call's
    sensitivities then equal those of Y_T itself, path by path and bit for
    bit, and its value is E[Y_T] - K."""
    H = S.Mlp.load(GBM_WEIGHTS)
    base = dict(model=W.GBM, theta=(0.3, 0.1), Y0=1.0, T=1.0, M=16, m=5, N=3000)
    pr0 = S.Problem(base["model"], base["theta"], base["Y0"], base["T"], base["M"], base["m"],
                    base["N"], K=1.0)
    g0, p0 = S.adjoint(pr0, H, prec=prec, seed=5, payoff=0, ckpt_every=4, per_path=True)
    p0 = p0.cpu().numpy()
    lo, hi = p0[:, 0].min(), p0[:, 0].max()
    prh = S.Problem(base["model"], base["theta"], base["Y0"], base["T"], base["M"], base["m"],
                    base["N"], K=2 * hi)
    gh, ph = S.adjoint(prh, H, prec=prec, seed=5, payoff=1, ckpt_every=4, per_path=True)
    assert gh["value"] == 0.0 and all(v == 0.0 for v in gh["grad"])
    assert not np.any(ph.cpu().numpy())
    prl = S.Problem(base["model"], base["theta"], base["Y0"], base["T"], base["M"], base["m"],
                    base["N"], K=0.5 * lo)
    gl, pl = S.adjoint(prl, H, prec=prec, seed=5, payoff=1, ckpt_every=4, per_path=True)
    pl = pl.cpu().numpy()
    assert np.array_equal(pl[:, 1:], p0[:, 1:])
    assert np.allclose(pl[:, 0], p0[:, 0] - np.float64(np.float32(0.5 * lo)), rtol=0, atol=1e-15)
