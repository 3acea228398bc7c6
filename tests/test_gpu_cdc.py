"""GPU parity of the 7L-CDC variant (sl7_simulate_cdc) against the oracle's
CDC (oracle.simulate_cdc), through the C ABI: per path 1e-12 in FP64 and
1e-5 in FP32 (relative, floor as for 7L: |Y| for GBM, 0.5 for OU, ybar for
CIR), path means 1e-12 / 1e-6.  Each step interpolates twice, in Y over the
marginal points and in X over the nodes; where either extrapolates, FP32
rounding is multiplied by that interpolant's Lebesgue function, and the FP32
bound of such a path is 1e-5 times the larger factor (Lambda over the
marginal points at the path's Y_i, relative to its largest value between
them; Lambda_m(X) relative to Lambda_m(4)), from the path's FP64 trajectory.
Maps: the analytic GBM map, the stored GBM network, the paper's OU network
(4 x 50 Softplus) at the Table 6.1 path counts and the CIR network; ragged
path counts, one and two steps and m = 2..8.  For maps affine in Y the
variant equals 7L path by path."""
import os

import numpy as np
import pytest
import torch

import oracle
import workloads as W
from lebesgue import X_REF, inside_max, lebesgue, lebesgue_nodes
from nets import network_with_m_outputs

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GBM_WEIGHTS = os.path.join(ROOT, "tests", "golden", "gbm_mlp_4x64.sl7w")
OU_WEIGHTS = os.path.join(ROOT, "tests", "golden", "ou_mlp_5x50_softplus.sl7w")
CIR_WEIGHTS = os.path.join(ROOT, "tests", "golden", "cir_mlp_5x64.sl7w")
TOL = {"f64": 1e-12, "f32": 1e-5}
MEAN_TOL = {"f64": 1e-12, "f32": 1e-6}


@pytest.fixture(scope="module")
def S():
    import paper_2302_05170_amd as S
    assert torch.cuda.is_available()
    return S


def run(S, pr, H, prec, seed):
    st, yt = S.simulate_cdc(pr, H, prec=prec, seed=seed, want_yt=True)
    torch.cuda.synchronize()
    return st, yt.double().cpu().numpy()


def oracle_cdc(pr, Ho, seed, N):
    opr = oracle.Problem(pr.model, pr.theta, pr.Y0, pr.T, pr.M, pr.m, pr.instance)
    return oracle.simulate_cdc(opr, Ho, seed, np.arange(N))


def amplification(pr, Ho, seed, N):
    """Per path, the largest Lebesgue factor of its two interpolations over
    the steps, from the FP64 trajectory rebuilt from the oracle's tables."""
    opr = oracle.Problem(pr.model, pr.theta, pr.Y0, pr.T, pr.M, pr.m, pr.instance)
    s, lams, ykj, _ = oracle.cdc_tables(opr, Ho)
    X = oracle.step_normals(seed, oracle.make_tag(0, pr.instance), np.arange(N), pr.M)
    x, _ = oracle.gh_nodes(pr.m)
    lam = oracle.bary_weights(x)
    fx = np.maximum(1.0, lebesgue(pr.m, np.abs(X)).max(axis=1) / lebesgue(pr.m, X_REF))
    fy = np.ones(N)
    Y = np.full(N, float(pr.Y0))
    for i in range(pr.M):
        if i == 0:
            y = np.broadcast_to(ykj[0, 0], (N, pr.m))
        else:
            fy = np.maximum(fy, lebesgue_nodes(s[i], Y) / inside_max(s[i]))
            with np.errstate(divide="ignore", invalid="ignore"):
                t = lams[i][None, :] / (Y[:, None] - s[i][None, :])
                y = (t[:, :, None] * ykj[i][None, :, :]).sum(1) / t.sum(1)[:, None]
        with np.errstate(divide="ignore", invalid="ignore"):
            tt = lam[None, :] / (X[:, i][:, None] - x[None, :])
            Y = (tt * y).sum(1) / tt.sum(1)
        if pr.model == W.CIR:
            Y = np.maximum(Y, 0.0)
    return np.maximum(fx, np.nan_to_num(fy, nan=1.0, posinf=1e6))


def check(S, pr, H, Ho, seed, floor, label, precs=("f64", "f32")):
    ref, ncl, nood = oracle_cdc(pr, Ho, seed, pr.N)
    amp = amplification(pr, Ho, seed, pr.N) if "f32" in precs else None
    for prec in precs:
        st, y = run(S, pr, H, prec, seed)
        e = np.abs(y - ref) / np.maximum(np.abs(ref), floor)
        bound = TOL[prec] * (amp if prec == "f32" else 1.0)
        inner = e[amp <= 1.0] if prec == "f32" else e
        print(f"CDC {label} {prec} N={pr.N} M={pr.M} m={pr.m}: max err {e.max():.3e}"
              + (f"; {inner.max() if inner.size else 0:.3e} on the {inner.size} paths with no "
                 f"extrapolation; max err/bound {(e / bound).max():.2f}" if prec == "f32" else ""),
              flush=True)
        assert st["n"] == pr.N
        assert np.all(e <= bound), (label, prec, e.max(), (e / bound).max())
        f = oracle.estimate(ref)
        assert abs(st["mean"][0] - f["mean"]) <= MEAN_TOL[prec] * max(abs(f["mean"]), floor), \
            (label, prec)
        if prec == "f64":
            assert st["n_clamped"] == ncl and st["n_out_of_domain"] == nood, label


def test_gbm_analytic_map(S):
    c = W.CONFIGS["gbm_analytic_1e5x4"]
    pr = S.Problem(c["model"], c["theta"], c["Y0"], c["T"], c["M"], c["m"], c["N"], K=c["K"])
    check(S, pr, None, None, c["seed"], 1e-12, "gbm analytic")


def test_equals_7l_for_the_analytic_gbm_map(S):
    """The analytic GBM map is affine in Y, so the global interpolation
    reproduces it exactly: CDC and 7L agree path by path (FP64)."""
    c = W.CONFIGS["gbm_analytic_1e5x4"]
    pr = S.Problem(c["model"], c["theta"], c["Y0"], c["T"], 9, c["m"], 20_000, K=c["K"])
    _, y7 = S.simulate(pr, None, prec="f64", seed=5, want_yt=True)
    _, yc = run(S, pr, None, "f64", 5)
    y7 = y7.cpu().numpy()
    assert np.max(np.abs(yc - y7) / np.abs(y7)) <= 1e-13


def test_gbm_network_16_steps(S):
    c = W.CONFIGS["gbm_mlp_2p22x16"]
    H, Ho = S.Mlp.load(GBM_WEIGHTS), oracle.load_mlp(GBM_WEIGHTS)
    pr = S.Problem(c["model"], c["theta"], c["Y0"], c["T"], c["M"], c["m"], 2 ** 17, K=c["K"])
    check(S, pr, H, Ho, c["seed"], 1e-12, "gbm network")


def test_ou_softplus_network_table61_counts(S):
    P = W.OU_PAPER
    H, Ho = S.Mlp.load(OU_WEIGHTS), oracle.load_mlp(OU_WEIGHTS)
    for N in P["path_counts"]:
        pr = S.Problem(P["model"], P["theta"], P["Y0"], P["T"], P["M"], P["m"], N, K=P["K"])
        check(S, pr, H, Ho, P["seed"], 0.5, "ou softplus")


def test_cir_network_instances(S):
    """CIR parameter sets of the batched workload over a horizon T = 0.8
    (M = 4), where the marginal points need the network at horizons t_i up
    to T - dt, inside its training range of dt (0.1 .. 1): the first four
    that satisfy the Feller condition (2 kappa ybar >= gamma^2) and whose
    marginal points all lie above ybar / 10.  Where the lower marginal
    points bunch near zero the global interpolation amplifies rounding
    without bound on both sides (reading 19)."""
    H, Ho = S.Mlp.load(CIR_WEIGHTS), oracle.load_mlp(CIR_WEIGHTS)
    picked = 0
    for d in W.cir_instances(256):
        kap, ybar, gam = d["theta"]
        if 2 * kap * ybar < gam ** 2:
            continue
        opr = oracle.Problem(d["model"], d["theta"], d["Y0"], 0.8, 4, d["m"], d["instance"])
        if oracle.cdc_tables(opr, Ho)[0][1:].min() < 0.1 * ybar:
            continue
        pr = S.Problem(d["model"], d["theta"], d["Y0"], 0.8, 4, d["m"], min(d["N"], 20_000),
                       K=ybar, instance=d["instance"])
        check(S, pr, H, Ho, 11, ybar, f"cir {d['instance']}")
        picked += 1
        if picked == 4:
            break
    assert picked == 4


@pytest.mark.parametrize("N,M", [(1, 1), (63, 2), (65, 1), (1000, 3), (4099, 7)])
def test_ragged_counts_and_few_steps(S, N, M):
    c = W.CONFIGS["gbm_mlp_2p22x16"]
    H, Ho = S.Mlp.load(GBM_WEIGHTS), oracle.load_mlp(GBM_WEIGHTS)
    pr = S.Problem(c["model"], c["theta"], c["Y0"], c["T"], M, c["m"], N, K=c["K"])
    check(S, pr, H, Ho, 3, 1e-12, "ragged")


@pytest.mark.parametrize("m2", [2, 3, 7, 8])
def test_node_counts(S, m2, tmp_path):
    H2, Ho2 = network_with_m_outputs(S, m2, str(tmp_path / f"gbm_m{m2}.sl7w"))
    c = W.CONFIGS["gbm_mlp_2p22x16"]
    pr = S.Problem(c["model"], c["theta"], c["Y0"], c["T"], 6, m2, 3000, K=c["K"])
    check(S, pr, H2, Ho2, 17, 1e-12, f"m={m2}")
    pa = S.Problem(W.GBM, (0.25, 0.05), 1.3, 0.7, 5, m2, 3000, K=1.2)
    check(S, pa, None, None, 17, 1e-12, f"analytic m={m2}")


def test_16_bit_modes_refused(S):
    from paper_2302_05170_amd import _lib as L
    H = S.Mlp.load(GBM_WEIGHTS)
    pr = S.Problem(W.GBM, (0.3, 0.1), 1.0, 1.0, 4, 5, 100)
    with pytest.raises(L.Sl7Error, match="F64 or F32"):
        S.simulate_cdc(pr, H, prec="bf16x3", seed=1)


def test_coinciding_marginal_points_are_reported(S, tmp_path):
    """A network whose outputs all equal 1 maps Y0 to coinciding marginal
    points: the table kernel counts them and the call returns SL7_ENUMERIC
    (the per-lane kernel meanwhile runs on infinite weights without fault)."""
    from paper_2302_05170_amd import _lib as L
    Ho = oracle.load_mlp(GBM_WEIGHTS)
    Wf = [np.array(w) for w in Ho.W]
    bf = [np.array(v) for v in Ho.b]
    Wf[-1][:] = 0.0
    bf[-1][:] = 1.0
    flat = oracle.Mlp(Ho.d_in, Ho.width, Ho.depth, Ho.m, Ho.act, Ho.model, Ho.in_scale,
                      Ho.in_shift, Ho.dom_lo, Ho.dom_hi, Wf, bf, dict(Ho.meta))
    path = str(tmp_path / "flat_head.sl7w")
    oracle.save_mlp(flat, path)
    H2 = S.Mlp.load(path)
    pr = S.Problem(W.GBM, (0.3, 0.1), 1.0, 1.0, 4, 5, 1000, K=1.0)
    for prec in ("f32", "f64"):
        with pytest.raises(L.Sl7Error, match="not distinct"):
            S.simulate_cdc(pr, H2, prec=prec, seed=1)
    # the library stays usable
    H = S.Mlp.load(GBM_WEIGHTS)
    st, _ = S.simulate_cdc(pr, H, prec="f32", seed=1)
    assert np.isfinite(st["mean"][0])
