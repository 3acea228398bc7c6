"""GPU parity of the piecewise-linear modes (SL7_PWL32 / SL7_PWL64): the
online stage with the ReLU network evaluated through its exact per-instance
piecewise-linear form in Y, against the FP64 oracle that evaluates the
network layer by layer.

Tolerances as for the other modes of the same lane arithmetic: per-path
relative error 1e-12 (PWL64) and 1e-5 (PWL32); path means 1e-12 / 1e-6.
"""
import os

import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GBM_W = os.path.join(ROOT, "tests", "golden", "gbm_mlp_4x64.sl7w")
CIR_W = os.path.join(ROOT, "tests", "golden", "cir_mlp_5x64.sl7w")
TOL = {"pwl64": 1e-12, "pwl32": 1e-5}


@pytest.fixture(scope="module")
def S():
    import paper_2302_05170_amd as S
    assert torch.cuda.is_available()
    return S


def rel(got, ref, floor=1e-12):
    return np.abs(got - ref) / np.maximum(np.abs(ref), floor)


def gpu_yt(S, pr, H, prec, seed, plan=None):
    st, yt = S.simulate(pr, H, prec=prec, seed=seed, want_yt=True, plan=plan)
    torch.cuda.synchronize()
    return st, yt.double().cpu().numpy()


def orc(pr, Ho, seed, paths):
    opr = oracle.Problem(pr.model, pr.theta, pr.Y0, pr.T, pr.M, pr.m, pr.instance)
    return oracle.simulate(opr, Ho, seed, paths)


@pytest.mark.parametrize("prec", ["pwl64", "pwl32"])
@pytest.mark.parametrize("N", [1, 63, 65, 4099])
def test_ragged_counts_all_paths(S, prec, N):
    H, Ho = S.Mlp.load(GBM_W), oracle.load_mlp(GBM_W)
    c = W.CONFIGS["gbm_mlp_2p22x16"]
    pr = S.Problem(c["model"], c["theta"], c["Y0"], c["T"], 7, c["m"], N, K=c["K"])
    ref, _, nood = orc(pr, Ho, 5, np.arange(N))
    st, y = gpu_yt(S, pr, H, prec, 5)
    assert st["n"] == N
    assert rel(y, ref).max() <= TOL[prec]
    e = oracle.estimate(ref)
    assert abs(st["mean"][0] - e["mean"]) <= (1e-12 if prec == "pwl64" else 1e-6) * abs(e["mean"])
    if prec == "pwl64":
        assert st["n_out_of_domain"] == nood


@pytest.mark.parametrize("prec", ["pwl64", "pwl32"])
def test_gbm_2p22x16_full_size_sampled(S, prec):
    H, Ho = S.Mlp.load(GBM_W), oracle.load_mlp(GBM_W)
    c = W.CONFIGS["gbm_mlp_2p22x16"]
    pr = S.Problem(c["model"], c["theta"], c["Y0"], c["T"], c["M"], c["m"], c["N"], K=c["K"])
    st, y = gpu_yt(S, pr, H, prec, c["seed"])
    sub = W.parity_subset(c["N"])
    ref, _, _ = orc(pr, Ho, c["seed"], sub)
    r = rel(y[sub], ref)
    print(f"GBM 2^22 x 16 {prec}: max rel err {r.max():.3e} over {len(sub)} paths")
    assert r.max() <= TOL[prec]


@pytest.mark.parametrize("prec", ["pwl64", "pwl32"])
def test_gbm_2p24x32_full_size_sampled(S, prec):
    H, Ho = S.Mlp.load(GBM_W), oracle.load_mlp(GBM_W)
    c = W.CONFIGS["gbm_mlp_2p24x32"]
    pr = S.Problem(c["model"], c["theta"], c["Y0"], c["T"], c["M"], c["m"], c["N"], K=c["K"])
    st, y = gpu_yt(S, pr, H, prec, c["seed"])
    sub = W.parity_subset(c["N"])[::4]
    ref, _, _ = orc(pr, Ho, c["seed"], sub)
    r = rel(y[sub], ref)
    print(f"GBM 2^24 x 32 {prec}: max rel err {r.max():.3e} over {len(sub)} paths")
    assert r.max() <= TOL[prec]
    assert st["n"] == c["N"] and np.isfinite(st["mean"][0])


def test_pwl_and_mfma_paths_agree(S):
    """The same paths through the FP32 MFMA network and the FP32 piecewise-
    linear form differ only by FP32 rounding."""
    H = S.Mlp.load(GBM_W)
    c = W.CONFIGS["gbm_mlp_2p22x16"]
    pr = S.Problem(c["model"], c["theta"], c["Y0"], c["T"], c["M"], c["m"], 1 << 18, K=c["K"])
    _, a = gpu_yt(S, pr, H, "f32", 3)
    _, b = gpu_yt(S, pr, H, "pwl32", 3)
    assert rel(a, b).max() <= 2e-5


@pytest.mark.parametrize("prec", ["pwl64", "pwl32"])
def test_results_independent_of_launch_plan(S, prec):
    H = S.Mlp.load(GBM_W)
    c = W.CONFIGS["gbm_mlp_2p22x16"]
    pr = S.Problem(c["model"], c["theta"], c["Y0"], c["T"], 9, c["m"], 50_001, K=c["K"])
    outs = [gpu_yt(S, pr, H, prec, 77, plan=plan)
            for plan in (None, dict(waves_per_block=1, blocks_per_cu=1, grab=1),
                         dict(waves_per_block=4, blocks_per_cu=3, grab=5))]
    for st, y in outs[1:]:
        assert np.array_equal(y, outs[0][1])
        assert st == outs[0][0]


def test_cir_batched_pwl32(S):
    """256 uneven CIR instances in one persistent launch through their
    compiled forms: every instance equals its single-instance run, and
    sampled paths match the oracle (CIR floor: the mean-reversion level)."""
    H, Ho = S.Mlp.load(CIR_W), oracle.load_mlp(CIR_W)
    ds = W.cir_instances(256)
    prs = [S.Problem(d["model"], d["theta"], d["Y0"], d["T"], d["M"], d["m"], d["N"],
                     K=d["theta"][1], instance=d["instance"]) for d in ds]
    batched = S.simulate_batched(prs, H, prec="pwl32", seed=11, use_graph=True)
    again = S.simulate_batched(prs, H, prec="pwl32", seed=11, use_graph=True)
    assert batched == again
    for k in (0, 17, 101, 255):
        st, y = gpu_yt(S, prs[k], H, "pwl32", 11)
        assert st == batched[k]
        sub = np.arange(min(prs[k].N, 2048))
        ref, _, _ = orc(prs[k], Ho, 11, sub)
        assert rel(y[sub], ref, floor=ds[k]["theta"][1]).max() <= TOL["pwl32"]
