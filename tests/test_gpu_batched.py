"""Batched uneven CIR instances (one persistent launch, longest-M-first work
queue, hipGraph replays) and the launch-plan autotuner.

Each instance's statistics from the batched launch must equal, bit for bit,
those of a single-instance launch of the same instance (same kernel, same
fixed-order 64-path block sums); single-instance runs are in turn checked
path by path against the oracle.  CIR per-path error is measured against
max(|Y|, ybar), the process's mean-reversion level: CIR paths spend time at
and near the zero clamp, where a relative error says nothing about the law
and FP32 arithmetic on network activations of order one leaves absolute
errors of ~1e-7.
"""
import os
import tempfile

import numpy as np
import pytest
import torch

import oracle
import workloads as W
from lebesgue import F32_TOL, f32_bound

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CIR_WEIGHTS = os.path.join(ROOT, "tests", "golden", "cir_mlp_5x64.sl7w")


@pytest.fixture(scope="module")
def S():
    import paper_2302_05170_amd as S
    assert torch.cuda.is_available()
    return S


@pytest.fixture(scope="module")
def H(S):
    return S.Mlp.load(CIR_WEIGHTS)


def problems(S, n=256, scale=1.0):
    out = []
    for d in W.cir_instances(n):
        out.append(S.Problem(d["model"], d["theta"], d["Y0"], d["T"], d["M"], d["m"],
                             max(1, int(d["N"] * scale)), K=d["theta"][1], instance=d["instance"]))
    return out


@pytest.mark.parametrize("prec", ["bf16x3", "f32", "bf16", "f16x3", "f16", "pwl32", "pwl64"])
def test_batched_equals_single_instance_runs(S, H, prec):
    prs = problems(S, 40, scale=0.25)
    got = S.simulate_batched(prs, H, prec=prec, seed=11, use_graph=False)
    for k, pr in enumerate(prs):
        st, _ = S.simulate(pr, H, prec=prec, seed=11)
        assert got[k] == st, k


def test_batched_graph_replays_match_eager(S, H):
    prs = problems(S, 64, scale=0.2)
    ref = S.simulate_batched(prs, H, prec="bf16x3", seed=11, use_graph=False)
    for r in range(3):
        got = S.simulate_batched(prs, H, prec="bf16x3", seed=11, use_graph=True)
        assert got == ref, r
        # eager work on the same device between replays
        S.simulate(prs[r], H, prec="f32", seed=5)
        torch.cuda.synchronize()


@pytest.mark.parametrize("prec", ["bf16x3", "pwl32"])
def test_graph_replays_follow_the_networks_parameters(S, prec):
    """A captured batch depends on the network's weights (the first-layer
    constants go into its instance table, the piecewise-linear tables into
    its workspace): after set_params, and for a new handle that replaces a
    freed one, replays must give what an eager launch gives."""
    prs = problems(S, 32, scale=0.1)
    H1 = S.Mlp.load(CIR_WEIGHTS)
    p0 = H1.params()
    first = S.simulate_batched(prs, H1, prec=prec, seed=3, use_graph=True)
    H1.set_params(p0 * np.float32(1.02))
    got = S.simulate_batched(prs, H1, prec=prec, seed=3, use_graph=True)
    ref = S.simulate_batched(prs, H1, prec=prec, seed=3, use_graph=False)
    assert got == ref
    assert got != first
    del H1
    for scale in (0.98, 1.0):
        H2 = S.Mlp.load(CIR_WEIGHTS)
        H2.set_params(p0 * np.float32(scale))
        got = S.simulate_batched(prs, H2, prec=prec, seed=3, use_graph=True)
        ref = S.simulate_batched(prs, H2, prec=prec, seed=3, use_graph=False)
        assert got == ref, scale
        del H2


def test_batched_result_independent_of_instance_order(S, H):
    prs = problems(S, 32, scale=0.2)
    a = S.simulate_batched(prs, H, prec="bf16x3", seed=11, use_graph=False)
    perm = np.random.default_rng(0).permutation(len(prs))
    b = S.simulate_batched([prs[i] for i in perm], H, prec="bf16x3", seed=11, use_graph=False)
    for j, i in enumerate(perm):
        assert b[j] == a[i]


def spanning_instances(prs, n_pick=64):
    """Every fourth instance in order of cost N*M, from the costliest down,
    plus the instances with the fewest and most paths and steps."""
    order = sorted(range(len(prs)), key=lambda k: prs[k].N * prs[k].M, reverse=True)
    pick = set(order[::len(prs) // n_pick])
    for key in (lambda k: prs[k].N, lambda k: prs[k].M):
        pick.add(min(range(len(prs)), key=key))
        pick.add(max(range(len(prs)), key=key))
    return sorted(pick)


@pytest.fixture(scope="module")
def cir_oracle_paths(S):
    """Oracle Y_T of every path of the spanning instances of the 256-instance
    CIR workload, at their full path counts, and each path's largest |X|."""
    Ho = oracle.load_mlp(CIR_WEIGHTS)
    prs = problems(S, 256)
    ref = {}
    for k in spanning_instances(prs):
        pr = prs[k]
        opr = oracle.Problem(pr.model, pr.theta, pr.Y0, pr.T, pr.M, pr.m, pr.instance)
        y, ncl, nood = oracle.simulate(opr, Ho, 11, np.arange(pr.N))
        X = oracle.step_normals(11, oracle.make_tag(0, pr.instance), np.arange(pr.N), pr.M)
        ref[k] = (y, ncl, nood, np.abs(X).max(axis=1))
    return prs, ref


@pytest.fixture(scope="module")
def cir_oracle_means(cir_oracle_paths):
    """The oracle's two payoff means (Y_T and max(Y_T - ybar, 0)) of every
    one of the 256 instances at its full path count (the spanning instances'
    from their stored paths)."""
    prs, ref = cir_oracle_paths
    Ho = oracle.load_mlp(CIR_WEIGHTS)
    means = {}
    for k, pr in enumerate(prs):
        if k in ref:
            y = ref[k][0]
        else:
            opr = oracle.Problem(pr.model, pr.theta, pr.Y0, pr.T, pr.M, pr.m, pr.instance)
            y = oracle.simulate(opr, Ho, 11, np.arange(pr.N))[0]
        means[k] = [oracle.estimate(f)["mean"] for f in oracle.payoffs(y, pr.K)]
    return prs, means


def test_batched_launch_means_match_oracle(S, H, cir_oracle_means):
    """The whole 256-instance batch in one persistent FP32 launch replayed
    from its graph: every instance's two payoff means (Y_T and
    max(Y_T - ybar, 0)) against the oracle's means over the same paths, at
    1e-6 relative to max(|mean|, ybar).  The call's mean can be a few
    thousandths, where 1e-6 of it is below the FP32 spacing of Y near ybar;
    ybar is the same floor as for the per-path errors.  The FP32 kernel
    carries the first-layer constant as two floats: rounded once to FP32 it
    would shift every path of an instance alike, by up to 8e-7 of ybar in
    the mean on this workload.  The plain relative error is printed."""
    prs, means = cir_oracle_means
    assert len(means) == 256
    got = S.simulate_batched(prs, H, prec="f32", seed=11, use_graph=True)
    worst = [0.0, 0.0]
    plain = [(0.0, -1, 0.0)] * 2
    miss = []
    for k, mk in means.items():
        assert got[k]["n"] == prs[k].N
        for j in range(2):
            diff = abs(got[k]["mean"][j] - mk[j])
            d = diff / max(abs(mk[j]), prs[k].theta[1])
            worst[j] = max(worst[j], d)
            rel = diff / max(abs(mk[j]), 1e-300)
            if rel > plain[j][0]:
                plain[j] = (rel, k, mk[j])
            if d > 1e-6:
                miss.append((k, j, d))
    print(f"batched f32 over {len(means)} instances at full N: max error of the means "
          f"{worst[0]:.2e} (Y_T), {worst[1]:.2e} (call) against max(|mean|, ybar); plain "
          f"relative {plain[0][0]:.2e} (instance {plain[0][1]}, mean {plain[0][2]:.3e}), "
          f"{plain[1][0]:.2e} (instance {plain[1][1]}, mean {plain[1][2]:.3e})")
    assert not miss, miss


# Absolute term per step for CIR.  The CIR network's inputs are scaled to
# [-1, 1] and its hidden activations are of order one, so its outputs
# (collocation values of order ybar, 0.02..0.1) carry the absolute error of
# the arithmetic at that scale whatever their own size -- a few units of
# 2^-23 in FP32, of 2^-16 in the split-BF16 mode (the dropped lo*lo terms) --
# and these add up over the M steps (neighbouring states round alike).
ATOL_STEP_CIR = {"f64": 0.0, "f32": 4 * 2.0 ** -23, "bf16x3": 2 * 2.0 ** -16}


@pytest.mark.parametrize("prec,tol", [("f64", 1e-12), ("f32", 1e-5), ("bf16x3", 2e-3)])
def test_cir_instances_match_oracle(S, H, cir_oracle_paths, prec, tol):
    """Every path of the spanning instances at full size, one single-instance
    launch each: |error| <= tol max(|Y|, ybar) + M atol (ybar the
    mean-reversion level; atol per step above, 0 in FP64), in FP32 scaled by
    the interpolant's Lebesgue function at the path's largest |X| beyond 4
    (tests/lebesgue.py).  The relative errors against the floors ybar and
    1e-3 ybar and the absolute error are printed."""
    prs, ref = cir_oracle_paths
    w_ybar = w_small = w_abs = w_inner = w_ratio = 0.0
    n_outer = n_over = 0
    fails = []
    for k, (y_ref, ncl, nood, xmax) in ref.items():
        pr = prs[k]
        st, yt = S.simulate(pr, H, prec=prec, seed=11, want_yt=True)
        torch.cuda.synchronize()
        y = yt.double().cpu().numpy()
        d = np.abs(y - y_ref)
        floor = np.maximum(np.abs(y_ref), pr.theta[1])
        e = d / floor
        bound = tol * floor + pr.M * ATOL_STEP_CIR[prec]
        if prec == "f32":
            bound = bound * (f32_bound(pr.m, xmax) / F32_TOL)
        n_over += int(np.count_nonzero(e > tol))
        ratio = d / bound
        w_ybar = max(w_ybar, e.max())
        w_small = max(w_small, (d / np.maximum(np.abs(y_ref), 1e-3 * pr.theta[1])).max())
        w_abs = max(w_abs, d.max())
        inner = xmax <= 4.0
        w_inner = max(w_inner, e[inner].max() if inner.any() else 0.0)
        n_outer += int(np.count_nonzero(~inner))
        w_ratio = max(w_ratio, ratio.max())
        if ratio.max() > 1.0:
            fails.append((k, float(e.max()), float(ratio.max())))
        if prec == "f64":
            assert st["n_clamped"] == ncl and st["n_out_of_domain"] == nood
    print(f"CIR {prec} over {len(ref)} instances: max err {w_ybar:.2e} (floor ybar), "
          f"{w_inner:.2e} on paths with all |X| <= 4, {n_outer} paths beyond; "
          f"{w_small:.2e} (floor 1e-3 ybar), max abs {w_abs:.2e}; max err/bound {w_ratio:.2f}; "
          f"{n_over} paths above {tol:g} at floor ybar")
    assert not fails, fails


def test_autotune_returns_valid_plan_and_caches(S, H):
    import ctypes
    from paper_2302_05170_amd import _lib as L
    pr = problems(S, 1)[0]
    pr = S.Problem(pr.model, pr.theta, pr.Y0, pr.T, 16, 7, 2 ** 16, K=pr.K)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "plans.jsonl").encode()
        plan = L.Plan()
        cp = pr.c()
        L.check(L.lib().sl7_autotune(ctypes.byref(cp), H.handle, L.BF16X3, path, ctypes.byref(plan),
                                     None))
        assert plan.waves_per_block in (1, 2, 4, 12) and 1 <= plan.blocks_per_cu <= 8
        text = open(path).read()
        assert '"key": "gfx950/prec4/din5/m7"' in text
        plan2 = L.Plan()
        L.check(L.lib().sl7_autotune(ctypes.byref(cp), H.handle, L.BF16X3, path, ctypes.byref(plan2),
                                     None))
        assert (plan2.waves_per_block, plan2.blocks_per_cu, plan2.grab) == \
            (plan.waves_per_block, plan.blocks_per_cu, plan.grab)
        assert open(path).read() == text  # second call read the cache


def test_autotune_batched_times_the_batch_and_caches(S, H):
    """The batch tuner returns a valid plan under a key naming the batch's
    shapes, reads it back, and the plan's results equal the default plan's."""
    prs = problems(S, 24)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "plans.jsonl")
        plan = S.autotune_batched(prs, H, prec="bf16x3", cache_path=path)
        assert plan["waves_per_block"] in (1, 2, 4, 12) and 1 <= plan["blocks_per_cu"] <= 16
        text = open(path).read()
        assert '"key": "gfx950/prec4/din5/m7/batch' in text
        assert S.autotune_batched(prs, H, prec="bf16x3", cache_path=path) == plan
        assert open(path).read() == text  # second call read the cache
        # another batch gets its own key
        S.autotune_batched(prs[:5], H, prec="bf16x3", cache_path=path)
        assert len(open(path).read().splitlines()) == 2
    tuned = S.simulate_batched(prs, H, prec="bf16x3", seed=11, plan=plan, use_graph=False)
    ref = S.simulate_batched(prs, H, prec="bf16x3", seed=11, use_graph=False)
    assert tuned == ref
