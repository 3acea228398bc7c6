"""GPU parity of the fused online stage (Algorithm I, steps 2-8) against the
FP64 oracle, through the C ABI.

Tolerances: per-path Y_T relative error max over the compared paths, 1e-12
in FP64, 1e-5 in FP32, 2e-3 in the BF16 mode that meets it (three-pass split
BF16, "bf16x3"; 5e-4 for the FP16 counterpart); path means 1e-6 relative in
FP32.  rel = |gpu - oracle| / max(|oracle|, 1e-12).  The one-pass BF16/FP16
modes carry a per-step rounding bias (weights rounded once) that grows with
M; they are checked against their measured bound (0.1 / 0.02 at M <= 32)
and their error is printed, not gated.
"""
import os

import numpy as np
import pytest
import torch

import oracle
import workloads as W
from lebesgue import f32_bound
from nets import network_with_m_outputs

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WEIGHTS = os.path.join(ROOT, "tests", "golden", "gbm_mlp_4x64.sl7w")
TOL = {"f64": 1e-12, "f32": 1e-5, "bf16x3": 2e-3, "f16x3": 5e-4, "bf16": 0.1, "f16": 0.02}


@pytest.fixture(scope="module")
def S():
    import paper_2302_05170_amd as S
    assert torch.cuda.is_available()
    return S


@pytest.fixture(scope="module")
def H(S):
    return S.Mlp.load(WEIGHTS)


@pytest.fixture(scope="module")
def Ho():
    return oracle.load_mlp(WEIGHTS)


def rel(got, ref):
    return np.abs(got - ref) / np.maximum(np.abs(ref), 1e-12)


def gpu_yt(S, pr, H, prec, seed, plan=None):
    st, yt = S.simulate(pr, H, prec=prec, seed=seed, want_yt=True, plan=plan)
    torch.cuda.synchronize()
    return st, yt.double().cpu().numpy()


def orc(pr, Ho, seed, paths):
    opr = oracle.Problem(pr.model, pr.theta, pr.Y0, pr.T, pr.M, pr.m, pr.instance)
    y, ncl, nood = oracle.simulate(opr, Ho, seed, paths)
    return y


def test_gbm_analytic_1e5x4_f64_all_paths(S):
    c = W.CONFIGS["gbm_analytic_1e5x4"]
    pr = S.Problem(c["model"], c["theta"], c["Y0"], c["T"], c["M"], c["m"], c["N"], K=c["K"])
    st, y = gpu_yt(S, pr, None, "f64", c["seed"])
    ref = orc(pr, None, c["seed"], np.arange(c["N"]))
    print("analytic 1e5 x 4 f64 max rel", rel(y, ref).max())
    assert rel(y, ref).max() <= TOL["f64"]
    for k, f in enumerate(oracle.payoffs(ref, c["K"])):
        e = oracle.estimate(f)
        assert abs(st["mean"][k] - e["mean"]) <= 1e-12 * abs(e["mean"])
        assert abs(st["var"][k] - e["var"]) <= 1e-9 * e["var"]
        assert abs(st["se"][k] - e["se"]) <= 1e-9 * e["se"]
    assert st["n"] == c["N"]


def test_gbm_analytic_1e5x4_f32_all_paths(S):
    c = W.CONFIGS["gbm_analytic_1e5x4"]
    pr = S.Problem(c["model"], c["theta"], c["Y0"], c["T"], c["M"], c["m"], c["N"], K=c["K"])
    st, y = gpu_yt(S, pr, None, "f32", c["seed"])
    ref = orc(pr, None, c["seed"], np.arange(c["N"]))
    r = rel(y, ref)
    print("analytic 1e5 x 4 f32 max rel", r.max(), "p99", np.quantile(r, 0.99))
    assert r.max() <= TOL["f32"]
    for k, f in enumerate(oracle.payoffs(ref, c["K"])):
        e = oracle.estimate(f)
        assert abs(st["mean"][k] - e["mean"]) <= 1e-6 * abs(e["mean"])


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_ou_analytic(S, prec):
    pr = S.Problem(W.OU, (0.5, 0.4, 1.7), 0.2, 2.0, 8, 5, 10_000, K=0.4, instance=3)
    st, y = gpu_yt(S, pr, None, prec, 9)
    ref = orc(pr, None, 9, np.arange(pr.N))
    # OU paths cross zero: compare against the path scale instead of |Y|
    err = np.abs(y - ref) / np.maximum(np.abs(ref), 0.5)
    assert err.max() <= TOL[prec]


@pytest.mark.parametrize("m", [2, 3, 4, 6, 7, 8])
def test_analytic_every_m_and_ragged_M(S, m):
    pr = S.Problem(W.GBM, (0.25, 0.05), 1.3, 0.7, 5, m, 3001, K=1.2)
    for prec in ("f64", "f32"):
        st, y = gpu_yt(S, pr, None, prec, 1234)
        ref = orc(pr, None, 1234, np.arange(pr.N))
        assert rel(y, ref).max() <= TOL[prec], (m, prec)


@pytest.mark.parametrize("N", [1, 15, 63, 65, 1000, 4099])
def test_ragged_path_counts(S, H, Ho, N):
    c = W.CONFIGS["gbm_mlp_2p22x16"]
    pr = S.Problem(c["model"], c["theta"], c["Y0"], c["T"], 7, c["m"], N, K=c["K"])
    ref = orc(pr, Ho, 5, np.arange(N))
    for prec in ("f64", "f32", "bf16", "f16", "bf16x3", "f16x3"):
        st, y = gpu_yt(S, pr, H, prec, 5)
        assert st["n"] == N
        assert rel(y, ref).max() <= TOL[prec], (N, prec)
        assert abs(st["mean"][0] - y.mean()) <= 1e-12 * abs(y.mean()) + 1e-7


def test_mlp_f64_matches_oracle(S, H, Ho):
    c = W.CONFIGS["gbm_mlp_2p22x16"]
    pr = S.Problem(c["model"], c["theta"], c["Y0"], c["T"], c["M"], c["m"], 4096, K=c["K"])
    st, y = gpu_yt(S, pr, H, "f64", c["seed"])
    ref = orc(pr, Ho, c["seed"], np.arange(pr.N))
    assert rel(y, ref).max() <= TOL["f64"]
    opr = oracle.Problem(c["model"], c["theta"], c["Y0"], c["T"], c["M"], c["m"])
    _, _, nood = oracle.simulate(opr, Ho, c["seed"], np.arange(pr.N))
    assert st["n_out_of_domain"] == nood


def test_mlp_f32_paths_and_means(S, H, Ho):
    """The 2^22 x 16 GBM setting on 2^17 paths: every path and both payoff means."""
    c = W.CONFIGS["gbm_mlp_2p22x16"]
    N = 2 ** 17
    pr = S.Problem(c["model"], c["theta"], c["Y0"], c["T"], c["M"], c["m"], N, K=c["K"])
    st, y = gpu_yt(S, pr, H, "f32", c["seed"])
    ref = orc(pr, Ho, c["seed"], np.arange(N))
    r = rel(y, ref)
    print(f"f32 GBM 16 steps, 2^17 paths: max rel {r.max():.3e} p99 {np.quantile(r, 0.99):.3e}")
    assert r.max() <= TOL["f32"]
    for k, f in enumerate(oracle.payoffs(ref, c["K"])):
        e = oracle.estimate(f)
        assert abs(st["mean"][k] - e["mean"]) <= 1e-6 * abs(e["mean"]), k


def test_gbm_2p22x16_full_size_every_path_and_means(S, H, Ho):
    """The full 2^22 x 16 workload in FP32 with the benchmark's default plan:
    the oracle recomputes every path, so each Y_T is checked -- at 1e-5
    while its normals stay within |X| <= 4, and at 1e-5 scaled by the
    interpolant's Lebesgue function at its largest |X| beyond that
    (tests/lebesgue.py) -- and both payoff means at 1e-6 relative."""
    c = W.CONFIGS["gbm_mlp_2p22x16"]
    pr = S.Problem(c["model"], c["theta"], c["Y0"], c["T"], c["M"], c["m"], c["N"], K=c["K"])
    st, y = gpu_yt(S, pr, H, "f32", c["seed"])
    paths = np.arange(c["N"])
    ref = orc(pr, Ho, c["seed"], paths)
    xmax = np.abs(oracle.step_normals(c["seed"], oracle.make_tag(0, 0), paths, c["M"])).max(axis=1)
    r = rel(y, ref)
    inner = xmax <= 4.0
    print(f"f32 GBM 2^22 x 16 full: max rel {r.max():.3e} p99 {np.quantile(r, 0.99):.3e} "
          f"over {c['N']} paths; {r[inner].max():.3e} on the paths with all |X| <= 4, "
          f"{np.count_nonzero(~inner)} beyond")
    assert r[inner].max() <= TOL["f32"]
    assert np.all(r <= f32_bound(c["m"], xmax)), (r / f32_bound(c["m"], xmax)).max()
    assert st["n"] == c["N"]
    for k, f in enumerate(oracle.payoffs(ref, c["K"])):
        e = oracle.estimate(f)
        d = abs(st["mean"][k] - e["mean"]) / abs(e["mean"])
        print(f"  payoff {k}: mean {st['mean'][k]:.9f} oracle {e['mean']:.9f} rel {d:.2e}")
        assert d <= 1e-6, k


@pytest.mark.parametrize("prec", ["bf16x3", "f16x3", "f32", "bf16", "f16"])
def test_gbm_2p24x32_full_size_sampled_paths(S, H, Ho, prec):
    c = W.CONFIGS["gbm_mlp_2p24x32"]
    pr = S.Problem(c["model"], c["theta"], c["Y0"], c["T"], c["M"], c["m"], c["N"], K=c["K"])
    st, y = gpu_yt(S, pr, H, prec, c["seed"])
    N = c["N"]
    sub = np.unique(np.concatenate([np.arange(4096), np.arange(N - 4096, N),
                                    np.arange(0, N, N // 8192)]))
    ref = orc(pr, Ho, c["seed"], sub)
    r = rel(y[sub], ref)
    print(f"{prec} GBM 2^24 x 32 full: max rel {r.max():.3e} p99 {np.quantile(r, 0.99):.3e} over {len(sub)}")
    assert r.max() <= TOL[prec]


def test_gbm_2p24x32_bf16x3_equal_weak_error_to_f32(S, H):
    """Same seed (common random numbers): the BF16x3 and FP32 means of Y_T
    differ by at most 2 SE of the paired difference or 10% of the FP32 weak
    error against the closed form E[Y_T] = Y0 exp(mu T)."""
    import math
    c = W.CONFIGS["gbm_mlp_2p24x32"]
    pr = S.Problem(c["model"], c["theta"], c["Y0"], c["T"], c["M"], c["m"], c["N"], K=c["K"])
    st32, y32 = gpu_yt(S, pr, H, "f32", c["seed"])
    stb, yb = gpu_yt(S, pr, H, "bf16x3", c["seed"])
    d = yb - y32
    se_pair = d.std(ddof=1) / math.sqrt(len(d))
    weak32 = abs(st32["mean"][0] - c["Y0"] * math.exp(c["theta"][1] * c["T"]))
    diff = abs(stb["mean"][0] - st32["mean"][0])
    print(f"mean bf16x3 - f32 = {diff:.3e}; paired SE {se_pair:.3e}; f32 weak error {weak32:.3e}")
    assert diff <= max(2 * se_pair, 0.1 * weak32)


def test_results_independent_of_launch_plan(S, H):
    c = W.CONFIGS["gbm_mlp_2p22x16"]
    pr = S.Problem(c["model"], c["theta"], c["Y0"], c["T"], 9, c["m"], 50_001, K=c["K"])
    for prec in ("bf16", "f32", "bf16x3", "f16x3"):
        outs = []
        plans = [None, dict(waves_per_block=1, blocks_per_cu=1, grab=1),
                 dict(waves_per_block=4, blocks_per_cu=1, grab=7),
                 dict(waves_per_block=2, blocks_per_cu=3, grab=2)]
        if prec.endswith("x3"):  # the split modes' all-LDS kernel: 12-wave workgroups
            plans += [dict(waves_per_block=12, blocks_per_cu=1, grab=1),
                      dict(waves_per_block=12, blocks_per_cu=2, grab=3)]
        for plan in plans:
            st, y = gpu_yt(S, pr, H, prec, 77, plan=plan)
            outs.append((st, y))
        for st, y in outs[1:]:
            assert np.array_equal(y, outs[0][1])
            assert st == outs[0][0]


def test_asynchronous_calls_on_two_streams(S, H):
    """Two calls that do not synchronise, on two streams, share the device's
    workspace: the second call's uploads must wait for the first call's
    kernels, and both results equal those of calls made one at a time."""
    c = W.CONFIGS["gbm_mlp_2p22x16"]
    pa = S.Problem(c["model"], c["theta"], c["Y0"], c["T"], c["M"], c["m"], c["N"], K=c["K"])
    pb = S.Problem(c["model"], (0.25, 0.02), 1.1, 0.5, 4, c["m"], 70_001, K=1.0)
    for prec in ("bf16x3", "pwl32", "f64"):
        ref_a = gpu_yt(S, pa, H, prec, 1)[1]
        ref_b = gpu_yt(S, pb, H, prec, 2)[1]
        dt = torch.float64 if prec == "f64" else torch.float32
        ya = torch.empty(pa.N, dtype=dt, device="cuda")
        yb = torch.empty(pb.N, dtype=dt, device="cuda")
        sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
        torch.cuda.synchronize()
        S.simulate(pa, H, prec=prec, seed=1, yt=ya, stats=False, stream=sa)
        S.simulate(pb, H, prec=prec, seed=2, yt=yb, stats=False, stream=sb)
        torch.cuda.synchronize()
        assert np.array_equal(ya.double().cpu().numpy(), ref_a), prec
        assert np.array_equal(yb.double().cpu().numpy(), ref_b), prec


def test_changing_a_network_waits_for_work_enqueued_with_it(S):
    """set_params and free release the network's device copies; a launch
    already enqueued with the old weights must still compute with them."""
    c = W.CONFIGS["gbm_mlp_2p22x16"]
    pr = S.Problem(c["model"], c["theta"], c["Y0"], c["T"], c["M"], c["m"], c["N"], K=c["K"])
    for prec in ("bf16x3", "f64"):
        H1 = S.Mlp.load(WEIGHTS)
        p0 = H1.params()
        ref = gpu_yt(S, pr, H1, prec, 5)[1]
        y = torch.empty(pr.N, dtype=torch.float64 if prec == "f64" else torch.float32, device="cuda")
        S.simulate(pr, H1, prec=prec, seed=5, yt=y, stats=False)
        H1.set_params(p0 * np.float32(1.5))
        torch.cuda.synchronize()
        assert np.array_equal(y.double().cpu().numpy(), ref), prec
        S.simulate(pr, H1, prec=prec, seed=5, yt=y, stats=False)
        del H1
        torch.cuda.synchronize()
        assert not np.array_equal(y.double().cpu().numpy(), ref), prec


def test_binding_refuses_mismatched_output_tensors(S, H):
    """Short, mistyped or strided output tensors are refused by the binding
    before the library could write past them."""
    pr = S.Problem(W.GBM, (0.3, 0.1), 1.0, 1.0, 4, 5, 1000)
    for bad in (torch.empty(999, device="cuda"), torch.empty(1000, dtype=torch.float64, device="cuda"),
                torch.empty(2000, device="cuda")[::2]):
        with pytest.raises(ValueError, match="yt must be"):
            S.simulate(pr, H, prec="f32", yt=bad)
    x = torch.zeros((10, 4), device="cuda")
    with pytest.raises(ValueError, match="out must be"):
        S.eval_H(H, x, prec="f32", out=torch.empty((10, 4), device="cuda"))


def test_path_offset_shards_compose(S, H):
    c = W.CONFIGS["gbm_mlp_2p22x16"]
    full = S.Problem(c["model"], c["theta"], c["Y0"], c["T"], 6, c["m"], 3000, K=c["K"])
    _, y = gpu_yt(S, full, H, "f32", 3)
    part = S.Problem(c["model"], c["theta"], c["Y0"], c["T"], 6, c["m"], 1000, K=c["K"],
                     path_offset=1500)
    _, yp = gpu_yt(S, part, H, "f32", 3)
    assert np.array_equal(yp, y[1500:2500])


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3", "f16x3", "pwl32", "pwl64"])
def test_path_indices_beyond_32_bits(S, H, Ho, prec):
    """Global path indices fill both 32-bit words of the Philox counter: a
    shard straddling 2^32 and the last shard of the 63-bit index range match
    the oracle at the same global indices."""
    c = W.CONFIGS["gbm_mlp_2p22x16"]
    tol = {"pwl32": TOL["f32"], "pwl64": TOL["f64"]}.get(prec, TOL.get(prec))
    N = 300
    for off in (2 ** 32 - 150, 2 ** 63 - 1 - N):
        pr = S.Problem(c["model"], c["theta"], c["Y0"], c["T"], 5, c["m"], N, K=c["K"],
                       path_offset=off)
        ref = orc(pr, Ho, 13, off + np.arange(N, dtype=np.int64))
        st, y = gpu_yt(S, pr, H, prec, 13)
        assert st["n"] == N
        assert rel(y, ref).max() <= tol, (prec, off)
    # the two shards differ from the first paths of the stream
    lo = S.Problem(c["model"], c["theta"], c["Y0"], c["T"], 5, c["m"], N, K=c["K"])
    assert not np.array_equal(gpu_yt(S, lo, H, prec, 13)[1], y)


def test_per_lane_kernel_beyond_2p32_paths(S):
    """The per-lane kernel (analytic map, FP32) at N = 2^32 + 1000 paths, one
    step: its blocks span both dimensions of the launch grid.  Paths sampled
    at the start, around 2^31 and 2^32 and at the end match the oracle, and
    every path is counted."""
    N = 2 ** 32 + 1000
    pr = S.Problem(W.GBM, (0.3, 0.1), 1.0, 0.25, 1, 5, N, K=1.0)
    st, yt = S.simulate(pr, None, prec="f32", seed=4, want_yt=True)
    torch.cuda.synchronize()
    idx = np.concatenate([np.arange(100), 2 ** 31 + np.arange(-50, 50), 2 ** 32 + np.arange(-50, 50),
                          N - 100 + np.arange(100)]).astype(np.int64)
    got = yt[torch.from_numpy(idx).cuda()].double().cpu().numpy()
    del yt
    ref = orc(pr, None, 4, idx)
    assert st["n"] == N
    assert rel(got, ref).max() <= TOL["f32"]
    # one step of the analytic map: E[Y_1] = Y0 sum_j w_j y_j exactly
    assert abs(st["mean"][0] - 1.0 * np.exp(0.1 * 0.25)) <= 5 * st["se"][0]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_per_lane_kernel_second_grid_row(S, H, Ho, prec):
    """Just past 2^16 blocks the per-lane launch grid gains a second row
    (N = 2^22 + 1000): sampled paths either side of the row boundary and at
    the end against the oracle."""
    N = 2 ** 22 + 1000
    c = W.CONFIGS["gbm_mlp_2p22x16"]
    pr = S.Problem(c["model"], c["theta"], c["Y0"], c["T"], 2, c["m"], N, K=c["K"])
    net, neto = (H, Ho) if prec == "f64" else (None, None)
    st, yt = S.simulate(pr, net, prec=prec, seed=6, want_yt=True)
    torch.cuda.synchronize()
    idx = np.concatenate([np.arange(64), 2 ** 22 + np.arange(-64, 64), N - 64 + np.arange(64)])
    got = yt.double().cpu().numpy()[idx]
    assert st["n"] == N
    assert rel(got, orc(pr, neto, 6, idx)).max() <= TOL[prec]


def test_eval_H_f64_second_grid_row(S, H, Ho):
    B = 2 ** 22 + 100
    x = W.gbm_features(B, seed=12).astype(np.float32)
    out = S.eval_H(H, torch.from_numpy(x).cuda(), prec="f64")
    torch.cuda.synchronize()
    idx = np.concatenate([np.arange(32), 2 ** 22 + np.arange(-32, 32), B - 32 + np.arange(32)])
    ref = Ho.forward(x[idx].astype(np.float64))
    got = out.double().cpu().numpy()[idx]
    assert np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 0.1)) <= 1.2e-7


@pytest.mark.parametrize("m2", [2, 3, 4, 6, 8])
def test_every_node_count_in_every_network_mode(S, m2, tmp_path):
    """Each kernel is specialised on m: networks with 2..8 outputs (other than
    the stored 5 and 7) against the oracle in every network mode."""
    H2, Ho2 = network_with_m_outputs(S, m2, str(tmp_path / f"gbm_m{m2}.sl7w"))
    c = W.CONFIGS["gbm_mlp_2p22x16"]
    pr = S.Problem(c["model"], c["theta"], c["Y0"], c["T"], 7, m2, 1000, K=c["K"])
    ref = orc(pr, Ho2, 17, np.arange(pr.N))
    assert np.all(np.isfinite(ref)) and ref.std() > 0.05
    for prec in ("f64", "f32", "bf16x3", "f16x3", "pwl32", "pwl64"):
        tol = {"pwl32": TOL["f32"], "pwl64": TOL["f64"]}.get(prec, TOL.get(prec))
        st, y = gpu_yt(S, pr, H2, prec, 17)
        assert st["n"] == pr.N
        assert rel(y, ref).max() <= tol, (m2, prec, rel(y, ref).max())


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16", "f16", "bf16x3", "f16x3"])
def test_eval_H_matches_oracle_forward(S, H, Ho, prec):
    x = W.gbm_features(5000, seed=99)
    ref = Ho.forward(x)
    out = S.eval_H(H, torch.tensor(x, dtype=torch.float32, device="cuda"), prec=prec)
    torch.cuda.synchronize()
    got = out.double().cpu().numpy()
    # inputs are rounded to FP32 before the call; compare against the oracle
    # on the same rounded inputs
    ref = Ho.forward(x.astype(np.float32).astype(np.float64))
    # outputs are FP32 in every mode
    # (the split BF16 form drops lo*lo, ~2^-16 of each product)
    tol = {"f64": 1.2e-7, "f32": 1e-5, "bf16": 2e-2, "f16": 5e-3, "bf16x3": 1e-4, "f16x3": 1e-5}[prec]
    assert np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 0.1)) <= tol


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3", "f16x3", "bf16", "f16", "pwl32", "pwl64"])
def test_degenerate_shapes(S, H, Ho, prec):
    """One step (M = 1), one path, a single 64-path block exactly, and the
    largest step of the training range, in every mode."""
    c = W.CONFIGS["gbm_mlp_2p22x16"]
    tol = {"pwl32": TOL["f32"], "pwl64": TOL["f64"]}.get(prec, TOL.get(prec))
    for T, M, N in ((0.5, 1, 1), (0.5, 1, 64), (1.0, 2, 129), (0.05, 1, 777)):
        pr = S.Problem(c["model"], c["theta"], c["Y0"], T, M, c["m"], N, K=c["K"])
        ref = orc(pr, Ho, 21, np.arange(N))
        st, y = gpu_yt(S, pr, H, prec, 21)
        assert st["n"] == N
        assert rel(y, ref).max() <= tol, (prec, T, M, N)


@pytest.mark.parametrize("m", [2, 8])
def test_analytic_extreme_node_counts_single_step(S, m):
    pr = S.Problem(W.GBM, (0.3, 0.1), 1.0, 0.25, 1, m, 1000, K=1.0)
    ref = orc(pr, None, 8, np.arange(pr.N))
    for prec in ("f64", "f32"):
        st, y = gpu_yt(S, pr, None, prec, 8)
        assert rel(y, ref).max() <= TOL[prec], (m, prec)
