"""GPU parity for the paper's own experiment: the Ornstein-Uhlenbeck SDE
(eq. 6.5) simulated with the paper's network shape (4 hidden layers of 50
Softplus units, Numerical Results section), at the path counts of Table 6.1.

The 50-unit layers run zero-padded to 64 on the MFMA kernels.  OU paths cross
zero, so the per-path error is taken against max(|oracle|, 0.5), the path
scale (the same reading as the analytic OU test).  Tolerances as for GBM
(FP64 1e-12, FP32 1e-5, split BF16 2e-3, split FP16 5e-4, the one-pass modes
against sanity bounds, 0.5 / 0.1, twice the worst error measured on this
network: the weights rounded once make a fixed bias in every step, which the
tail paths below amplify).

FP32: 1e-5 for every path.  A path that draws some |X| > 4 extrapolates the
degree-4 interpolant there, which multiplies the network's FP32 output error
by the Lebesgue function (22.6 at |X| = 4, 43 at 4.5, 89 at 5.2); those
paths (97 of the 2e5) stay within the gate because the kernel carries the
first-layer constant as two floats.  Rounded once to FP32, that constant
shifted every output of a step alike, and the extrapolating paths reached
1.26e-5.  Errors are printed separately for paths with all |X| <= 4.
"""
import os

import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WEIGHTS = os.path.join(ROOT, "tests", "golden", "ou_mlp_5x50_softplus.sl7w")
TOL = {"f64": 1e-12, "f32": 1e-5, "bf16x3": 2e-3, "f16x3": 5e-4, "bf16": 0.5, "f16": 0.1}
PAPER = W.OU_PAPER


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


def err(got, ref):
    return np.abs(got - ref) / np.maximum(np.abs(ref), 0.5)


def problem(S, N, M=PAPER["M"]):
    return S.Problem(PAPER["model"], PAPER["theta"], PAPER["Y0"], PAPER["T"], M, PAPER["m"], N,
                     K=PAPER["K"])


def gpu_yt(S, pr, H, prec, seed):
    st, yt = S.simulate(pr, H, prec=prec, seed=seed, want_yt=True)
    torch.cuda.synchronize()
    return st, yt.double().cpu().numpy()


@pytest.fixture(scope="module")
def ref_paths(S, Ho):
    """Oracle Y_T for every path at the largest path count of Table 6.1 (the
    smaller counts are prefixes of it: same seed, global path indices) and
    each path's largest |X| over the steps."""
    N = max(PAPER["path_counts"])
    pr = problem(S, N)
    opr = oracle.Problem(pr.model, pr.theta, pr.Y0, pr.T, pr.M, pr.m, pr.instance)
    y, _, _ = oracle.simulate(opr, Ho, PAPER["seed"], np.arange(N))
    X = oracle.step_normals(PAPER["seed"], oracle.make_tag(0, pr.instance), np.arange(N), pr.M)
    return y, np.abs(X).max(axis=1)


def test_network_is_the_papers_shape(H, Ho):
    d = H.desc()
    assert (d.d_in, d.width, d.depth, d.m, d.act, d.model) == (5, 50, 4, 5, oracle.ACT_SOFTPLUS,
                                                               W.OU)
    assert (Ho.width, Ho.act) == (50, oracle.ACT_SOFTPLUS)


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3", "f16x3", "bf16", "f16"])
def test_table61_path_counts(S, H, ref_paths, prec):
    ref_all, xmax_all = ref_paths
    for N in PAPER["path_counts"]:
        st, y = gpu_yt(S, problem(S, N), H, prec, PAPER["seed"])
        e = err(y, ref_all[:N])
        inner = xmax_all[:N] <= 4.0
        print(f"OU softplus {prec} N={N} max err {e.max():.3e}; paths with all |X| <= 4: "
              f"{e[inner].max():.3e}; {np.count_nonzero(~inner)} extrapolating paths: "
              f"{e[~inner].max() if np.any(~inner) else 0.0:.3e}")
        assert st["n"] == N
        assert e.max() <= TOL[prec], (prec, N, e.max())
        if prec in ("f64", "f32"):
            f = oracle.estimate(ref_all[:N])
            assert abs(st["mean"][0] - f["mean"]) <= (1e-12 if prec == "f64" else 1e-6) * max(
                abs(f["mean"]), 0.5)


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3"])
def test_ragged_counts_and_steps(S, H, Ho, prec):
    for N, M in ((1, 3), (63, 5), (65, 11), (1001, 2)):
        pr = problem(S, N, M=M)
        opr = oracle.Problem(pr.model, pr.theta, pr.Y0, pr.T, pr.M, pr.m, pr.instance)
        ref, _, _ = oracle.simulate(opr, Ho, 3, np.arange(N))
        st, y = gpu_yt(S, pr, H, prec, 3)
        assert err(y, ref).max() <= TOL[prec], (prec, N, M)


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3", "f16x3"])
def test_eval_H_softplus_matches_oracle_forward(S, H, Ho, prec):
    x = W.ou_features(5000, seed=99).astype(np.float32).astype(np.float64)
    ref = Ho.forward(x)
    out = S.eval_H(H, torch.tensor(x, dtype=torch.float32, device="cuda"), prec=prec)
    torch.cuda.synchronize()
    got = out.double().cpu().numpy()
    # Softplus keeps every unit active, so the split modes' dropped lo*lo
    # products (2^-16 of each product in BF16, 2^-22 in FP16) add up over all
    # 50 units of a layer; the 16-bit kernels also use the hardware exp2 and
    # log2 for Softplus.  Bounds: 1e-3 (BF16 split), 5e-5 (FP16 split).
    tol = {"f64": 1.2e-7, "f32": 1e-5, "bf16x3": 1e-3, "f16x3": 5e-5}[prec]
    e = np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 0.1))
    print(f"eval_H OU softplus {prec}: max rel err {e:.3e}")
    assert e <= tol
