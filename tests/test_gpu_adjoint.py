"""GPU reverse-mode sensitivities against the oracle's forward-mode tangents,
central finite differences with common random numbers and Black-Scholes.

Per-path parity (FP64): the adjoint's df/d(Y0, theta) per path equals
f'(Y_T) dY_T/d(Y0, theta) from the oracle's dual-number pass to 1e-10
relative (two independent differentiation modes of the same discrete scheme).
"""
import math
import os

import numpy as np
import pytest
import torch
from scipy.stats import norm

import oracle
import workloads as W
from nets import network_with_m_outputs

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WEIGHTS = os.path.join(ROOT, "tests", "golden", "gbm_mlp_4x64.sl7w")


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


def oracle_pathwise(pr, Ho, seed, payoff, N):
    opr = oracle.Problem(pr.model, pr.theta, pr.Y0, pr.T, pr.M, pr.m, pr.instance)
    YT, dY = oracle.simulate_tangent(opr, Ho, seed, np.arange(N))
    if payoff == 0:
        return YT, dY
    ind = (YT > pr.K).astype(float)
    return np.maximum(YT - pr.K, 0.0), dY * ind[:, None]


@pytest.mark.parametrize("case", ["gbm_analytic", "ou_analytic", "gbm_network"])
@pytest.mark.parametrize("payoff", [0, 1])
def test_per_path_sensitivities_match_oracle_tangents(S, H, Ho, case, payoff):
    if case == "gbm_analytic":
        pr, net, neto = S.Problem(W.GBM, (0.3, 0.1), 1.0, 1.0, 4, 5, 4096, K=1.0), None, None
    elif case == "ou_analytic":
        pr, net, neto = S.Problem(W.OU, (0.5, 0.4, 1.7), 0.2, 2.0, 7, 5, 4096, K=0.4), None, None
    else:
        pr, net, neto = S.Problem(W.GBM, (0.3, 0.1), 1.0, 1.0, 16, 5, 2048, K=1.0), H, Ho
    g, pp = S.adjoint(pr, net, prec="f64", seed=42, payoff=payoff, ckpt_every=4, per_path=True)
    pp = pp.cpu().numpy()
    f, df = oracle_pathwise(pr, neto, 42, payoff, pr.N)
    assert np.max(np.abs(pp[:, 0] - f)) <= 1e-12 * (1 + np.max(np.abs(f)))
    scale = 1 + np.max(np.abs(df), axis=0)
    err = np.max(np.abs(pp[:, 1:] - df), axis=0) / scale
    print(case, payoff, "max pathwise gradient error", err)
    assert np.all(err <= 1e-10)
    for q in range(df.shape[1]):
        assert abs(g["grad"][q] - df[:, q].mean()) <= 1e-11 * scale[q]


OU_WEIGHTS = os.path.join(ROOT, "tests", "golden", "ou_mlp_5x50_softplus.sl7w")
CIR_WEIGHTS = os.path.join(ROOT, "tests", "golden", "cir_mlp_5x64.sl7w")


def check_pathwise(pp, f, df, g, tol=1e-10):
    assert np.max(np.abs(pp[:, 0] - f)) <= 1e-12 * (1 + np.max(np.abs(f)))
    scale = 1 + np.max(np.abs(df), axis=0)
    err = np.max(np.abs(pp[:, 1:] - df), axis=0) / scale
    assert np.all(err <= tol), err
    for q in range(df.shape[1]):
        assert abs(g["grad"][q] - df[:, q].mean()) <= 1e-11 * scale[q]
    return err


@pytest.mark.parametrize("payoff", [0, 1])
def test_cir_network_adjoint_matches_oracle_tangents(S, payoff):
    """CIR with its 5-input, 7-output ReLU network: three parameters, the
    clamp at zero (a clamped step passes no gradient), FP64 per path."""
    Hc, Hco = S.Mlp.load(CIR_WEIGHTS), oracle.load_mlp(CIR_WEIGHTS)
    d = W.cir_instances(4)[2]
    pr = S.Problem(d["model"], d["theta"], d["Y0"], d["T"], d["M"], d["m"], 3000,
                   K=d["theta"][1])
    g, pp = S.adjoint(pr, Hc, prec="f64", seed=9, payoff=payoff, ckpt_every=3, per_path=True)
    f, df = oracle_pathwise(pr, Hco, 9, payoff, pr.N)
    err = check_pathwise(pp.cpu().numpy(), f, df, g)
    print("cir network", payoff, "max pathwise gradient error", err)


@pytest.mark.parametrize("payoff", [0, 1])
def test_softplus_network_adjoint_matches_oracle_tangents(S, payoff):
    """The paper's network (4 x 50 Softplus, padded to 64) on the OU model:
    the reverse pass recomputes each layer's pre-activation for the logistic
    derivative; FP64 per path against the oracle's dual-number pass, with
    ragged N and a checkpoint interval that does not divide M."""
    Ho_, Hoo = S.Mlp.load(OU_WEIGHTS), oracle.load_mlp(OU_WEIGHTS)
    P = W.OU_PAPER
    pr = S.Problem(P["model"], P["theta"], P["Y0"], P["T"], P["M"], P["m"], 1000, K=P["K"])
    g, pp = S.adjoint(pr, Ho_, prec="f64", seed=P["seed"], payoff=payoff, ckpt_every=3,
                      per_path=True)
    f, df = oracle_pathwise(pr, Hoo, P["seed"], payoff, pr.N)
    err = check_pathwise(pp.cpu().numpy(), f, df, g)
    print("ou softplus", payoff, "max pathwise gradient error", err)
    g32 = S.adjoint(pr, Ho_, prec="f32", seed=P["seed"], payoff=payoff, ckpt_every=3)
    for a, b, se in zip(g32["grad"], g["grad"], g["grad_se"]):
        assert abs(a - b) <= 1e-4 * abs(b) + 1e-3 * se, (a, b)
    for k in (1, 8):
        assert S.adjoint(pr, Ho_, prec="f64", seed=P["seed"], payoff=payoff, ckpt_every=k) == g


def test_adjoint_full_size_sampled_paths(S, H, Ho):
    """The adjoint workload at full size (N = 2^22, M = 16, checkpoint every
    4, the launch bench.py times): per-path df/d(Y0, sigma, mu) in FP64 on
    2048 sampled paths (first, last and strided) against the oracle's
    dual-number pass on the same global path indices."""
    c = W.CONFIGS["gbm_adjoint_2p22x16"]
    pr = S.Problem(c["model"], c["theta"], c["Y0"], c["T"], c["M"], c["m"], c["N"], K=c["K"])
    g, pp = S.adjoint(pr, H, prec="f64", seed=c["seed"], payoff=1, ckpt_every=c["ckpt"],
                      per_path=True)
    idx = np.unique(np.concatenate([np.arange(512), np.arange(pr.N - 512, pr.N),
                                    np.linspace(0, pr.N - 1, 1024).astype(np.int64)]))
    pp = pp[torch.from_numpy(idx).cuda()].cpu().numpy()
    opr = oracle.Problem(pr.model, pr.theta, pr.Y0, pr.T, pr.M, pr.m, pr.instance)
    YT, dY = oracle.simulate_tangent(opr, Ho, c["seed"], idx)
    ind = (YT > pr.K).astype(float)
    f, df = np.maximum(YT - pr.K, 0.0), dY * ind[:, None]
    assert np.max(np.abs(pp[:, 0] - f)) <= 1e-12 * (1 + np.max(np.abs(f)))
    err = np.max(np.abs(pp[:, 1:] - df), axis=0) / (1 + np.max(np.abs(df), axis=0))
    print("full-size sampled pathwise gradient error", err)
    assert np.all(err <= 1e-10)


def test_checkpoint_interval_does_not_change_results(S, H):
    pr = S.Problem(W.GBM, (0.3, 0.1), 1.0, 1.0, 16, 5, 3000, K=1.0)
    ref = S.adjoint(pr, H, prec="f64", seed=3, payoff=1, ckpt_every=1)
    for k in (3, 4, 16, 32):
        g = S.adjoint(pr, H, prec="f64", seed=3, payoff=1, ckpt_every=k)
        assert g == ref, k


def test_adjoint_vs_central_differences_with_crn(S, H):
    """The adjoint workload: N = 2^22, M = 16, K = 1, checkpoint every 4; bumps 1e-4 on Y0,
    sigma and mu; FP64 differences; gate 1e-3 relative for the FP64 sweep and
    for the FP32 and BF16X3 sweeps on MFMA."""
    c = W.CONFIGS["gbm_adjoint_2p22x16"]
    pr = S.Problem(c["model"], c["theta"], c["Y0"], c["T"], c["M"], c["m"], c["N"], K=c["K"])
    g = S.adjoint(pr, H, prec="f64", seed=c["seed"], payoff=1, ckpt_every=c["ckpt"])
    g32 = S.adjoint(pr, H, prec="f32", seed=c["seed"], payoff=1, ckpt_every=c["ckpt"])
    gx3 = S.adjoint(pr, H, prec="bf16x3", seed=c["seed"], payoff=1, ckpt_every=c["ckpt"])
    h = 1e-4
    for q in range(3):
        def bumped(d):
            th = list(c["theta"])
            y0 = c["Y0"]
            if q == 0:
                y0 += d
            else:
                th[q - 1] += d
            p2 = S.Problem(c["model"], tuple(th), y0, c["T"], c["M"], c["m"], c["N"], K=c["K"])
            st, _ = S.simulate(p2, H, prec="f64", seed=c["seed"])
            return st["mean"][1]
        fd = (bumped(h) - bumped(-h)) / (2 * h)
        print(f"param {q}: adjoint {g['grad'][q]:.8f} (FP32 MFMA {g32['grad'][q]:.8f}, "
              f"BF16X3 MFMA {gx3['grad'][q]:.8f}) fd {fd:.8f}")
        assert abs(g["grad"][q] - fd) <= 1e-3 * abs(fd)
        assert abs(g32["grad"][q] - fd) <= 1e-3 * abs(fd)
        assert abs(gx3["grad"][q] - fd) <= 1e-3 * abs(fd)


def test_analytic_map_greeks_vs_black_scholes(S):
    """Analytic GBM map, N = 2^22: delta, vega and d/dmu of the call within
    4 SE of Black-Scholes with drift (the 7L interpolation bias is ~1e-7)."""
    sig, mu, T, K, Y0 = 0.3, 0.1, 1.0, 1.0, 1.0
    pr = S.Problem(W.GBM, (sig, mu), Y0, T, 16, 5, 2 ** 22, K=K)
    g = S.adjoint(pr, None, prec="f64", seed=42, payoff=1, ckpt_every=4)
    d1 = (math.log(Y0 / K) + (mu + 0.5 * sig ** 2) * T) / (sig * math.sqrt(T))
    delta = math.exp(mu * T) * norm.cdf(d1)
    vega = Y0 * math.exp(mu * T) * math.sqrt(T) * norm.pdf(d1)
    dmu = T * Y0 * math.exp(mu * T) * norm.cdf(d1)
    assert abs(delta - 0.757672537048) < 1e-9 and abs(vega - 0.392293855456) < 1e-9
    for got, se, ref in zip(g["grad"], g["grad_se"], (delta, vega, dmu)):
        print(f"adjoint {got:.6f} +- {se:.1e} vs Black-Scholes {ref:.6f}")
        assert abs(got - ref) <= 4 * se + 1e-5


def test_f32_adjoint_close_to_f64(S, H):
    pr = S.Problem(W.GBM, (0.3, 0.1), 1.0, 1.0, 16, 5, 2 ** 16, K=1.0)
    g64 = S.adjoint(pr, H, prec="f64", seed=42, payoff=1)
    g32 = S.adjoint(pr, H, prec="f32", seed=42, payoff=1)
    for a, b in zip(g32["grad"], g64["grad"]):
        assert abs(a - b) <= 1e-3 * abs(b)


def test_autograd_function(S, H):
    pr = S.Problem(W.GBM, (0.3, 0.1), 1.0, 1.0, 8, 5, 8192, K=1.0)
    Y0 = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
    th = torch.tensor([0.3, 0.1], dtype=torch.float64, requires_grad=True)
    v = S.SL7Adjoint.apply(Y0, th, pr, H, "f64", 7, 1, 4)
    (2.0 * v).backward()
    g = S.adjoint(pr, H, prec="f64", seed=7, payoff=1, ckpt_every=4)
    assert abs(v.item() - g["value"]) == 0.0
    assert abs(Y0.grad.item() - 2 * g["grad"][0]) <= 1e-15
    assert np.allclose(th.grad.numpy(), 2 * np.array(g["grad"][1:]), rtol=0, atol=1e-15)


def test_autograd_function_on_device_tensors(S, H):
    """Y0 and theta as CUDA tensors (float64 and float32): the value and
    both gradients come back on their devices and in their dtypes."""
    pr = S.Problem(W.GBM, (0.3, 0.1), 1.0, 1.0, 8, 5, 8192, K=1.0)
    g = S.adjoint(pr, H, prec="f64", seed=7, payoff=1, ckpt_every=4)
    for dt in (torch.float64, torch.float32):
        Y0 = torch.tensor(1.0, dtype=dt, device="cuda", requires_grad=True)
        th = torch.tensor([0.3, 0.1], dtype=dt, device="cuda", requires_grad=True)
        v = S.SL7Adjoint.apply(Y0, th, pr, H, "f64", 7, 1, 4)
        assert v.is_cuda and v.dtype == dt
        (3.0 * v).backward()
        assert Y0.grad.is_cuda and Y0.grad.dtype == dt and th.grad.is_cuda and th.grad.dtype == dt
        tol = 1e-15 if dt == torch.float64 else 1e-6
        assert abs(Y0.grad.item() - 3 * g["grad"][0]) <= tol * max(1.0, abs(3 * g["grad"][0]))
        assert np.allclose(th.grad.double().cpu().numpy(), 3 * np.array(g["grad"][1:]), rtol=tol,
                           atol=0)


def test_training_loss_function_gives_the_weight_gradient(S, Ho):
    """SL7TrainLoss: the MSE training loss as a function of H's parameters;
    backward yields the weight gradient from the library's trainer kernels,
    checked against the oracle's FP64 back-propagation at 1e-4."""
    H = S.Mlp.load(WEIGHTS)
    X = W.gbm_features(1024, seed=34).astype(np.float32).astype(np.float64)
    Y = (Ho.forward(X) * 1.01).astype(np.float32).astype(np.float64)
    p = torch.tensor(H.params(), device="cuda", requires_grad=True)
    loss = S.SL7TrainLoss.apply(p, H, torch.tensor(X, dtype=torch.float32, device="cuda"),
                                torch.tensor(Y, dtype=torch.float32, device="cuda"))
    (0.5 * loss).backward()
    lo, dW, db = oracle.mse_loss_and_grads(Ho, X, Y)
    ref = 0.5 * oracle.flatten(dW, db)
    assert p.grad.is_cuda and p.grad.dtype == torch.float32
    assert abs(loss.item() - lo) <= 1e-4 * lo
    g = p.grad.double().cpu().numpy()
    assert np.max(np.abs(g - ref)) <= 1e-4 * np.max(np.abs(ref))


@pytest.mark.parametrize("payoff", [0, 1])
def test_piecewise_linear_adjoint_matches_oracle_tangents(S, H, Ho, payoff):
    """The reverse sweep through the compiled piecewise-linear form (slope in
    Y and compiled theta derivatives per piece) against the oracle's dual-
    number pass through the network, per path, FP64."""
    pr = S.Problem(W.GBM, (0.3, 0.1), 1.0, 1.0, 16, 5, 4096, K=1.0)
    g, pp = S.adjoint(pr, H, prec="pwl64", seed=42, payoff=payoff, ckpt_every=4, per_path=True)
    pp = pp.cpu().numpy()
    f, df = oracle_pathwise(pr, Ho, 42, payoff, pr.N)
    assert np.max(np.abs(pp[:, 0] - f)) <= 1e-12 * (1 + np.max(np.abs(f)))
    scale = 1 + np.max(np.abs(df), axis=0)
    err = np.max(np.abs(pp[:, 1:] - df), axis=0) / scale
    print("pwl64", payoff, "max pathwise gradient error", err)
    assert np.all(err <= 1e-10)


def test_piecewise_linear_adjoint_fp32_and_checkpoints(S, H):
    pr = S.Problem(W.GBM, (0.3, 0.1), 1.0, 1.0, 16, 5, 20_000, K=1.0)
    ref = S.adjoint(pr, H, prec="pwl64", seed=5, payoff=1, ckpt_every=4)
    for k in (1, 7):
        assert S.adjoint(pr, H, prec="pwl64", seed=5, payoff=1, ckpt_every=k) == ref
    g32 = S.adjoint(pr, H, prec="pwl32", seed=5, payoff=1, ckpt_every=4)
    for q in range(3):
        assert abs(g32["grad"][q] - ref["grad"][q]) <= 1e-4 * abs(ref["grad"][q]) + 1e-6


def test_piecewise_linear_adjoint_on_cir(S):
    """CIR (three parameters, zero clamp) through the compiled form against
    the network's own lane back-propagation, per path, FP64."""
    Hc = S.Mlp.load(os.path.join(ROOT, "tests", "golden", "cir_mlp_5x64.sl7w"))
    d = W.cir_instances(4)[2]
    pr = S.Problem(d["model"], d["theta"], d["Y0"], d["T"], d["M"], d["m"], 3000, K=d["theta"][1])
    _, a = S.adjoint(pr, Hc, prec="pwl64", seed=9, payoff=1, ckpt_every=4, per_path=True)
    _, b = S.adjoint(pr, Hc, prec="f64", seed=9, payoff=1, ckpt_every=4, per_path=True)
    a, b = a.cpu().numpy(), b.cpu().numpy()
    scale = 1 + np.max(np.abs(b), axis=0)
    assert np.all(np.max(np.abs(a - b), axis=0) / scale <= 1e-10)


@pytest.mark.parametrize("m2", [3, 8])
def test_adjoint_other_node_counts(S, m2, tmp_path):
    """Networks with 3 and 8 outputs (the stored head re-interpolated onto
    the other node sets): network and piecewise-linear reverse sweeps against
    the oracle's per-path tangents, FP64."""
    H2, Ho2 = network_with_m_outputs(S, m2, str(tmp_path / f"gbm_m{m2}.sl7w"))
    pr = S.Problem(W.GBM, (0.3, 0.1), 1.0, 1.0, 9, m2, 1500, K=1.0)
    f, df = oracle_pathwise(pr, Ho2, 23, 1, pr.N)
    for prec in ("f64", "pwl64"):
        g, pp = S.adjoint(pr, H2, prec=prec, seed=23, payoff=1, ckpt_every=4, per_path=True)
        err = check_pathwise(pp.cpu().numpy(), f, df, g)
        print(m2, prec, "max pathwise gradient error", err)


def test_adjoint_second_grid_row(S):
    """Just past 2^16 blocks (N = 2^22 + 1000) the adjoint's launch grid gains
    a second row: analytic map, FP64, sampled paths either side of the row
    boundary and at the end against the oracle's tangents."""
    N = 2 ** 22 + 1000
    pr = S.Problem(W.GBM, (0.3, 0.1), 1.0, 1.0, 3, 5, N, K=1.0)
    g, pp = S.adjoint(pr, None, prec="f64", seed=31, payoff=0, ckpt_every=2, per_path=True)
    idx = np.concatenate([np.arange(64), 2 ** 22 + np.arange(-64, 64), N - 64 + np.arange(64)])
    pp = pp[torch.from_numpy(idx).cuda()].cpu().numpy()
    opr = oracle.Problem(pr.model, pr.theta, pr.Y0, pr.T, pr.M, pr.m, pr.instance)
    f, df = oracle.simulate_tangent(opr, None, 31, idx)
    assert np.max(np.abs(pp[:, 0] - f)) <= 1e-12 * (1 + np.max(np.abs(f)))
    assert np.max(np.abs(pp[:, 1:] - df) / (1 + np.abs(df))) <= 1e-10


@pytest.mark.parametrize("prec", ["f64", "pwl64"])
def test_adjoint_path_indices_beyond_32_bits(S, H, Ho, prec):
    """A shard straddling global path index 2^32 (both Philox path words):
    per-path sensitivities against the oracle's tangents at the same global
    indices, network and piecewise-linear sweeps."""
    off, N = 2 ** 32 - 500, 1000
    pr = S.Problem(W.GBM, (0.3, 0.1), 1.0, 1.0, 6, 5, N, K=1.0, path_offset=off)
    g, pp = S.adjoint(pr, H, prec=prec, seed=19, payoff=0, ckpt_every=4, per_path=True)
    opr = oracle.Problem(pr.model, pr.theta, pr.Y0, pr.T, pr.M, pr.m, pr.instance)
    f, df = oracle.simulate_tangent(opr, Ho, 19, off + np.arange(N, dtype=np.int64))
    check_pathwise(pp.cpu().numpy(), f, df, g)
