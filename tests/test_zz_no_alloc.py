"""sl7_simulate_noalloc (scratch in the library's fixed per-device array, no
allocation) against sl7_simulate on the same inputs, through the C ABI: Y_T
and the statistics must be identical, bit for bit, on two calls in a row,
the second with a smaller input (the array keeps the first call's contents),
at the largest size the array takes, and in each kernel family (network on
MFMA, network and analytic map one path per lane).  Sizes beyond the array,
the piecewise-linear modes and a network without a device copy are refused
before any device work."""
import os

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WEIGHTS = os.path.join(ROOT, "tests", "golden", "gbm_mlp_4x64.sl7w")
MAX_N = 2 ** 24


@pytest.fixture(scope="module")
def S():
    import paper_2302_05170_amd as S
    assert torch.cuda.is_available()
    return S


@pytest.fixture(scope="module")
def H(S):
    return S.Mlp.load(WEIGHTS)


def problem(S, N, M=9):
    c = W.CONFIGS["gbm_mlp_2p22x16"]
    return S.Problem(c["model"], c["theta"], c["Y0"], c["T"], M, c["m"], N, K=c["K"])


def regular(S, pr, H, prec, seed):
    st, yt = S.simulate(pr, H, prec=prec, seed=seed, want_yt=True)
    torch.cuda.synchronize()
    return st, yt.cpu()


def noalloc(S, pr, H, prec, seed):
    dt = torch.float64 if prec == "f64" else torch.float32
    yt = torch.full((int(pr.N),), float("nan"), dtype=dt, device="cuda")
    stats = torch.full((S.api.STATS_DOUBLES,), float("nan"), dtype=torch.float64, device="cuda")
    S.simulate_noalloc(pr, H, prec=prec, seed=seed, yt=yt, stats=stats)
    torch.cuda.synchronize()
    return S.stats_from_tensor(stats), yt.cpu()


@pytest.mark.parametrize("prec,net", [("f32", True), ("bf16x3", True), ("bf16", True),
                                      ("f64", True), ("f32", False), ("f64", False)])
def test_two_calls_in_a_row_match_the_allocating_entry_point(S, H, prec, net):
    Hn = H if net else None
    for N, seed in ((200_003, 7), (1_000, 8)):
        pr = problem(S, N)
        ref_st, ref_yt = regular(S, pr, Hn, prec, seed)
        print(f"noalloc {prec} net={net} N={N} seed={seed}", flush=True)
        st, yt = noalloc(S, pr, Hn, prec, seed)
        assert torch.equal(yt, ref_yt), (prec, N)
        assert st == ref_st, (prec, N)


def test_largest_size_the_array_takes(S, H):
    c = W.CONFIGS["gbm_mlp_2p24x32"]
    pr = S.Problem(c["model"], c["theta"], c["Y0"], c["T"], c["M"], c["m"], MAX_N, K=c["K"])
    ref_st, ref_yt = regular(S, pr, H, "bf16x3", c["seed"])
    print("noalloc bf16x3 N=2^24", flush=True)
    st, yt = noalloc(S, pr, H, "bf16x3", c["seed"])
    assert torch.equal(yt, ref_yt)
    assert st == ref_st
    # then a smaller call: the stale partials of the large one are not read
    pr2 = problem(S, 4097)
    ref_st2, ref_yt2 = regular(S, pr2, H, "bf16x3", 3)
    st2, yt2 = noalloc(S, pr2, H, "bf16x3", 3)
    assert torch.equal(yt2, ref_yt2) and st2 == ref_st2


def test_refusals_before_any_device_work(S, H):
    from paper_2302_05170_amd import _lib as L
    with pytest.raises(L.Sl7Error, match="exceeds the fixed scratch"):
        S.simulate_noalloc(problem(S, MAX_N + 1), H, prec="bf16x3", seed=1)
    with pytest.raises(L.Sl7Error, match="piecewise-linear"):
        S.simulate_noalloc(problem(S, 1000), H, prec="pwl32", seed=1)
    fresh = S.Mlp.load(WEIGHTS)
    with pytest.raises(L.Sl7Error, match="no device copy"):
        S.simulate_noalloc(problem(S, 1000), fresh, prec="f16x3", seed=1)
    # an allocating call makes the copy; then the call goes through
    ref_st, ref_yt = regular(S, problem(S, 1000), fresh, "f16x3", 1)
    st, yt = noalloc(S, problem(S, 1000), fresh, "f16x3", 1)
    assert torch.equal(yt, ref_yt) and st == ref_st
