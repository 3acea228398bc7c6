"""CPU-side checks of the C ABI: every declared symbol is exported, host logic
(Gauss-Hermite nodes, weight file, argument validation) behaves as the
header states.  No GPU work is launched here."""
import ctypes
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sl7.h")
WEIGHTS = os.path.join(ROOT, "tests", "golden", "gbm_mlp_4x64.sl7w")


@pytest.fixture(scope="module")
def L():
    from paper_2302_05170_amd import _lib
    _lib.lib()
    return _lib


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sl7_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(L):
    names = declared_functions()
    assert len(names) >= 10
    missing = [n for n in names if not hasattr(L.lib(), n)]
    assert not missing, missing


def test_version_and_error_string(L):
    assert b"gfx950" in L.lib().sl7_version()
    assert L.lib().sl7_gh_nodes(0, None, None) == L.SL7_EINVAL
    assert b"m=0" in L.lib().sl7_last_error()


@pytest.mark.parametrize("m", range(1, 17))
def test_gh_nodes_match_oracle(L, m):
    import paper_2302_05170_amd as S
    x, w = S.gh_nodes(m)
    xo, wo = oracle.gh_nodes(m)
    assert np.max(np.abs(x - xo)) <= 1e-13 * max(1.0, np.max(np.abs(xo)))
    assert np.max(np.abs(w - wo)) <= 1e-13
    if m % 2:
        assert x[m // 2] == 0.0


def test_weight_file_read_by_both_sides(L):
    import paper_2302_05170_amd as S
    H = S.Mlp.load(WEIGHTS)
    Ho = oracle.load_mlp(WEIGHTS)
    d = H.desc()
    assert (d.d_in, d.width, d.depth, d.m, d.act, d.model) == (Ho.d_in, Ho.width, Ho.depth, Ho.m,
                                                               Ho.act, Ho.model)
    assert np.array_equal(H.params(), Ho.params_f32())
    assert [d.in_scale[k] for k in range(4)] == list(Ho.in_scale)
    with tempfile.TemporaryDirectory() as tmp:
        p = os.path.join(tmp, "copy.sl7w")
        H.save(p)
        assert open(p, "rb").read() == open(WEIGHTS, "rb").read()


def test_bad_weight_files(L):
    import paper_2302_05170_amd as S
    with tempfile.TemporaryDirectory() as tmp:
        p = os.path.join(tmp, "bad.sl7w")
        open(p, "wb").write(b"NOPE" + bytes(64))
        with pytest.raises(S.Sl7Error) as e:
            S.Mlp.load(p)
        assert e.value.code == L.SL7_EINVAL
        open(p, "wb").write(open(WEIGHTS, "rb").read()[:200])
        with pytest.raises(S.Sl7Error) as e:
            S.Mlp.load(p)
        assert e.value.code == L.SL7_EINVAL
        with pytest.raises(S.Sl7Error) as e:
            S.Mlp.load(os.path.join(tmp, "missing.sl7w"))
        assert e.value.code == L.SL7_EIO


def test_create_rejects_nonfinite_and_bad_shapes(L):
    import paper_2302_05170_amd as S
    p = W.glorot_params(4, 5, seed=1)
    args = (4, 5, W.GBM)
    aff = ([1.0] * 4, [0.0] * 4, W.GBM_DOMAIN_LO, W.GBM_DOMAIN_HI)
    S.Mlp.create(*args, p, *aff)
    bad = p.copy()
    bad[17] = np.nan
    with pytest.raises(S.Sl7Error) as e:
        S.Mlp.create(*args, bad, *aff)
    assert e.value.code == L.SL7_ENUMERIC
    with pytest.raises(S.Sl7Error) as e:
        S.Mlp.create(4, 9, W.GBM, W.glorot_params(4, 9), *aff)  # m > 8
    assert e.value.code == L.SL7_EINVAL


def _sim_rc(L, H=None, prec=1, **kw):
    import paper_2302_05170_amd as S
    base = dict(model=W.GBM, theta=(0.3, 0.1), Y0=1.0, T=1.0, M=4, m=5, N=100)
    base.update(kw)
    pr = S.Problem(**base).c()
    st = L.Stats()
    rc = L.lib().sl7_simulate(ctypes.byref(pr), H.handle if H else None, prec, 42, None,
                              ctypes.byref(st), None, None)
    return rc, L.lib().sl7_last_error().decode()


@pytest.mark.parametrize("kw,needle", [
    (dict(m=1), "m=1"), (dict(m=9), "m=9"), (dict(M=0), "M=0"), (dict(N=0), "N=0"),
    (dict(T=0.0), "T"), (dict(T=float("nan")), "T"), (dict(theta=(-0.1, 0.1)), "sigma"),
    (dict(Y0=float("inf")), "Y0"), (dict(model=7), "model"),
    (dict(model=W.CIR, theta=(1.0, 0.05, 0.2), Y0=-0.1), "Y0"),
    (dict(model=W.OU, theta=(0.5, 0.3, 0.0)), "lambda"),
    (dict(path_offset=-1), "path_offset"), (dict(path_offset=2 ** 63 - 100), "63-bit"),
    (dict(N=2 ** 40 + 1), "too large"),
])
def test_simulate_rejects_bad_problems(L, kw, needle):
    rc, msg = _sim_rc(L, **kw)
    assert rc == L.SL7_EINVAL and needle in msg, (rc, msg)


def test_simulate_rejects_mismatched_network_and_precision(L):
    import paper_2302_05170_amd as S
    H = S.Mlp.load(WEIGHTS)
    rc, msg = _sim_rc(L, H=H, m=7)
    assert rc == L.SL7_EINVAL and "m=7" in msg
    rc, msg = _sim_rc(L, H=H, model=W.OU, theta=(0.5, 0.3, 1.0))
    assert rc == L.SL7_EINVAL
    rc, msg = _sim_rc(L, prec=L.BF16)  # analytic map has no BF16 form
    assert rc == L.SL7_EUNSUPPORTED
    rc, msg = _sim_rc(L, model=W.CIR, theta=(1.0, 0.05, 0.2), Y0=0.05, m=5)
    assert rc == L.SL7_EUNSUPPORTED
    rc, msg = _sim_rc(L, prec=9)
    assert rc == L.SL7_EINVAL


def test_plans_beyond_the_kernels_launch_bounds_are_rejected(L):
    import paper_2302_05170_amd as S
    H = S.Mlp.load(WEIGHTS)
    pr = S.Problem(W.GBM, (0.3, 0.1), 1.0, 1.0, 4, 5, 100).c()
    # L.BF16 (one pass) takes at most four waves per workgroup; 12 is for
    # the split modes only
    for bad in (dict(waves_per_block=8), dict(waves_per_block=3), dict(waves_per_block=12),
                dict(blocks_per_cu=0), dict(grab=0)):
        plan = L.Plan()
        plan.waves_per_block, plan.blocks_per_cu, plan.grab = 4, 1, 1
        for k, v in bad.items():
            setattr(plan, k, v)
        rc = L.lib().sl7_simulate(ctypes.byref(pr), H.handle, L.BF16, 1, None, None,
                                  ctypes.byref(plan), None)
        assert rc == L.SL7_EINVAL, bad


def test_narrow_softplus_network_rejected_by_piecewise_linear_adjoint(L):
    import paper_2302_05170_amd as S
    p = W.glorot_params(5, 5, seed=2, width=W.OU_WIDTH)
    H = S.Mlp.create(5, 5, W.OU, p, [1.0] * 5, [0.0] * 5, W.OU_DOMAIN_LO, W.OU_DOMAIN_HI,
                     width=W.OU_WIDTH, act=L.SOFTPLUS)
    d = H.desc()
    assert (d.width, d.act) == (W.OU_WIDTH, L.SOFTPLUS)
    assert np.array_equal(H.params(), p)
    pr = S.Problem(W.OU, (0.5, 0.3, 1.0), 0.2, 2.0, 8, 5, 100).c()
    g = L.Greeks()
    ws = ctypes.create_string_buffer(1 << 16)  # host memory; rejected before any use
    rc = L.lib().sl7_adjoint(ctypes.byref(pr), H.handle, L.PWL64, 1, 1, 4, ctypes.byref(g), None,
                             ctypes.cast(ws, ctypes.c_void_p), len(ws), None)
    assert rc == L.SL7_EUNSUPPORTED and "ReLU" in L.lib().sl7_last_error().decode()
    # wider than the kernels' 64 units: a valid network, rejected by the simulator
    H65 = S.Mlp.create(5, 5, W.OU, W.glorot_params(5, 5, width=65), [1.0] * 5, [0.0] * 5,
                       W.OU_DOMAIN_LO, W.OU_DOMAIN_HI, width=65, act=L.SOFTPLUS)
    rc, msg = _sim_rc(L, H=H65, model=W.OU, theta=(0.5, 0.3, 1.0))
    assert rc == L.SL7_EUNSUPPORTED and "width" in msg, msg


def test_adjoint_workspace_size(L):
    """sl7_adjoint_ws_bytes covers its documented parts: ceil(M / k) x N
    checkpoints (8 or 4 bytes), k x N x 32 bytes of per-step network state
    in FP64 (k x N x 128 in the MFMA modes F32 and BF16X3, 4 bytes of piece
    index in the PWL modes) and one 96-byte partial per 64-path block; 0 for
    bad arguments."""
    import paper_2302_05170_amd as S
    f = L.lib().sl7_adjoint_ws_bytes
    for N, M, k in ((1, 1, 1), (1000, 16, 4), (2 ** 22, 16, 4), (4097, 7, 3), (64, 32, 32)):
        pr = S.Problem(W.GBM, (0.3, 0.1), 1.0, 1.0, M, 5, N).c()
        nseg, nb = -(-M // k), -(-N // 64)
        for prec, el, words in ((L.F64, 8, 8), (L.F32, 4, 32), (L.BF16X3, 4, 32), (L.PWL64, 8, 1),
                                (L.PWL32, 4, 1)):
            need = el * nseg * N + 4 * words * k * 64 * nb + 96 * nb
            got = f(ctypes.byref(pr), prec, k)
            assert need <= got <= need + 4 * 256, (N, M, k, prec, got, need)
    pr = S.Problem(W.GBM, (0.3, 0.1), 1.0, 1.0, 16, 5, 1000).c()
    assert f(ctypes.byref(pr), L.F64, 0) == 0
    assert f(None, L.F64, 4) == 0


def test_batch_tuner_rejects_bad_batches(L):
    """sl7_autotune_batched checks its batch as sl7_simulate_batched does,
    before any device work."""
    import paper_2302_05170_amd as S
    plan = L.Plan()
    H = S.Mlp.load(os.path.join(ROOT, "tests", "golden", "cir_mlp_5x64.sl7w"))
    f = L.lib().sl7_autotune_batched
    assert f(None, 1, H.handle, L.BF16X3, None, ctypes.byref(plan), None) == L.SL7_EINVAL
    arr = (L.Problem * 2)(*[S.Problem(W.CIR, (1.0, 0.05, 0.3), 0.05, 1.0, 4, 7, 100).c()] * 2)
    assert f(arr, 0, H.handle, L.BF16X3, None, ctypes.byref(plan), None) == L.SL7_EINVAL
    assert f(arr, 2, None, L.BF16X3, None, ctypes.byref(plan), None) == L.SL7_EUNSUPPORTED
    assert f(arr, 2, H.handle, L.F64, None, ctypes.byref(plan), None) == L.SL7_EUNSUPPORTED
    assert f(arr, 2, H.handle, L.BF16X3, None, None, None) == L.SL7_EINVAL
    arr[1].m = 5
    assert f(arr, 2, H.handle, L.BF16X3, None, ctypes.byref(plan), None) == L.SL7_EINVAL


def test_binding_fails_loudly_without_the_library(L, monkeypatch, tmp_path):
    """With libsl7.so absent the binding raises on first use: there is no
    other implementation behind it to fall back to."""
    import paper_2302_05170_amd as S
    monkeypatch.setattr(L, "LIB_PATH", str(tmp_path / "libsl7.so"))
    monkeypatch.setattr(L, "_lib", None)
    with pytest.raises(RuntimeError, match="is missing"):
        L.lib()
    with pytest.raises(RuntimeError, match="is missing"):
        S.Mlp.load(WEIGHTS)
    with pytest.raises(RuntimeError, match="is missing"):
        S.gh_nodes(5)


def test_binding_refuses_tensors_it_cannot_size(L):
    """The C ABI takes bare device pointers; the binding checks every caller
    tensor against the shape the library will read or write before the call
    (here a host tensor, refused without touching a device)."""
    import torch
    import paper_2302_05170_amd as S
    pr = S.Problem(W.GBM, (0.3, 0.1), 1.0, 1.0, 4, 5, 100)
    with pytest.raises(ValueError, match="yt must be"):
        S.simulate(pr, None, prec="f32", yt=torch.empty(100))


def test_default_plan_takes_the_all_lds_split_kernel_for_large_launches(L):
    """sl7_default_plan (host only): the split modes run 12-wave workgroups
    from 64 blocks of 64 paths per compute unit and 4-wave ones below; no
    other mode takes 12 waves; every default passes the calls' own checks."""
    def plan(prec, blocks, n_cu=256):
        p = L.Plan()
        L.check(L.lib().sl7_default_plan(prec, blocks, n_cu, ctypes.byref(p)))
        return (p.waves_per_block, p.blocks_per_cu, p.grab)
    for prec in (L.BF16X3, L.F16X3):
        assert plan(prec, 64 * 256) == (12, 1, 1)
        assert plan(prec, 2 ** 18) == (12, 1, 1)
        assert plan(prec, 64 * 256 - 1)[0] == 4
        assert plan(prec, 3125)[0] == 4  # the paper's OU shape, 2e5 paths
        assert plan(prec, 64 * 80, n_cu=80) == (12, 1, 1)
    for prec in (L.F32, L.BF16, L.F16, L.PWL32, L.PWL64, L.F64):
        assert plan(prec, 2 ** 20)[0] in (1, 2, 4)
    p = L.Plan()
    assert L.lib().sl7_default_plan(L.BF16X3, 100, 0, ctypes.byref(p)) == L.SL7_EINVAL
    assert L.lib().sl7_default_plan(99, 100, 256, ctypes.byref(p)) == L.SL7_EINVAL
    assert L.lib().sl7_default_plan(L.BF16X3, 100, 256, None) == L.SL7_EINVAL


def test_c_program_links_and_calls_host_entry_points(L, tmp_path):
    """The boundary is plain C: a C99 program includes sl7.h, links
    libsl7.so and calls two host-only entry points (no device needed): the
    Gauss-Hermite nodes for m = 3 (0, +-sqrt(3)) and the default plan."""
    import shutil
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    src = tmp_path / "abi_check.c"
    src.write_text(r'''
#include <math.h>
#include <stdio.h>
#include "sl7.h"
int main(void) {
  double x[3], w[3];
  if (sl7_gh_nodes(3, x, w) != SL7_OK) return 1;
  if (fabs(x[0] + sqrt(3.0)) > 1e-14 || fabs(x[1]) > 1e-15 || fabs(x[2] - sqrt(3.0)) > 1e-14)
    return 2;
  sl7_plan p;
  if (sl7_default_plan(SL7_BF16X3, 1 << 20, 256, &p) != SL7_OK || p.waves_per_block != 12) return 3;
  if (sl7_default_plan(SL7_F32, 1 << 20, 256, &p) != SL7_OK || p.waves_per_block != 4) return 4;
  if (sl7_default_plan(SL7_F32, 1, 0, &p) != SL7_EINVAL) return 5;
  printf("ok %s\n", sl7_version());
  return 0;
}
''')
    exe = tmp_path / "abi_check"
    libdir = os.path.dirname(L.LIB_PATH)
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                        str(src), "-o", str(exe), "-L", libdir, "-lsl7", "-lm",
                        f"-Wl,-rpath,{libdir}"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.startswith("ok"), (r.returncode, r.stdout, r.stderr)
