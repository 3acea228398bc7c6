"""Python face of the C ABI: the same calls, with torch tensors as device
buffers and torch's current stream as the HIP stream."""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib as L

PRECISIONS = {"f64": L.F64, "f32": L.F32, "bf16": L.BF16, "f16": L.F16, "bf16x3": L.BF16X3,
              "f16x3": L.F16X3, "pwl32": L.PWL32, "pwl64": L.PWL64}


def _prec(p) -> int:
    if isinstance(p, str):
        return PRECISIONS[p]
    return int(p)


def _stream(stream=None) -> int:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _ptr(t) -> int | None:
    if t is None:
        return None
    return t.data_ptr()


def _check_tensor(name: str, t: torch.Tensor, dtype, shape) -> None:
    """The library reads or writes `t` as a dense device array of `shape`:
    refuse anything else here, where the tensor's size is still known."""
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dtype \
            or tuple(t.shape) != tuple(int(v) for v in shape) or not t.is_contiguous():
        got = (f"{tuple(t.shape)} {t.dtype} on {t.device}"
               f"{'' if t.is_contiguous() else ', not contiguous'}"
               if isinstance(t, torch.Tensor) else type(t).__name__)
        raise ValueError(f"{name} must be a contiguous CUDA {dtype} tensor of shape "
                         f"{tuple(int(v) for v in shape)}; got {got}")


def gh_nodes(m: int):
    """Probabilists' Gauss-Hermite nodes and weights (weights sum to 1)."""
    x = np.zeros(m)
    w = np.zeros(m)
    L.check(L.lib().sl7_gh_nodes(m, x.ctypes.data, w.ctypes.data))
    return x, w


@dataclass
class Problem:
    """One simulation instance (sl7_problem).  theta: GBM (sigma, mu); OU
    (ybar, sigma, lambda); CIR (kappa, ybar, gamma)."""
    model: int
    theta: tuple
    Y0: float
    T: float
    M: int
    m: int
    N: int
    K: float = 1.0
    path_offset: int = 0
    instance: int = 0

    def c(self) -> L.Problem:
        p = L.Problem()
        p.model, p.m, p.M, p.N = int(self.model), int(self.m), int(self.M), int(self.N)
        for k, v in enumerate(self.theta):
            p.theta[k] = float(v)
        p.Y0, p.T, p.K = float(self.Y0), float(self.T), float(self.K)
        p.path_offset, p.instance = int(self.path_offset), int(self.instance)
        return p


class Mlp:
    """Handle of the collocation network H (sl7_mlp)."""

    def __init__(self, handle: ctypes.c_void_p):
        self._h = handle

    @classmethod
    def load(cls, path: str) -> "Mlp":
        h = ctypes.c_void_p()
        L.check(L.lib().sl7_mlp_load(path.encode(), ctypes.byref(h)))
        return cls(h)

    @classmethod
    def create(cls, d_in: int, m: int, model: int, params, in_scale, in_shift, dom_lo, dom_hi,
               width: int = 64, depth: int = 4, act: int = L.RELU) -> "Mlp":
        d = L.MlpDesc()
        d.d_in, d.width, d.depth, d.m, d.act, d.model = d_in, width, depth, m, act, model
        for k in range(d_in):
            d.in_scale[k], d.in_shift[k] = float(in_scale[k]), float(in_shift[k])
            d.dom_lo[k], d.dom_hi[k] = float(dom_lo[k]), float(dom_hi[k])
        p = np.ascontiguousarray(params, dtype=np.float32)
        n = L.lib().sl7_mlp_n_params(ctypes.byref(d))
        if n < 0:
            L.check(L.SL7_EINVAL)
        if p.size != n:
            raise ValueError(f"expected {n} parameters, got {p.size}")
        h = ctypes.c_void_p()
        L.check(L.lib().sl7_mlp_create(ctypes.byref(d), p.ctypes.data, ctypes.byref(h)))
        return cls(h)

    @property
    def handle(self):
        return self._h

    def desc(self) -> L.MlpDesc:
        d = L.MlpDesc()
        L.check(L.lib().sl7_mlp_get_desc(self._h, ctypes.byref(d)))
        return d

    def n_params(self) -> int:
        d = self.desc()
        return int(L.lib().sl7_mlp_n_params(ctypes.byref(d)))

    def params(self) -> np.ndarray:
        out = np.empty(self.n_params(), np.float32)
        L.check(L.lib().sl7_mlp_get_params(self._h, out.ctypes.data))
        return out

    def set_params(self, p) -> None:
        p = np.ascontiguousarray(p, dtype=np.float32)
        if p.size != self.n_params():
            raise ValueError("parameter count mismatch")
        L.check(L.lib().sl7_mlp_set_params(self._h, p.ctypes.data))

    def save(self, path: str) -> None:
        L.check(L.lib().sl7_mlp_save(self._h, path.encode()))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and L._lib is not None:
            L._lib.sl7_mlp_free(h)
            self._h = None


def _plan(plan):
    if plan is None:
        return None
    p = L.Plan()
    p.waves_per_block = int(plan.get("waves_per_block", 4))
    p.blocks_per_cu = int(plan.get("blocks_per_cu", 1))
    p.grab = int(plan.get("grab", 1))
    return p


def _stats_dict(s: L.Stats) -> dict:
    return {"mean": [s.mean[0], s.mean[1]], "var": [s.var[0], s.var[1]],
            "se": [s.se[0], s.se[1]], "n": s.n, "n_clamped": s.n_clamped,
            "n_out_of_domain": s.n_out_of_domain}


def simulate(pr: Problem, H: Mlp | None = None, prec="f32", seed: int = 42, want_yt: bool = False,
             yt: torch.Tensor | None = None, plan: dict | None = None, stats: bool = True,
             stream=None):
    """Runs sl7_simulate.  Returns (stats dict or None, Y_T tensor or None)."""
    p = _prec(prec)
    dt = torch.float64 if p in (L.F64, L.PWL64) else torch.float32
    if want_yt and yt is None:
        yt = torch.empty(int(pr.N), dtype=dt, device="cuda")
    if yt is not None:
        _check_tensor("yt", yt, dt, (int(pr.N),))
    st = L.Stats()
    pl = _plan(plan)
    cp = pr.c()
    L.check(L.lib().sl7_simulate(ctypes.byref(cp), H.handle if H is not None else None, p,
                                 int(seed) & 0xFFFFFFFFFFFFFFFF, _ptr(yt),
                                 ctypes.byref(st) if stats else None,
                                 ctypes.byref(pl) if pl is not None else None, _stream(stream)))
    return (_stats_dict(st) if stats else None), yt


def simulate_cdc(pr: Problem, H: Mlp | None = None, prec="f32", seed: int = 42,
                 want_yt: bool = False, yt: torch.Tensor | None = None, stats: bool = True,
                 stream=None):
    """Runs sl7_simulate_cdc (the 7L-CDC variant; prec "f64" or "f32").
    Returns (stats dict or None, Y_T tensor or None)."""
    p = _prec(prec)
    dt = torch.float64 if p == L.F64 else torch.float32
    if want_yt and yt is None:
        yt = torch.empty(int(pr.N), dtype=dt, device="cuda")
    if yt is not None:
        _check_tensor("yt", yt, dt, (int(pr.N),))
    st = L.Stats()
    cp = pr.c()
    L.check(L.lib().sl7_simulate_cdc(ctypes.byref(cp), H.handle if H is not None else None, p,
                                     int(seed) & 0xFFFFFFFFFFFFFFFF, _ptr(yt),
                                     ctypes.byref(st) if stats else None, _stream(stream)))
    return (_stats_dict(st) if stats else None), yt


STATS_DOUBLES = ctypes.sizeof(L.Stats) // 8


def stats_from_tensor(t: torch.Tensor) -> dict:
    """Statistics dict from the device sl7_stats that simulate_noalloc filled
    (copies to the host, so it waits for the call's work)."""
    s = L.Stats.from_buffer_copy(t.cpu().numpy().tobytes())
    return _stats_dict(s)


def simulate_noalloc(pr: Problem, H: Mlp | None = None, prec="f32", seed: int = 42,
                     yt: torch.Tensor | None = None, stats: torch.Tensor | None = None,
                     plan: dict | None = None, stream=None) -> None:
    """Runs sl7_simulate_noalloc with caller-owned device buffers: yt (N
    values, or None) and stats (a float64 CUDA tensor of STATS_DOUBLES
    values that receives the sl7_stats, or None).  Enqueues work only; read
    stats with stats_from_tensor."""
    p = _prec(prec)
    dt = torch.float64 if p in (L.F64, L.PWL64) else torch.float32
    if yt is not None:
        _check_tensor("yt", yt, dt, (int(pr.N),))
    if stats is not None:
        _check_tensor("stats", stats, torch.float64, (STATS_DOUBLES,))
    pl = _plan(plan)
    cp = pr.c()
    L.check(L.lib().sl7_simulate_noalloc(ctypes.byref(cp), H.handle if H is not None else None, p,
                                         int(seed) & 0xFFFFFFFFFFFFFFFF, _ptr(yt), _ptr(stats),
                                         ctypes.byref(pl) if pl is not None else None,
                                         _stream(stream)))


def pwl_compile(H: Mlp, pr: Problem, max_pieces: int = 1 << 16) -> dict:
    """The exact piecewise-linear form of the ReLU network H along Y for
    instance pr (sl7_pwl_compile, host only): breakpoints [P-1], anchors [P],
    slopes and values [P, m] with y_j = value + slope (Y - anchor)."""
    import numpy as np
    cp = pr.c()
    n = ctypes.c_int(0)
    L.check(L.lib().sl7_pwl_compile(H.handle, ctypes.byref(cp), int(max_pieces), ctypes.byref(n),
                                    None, None, None, None))
    P, m = n.value, int(pr.m)
    brk, anc = np.zeros(max(P - 1, 0)), np.zeros(P)
    slope, value = np.zeros((P, m)), np.zeros((P, m))
    ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p) if a.size else ctypes.c_void_p(
        ctypes.addressof(ctypes.c_double()))
    L.check(L.lib().sl7_pwl_compile(H.handle, ctypes.byref(cp), int(max_pieces), ctypes.byref(n),
                                    ptr(brk), ptr(anc), ptr(slope), ptr(value)))
    return {"breaks": brk, "anchor": anc, "slope": slope, "value": value}


def autotune(shape: Problem, H: Mlp, prec="bf16x3", cache_path: str | None = None,
             stream=None) -> dict:
    """Fastest launch plan for problems shaped like `shape` (sl7_autotune)."""
    cp = shape.c()
    plan = L.Plan()
    L.check(L.lib().sl7_autotune(ctypes.byref(cp), H.handle, _prec(prec),
                                 cache_path.encode() if cache_path else None, ctypes.byref(plan),
                                 _stream(stream)))
    return {"waves_per_block": plan.waves_per_block, "blocks_per_cu": plan.blocks_per_cu,
            "grab": plan.grab}


def autotune_batched(prs: list, H: Mlp, prec="bf16x3", cache_path: str | None = None,
                     stream=None) -> dict:
    """Fastest launch plan for the batch prs itself (sl7_autotune_batched)."""
    arr = (L.Problem * len(prs))(*[p.c() for p in prs])
    plan = L.Plan()
    L.check(L.lib().sl7_autotune_batched(arr, len(prs), H.handle, _prec(prec),
                                         cache_path.encode() if cache_path else None,
                                         ctypes.byref(plan), _stream(stream)))
    return {"waves_per_block": plan.waves_per_block, "blocks_per_cu": plan.blocks_per_cu,
            "grab": plan.grab}


def simulate_batched(prs: list, H: Mlp, prec="bf16", seed: int = 11, plan: dict | None = None,
                     use_graph: bool = True, stream=None) -> list:
    """Runs sl7_simulate_batched; returns one stats dict per instance."""
    n = len(prs)
    arr = (L.Problem * n)(*[p.c() for p in prs])
    st = (L.Stats * n)()
    pl = _plan(plan)
    L.check(L.lib().sl7_simulate_batched(arr, n, H.handle, _prec(prec), int(seed), st,
                                         ctypes.byref(pl) if pl is not None else None,
                                         1 if use_graph else 0, _stream(stream)))
    return [_stats_dict(st[k]) for k in range(n)]


def eval_H(H: Mlp, inputs: torch.Tensor, prec="f32", out: torch.Tensor | None = None,
           stream=None) -> torch.Tensor:
    """Batched forward pass: inputs [B, d_in] float32 on the GPU -> [B, m]."""
    d = H.desc()
    if inputs.dtype != torch.float32 or not inputs.is_cuda or inputs.dim() != 2 \
            or inputs.shape[1] != d.d_in:
        raise ValueError(f"inputs must be a CUDA float32 tensor [B, {d.d_in}]")
    inputs = inputs.contiguous()
    B = inputs.shape[0]
    if out is None:
        out = torch.empty((B, d.m), dtype=torch.float32, device=inputs.device)
    _check_tensor("out", out, torch.float32, (B, d.m))
    L.check(L.lib().sl7_eval_H(H.handle, _prec(prec), _ptr(inputs), B, _ptr(out), _stream(stream)))
    return out


def labels(model: int, m: int, feats: torch.Tensor, n_paths: int = 10_000, substeps: int = 100,
           seed: int = 7, label0: int = 0, out: torch.Tensor | None = None, stream=None):
    """Euler-Maruyama quantile labels for feats [n, d_in] (CUDA float32)."""
    feats = feats.contiguous()
    n = feats.shape[0]
    _check_tensor("feats", feats, torch.float32, (n, 2 + (2 if int(model) == L.GBM else 3)))
    if out is None:
        out = torch.empty((n, m), dtype=torch.float32, device=feats.device)
    _check_tensor("out", out, torch.float32, (n, int(m)))
    L.check(L.lib().sl7_labels(int(model), int(m), _ptr(feats), n, int(n_paths), int(substeps),
                               int(seed), int(label0), _ptr(out), _stream(stream)))
    return out


def train(H: Mlp, X: torch.Tensor, Y: torch.Tensor, epochs: int, batch: int = 1024,
          lr: float = 1e-3, order: torch.Tensor | None = None, betas=(0.9, 0.999),
          eps: float = 1e-8, stream=None) -> np.ndarray:
    """Adam training of H in place on the GPU; returns the minibatch losses."""
    X = X.contiguous()
    Y = Y.contiguous()
    n = X.shape[0]
    d = H.desc()
    _check_tensor("X", X, torch.float32, (n, d.d_in))
    _check_tensor("Y", Y, torch.float32, (n, d.m))
    spec = L.TrainSpec()
    spec.epochs, spec.batch, spec.lr = int(epochs), int(batch), float(lr)
    spec.beta1, spec.beta2, spec.eps = float(betas[0]), float(betas[1]), float(eps)
    hist = np.zeros(int(epochs) * (n // int(batch)))
    if order is not None:
        order = order.to(device=X.device, dtype=torch.int32).contiguous().reshape(-1)
        _check_tensor("order", order, torch.int32, (int(epochs) * n,))
    L.check(L.lib().sl7_train(H.handle, ctypes.byref(spec), _ptr(X), _ptr(Y), n, _ptr(order),
                              hist.ctypes.data, _stream(stream)))
    return hist


def train_grad(H: Mlp, X: torch.Tensor, Y: torch.Tensor, stream=None):
    """Loss and its gradient over all rows of (X, Y): (loss, grad [n_params])."""
    X = X.contiguous()
    Y = Y.contiguous()
    d = H.desc()
    _check_tensor("X", X, torch.float32, (X.shape[0], d.d_in))
    _check_tensor("Y", Y, torch.float32, (X.shape[0], d.m))
    g = torch.empty(H.n_params(), dtype=torch.float32, device=X.device)
    loss = ctypes.c_double()
    L.check(L.lib().sl7_train_grad(H.handle, _ptr(X), _ptr(Y), X.shape[0], _ptr(g),
                                   ctypes.byref(loss), _stream(stream)))
    return loss.value, g


def adjoint(pr: Problem, H: Mlp | None = None, prec="f64", seed: int = 42, payoff: int = 1,
            ckpt_every: int = 4, per_path: bool = False, stream=None):
    """Pathwise Greeks by the reverse sweep (sl7_adjoint).  Returns a dict
    with value, value_se, grad [dE/dY0, dE/dtheta...], grad_se and, when
    per_path, a [N, 2 + n_theta] float64 tensor of (f, df/dY0, df/dtheta)."""
    p = _prec(prec)
    cp = pr.c()
    nbytes = L.lib().sl7_adjoint_ws_bytes(ctypes.byref(cp), p, int(ckpt_every))
    if nbytes == 0:
        L.check(L.SL7_EINVAL)
    ws = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
    nth = 2 if pr.model == L.GBM else 3
    pp = torch.empty((int(pr.N), 2 + nth), dtype=torch.float64, device="cuda") if per_path else None
    g = L.Greeks()
    L.check(L.lib().sl7_adjoint(ctypes.byref(cp), H.handle if H is not None else None, p,
                                int(seed), int(payoff), int(ckpt_every), ctypes.byref(g), _ptr(pp),
                                _ptr(ws), int(nbytes), _stream(stream)))
    out = {"value": g.value, "value_se": g.value_se,
           "grad": [g.grad[k] for k in range(g.n_grad)],
           "grad_se": [g.grad_se[k] for k in range(g.n_grad)]}
    return (out, pp) if per_path else out


class SL7Adjoint(torch.autograd.Function):
    """E[f(Y_T)] as a differentiable function of (Y0, theta): forward runs the
    adjoint sweep once (value and pathwise Greeks); backward scales the stored
    Greeks by the incoming gradient.  The value and the gradients take the
    device and dtype of Y0 and theta.

        value = SL7Adjoint.apply(Y0, theta, problem, H, prec, seed, payoff, ckpt)
    """

    @staticmethod
    def forward(ctx, Y0, theta, problem: Problem, H, prec="f64", seed=42, payoff=1, ckpt=4):
        pr = Problem(problem.model, tuple(float(v) for v in theta.detach().cpu().tolist()),
                     float(Y0.detach().cpu()), problem.T, problem.M, problem.m, problem.N,
                     problem.K, problem.path_offset, problem.instance)
        g = adjoint(pr, H, prec=prec, seed=seed, payoff=payoff, ckpt_every=ckpt)
        ctx.save_for_backward(torch.tensor(g["grad"], dtype=torch.float64))
        ctx.meta = (Y0.device, Y0.dtype, theta.device, theta.dtype)
        return torch.tensor(g["value"], dtype=Y0.dtype, device=Y0.device)

    @staticmethod
    def backward(ctx, gout):
        (grad,) = ctx.saved_tensors
        dev0, dt0, devt, dtt = ctx.meta
        gout = gout.detach().to(torch.float64).cpu()
        g_y0 = (gout * grad[0]).to(device=dev0, dtype=dt0)
        g_th = (gout * grad[1:]).to(device=devt, dtype=dtt)
        return g_y0, g_th, None, None, None, None, None, None


class SL7TrainLoss(torch.autograd.Function):
    """The training loss of H (mean squared error over all rows of the labels,
    Algorithm I step 1) as a differentiable function of H's flat parameter
    vector: forward and backward run on the GPU through sl7_train_grad (the
    trainer's MFMA forward and backward kernels).  Forward loads `params`
    into H; the gradient returned has the device and dtype of `params`.

        loss = SL7TrainLoss.apply(params, H, X, Y)
    """

    @staticmethod
    def forward(ctx, params, H, X, Y):
        H.set_params(params.detach().to(torch.float32).cpu().numpy())
        loss, g = train_grad(H, X, Y)
        ctx.save_for_backward(g)
        ctx.meta = (params.device, params.dtype)
        return torch.tensor(loss, dtype=params.dtype, device=params.device)

    @staticmethod
    def backward(ctx, gout):
        (g,) = ctx.saved_tensors
        dev, dt = ctx.meta
        return (g.to(device=dev, dtype=dt) * gout.to(device=dev, dtype=dt)), None, None, None
