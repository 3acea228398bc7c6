"""FP64 CPU oracle for the Seven-League (7L) online stage.

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only ``tests/``, the smoke check in
``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may import this
package.  It shares no code with the GPU library (``paper_2302_05170_amd``)
and never imports it; the two meet only through the seeded input generators
in ``workloads`` and through weight files, which both sides parse with their
own readers.

What it computes (arXiv 2302.05170):
  * Gauss-Hermite collocation nodes x_j of N(0,1) (Methodology section),
    by Golub-Welsch on the Jacobi matrix of the probabilists' Hermite
    polynomials;
  * barycentric weights and the barycentric interpolant g_m (Parallelization
    section, the paper's ref. [8]);
  * the 7L step Y_{i+1} = g_m(X_{i+1}) with collocation points from the
    network H (eq. 6.3/6.4) or from an analytic transition law, looped over
    the M large steps of Algorithm I (online stage);
  * Euler-Maruyama (eq. 6.2) for the offline labels and as the large-step
    baseline;
  * the network's forward and backward passes and an Adam step for the
    offline training stage (Algorithm I step 1, Numerical Results);
  * forward-mode tangents of Y_T for pathwise sensitivities.
The per-path loops live in ``sl7_oracle.c`` (plain C, double precision, one
path at a time); this module adds the node computation, the batched network
maths used for training checks, the estimators, the weight-file reader and a
thread pool over independent paths.

Parity status: every routine here is pinned by closed forms, library routines,
published values or invariants in ``tests/test_oracle_*.py``; the Philox
generator by the known-answer vectors published with its reference
implementation (``tests/golden/philox4x32_10_kat.txt``).
"""
from __future__ import annotations

import ctypes
import json
import math
import os
import struct
import subprocess
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sl7_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libsl7oracle.so")

GBM, OU, CIR = 0, 1, 2
N_THETA = {GBM: 2, OU: 3, CIR: 3}
SIMULATE_DOMAIN = 0
LABEL_DOMAIN = 1


def build(verbose: bool = False) -> str:
    """Compiles the C part of the oracle with gcc (no fast-math, no FMA
    contraction, so the arithmetic is the plain IEEE sequence written)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-o", _LIB_PATH + ".tmp", _SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        _lib = _declare(ctypes.CDLL(_LIB_PATH))
    return _lib


class _Mlp(ctypes.Structure):
    _fields_ = [("d_in", ctypes.c_int32), ("width", ctypes.c_int32),
                ("depth", ctypes.c_int32), ("m", ctypes.c_int32),
                ("act", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("in_scale", ctypes.c_void_p), ("in_shift", ctypes.c_void_p),
                ("W", ctypes.c_void_p * 9), ("b", ctypes.c_void_p * 9)]


class _Problem(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int32), ("m", ctypes.c_int32),
                ("M", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("theta", ctypes.c_double * 4), ("Y0", ctypes.c_double),
                ("T", ctypes.c_double), ("tag", ctypes.c_uint32),
                ("pad2_", ctypes.c_int32), ("dom_lo", ctypes.c_double),
                ("dom_hi", ctypes.c_double)]


_P = ctypes.c_void_p


def _declare(L):
    L.orc_philox4x32.argtypes = [_P, _P, ctypes.c_int, _P]
    L.orc_normals4.argtypes = [ctypes.c_uint64] + [ctypes.c_uint32] * 4 + [_P]
    L.orc_step_normal.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int64, ctypes.c_int]
    L.orc_step_normal.restype = ctypes.c_double
    L.orc_step_normals.argtypes = [ctypes.c_uint64, ctypes.c_uint32, _P, ctypes.c_int64,
                                   ctypes.c_int, _P]
    L.orc_Phi.argtypes = [ctypes.c_double]
    L.orc_Phi.restype = ctypes.c_double
    L.orc_bary.argtypes = [ctypes.c_int, _P, _P, _P, ctypes.c_double]
    L.orc_bary.restype = ctypes.c_double
    L.orc_mlp_forward.argtypes = [_P, _P, _P]
    L.orc_simulate.argtypes = [_P, _P, _P, _P, ctypes.c_uint64, _P, ctypes.c_int64, _P, _P]
    L.orc_simulate_tangent.argtypes = [_P, _P, _P, _P, ctypes.c_uint64, _P, ctypes.c_int64, _P, _P]
    L.orc_cdc_tables.argtypes = [_P, _P, _P, _P, _P, _P, _P]
    L.orc_cdc_tables.restype = ctypes.c_int
    L.orc_cdc_collocation.argtypes = [ctypes.c_int, ctypes.c_int, _P, _P, _P, ctypes.c_double, _P]
    L.orc_simulate_cdc.argtypes = [_P, _P, _P, _P, _P, _P, ctypes.c_uint64, _P, ctypes.c_int64,
                                   _P, _P]
    L.orc_em_paths.argtypes = [ctypes.c_int, _P, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                               ctypes.c_uint64, ctypes.c_uint32, _P, ctypes.c_int64, _P]
    L.orc_em_label.argtypes = [ctypes.c_int, _P, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                               ctypes.c_int, ctypes.c_int, _P, ctypes.c_uint64, ctypes.c_uint32,
                               ctypes.c_uint32, _P]
    L.orc_em_label.restype = ctypes.c_int
    L.orc_type7_quantiles.argtypes = [_P, ctypes.c_int, ctypes.c_int, _P, _P]
    L.orc_gammainc_lower.argtypes = [ctypes.c_double, ctypes.c_double]
    L.orc_gammainc_lower.restype = ctypes.c_double
    L.orc_ncx2_cdf.argtypes = [ctypes.c_double] * 3
    L.orc_ncx2_cdf.restype = ctypes.c_double
    L.orc_ncx2_ppf.argtypes = [ctypes.c_double] * 3
    L.orc_ncx2_ppf.restype = ctypes.c_double
    return L


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def n_threads() -> int:
    return int(os.environ.get("SL7_ORACLE_THREADS", os.cpu_count() or 1))


# ---------------------------------------------------------------------------
# Collocation nodes (Methodology section: x_j from N(0,1), Gauss-Hermite).
# ---------------------------------------------------------------------------
def gh_nodes(m: int):
    """Probabilists' Gauss-Hermite nodes and weights (weights sum to 1).

    Golub-Welsch: the three-term recurrence He_{k+1} = x He_k - k He_{k-1}
    gives a symmetric Jacobi matrix with zero diagonal and off-diagonal
    sqrt(k), k = 1..m-1.  Its eigenvalues are the nodes and the squared first
    components of its unit eigenvectors are the weights.  The result is
    symmetrised about 0 (the middle node is exactly 0 for odd m)."""
    if m < 1:
        raise ValueError("m must be >= 1")
    J = np.zeros((m, m))
    for k in range(1, m):
        J[k - 1, k] = J[k, k - 1] = math.sqrt(k)
    vals, vecs = np.linalg.eigh(J)
    order = np.argsort(vals)
    x = vals[order]
    w = vecs[0, order] ** 2
    x = 0.5 * (x - x[::-1])
    w = 0.5 * (w + w[::-1])
    if m % 2 == 1:
        x[m // 2] = 0.0
    return x, w / w.sum()


def bary_weights(x: np.ndarray) -> np.ndarray:
    """lambda_j = 1 / prod_{k != j} (x_j - x_k)."""
    m = len(x)
    lam = np.empty(m)
    for j in range(m):
        p = 1.0
        for k in range(m):
            if k != j:
                p *= x[j] - x[k]
        lam[j] = 1.0 / p
    return lam


def bary(x, lam, y, X: float) -> float:
    x = np.ascontiguousarray(x, dtype=np.float64)
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    return lib().orc_bary(len(x), _ptr(x), _ptr(lam), _ptr(y), float(X))


def Phi(x: float) -> float:
    return lib().orc_Phi(float(x))


# ---------------------------------------------------------------------------
# Random numbers: Philox4x32-10 + Box-Muller (project convention).
# ---------------------------------------------------------------------------
def philox4x32(ctr, key, rounds: int = 10) -> np.ndarray:
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32(_ptr(c), _ptr(k), rounds, _ptr(out))
    return out


def normals4(seed: int, c0: int, c1: int, c2: int, c3: int) -> np.ndarray:
    out = np.zeros(4)
    lib().orc_normals4(seed, c0, c1, c2, c3, _ptr(out))
    return out


def make_tag(domain: int, instance: int) -> int:
    return ((domain & 0xFF) << 24) | (instance & 0xFFFFFF)


def step_normals(seed: int, tag: int, paths, M: int, threads: int | None = None) -> np.ndarray:
    """X[c, i]: the normal driving large step i of global path paths[c]."""
    paths = np.ascontiguousarray(paths, dtype=np.int64)
    out = np.empty((len(paths), M))

    def run(rng):
        a, b = rng
        lib().orc_step_normals(seed, tag, _ptr(paths[a:b]), b - a, M, _ptr(out[a:b]))

    nt = threads or n_threads()
    with ThreadPoolExecutor(nt) as ex:
        list(ex.map(run, _chunks(paths, nt)))
    return out


# ---------------------------------------------------------------------------
# The network H and its weight file.
# ---------------------------------------------------------------------------
ACT_RELU, ACT_SOFTPLUS = 0, 1
_MAGIC = b"SL7W"


@dataclass
class Mlp:
    """Collocation network H: (Y, dt, theta) -> (y_0..y_{m-1}).

    h0 = in_scale * input + in_shift; h_l = act(W_l h_{l-1} + b_l) for the
    hidden layers; y = W_out h_depth + b_out.  Values are the stored FP32
    numbers widened exactly to FP64."""
    d_in: int
    width: int
    depth: int
    m: int
    act: int
    model: int
    in_scale: np.ndarray
    in_shift: np.ndarray
    dom_lo: np.ndarray
    dom_hi: np.ndarray
    W: list
    b: list
    meta: dict = field(default_factory=dict)

    def layer_shapes(self):
        shapes, n_in = [], self.d_in
        for l in range(self.depth + 1):
            n_out = self.m if l == self.depth else self.width
            shapes.append((n_out, n_in))
            n_in = n_out
        return shapes

    def n_params(self) -> int:
        return sum(o * i + o for o, i in self.layer_shapes())

    def params_f32(self) -> np.ndarray:
        parts = []
        for W, b in zip(self.W, self.b):
            parts += [np.asarray(W, np.float32).ravel(), np.asarray(b, np.float32).ravel()]
        return np.concatenate(parts)

    def with_params(self, flat) -> "Mlp":
        flat = np.asarray(flat, dtype=np.float64)
        W, b, off = [], [], 0
        for o, i in self.layer_shapes():
            W.append(flat[off:off + o * i].reshape(o, i).copy()); off += o * i
            b.append(flat[off:off + o].copy()); off += o
        assert off == len(flat)
        return Mlp(self.d_in, self.width, self.depth, self.m, self.act, self.model,
                   self.in_scale, self.in_shift, self.dom_lo, self.dom_hi, W, b, dict(self.meta))

    def _struct(self):
        keep = [np.ascontiguousarray(self.in_scale, np.float64),
                np.ascontiguousarray(self.in_shift, np.float64)]
        s = _Mlp()
        s.d_in, s.width, s.depth, s.m, s.act = self.d_in, self.width, self.depth, self.m, self.act
        s.in_scale, s.in_shift = keep[0].ctypes.data, keep[1].ctypes.data
        for l in range(self.depth + 1):
            Wl = np.ascontiguousarray(self.W[l], np.float64)
            bl = np.ascontiguousarray(self.b[l], np.float64)
            keep += [Wl, bl]
            s.W[l], s.b[l] = Wl.ctypes.data, bl.ctypes.data
        return s, keep

    def forward(self, inputs: np.ndarray) -> np.ndarray:
        """Per-row forward pass through the C routine (one input at a time)."""
        inputs = np.ascontiguousarray(inputs, np.float64)
        s, keep = self._struct()
        out = np.empty((inputs.shape[0], self.m))
        row_out = np.empty(self.m)
        for r in range(inputs.shape[0]):
            row = np.ascontiguousarray(inputs[r])
            lib().orc_mlp_forward(ctypes.byref(s), _ptr(row), _ptr(row_out))
            out[r] = row_out
        return out


def save_mlp(H: Mlp, path: str) -> None:
    """Writes the shared little-endian weight file: magic 'SL7W', u32 version
    1, u32 (d_in, width, depth, m, act, model), f64 in_scale/in_shift/
    dom_lo/dom_hi [d_in each], then per layer W (out x in row-major) and b as
    f32, then u32 meta length and UTF-8 JSON metadata."""
    with open(path, "wb") as f:
        f.write(_MAGIC)
        f.write(struct.pack("<7I", 1, H.d_in, H.width, H.depth, H.m, H.act, H.model))
        for arr in (H.in_scale, H.in_shift, H.dom_lo, H.dom_hi):
            f.write(np.asarray(arr, "<f8").tobytes())
        for W, b in zip(H.W, H.b):
            f.write(np.asarray(W, "<f4").tobytes())
            f.write(np.asarray(b, "<f4").tobytes())
        meta = json.dumps(H.meta, sort_keys=True).encode()
        f.write(struct.pack("<I", len(meta)))
        f.write(meta)


def load_mlp(path: str) -> Mlp:
    with open(path, "rb") as f:
        data = f.read()
    if data[:4] != _MAGIC:
        raise ValueError(f"{path}: not a weight file")
    ver, d_in, width, depth, m, act, model = struct.unpack_from("<7I", data, 4)
    if ver != 1:
        raise ValueError(f"{path}: unsupported version {ver}")
    off = 4 + 28
    vecs = []
    for _ in range(4):
        vecs.append(np.frombuffer(data, "<f8", d_in, off).astype(np.float64)); off += 8 * d_in
    H = Mlp(d_in, width, depth, m, act, model, *vecs, W=[], b=[])
    for o, i in H.layer_shapes():
        H.W.append(np.frombuffer(data, "<f4", o * i, off).astype(np.float64).reshape(o, i)); off += 4 * o * i
        H.b.append(np.frombuffer(data, "<f4", o, off).astype(np.float64)); off += 4 * o
    (n_meta,) = struct.unpack_from("<I", data, off); off += 4
    H.meta = json.loads(data[off:off + n_meta].decode()) if n_meta else {}
    return H


def glorot_mlp(d_in, width, depth, m, model, in_lo, in_hi, flat_params, act=ACT_RELU) -> Mlp:
    """Network with the input affine mapping [in_lo, in_hi] to [-1, 1] and the
    given flat parameter vector (rounded to FP32 as the file stores it)."""
    in_lo = np.asarray(in_lo, np.float64); in_hi = np.asarray(in_hi, np.float64)
    scale = 2.0 / (in_hi - in_lo)
    shift = -(in_hi + in_lo) / (in_hi - in_lo)
    H = Mlp(d_in, width, depth, m, act, model, scale, shift, in_lo.copy(), in_hi.copy(), [], [])
    return H.with_params(np.asarray(flat_params, np.float32).astype(np.float64))


# ---------------------------------------------------------------------------
# The online stage (Algorithm I), per path.
# ---------------------------------------------------------------------------
@dataclass
class Problem:
    model: int
    theta: tuple
    Y0: float
    T: float
    M: int
    m: int
    instance: int = 0


def _problem_struct(pr: Problem, H: Mlp | None):
    s = _Problem()
    s.model, s.m, s.M = pr.model, pr.m, pr.M
    for k, v in enumerate(pr.theta):
        s.theta[k] = float(v)
    s.Y0, s.T = float(pr.Y0), float(pr.T)
    s.tag = make_tag(SIMULATE_DOMAIN, pr.instance)
    if H is not None:
        s.dom_lo, s.dom_hi = float(H.dom_lo[0]), float(H.dom_hi[0])
    else:
        s.dom_lo, s.dom_hi = -np.inf, np.inf
    return s


def _chunks(paths: np.ndarray, nt: int):
    nt = max(1, min(nt, len(paths)))
    bounds = np.linspace(0, len(paths), nt + 1).astype(np.int64)
    return [(int(bounds[k]), int(bounds[k + 1])) for k in range(nt) if bounds[k + 1] > bounds[k]]


def simulate(pr: Problem, H: Mlp | None, seed: int, paths, threads: int | None = None):
    """Y_T for the listed global paths.  H=None selects the analytic map.
    Returns (YT, n_clamped, n_out_of_domain)."""
    paths = np.ascontiguousarray(paths, dtype=np.int64)
    x, _ = gh_nodes(pr.m)
    lam = bary_weights(x)
    ps = _problem_struct(pr, H)
    hs, keep = (H._struct() if H is not None else (None, None))
    YT = np.empty(len(paths))
    counts = []

    def run(rng):
        a, b = rng
        cnt = np.zeros(2, dtype=np.int64)
        lib().orc_simulate(ctypes.byref(ps), ctypes.byref(hs) if hs is not None else None,
                           _ptr(x), _ptr(lam), seed, _ptr(paths[a:b]), b - a,
                           _ptr(YT[a:b]), _ptr(cnt))
        return cnt

    with ThreadPoolExecutor(threads or n_threads()) as ex:
        for cnt in ex.map(run, _chunks(paths, threads or n_threads())):
            counts.append(cnt)
    tot = np.sum(counts, axis=0) if counts else np.zeros(2, np.int64)
    return YT, int(tot[0]), int(tot[1])


def simulate_tangent(pr: Problem, H: Mlp | None, seed: int, paths, threads: int | None = None):
    """(YT, dYT) with dYT[c, p] = dY_T/d(Y0, theta_0, ...)[p] by forward mode."""
    paths = np.ascontiguousarray(paths, dtype=np.int64)
    x, _ = gh_nodes(pr.m)
    lam = bary_weights(x)
    ps = _problem_struct(pr, H)
    hs, keep = (H._struct() if H is not None else (None, None))
    npar = 1 + N_THETA[pr.model]
    YT = np.empty(len(paths))
    dYT = np.empty((len(paths), npar))

    def run(rng):
        a, b = rng
        lib().orc_simulate_tangent(ctypes.byref(ps), ctypes.byref(hs) if hs is not None else None,
                                   _ptr(x), _ptr(lam), seed, _ptr(paths[a:b]), b - a,
                                   _ptr(YT[a:b]), _ptr(dYT[a:b]))

    with ThreadPoolExecutor(threads or n_threads()) as ex:
        list(ex.map(run, _chunks(paths, threads or n_threads())))
    return YT, dYT


def cdc_tables(pr: Problem, H: Mlp | None):
    """Per-step tables of the 7L-CDC variant: marginal points s [M, m], their
    barycentric weights [M, m] and the conditional points at them ykj
    [M, m, m] (row 0: the conditional points at Y0 in k = 0).  Also returns
    the count of network inputs outside the training domain."""
    x, _ = gh_nodes(pr.m)
    ps = _problem_struct(pr, H)
    hs, keep = (H._struct() if H is not None else (None, None))
    s = np.zeros((pr.M, pr.m))
    lams = np.zeros((pr.M, pr.m))
    ykj = np.zeros((pr.M, pr.m, pr.m))
    cnt = np.zeros(2, dtype=np.int64)
    rc = lib().orc_cdc_tables(ctypes.byref(ps), ctypes.byref(hs) if hs is not None else None,
                              _ptr(x), _ptr(s), _ptr(lams), _ptr(ykj), _ptr(cnt))
    if rc != 0:
        raise ValueError(f"7L-CDC: marginal collocation points of step {-1 - rc} are not distinct")
    return s, lams, ykj, int(cnt[1])


def cdc_collocation(tables, i: int, Y: float) -> np.ndarray:
    """Conditional collocation points of a path at Y in step i (the global
    interpolation)."""
    s, lams, ykj = (np.ascontiguousarray(t, np.float64) for t in tables[:3])
    m = s.shape[1]
    out = np.zeros(m)
    lib().orc_cdc_collocation(m, i, _ptr(s), _ptr(lams), _ptr(ykj), float(Y), _ptr(out))
    return out


def simulate_cdc(pr: Problem, H: Mlp | None, seed: int, paths, threads: int | None = None):
    """Y_T of the listed global paths under the 7L-CDC variant.  Returns
    (YT, n_clamped, n_out_of_domain of the table evaluations)."""
    paths = np.ascontiguousarray(paths, dtype=np.int64)
    x, _ = gh_nodes(pr.m)
    lam = bary_weights(x)
    s, lams, ykj, nood = cdc_tables(pr, H)
    ps = _problem_struct(pr, H)
    YT = np.empty(len(paths))
    counts = []

    def run(rng):
        a, b = rng
        cnt = np.zeros(2, dtype=np.int64)
        lib().orc_simulate_cdc(ctypes.byref(ps), _ptr(x), _ptr(lam), _ptr(s), _ptr(lams),
                               _ptr(ykj), seed, _ptr(paths[a:b]), b - a, _ptr(YT[a:b]),
                               _ptr(cnt))
        return cnt

    with ThreadPoolExecutor(threads or n_threads()) as ex:
        for cnt in ex.map(run, _chunks(paths, threads or n_threads())):
            counts.append(cnt)
    tot = np.sum(counts, axis=0) if counts else np.zeros(2, np.int64)
    return YT, int(tot[0]), nood


def em_paths(pr: Problem, seed: int, paths) -> np.ndarray:
    """Large-step Euler-Maruyama (eq. 6.2) with the same normals as 7L."""
    paths = np.ascontiguousarray(paths, dtype=np.int64)
    th = np.ascontiguousarray(pr.theta, np.float64)
    YT = np.empty(len(paths))
    lib().orc_em_paths(pr.model, _ptr(th), pr.Y0, pr.T, pr.M, seed,
                       make_tag(SIMULATE_DOMAIN, pr.instance), _ptr(paths), len(paths), _ptr(YT))
    return YT


def em_labels(model: int, features: np.ndarray, m: int, n_paths: int, substeps: int,
              seed: int, first_label: int = 0, threads: int | None = None) -> np.ndarray:
    """Offline labels (Algorithm I step 1): features[r] = (Y, dt, theta...);
    label r is computed with Philox counter word 2 = first_label + r."""
    features = np.ascontiguousarray(features, np.float64)
    x, _ = gh_nodes(m)
    out = np.empty((features.shape[0], m))
    tag = make_tag(LABEL_DOMAIN, 0)

    def run(rng):
        a, b = rng
        for r in range(a, b):
            th = np.ascontiguousarray(features[r, 2:])
            row = np.empty(m)
            rc = lib().orc_em_label(model, _ptr(th), features[r, 0], features[r, 1], n_paths,
                                    substeps, m, _ptr(x), seed, first_label + r, tag, _ptr(row))
            if rc != 0:
                raise MemoryError("orc_em_label")
            out[r] = row

    idx = np.arange(features.shape[0])
    with ThreadPoolExecutor(threads or n_threads()) as ex:
        list(ex.map(run, _chunks(idx, 4 * (threads or n_threads()))))
    return out


def ncx2_cdf(x, k, nc):
    return lib().orc_ncx2_cdf(float(x), float(k), float(nc))


def ncx2_ppf(p, k, nc):
    return lib().orc_ncx2_ppf(float(p), float(k), float(nc))


def gammainc_lower(a, z):
    return lib().orc_gammainc_lower(float(a), float(z))


# ---------------------------------------------------------------------------
# Estimators.
# ---------------------------------------------------------------------------
def neumaier_sum(v) -> float:
    s, c = 0.0, 0.0
    for t in np.asarray(v, np.float64).tolist():
        u = s + t
        if abs(s) >= abs(t):
            c += (s - u) + t
        else:
            c += (t - u) + s
        s = u
    return s + c


def payoffs(YT, K: float):
    YT = np.asarray(YT, np.float64)
    return YT, np.maximum(YT - K, 0.0)


def estimate(f) -> dict:
    """Mean (compensated, path order), variance (two-pass, N-1), SE."""
    f = np.asarray(f, np.float64)
    n = len(f)
    mean = neumaier_sum(f) / n
    var = neumaier_sum((f - mean) ** 2) / (n - 1) if n > 1 else 0.0
    return {"mean": mean, "var": var, "se": math.sqrt(var / n), "n": n}


# ---------------------------------------------------------------------------
# Offline training maths (Numerical Results: Glorot init, Adam, batch 1024,
# learning rate 1e-3; loss: mean squared error over batch and outputs).
# ---------------------------------------------------------------------------
def _act(act, z):
    if act == ACT_RELU:
        return np.maximum(z, 0.0)
    return np.where(z > 0, z + np.log1p(np.exp(-np.abs(z))), np.log1p(np.exp(np.minimum(z, 0.0))))


def _act_deriv(act, z):
    if act == ACT_RELU:
        return (z > 0).astype(np.float64)
    return 1.0 / (1.0 + np.exp(-z))


def mlp_forward_batch(H: Mlp, inputs: np.ndarray):
    """Returns (y, cache) for a batch of raw inputs [B, d_in]."""
    h = inputs * H.in_scale + H.in_shift
    hs, zs = [h], []
    for l in range(H.depth + 1):
        z = h @ H.W[l].T + H.b[l]
        zs.append(z)
        h = z if l == H.depth else _act(H.act, z)
        hs.append(h)
    return h, (hs, zs)


def mse_loss_and_grads(H: Mlp, inputs: np.ndarray, labels: np.ndarray):
    """Loss = mean over batch and outputs of (y - label)^2 and its gradient
    with respect to every W_l and b_l, by reverse-mode differentiation."""
    y, (hs, zs) = mlp_forward_batch(H, inputs)
    B, m = labels.shape
    r = y - labels
    loss = float(np.sum(r * r) / (B * m))
    g = 2.0 * r / (B * m)
    dW, db = [None] * (H.depth + 1), [None] * (H.depth + 1)
    for l in range(H.depth, -1, -1):
        if l < H.depth:
            g = g * _act_deriv(H.act, zs[l])
        dW[l] = g.T @ hs[l]
        db[l] = g.sum(axis=0)
        g = g @ H.W[l]
    return loss, dW, db


def flatten(W, b) -> np.ndarray:
    parts = []
    for Wl, bl in zip(W, b):
        parts += [np.ravel(Wl), np.ravel(bl)]
    return np.concatenate(parts)


@dataclass
class AdamState:
    m: np.ndarray
    v: np.ndarray
    t: int = 0


def adam_step(params: np.ndarray, grad: np.ndarray, st: AdamState, lr=1e-3,
              b1=0.9, b2=0.999, eps=1e-8) -> np.ndarray:
    st.t += 1
    st.m = b1 * st.m + (1 - b1) * grad
    st.v = b2 * st.v + (1 - b2) * grad * grad
    mhat = st.m / (1 - b1 ** st.t)
    vhat = st.v / (1 - b2 ** st.t)
    return params - lr * mhat / (np.sqrt(vhat) + eps)


def train(H: Mlp, features: np.ndarray, labels: np.ndarray, order: np.ndarray,
          batch: int = 1024, lr: float = 1e-3, log_every: int = 0):
    """Plain Adam over the given minibatch order (rows of ``order`` are
    epochs, each a permutation of the label indices).  Returns the trained
    network and the per-step loss history."""
    p = flatten(H.W, H.b)
    st = AdamState(np.zeros_like(p), np.zeros_like(p))
    hist = []
    for ep in range(order.shape[0]):
        perm = order[ep]
        for s in range(0, len(perm) - batch + 1, batch):
            idx = perm[s:s + batch]
            cur = H.with_params(p)
            loss, dW, db = mse_loss_and_grads(cur, features[idx], labels[idx])
            p = adam_step(p, flatten(dW, db), st, lr=lr)
            hist.append(loss)
        if log_every and (ep + 1) % log_every == 0:
            print(f"epoch {ep + 1}: loss {np.mean(hist[-(len(perm) // batch):]):.4e}", flush=True)
    return H.with_params(p), np.asarray(hist)
