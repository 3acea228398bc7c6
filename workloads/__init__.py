"""Seeded synthetic inputs for the Seven-League workloads.

This module is shared by the GPU library's tests and benchmark and by the
oracle's tests.  It holds no arithmetic of the method itself: only parameter
sets, uniform draws of training features, initial network weights, minibatch
orders and path subsets, all from numpy's seeded generator.  The normals that
drive the paths are not drawn here; each side derives them from its own
counter-based generator.

Workloads (synthetic; the paper uses no public dataset):
  gbm_analytic_1e5x4   GBM, analytic collocation map, FP64: mu 0.1,
                       sigma 0.3, Y0 1, T 1, M 4, m 5, N 1e5, seed 42.
  gbm_mlp_2p22x16      GBM, MLP map (4 inputs, 4x64 ReLU, 5 outputs), FP32:
                       sigma 0.3, mu 0.1, Y0 1, T 1, M 16, N 2^22, seed 42.
  gbm_mlp_2p24x32      same network, GEMMs in BF16 / FP16: sigma 0.4,
                       mu 0.05, T 2, M 32, N 2^24.
  gbm_adjoint_2p22x16  adjoint of E[max(Y_T - 1, 0)] in the 2^22 x 16
                       setting, checkpoint every 4.
  cir_instances(256)   256 CIR instances of uneven size (kappa, ybar, gamma,
                       Y0, dt, M, N drawn from seed 11), MLP with 5 inputs and
                       7 outputs, BF16.
"""
from __future__ import annotations

import numpy as np

GBM, OU, CIR = 0, 1, 2

# GBM parameter vector order is (sigma, mu): the network's input order is
# (Y, dt, sigma, mu).  OU: (ybar, sigma, lambda).  CIR: (kappa, ybar, gamma).
CONFIGS = {
    "gbm_analytic_1e5x4": dict(model=GBM, theta=(0.3, 0.1), Y0=1.0, T=1.0, M=4, m=5, N=100_000,
               seed=42, K=1.0),
    "gbm_mlp_2p22x16": dict(model=GBM, theta=(0.3, 0.1), Y0=1.0, T=1.0, M=16, m=5, N=2 ** 22,
               seed=42, K=1.0),
    "gbm_mlp_2p24x32": dict(model=GBM, theta=(0.4, 0.05), Y0=1.0, T=2.0, M=32, m=5, N=2 ** 24,
               seed=42, K=1.0),
    "gbm_adjoint_2p22x16": dict(model=GBM, theta=(0.3, 0.1), Y0=1.0, T=1.0, M=16, m=5, N=2 ** 22,
               seed=42, K=1.0, ckpt=4),
}

# Training domain of the GBM network, feature order (Y, dt, sigma, mu).
GBM_DOMAIN_LO = np.array([0.5, 0.05, 0.1, 0.0])
GBM_DOMAIN_HI = np.array([1.5, 0.5, 0.5, 0.2])
# Training domain of the OU network (the paper's experiment, eq. 6.5), feature
# order (Y, dt, ybar, sigma, lambda).
OU_DOMAIN_LO = np.array([-1.0, 0.05, 0.0, 0.1, 0.5])
OU_DOMAIN_HI = np.array([2.0, 0.5, 1.0, 0.5, 2.5])
# The paper's network for OU: 4 hidden layers of 50 Softplus units.
OU_WIDTH = 50
# Training domain of the CIR network, feature order (Y, dt, kappa, ybar, gamma).
CIR_DOMAIN_LO = np.array([0.0, 0.1, 0.5, 0.02, 0.1])
CIR_DOMAIN_HI = np.array([1.3, 1.0, 3.0, 0.1, 0.5])

WIDTH, DEPTH = 64, 4
TRAIN_SEED = 7
N_LABELS = 2 ** 16
LABEL_PATHS = 10_000
LABEL_SUBSTEPS = 100
BATCH = 1024


def layer_shapes(d_in: int, m: int, width: int = WIDTH, depth: int = DEPTH):
    shapes, n_in = [], d_in
    for l in range(depth + 1):
        n_out = m if l == depth else width
        shapes.append((n_out, n_in))
        n_in = n_out
    return shapes


def glorot_params(d_in: int, m: int, seed: int = TRAIN_SEED, width: int = WIDTH,
                  depth: int = DEPTH) -> np.ndarray:
    """Glorot-uniform weights U(+-sqrt(6/(fan_in+fan_out))), zero biases,
    flattened as [W_0, b_0, W_1, b_1, ...] (W row-major out x in), FP32."""
    rng = np.random.default_rng(seed)
    parts = []
    for o, i in layer_shapes(d_in, m, width, depth):
        lim = np.sqrt(6.0 / (i + o))
        parts.append(rng.uniform(-lim, lim, size=(o, i)).astype(np.float32).ravel())
        parts.append(np.zeros(o, np.float32))
    return np.concatenate(parts)


def gbm_features(n: int = N_LABELS, seed: int = TRAIN_SEED) -> np.ndarray:
    """Rows (Y, dt, sigma, mu) uniform over the GBM training domain."""
    rng = np.random.default_rng(seed + 1000)
    return rng.uniform(GBM_DOMAIN_LO, GBM_DOMAIN_HI, size=(n, 4))


def ou_features(n: int = N_LABELS, seed: int = TRAIN_SEED) -> np.ndarray:
    """Rows (Y, dt, ybar, sigma, lambda) uniform over the OU training domain."""
    rng = np.random.default_rng(seed + 4000)
    return rng.uniform(OU_DOMAIN_LO, OU_DOMAIN_HI, size=(n, 5))


# The paper's OU experiment (Table 6.1) does not state T, M, theta or Y0;
# these are chosen here, with the paper's path counts.
OU_PAPER = dict(model=OU, theta=(0.5, 0.3, 1.0), Y0=0.2, T=2.0, M=8, m=5, seed=42, K=0.5,
                path_counts=(1_000, 50_000, 100_000, 200_000))


def cir_features(n: int = N_LABELS, seed: int = TRAIN_SEED) -> np.ndarray:
    """Rows (Y, dt, kappa, ybar, gamma) uniform over the CIR training domain."""
    rng = np.random.default_rng(seed + 2000)
    return rng.uniform(CIR_DOMAIN_LO, CIR_DOMAIN_HI, size=(n, 5))


def minibatch_order(n: int, epochs: int, seed: int = TRAIN_SEED) -> np.ndarray:
    """One permutation of range(n) per epoch, int32 [epochs, n]."""
    rng = np.random.default_rng(seed + 3000)
    return np.stack([rng.permutation(n) for _ in range(epochs)]).astype(np.int32)


def parity_subset(N: int) -> np.ndarray:
    """Paths compared one by one at full size: the first and last 2^15 and a
    strided 2^16 (all paths when N <= 2^17)."""
    if N <= 2 ** 17:
        return np.arange(N, dtype=np.int64)
    first = np.arange(2 ** 15, dtype=np.int64)
    last = np.arange(N - 2 ** 15, N, dtype=np.int64)
    strided = np.arange(0, N, N // 2 ** 16, dtype=np.int64)[: 2 ** 16]
    return np.unique(np.concatenate([first, strided, last]))


def cir_instances(n: int = 256, seed: int = 11) -> list:
    """Uneven CIR instances: kappa~U[0.5,3], ybar~U[0.02,0.1], gamma~U[0.1,0.5],
    Y0~U[0.01,0.1], dt~U[0.1,1], M~U{4..32}, N log-uniform in [2^12, 2^18];
    drawn in that order per instance.  T = M * dt."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        kap = rng.uniform(0.5, 3.0)
        ybar = rng.uniform(0.02, 0.1)
        gam = rng.uniform(0.1, 0.5)
        y0 = rng.uniform(0.01, 0.1)
        dt = rng.uniform(0.1, 1.0)
        M = int(rng.integers(4, 33))
        N = int(round(2.0 ** rng.uniform(12.0, 18.0)))
        out.append(dict(model=CIR, theta=(kap, ybar, gam), Y0=y0, T=M * dt, M=M, m=7,
                        N=N, instance=k))
    return out
