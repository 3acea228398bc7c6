"""Networks derived from the stored ones for tests (test support, no tests).

Built and written with the oracle's own reader and writer; both sides then
read the file, so no input passes through the library."""
import os

import numpy as np

import oracle

GBM_WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                           "gbm_mlp_4x64.sl7w")


def network_with_m_outputs(S, m2, path, src=GBM_WEIGHTS):
    """The stored GBM network with its head re-interpolated onto the m2
    Gauss-Hermite nodes: head row k becomes sum_j l_j(x'_k) row_j (Lagrange
    basis on the stored network's nodes), so the outputs stay
    collocation-point shaped.  Returns (library handle, oracle network)."""
    Ho = oracle.load_mlp(src)
    x0, _ = oracle.gh_nodes(Ho.m)
    x2, _ = oracle.gh_nodes(m2)
    Lm = np.array([[np.prod([(xk - x0[i]) / (x0[j] - x0[i]) for i in range(Ho.m) if i != j])
                    for j in range(Ho.m)] for xk in x2])
    W = [np.array(w) for w in Ho.W]
    b = [np.array(v) for v in Ho.b]
    W[-1] = (Lm @ W[-1]).astype(np.float32).astype(np.float64)
    b[-1] = (Lm @ b[-1]).astype(np.float32).astype(np.float64)
    H2o = oracle.Mlp(Ho.d_in, Ho.width, Ho.depth, m2, Ho.act, Ho.model, Ho.in_scale, Ho.in_shift,
                     Ho.dom_lo, Ho.dom_hi, W, b, dict(Ho.meta))
    oracle.save_mlp(H2o, path)
    return S.Mlp.load(path), oracle.load_mlp(path)
