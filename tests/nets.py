"""Networks derived from the stored ones for tests (test support, no tests)."""
import numpy as np

import oracle


def network_with_m_outputs(S, H, m2, path):
    """The stored GBM network with its head re-interpolated onto the m2
    Gauss-Hermite nodes: head row k becomes sum_j l_j(x'_k) row_j (Lagrange
    basis on the 5 nodes), so the outputs stay collocation-point shaped."""
    d = H.desc()
    x5, _ = oracle.gh_nodes(d.m)
    x2, _ = oracle.gh_nodes(m2)
    Lm = np.array([[np.prod([(xk - x5[i]) / (x5[j] - x5[i]) for i in range(d.m) if i != j])
                    for j in range(d.m)] for xk in x2])
    p = H.params().astype(np.float64)
    nb, nw = d.m, d.m * d.width
    Wh, bh = p[-nb - nw:-nb].reshape(d.m, d.width), p[-nb:]
    p2 = np.concatenate([p[:-nb - nw], (Lm @ Wh).ravel(), Lm @ bh]).astype(np.float32)
    H2 = S.Mlp.create(d.d_in, m2, d.model, p2, list(d.in_scale)[:d.d_in], list(d.in_shift)[:d.d_in],
                      list(d.dom_lo)[:d.d_in], list(d.dom_hi)[:d.d_in], width=d.width)
    H2.save(path)
    return H2, oracle.load_mlp(path)
