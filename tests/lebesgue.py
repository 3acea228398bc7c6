"""The Lebesgue function of the step's interpolant and the FP32 per-path
bound that follows from it.

An FP32 network output error e in the collocation points y_j moves the
interpolant at X by at most Lambda_m(X) e, Lambda_m(X) = sum_j |l_j(X)| over
the Lagrange basis l_j on the m Gauss-Hermite nodes.  Inside the nodes
Lambda_m is a few units; beyond the outer node it grows like |X|^(m-1).
The FP32 tolerance 1e-5 holds while every normal of a path stays within
|X| <= 4; a path that draws a larger |X| is held to 1e-5 scaled by
Lambda_m at that draw over Lambda_m(4)."""
import numpy as np

import oracle

F32_TOL = 1e-5
X_REF = 4.0


def lebesgue(m: int, X) -> np.ndarray:
    x, _ = oracle.gh_nodes(m)
    X = np.asarray(X, dtype=np.float64)
    tot = np.zeros_like(X)
    for j in range(m):
        p = np.ones_like(X)
        for k in range(m):
            if k != j:
                p = p * (X - x[k]) / (x[j] - x[k])
        tot += np.abs(p)
    return tot


def f32_bound(m: int, xmax) -> np.ndarray:
    """Per-path FP32 bound for paths whose largest |X| over the steps is xmax."""
    xmax = np.asarray(xmax, dtype=np.float64)
    scale = np.where(xmax > X_REF, lebesgue(m, xmax) / lebesgue(m, X_REF), 1.0)
    return F32_TOL * np.maximum(scale, 1.0)


def lebesgue_nodes(nodes, Y) -> np.ndarray:
    """Lambda over arbitrary distinct nodes (e.g. a step's marginal points)."""
    nodes = np.asarray(nodes, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    tot = np.zeros_like(Y)
    for j in range(len(nodes)):
        p = np.ones_like(Y)
        for k in range(len(nodes)):
            if k != j:
                p = p * (Y - nodes[k]) / (nodes[j] - nodes[k])
        tot += np.abs(p)
    return tot


def inside_max(nodes) -> float:
    """Largest Lambda between the outer nodes (sampled finely)."""
    nodes = np.sort(np.asarray(nodes, dtype=np.float64))
    return float(lebesgue_nodes(nodes, np.linspace(nodes[0], nodes[-1], 4001)).max())
