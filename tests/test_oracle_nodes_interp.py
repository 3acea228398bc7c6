"""Pins for the oracle's collocation nodes and barycentric interpolation.

Gauss-Hermite nodes of N(0,1) (Methodology section) are pinned by their
closed forms, by numpy's independent hermegauss routine and by the
quadrature's moment exactness; the barycentric interpolant (Parallelization
section, ref. [8]) by exact reproduction of polynomials of degree < m and by
the Lagrange remainder bound for the GBM collocation map.
"""
import math

import numpy as np
import pytest
from numpy.polynomial.hermite_e import hermegauss


def test_nodes_closed_forms(orc):
    x, w = orc.gh_nodes(2)
    assert np.array_equal(x, [-1.0, 1.0]) or np.allclose(x, [-1, 1], atol=1e-15, rtol=0)
    assert np.allclose(w, [0.5, 0.5], atol=1e-15)
    x, w = orc.gh_nodes(3)
    assert x[1] == 0.0
    assert np.allclose(x, [-math.sqrt(3), 0, math.sqrt(3)], rtol=1e-15, atol=1e-15)
    assert np.allclose(w, [1 / 6, 2 / 3, 1 / 6], rtol=1e-14)
    x, w = orc.gh_nodes(5)
    a, b = math.sqrt(5 - math.sqrt(10)), math.sqrt(5 + math.sqrt(10))
    assert x[2] == 0.0
    assert np.allclose(x, [-b, -a, 0, a, b], rtol=1e-14, atol=1e-15)
    assert np.allclose(x[3:], [1.355626179974266, 2.856970013872806], rtol=1e-14)
    assert np.allclose(w[:3], [0.011257411327721, 0.222075922005613, 0.533333333333334],
                       rtol=1e-12)
    x, _ = orc.gh_nodes(7)
    assert np.allclose(x[4:], [1.154405394739968, 2.366759410734541, 3.750439717725742],
                       rtol=1e-14)


@pytest.mark.parametrize("m", range(1, 11))
def test_nodes_vs_numpy_hermegauss(orc, m):
    x, w = orc.gh_nodes(m)
    xr, wr = hermegauss(m)
    assert np.allclose(x, xr, rtol=1e-13, atol=1e-14)
    assert np.allclose(w, wr / math.sqrt(2 * math.pi), rtol=1e-12, atol=1e-16)
    assert np.all(np.diff(x) > 0)
    assert np.allclose(x, -x[::-1], rtol=0, atol=0)


@pytest.mark.parametrize("m", [2, 3, 4, 5, 6, 7, 8])
def test_quadrature_moments(orc, m):
    """sum_j w_j x_j^k equals E[X^k] for k <= 2m-1: 0 for odd k and
    (k-1)!! for even k."""
    x, w = orc.gh_nodes(m)
    for k in range(2 * m):
        exact = 0.0 if k % 2 else float(np.prod(np.arange(k - 1, 0, -2))) if k else 1.0
        assert abs(np.sum(w * x ** k) - exact) <= 1e-12 * max(1.0, exact)


def test_bary_weights_closed_forms(orc):
    assert np.allclose(orc.bary_weights(orc.gh_nodes(2)[0]), [-0.5, 0.5], rtol=1e-15)
    assert np.allclose(orc.bary_weights(orc.gh_nodes(3)[0]), [1 / 6, -1 / 3, 1 / 6], rtol=1e-14)
    lam5 = orc.bary_weights(orc.gh_nodes(5)[0])
    assert abs(lam5[2] - 1.0 / 15.0) < 1e-15
    assert np.allclose(lam5, lam5[::-1], rtol=1e-14)


@pytest.mark.parametrize("m", [2, 3, 4, 5, 6, 7, 8])
def test_interpolant_reproduces_low_degree_polynomials(orc, m):
    x, _ = orc.gh_nodes(m)
    lam = orc.bary_weights(x)
    rng = np.random.default_rng(m)
    for deg in range(m):
        c = rng.normal(size=deg + 1)
        y = np.polyval(c, x)
        for X in [-7.3, -x[-1] - 0.5, -0.91, 0.0137, 0.5 * x[-1], x[-1] + 1.25, 6.1]:
            if np.any(X == x):
                continue
            got = orc.bary(x, lam, y, X)
            ref = np.polyval(c, X)
            # the second form's forward error grows with the Lebesgue
            # function Lambda(X) = sum_j |l_j(X)| (Higham, 2004)
            leb = sum(abs(np.prod([(X - x[k]) / (x[j] - x[k]) for k in range(m) if k != j]))
                      for j in range(m))
            scale = leb * max(np.max(np.abs(y)), abs(ref)) + 1.0
            assert abs(got - ref) <= (3 * m + 4) * 2.3e-16 * scale, (m, deg, X, got, ref)


@pytest.mark.parametrize("m", [3, 5, 7])
def test_interpolant_node_hits_are_exact(orc, m):
    x, _ = orc.gh_nodes(m)
    lam = orc.bary_weights(x)
    y = np.random.default_rng(0).normal(size=m)
    for j in range(m):
        assert orc.bary(x, lam, y, x[j]) == y[j]
    # X = 0 is the middle node for odd m: no division by zero
    assert orc.bary(x, lam, y, 0.0) == y[m // 2]
    # the basis sums to one just off a node
    assert abs(orc.bary(x, lam, np.ones(m), x[0] + 1e-300) - 1.0) < 1e-15


def test_gbm_map_within_lagrange_bound(orc):
    """|g_m(X) - Y e^{a+bX}| <= Y e^{a+b max(X, x_max)} b^m/m! prod|X - x_j|."""
    m = 5
    x, _ = orc.gh_nodes(m)
    lam = orc.bary_weights(x)
    sig, mu, dt, Y = 0.3, 0.1, 0.25, 1.3
    a, b = (mu - 0.5 * sig * sig) * dt, sig * math.sqrt(dt)
    y = Y * np.exp(a + b * x)
    for X in np.linspace(-4.5, 4.5, 181):
        if np.any(X == x):
            continue
        err = abs(orc.bary(x, lam, y, X) - Y * math.exp(a + b * X))
        bound = Y * math.exp(a + b * max(X, x[-1])) * b ** m / math.factorial(m) * np.prod(np.abs(X - x))
        assert err <= bound * (1 + 1e-9) + 1e-15
