"""Pins of the oracle's 1D reference data (Sec. 2: Lagrange basis on GLL
points; Sec. 2.1: 1D mass/stiffness matrices and face evaluators)."""
import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

from oracle import basis1d


def test_closed_forms_k1_k2():
    M, K = basis1d.mass_stiffness(1)
    np.testing.assert_allclose(M, [[1 / 3, 1 / 6], [1 / 6, 1 / 3]], atol=1e-15)
    np.testing.assert_allclose(K, [[1, -1], [-1, 1]], atol=1e-14)
    M, K = basis1d.mass_stiffness(2)
    np.testing.assert_allclose(M, np.array([[4, 2, -1], [2, 16, 2], [-1, 2, 4]]) / 30, atol=1e-15)
    np.testing.assert_allclose(K, np.array([[7, -8, 1], [-8, 16, -8], [1, -8, 7]]) / 3, atol=1e-13)


def test_gll_nodes_closed_form():
    np.testing.assert_allclose(basis1d.gll_nodes(1), [0, 1])
    np.testing.assert_allclose(basis1d.gll_nodes(2), [0, 0.5, 1], atol=1e-15)
    s = 1 / (2 * np.sqrt(5))
    np.testing.assert_allclose(basis1d.gll_nodes(3), [0, 0.5 - s, 0.5 + s, 1], atol=1e-15)
    # k = 4: interior nodes 1/2 and 1/2 -+ sqrt(3/7)/2
    r = np.sqrt(3 / 7) / 2
    np.testing.assert_allclose(basis1d.gll_nodes(4), [0, 0.5 - r, 0.5, 0.5 + r, 1], atol=1e-15)


@pytest.mark.parametrize("k", range(1, 8))
def test_partition_of_unity_and_cardinality(k):
    x = basis1d.gll_nodes(k)
    np.testing.assert_allclose(basis1d.lagrange_values(x, x), np.eye(k + 1), atol=1e-13)
    t = np.random.default_rng(k).uniform(0, 1, 17)
    np.testing.assert_allclose(basis1d.lagrange_values(x, t).sum(1), 1.0, atol=1e-12)
    np.testing.assert_allclose(basis1d.lagrange_derivs(x, t).sum(1), 0.0, atol=1e-10)


@pytest.mark.parametrize("k", range(1, 8))
def test_derivative_reproduces_polynomials(k):
    """phi' applied to nodal values of t^m gives m t^(m-1) for m <= k."""
    x = basis1d.gll_nodes(k)
    t = np.random.default_rng(10 + k).uniform(0, 1, 9)
    D = basis1d.lagrange_derivs(x, t)
    for m in range(k + 1):
        exact = m * t ** (m - 1) if m > 0 else 0 * t
        np.testing.assert_allclose(D @ x ** m, exact, atol=1e-10)


@pytest.mark.parametrize("n", range(1, 10))
def test_gauss_rule_exactness(n):
    x, w = basis1d.gauss_rule(n)
    for m in range(2 * n):
        assert abs(np.sum(w * x ** m) - 1.0 / (m + 1)) < 1e-14


@pytest.mark.parametrize("k", range(1, 8))
def test_mass_row_sums_are_gll_weights(k):
    """sum_b Mhat_ab = int phi_a = GLL weight 1/(k(k+1) P_k(t_a)^2) on
    [0, 1] (half of the classical weight on [-1, 1])."""
    M, K = basis1d.mass_stiffness(k)
    t = 2 * basis1d.gll_nodes(k) - 1
    c = np.zeros(k + 1)
    c[k] = 1
    w = 1.0 / (k * (k + 1) * npleg.legval(t, c) ** 2)
    np.testing.assert_allclose(M.sum(1), w, rtol=1e-12)
    # stiffness annihilates constants and maps x to phi(1) - phi(0)
    x = basis1d.gll_nodes(k)
    s0, s1, d0, d1 = basis1d.end_vectors(k)
    np.testing.assert_allclose(K @ np.ones(k + 1), 0, atol=1e-11)
    np.testing.assert_allclose(K @ x, s1 - s0, atol=1e-11)
    assert np.all(np.linalg.eigvalsh(M) > 0)
    np.testing.assert_allclose(M, M.T, atol=1e-15)
    np.testing.assert_allclose(K, K.T, atol=1e-12)


@pytest.mark.parametrize("k", range(1, 8))
def test_end_vectors(k):
    s0, s1, d0, d1 = basis1d.end_vectors(k)
    e = np.eye(k + 1)
    np.testing.assert_allclose(s0, e[0], atol=1e-13)
    np.testing.assert_allclose(s1, e[k], atol=1e-13)
    x = basis1d.gll_nodes(k)
    if k >= 2:
        assert abs(d0 @ x ** 2) < 1e-10 and abs(d1 @ x ** 2 - 2.0) < 1e-10
    assert abs(d0 @ x - 1) < 1e-11 and abs(d1 @ x - 1) < 1e-11
