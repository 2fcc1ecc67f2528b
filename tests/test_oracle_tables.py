"""Pins for the oracle's node and basis tables (Sec. 3, eqs. gaussquad, 3.4, 3.5)."""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import tables


@pytest.mark.parametrize("n", list(range(1, 33)))
def test_gl_nodes_match_numpy_leggauss(n):
    # numpy computes the same roots by a different route (companion eigenvalues + Newton)
    x, w = np.polynomial.legendre.leggauss(n)
    ref_nodes = (x + 1.0) / 2.0
    ours = np.asarray(tables.nodes(n, "gl"))
    assert np.all(np.diff(ours) > 0)
    assert np.all((ours > 0) & (ours < 1))
    np.testing.assert_allclose(ours, ref_nodes, rtol=0, atol=1.5e-15)
    np.testing.assert_allclose(np.asarray(tables.weights(n, "gl")), w / 2.0, rtol=1e-12, atol=0)


@pytest.mark.parametrize("n", [2, 3, 5, 8, 12, 16, 24])
def test_gl_quadrature_exact_to_degree_2n_minus_1(n):
    xi = np.asarray(tables.nodes(n))
    w = np.asarray(tables.weights(n))
    assert abs(w.sum() - 1.0) < 1e-15
    for k in range(2 * n):
        assert abs(np.dot(w, xi ** k) - 1.0 / (k + 1)) < 2e-15, k
    # and not exact at degree 2n (Gauss rules are exact to 2n-1 only; visible for small n)
    if n <= 5:
        assert abs(np.dot(w, xi ** (2 * n)) - 1.0 / (2 * n + 1)) > 1e-8


@pytest.mark.parametrize("n", [2, 3, 4, 7, 10])
def test_cg_nodes_closed_form(n):
    ours = np.asarray(tables.nodes(n, "cg"))
    ref = np.array([(1 - math.cos((2 * i + 1) * math.pi / (2 * n))) / 2 for i in range(n)])
    np.testing.assert_allclose(ours, ref, rtol=0, atol=4.5e-16)
    w = np.asarray(tables.weights(n, "cg"))
    for k in range(n):
        assert abs(np.dot(w, ours ** k) - 1.0 / (k + 1)) < 1e-13


@pytest.mark.parametrize("n", [2, 4, 8, 13])
def test_legendre_basis_orthonormal_under_gl(n):
    xi = np.asarray(tables.nodes(n))
    w = np.asarray(tables.weights(n))
    psi = tables.legendre_basis(xi, n)
    np.testing.assert_allclose(psi.T @ (w[:, None] * psi), np.eye(n), atol=1e-13)


def test_legendre_basis_small_closed_forms():
    t = np.linspace(-0.5, 1.5, 9)
    psi = tables.legendre_basis(t, 4)
    x = 2 * t - 1
    np.testing.assert_allclose(psi[:, 0], 1.0)
    np.testing.assert_allclose(psi[:, 1], math.sqrt(3) * x, rtol=1e-15)
    np.testing.assert_allclose(psi[:, 2], math.sqrt(5) * (3 * x * x - 1) / 2, rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(psi[:, 3], math.sqrt(7) * (5 * x ** 3 - 3 * x) / 2, rtol=1e-14, atol=1e-14)


def test_gl_nodes_correctly_rounded_small_n():
    # exact roots for n = 2, 3: xi = (1 -+ 1/sqrt(3))/2 and (1 - sqrt(3/5))/2, 1/2, ...
    def cr(fr_hi):
        return float(fr_hi)
    import mpmath
    with mpmath.workdps(60):
        r2 = [(1 - 1 / mpmath.sqrt(3)) / 2, (1 + 1 / mpmath.sqrt(3)) / 2]
        r3 = [(1 - mpmath.sqrt(mpmath.mpf(3) / 5)) / 2, mpmath.mpf(1) / 2, (1 + mpmath.sqrt(mpmath.mpf(3) / 5)) / 2]
        assert list(tables.nodes(2)) == [float(v) for v in r2]
        assert list(tables.nodes(3)) == [float(v) for v in r3]
    assert Fraction(tables.nodes(3)[1]) == Fraction(1, 2)
