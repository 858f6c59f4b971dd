"""Pins of the oracle's B-spline layer against facts the paper and mathematics fix.

Paper: Section 2.3 (open knots, Cox-de Boor eq. (5), Proposition 3), Section 2.4
(Table 1: 1D discretisation errors), Section 2 (prolongation P, R = P^T).
"""
import math
import os

import numpy as np
import pytest

from oracle import bspline

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("n_el", [1, 3, 8])
def test_proposition3_properties(p, n_el):
    """Partition of unity, non-negativity and local support (Proposition 3)."""
    t = bspline.open_uniform_knots(n_el, p)
    x = np.concatenate([np.random.default_rng(1).uniform(0, 1, 200), [0.0, 1.0], t])
    N = bspline.cox_de_boor(t, p, x)
    assert N.shape[1] == n_el + p
    np.testing.assert_allclose(N.sum(axis=1), 1.0, atol=1e-14)
    assert (N >= -1e-15).all()
    for j in range(N.shape[1]):
        outside = (x < t[j]) | (x > t[j + p + 1])
        assert np.all(N[outside, j] == 0.0)
    # at most p+1 functions are nonzero at any point (second item of Prop. 3)
    assert ((N > 0).sum(axis=1) <= p + 1).all()


def test_hat_functions_p1():
    """Degree 1 on a uniform grid gives the piecewise-linear hat functions."""
    n_el = 5
    t = bspline.open_uniform_knots(n_el, 1)
    x = np.linspace(0, 1, 101)
    N = bspline.cox_de_boor(t, 1, x)
    for j in range(n_el + 1):
        hat = np.maximum(0.0, 1.0 - np.abs(x * n_el - j))
        np.testing.assert_allclose(N[:, j], hat, atol=1e-14)


@pytest.mark.parametrize("p", [1, 2, 3, 5, 7])
def test_single_element_is_bernstein(p):
    """Knots (0^{p+1}, 1^{p+1}) give the Bernstein polynomials and their derivatives."""
    t = bspline.open_uniform_knots(1, p)
    x = np.linspace(0, 1, 37)
    N = bspline.cox_de_boor(t, p, x)
    D = bspline.cox_de_boor_derivative(t, p, x)
    for k in range(p + 1):
        B = math.comb(p, k) * x ** k * (1 - x) ** (p - k)
        dB = math.comb(p, k) * (k * x ** max(k - 1, 0) * (1 - x) ** (p - k) * (k > 0) -
                                (p - k) * x ** k * (1 - x) ** max(p - k - 1, 0) * (k < p))
        np.testing.assert_allclose(N[:, k], B, atol=1e-13)
        np.testing.assert_allclose(D[:, k], dB, atol=1e-11)


@pytest.mark.parametrize("p", [2, 3, 4])
def test_derivative_central_difference(p):
    t = bspline.open_uniform_knots(6, p)
    x = np.random.default_rng(2).uniform(0.01, 0.99, 50)
    h = 1e-6
    fd = (bspline.cox_de_boor(t, p, x + h) - bspline.cox_de_boor(t, p, x - h)) / (2 * h)
    np.testing.assert_allclose(bspline.cox_de_boor_derivative(t, p, x), fd, atol=2e-6)


def _cardinal_bspline(order, x, deriv=0):
    """Cardinal B-spline of the given order (support [0, order]) by the
    truncated-power formula M(x) = 1/(k-1)! sum_j (-1)^j C(k, j) (x - j)_+^{k-1}."""
    k = order
    tot = 0.0
    for j in range(k + 1):
        y = x - j
        if y <= 0:
            continue
        e = k - 1 - deriv
        coef = math.factorial(k - 1) / math.factorial(e) if e >= 0 else 0.0
        tot += (-1) ** j * math.comb(k, j) * coef * y ** e
    return tot / math.factorial(k - 1)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_interior_mass_stiffness_rows_are_cardinal_values(p):
    """Away from the boundary, M1/h and K1*h are samples of the cardinal B-spline
    of degree 2p+1 (and minus its second derivative) at the integer shifts."""
    n_el = 20
    K, M = bspline.stiffness_mass_1d(n_el, p)
    h = 1.0 / n_el
    i = n_el // 2
    for d in range(-p, p + 1):
        m_ref = _cardinal_bspline(2 * p + 2, p + 1 + d)
        k_ref = -_cardinal_bspline(2 * p + 2, p + 1 + d, deriv=2)
        assert abs(M[i, i + d] / h - m_ref) < 1e-13
        assert abs(K[i, i + d] * h - k_ref) < 1e-12
    # explicit values for p = 2
    if p == 2:
        np.testing.assert_allclose(M[i, i - 2:i + 3] / h, np.array([1, 26, 66, 26, 1]) / 120,
                                   atol=1e-14)
        np.testing.assert_allclose(K[i, i - 2:i + 3] * h, [-1 / 6, -1 / 3, 1, -1 / 3, -1 / 6],
                                   atol=1e-13)


@pytest.mark.parametrize("p", [1, 2, 3, 5])
def test_mass_stiffness_spd(p):
    K, M = bspline.stiffness_mass_1d(9, p)
    for A in (K, M):
        np.testing.assert_allclose(A, A.T, atol=1e-14)
        assert np.linalg.eigvalsh(A).min() > 0


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_prolongation_interior_columns_binomial(p):
    """Midpoint knot insertion: interior columns of P1 are 2^-p C(p+1, k)."""
    nc = 16
    P = bspline.prolongation_1d(nc, p, interior=False)
    J = nc // 2 + 1
    col = P[:, J]
    nz = np.nonzero(np.abs(col) > 1e-14)[0]
    ref = np.array([math.comb(p + 1, k) for k in range(p + 2)]) / 2 ** p
    np.testing.assert_allclose(col[nz], ref, atol=1e-14)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_prolongation_partition_and_function_identity(p):
    nc = 8
    P = bspline.prolongation_1d(nc, p, interior=False)
    np.testing.assert_allclose(P.sum(axis=1), 1.0, atol=1e-14)   # partition of unity
    assert (P >= -1e-15).all()
    rng = np.random.default_rng(p)
    c = rng.standard_normal(nc + p)
    x = rng.uniform(0, 1, 100)
    tc = bspline.open_uniform_knots(nc, p)
    tf = bspline.open_uniform_knots(2 * nc, p)
    np.testing.assert_allclose(bspline.cox_de_boor(tc, p, x) @ c,
                               bspline.cox_de_boor(tf, p, x) @ (P @ c), atol=1e-13)
    # interior block: boundary fine rows carry no interior coarse entries
    assert np.all(P[0, 1:-1] == 0) and np.all(P[-1, 1:-1] == 0)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_galerkin_1d_equals_direct_coarse_assembly(p):
    """On nested spaces P1^T K_h P1 = K_2h and likewise for M (eq. (4))."""
    Kf, Mf = bspline.stiffness_mass_1d(16, p)
    Kc, Mc = bspline.stiffness_mass_1d(8, p)
    P = bspline.prolongation_1d(8, p)
    np.testing.assert_allclose(P.T @ Kf @ P, Kc, atol=1e-12 * np.abs(Kc).max())
    np.testing.assert_allclose(P.T @ Mf @ P, Mc, atol=1e-14)
