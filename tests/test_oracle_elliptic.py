"""Pins of the oracle's full elliptic operator (Section 4.3) and its geometry.

The bilinear form a(u, v) = int A grad u . grad v + (B . grad u) v + c u v with
the two coefficient sets of Section 4.3; the quarter annulus with exact
(rational) arcs for the manufactured solution of the second problem.
"""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import assemble, bspline, elliptic as el, multigrid as mg


def test_laplace_set_equals_independent_assemblies():
    """A = I, B = 0, c = 0 reproduces the C element-scatter assembly on the
    annulus and the Kronecker form K1 (x) M1 + M1 (x) K1 on the square."""
    for p in (2, 3):
        A1 = el.assemble(6, p, "annulus", el.CSET_LAPLACE, 1.0, 2.0)
        A2 = assemble.mapped_stiffness_2d(6, p)
        assert abs(A1 - A2).max() < 1e-14 * abs(A2).max()
        A3 = el.assemble(6, p, "square", el.CSET_LAPLACE)
        A4 = assemble.kron_operator_2d(6, p)
        assert abs(A3 - A4).max() < 1e-14 * abs(A4).max()


@pytest.mark.parametrize("p", [1, 2, 3])
def test_divergence_free_convection_is_skew_on_the_square(p):
    """B = (-5y, 5x) has zero divergence and the interior functions vanish on
    the boundary, so int (B . grad phi_J) phi_I = -int (B . grad phi_I) phi_J;
    on the square the Gauss rule integrates these polynomials exactly."""
    C = el.assemble(6, p, "square", el.CSET_ANNULUS, terms=("convection",)).toarray()
    assert abs(C + C.T).max() < 1e-13 * abs(C).max()
    assert abs(C).max() > 1e-3


@pytest.mark.parametrize("p", [1, 2, 3])
def test_advection_diffusion_parts(p):
    """A = 0.1 I, B = (1, 1): the diffusion part is 0.1 times the Laplace
    assembly, the constant convection is exactly skew-symmetric."""
    D = el.assemble(6, p, "square", el.CSET_ADVDIFF, terms=("diffusion",))
    assert abs(D - 0.1 * assemble.kron_operator_2d(6, p)).max() < 1e-15
    C = el.assemble(6, p, "square", el.CSET_ADVDIFF, terms=("convection",)).toarray()
    assert abs(C + C.T).max() < 1e-14 * abs(C).max()


@pytest.mark.parametrize("p", [1, 2, 4])
def test_reaction_with_c_one_integrates_the_area(p):
    """c = 1 over all functions: sum_IJ int phi_I phi_J = int 1 = 1 (partition of unity)."""
    M = el.assemble(5, p, "square", el.CSET_SQUARE, interior=False, terms=("reaction",))
    assert abs(M.sum() - 1.0) < 1e-13


def test_variable_diffusion_energy_identities():
    """With u = x and v = y (coefficients: Greville abscissae, all functions),
    u^T K u = int a11, v^T K v = int a22, u^T K v = int a12 over the unit square,
    in closed form: 1.5 (2 + sin 1), 1.5 (3 - cos 1), (2 sin 2 - sin 4) / 8."""
    p, ne = 3, 8
    K = el.assemble(ne, p, "square", el.CSET_SQUARE, interior=False, terms=("diffusion",)).toarray()
    g = bspline.greville(bspline.open_uniform_knots(ne, p), p)
    n = ne + p
    X = np.tile(g, n)            # coefficient of phi_{i + n j} for u = x
    Y = np.repeat(g, n)
    assert abs(X @ K @ X - 1.5 * (2.0 + math.sin(1.0))) < 1e-10
    assert abs(Y @ K @ Y - 1.5 * (3.0 - math.cos(1.0))) < 1e-10
    assert abs(X @ K @ Y - (2.0 * math.sin(2.0) - math.sin(4.0)) / 8.0) < 1e-10
    # rows of the diffusion part annihilate constants (sum_J grad phi_J = 0)
    assert abs(K.sum(axis=1)).max() < 1e-12 * abs(K).max()


def test_exact_annulus_arcs_and_area():
    """The rational surface's arcs lie on the circles r_in and r_out, the side
    eta = 0 on the x axis, eta = 1 on the y axis; its area is pi (R^2 - r^2) / 4."""
    r, R = 0.2, 1.0
    eta = np.linspace(0.0, 1.0, 101)
    for xi, rad in ((0.0, r), (1.0, R)):
        x, y, *_ = el.geometry("annulus_exact", np.full_like(eta, xi), eta, r, R)
        np.testing.assert_allclose(np.hypot(x, y), rad, rtol=1e-15)
    xi = np.linspace(0.0, 1.0, 11)
    x, y, *_ = el.geometry("annulus_exact", xi, np.zeros_like(xi), r, R)
    assert np.all(y == 0.0)
    x, y, *_ = el.geometry("annulus_exact", xi, np.ones_like(xi), r, R)
    assert np.all(np.abs(x) < 1e-16)
    xg, wg = np.polynomial.legendre.leggauss(40)
    xg, wg = (xg + 1) / 2, wg / 2
    XI, ETA = np.meshgrid(xg, xg)
    _, _, j11, j12, j21, j22 = el.geometry("annulus_exact", XI, ETA, r, R)
    area = np.sum(np.outer(wg, wg) * np.abs(j11 * j22 - j12 * j21))
    assert abs(area - math.pi * (R * R - r * r) / 4.0) < 1e-12


def test_manufactured_rhs_matches_finite_differences():
    """The closed-form f equals -div(A grad u) + B . grad u + c u evaluated by
    central differences of u and of the flux A grad u."""
    rng = np.random.default_rng(7)
    x, y = rng.uniform(0.2, 0.7, (2, 25))
    h, H = 1e-4, 1e-3
    u = el.manufactured_u

    def flux(x, y):
        ux = (u(x + h, y) - u(x - h, y)) / (2 * h)
        uy = (u(x, y + h) - u(x, y - h)) / (2 * h)
        a11, a12, a22, *_ = el.coefficients(el.CSET_ANNULUS, x, y)
        return a11 * ux + a12 * uy, a12 * ux + a22 * uy

    div = ((flux(x + H, y)[0] - flux(x - H, y)[0]) + (flux(x, y + H)[1] - flux(x, y - H)[1])) / (2 * H)
    ux = (u(x + h, y) - u(x - h, y)) / (2 * h)
    uy = (u(x, y + h) - u(x, y - h)) / (2 * h)
    f_fd = -div - 5.0 * y * ux + 5.0 * x * uy + x * y * u(x, y)
    f = el.manufactured_f(x, y)
    assert np.max(np.abs(f - f_fd)) < 1e-5 * np.max(np.abs(f))
    # u vanishes on the boundary of the exact annulus
    eta = np.linspace(0, 1, 17)
    for xi in (0.0, 1.0):
        bx, by, *_ = el.geometry("annulus_exact", np.full_like(eta, xi), eta, 0.2, 1.0)
        assert np.max(np.abs(u(bx, by))) < 1e-16


@pytest.mark.parametrize("p", [2, 3])
def test_manufactured_solution_converges_at_order_p_plus_1(p):
    """Galerkin solutions of the second Section 4.3 problem on the exact annulus
    (radii 0.2, 1): the relative L2 error decays like h^(p+1)."""
    errs = []
    for ne in (8, 16, 32):
        A = el.assemble(ne, p, "annulus_exact", el.CSET_ANNULUS, 0.2, 1.0)
        b = el.load(ne, p, "annulus_exact", el.manufactured_f, 0.2, 1.0)
        uh = spla.spsolve(A.tocsc(), b)
        e, r = el.l2_error(ne, p, "annulus_exact", uh, el.manufactured_u, 0.2, 1.0)
        errs.append(e / r)
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert abs(rates[-1] - (p + 1)) < 0.25, rates
    assert errs[-1] < 1e-4


def test_nonsymmetric_hierarchy_uses_lu_and_solves():
    """The coarsest operator of the full elliptic problem is nonsymmetric; its
    direct solve (LU) returns A0^-1 b."""
    H = mg.build_elliptic_hierarchy("square", 16, 2, el.CSET_SQUARE)
    assert not H.symmetric
    A0 = H.levels[0].A.toarray()
    b = np.random.default_rng(1).standard_normal(A0.shape[0])
    x = H.coarse_solve(b)
    assert np.linalg.norm(A0 @ x - b) < 1e-12 * np.linalg.norm(b)
