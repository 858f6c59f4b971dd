"""Pins of the oracle's 2D/3D operators and load vectors.

Paper: Section 2 (A SPD, eq. (2); Galerkin operator eq. (4)); Section 4.2
(2D Poisson, eq. (12)); Section 4.3 (quarter annulus as a B-spline surface);
Section 4.2 (Table 11: 2D discretisation errors).
"""
import math
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from oracle import assemble, bspline, multigrid


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_identity_mapping_equals_kronecker(p):
    """Two independent code paths: element scatter with F = id vs K1(x)M1 + M1(x)K1."""
    n_el = 7
    A1 = assemble.mapped_stiffness_2d(n_el, p, geom=assemble.GEOM_IDENTITY)
    A2 = assemble.kron_operator_2d(n_el, p)
    assert abs(A1 - A2).max() < 1e-14 * abs(A2).max()


def test_annulus_closed_form_is_the_bspline_surface():
    """F(xi, eta) = (1+xi)(1-eta^2, 2eta-eta^2) equals the degree-2 B-spline surface
    with knots (0,0,0,1,1,1)^2 and control net rho_i * {(1,0), (1,1), (0,1)}_j,
    rho = (1, 1.5, 2)."""
    t = bspline.open_uniform_knots(1, 2)
    rng = np.random.default_rng(0)
    xi, eta = rng.uniform(0, 1, 50), rng.uniform(0, 1, 50)
    Bx, By = bspline.cox_de_boor(t, 2, xi), bspline.cox_de_boor(t, 2, eta)
    rho = np.array([1.0, 1.5, 2.0])
    net = np.array([[1.0, 0.0], [1.0, 1.0], [0.0, 1.0]])
    XY = np.einsum("qi,qj,i,jc->qc", Bx, By, rho, net)
    F = np.column_stack([(1 + xi) * (1 - eta ** 2), (1 + xi) * (2 * eta - eta ** 2)])
    np.testing.assert_allclose(XY, F, atol=1e-15)


def _spline_coefficients_of_xy(n_el, p):
    """Tensor B-spline coefficients (all functions, x fastest) of the physical
    coordinates x(xi, eta), y(xi, eta) of the annulus, by 1D interpolation at
    the Greville points (F is biquadratic, so it lies in the space for p >= 2)."""
    t = bspline.open_uniform_knots(n_el, p)
    g = bspline.greville(t, p)
    B = bspline.cox_de_boor(t, p, g)
    Binv = np.linalg.inv(B)
    XI, ETA = np.meshgrid(g, g, indexing="xy")    # [j, i]
    X = (1 + XI) * (1 - ETA ** 2)
    Y = (1 + XI) * (2 * ETA - ETA ** 2)
    cx = Binv @ X @ Binv.T     # rows eta-index j, cols xi-index i
    cy = Binv @ Y @ Binv.T
    return cx.reshape(-1), cy.reshape(-1)


@pytest.mark.parametrize("p", [2, 3, 4])
def test_annulus_energy_identities(p):
    """Exact weak-form identities on the mapped domain:
    int |grad x|^2 = int |grad y|^2 = area = 5/2, int grad x . grad y = 0."""
    n_el = 6
    A = assemble.mapped_stiffness_2d(n_el, p, interior=False)
    cx, cy = _spline_coefficients_of_xy(n_el, p)
    assert abs(cx @ (A @ cx) - 2.5) < 1e-12
    assert abs(cy @ (A @ cy) - 2.5) < 1e-12
    assert abs(cx @ (A @ cy)) < 1e-12


@pytest.mark.parametrize("p", [2, 3, 5])
def test_annulus_stencil_symmetric_positive_definite(p):
    n_el = 8
    st = assemble.mapped_stiffness_2d(n_el, p, as_stencil=True)
    n = n_el + p - 2
    A = assemble.stencil_to_csr(st, n, p)
    assert abs(A - A.T).max() < 1e-14 * abs(A).max()
    ev = np.linalg.eigvalsh(A.toarray())
    assert ev.min() > 0
    np.linalg.cholesky(A.toarray())


def test_annulus_jacobian_bounds():
    """det J = (1+xi)(2 - 2 eta + 2 eta^2) lies in [1.5, 4] on the unit square."""
    xi, eta = np.meshgrid(np.linspace(0, 1, 101), np.linspace(0, 1, 101))
    det = (1 + xi) * (2 - 2 * eta + 2 * eta ** 2)
    assert abs(det.min() - 1.5) < 1e-12 and abs(det.max() - 4.0) < 1e-12


@pytest.mark.parametrize("dim,n_el,p", [(2, 12, 3), (2, 8, 5), (3, 4, 2), (3, 8, 3)])
def test_fast_diagonalisation_equals_sparse_solve(dim, n_el, p):
    """A^{-1} = (V (x) V ..)(Lambda (+) Lambda ..)^{-1}(V (x) V ..)^T from K1 V = M1 V Lambda."""
    from oracle import fastdiag
    N = (n_el + p - 2) ** dim
    b = synth.random_vector(N, 3)
    A = assemble.kron_operator_2d(n_el, p) if dim == 2 else assemble.kron_operator_3d(n_el, p)
    x = spla.spsolve(A.tocsc(), b)
    np.testing.assert_allclose(fastdiag.solve_kronecker(n_el, p, b, dim), x, rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize("p", [2, 3])
def test_2d_discretisation_rate(p):
    """L2 error of the exact discrete solution decays like h^{p+1} (the rate of
    Table 1, observed here in 2D for u = sin(pi x) sin(pi y))."""
    errs = []
    sizes = [8, 16, 32]
    for n_el in sizes:
        A = assemble.kron_operator_2d(n_el, p)
        b = assemble.kron_load_2d(n_el, p, synth.manufactured_sine_modes_2d())
        u = spla.spsolve(A.tocsc(), b)
        n = n_el + p - 2
        U = np.zeros((n + 2, n + 2))
        U[1:-1, 1:-1] = u.reshape(n, n)
        xq, wq, V, _ = bspline.local_basis_tables(n_el, p, p + 1)
        err = 0.0
        for ey in range(n_el):
            for ex in range(n_el):
                c = U[ey:ey + p + 1, ex:ex + p + 1]
                uh = np.einsum("qa,rb,ba->rq", V[ex], V[ey], c)   # [qy, qx]
                ue = np.sin(np.pi * xq[ex])[None, :] * np.sin(np.pi * xq[ey])[:, None]
                err += np.sum(wq[ey][:, None] * wq[ex][None, :] * (uh - ue) ** 2)
        errs.append(math.sqrt(err))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert abs(rates[-1] - (p + 1)) < 0.2, rates


def test_load_vector_3d_matches_2d_structure():
    """3D load of a product f(x,y) g(z) factorises: compare a z-constant mode table
    with the 2D load times the 1D integral of the z factor."""
    n_el, p = 4, 2
    modes3 = np.array([[1.0, 1.0, 2.0, 0.0, 0.3]])
    b3 = assemble.load_vector_3d(n_el, p, modes3)
    b2 = assemble.kron_load_2d(n_el, p, np.array([[1.0, 1.0, 2.0, 0.3]]))
    xq, wq, V, _ = bspline.local_basis_tables(n_el, p, p + 1)
    mz = np.zeros(n_el + p)
    for e in range(n_el):
        mz[e:e + p + 1] += V[e].T @ wq[e]
    ref = (mz[1:-1][:, None] * b2[None, :]).reshape(-1)
    np.testing.assert_allclose(b3, ref, atol=1e-14)


@pytest.mark.parametrize("dim,n_el,p", [(2, 16, 2), (2, 16, 3), (3, 8, 2)])
def test_colouring_has_no_same_colour_coupling(dim, n_el, p):
    geom = "square" if dim == 2 else "cube"
    H = multigrid.build_hierarchy(geom, n_el, p)
    for lev in H.levels:
        col = multigrid.colours(lev.n, p, dim)
        A = lev.A.tocoo()
        off = A.row != A.col
        assert not np.any(col[A.row[off]] == col[A.col[off]])


def test_galerkin_square_equals_rediscretisation():
    """On the unit square the Galerkin coarse operator equals direct assembly."""
    H = multigrid.build_hierarchy("square", 16, 3)
    Ac = assemble.kron_operator_2d(8, 3)
    assert abs(H.levels[-2].A - Ac).max() < 1e-12 * abs(Ac).max()


def _l2_error_2d(n_el, p, modes, exact):
    """L2 error of the exact discrete solution (p+3 Gauss points per direction)."""
    A = assemble.kron_operator_2d(n_el, p)
    b = assemble.kron_load_2d(n_el, p, modes)
    u = spla.spsolve(A.tocsc(), b)
    n = n_el + p - 2
    U = np.zeros((n + 2, n + 2))
    U[1:-1, 1:-1] = u.reshape(n, n)
    xq, wq, V, _ = bspline.local_basis_tables(n_el, p, p + 3)
    err = 0.0
    for ey in range(n_el):
        for ex in range(n_el):
            c = U[ey:ey + p + 1, ex:ex + p + 1]
            uh = np.einsum("qa,rb,ba->rq", V[ex], V[ey], c)   # [qy, qx]
            ue = exact(xq[ex][None, :], xq[ey][:, None])
            err += np.sum(wq[ey][:, None] * wq[ex][None, :] * (uh - ue) ** 2)
    return math.sqrt(err)


def test_table11_l2_errors_reproduced():
    """Table 11's L2-err column for the Section 4.2 model problem on 64 x 64
    elements: reproduced to 3 % for p = 3, 4, 5.  For p = 1, 2 the printed
    values are 15-20 % below the exact 2D discrete solution's error (for p = 2..5
    they equal the 1D values of Table 1 at 64 elements, which the 2D error of
    this product solution approaches only as the error shrinks); there the
    error is required to be within 25 % and above the printed value."""
    golden = os.path.join(os.path.dirname(__file__), "golden", "table11_l2err_2d.txt")
    rows = [l.split() for l in open(golden) if l.strip() and not l.startswith("#")]
    exact = lambda x, y: np.sin(2 * np.pi * x) * np.sin(2 * np.pi * y)
    modes = synth.poisson_2d_sine_modes(1)
    for ne, p, v in rows:
        ne, p, v = int(ne), int(p), float(v)
        e = _l2_error_2d(ne, p, modes, exact)
        if p >= 3:
            assert abs(e / v - 1) < 0.03, (p, v, e)
        else:
            assert 1.0 < e / v < 1.25, (p, v, e)


def test_poisson_2d_modes_reproduce_f():
    """The mode table of the Section 4.2 model problem evaluates to
    f = 2 (2 k pi)^2 sin(2 k pi x) sin(2 k pi y)."""
    rng = np.random.default_rng(3)
    x, y = rng.uniform(0, 1, 100), rng.uniform(0, 1, 100)
    for k in (1, 2):
        m = synth.poisson_2d_sine_modes(k)
        f = sum(a * np.sin(np.pi * (kx * x + ky * y) + ph) for a, kx, ky, ph in m)
        ref = 2 * (2 * k * np.pi) ** 2 * np.sin(2 * k * np.pi * x) * np.sin(2 * k * np.pi * y)
        np.testing.assert_allclose(f, ref, atol=1e-12)


# ---- load vector on the quarter annulus -------------------------------------

def _mode_sum(modes):
    m = np.asarray(modes, dtype=np.float64).reshape(-1, 4)

    def f(x, y):
        out = np.zeros_like(np.asarray(x, dtype=np.float64))
        for a, k, l, ph in m:
            out = out + a * np.sin(np.pi * (k * x + l * y) + ph)
        return out
    return f


@pytest.mark.parametrize("p", [2, 3, 4, 5])
def test_annulus_load_equals_independent_numpy_assembly(p):
    """The C element-scatter load vector on the annulus equals the separate
    numpy assembly of the full elliptic oracle (its own geometry evaluation,
    Jacobian, physical point and element loop), for the benchmark's random
    field: b_I = int f(F(xi)) phi_I |det J| (Section 2, eq. (2); Section 4.3)."""
    from oracle import elliptic
    n_el = 12
    modes = synth.random_field_modes(2000 + p)
    b1 = assemble.load_vector_2d(n_el, p, modes)
    b2 = elliptic.load(n_el, p, "annulus", _mode_sum(modes))
    assert np.max(np.abs(b1 - b2)) <= 1e-14 * np.max(np.abs(b2))


@pytest.mark.parametrize("p", [2, 3, 5])
def test_annulus_load_integrates_area_and_moments(p):
    """Partition of unity (Section 2.3, Proposition 3): with every function kept,
    sum_I b_I = int_Omega f.  For f = 1 this is the area of the degree-2 annulus
    surface, |det J| = (1 + xi)(2 - 2 eta + 2 eta^2), whose integral is exactly
    3/2 * 5/3 = 5/2; the Gauss rule integrates it exactly.  For a
    non-constant f evaluated at the physical point, the sum equals an adaptive
    quadrature of f(F) |det J| over the reference square within the error of
    the (p+1)-point Gauss rule, O(h^(2p+2)) (f taken at (xi, eta), or |det J|
    dropped, would change it by O(1))."""
    import scipy.integrate as si
    n_el = 16
    one = [[1.0, 0.0, 0.0, np.pi / 2]]
    b = assemble.load_vector_2d(n_el, p, one, interior=False)
    assert b.shape == ((n_el + p) ** 2,)
    assert abs(b.sum() - 2.5) <= 1e-13
    assert np.all(b > 0)
    modes = [[1.0, 1.0, 0.0, 0.3], [-0.7, 0.0, 2.0, 1.1], [0.4, 2.0, 1.0, 0.0]]
    f = _mode_sum(modes)
    b = assemble.load_vector_2d(n_el, p, modes, interior=False)

    def integrand(eta, xi):
        x, y = (1 + xi) * (1 - eta ** 2), (1 + xi) * (2 * eta - eta ** 2)
        return f(x, y) * (1 + xi) * (2 - 2 * eta + 2 * eta ** 2)
    ref, err = si.dblquad(integrand, 0.0, 1.0, 0.0, 1.0, epsabs=1e-14, epsrel=1e-14)
    assert err < 1e-12
    h = 1.0 / n_el
    assert abs(b.sum() - ref) <= 20.0 * h ** (2 * p + 2) + 1e-14
    # the interior load vector is the interior block of the full one
    bi = assemble.load_vector_2d(n_el, p, modes)
    n = n_el + p
    np.testing.assert_array_equal(bi, b.reshape(n, n)[1:-1, 1:-1].reshape(-1))
