"""Pins of the oracle's smoothers and multigrid cycle.

Paper: Section 2.1 (Algorithm 2), Section 2.2 (Propositions 1 and 2: the cycle
is an affine map with a recursively defined iteration matrix), Section 2.4
(Gauss-Seidel and Jacobi smoothers).
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import synth
from oracle import assemble, multigrid as mg


def _tiny(geom="annulus", n_el=8, p=2):
    return mg.build_hierarchy(geom, n_el, p)


def test_lexicographic_gs_is_triangular_solve():
    """One forward GS sweep is x + (D + L)^{-1} (b - A x)."""
    H = _tiny("annulus", 8, 3)
    lev = H.fine
    b = synth.random_vector(lev.A.shape[0], 1)
    x0 = synth.random_vector(lev.A.shape[0], 2)
    x = mg.smooth(lev, b, x0.copy(), mg.SMOOTH_LEXGS, 1)
    DL = sp.tril(lev.A, format="csr")
    ref = x0 + spla.spsolve_triangular(DL, b - lev.A @ x0, lower=True)
    np.testing.assert_allclose(x, ref, rtol=1e-13, atol=1e-13)


def test_multicolour_gs_is_product_of_colour_steps_and_order_free():
    """A multicolour sweep equals the product over colours of
    x <- x + E_c D^{-1} (b - A x) (E_c selects colour c), and reshuffling the rows
    inside a colour changes nothing."""
    H = _tiny("annulus", 8, 2)
    lev = H.fine
    N = lev.A.shape[0]
    b = synth.random_vector(N, 3)
    x0 = synth.random_vector(N, 4)
    x = mg.smooth(lev, b, x0.copy(), mg.SMOOTH_MCGS, 1)
    col = mg.colours(lev.n, lev.p, 2)
    ref = x0.copy()
    for c in range(col.max() + 1):
        E = (col == c)
        ref = ref + E * (b - lev.A @ ref) / lev.diag
    np.testing.assert_allclose(x, ref, rtol=1e-13, atol=1e-14)
    rng = np.random.default_rng(0)
    lev.colour_rows = [np.ascontiguousarray(rng.permutation(r)) for r in lev.colour_rows]
    x2 = mg.smooth(lev, b, x0.copy(), mg.SMOOTH_MCGS, 1)
    np.testing.assert_array_equal(x, x2)


def _smoother_matrix(lev, kind):
    A = lev.A.toarray()
    N = A.shape[0]
    if kind == mg.SMOOTH_LEXGS:
        return np.eye(N) - np.linalg.solve(np.tril(A), A)
    if kind == mg.SMOOTH_JACOBI:
        return np.eye(N) - (2.0 / 3.0) * A / np.diag(A)[:, None]
    col = mg.colours(lev.n, lev.p, 2)
    S = np.eye(N)
    for c in range(col.max() + 1):
        E = np.diag((col == c).astype(float))
        S = (np.eye(N) - E @ np.diag(1 / np.diag(A)) @ A) @ S
    return S


def _prop2_matrix(H, l, kind, nu1, nu2, mu):
    """Iteration matrix of Proposition 2 built from dense blocks."""
    if l == 0:
        return np.zeros((H.levels[0].A.shape[0],) * 2)
    lev = H.levels[l]
    A = lev.A.toarray()
    Ac = H.levels[l - 1].A.toarray()
    P = lev.P.toarray()
    S = _smoother_matrix(lev, kind)
    Bc = _prop2_matrix(H, l - 1, kind, nu1, nu2, mu)
    inner = np.eye(len(A)) - P @ (np.eye(len(Ac)) - np.linalg.matrix_power(Bc, mu)) @ \
        np.linalg.solve(Ac, P.T @ A)
    return np.linalg.matrix_power(S, nu2) @ inner @ np.linalg.matrix_power(S, nu1)


@pytest.mark.parametrize("kind", [mg.SMOOTH_MCGS, mg.SMOOTH_LEXGS, mg.SMOOTH_JACOBI])
@pytest.mark.parametrize("mu", [1, 2])
def test_cycle_matches_proposition2(kind, mu):
    """G(x) = B x + c with B from Proposition 2 (three levels, tiny grid);
    for two levels B is Proposition 1's two-grid matrix."""
    H = mg.build_hierarchy("annulus", 16, 2)
    L = len(H.levels) - 1
    N = H.fine.A.shape[0]
    b = synth.random_vector(N, 5)
    nu1, nu2 = 2, 1
    G = lambda x: mg.mu_cycle(H, L, b, x, kind, nu1, nu2, mu)
    c = G(np.zeros(N))
    cols = [G(np.eye(N)[:, i]) - c for i in range(N)]
    Bnum = np.column_stack(cols)
    Bref = _prop2_matrix(H, L, kind, nu1, nu2, mu)
    assert np.abs(Bnum - Bref).max() < 1e-11
    assert max(abs(np.linalg.eigvals(Bref))) < 1.0
    # affine: G(x) = B x + c for a random x
    x = synth.random_vector(N, 6)
    np.testing.assert_allclose(G(x), Bref @ x + c, atol=1e-11)


def test_adjoint_restriction_is_transpose():
    H = _tiny("annulus", 8, 3)
    P = H.fine.P
    rng = np.random.default_rng(0)
    r, e = rng.standard_normal(P.shape[0]), rng.standard_normal(P.shape[1])
    assert abs((P.T @ r) @ e - r @ (P @ e)) < 1e-12


def test_fixed_point_is_discrete_solution():
    H = mg.build_hierarchy("annulus", 16, 3)
    b = assemble.load_vector_2d(16, 3, synth.random_field_modes(2003))
    u = spla.spsolve(H.fine.A.tocsc(), b)
    np.testing.assert_allclose(mg.vcycle(H, b, u), u, rtol=1e-12, atol=1e-14)
