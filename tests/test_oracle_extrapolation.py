"""Pins of the oracle's RRE / MPE (Algorithms 3-4) and restarted driver (Algorithm 5).

Paper: Section 3, eqs. (8)-(10); Section 3.1, Algorithms 3 and 4; Section 3.2,
Algorithm 5.  Textbook facts used as pins: on a linear fixed-point iteration
s_{j+1} = B s_j + c, RRE is GMRES and MPE is FOM (the Arnoldi/Galerkin method) on
(I - B) x = c started from s_0 with q Krylov steps (t - s_0 lies in the span of
Delta s_0 .. Delta s_{q-1}), and both are exact once q reaches the degree of the
minimal polynomial of B with respect to the initial error.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from oracle import assemble, extrapolation as ex, multigrid as mg


def _linear_sequence(N=40, q=5, seed=0, rank=None):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((N, N)))
    lam = rng.uniform(-0.9, 0.95, N)
    if rank is not None:
        lam[rank:] = 0.0
    B = (Q * lam) @ Q.T
    c = rng.standard_normal(N)
    S = [rng.standard_normal(N)]
    for _ in range(q + 1):
        S.append(B @ S[-1] + c)
    return B, c, S


def _krylov(A, r0, m):
    K = [r0]
    for _ in range(m - 1):
        K.append(A @ K[-1])
    Q, _ = np.linalg.qr(np.column_stack(K))
    return Q


@pytest.mark.parametrize("q", [1, 3, 5, 8])
@pytest.mark.parametrize("method", [ex.RRE, ex.MPE])
def test_weighted_sum_equals_qr_form(q, method):
    """t = sum_j gamma_j s_j (the definition) equals the algorithms' QR form
    s_0 + Q_q R_q a, a_j = 1 - sum_{i<=j} gamma_i (summation by parts), on a
    linear sequence and on FP64 V-cycle iterates of the annulus."""
    _, _, S = _linear_sequence(q=q, seed=10 + q)
    t, g, _ = ex.extrapolate(S, method)
    t2, g2, _ = ex.extrapolate_qr_form(S, method)
    assert np.array_equal(g, g2)
    np.testing.assert_allclose(t, t2, rtol=1e-12, atol=1e-13 * np.abs(t).max())
    H = mg.build_hierarchy("annulus", 16, 3)
    b = assemble.load_vector_2d(16, 3, synth.random_field_modes(2003))
    V = [np.zeros(len(b))]
    for _ in range(q + 1):
        V.append(mg.vcycle(H, b, V[-1]))
    t, _, _ = ex.extrapolate(V, method)
    t2, _, _ = ex.extrapolate_qr_form(V, method)
    assert np.linalg.norm(t - t2) <= 1e-13 * np.linalg.norm(t)


@pytest.mark.parametrize("q", [1, 3, 5, 8])
def test_algorithms_match_closed_forms(q):
    _, _, S = _linear_sequence(q=q, seed=q)
    t_rre, g, _ = ex.extrapolate(S, ex.RRE)
    assert abs(g.sum() - 1) < 1e-13
    np.testing.assert_allclose(t_rre, ex.extrapolate_schur(S, ex.RRE), rtol=1e-9, atol=1e-10)
    np.testing.assert_allclose(t_rre, ex.extrapolate_pinv(S), rtol=1e-9, atol=1e-10)
    t_mpe, g2, _ = ex.extrapolate(S, ex.MPE)
    assert abs(g2.sum() - 1) < 1e-13
    np.testing.assert_allclose(t_mpe, ex.extrapolate_schur(S, ex.MPE), rtol=1e-9, atol=1e-10)
    # t equals sum gamma_j s_j (eq. (8))
    np.testing.assert_allclose(t_rre, sum(gj * s for gj, s in zip(g, S)), atol=1e-10)


@pytest.mark.parametrize("q", [2, 4, 6])
def test_rre_is_gmres_and_mpe_is_fom(q):
    B, c, S = _linear_sequence(q=q, seed=10 + q)
    A = np.eye(len(c)) - B
    r0 = c - A @ S[0]
    V = _krylov(A, r0, q)
    # GMRES: minimise ||c - A(s0 + V y)||
    y, *_ = np.linalg.lstsq(A @ V, r0, rcond=None)
    x_gmres = S[0] + V @ y
    # FOM: residual orthogonal to the Krylov space
    y2 = np.linalg.solve(V.T @ A @ V, V.T @ r0)
    x_fom = S[0] + V @ y2
    t_rre, _, _ = ex.extrapolate(S, ex.RRE)
    t_mpe, _, _ = ex.extrapolate(S, ex.MPE)
    np.testing.assert_allclose(t_rre, x_gmres, rtol=1e-9, atol=1e-10)
    np.testing.assert_allclose(t_mpe, x_fom, rtol=1e-9, atol=1e-10)


@pytest.mark.parametrize("k", [2, 3, 5])
def test_exact_when_q_reaches_minimal_polynomial_degree(k):
    """A k-dimensional linear map is extrapolated exactly with q = k (k+1
    differences, the last one dependent: lucky breakdown), but not with q = k-1.
    In dimension 30 with rank(B) = k the minimal polynomial has degree k+1
    (eigenvalue 0 included), so q = k+1 is exact and q = k is not."""
    for N, q_exact in ((k, k), (30, k + 1)):
        B, c, S = _linear_sequence(N=N, q=q_exact, seed=20 + k,
                                   rank=None if N == k else k)
        xs = np.linalg.solve(np.eye(N) - B, c)
        for method in (ex.RRE, ex.MPE):
            t, _, _ = ex.extrapolate(S, method)
            assert np.linalg.norm(t - xs) / np.linalg.norm(xs) < 1e-10, (N, method)
            t2, _, _ = ex.extrapolate(S[:-1], method)
            assert np.linalg.norm(t2 - xs) / np.linalg.norm(xs) > 1e-6, (N, method)


def test_rre_residual_not_worse_than_any_difference():
    _, _, S = _linear_sequence(q=5, seed=3)
    _, g, _ = ex.extrapolate(S, ex.RRE)
    U = ex.differences(S)
    assert np.linalg.norm(U @ g) <= np.linalg.norm(U, axis=0).min() * (1 + 1e-12)


def test_drifting_sequence_breaks_down():
    """s_j = j v has no fixed point: every difference equals v."""
    v = synth.random_vector(20, 1)
    S = [j * v for j in range(7)]
    for method in (ex.RRE, ex.MPE):
        with pytest.raises(ex.Breakdown):
            ex.extrapolate(S, method)


def test_lucky_breakdown_returns_fixed_point():
    """If the iteration reaches its fixed point inside a cycle, the extrapolation
    returns it exactly."""
    xs = synth.random_vector(20, 2)
    a, b = synth.random_vector(20, 3), synth.random_vector(20, 4)
    for S in ([xs + a, xs + b, xs, xs, xs, xs], [xs, xs, xs, xs]):
        for method in (ex.RRE, ex.MPE):
            t, _, info = ex.extrapolate(S, method)
            assert info == "lucky"
            np.testing.assert_allclose(t, xs, atol=1e-13)


def test_restarted_driver_counts_and_converges():
    """Algorithm 5 on the C1-type problem (unit square 16^2, p = 3, V(2,2) MCGS)."""
    H = mg.build_hierarchy("square", 16, 3)
    b = assemble.kron_load_2d(16, 3, synth.manufactured_sine_modes_2d())
    A = H.fine.A
    nb = np.linalg.norm(b)
    G = lambda x: mg.vcycle(H, b, x)
    rn = lambda x: np.linalg.norm(b - A @ x) / nb
    u = spla.spsolve(A.tocsc(), b)
    for method in (ex.RRE, ex.MPE, None):
        x, st, its = ex.restarted_solve(G, rn, np.zeros(len(b)), 5, method, tol=1e-10,
                                        max_restarts=400, keep_iterates=True)
        assert st.converged and st.rel_residual <= 1e-10
        if method is not None:
            assert st.vcycles == 6 * st.restarts
            assert len(its) == 7 * st.restarts
        assert np.linalg.norm(x - u) / np.linalg.norm(u) < 1e-8


def test_paper_qualitative_degree_robustness():
    """Plain V-cycle counts grow steeply with p while RRE restart counts stay small
    (Tables 11 and 2D RRE(8): bounded restarts as p grows)."""
    counts = {}
    for p in (2, 4):
        H = mg.build_hierarchy("square", 32, p)
        b = assemble.kron_load_2d(32, p, synth.manufactured_sine_modes_2d())
        A = H.fine.A
        nb = np.linalg.norm(b)
        G = lambda x, H=H, b=b: mg.vcycle(H, b, x)
        rn = lambda x, A=A, b=b, nb=nb: np.linalg.norm(b - A @ x) / nb
        _, s_plain, _ = ex.restarted_solve(G, rn, np.zeros(len(b)), 8, None, 1e-10, 2000)
        _, s_rre, _ = ex.restarted_solve(G, rn, np.zeros(len(b)), 8, ex.RRE, 1e-10, 100)
        counts[p] = (s_plain.vcycles, s_rre.restarts)
    assert counts[4][0] > 4 * counts[2][0]
    assert counts[4][1] <= 4 and counts[2][1] <= 2
    assert counts[4][1] * 9 < counts[4][0]


@pytest.mark.parametrize("method", [ex.RRE, ex.MPE])
@pytest.mark.parametrize("q", [2, 5, 8])
def test_generalized_residual_is_one_step_of_the_map(method, q):
    """Section 3, eq. (11): r~(t) = t~ - t.  On an affine map s -> B s + c with
    sum gamma_j = 1, t~ = B t + c, so r~(t) = G(t) - t; it also equals the
    closed form Delta s_0 - Delta^2 S (Y^T Delta^2 S)^-1 Y^T Delta s_0."""
    B, c, S = _linear_sequence(N=60, q=q, seed=3)
    t, gamma, info = ex.extrapolate(S, method)
    assert info == "ok"
    r = ex.generalized_residual(S, gamma)
    g = B @ t + c - t
    assert np.linalg.norm(r - g) < 1e-10 * np.linalg.norm(g)
    rc = ex.generalized_residual_closed(S, method)
    assert np.linalg.norm(r - rc) < 1e-10 * np.linalg.norm(rc)


def test_rre_generalized_residual_is_the_constrained_minimum():
    """RRE's gamma minimises ||sum gamma_j Delta s_j|| subject to sum gamma_j = 1:
    no other weights (random, summing to one) give a smaller generalised residual."""
    _, _, S = _linear_sequence(N=50, q=5, seed=4)
    _, gamma, _ = ex.extrapolate(S, ex.RRE)
    best = np.linalg.norm(ex.generalized_residual(S, gamma))
    U = ex.differences(S)
    rng = np.random.default_rng(5)
    for _ in range(200):
        w = rng.standard_normal(len(gamma))
        w += (1.0 - w.sum()) / len(w)
        assert np.linalg.norm(U @ w) >= best * (1 - 1e-12)
