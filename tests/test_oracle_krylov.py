"""Pins of the oracle's flexible GMRES (the extrapolated cycle as preconditioner)."""
import numpy as np
import pytest

import synth
from oracle import elliptic as el, extrapolation as ex, krylov, multigrid as mg


def _system(N=60, seed=0):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((N, N)) / np.sqrt(N) + 3.0 * np.eye(N)
    return A, rng.standard_normal(N)


@pytest.mark.parametrize("k", [1, 4, 9])
def test_identity_preconditioner_is_minimal_residual_over_krylov_space(k):
    """With M = I, after k steps x minimises ||b - A x|| over span{b, Ab, .., A^(k-1) b}."""
    A, b = _system()
    x, it = krylov.fgmres(A, b, lambda v: v.copy(), m=30, fixed_iters=k)
    K = [b]
    for _ in range(k - 1):
        K.append(A @ K[-1])
    K = np.column_stack(K)
    c, *_ = np.linalg.lstsq(A @ K, b, rcond=None)
    np.testing.assert_allclose(x, K @ c, rtol=1e-9, atol=1e-12)


def test_exact_preconditioner_converges_in_one_step():
    A, b = _system(seed=1)
    Ainv = np.linalg.inv(A)
    x, it = krylov.fgmres(A, b, lambda v: Ainv @ v, tol=1e-12, m=10)
    assert it == 1
    assert np.linalg.norm(b - A @ x) <= 1e-12 * np.linalg.norm(b)


def test_restart_keeps_reducing_the_residual():
    A, b = _system(seed=2)
    x, it = krylov.fgmres(A, b, lambda v: v.copy(), tol=1e-11, m=3, max_iters=400)
    assert np.linalg.norm(b - A @ x) <= 1e-11 * np.linalg.norm(b)


@pytest.mark.parametrize("method", [None, ex.RRE])
def test_extrapolated_cycle_preconditions_the_nonsymmetric_problem(method):
    """FGMRES with one V-cycle or one RRE(3) restart cycle as preconditioner
    reaches 1e-10 on the first Section 4.3 problem in fewer iterations than the
    identity preconditioner reaches in 200."""
    H = mg.build_elliptic_hierarchy("square", 16, 2, el.CSET_SQUARE)
    b = el.load(16, 2, "square", lambda x, y: np.ones_like(x))
    A = H.fine.A
    x, it = krylov.fgmres(A, b, krylov.extrapolated_cycle(H, 3, method), tol=1e-10, m=20)
    assert np.linalg.norm(b - A @ x) <= 1e-10 * np.linalg.norm(b)
    assert it <= 12
