"""Flexible GMRES with the extrapolated multigrid cycle as preconditioner (FP64).

Paper: Section 1 and the conclusions state that the extrapolated V-cycle can
serve as a preconditioner for the Galerkin systems; since one restart cycle of
RRE/MPE (Algorithm 5's body from a zero start) depends nonlinearly on its
right-hand side, it is used inside flexible GMRES (right preconditioning with
the preconditioned directions kept), restarted every m steps.  The
orthogonalisation is classical Gram-Schmidt applied twice.

Test infrastructure only.
"""
import numpy as np

from . import extrapolation as ex, multigrid as mg


def extrapolated_cycle(H, q, method, kind=mg.SMOOTH_MCGS, nu1=2, nu2=2):
    """M(v): one restart cycle for A z = v from z = 0 (q+1 V-cycles, then t);
    method None gives one V-cycle."""
    L = len(H.levels) - 1

    def M(v):
        if method is None:
            return mg.mu_cycle(H, L, v, np.zeros(len(v)), kind, nu1, nu2, 1)
        S = [np.zeros(len(v))]
        for _ in range(q + 1):
            S.append(mg.mu_cycle(H, L, v, S[-1], kind, nu1, nu2, 1))
        t, _, _ = ex.extrapolate(S, method)
        return t
    return M


def fgmres(A, b, M, x0=None, tol=1e-10, m=20, max_iters=200, fixed_iters=None):
    """Right-preconditioned flexible GMRES(m).  Stops when the Arnoldi residual
    estimate |g_{j+1}| <= tol ||b|| (then the true residual is checked at the next
    restart), or after fixed_iters iterations when given.  Returns (x, iters)."""
    x = np.zeros(len(b)) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    nb = np.linalg.norm(b)
    iters = 0
    while True:
        r = b - A @ x
        beta = np.linalg.norm(r)
        if fixed_iters is None and beta <= tol * nb:
            return x, iters
        if iters >= (fixed_iters if fixed_iters is not None else max_iters):
            return x, iters
        V = [r / beta]
        Z = []
        Hm = np.zeros((m + 1, m))
        k = 0
        for j in range(m):
            Z.append(M(V[j]))
            w = A @ Z[j]
            Vj = np.column_stack(V)
            h = Vj.T @ w
            w = w - Vj @ h
            h2 = Vj.T @ w
            w = w - Vj @ h2
            Hm[:j + 1, j] = h + h2
            Hm[j + 1, j] = np.linalg.norm(w)
            V.append(w / Hm[j + 1, j])
            k = j + 1
            iters += 1
            e1 = np.zeros(k + 1)
            e1[0] = beta
            y, *_ = np.linalg.lstsq(Hm[:k + 1, :k], e1, rcond=None)
            est = np.linalg.norm(e1 - Hm[:k + 1, :k] @ y)
            if fixed_iters is not None and iters >= fixed_iters:
                break
            if fixed_iters is None and (est <= tol * nb or iters >= max_iters):
                break
        x = x + np.column_stack(Z) @ y
