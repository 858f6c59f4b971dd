"""Geometric multigrid on nested B-spline spaces (FP64, CSR).

Paper: Section 2 (residual equation eq. (3), prolongation P and restriction
R = P^T, Galerkin coarse operator eq. (4)); Section 2.1, Algorithm 2 (the
mu-cycle with a direct solve on the coarsest grid; mu = 1 is the V-cycle);
Section 2.2, Propositions 1-2 (the cycle is an affine fixed-point map);
Section 4.1 (weighted Jacobi with omega = 2/3, zero initial guess).

Readings where the paper is silent:
  * Levels l = 0 (coarsest) .. L (finest), each halving N_el per direction,
    down to a coarsest grid of N_el0 elements per direction.
  * Multicolour Gauss-Seidel: colour c(I) = sum_d (i_d mod (p+1)) (p+1)^d,
    colours swept in increasing order, each colour updated from the values
    at the start of that colour; the same ordering for pre- and post-smoothing.
  * Lexicographic Gauss-Seidel: forward, x index fastest.
  * The coarse-grid correction starts from a zero coarse error (Algorithm 2).
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import assemble, bspline
from ._clib import lib

SMOOTH_MCGS = "mcgs"
SMOOTH_LEXGS = "lexgs"
SMOOTH_JACOBI = "jacobi"


def prolongation(n_el_coarse, p, dim):
    """P = P1 (x) P1 [(x) P1] in the I = i + n j (+ n^2 k) ordering."""
    P1 = sp.csr_matrix(bspline.prolongation_1d(n_el_coarse, p))
    P = P1
    for _ in range(dim - 1):
        P = sp.kron(P1, P)
    return P.tocsr()


def colours(n, p, dim):
    """Colour index c(I) = sum_d (i_d mod (p+1)) (p+1)^d for every unknown."""
    idx = np.indices((n,) * dim)  # idx[d] along axis ordering (slowest..fastest)
    c = np.zeros((n,) * dim, dtype=np.int64)
    # axis dim-1 is x (fastest), weight (p+1)^0
    for d in range(dim):
        c += (idx[dim - 1 - d] % (p + 1)) * (p + 1) ** d
    return c.reshape(-1)


class Level:
    def __init__(self, A, n_el, p, dim):
        self.A = A.tocsr()
        self.A.eliminate_zeros()
        self.A.sort_indices()
        self.n_el = n_el
        self.n = n_el + p - 2
        self.p = p
        self.dim = dim
        self.diag = np.ascontiguousarray(self.A.diagonal())
        self.indptr = self.A.indptr.astype(np.int32)
        self.indices = self.A.indices.astype(np.int32)
        self.data = np.ascontiguousarray(self.A.data, dtype=np.float64)
        col = colours(self.n, p, dim)
        self.colour_rows = [np.ascontiguousarray(np.nonzero(col == c)[0].astype(np.int32))
                            for c in range((p + 1) ** dim)]
        self.P = None  # prolongation from level l-1 to this level


class Hierarchy:
    """Levels 0..L with Galerkin coarse operators A_{l-1} = P_l^T A_l P_l (eq. (4))."""

    def __init__(self, A_fine, n_el, p, dim, n_el_coarsest=4):
        if n_el % n_el_coarsest:
            raise ValueError("n_el must be n_el_coarsest * 2^k")
        levels = [Level(A_fine, n_el, p, dim)]
        ne = n_el
        while ne > n_el_coarsest:
            if ne % 2:
                raise ValueError("n_el must be n_el_coarsest * 2^k")
            P = prolongation(ne // 2, p, dim)
            levels[0].P = P
            Ac = (P.T @ levels[0].A @ P).tocsr()
            ne //= 2
            levels.insert(0, Level(Ac, ne, p, dim))
        self.levels = levels
        A0 = levels[0].A.toarray()
        # Cholesky for the symmetric operators, LU with partial pivoting for
        # the nonsymmetric ones (convection terms of the full elliptic problem)
        self.symmetric = np.allclose(A0, A0.T, rtol=0.0, atol=1e-13 * np.abs(A0).max())
        if self.symmetric:
            self.coarse_chol = sla.cho_factor(A0, lower=True)
        else:
            self.coarse_lu = sla.lu_factor(A0)
        self.p = p
        self.dim = dim

    @property
    def fine(self):
        return self.levels[-1]

    def coarse_solve(self, b):
        """Direct solve on the coarsest grid (Algorithm 2): dense Cholesky, or LU
        for a nonsymmetric operator."""
        if self.symmetric:
            return sla.cho_solve(self.coarse_chol, b)
        return sla.lu_solve(self.coarse_lu, b)


def build_elliptic_hierarchy(kind, n_el, p, cset, r_in=1.0, r_out=2.0, n_el_coarsest=4):
    """Hierarchy of the full elliptic operator of Section 4.3 (oracle.elliptic)."""
    from . import elliptic
    A = elliptic.assemble(n_el, p, kind, cset, r_in, r_out)
    return Hierarchy(A, n_el, p, 2, n_el_coarsest)


def build_hierarchy(geometry, n_el, p, n_el_coarsest=4):
    """Hierarchy for 'square' (Kronecker), 'cube' (Kronecker 3D) or 'annulus'."""
    if geometry == "square":
        return Hierarchy(assemble.kron_operator_2d(n_el, p), n_el, p, 2, n_el_coarsest)
    if geometry == "cube":
        return Hierarchy(assemble.kron_operator_3d(n_el, p), n_el, p, 3, n_el_coarsest)
    if geometry == "annulus":
        return Hierarchy(assemble.mapped_stiffness_2d(n_el, p), n_el, p, 2, n_el_coarsest)
    raise ValueError(geometry)


def smooth(lev, b, x, kind, nsweeps, omega=2.0 / 3.0):
    """nsweeps smoothing steps on A x = b; x is updated in place and returned."""
    L = lib()
    x = np.ascontiguousarray(x, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    N = lev.A.shape[0]
    for _ in range(nsweeps):
        if kind == SMOOTH_LEXGS:
            L.orc_gs_lex(N, lev.indptr, lev.indices, lev.data, lev.diag, b, x)
        elif kind == SMOOTH_MCGS:
            for rows in lev.colour_rows:
                tmp = np.empty(len(rows))
                L.orc_gs_colour(len(rows), rows, lev.indptr, lev.indices, lev.data,
                                lev.diag, b, x, tmp)
        elif kind == SMOOTH_JACOBI:
            x += omega * (b - lev.A @ x) / lev.diag
        else:
            raise ValueError(kind)
    return x


def residual(lev, b, x):
    """r = b - A x (eq. (3))."""
    return b - lev.A @ x


def mu_cycle(H, l, b, x, kind=SMOOTH_MCGS, nu1=2, nu2=2, mu=1, omega=2.0 / 3.0):
    """One mu-cycle on level l (Algorithm 2): returns the new approximation."""
    if l == 0:
        return H.coarse_solve(b)
    lev = H.levels[l]
    x = smooth(lev, b, np.array(x, dtype=np.float64, copy=True), kind, nu1, omega)
    r = residual(lev, b, x)
    rc = lev.P.T @ r
    e = np.zeros(len(rc))
    for _ in range(mu):
        e = mu_cycle(H, l - 1, rc, e, kind, nu1, nu2, mu, omega)
    x = x + lev.P @ e
    return smooth(lev, b, x, kind, nu2, omega)


def vcycle(H, b, x, kind=SMOOTH_MCGS, nu1=2, nu2=2, omega=2.0 / 3.0):
    """G(x): one V-cycle (mu = 1) on the finest level, eq. (7)."""
    return mu_cycle(H, len(H.levels) - 1, b, x, kind, nu1, nu2, 1, omega)
