"""The 1D model problem of Section 2.4 (FP64): -u'' = f on (0, 1), u(0) = u(1) = 0,
with f(x) = (2 pi)^2 sin(2 pi x) and exact solution u(x) = sin(2 pi x) (eq. (6)).

Discretisation as in Section 2: B-splines of degree p on N_el uniform elements
with open knot vectors, the two Dirichlet functions removed (n = N_el + p - 2
unknowns); stiffness and load by Gauss quadrature with p+1 points per element.
The multigrid hierarchy has nlevels levels (Table 1's nlevels = 4: the coarsest
grid has N_el / 2^(nlevels-1) elements) with Galerkin coarse matrices (eq. (4))
and the smoothers and mu-cycle of oracle.multigrid.  The L2 error of a discrete
solution is evaluated with p+1 Gauss points per element (reading of Table 1's
error norm).

Test infrastructure only: nothing in the library imports this module.
"""
import math

import numpy as np
import scipy.sparse as sp

from . import bspline, multigrid as mg


def f(x):
    """Right-hand side of eq. (6)."""
    return (2.0 * np.pi) ** 2 * np.sin(2.0 * np.pi * x)


def exact_u(x):
    return np.sin(2.0 * np.pi * x)


def operator(n_el, p):
    """Interior stiffness matrix K_ij = int N_i' N_j' (CSR, n x n)."""
    K, _ = bspline.stiffness_mass_1d(n_el, p)
    return sp.csr_matrix(K)


def load(n_el, p):
    """Interior load vector b_i = int f N_i, accumulated element by element."""
    xq, wq, V, _ = bspline.local_basis_tables(n_el, p, p + 1)
    fq = f(xq)
    b = np.zeros(n_el + p)
    for e in range(n_el):
        b[e:e + p + 1] += V[e].T @ (wq[e] * fq[e])
    return b[1:-1]


def hierarchy(n_el, p, nlevels):
    """Levels 0 .. nlevels-1 with Galerkin coarse operators; the coarsest grid
    has N_el / 2^(nlevels-1) elements."""
    if nlevels < 1 or n_el % (1 << (nlevels - 1)):
        raise ValueError("N_el must be a multiple of 2^(nlevels-1)")
    return mg.Hierarchy(operator(n_el, p), n_el, p, 1, n_el_coarsest=n_el >> (nlevels - 1))


def l2_error(n_el, p, x):
    """|| u_h - u ||_L2 for the interior coefficients x (boundary coefficients 0)."""
    xq, wq, V, _ = bspline.local_basis_tables(n_el, p, p + 1)
    c = np.zeros(n_el + p)
    c[1:-1] = x
    uh = np.einsum("eqa,ea->eq", V, np.array([c[e:e + p + 1] for e in range(n_el)]))
    return math.sqrt(float(np.sum(wq * (uh - exact_u(xq)) ** 2)))
