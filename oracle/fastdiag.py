"""Exact discrete solutions of the unit-square and unit-cube systems by fast
diagonalisation (test infrastructure only).

Paper: Section 2, eq. (2) (A u = b).  With the generalised eigendecomposition
K1 V = M1 V Lambda (V^T M1 V = I) of the 1D factors, the Kronecker operator
K1(x)M1 + M1(x)K1 [+ third term] is diagonalised by V(x)V[(x)V]:
A^{-1} = (V(x)V(x)V) (Lambda(+)Lambda(+)Lambda)^{-1} (V(x)V(x)V)^T.
"""
import numpy as np
import scipy.linalg as sla

from . import bspline


def solve_kronecker(n_el, p, b, dim):
    """u = A^{-1} b for the unit square (dim 2) or cube (dim 3), natural order."""
    K, M = bspline.stiffness_mass_1d(n_el, p)
    lam, V = sla.eigh(K, M)
    n = K.shape[0]
    B = np.asarray(b, dtype=np.float64).reshape((n,) * dim)
    # apply V^T along every axis
    U = B
    for ax in range(dim):
        U = np.moveaxis(np.tensordot(V.T, np.moveaxis(U, ax, 0), axes=(1, 0)), 0, ax)
    den = np.zeros((n,) * dim)
    for ax in range(dim):
        shape = [1] * dim
        shape[ax] = n
        den = den + lam.reshape(shape)
    U = U / den
    for ax in range(dim):
        U = np.moveaxis(np.tensordot(V, np.moveaxis(U, ax, 0), axes=(1, 0)), 0, ax)
    return U.reshape(-1)
