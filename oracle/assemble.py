"""Galerkin operators and load vectors (FP64, sparse CSR).

Paper: Section 2, eq. (2) (the SPD stiffness system A u = b) and eq. (4) (the
Galerkin coarse operator R A P); Section 4.2, eq. (12) (2D Poisson); Section
4.3 (quarter annulus given as a B-spline surface).

Index convention: interior unknown (i, j[, k]) has global index
I = i + n j (+ n^2 k), x index fastest, n = N_el + p - 2 per direction.
"""
import numpy as np
import scipy.sparse as sp

from . import bspline
from ._clib import lib

GEOM_IDENTITY = 0
GEOM_ANNULUS = 1


def kron_operator_2d(n_el, p):
    """Unit-square stiffness K1 (x) M1 + M1 (x) K1 as CSR (exact quadrature)."""
    K, M = bspline.stiffness_mass_1d(n_el, p)
    K = sp.csr_matrix(K)
    M = sp.csr_matrix(M)
    A = (sp.kron(M, K) + sp.kron(K, M)).tocsr()
    A.eliminate_zeros()   # kron may store explicit zeros (block format)
    return A


def kron_operator_3d(n_el, p):
    """Unit-cube stiffness K(x)M(x)M + M(x)K(x)M + M(x)M(x)K as CSR."""
    K, M = bspline.stiffness_mass_1d(n_el, p)
    K = sp.csr_matrix(K)
    M = sp.csr_matrix(M)
    A = (sp.kron(sp.kron(K, M), M) + sp.kron(sp.kron(M, K), M) +
         sp.kron(sp.kron(M, M), K)).tocsr()
    A.eliminate_zeros()   # kron may store explicit zeros (block format)
    return A


def stencil_to_csr(st, n, p):
    """Convert stencil rows (n*n, (2p+1)^2) to a CSR matrix, dropping empty slots."""
    W = 2 * p + 1
    N = n * n
    I = np.arange(N)
    i, j = I % n, I // n
    rows, cols, vals = [], [], []
    for o in range(W * W):
        di, dj = o % W - p, o // W - p
        ii, jj = i + di, j + dj
        ok = (ii >= 0) & (ii < n) & (jj >= 0) & (jj < n)
        rows.append(I[ok])
        cols.append((ii + n * jj)[ok])
        vals.append(st[ok, o])
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N))
    A.sum_duplicates()
    return A


def mapped_stiffness_2d(n_el, p, geom=GEOM_ANNULUS, as_stencil=False, interior=True):
    """Stiffness matrix on the mapped square by element-scatter quadrature.

    p+1 Gauss points per element and direction; A_IJ = sum over quadrature points
    of w |det J| (J^-T grad phi_I) . (J^-T grad phi_J).  The geometry is the
    quarter annulus F(xi, eta) = (1 + xi)(1 - eta^2, 2 eta - eta^2), i.e. the
    degree-2 B-spline surface of radii 1 and 2 (reading of Section 4.3), or the
    identity.  interior=False keeps the Dirichlet functions (n = N_el + p).
    """
    nq = p + 1
    xq, wq, V, D = bspline.local_basis_tables(n_el, p, nq)
    first = 1 if interior else 0
    n = n_el + p - 2 * first
    S = (2 * p + 1) ** 2
    out = np.zeros(n * n * S)
    lib().orc_assemble_stiffness_2d(n_el, p, nq, geom, first, np.ascontiguousarray(xq.ravel()),
                                    np.ascontiguousarray(wq.ravel()),
                                    np.ascontiguousarray(V.ravel()),
                                    np.ascontiguousarray(D.ravel()), out)
    st = out.reshape(n * n, S)
    if as_stencil:
        return st
    return stencil_to_csr(st, n, p)


def load_vector_2d(n_el, p, modes, geom=GEOM_ANNULUS, interior=True):
    """b_I = int f phi_I with f = sum_m a_m sin(pi (k_m x + l_m y) + phi_m).

    f is evaluated in physical coordinates; p+1 Gauss points per direction.
    interior=False keeps the Dirichlet functions (n = N_el + p), so that by the
    partition of unity (Section 2.3, Proposition 3) the entries sum to int f.
    """
    nq = p + 1
    xq, wq, V, _ = bspline.local_basis_tables(n_el, p, nq)
    first = 1 if interior else 0
    n = n_el + p - 2 * first
    out = np.zeros(n * n)
    modes = np.ascontiguousarray(np.asarray(modes, dtype=np.float64).reshape(-1, 4))
    lib().orc_assemble_load_2d(n_el, p, nq, geom, first, np.ascontiguousarray(xq.ravel()),
                               np.ascontiguousarray(wq.ravel()),
                               np.ascontiguousarray(V.ravel()), modes.ravel().copy(),
                               len(modes), out)
    return out


def load_vector_3d(n_el, p, modes):
    """Unit-cube load vector for f = sum_m a_m sin(pi (k x + l y + m z) + phi).

    The integral over each element is a tensor Gauss rule with p+1 points per
    direction; evaluated with dense numpy sums per z-layer of elements.
    """
    nq = p + 1
    xq, wq, V, _ = bspline.local_basis_tables(n_el, p, nq)
    n = n_el + p - 2
    n_tot = n_el + p
    modes = np.asarray(modes, dtype=np.float64).reshape(-1, 5)
    # B[q, f]: value of 1D function f at flat quadrature point q
    nqt = n_el * nq
    B = np.zeros((nqt, n_tot))
    for e in range(n_el):
        B[e * nq:(e + 1) * nq, e:e + p + 1] = V[e]
    x = xq.ravel()
    w = wq.ravel()
    out = np.zeros((n_tot, n_tot, n_tot))  # indexed [k, j, i]
    for iz in range(nqt):
        X, Y = np.meshgrid(x, x, indexing="xy")  # X[jy, ix]
        f = np.zeros_like(X)
        for a, kx, ly, mz, ph in modes:
            f += a * np.sin(np.pi * (kx * X + ly * Y + mz * x[iz]) + ph)
        g = f * w[None, :] * w[:, None] * w[iz]          # [qy, qx]
        layer = B.T @ g @ B                               # [j, i]
        out += B[iz][:, None, None] * layer[None, :, :]
    return out[1:-1, 1:-1, 1:-1].reshape(-1).copy() if n > 0 else np.zeros(0)


def kron_load_2d(n_el, p, modes):
    """Unit-square load vector (identity geometry) for a 2D mode table."""
    return load_vector_2d(n_el, p, modes, geom=GEOM_IDENTITY)
