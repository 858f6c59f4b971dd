"""Full elliptic operator -div(A grad u) + B . grad u + c u (FP64, test oracle).

Paper: Section 4.3, the full elliptic problem with homogeneous Dirichlet
conditions: on the unit square with the first coefficient set (right-hand side
f = 1, Table 13) and on a quarter annulus with radii 0.2 and 1 with the second
coefficient set and a manufactured solution (Table 15); the discretisation is
the Galerkin method of Section 2 on the B-spline space of Section 2.3.

The bilinear form is a(u, v) = int A grad u . grad v + (B . grad u) v + c u v,
so that row I (test function phi_I), column J (trial function phi_J) of the
matrix is a(phi_J, phi_I).  The integrals use p+1 Gauss points per element and
direction in the reference square; physical gradients are J^-T times the
reference gradients, and the measure is |det J|.

Readings (where the paper is silent):
  * The quarter annulus of radii r_in < r_out is either the polynomial
    degree-2 B-spline surface (r_in + (r_out - r_in) xi)(1 - eta^2, 2 eta - eta^2)
    (the radii 1 and 2 case is the geometry of the Poisson workloads) or, for
    the manufactured-solution problem, its rational (NURBS) counterpart with
    exact circular arcs: the manufactured u vanishes on circles, and on the
    polynomial surface (whose arcs are up to 6 % off the circle) it does not.
  * The coefficients are evaluated at the physical quadrature points.

Test infrastructure only: the library shares no code with this module.
"""
import math

import numpy as np
import scipy.sparse as sp

from . import bspline

CSET_LAPLACE = "laplace"
CSET_SQUARE = "square"     # Section 4.3, unit square: A, B of Table 13's problem, c = 1
CSET_ANNULUS = "annulus"   # Section 4.3, quarter annulus: same A, B = (-5y, 5x), c = xy
CSET_ADVDIFF = "advdiff"   # Section 4.3, advection-diffusion (Table 14): A = 0.1 I, B = (1, 1), c = 0


def _A(x, y):
    """Diffusion tensor of both Section 4.3 problems (symmetric positive definite)."""
    a11 = (2.0 + np.cos(x)) * (1.0 + y)
    a12 = np.cos(x + y) * np.sin(x + y)
    a22 = (2.0 + np.sin(y)) * (1.0 + x)
    return a11, a12, a22


def coefficients(cset, x, y):
    """(a11, a12, a22, b1, b2, c) at the physical points (x, y)."""
    z = np.zeros_like(x)
    if cset == CSET_LAPLACE:
        return np.ones_like(x), z, np.ones_like(x), z, z, z
    if cset == CSET_ADVDIFF:
        eps = np.full_like(x, 0.1)
        return eps, z, eps, np.ones_like(x), np.ones_like(x), z
    a11, a12, a22 = _A(x, y)
    if cset == CSET_SQUARE:
        cc = np.cos(x + y) ** 2
        b1 = 11.0 + np.sin(x) + y * np.sin(x) - 2.0 * cc
        b2 = -9.0 - np.cos(y) - x * np.cos(y) - 2.0 * cc
        return a11, a12, a22, b1, b2, np.ones_like(x)
    if cset == CSET_ANNULUS:
        return a11, a12, a22, -5.0 * y, 5.0 * x, x * y
    raise ValueError(cset)


def geometry(kind, xi, eta, r_in=1.0, r_out=2.0):
    """Physical point and Jacobian entries (dx/dxi, dx/deta, dy/dxi, dy/deta).

    kind "square": identity; "annulus": the polynomial degree-2 surface
    rho(xi) (1 - eta^2, 2 eta - eta^2); "annulus_exact": rho(xi) C(eta) with C
    the rational quadratic quarter circle (control points (1,0), (1,1), (0,1),
    weights 1, 1/sqrt 2, 1), whose boundary arcs are exact circles.
    """
    if kind == "square":
        one, zero = np.ones_like(xi), np.zeros_like(xi)
        return xi, eta, one, zero, zero, one
    rho = r_in + (r_out - r_in) * xi
    if kind == "annulus_exact":
        w = 1.0 / math.sqrt(2.0)
        b0, b1, b2 = (1.0 - eta) ** 2, 2.0 * eta * (1.0 - eta), eta ** 2
        d0, d1, d2 = -2.0 * (1.0 - eta), 2.0 - 4.0 * eta, 2.0 * eta
        den = b0 + w * b1 + b2
        nx, ny = b0 + w * b1, w * b1 + b2
        dden = d0 + w * d1 + d2
        dnx, dny = d0 + w * d1, w * d1 + d2
        cx, cy = nx / den, ny / den
        dcx, dcy = (dnx * den - nx * dden) / den ** 2, (dny * den - ny * dden) / den ** 2
        return (rho * cx, rho * cy, (r_out - r_in) * cx, rho * dcx, (r_out - r_in) * cy, rho * dcy)
    cx, cy = 1.0 - eta ** 2, 2.0 * eta - eta ** 2
    return (rho * cx, rho * cy, (r_out - r_in) * cx, rho * (-2.0 * eta),
            (r_out - r_in) * cy, rho * (2.0 - 2.0 * eta))


def _element_tables(n_el, p):
    nq = p + 1
    xq, wq, V, D = bspline.local_basis_tables(n_el, p, nq)
    return nq, xq, wq, V, D


def assemble(n_el, p, kind, cset, r_in=1.0, r_out=2.0, interior=True,
             terms=("diffusion", "convection", "reaction")):
    """Sparse matrix of a(phi_J, phi_I) over the interior (or all) functions;
    `terms` selects the parts of the bilinear form that are summed."""
    nq, xq, wq, V, D = _element_tables(n_el, p)
    first = 1 if interior else 0
    n = n_el + p - 2 * first
    nf = p + 1
    rows, cols, vals = [], [], []
    for ey in range(n_el):
        for ex in range(n_el):
            XI, ETA = np.meshgrid(xq[ex], xq[ey], indexing="xy")    # [qy, qx]
            W = np.outer(wq[ey], wq[ex])
            X, Y, j11, j12, j21, j22 = geometry(kind, XI, ETA, r_in, r_out)
            det = j11 * j22 - j12 * j21
            a11, a12, a22, b1, b2, c = coefficients(cset, X, Y)
            # local functions k = a1 + (p+1) a2: value and reference gradient
            val = np.einsum("ya,xb->abyx", V[ey], V[ex])         # [a2, a1, qy, qx]
            gxi = np.einsum("ya,xb->abyx", V[ey], D[ex])
            geta = np.einsum("ya,xb->abyx", D[ey], V[ex])
            val = val.reshape(nf * nf, nq, nq)
            gxi = gxi.reshape(nf * nf, nq, nq)
            geta = geta.reshape(nf * nf, nq, nq)
            # physical gradient = J^-T (d/dxi, d/deta)
            gx = (j22 * gxi - j21 * geta) / det
            gy = (-j12 * gxi + j11 * geta) / det
            m = W * np.abs(det)
            # K[test, trial]
            diff = (np.einsum("iyx,jyx->ij", gx, a11 * gx * m) +
                    np.einsum("iyx,jyx->ij", gx, a12 * gy * m) +
                    np.einsum("iyx,jyx->ij", gy, a12 * gx * m) +
                    np.einsum("iyx,jyx->ij", gy, a22 * gy * m))
            conv = np.einsum("iyx,jyx->ij", val, (b1 * gx + b2 * gy) * m)
            reac = np.einsum("iyx,jyx->ij", val, c * val * m)
            K = (diff if "diffusion" in terms else 0.0) + (conv if "convection" in terms else 0.0) + \
                (reac if "reaction" in terms else 0.0)
            gi = (ex + np.arange(nf)[None, :]) + 0 * np.arange(nf)[:, None]   # [a2, a1]
            gj = (ey + np.arange(nf)[:, None]) + 0 * np.arange(nf)[None, :]
            gi = gi.reshape(-1) - first
            gj = gj.reshape(-1) - first
            ok = (gi >= 0) & (gi < n) & (gj >= 0) & (gj < n)
            idx = gi + n * gj
            sel = np.nonzero(ok)[0]
            for a in sel:
                rows.extend([idx[a]] * len(sel))
                cols.extend(idx[sel])
                vals.extend(K[a, sel])
    return sp.csr_matrix((vals, (rows, cols)), shape=(n * n, n * n))


def load(n_el, p, kind, f, r_in=1.0, r_out=2.0):
    """b_I = int f phi_I over the interior functions; f(x, y) a callable."""
    nq, xq, wq, V, _ = _element_tables(n_el, p)
    n = n_el + p - 2
    nf = p + 1
    b = np.zeros(n * n)
    for ey in range(n_el):
        for ex in range(n_el):
            XI, ETA = np.meshgrid(xq[ex], xq[ey], indexing="xy")
            W = np.outer(wq[ey], wq[ex])
            X, Y, j11, j12, j21, j22 = geometry(kind, XI, ETA, r_in, r_out)
            m = W * np.abs(j11 * j22 - j12 * j21) * f(X, Y)
            val = np.einsum("ya,xb->abyx", V[ey], V[ex]).reshape(nf * nf, nq, nq)
            loc = np.einsum("iyx,yx->i", val, m)
            for a2 in range(nf):
                for a1 in range(nf):
                    i, j = ex + a1 - 1, ey + a2 - 1
                    if 0 <= i < n and 0 <= j < n:
                        b[i + n * j] += loc[a1 + nf * a2]
    return b


# ---- manufactured solution on the quarter annulus (radii 0.2 and 1) -------

MANUFACTURED_R_IN, MANUFACTURED_R_OUT = 0.2, 1.0


def manufactured_u(x, y):
    """u = (x^2 + y^2 - 0.2^2)(x^2 + y^2 - 1) sin x sin y (zero on the boundary)."""
    r2 = x * x + y * y
    return (r2 - 0.04) * (r2 - 1.0) * np.sin(x) * np.sin(y)


def manufactured_f(x, y):
    """f = -div(A grad u) + B . grad u + c u for the annulus coefficient set,
    from the derivatives of u = g s, g = (r^2 - 0.04)(r^2 - 1), s = sin x sin y."""
    r2 = x * x + y * y
    h = 2.0 * r2 - 1.04                 # dg/d(r^2)
    g = (r2 - 0.04) * (r2 - 1.0)
    gx, gy = 2.0 * x * h, 2.0 * y * h
    gxx, gyy, gxy = 8.0 * x * x + 2.0 * h, 8.0 * y * y + 2.0 * h, 8.0 * x * y
    s = np.sin(x) * np.sin(y)
    sx, sy = np.cos(x) * np.sin(y), np.sin(x) * np.cos(y)
    sxx, syy, sxy = -s, -s, np.cos(x) * np.cos(y)
    u = g * s
    ux, uy = gx * s + g * sx, gy * s + g * sy
    uxx = gxx * s + 2.0 * gx * sx + g * sxx
    uyy = gyy * s + 2.0 * gy * sy + g * syy
    uxy = gxy * s + gx * sy + gy * sx + g * sxy
    a11, a12, a22 = _A(x, y)
    a11_x = -np.sin(x) * (1.0 + y)
    a12_x = a12_y = np.cos(2.0 * (x + y))
    a22_y = np.cos(y) * (1.0 + x)
    div = (a11_x * ux + a11 * uxx + a12_x * uy + a12 * uxy +
           a12_y * ux + a12 * uxy + a22_y * uy + a22 * uyy)
    return -div + (-5.0 * y) * ux + (5.0 * x) * uy + x * y * u


def l2_error(n_el, p, kind, coeffs, u_exact, r_in=1.0, r_out=2.0, extra=3):
    """(||u - u_h||_L2, ||u||_L2) with p+extra Gauss points per direction;
    coeffs are the interior coefficients (x fastest)."""
    nq = p + extra
    xq, wq, V, _ = bspline.local_basis_tables(n_el, p, nq)
    n = n_el + p - 2
    U = np.zeros((n + 2, n + 2))
    U[1:-1, 1:-1] = np.asarray(coeffs).reshape(n, n)
    err = ref = 0.0
    for ey in range(n_el):
        for ex in range(n_el):
            XI, ETA = np.meshgrid(xq[ex], xq[ey], indexing="xy")
            W = np.outer(wq[ey], wq[ex])
            X, Y, j11, j12, j21, j22 = geometry(kind, XI, ETA, r_in, r_out)
            m = W * np.abs(j11 * j22 - j12 * j21)
            c = U[ey:ey + p + 1, ex:ex + p + 1]
            uh = np.einsum("qa,rb,ba->rq", V[ex], V[ey], c)
            ue = u_exact(X, Y)
            err += np.sum(m * (uh - ue) ** 2)
            ref += np.sum(m * ue ** 2)
    return math.sqrt(err), math.sqrt(ref)
