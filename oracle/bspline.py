"""Univariate B-spline spaces, quadrature and 1D Galerkin matrices (FP64).

Paper: Section 2.3 "B-splines & IGA" (open uniform knot vectors, the
Cox-de Boor recursion, eq. (5), and Proposition 3), and Section 2 (the SPD
system A u = b, eq. (2), and the Galerkin coarse operator, eq. (4)).

Conventions (readings where the paper is silent):
  * N_el elements on [0, 1]; open uniform knots
    t = (0^{p+1}, 1/N_el, ..., (N_el-1)/N_el, 1^{p+1}); n_tot = N_el + p
    basis functions.
  * Degree-0 functions are indicators of half-open spans [t_j, t_{j+1}); the
    point x = 1 is assigned to the last non-empty span.  0/0 := 0 in eq. (5).
  * Homogeneous Dirichlet conditions are imposed by dropping the first and last
    basis function: the n = N_el + p - 2 unknowns are functions 1 .. n_tot-2.
"""
import numpy as np


def open_uniform_knots(n_el, p):
    """Open uniform knot vector with p+1 repeated end knots (Section 2.3)."""
    inner = np.arange(1, n_el, dtype=np.float64) / n_el
    return np.concatenate([np.zeros(p + 1), inner, np.ones(p + 1)])


def _last_nonempty_span(t):
    for j in range(len(t) - 2, -1, -1):
        if t[j] < t[j + 1]:
            return j
    raise ValueError("degenerate knot vector")


def cox_de_boor(t, p, x):
    """Values N_j^p(x) of all B-splines on knot vector t, by eq. (5).

    Returns an array of shape (len(x), len(t) - p - 1).  The recursion is run
    literally from degree 0 upwards, with 0/0 := 0.
    """
    t = np.asarray(t, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    m = len(t) - 1
    N = np.zeros((len(x), m))
    for j in range(m):
        N[:, j] = ((t[j] <= x) & (x < t[j + 1])).astype(np.float64)
    N[x == t[-1], _last_nonempty_span(t)] = 1.0
    for k in range(1, p + 1):
        Nk = np.zeros((len(x), m - k))
        for j in range(m - k):
            left = t[j + k] - t[j]
            right = t[j + k + 1] - t[j + 1]
            v = np.zeros(len(x))
            if left > 0.0:
                v += (x - t[j]) / left * N[:, j]
            if right > 0.0:
                v += (t[j + k + 1] - x) / right * N[:, j + 1]
            Nk[:, j] = v
        N = Nk
    return N


def cox_de_boor_derivative(t, p, x):
    """First derivatives of all degree-p B-splines, from the degree p-1 ones.

    Differentiating eq. (5) gives the standard rule
    N_j^p' = p/(t_{j+p}-t_j) N_j^{p-1} - p/(t_{j+p+1}-t_{j+1}) N_{j+1}^{p-1}.
    """
    t = np.asarray(t, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    nb = len(t) - p - 1
    if p == 0:
        return np.zeros((len(x), nb))
    Nm = cox_de_boor(t, p - 1, x)
    D = np.zeros((len(x), nb))
    for j in range(nb):
        left = t[j + p] - t[j]
        right = t[j + p + 1] - t[j + 1]
        if left > 0.0:
            D[:, j] += p / left * Nm[:, j]
        if right > 0.0:
            D[:, j] -= p / right * Nm[:, j + 1]
    return D


def gauss_legendre(nq):
    """Gauss-Legendre rule on [-1, 1] (library routine)."""
    return np.polynomial.legendre.leggauss(nq)


def element_quadrature(n_el, nq):
    """Physical Gauss points and weights on every element of [0, 1].

    Returns (xq, wq), both of shape (n_el, nq).  Element e is [e/N_el, (e+1)/N_el].
    """
    g, w = gauss_legendre(nq)
    a = np.arange(n_el, dtype=np.float64) / n_el
    b = np.arange(1, n_el + 1, dtype=np.float64) / n_el
    xq = 0.5 * (a + b)[:, None] + 0.5 * (b - a)[:, None] * g[None, :]
    wq = 0.5 * (b - a)[:, None] * w[None, :]
    return xq, wq


def local_basis_tables(n_el, p, nq):
    """Values and derivatives of the p+1 functions alive on each element.

    On element e (span [t_{p+e}, t_{p+e+1})) the nonzero functions are
    N_e .. N_{e+p} (Proposition 3, second item).  Returns (xq, wq, V, D) with
    V, D of shape (n_el, nq, p+1): V[e, q, a] = N_{e+a}(xq[e, q]).
    """
    t = open_uniform_knots(n_el, p)
    xq, wq = element_quadrature(n_el, nq)
    flat = xq.reshape(-1)
    Nall = cox_de_boor(t, p, flat).reshape(n_el, nq, -1)
    Dall = cox_de_boor_derivative(t, p, flat).reshape(n_el, nq, -1)
    V = np.zeros((n_el, nq, p + 1))
    D = np.zeros((n_el, nq, p + 1))
    for e in range(n_el):
        V[e] = Nall[e, :, e:e + p + 1]
        D[e] = Dall[e, :, e:e + p + 1]
    return xq, wq, V, D


def stiffness_mass_1d(n_el, p, interior=True):
    """1D stiffness K1_ab = int N_a' N_b' and mass M1_ab = int N_a N_b.

    Gauss quadrature with p+1 points per element, which is exact for these
    piecewise polynomial integrands.  With interior=True the first and last
    rows/columns (Dirichlet functions) are dropped.  Dense (small n only).
    """
    n_tot = n_el + p
    _, wq, V, D = local_basis_tables(n_el, p, p + 1)
    K = np.zeros((n_tot, n_tot))
    M = np.zeros((n_tot, n_tot))
    for e in range(n_el):
        sl = slice(e, e + p + 1)
        K[sl, sl] += (D[e].T * wq[e]) @ D[e]
        M[sl, sl] += (V[e].T * wq[e]) @ V[e]
    if interior:
        K = K[1:-1, 1:-1]
        M = M[1:-1, 1:-1]
    return K, M


def greville(t, p):
    """Greville abscissae g_i = (t_{i+1} + ... + t_{i+p}) / p."""
    nb = len(t) - p - 1
    return np.array([np.mean(t[i + 1:i + p + 1]) for i in range(nb)])


def prolongation_1d(n_el_coarse, p, interior=True):
    """1D prolongation from N_el/2 to N_el elements (Section 2, P_{2h}^h).

    The coarse space is contained in the fine one (the fine knots refine the
    coarse knots), so each coarse function is a combination of fine functions.
    The coefficients are found by collocation: the fine basis matrix at the
    fine Greville points is nonsingular (Schoenberg-Whitney), and
    P1 = B_f(g)^{-1} B_c(g).  With interior=True the Dirichlet rows and columns
    are dropped.  (The GPU library uses knot insertion instead.)
    """
    p = int(p)
    tc = open_uniform_knots(n_el_coarse, p)
    tf = open_uniform_knots(2 * n_el_coarse, p)
    g = greville(tf, p)
    Bf = cox_de_boor(tf, p, g)
    Bc = cox_de_boor(tc, p, g)
    P = np.linalg.solve(Bf, Bc)
    P[np.abs(P) < 1e-15] = 0.0
    if interior:
        P = P[1:-1, 1:-1]
    return P
