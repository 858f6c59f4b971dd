"""CPU checks of libigamg.so without a GPU: it loads, exports every function the
public headers declare, and its host-side setup arithmetic (Gauss rule, de Boor
basis evaluation, knot-insertion prolongation, Galerkin bands) agrees with the
oracle's independent constructions (Cox-de Boor recursion, collocation
prolongation, sparse Galerkin products)."""
import os
import re

import numpy as np
import pytest

from oracle import assemble, bspline
from paper_2412_20205_amd import igamg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if not h.endswith(".h"):
            continue
        src = open(os.path.join(ROOT, "include", h)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"\b(igamg_\w+)\s*\(", src):
            names.add(m.group(1))
    return names


def test_library_exports_every_declared_symbol():
    L = igamg.lib()
    names = _declared_functions()
    assert len(names) >= 20
    for n in sorted(names):
        assert hasattr(L, n), n
    # the binding covers the whole ABI
    assert names <= set(igamg._SIGNATURES)


@pytest.mark.parametrize("m", [1, 2, 3, 4, 6, 9])
def test_gauss_legendre_matches_library_routine(m):
    x, w = igamg.host_gauss_legendre(m)
    xr, wr = np.polynomial.legendre.leggauss(m)
    np.testing.assert_allclose(x, xr, atol=1e-15)
    np.testing.assert_allclose(w, wr, atol=1e-15)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 8, 9])
def test_basis_matches_cox_de_boor(p):
    ne = 7
    t = bspline.open_uniform_knots(ne, p)
    for u in np.linspace(0, 1, 29):
        first, N, D = igamg.host_basis(ne, p, u)
        Nr = bspline.cox_de_boor(t, p, [u])[0]
        Dr = bspline.cox_de_boor_derivative(t, p, [u])[0]
        np.testing.assert_allclose(N, Nr[first:first + p + 1], atol=1e-14)
        np.testing.assert_allclose(D, Dr[first:first + p + 1], atol=1e-11)
        assert abs(Nr.sum() - N.sum()) < 1e-14   # every nonzero function is in the window


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 9])
@pytest.mark.parametrize("nc", [4, 5, 16])
def test_knot_insertion_equals_collocation(p, nc):
    Pb = igamg.host_prolongation_1d(nc, p)
    Pc = bspline.prolongation_1d(nc, p, interior=False)
    np.testing.assert_allclose(Pb, Pc, atol=1e-14)


@pytest.mark.parametrize("p", [2, 3, 5, 8, 9])
def test_galerkin_bands_match_oracle(p):
    ne, nc0 = 32, 4
    K, M = bspline.stiffness_mass_1d(ne, p)
    levels = [(K, M)]
    e = ne
    while e > nc0:
        P = bspline.prolongation_1d(e // 2, p)
        K, M = P.T @ K @ P, P.T @ M @ P
        levels.insert(0, (K, M))
        e //= 2
    for lev, (Kr, Mr) in enumerate(levels):
        Kb, Mb = igamg.host_bands(ne, nc0, lev, p)
        n = Kr.shape[0]
        for d in range(-p, p + 1):
            for i in range(n):
                j = i + d
                kr = Kr[i, j] if 0 <= j < n else 0.0
                mr = Mr[i, j] if 0 <= j < n else 0.0
                assert abs(Kb[i, d + p] - kr) < 1e-12 * np.abs(Kr).max()
                assert abs(Mb[i, d + p] - mr) < 1e-14


def test_host_degree_limit():
    """Degrees up to 9 (the 1D problems) are accepted; 10 is refused."""
    igamg.host_basis(4, 9, 0.3)
    with pytest.raises(ValueError):
        igamg.host_basis(4, 10, 0.3)


@pytest.mark.parametrize("p", [2, 3, 5])
def test_coarse_inverse_of_the_coarsest_operator(p):
    """The setup's coarsest inverse (Cholesky of the SPD operator, Section 2)
    of the oracle's 4 x 4-element annulus operator equals the dense inverse."""
    A = assemble.mapped_stiffness_2d(4, p).toarray()
    st, inv = igamg.host_coarse_inverse(A, symmetric=True)
    assert st == 0
    ref = np.linalg.inv(A)
    assert np.abs(inv - ref).max() <= 1e-12 * np.abs(ref).max()
    # the nonsymmetric path (LU) agrees on the same matrix
    st2, inv2 = igamg.host_coarse_inverse(A, symmetric=False)
    assert st2 == 0
    assert np.abs(inv2 - ref).max() <= 1e-12 * np.abs(ref).max()


def test_coarse_inverse_refuses_indefinite_and_singular():
    """A symmetric matrix that is not positive definite gives ENOTSPD (-4),
    as does a singular one on the LU path; the output is left untouched."""
    A = assemble.mapped_stiffness_2d(4, 3).toarray()
    lam = np.linalg.eigvalsh(A)
    B = A - 0.5 * (lam[0] + lam[1]) * np.eye(len(A))   # one negative eigenvalue
    st, inv = igamg.host_coarse_inverse(B, symmetric=True)
    assert st == igamg.ENOTSPD
    assert not inv.any()
    C = A.copy()
    C[:, 3] = C[:, 1]                                    # rank deficient
    C[3, :] = C[1, :]
    st, inv = igamg.host_coarse_inverse(C, symmetric=False)
    assert st == igamg.ENOTSPD
    assert not inv.any()
    st, _ = igamg.host_coarse_inverse(-A, symmetric=True)
    assert st == igamg.ENOTSPD
