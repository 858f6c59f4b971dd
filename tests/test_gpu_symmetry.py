"""Symmetry of the stored Poisson stencils and the full-size product.

The Poisson operator is symmetric (Section 2, eq. (2)): a lower-half stencil
entry A[I, I+o] equals the upper-half entry A[J, J-o] stored at J = I + o.
The library makes every stored Poisson level exactly symmetric at setup (its
assembly and Galerkin products give it up to rounding).  Checked here: exact
symmetry of every level, and at 1024^2 the products and residual norms against
the oracle's independent assembly."""
import numpy as np
import pytest
import torch

import synth
from oracle import assemble
from paper_2412_20205_amd import igamg

from test_gpu_parity import DEV, _offsets, host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("p", [2, 3, 5])
def test_stored_stencils_exactly_symmetric(p):
    print("[symmetry] annulus 64 p=%d" % p, flush=True)
    s = igamg.Solver(igamg.QUARTER_ANNULUS, 64, p)
    di, dj, _ = _offsets(p, 2)
    S = len(di)
    for level in range(s.num_levels):
        N = s.level_ndof(level)
        n = int(round(N ** 0.5))
        rows = np.arange(N)
        got = s.operator_rows(level, rows)
        i, j = rows % n, rows // n
        for o in range(S):
            ii, jj = i + di[o], j + dj[o]
            ok = (ii >= 0) & (ii < n) & (jj >= 0) & (jj < n)
            J = (ii + n * jj)[ok]
            assert np.array_equal(got[rows[ok], o], got[J, S - 1 - o]), (level, o)
    s.close()


def test_products_fullsize():
    """y = A x and ||b - A x|| / ||b|| on the 1024^2 annulus (p = 3) against
    the oracle's assembly, elementwise within 1e-13 of |A| |x|."""
    print("[symmetry] oracle assembly 1024^2 p=3", flush=True)
    A = assemble.mapped_stiffness_2d(1024, 3).tocsr()
    b = assemble.load_vector_2d(1024, 3, synth.random_field_modes(2003))
    s = igamg.Solver(igamg.QUARTER_ANNULUS, 1024, 3)
    s.set_rhs_field(synth.random_field_modes(2003))
    L = s.num_levels - 1
    rng = np.random.default_rng(11)
    x = rng.standard_normal(s.ndof)
    y = torch.zeros(s.ndof, dtype=torch.float64, device=DEV)
    s.apply(L, torch.tensor(x, device=DEV), y)
    ref = A @ x
    bound = abs(A) @ abs(x)
    err = np.abs(host(y) - ref)
    print("[symmetry] apply max err / (|A||x|) %.2e" % (err / bound).max(), flush=True)
    assert np.all(err <= 1e-13 * bound)
    for xv in (x, np.zeros(s.ndof)):
        rel = s.residual(torch.tensor(xv, device=DEV))
        rel_o = np.linalg.norm(b - A @ xv) / np.linalg.norm(b)
        assert abs(rel - rel_o) <= 1e-13 * rel_o
    s.close()
