"""Parity of the full elliptic operators of Section 4.3 (nonsymmetric stored
stencils) with the FP64 CPU oracle, through the C ABI.

Problems: ELLIPTIC_1 on the unit square (f = 1) and ELLIPTIC_2 on the quarter
annulus with exact arcs and radii 0.2 and 1 (manufactured solution); also
ELLIPTIC_2 on the polynomial annulus of radii 1 and 2.  Bars: operator rows of
every level, load vectors, products and the coarse solve to 1e-13 (1e-12 for
the coarse solve), two sweeps to 1e-13, V-cycle iterates to 1e-12 per iterate,
RRE(8) solves to 1e-12 with the oracle's V-cycle and restart counts.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import elliptic as el, extrapolation as ex, multigrid as mg
from paper_2412_20205_amd import igamg

from test_gpu_parity import DEV, _offsets, dev, host, rel

pytestmark = pytest.mark.gpu

PROBLEMS = {
    # name: (library geometry, oracle kind, coefficient set, pde, radii, oracle f)
    "square1": (igamg.UNIT_SQUARE, "square", el.CSET_SQUARE, igamg.PDE_ELLIPTIC_1, (0.0, 0.0),
                lambda x, y: np.ones_like(x)),
    "exact2": (igamg.QUARTER_ANNULUS_EXACT, "annulus_exact", el.CSET_ANNULUS, igamg.PDE_ELLIPTIC_2,
               (0.2, 1.0), el.manufactured_f),
    "poly2": (igamg.QUARTER_ANNULUS, "annulus", el.CSET_ANNULUS, igamg.PDE_ELLIPTIC_2, (0.0, 0.0),
              el.manufactured_f),
    "advdiff": (igamg.UNIT_SQUARE, "square", el.CSET_ADVDIFF, igamg.PDE_ADVECTION_DIFFUSION, (0.0, 0.0),
                lambda x, y: np.ones_like(x)),
}
_cache = {}


def case(name, n_el, p, **opts):
    key = (name, n_el, p, tuple(sorted(opts.items())))
    if key not in _cache:
        print("[elliptic] %s n_el=%d p=%d %s" % (name, n_el, p, opts), flush=True)
        g, kind, cset, pde, radii, f = PROBLEMS[name]
        s = igamg.Solver(g, n_el, p, radii=radii, pde=pde, **opts)
        s.set_rhs_builtin()
        ri, ro = (radii if radii[0] > 0 else (1.0, 2.0))
        H = mg.build_elliptic_hierarchy(kind, n_el, p, cset, ri, ro)
        b = el.load(n_el, p, kind, f, ri, ro)
        _cache[key] = (s, H, b)
    return _cache[key]


CASES = [("square1", 16, 1), ("square1", 16, 2), ("square1", 32, 3), ("square1", 16, 4), ("square1", 16, 5),
         ("exact2", 16, 2), ("exact2", 32, 3), ("exact2", 16, 4), ("exact2", 16, 5), ("poly2", 16, 3),
         ("advdiff", 16, 2), ("advdiff", 32, 4)]


@pytest.mark.parametrize("name,n_el,p", CASES)
def test_rows_rhs_products_coarse(name, n_el, p):
    s, H, b = case(name, n_el, p)
    di, dj, _ = _offsets(p, 2)
    assert s.num_levels == len(H.levels)
    for l, lev in enumerate(H.levels):
        n, N = lev.n, lev.A.shape[0]
        rows = np.arange(N)
        got = s.operator_rows(l, rows)
        A = lev.A.tocsr()
        i, j = rows % n, rows // n
        scale = abs(A).max()
        for o in range(got.shape[1]):
            ii, jj = i + di[o], j + dj[o]
            ok = (ii >= 0) & (ii < n) & (jj >= 0) & (jj < n)
            ref = np.zeros(N)
            ref[ok] = np.asarray(A[rows[ok], (ii + n * jj)[ok]]).ravel()
            assert np.all(got[~ok, o] == 0.0)
            assert np.abs(got[:, o] - ref).max() <= 1e-13 * scale, (l, o)
        x = synth.random_vector(N, 10 + l)
        y = torch.zeros(N, dtype=torch.float64, device=DEV)
        s.apply(l, dev(x), y)
        assert rel(host(y), lev.A @ x) < 1e-13
    bd = torch.zeros(s.ndof, dtype=torch.float64, device=DEV)
    s.get_rhs(bd)
    assert rel(host(bd), b) < 1e-13
    b0 = synth.random_vector(H.levels[0].A.shape[0], 30)
    x0 = torch.zeros(len(b0), dtype=torch.float64, device=DEV)
    s.coarse_solve(dev(b0), x0)
    assert rel(host(x0), H.coarse_solve(b0)) < 1e-12


@pytest.mark.parametrize("name,n_el,p", [("square1", 32, 2), ("exact2", 32, 3), ("exact2", 16, 5)])
def test_sweeps_and_vcycle_iterates(name, n_el, p):
    for tail in (0, 32):
        s, H, b = case(name, n_el, p, tail_items=tail)
        for l in range(1, len(H.levels)):
            lev = H.levels[l]
            bl = synth.random_vector(lev.A.shape[0], 40 + l)
            x0 = synth.random_vector(lev.A.shape[0], 50 + l)
            xg = dev(x0)
            s.smooth(l, dev(bl), xg, 2)
            assert rel(host(xg), mg.smooth(lev, bl, x0.copy(), mg.SMOOTH_MCGS, 2)) < 1e-13
        L = len(H.levels) - 1
        xg = torch.zeros(len(b), dtype=torch.float64, device=DEV)
        xr = np.zeros(len(b))
        for it in range(5):
            s.vcycle(xg)
            xr = mg.mu_cycle(H, L, b, xr, mg.SMOOTH_MCGS, 2, 2, 1)
            assert rel(host(xg), xr) < 1e-12, (tail, it)


@pytest.mark.parametrize("name,n_el,p", [("square1", 32, 1), ("square1", 32, 4), ("exact2", 32, 2),
                                         ("exact2", 64, 3), ("exact2", 32, 5), ("advdiff", 64, 3)])
def test_rre8_solve_matches_oracle(name, n_el, p):
    """RRE(8), relative residual 1e-12 (the setting of Tables 13 and 15)."""
    s, H, b = case(name, n_el, p)
    L = len(H.levels) - 1
    A = H.fine.A
    nb = np.linalg.norm(b)
    G = lambda x: mg.mu_cycle(H, L, b, x, mg.SMOOTH_MCGS, 2, 2, 1)
    rn = lambda x: np.linalg.norm(b - A @ x) / nb
    xr, st_r, _ = ex.restarted_solve(G, rn, np.zeros(len(b)), 8, ex.RRE, tol=1e-12, max_restarts=300)
    assert st_r.converged
    xg = torch.zeros(len(b), dtype=torch.float64, device=DEV)
    st, _ = s.solve(xg, tol=1e-12, max_restarts=300, method=igamg.RRE, q=8)
    x = host(xg)
    assert st.vcycles == st_r.vcycles and st.restarts == st_r.restarts
    assert rn(x) <= 1.0000001e-12
    assert rel(x, xr) < 1e-10


@pytest.mark.parametrize("name,n_el,p", [("square1", 64, 3), ("exact2", 64, 3)])
def test_fp32_refinement_reaches_tolerance(name, n_el, p):
    s, H, b = case(name, n_el, p, precision=igamg.FP32_IR)
    xg = torch.zeros(len(b), dtype=torch.float64, device=DEV)
    st, _ = s.solve(xg, tol=1e-10, max_restarts=300, method=igamg.RRE, q=8)
    A = H.fine.A
    assert np.linalg.norm(b - A @ host(xg)) / np.linalg.norm(b) <= 1.0000001e-10


def test_manufactured_solution_error():
    """The GPU solution of the annulus problem approximates the manufactured u
    with the discretisation error of the oracle's own exact discrete solution."""
    import scipy.sparse.linalg as spla
    s, H, b = case("exact2", 32, 3)
    xg = torch.zeros(len(b), dtype=torch.float64, device=DEV)
    s.solve(xg, tol=1e-12, max_restarts=300, method=igamg.RRE, q=8)
    e_gpu, r = el.l2_error(32, 3, "annulus_exact", host(xg), el.manufactured_u, 0.2, 1.0)
    u = spla.spsolve(H.fine.A.tocsc(), b)
    e_ref, _ = el.l2_error(32, 3, "annulus_exact", u, el.manufactured_u, 0.2, 1.0)
    assert abs(e_gpu - e_ref) <= 1e-6 * e_ref
    assert e_gpu / r < 1e-5


def test_elliptic_argument_errors():
    with pytest.raises(igamg.IgamgError):
        igamg.Solver(igamg.UNIT_CUBE, 8, 2, pde=igamg.PDE_ELLIPTIC_1)
    with pytest.raises(igamg.IgamgError):
        igamg.Solver(igamg.QUARTER_ANNULUS_EXACT, 16, 2, radii=(1.0, 0.5))
    s = igamg.Solver(igamg.UNIT_SQUARE, 16, 2)
    with pytest.raises(igamg.IgamgError):
        s.set_rhs_builtin()
    s.close()
