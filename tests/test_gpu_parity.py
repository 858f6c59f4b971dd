"""Parity of the HIP library (through its C ABI) with the FP64 CPU oracle.

Bars: integer/index work bit-exact; FP64 operator rows, transfers and the
coarse solve to 1e-13 relative; FP64 multicolour iterates (V-cycles and
extrapolated iterates) to 1e-12 relative per iterate; every solve to a final
relative residual of 1e-10.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import assemble, bspline, extrapolation as ex, multigrid as mg
from paper_2412_20205_amd import igamg

pytestmark = pytest.mark.gpu

GEOM = {"square": igamg.UNIT_SQUARE, "annulus": igamg.QUARTER_ANNULUS, "cube": igamg.UNIT_CUBE}
DEV = "cuda:0"


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=DEV).contiguous()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def oracle_rhs(geom, n_el, p, modes):
    if geom == "cube":
        return assemble.load_vector_3d(n_el, p, modes)
    g = assemble.GEOM_ANNULUS if geom == "annulus" else assemble.GEOM_IDENTITY
    return assemble.load_vector_2d(n_el, p, modes, geom=g)


def modes_for(geom, seed):
    if geom == "cube":
        return synth.manufactured_sine_modes_3d()
    return synth.random_field_modes(seed)


_cache = {}


def case(geom, n_el, p, **opts):
    key = (geom, n_el, p, tuple(sorted(opts.items())))
    if key not in _cache:
        print("[case] %s n_el=%d p=%d %s" % (geom, n_el, p, opts), flush=True)
        s = igamg.Solver(GEOM[geom], n_el, p, **opts)
        H = mg.build_hierarchy(geom, n_el, p)
        modes = modes_for(geom, 2000 + p)
        s.set_rhs_field(modes)
        b = oracle_rhs(geom, n_el, p, modes)
        _cache[key] = (s, H, b)
    return _cache[key]


CASES_2D = [("annulus", 16, 2), ("annulus", 32, 3), ("annulus", 32, 4), ("annulus", 16, 5),
            ("square", 32, 2), ("square", 16, 3), ("square", 8, 1)]
CASES_ALL = CASES_2D + [("cube", 8, 2), ("cube", 8, 3)]


def _offsets(p, dim):
    W = 2 * p + 1
    S = W ** dim
    o = np.arange(S)
    return o % W - p, (o // W) % W - p, (o // (W * W)) - p if dim == 3 else np.zeros(S, int)


@pytest.mark.parametrize("geom,n_el,p", CASES_ALL)
def test_operator_rows_every_level(geom, n_el, p):
    s, H, _ = case(geom, n_el, p)
    dim = 3 if geom == "cube" else 2
    di, dj, dk = _offsets(p, dim)
    assert s.num_levels == len(H.levels)
    for l, lev in enumerate(H.levels):
        n = lev.n
        N = lev.A.shape[0]
        assert s.level_ndof(l) == N
        rows = np.arange(N)
        got = s.operator_rows(l, rows)
        A = lev.A.tocsr()
        i, j, k = rows % n, (rows // n) % n, rows // (n * n) if dim == 3 else 0 * rows
        scale = abs(A).max()
        for o in range(got.shape[1]):
            ii, jj, kk = i + di[o], j + dj[o], k + dk[o]
            ok = (ii >= 0) & (ii < n) & (jj >= 0) & (jj < n) & (kk >= 0) & (kk < n)
            J = ii + n * jj + (n * n * kk if dim == 3 else 0)
            ref = np.zeros(N)
            ref[ok] = np.asarray(A[rows[ok], J[ok]]).ravel()
            assert np.all(got[~ok, o] == 0.0)
            assert np.abs(got[:, o] - ref).max() <= 1e-13 * scale, (l, o)


@pytest.mark.parametrize("geom,n_el,p", CASES_ALL)
def test_rhs_apply_restrict_prolong_coarse(geom, n_el, p):
    s, H, b = case(geom, n_el, p)
    bd = torch.zeros(s.ndof, dtype=torch.float64, device=DEV)
    s.get_rhs(bd)
    assert rel(host(bd), b) < 1e-13
    L = len(H.levels) - 1
    for l in range(L + 1):
        lev = H.levels[l]
        x = synth.random_vector(lev.A.shape[0], 10 + l)
        y = torch.zeros(len(x), dtype=torch.float64, device=DEV)
        s.apply(l, dev(x), y)
        assert rel(host(y), lev.A @ x) < 1e-13
        if l >= 1:
            nc = H.levels[l - 1].A.shape[0]
            rc = torch.zeros(nc, dtype=torch.float64, device=DEV)
            s.restrict(l, dev(x), rc)
            assert rel(host(rc), lev.P.T @ x) < 1e-14
            e = synth.random_vector(nc, 20 + l)
            xf = dev(x)
            s.prolong_add(l, dev(e), xf)
            assert rel(host(xf), x + lev.P @ e) < 1e-14
    b0 = synth.random_vector(H.levels[0].A.shape[0], 30)
    x0 = torch.zeros(len(b0), dtype=torch.float64, device=DEV)
    s.coarse_solve(dev(b0), x0)
    assert rel(host(x0), H.coarse_solve(b0)) < 1e-12


@pytest.mark.parametrize("geom,n_el,p", CASES_ALL)
def test_multicolour_sweeps(geom, n_el, p):
    s, H, _ = case(geom, n_el, p)
    for l in range(1, len(H.levels)):
        lev = H.levels[l]
        bl = synth.random_vector(lev.A.shape[0], 40 + l)
        x0 = synth.random_vector(lev.A.shape[0], 50 + l)
        xg = dev(x0)
        s.smooth(l, dev(bl), xg, 2)
        xr = mg.smooth(lev, bl, x0.copy(), mg.SMOOTH_MCGS, 2)
        assert rel(host(xg), xr) < 1e-13


# tail = 512: the single-workgroup kernel takes every level whose iterates
# (with those of the coarser levels) fit its LDS store
VCYCLE_CASES = ([(g, n, p, 32) for g, n, p in CASES_ALL] + [(g, n, p, 0) for g, n, p in CASES_ALL] +
                [("annulus", 128, 3, 32), ("square", 128, 2, 32), ("annulus", 64, 5, 32),
                 ("cube", 16, 2, 32), ("annulus", 128, 3, 512), ("square", 128, 2, 512),
                 ("annulus", 64, 5, 512), ("cube", 16, 3, 512), ("annulus", 32, 4, 512)])


@pytest.mark.parametrize("geom,n_el,p,tail", VCYCLE_CASES)
def test_vcycle_iterates(geom, n_el, p, tail):
    """Per-iterate parity of V-cycles; tail = 0 runs every level with
    multi-block launches, tail = 32 runs the small levels in the
    single-workgroup kernel (the larger grids use both paths)."""
    s, H, b = case(geom, n_el, p, tail_items=tail)
    N = len(b)
    xg = torch.zeros(N, dtype=torch.float64, device=DEV)
    xr = np.zeros(N)
    for it in range(6):
        s.vcycle(xg)
        xr = mg.vcycle(H, b, xr)
        assert rel(host(xg), xr) < 1e-12, it


@pytest.mark.parametrize("geom,n_el,p", [("annulus", 32, 3), ("annulus", 16, 5), ("square", 32, 2),
                                         ("cube", 8, 3)])
@pytest.mark.parametrize("method", [igamg.RRE, igamg.MPE])
def test_extrapolated_iterates(geom, n_el, p, method):
    s, H, b = case(geom, n_el, p)
    N = len(b)
    q = 5
    xg = torch.zeros(N, dtype=torch.float64, device=DEV)
    its = torch.zeros((q + 2) * N, dtype=torch.float64, device=DEV)
    x = np.zeros(N)
    om = ex.RRE if method == igamg.RRE else ex.MPE
    for cycle in range(2):
        gam = s.extrapolate(method, q, xg, its)
        S = [x]
        for j in range(q + 1):
            S.append(mg.vcycle(H, b, S[-1]))
        Sg = host(its).reshape(q + 2, N)
        for j in range(q + 2):
            assert rel(Sg[j], S[j]) < 1e-12, (cycle, j)
        t, gr, _ = ex.extrapolate(S, om)
        assert rel(host(xg), t) < 1e-12, cycle
        # gamma itself is ill-determined when Delta S is ill-conditioned (strong
        # contraction); t, compared above, is what the method fixes uniquely
        assert abs(gam.sum() - 1.0) < 1e-12
        x = t


def _linear_sequence(N, q, seed):
    rng = np.random.default_rng(seed)
    lam = rng.uniform(0.3, 0.95, N)
    c = rng.standard_normal(N)
    S = [rng.standard_normal(N)]
    for _ in range(q + 1):
        S.append(lam * S[-1] + c)
    return S


@pytest.mark.parametrize("q", [1, 3, 5, 8])
def test_tsqr_coefficients_tree(q):
    """Tall-skinny QR over several tree levels (N = 1e6 + ragged tail)."""
    if "tsqr" not in _cache:
        print("[case] annulus n_el=1024 p=2 (extrapolation only)", flush=True)
        _cache["tsqr"] = igamg.Solver(igamg.QUARTER_ANNULUS, 1024, 2)
    s = _cache["tsqr"]
    N = s.ndof
    S = _linear_sequence(N, q, q)
    its = dev(np.concatenate(S))
    for method, om in ((igamg.RRE, ex.RRE), (igamg.MPE, ex.MPE)):
        g, info = s.extrap_coeffs(method, q, its)
        _, gr, _ = ex.extrapolate(S, om)
        assert info == 0
        assert np.abs(g - gr).max() < 1e-9 * np.abs(gr).max()


def test_breakdown_rules():
    s, _, _ = case("annulus", 16, 2)
    N = s.ndof
    v = synth.random_vector(N, 1)
    drift = dev(np.concatenate([j * v for j in range(7)]))
    for method in (igamg.RRE, igamg.MPE):
        _, info = s.extrap_coeffs(method, 5, drift)
        assert info == -1
    xs = synth.random_vector(N, 2)
    a, b2 = synth.random_vector(N, 3), synth.random_vector(N, 4)
    lucky = [xs + a, xs + b2, xs, xs, xs, xs, xs]
    for method, om in ((igamg.RRE, ex.RRE), (igamg.MPE, ex.MPE)):
        g, info = s.extrap_coeffs(method, 5, dev(np.concatenate(lucky)))
        _, gr, _ = ex.extrapolate(lucky, om)
        assert info == 1
        np.testing.assert_allclose(g, gr, atol=1e-12)


@pytest.mark.parametrize("geom,n_el,p,tail", [("annulus", 32, 3, 32), ("annulus", 32, 5, 0),
                                              ("square", 64, 2, 32), ("square", 32, 4, 0),
                                              ("cube", 8, 2, 32), ("annulus", 128, 4, 32)])
@pytest.mark.parametrize("method", [igamg.EXTRAP_NONE, igamg.RRE, igamg.MPE])
def test_solve_matches_oracle(geom, n_el, p, tail, method):
    s, H, b = case(geom, n_el, p, tail_items=tail)
    N = len(b)
    A = H.fine.A
    nb = np.linalg.norm(b)
    G = lambda x: mg.vcycle(H, b, x)
    rn = lambda x: np.linalg.norm(b - A @ x) / nb
    om = {igamg.EXTRAP_NONE: None, igamg.RRE: ex.RRE, igamg.MPE: ex.MPE}[method]
    xr, st_r, _ = ex.restarted_solve(G, rn, np.zeros(N), 5, om, tol=1e-10, max_restarts=600)
    xg = torch.zeros(N, dtype=torch.float64, device=DEV)
    st, _ = s.solve(xg, tol=1e-10, max_restarts=600, method=method, q=5)
    x = host(xg)
    assert st.rel_residual <= 1e-10 and rn(x) <= 1.0000001e-10
    assert st.vcycles == st_r.vcycles and st.restarts == st_r.restarts
    assert rel(x, xr) < 1e-11


@pytest.mark.parametrize("geom,n_el,p", [("annulus", 64, 3), ("annulus", 32, 5), ("square", 64, 2),
                                         ("cube", 16, 3)])
@pytest.mark.parametrize("method", [igamg.EXTRAP_NONE, igamg.RRE])
def test_fp32_refinement_reaches_tolerance(geom, n_el, p, method):
    """FP32 V-cycles inside FP64 refinement reach the FP64 tolerance; the error
    against the oracle's exact discrete solution is stated and bounded."""
    import scipy.sparse.linalg as spla
    s, H, b = case(geom, n_el, p, precision=igamg.FP32_IR)
    N = len(b)
    xg = torch.zeros(N, dtype=torch.float64, device=DEV)
    st, _ = s.solve(xg, tol=1e-10, max_restarts=800, method=method, q=5)
    x = host(xg)
    A = H.fine.A
    assert np.linalg.norm(b - A @ x) / np.linalg.norm(b) <= 1.0000001e-10
    u = spla.spsolve(A.tocsc(), b)
    err = rel(x, u)
    print("[fp32-ir] %s n_el=%d p=%d method=%d vcycles=%d err_vs_exact=%.2e"
          % (geom, n_el, p, method, st.vcycles, err))
    assert err < 1e-6


@pytest.mark.parametrize("geom,n_el,p", [("annulus", 128, 3), ("cube", 16, 2), ("annulus", 64, 5),
                                         ("annulus", 64, 4), ("annulus", 64, 1), ("square", 64, 2)])
def test_fp32_large_tail_matches_multiblock(geom, n_el, p):
    """FP32 V-cycles with the small levels in the single-workgroup kernel (its
    LDS store holds twice as many FP32 unknowns) agree with all-multi-block
    FP32 V-cycles to FP32 rounding, and both reach the FP64 tolerance."""
    res = {}
    for tail in (0, 512):
        s, H, b = case(geom, n_el, p, precision=igamg.FP32_IR, tail_items=tail)
        N = len(b)
        xg = torch.zeros(N, dtype=torch.float64, device=DEV)
        for _ in range(3):
            s.vcycle(xg)
        x3 = host(xg)
        xg.zero_()
        st, _ = s.solve(xg, tol=1e-10, max_restarts=400, method=igamg.RRE, q=5)
        A = H.fine.A
        assert np.linalg.norm(b - A @ host(xg)) / np.linalg.norm(b) <= 1.0000001e-10
        res[tail] = (x3, host(xg), st.vcycles)
    assert rel(res[512][0], res[0][0]) < 1e-5
    assert rel(res[512][1], res[0][1]) < 1e-8
    assert abs(res[512][2] - res[0][2]) <= 6


def test_error_paths():
    with pytest.raises(igamg.IgamgError) as e:
        igamg.Solver(igamg.QUARTER_ANNULUS, 12, 3)
    assert e.value.status == igamg.EINVAL
    with pytest.raises(igamg.IgamgError) as e:
        igamg.Solver(igamg.UNIT_CUBE, 8, 4)
    assert e.value.status == igamg.EINVAL
    s, H, b = case("annulus", 32, 4)
    N = len(b)
    xg = torch.zeros(N, dtype=torch.float64, device=DEV)
    st, status = s.solve(xg, tol=1e-10, max_restarts=2, method=igamg.EXTRAP_NONE, check=False)
    assert status == igamg.ENOCONV and st.vcycles == 2 and st.rel_residual > 1e-10
    s2 = igamg.Solver(igamg.QUARTER_ANNULUS, 16, 2)
    bad = np.ones(s2.ndof)
    bad[3] = np.nan
    with pytest.raises(igamg.IgamgError) as e:
        s2.set_rhs(bad)
    assert e.value.status == igamg.ENONFINITE
    with pytest.raises(igamg.IgamgError) as e:
        s.extrapolate(igamg.RRE, 9, xg)
    assert e.value.status == igamg.EINVAL


def test_single_level_is_direct_solve():
    s = igamg.Solver(igamg.QUARTER_ANNULUS, 4, 3)
    H = mg.build_hierarchy("annulus", 4, 3)
    modes = synth.random_field_modes(7)
    s.set_rhs_field(modes)
    b = assemble.load_vector_2d(4, 3, modes)
    xg = torch.zeros(s.ndof, dtype=torch.float64, device=DEV)
    s.vcycle(xg)
    assert rel(host(xg), H.coarse_solve(b)) < 1e-12


@pytest.mark.parametrize("geom,n_el,p", [("square", 32, 2), ("annulus", 16, 3), ("annulus", 16, 5),
                                         ("square", 32, 4)])
def test_lexicographic_sweeps(geom, n_el, p):
    s, H, _ = case(geom, n_el, p, smoother=igamg.SMOOTH_LEXGS)
    for l in range(1, len(H.levels)):
        lev = H.levels[l]
        bl = synth.random_vector(lev.A.shape[0], 60 + l)
        x0 = synth.random_vector(lev.A.shape[0], 70 + l)
        xg = dev(x0)
        s.smooth(l, dev(bl), xg, 2)
        xr = mg.smooth(lev, bl, x0.copy(), mg.SMOOTH_LEXGS, 2)
        assert rel(host(xg), xr) < 1e-13, l


@pytest.mark.parametrize("method", [igamg.EXTRAP_NONE, igamg.RRE, igamg.MPE])
def test_lexicographic_c1_solve(method):
    """The unit-square workload of 64^2 elements, p = 2, lexicographic V(2,2)."""
    s, H, b = case("square", 64, 2, smoother=igamg.SMOOTH_LEXGS)
    N = len(b)
    A = H.fine.A
    nb = np.linalg.norm(b)
    G = lambda x: mg.vcycle(H, b, x, mg.SMOOTH_LEXGS)
    xg = torch.zeros(N, dtype=torch.float64, device=DEV)
    xr = np.zeros(N)
    for it in range(4):
        s.vcycle(xg)
        xr = G(xr)
        assert rel(host(xg), xr) < 1e-12, it
    om = {igamg.EXTRAP_NONE: None, igamg.RRE: ex.RRE, igamg.MPE: ex.MPE}[method]
    xo, st_r, _ = ex.restarted_solve(G, lambda x: np.linalg.norm(b - A @ x) / nb, np.zeros(N), 5, om,
                                     tol=1e-10, max_restarts=200)
    x = torch.zeros(N, dtype=torch.float64, device=DEV)
    st, _ = s.solve(x, tol=1e-10, max_restarts=200, method=method, q=5)
    assert st.vcycles == st_r.vcycles
    assert rel(host(x), xo) < 1e-11


@pytest.mark.parametrize("geom,n_el,p,extra", [("annulus", 64, 1, {}), ("annulus", 64, 2, {}),
                                               ("annulus", 128, 3, {}), ("annulus", 32, 4, {}),
                                               ("annulus", 64, 5, {}), ("square", 64, 2, {"stored_stencil": 1}),
                                               ("annulus", 1024, 3, {})])
@pytest.mark.parametrize("prec", [igamg.FP64, igamg.FP32_IR])
def test_row_class_sweeps_equal_colour_passes(geom, n_el, p, extra, prec):
    """Sweeping the p+1 colours of a row class in one launch gives the same
    V-cycle iterates, bit for bit, as one launch per colour (every level
    multi-block, so every level's sweeps go through the kernel under test)."""
    out = []
    for rows in (0, 1):
        print("[rows] %s n_el=%d p=%d prec=%d rows=%d" % (geom, n_el, p, prec, rows), flush=True)
        s = igamg.Solver(GEOM[geom], n_el, p, tail_items=0, precision=prec, row_sweeps=rows, **extra)
        s.set_rhs_field(modes_for(geom, 2000 + p))
        x = torch.zeros(s.ndof, dtype=torch.float64, device=DEV)
        for _ in range(2 if n_el >= 1024 else 3):
            s.vcycle(x)
        out.append(host(x))
        s.close()
    assert np.array_equal(out[0], out[1])


def _with_shape(s, shape):
    """Sets every level's sweep launch shape (0 per colour, 1 per row class,
    2 per plane class where it applies: cubes) and the multi-block split 0."""
    t = s.tuning()
    t["tail_items"] = 0
    t["row_class"] = [shape] * t["num_levels"]
    s.set_tuning(t)
    return s.tuning()["row_class"]


KRON_ROW_CASES = ([("cube", n, p) for n, p in [(16, 1), (32, 1), (16, 2), (32, 2), (16, 3), (32, 3)]] +
                  [("square", n, p) for n, p in [(16, 1), (64, 2), (32, 3), (16, 4), (32, 5)]])


@pytest.mark.parametrize("geom,n_el,p", KRON_ROW_CASES)
def test_kron_row_class_sweeps_and_products(geom, n_el, p):
    """Sum-factorised levels (unit square and cube): the row-class sweep (one
    launch per row class, j (and k) fixed mod p+1, each row's product factored
    through the y (and z) bands), on the cube also the plane-class sweep (one
    launch per plane class, one workgroup per plane), and the
    one-workgroup-per-row products (A x, damped Jacobi) equal the oracle's
    multicolour sweeps, A x and Jacobi steps on every level (1e-13), as do the
    per-colour kernels.  Row- and plane-class sweeps are equal bit for bit; the
    per-colour kernels sum in another order and agree with them to the same
    bar.  With n = n_el + p - 2 unknowns per direction most levels leave ragged
    classes (n not a multiple of p + 1)."""
    H = mg.build_hierarchy(geom, n_el, p)
    got = {}
    for rows in (0, 1):
        s = igamg.Solver(GEOM[geom], n_el, p, tail_items=0, row_sweeps=rows)
        sj = igamg.Solver(GEOM[geom], n_el, p, tail_items=0, row_sweeps=rows, smoother=igamg.SMOOTH_JACOBI)
        shapes = (0,) if rows == 0 else ((1, 2) if geom == "cube" else (1,))
        for shape in shapes:
            print("[kron shapes] %s n_el=%d p=%d rows=%d shape=%d" % (geom, n_el, p, rows, shape), flush=True)
            used = _with_shape(s, shape)
            if shape == 2:
                assert 2 in used  # the plane-class kernel applies on the finest level at least
            for l in range(1, len(H.levels)):
                lev = H.levels[l]
                N = lev.A.shape[0]
                bl = synth.random_vector(N, 140 + l)
                x0 = synth.random_vector(N, 150 + l)
                xg = dev(x0)
                s.smooth(l, dev(bl), xg, 2)
                xr = mg.smooth(lev, bl, x0.copy(), mg.SMOOTH_MCGS, 2)
                assert rel(host(xg), xr) < 1e-13, (shape, l)
                y = torch.zeros(N, dtype=torch.float64, device=DEV)
                s.apply(l, dev(x0), y)
                assert rel(host(y), lev.A @ x0) < 1e-13, (shape, l)
                xj = dev(x0)
                sj.smooth(l, dev(bl), xj, 2)
                assert rel(host(xj), mg.smooth(lev, bl, x0.copy(), mg.SMOOTH_JACOBI, 2)) < 1e-13, (shape, l)
                got[shape, l] = (host(xg), host(y), host(xj))
        s.close()
        sj.close()
    for l in range(1, len(H.levels)):
        if geom == "cube":
            assert all(np.array_equal(a, b) for a, b in zip(got[1, l], got[2, l])), l
        for a, b in zip(got[0, l], got[1, l]):
            assert rel(b, a) < 1e-13, l


def _cube_apply(n_el, p, x):
    """A x and diag(A) for the unit-cube operator K(x)M(x)M + M(x)K(x)M +
    M(x)M(x)K (first factor on k, x index fastest), from the oracle's 1D
    stiffness and mass matrices by dense tensor contractions (grids too large
    for the assembled matrix)."""
    K, M = (np.asarray(a.todense()) if hasattr(a, "todense") else np.asarray(a)
            for a in bspline.stiffness_mass_1d(n_el, p))
    n = K.shape[0]
    X = x.reshape(n, n, n)
    ax = lambda F, Y: Y @ F.T                            # along i
    ay = lambda F, Y: np.matmul(F, Y)                    # along j
    az = lambda F, Y: np.tensordot(F, Y, axes=(1, 0))    # along k
    Xm = ax(M, X)
    y = az(K, ay(M, Xm)) + az(M, ay(K, Xm)) + az(M, ay(M, ax(K, X)))
    kd, md = np.diag(K), np.diag(M)
    d = (kd[:, None, None] * md[None, :, None] * md[None, None, :] +
         md[:, None, None] * kd[None, :, None] * md[None, None, :] +
         md[:, None, None] * md[None, :, None] * kd[None, None, :])
    return y.ravel(), d.ravel()


@pytest.mark.parametrize("n_el,p", [(96, 2), (96, 3), (128, 1), (128, 3)])
def test_cube_products_rolling_planes(n_el, p):
    """The products of the large 3D levels (one workgroup per x-row and run
    of 8 planes, the y-contractions of the planes kept in a window as the
    plane advances): A x, the damped Jacobi step and the relative residual
    from the per-row sums of squares equal the operator's definition applied
    to random vectors (1e-13).  n = 96 (whole runs), 97 and 129 (a last run of
    one plane, shorter than the window of 2p+1 planes), 127 (a last run of
    seven)."""
    n = n_el + p - 2
    N = n ** 3
    x = synth.random_vector(N, 170 + p)
    b = synth.random_vector(N, 171 + p)
    Ax, d = _cube_apply(n_el, p, x)
    print("[cube rolling] n_el=%d p=%d" % (n_el, p), flush=True)
    s = igamg.Solver(igamg.UNIT_CUBE, n_el, p, n_el_coarsest=0)
    fine = s.num_levels - 1
    assert s.level_ndof(fine) == N
    y = torch.zeros(N, dtype=torch.float64, device=DEV)
    s.apply(fine, dev(x), y)
    assert rel(host(y), Ax) < 1e-13
    s.set_rhs(dev(b))
    ref = np.linalg.norm(b - Ax) / np.linalg.norm(b)
    got = s.residual(dev(x))
    assert abs(got - ref) <= 1e-13 * ref
    s.close()
    sj = igamg.Solver(igamg.UNIT_CUBE, n_el, p, n_el_coarsest=0, smoother=igamg.SMOOTH_JACOBI)
    xj = dev(x)
    sj.smooth(fine, dev(b), xj, 1)
    assert rel(host(xj), x + (2.0 / 3.0) * (b - Ax) / d) < 1e-13
    sj.close()


@pytest.mark.parametrize("prec,method", [(igamg.FP32_IR, igamg.MPE), (igamg.FP64, igamg.RRE)])
def test_cube_large_solve_reaches_tolerance(prec, method):
    """A 97^3 cube (n_el = 96, p = 3: the residuals of the finest level by the
    windowed kernel, FP64 in and FP32 out for the refinement's right-hand side)
    solved to 1e-10 from zero for a random right-hand side: the relative
    residual of the returned x, recomputed on the host from the operator's
    Kronecker definition, is within the tolerance (up to the rounding of the
    two computations)."""
    n_el, p = 96, 3
    n = n_el + p - 2
    b = synth.random_vector(n ** 3, 181)
    print("[cube large solve] prec=%d method=%d" % (prec, method), flush=True)
    s = igamg.Solver(igamg.UNIT_CUBE, n_el, p, n_el_coarsest=0, precision=prec)
    s.set_rhs(dev(b))
    x = torch.zeros(n ** 3, dtype=torch.float64, device=DEV)
    st, _ = s.solve(x, tol=1e-10, max_restarts=200, method=method, q=4)
    s.close()
    Ax, _ = _cube_apply(n_el, p, host(x))
    got = np.linalg.norm(b - Ax) / np.linalg.norm(b)
    print("[cube large solve] vcycles=%d restarts=%d rel=%.3e host=%.3e"
          % (st.vcycles, st.restarts, st.rel_residual, got), flush=True)
    assert st.rel_residual <= 1e-10
    assert got <= 1.0001e-10


@pytest.mark.parametrize("n_el,p", [(32, 1), (32, 2), (32, 3), (64, 2), (64, 3)])
@pytest.mark.parametrize("prec", [igamg.FP64, igamg.FP32_IR])
def test_cube_plane_class_equals_row_class_bitwise(n_el, p, prec):
    """V-cycles with every cube level multi-block: one launch per plane class
    (where it applies: at most 64 unknowns per direction, with the 2p+1
    planes of x, the plane of b and the bands in LDS, so the 64^3 level of
    n_el = 64, p = 2 in FP32 but not in FP64, and not the 65^3 one of p = 3)
    gives the iterates of one launch per row class bit for bit.  (n = 64 also
    checks the rows' zero pads when no thread lies past the row's last
    point.)"""
    out = []
    for shape in (1, 2):
        print("[cube plane] n_el=%d p=%d prec=%d shape=%d" % (n_el, p, prec, shape), flush=True)
        s = igamg.Solver(igamg.UNIT_CUBE, n_el, p, precision=prec)
        s.set_rhs_field(modes_for("cube", 2000 + p))
        used = _with_shape(s, shape)
        assert (2 in used) == (shape == 2)
        x = torch.zeros(s.ndof, dtype=torch.float64, device=DEV)
        for _ in range(3):
            s.vcycle(x)
        out.append(host(x))
        s.close()
    assert np.all(np.isfinite(out[0]))
    assert np.array_equal(out[0], out[1])


@pytest.mark.parametrize("geom,n_el,p", [("cube", 16, 1), ("cube", 16, 2), ("cube", 16, 3), ("cube", 32, 3),
                                         ("square", 64, 2), ("square", 32, 3), ("square", 16, 5)])
@pytest.mark.parametrize("prec", [igamg.FP64, igamg.FP32_IR])
@pytest.mark.parametrize("mu", [1, 2])
def test_kron_tail_equals_multiblock_bitwise(geom, n_el, p, prec, mu):
    """Sum-factorised levels in the single-workgroup kernel (rows of at most 64
    unknowns) sweep in row classes with the arithmetic of the multi-block
    row-class kernels (same contraction and summation order; the same
    transfers and coarse solve), so V- and W-cycle iterates with the small
    levels in one workgroup equal, bit for bit, those with every level
    multi-block."""
    out = []
    for tail in (0, 512):
        print("[kron tail] %s n_el=%d p=%d prec=%d mu=%d tail=%d" % (geom, n_el, p, prec, mu, tail), flush=True)
        s = igamg.Solver(GEOM[geom], n_el, p, tail_items=tail, precision=prec, mu=mu)
        s.set_rhs_field(modes_for(geom, 2000 + p))
        assert (s.tuning()["tail_top"] >= 2) == (tail > 0)
        x = torch.zeros(s.ndof, dtype=torch.float64, device=DEV)
        for _ in range(3):
            s.vcycle(x)
        out.append(host(x))
        s.close()
    assert np.array_equal(out[0], out[1])
