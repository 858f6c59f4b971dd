"""The generalised residual t~ - t of eq. (11) from the library's R factor, and
the solve mode that uses it as a monitor (no product with A until it predicts
convergence), against the oracle and against one more application of G."""
import numpy as np
import pytest
import torch

from oracle import extrapolation as ex, multigrid as mg
from paper_2412_20205_amd import igamg

from test_gpu_parity import DEV, case, host, rel

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("geom,n_el,p", [("annulus", 32, 3), ("square", 32, 2), ("cube", 8, 2)])
@pytest.mark.parametrize("method", [igamg.RRE, igamg.MPE])
def test_generalized_residual_matches_oracle_and_one_vcycle(geom, n_el, p, method):
    s, H, b = case(geom, n_el, p)
    N = len(b)
    q = 5
    xg = torch.zeros(N, dtype=torch.float64, device=DEV)
    its = torch.zeros((q + 2) * N, dtype=torch.float64, device=DEV)
    gam = s.extrapolate(method, q, xg, its)
    g_gpu = s.generalized_residual()
    Sg = list(host(its).reshape(q + 2, N))
    # oracle: the same iterates, its own gamma and t~ - t
    S = [np.zeros(N)]
    for j in range(q + 1):
        S.append(mg.vcycle(H, b, S[-1]))
    om = ex.RRE if method == igamg.RRE else ex.MPE
    t, gamma, _ = ex.extrapolate(S, om)
    g_orc = np.linalg.norm(ex.generalized_residual(S, gamma))
    d0 = np.linalg.norm(S[1] - S[0])
    assert abs(g_gpu - g_orc) <= 1e-9 * d0
    # the V-cycle is an affine map: t~ - t = G(t) - t
    t_gpu = host(xg)
    s.vcycle(xg)
    g_map = np.linalg.norm(host(xg) - t_gpu)
    assert abs(g_gpu - g_map) <= 1e-9 * d0 + 1e-6 * g_map


@pytest.mark.parametrize("geom,n_el,p,prec", [("annulus", 64, 3, igamg.FP64), ("annulus", 64, 5, igamg.FP64),
                                              ("annulus", 128, 3, igamg.FP32_IR), ("cube", 16, 3, igamg.FP64)])
def test_monitor_solve_reaches_tolerance_with_fewer_residuals(geom, n_el, p, prec):
    base, H, b = case(geom, n_el, p, precision=prec)
    mon, _, _ = case(geom, n_el, p, precision=prec, monitor=1)
    N = len(b)
    x0 = torch.zeros(N, dtype=torch.float64, device=DEV)
    x1 = torch.zeros(N, dtype=torch.float64, device=DEV)
    st0, _ = base.solve(x0, tol=1e-10, max_restarts=400, method=igamg.RRE, q=5)
    st1, _ = mon.solve(x1, tol=1e-10, max_restarts=400, method=igamg.RRE, q=5)
    A = H.fine.A
    assert np.linalg.norm(b - A @ host(x1)) / np.linalg.norm(b) <= 1.0000001e-10
    assert st1.rel_residual <= 1e-10
    # same iterates until the stop; at most one more cycle than testing every cycle
    assert st0.restarts <= st1.restarts <= st0.restarts + 1
    assert st1.residual_checks <= st1.restarts
    assert st0.residual_checks == st0.restarts
    if st1.restarts == st0.restarts:
        assert rel(host(x1), host(x0)) < 1e-13
    assert 0.0 < st1.gen_residual < 1e-6
