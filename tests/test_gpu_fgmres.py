"""Flexible GMRES preconditioned by one V-cycle or by one RRE/MPE restart cycle
(the extrapolated cycle as a preconditioner), against the oracle's FGMRES with
the same preconditioners: iterates after a fixed number of steps to 1e-12
relative (the FP64 per-iterate bar; measured 1.3e-15 to 4.6e-15, while a
one-ulp change of b moves the oracle's own iterates by up to 1.4e-15), and
solves to 1e-10 with exactly the oracle's iteration counts and x within 1e-12."""
import numpy as np
import pytest
import torch

from oracle import elliptic as el, extrapolation as ex, krylov
from paper_2412_20205_amd import igamg

from test_gpu_elliptic import case as ell_case
from test_gpu_parity import DEV, case, host, rel

pytestmark = pytest.mark.gpu

PRE = {igamg.PRECOND_VCYCLE: None, igamg.PRECOND_RRE: ex.RRE, igamg.PRECOND_MPE: ex.MPE}


def _problem(kind, n_el, p):
    if kind == "annulus":
        return case("annulus", n_el, p)
    return ell_case(kind, n_el, p)


@pytest.mark.parametrize("kind,n_el,p", [("annulus", 32, 3), ("square1", 32, 2), ("exact2", 32, 3)])
@pytest.mark.parametrize("precond", [igamg.PRECOND_VCYCLE, igamg.PRECOND_RRE, igamg.PRECOND_MPE])
def test_fixed_iterations_match_oracle(kind, n_el, p, precond):
    s, H, b = _problem(kind, n_el, p)
    A = H.fine.A
    M = krylov.extrapolated_cycle(H, 3, PRE[precond])
    for k in (1, 3, 5):
        xg = torch.zeros(len(b), dtype=torch.float64, device=DEV)
        st, status = s.solve_fgmres(xg, tol=1e-300, max_iters=k, m=20, precond=precond, q=3, check=False)
        assert status == igamg.ENOCONV and st.restarts == k
        xr, it = krylov.fgmres(A, b, M, m=20, fixed_iters=k)
        assert rel(host(xg), xr) < 1e-12, k


@pytest.mark.parametrize("kind,n_el,p", [("annulus", 64, 3), ("square1", 64, 3), ("exact2", 64, 4)])
@pytest.mark.parametrize("precond", [igamg.PRECOND_VCYCLE, igamg.PRECOND_RRE])
def test_solve_matches_oracle_counts(kind, n_el, p, precond):
    s, H, b = _problem(kind, n_el, p)
    A = H.fine.A
    xr, it = krylov.fgmres(A, b, krylov.extrapolated_cycle(H, 3, PRE[precond]), tol=1e-10, m=20)
    xg = torch.zeros(len(b), dtype=torch.float64, device=DEV)
    st, _ = s.solve_fgmres(xg, tol=1e-10, max_iters=200, m=20, precond=precond, q=3)
    x = host(xg)
    assert np.linalg.norm(b - A @ x) / np.linalg.norm(b) <= 1.0000001e-10
    assert st.restarts == it
    assert rel(x, xr) < 1e-12
    assert st.vcycles == st.restarts * (1 if precond == igamg.PRECOND_VCYCLE else 4)


def test_fgmres_argument_errors():
    s, _, b = case("annulus", 16, 2)
    x = torch.zeros(len(b), dtype=torch.float64, device=DEV)
    for kw in ({"m": 0}, {"m": 31}, {"precond": 7}, {"precond": igamg.PRECOND_RRE, "q": 0}):
        args = dict(tol=1e-10, max_iters=10, m=10, precond=igamg.PRECOND_VCYCLE, q=3)
        args.update(kw)
        with pytest.raises(igamg.IgamgError):
            s.solve_fgmres(x, **args)
