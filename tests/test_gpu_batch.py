"""Batched solves: every problem of a batch must equal its standalone solve
(same kernels, same order) and reach the tolerance by its true residual; the
unit-square stored-stencil form must equal the Kronecker form."""
import numpy as np
import pytest
import torch

import synth
from oracle import assemble
from paper_2412_20205_amd import igamg

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

PROBLEMS = [(igamg.QUARTER_ANNULUS, 32, 3), (igamg.UNIT_SQUARE, 40, 2), (igamg.QUARTER_ANNULUS, 56, 5),
            (igamg.UNIT_SQUARE, 48, 4), (igamg.QUARTER_ANNULUS, 80, 2), (igamg.UNIT_SQUARE, 112, 5),
            (igamg.QUARTER_ANNULUS, 64, 4), (igamg.QUARTER_ANNULUS, 28 * 4, 3)]


def test_stored_stencil_square_equals_kronecker():
    a = igamg.Solver(igamg.UNIT_SQUARE, 32, 3)
    b = igamg.Solver(igamg.UNIT_SQUARE, 32, 3, stored_stencil=1)
    for l in range(a.num_levels):
        rows = np.arange(a.level_ndof(l))
        assert np.abs(a.operator_rows(l, rows) - b.operator_rows(l, rows)).max() < 1e-15 * 100


def test_batch_equals_standalone_and_converges():
    print("[case] batch of %d" % len(PROBLEMS), flush=True)
    B = igamg.Batch(PROBLEMS)
    xs = []
    for i, (g, e, d) in enumerate(PROBLEMS):
        B.instances[i].set_rhs_field(synth.random_field_modes(4000 + i))
        xs.append(torch.zeros(B.instances[i].ndof, dtype=torch.float64, device=DEV))
    stats, _ = B.solve(xs, tol=1e-10, max_restarts=60, q=5)
    for i, (g, e, d) in enumerate(PROBLEMS):
        rel = B.instances[i].residual(xs[i])
        s = igamg.Solver(g, e, d, precision=igamg.FP32_IR, stored_stencil=1, tail_items=32,
                         n_el_coarsest=0)
        s.set_rhs_field(synth.random_field_modes(4000 + i))
        x = torch.zeros(s.ndof, dtype=torch.float64, device=DEV)
        st, _ = s.solve(x, tol=1e-10, max_restarts=60, method=igamg.RRE, q=5)
        diff = (torch.linalg.norm(x - xs[i]) / torch.linalg.norm(x)).item()
        print("[batch] problem %d geom=%d n_el=%d p=%d restarts=%d/%d rel=%.2e diff=%.1e"
              % (i, g, e, d, stats[i].restarts, st.restarts, rel, diff))
        assert rel <= 1.0000001e-10
        assert stats[i].restarts == st.restarts
        assert diff < 1e-13
    # true residual by the oracle for two problems
    for i in (0, 1):
        g, e, d = PROBLEMS[i]
        if g == igamg.QUARTER_ANNULUS:
            A = assemble.mapped_stiffness_2d(e, d)
            bb = assemble.load_vector_2d(e, d, synth.random_field_modes(4000 + i))
        else:
            A = assemble.kron_operator_2d(e, d)
            bb = assemble.kron_load_2d(e, d, synth.random_field_modes(4000 + i))
        xv = xs[i].cpu().numpy()
        assert np.linalg.norm(bb - A @ xv) / np.linalg.norm(bb) <= 1.0000001e-10
    B.close()


def test_autotune_choice_is_cached_and_used():
    s = igamg.Solver(igamg.QUARTER_ANNULUS, 128, 4)
    items, ms = s.autotune()
    tu = s.tuning()
    print("[autotune] annulus 128 p=4 -> tail_items=%d (%.3f ms per V-cycle) %s" % (items, ms, tu))
    assert items in (0, 8, 16, 32, 64, 128, 256, 512) and ms > 0
    assert tu["tail_items"] == items and tu["vcycle_ms"] == ms and tu["num_levels"] == s.num_levels
    assert set(tu["row_class"]) <= {0, 1} and set(tu["learned_kernel"]) <= {0, 12, 28, 29}
    t = igamg.Solver(igamg.QUARTER_ANNULUS, 128, 4, tail_items=-1)
    assert t.options.tail_items == -1  # resolved inside the library
    assert t.tuning() == tu  # every tuned shape comes from the cache
    modes = synth.random_field_modes(77)
    for solver in (s, t):
        solver.set_rhs_field(modes)
    xa = torch.zeros(s.ndof, dtype=torch.float64, device=DEV)
    xb = torch.zeros(t.ndof, dtype=torch.float64, device=DEV)
    sa, _ = s.solve(xa, tol=1e-10, method=igamg.RRE, q=5)
    sb, _ = t.solve(xb, tol=1e-10, method=igamg.RRE, q=5)
    assert sa.vcycles == sb.vcycles
    assert torch.equal(xa, xb)
    # the sweep launch shape changes times, not iterates: flipping every
    # level's row-class choice gives the same solve bit for bit
    u = dict(tu, row_class=[1 - r for r in tu["row_class"]])
    t.set_tuning(u)
    xc = torch.zeros(t.ndof, dtype=torch.float64, device=DEV)
    sc, _ = t.solve(xc, tol=1e-10, method=igamg.RRE, q=5)
    assert sc.vcycles == sa.vcycles
    assert torch.equal(xc, xa)


def test_batch_row_class_sweeps_equal_colour_launches():
    """The batched row-class sweep (one launch per row class for every problem
    of a degree, a workgroup per row) gives the iterates of one launch per
    colour, bit for bit, and the same counts."""
    out = []
    for rows in (0, 1):
        print("[batch rows] row_sweeps=%d" % rows, flush=True)
        B = igamg.Batch(PROBLEMS, row_sweeps=rows)
        xs = []
        for i in range(len(PROBLEMS)):
            B.instances[i].set_rhs_field(synth.random_field_modes(4100 + i))
            xs.append(torch.zeros(B.instances[i].ndof, dtype=torch.float64, device=DEV))
        stats, _ = B.solve(xs, tol=1e-10, max_restarts=60, q=5)
        out.append(([x.cpu().numpy() for x in xs], [(st.restarts, st.vcycles) for st in stats]))
        B.close()
    for a, b in zip(out[0][0], out[1][0]):
        assert np.array_equal(a, b)
    assert out[0][1] == out[1][1]
