"""Benchmark: time to a 1e-10 relative residual on the quarter-annulus workload.

Workload: Poisson problem on the quarter annulus (radii 1 and 2, degree-2
B-spline map), B-spline degree p in {3, 4, 5}, 1024 x 1024 elements, stored
(2p+1)^2 stencils, 9-level dyadic hierarchy (coarsest 4 x 4 elements, FP64
Cholesky), V(2,2) multicolour Gauss-Seidel, seeded random-field right-hand
side (64 sine modes, seed 2000 + p), x_0 = 0.

A step is one complete solve to ||b - A x||_2 / ||b||_2 <= 1e-10 with the
right-hand side already on the device.  Forms timed per degree:
  plain_fp64  -- plain FP64 V-cycles, residual tested after each one;
  rre_fp64    -- restarted RRE(5) around FP64 V-cycles;
  ir_rre      -- restarted RRE(5) around FP32 V-cycles inside FP64 refinement;
  chosen      -- ir_rre with the learned smoother (headline degree p = 3: per-level
                 networks trained on the device before timing, on residual/target
                 pairs from plain V-cycles with RHS seeds 5000..5015, accepted by the
                 measured contraction on seed 5900; other degrees: ir_rre).
`value` is the chosen form's ms per solve at the headline degree.

Extra legs (not timed into `value`): the unit square 64^2 p = 2 and the unit
cube 128^3 p = 3 workloads, the batch of 96 problems, the paper's own 2D
setting of Table 11 (64^2 elements, 4 levels, weighted Jacobi V(1,1)/W(1,1),
plain and RRE/MPE, p = 1..5, relative residual 1e-12), the full elliptic
problems of Section 4.3 (Tables 13-15; RRE(8)) and the 1D model problem
(Tables 1 and 4).  Each leg and the per-degree results are written as one JSON
object per line to stderr and, together, to the detail file (--detail-out);
stdout carries exactly one compact JSON line, the last one.

The roofline entry is the finest-level smoother of the chosen form (the
HBM-bound kernel): one row-class launch of the finest-level FP32 multicolour
Gauss-Seidel (the p+1 colours of the rows j = r mod p+1), timed live with HIP
events around a replayed graph of sweeps (igamg_profile_smoother).  The CPU
baseline is the FP64 oracle's own restarted RRE(5) solve of the same workload
on the host.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
       python bench.py --only-smoother --degree P   (kernel profiling runs)
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Counter-derived HBM traffic per launch of the finest-level row-class sweep (FETCH_SIZE x 2.0
# + WRITE_SIZE, calibrated on a 1 GiB copy), from the committed counter profile of that
# kernel.  Valid only for the kernel as profiled; entries are removed when the kernel changes.
MEASURED_TRAFFIC = {(3, "double"): 119.70e6, (3, "float"): 58.67e6}
TOL = 1e-10
Q = 5
N_EL = 1024
METRIC = "ms to 1e-10 rel. residual + smoother HBM GB/s, plain FP64 vs chosen form"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def dof_updates(s, vcycles, nu):
    tot = 0
    for l in range(1, s.num_levels):
        tot += s.level_ndof(l)
    return tot * nu * vcycles


def time_form(s, igamg, torch, method, precision, steps, warmup, learned=False, trained=False):
    s.set_precision(precision)
    if trained:
        s.set_learned(learned)
    x = torch.zeros(s.ndof, dtype=torch.float64, device="cuda:0")
    for _ in range(warmup):
        x.zero_()
        s.solve(x, tol=TOL, max_restarts=2000, method=method, q=Q)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = None
    for _ in range(steps):
        x.zero_()
        st, _ = s.solve(x, tol=TOL, max_restarts=2000, method=method, q=Q)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    return ms, st, x.clone()


def smoother_roofline(s, igamg, precision, nsweeps=8):
    L = s.num_levels - 1
    ms, by, n = s.profile_smoother(L, precision, nsweeps)
    gbs = by / (ms * 1e-3) / 1e9
    tname = "double" if precision == igamg.FP64 else "float"
    p = s.degree
    if n == nsweeps * (p + 1):
        kernel = "k_gs_rowclass<Stencil2D<%d,%s>> (finest level; the p+1 colours of a row " \
                 "class per launch)" % (p, tname)
        traffic = MEASURED_TRAFFIC.get((p, tname))
    else:
        kernel = "k_gs_colour_sliced<Stencil2D<%d,%s>> (finest level; one colour per launch)" \
                 % (p, tname)
        traffic = None
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": kernel,
            "avg_launch_us": round(ms * 1e3, 3), "bytes_per_launch": int(by), "launches": n}


def batch_measure(igamg, torch, synth, steps, warmup, sequential=True):
    """96 independent 2D problems (seeded sizes 32^2..512^2, p in 2..5, square or
    annulus, RHS seed 4000 + i) solved by one batch, RRE(5) around FP32 V-cycles
    in FP64 refinement; the same problems solved one after another beside it
    (unless not sequential)."""
    probs = synth.batch_instances(96, 4)
    geo = {0: igamg.UNIT_SQUARE, 1: igamg.QUARTER_ANNULUS}
    t0 = time.perf_counter()
    B = igamg.Batch([(geo[g], ne, p) for ne, p, g, _ in probs], tail_items=-1)
    setup_s = time.perf_counter() - t0
    xs = []
    ndof = 0
    for i, (ne, p, g, seed) in enumerate(probs):
        B.instances[i].set_rhs_field(synth.random_field_modes(seed))
        xs.append(torch.zeros(B.instances[i].ndof, dtype=torch.float64, device="cuda:0"))
        ndof += B.instances[i].ndof
    for _ in range(warmup):
        for x in xs:
            x.zero_()
        B.solve(xs, tol=TOL, max_restarts=200, q=Q)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for x in xs:
            x.zero_()
        stats, _ = B.solve(xs, tol=TOL, max_restarts=200, q=Q)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    worst = max(B.instances[i].residual(xs[i]) for i in range(len(xs)))
    upd = 0
    for i, st in enumerate(stats):
        inst = B.instances[i]
        upd += sum(inst.level_ndof(l) for l in range(1, inst.num_levels)) * 4 * st.vcycles
    B.close()
    if not sequential:
        return {"problems": len(probs), "ndof": ndof, "batch_ms": round(ms, 2),
                "max_restarts": max(st.restarts for st in stats), "setup_s": round(setup_s, 2)}
    # the same problems one by one (default single-problem path)
    seq_ms = 0.0
    for i, (ne, p, g, seed) in enumerate(probs):
        s = igamg.Solver(geo[g], ne, p, precision=igamg.FP32_IR, n_el_coarsest=0, tail_items=-1)
        s.set_rhs_field(synth.random_field_modes(seed))
        x = torch.zeros(s.ndof, dtype=torch.float64, device="cuda:0")
        s.solve(x, tol=TOL, max_restarts=200, method=igamg.RRE, q=Q)
        x.zero_()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        s.solve(x, tol=TOL, max_restarts=200, method=igamg.RRE, q=Q)
        torch.cuda.synchronize()
        seq_ms += (time.perf_counter() - t1) * 1e3
        s.close()
    return {"problems": len(probs), "ndof": ndof, "batch_ms": round(ms, 2),
            "split": "autotuned per (geometry, degree, grid)",
            "sequential_ms": round(seq_ms, 2), "speedup": round(seq_ms / ms, 2),
            "dof_updates_per_s": round(upd / (ms * 1e-3), 1),
            "max_restarts": max(s.restarts for s in stats), "worst_rel_residual": worst,
            "setup_s": round(setup_s, 2)}


def c1_measure(igamg, torch, synth, steps, forms=None, tuning=None):
    """Unit square, p = 2, 64^2 elements, f = 2 pi^2 sin(pi x) sin(pi y), FP64:
    {multicolour, lexicographic} V(2,2) x {plain, RRE(5), MPE(5)} (forms: a
    subset of their names, e.g. "mcgs_rre5")."""
    out = {}
    for sm_name, sm in (("mcgs", igamg.SMOOTH_MCGS), ("lexgs", igamg.SMOOTH_LEXGS)):
        if forms is not None and not any(f.startswith(sm_name) for f in forms):
            continue
        s = igamg.Solver(igamg.UNIT_SQUARE, 64, 2, smoother=sm)
        s.set_rhs_field(synth.manufactured_sine_modes_2d())
        if sm == igamg.SMOOTH_MCGS:
            if tuning is not None:  # launch shapes given (profiled runs)
                s.set_tuning(tuning)
            else:
                s.autotune()  # sweep launch shapes and the single-workgroup split
            out["mcgs_tuning"] = s.tuning()
        for m_name, m in (("plain", igamg.EXTRAP_NONE), ("rre5", igamg.RRE), ("mpe5", igamg.MPE)):
            if forms is not None and "%s_%s" % (sm_name, m_name) not in forms:
                continue
            ms, st, _ = time_form(s, igamg, torch, m, igamg.FP64, steps, 1)
            out["%s_%s" % (sm_name, m_name)] = {"ms": round(ms, 3), "vcycles": st.vcycles,
                                                "restarts": st.restarts,
                                                "rel_residual": st.rel_residual}
        s.close()
    return out


# Iteration counts printed in Table 11 (2D Poisson, 64 x 64 elements, V(1,1)
# weighted Jacobi with omega = 2/3, tolerance 1e-12): V-cycle, W-cycle, and
# restart cycles of RRE(q) and MPE(q) with q = 4 (p <= 2) or 8 (p >= 3).
PAPER_TABLE11_ITER = {1: (10, 4, 2, 2), 2: (13, 9, 2, 2), 3: (49, 33, 3, 3), 4: (161, 108, 5, 5),
                      5: (466, 352, 8, 8)}


def paper_setting_measure(igamg, torch, synth, steps):
    """The paper's own 2D setting (Section 4.2, Table 11): unit square, 64^2
    elements, 4 levels, weighted Jacobi V(1,1)/W(1,1), f of the model problem
    with exact u = sin(2 pi x) sin(2 pi y), relative residual 1e-12, FP64.
    Reports V-cycle counts, restart counts and ms per solve beside the
    paper's printed counts (its stopping norm is not stated; context only)."""
    out = {}
    for p in range(1, 6):
        q = 4 if p <= 2 else 8
        row = {"q": q, "paper_iter": dict(zip(("v", "w", "rre", "mpe"), PAPER_TABLE11_ITER[p]))}
        for name, mu, m in (("v", 1, igamg.EXTRAP_NONE), ("w", 2, igamg.EXTRAP_NONE),
                            ("rre", 1, igamg.RRE), ("mpe", 1, igamg.MPE)):
            s = igamg.Solver(igamg.UNIT_SQUARE, 64, p, levels=4, smoother=igamg.SMOOTH_JACOBI,
                             nu1=1, nu2=1, mu=mu)
            s.set_rhs_field(synth.poisson_2d_sine_modes(1))
            x = torch.zeros(s.ndof, dtype=torch.float64, device="cuda:0")
            s.solve(x, tol=1e-12, max_restarts=5000, method=m, q=q)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                x.zero_()
                st, _ = s.solve(x, tol=1e-12, max_restarts=5000, method=m, q=q)
            torch.cuda.synchronize()
            row[name] = {"ms": round((time.perf_counter() - t0) * 1e3 / steps, 3), "vcycles": st.vcycles,
                         "restarts": st.restarts, "rel_residual": st.rel_residual}
            s.close()
        out["p%d" % p] = row
    return out


# Table 4 (1D, N = 64): V-cycle, W-cycle, RRE(q), MPE(q) iteration counts and the
# paper's CPU seconds, p = 2..8 (q = 4 for p <= 3, 8 above).
PAPER_TABLE4 = {2: ((6, 4, 2, 2), (0.27, 0.39, 0.30, 0.29)), 3: ((10, 7, 2, 2), (0.74, 1.01, 0.68, 0.71)),
                4: ((20, 14, 2, 2), (2.21, 4.15, 1.79, 1.32)), 5: ((40, 27, 2, 3), (7.13, 9.28, 3.56, 3.83)),
                6: ((81, 54, 4, 4), (19.31, 27.85, 6.37, 6.43)), 7: ((164, 109, 5, 5), (51.10, 71.94, 12.24, 12.72)),
                8: ((347, 232, 7, 7), (141.41, 199.82, 23.86, 22.81))}
# Table 1 (1D V-cycle(1,1), nlevels = 4): iterations per grid for p = 2..6.
PAPER_TABLE1_ITER = {16: (6, 11, 22, 39, 87), 32: (6, 10, 20, 40, 81), 64: (6, 10, 20, 40, 81),
                     128: (6, 10, 20, 39, 79), 256: (8, 13, 19, 38, 78)}


def oned_measure(igamg, torch, steps):
    """The 1D model problem of Section 2.4 (-u'' = (2 pi)^2 sin(2 pi x)), each
    problem in one workgroup of one launch, FP64, weighted Jacobi (omega = 2/3)
    V(1,1) on 4 levels, relative residual 1e-12.  Table 4: N = 64, p = 2..8,
    V, W, RRE(q), MPE(q) solved one set per method (one launch), cycles /
    restarts, L2 error and ms beside the paper's counts and CPU seconds
    (other hardware, context only).  Table 1: its 25 problems (N = 16..256,
    p = 2..6, plain V-cycles) as ONE set in one launch."""
    def run(probs):
        with igamg.Set1D(probs) as s:
            xs = [torch.zeros(s.ndof(i), dtype=torch.float64, device="cuda:0") for i in range(len(probs))]
            stats, _ = s.solve(xs, tol=1e-12, max_iters=5000)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                for x in xs:
                    x.zero_()
                stats, _ = s.solve(xs, tol=1e-12, max_iters=5000)
            torch.cuda.synchronize()
            return stats, (time.perf_counter() - t0) * 1e3 / steps
    t4 = {}
    methods = (("v", 1, igamg.EXTRAP_NONE), ("w", 2, igamg.EXTRAP_NONE), ("rre", 1, igamg.RRE),
               ("mpe", 1, igamg.MPE))
    for k, (name, mu, m) in enumerate(methods):
        probs = [dict(n_el=64, degree=p, levels=4, mu=mu, method=m, q=4 if p <= 3 else 8) for p in range(2, 9)]
        # one problem per set, so each time is that problem's own solve
        for p, pr in zip(range(2, 9), probs):
            (st,), ms = run([pr])
            row = t4.setdefault("p%d" % p, {"q": pr["q"]})
            row[name] = {"iter": st.restarts, "vcycles": st.vcycles, "rel_residual": st.rel_residual,
                         "l2_error": st.l2_error, "ms": round(ms, 3),
                         "paper_iter": PAPER_TABLE4[p][0][k], "paper_cpu_s": PAPER_TABLE4[p][1][k]}
    grids = sorted(PAPER_TABLE1_ITER)
    probs = [dict(n_el=ne, degree=p, levels=4) for ne in grids for p in range(2, 7)]
    stats, ms = run(probs)
    t1 = {"ms_all_25_one_launch": round(ms, 3), "rows": {}}
    for pr, st in zip(probs, stats):
        t1["rows"]["N%d_p%d" % (pr["n_el"], pr["degree"])] = {
            "iter": st.vcycles, "l2_error": st.l2_error,
            "paper_iter": PAPER_TABLE1_ITER[pr["n_el"]][pr["degree"] - 2]}
    return {"table4_n64": t4, "table1_set": t1}


# Restart cycles printed in Tables 13 and 15 (RRE(8), tolerance 1e-12), per grid
# (16, 32, 64 elements per direction) and degree p = 1..5.
PAPER_TABLE13 = {16: (2, 3, 4, 6, 9), 32: (3, 3, 4, 8, 9), 64: (4, 4, 5, 9, 10)}
PAPER_TABLE15 = {16: (2, 2, 2, 4, 9), 32: (2, 2, 2, 4, 7), 64: (2, 2, 3, 5, 6)}
PAPER_TABLE14 = {16: (2, 2, 4, 6), 32: (2, 2, 4, 5), 64: (2, 2, 3, 6)}   # p = 1..4


def elliptic_measure(igamg, torch, steps):
    """The full elliptic problems of Section 4.3: the unit square with the first
    coefficient set and f = 1 (Table 13), the quarter annulus with exact arcs,
    radii 0.2 and 1, the second coefficient set and the manufactured solution
    (Table 15), and the advection-diffusion problem with f = 1 (Table 14); RRE(8) around FP64 V(2,2) multicolour Gauss-Seidel cycles,
    relative residual 1e-12; restart cycles and ms per solve beside the paper's
    counts.  Also flexible GMRES(20) on the annulus problem preconditioned by one
    V-cycle or one RRE(3) restart cycle (relative residual 1e-10), and the
    annulus problem at 1024^2, p = 3, RRE(8) around FP32 V-cycles in FP64
    refinement, relative residual 1e-10."""
    out = {}
    probs = (("table13_square", igamg.UNIT_SQUARE, igamg.PDE_ELLIPTIC_1, (0.0, 0.0), PAPER_TABLE13),
             ("table15_annulus", igamg.QUARTER_ANNULUS_EXACT, igamg.PDE_ELLIPTIC_2, (0.2, 1.0), PAPER_TABLE15),
             ("table14_advection_diffusion", igamg.UNIT_SQUARE, igamg.PDE_ADVECTION_DIFFUSION, (0.0, 0.0),
              PAPER_TABLE14))
    for name, g, pde, radii, paper in probs:
        rows = {}
        for ne in (16, 32, 64):
            row = {}
            for p in range(1, len(paper[ne]) + 1):
                s = igamg.Solver(g, ne, p, radii=radii, pde=pde)
                s.set_rhs_builtin()
                x = torch.zeros(s.ndof, dtype=torch.float64, device="cuda:0")
                s.solve(x, tol=1e-12, max_restarts=500, method=igamg.RRE, q=8)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(steps):
                    x.zero_()
                    st, _ = s.solve(x, tol=1e-12, max_restarts=500, method=igamg.RRE, q=8)
                torch.cuda.synchronize()
                row["p%d" % p] = {"restarts": st.restarts, "vcycles": st.vcycles,
                                  "ms": round((time.perf_counter() - t0) * 1e3 / steps, 3),
                                  "paper_restarts": paper[ne][p - 1]}
                s.close()
            rows["n_el_%d" % ne] = row
        out[name] = rows
    # flexible GMRES(20) preconditioned by one V-cycle or one RRE(3) restart cycle
    fg = {}
    for ne, p in ((64, 4), (256, 3)):
        s = igamg.Solver(igamg.QUARTER_ANNULUS_EXACT, ne, p, radii=(0.2, 1.0), pde=igamg.PDE_ELLIPTIC_2)
        s.set_rhs_builtin()
        for pname, pc in (("vcycle", igamg.PRECOND_VCYCLE), ("rre3", igamg.PRECOND_RRE)):
            x = torch.zeros(s.ndof, dtype=torch.float64, device="cuda:0")
            s.solve_fgmres(x, tol=1e-10, max_iters=300, m=20, precond=pc, q=3)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                x.zero_()
                st, _ = s.solve_fgmres(x, tol=1e-10, max_iters=300, m=20, precond=pc, q=3)
            torch.cuda.synchronize()
            fg["annulus_%d_p%d_%s" % (ne, p, pname)] = {
                "iterations": st.restarts, "vcycles": st.vcycles, "rel_residual": st.rel_residual,
                "ms": round((time.perf_counter() - t0) * 1e3 / steps, 3)}
        s.close()
    out["fgmres_table15_problem"] = fg
    s = igamg.Solver(igamg.QUARTER_ANNULUS_EXACT, N_EL, 3, radii=(0.2, 1.0), pde=igamg.PDE_ELLIPTIC_2,
                     precision=igamg.FP32_IR)
    s.set_rhs_builtin()
    x = torch.zeros(s.ndof, dtype=torch.float64, device="cuda:0")
    s.solve(x, tol=TOL, max_restarts=500, method=igamg.RRE, q=8)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        x.zero_()
        st, _ = s.solve(x, tol=TOL, max_restarts=500, method=igamg.RRE, q=8)
    torch.cuda.synchronize()
    out["annulus_1024_p3_fp32ir_rre8"] = {"ms": round((time.perf_counter() - t0) * 1e3 / steps, 3),
                                          "vcycles": st.vcycles, "restarts": st.restarts,
                                          "rel_residual": st.rel_residual}
    s.close()
    return out


def c3_measure(igamg, torch, synth, steps, forms=None, tuning=None):
    """Unit cube, p = 3, 128^3 elements, f = 3 pi^2 prod sin(pi x_d), V(2,2)
    multicolour GS (64 colours in 16 row classes): plain FP64 V-cycles, FP64
    MPE(4), and MPE(4) around FP32 V-cycles in FP64 refinement; launch shapes
    and the single-workgroup split autotuned per precision."""
    s = igamg.Solver(igamg.UNIT_CUBE, 128, 3)
    s.set_rhs_field(synth.manufactured_sine_modes_3d())
    out = {"ndof": s.ndof, "tuning": {}}
    xs = {}
    tuned = set()
    for name, m, prec in (("plain_fp64", igamg.EXTRAP_NONE, igamg.FP64), ("mpe4_fp64", igamg.MPE, igamg.FP64),
                          ("mpe4_ir", igamg.MPE, igamg.FP32_IR)):
        if forms is not None and name not in forms:
            continue
        s.set_precision(prec)
        if prec not in tuned:
            if tuning is not None:  # launch shapes given (profiled runs)
                s.set_tuning(tuning)
            else:
                s.autotune()
            tuned.add(prec)
            out["tuning"]["fp64" if prec == igamg.FP64 else "fp32"] = s.tuning()
        x = torch.zeros(s.ndof, dtype=torch.float64, device="cuda:0")
        s.solve(x, tol=TOL, max_restarts=2000, method=m, q=4)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            x.zero_()
            st, _ = s.solve(x, tol=TOL, max_restarts=2000, method=m, q=4)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        out[name] = {"ms": round(ms, 2), "vcycles": st.vcycles, "ms_per_vcycle": round(ms / st.vcycles, 3),
                     "rel_residual": st.rel_residual}
        xs[name] = x.clone()
    s.close()
    return out, xs


def c3_oracle_error(xs):
    """Distance of the GPU solutions to the oracle's exact discrete solution
    (fast diagonalisation of the oracle's own assembly)."""
    import numpy as np

    import synth
    from oracle import assemble, fastdiag
    b = assemble.load_vector_3d(128, 3, synth.manufactured_sine_modes_3d())
    u = fastdiag.solve_kronecker(128, 3, b, 3)
    nu = np.linalg.norm(u)
    return {k: float(np.linalg.norm(v.cpu().numpy() - u) / nu) for k, v in xs.items()}


def host_cpu():
    """Host CPU model and the logical CPUs this process may run on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0))


def cpu_baseline(p):
    """The FP64 oracle's restarted RRE(5) solve of the same workload (p, 1024^2),
    from x0 = 0 to the same tolerance, with its own restart bound."""
    import numpy as np

    import synth
    from oracle import assemble, extrapolation as ex, multigrid as mg
    t0 = time.perf_counter()
    H = mg.Hierarchy(assemble.mapped_stiffness_2d(N_EL, p), N_EL, p, 2)
    b = assemble.load_vector_2d(N_EL, p, synth.random_field_modes(2000 + p))
    setup_s = time.perf_counter() - t0
    A = H.fine.A
    nb = np.linalg.norm(b)
    t0 = time.perf_counter()
    x, st, _ = ex.restarted_solve(lambda v: mg.vcycle(H, b, v),
                                  lambda v: np.linalg.norm(b - A @ v) / nb,
                                  np.zeros(len(b)), Q, ex.RRE, tol=TOL, max_restarts=50)
    solve_s = time.perf_counter() - t0
    model, ncpu = host_cpu()
    # the oracle's Gauss-Seidel colour loops and residuals run on OpenMP threads
    # (OMP_NUM_THREADS, else every CPU of the affinity mask); its transfers,
    # sparse products and QR are single-threaded numpy / scipy
    threads = int(os.environ.get("OMP_NUM_THREADS", ncpu))
    # the same DOF-update count as the GPU forms: unknowns of every smoothed level
    # x 4 sweeps (V(2,2)) x V-cycles
    upd = sum(lev.A.shape[0] for lev in H.levels[1:]) * 4 * st.vcycles
    return x, {"value": round(solve_s * 1e3, 1), "unit": "ms", "cores": threads, "kind": "oracle",
               "sample": "one full FP64 restarted RRE(5) solve, quarter annulus p=%d 1024^2, x0=0, "
                         "tol 1e-10 (oracle setup %.1f s excluded); restarts=%d vcycles=%d; "
                         "OpenMP in the GS colour loops and residuals only, the rest "
                         "single-threaded numpy/scipy" % (p, setup_s, st.restarts, st.vcycles),
               "dof_updates_per_s": round(upd / solve_s, 1),
               "host_cpu": model, "host_ncpu": ncpu, "converged": bool(st.converged)}


def cpu_baseline_1d():
    """The oracle on Table 4's p = 8 problem (N = 64, 4 levels, weighted Jacobi
    V(1,1), relative residual 1e-12): RRE(8) and plain V-cycles, ms per solve."""
    import numpy as np

    from oracle import extrapolation as ex, multigrid as mg, poisson1d as p1
    H = p1.hierarchy(64, 8, 4)
    A = H.fine.A
    b = p1.load(64, 8)
    nb = np.linalg.norm(b)
    G = lambda v: mg.mu_cycle(H, 3, b, v, mg.SMOOTH_JACOBI, 1, 1, 1)
    rn = lambda v: np.linalg.norm(b - A @ v) / nb
    out = {}
    for name, method in (("rre8", ex.RRE), ("v_cycle", None)):
        t0 = time.perf_counter()
        _, st, _ = ex.restarted_solve(G, rn, np.zeros(len(b)), 8, method, tol=1e-12, max_restarts=5000)
        out[name] = {"ms": round((time.perf_counter() - t0) * 1e3, 1), "vcycles": st.vcycles}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--degrees", default="3,4,5")
    ap.add_argument("--headline-degree", type=int, default=3)
    ap.add_argument("--degree", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-c1c3", action="store_true")
    ap.add_argument("--no-paper-setting", action="store_true")
    ap.add_argument("--no-elliptic", action="store_true")
    ap.add_argument("--no-1d", action="store_true")
    ap.add_argument("--only-batch", action="store_true")
    ap.add_argument("--only-chosen", action="store_true",
                    help="setup, tuning and training, then only the chosen-form solves (kernel profiles)")
    ap.add_argument("--only-cube", action="store_true",
                    help="only the 128^3 cube's FP32-in-FP64 MPE(4) solves, autotuned (kernel profiles)")
    ap.add_argument("--tuning", default=None,
                    help="with --only-cube or --only-square: launch shapes as JSON (tuning() of an "
                         "unprofiled run) instead of autotuning")
    ap.add_argument("--only-square", action="store_true",
                    help="only the 64^2 unit square's multicolour FP64 RRE(5) solves, autotuned (kernel profiles)")
    ap.add_argument("--no-sequential", action="store_true",
                    help="with --only-batch: skip the one-by-one comparison (kernel profiles)")
    ap.add_argument("--only-1d", action="store_true",
                    help="only the 1D model problem leg (Tables 1 and 4), printed as its own JSON line")
    ap.add_argument("--epochs", type=int, default=10)
    ap.add_argument("--tail-items", type=int, default=-1,
                    help="single-workgroup V-cycle threshold (0 = one launch per step everywhere, "
                         "-1 = autotuned per precision)")
    ap.add_argument("--colour-launches", action="store_true",
                    help="with --only-smoother: one launch per colour instead of per row class")
    ap.add_argument("--detail-out", default=None,
                    help="also write the per-degree results and extra legs to this JSON file")
    ap.add_argument("--only-smoother", action="store_true",
                    help="setup + finest-level smoother sweeps only (for kernel profiling)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(requested --gpus %d, WORLD_SIZE %d)" % (args.gpus, world), flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_2412_20205_amd import igamg

    if not os.path.exists(igamg.LIB_PATH):
        from paper_2412_20205_amd import build as _b
        _b.build(force=True)

    if args.only_smoother:
        p = args.degree
        s = igamg.Solver(igamg.QUARTER_ANNULUS, N_EL, p, row_sweeps=0 if args.colour_launches else 1)
        out = {}
        for prec, name in ((igamg.FP64, "fp64"), (igamg.FP32_IR, "fp32")):
            out[name] = smoother_roofline(s, igamg, prec, nsweeps=16)
            if args.colour_launches:
                out[name]["kernel"] = "k_gs_colour_sliced (one launch per colour)"
                out[name]["traffic"] = None
        # a plain copy of known size (calibration of the traffic counters)
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda:0").fill_(1.0)
        bcopy = torch.empty_like(a)
        for _ in range(4):
            bcopy.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"only_smoother": True, "degree": p, "copy_bytes": 2 * a.numel() * 8,
                          **out}), flush=True)
        return

    if args.only_chosen:
        # setup, tuning and training as in the full run, then only the timed
        # chosen-form solves (a short run for kernel profiles)
        p = args.headline_degree
        s = igamg.Solver(igamg.QUARTER_ANNULUS, N_EL, p, tail_items=-1)
        s.set_precision(igamg.FP32_IR)
        s.autotune()
        rep = s.train_smoother([synth.random_field_modes(5000 + k) for k in range(16)],
                               val_modes=synth.random_field_modes(5900), epochs=args.epochs)
        s.set_rhs_field(synth.random_field_modes(2000 + p))
        ms, st, _ = time_form(s, igamg, torch, igamg.RRE, igamg.FP32_IR, args.steps, args.warmup, True,
                              bool(rep["accepted"]))
        L = s.num_levels
        print(json.dumps({"only_chosen": True, "degree": p, "ms": round(ms, 3), "vcycles": st.vcycles,
                          "restarts": st.restarts, "learned": bool(rep["accepted"]),
                          "accepted_level": rep["accepted_level"][:L],
                          "rho_plain_level": [round(v, 4) for v in rep["rho_plain_level"][:L]],
                          "rho_learned_level": [round(v, 4) for v in rep["rho_learned_level"][:L]],
                          "tuning": s.tuning()}), flush=True)
        return

    if args.only_cube:
        c3, _ = c3_measure(igamg, torch, synth, args.steps, forms=("mpe4_ir",),
                           tuning=json.loads(args.tuning) if args.tuning else None)
        # a plain copy of known size (calibration of the traffic counters)
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda:0").fill_(1.0)
        bcopy = torch.empty_like(a)
        for _ in range(2):
            bcopy.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"only_cube": True, "copy_bytes": 2 * a.numel() * 8, **c3}), flush=True)
        return

    if args.only_batch:
        print(json.dumps({"batch": batch_measure(igamg, torch, synth, args.steps, args.warmup,
                                                 sequential=not args.no_sequential)}), flush=True)
        return

    if args.only_square:
        print(json.dumps({"only_square": True,
                          **c1_measure(igamg, torch, synth, args.steps, forms=("mcgs_rre5",),
                                       tuning=json.loads(args.tuning) if args.tuning else None)}), flush=True)
        return

    if args.only_1d:
        print(json.dumps({"poisson_1d": oned_measure(igamg, torch, args.steps)}), flush=True)
        return

    degrees = [int(v) for v in args.degrees.split(",")]
    results = {}
    headline = None
    xsol = {}
    for p in degrees:
        log("[bench] setup quarter annulus %d^2 p=%d" % (N_EL, p))
        s = igamg.Solver(igamg.QUARTER_ANNULUS, N_EL, p, tail_items=args.tail_items)
        res = {}
        if args.tail_items < 0:
            # launch shapes (sweep launches and learned kernel per level, the
            # split between multi-block levels and the single-workgroup
            # kernel), tuned per precision (the FP32 form trains above its own split)
            s.autotune()
            tun64 = s.tuning()
            s.set_precision(igamg.FP32_IR)
            s.autotune()
            res["tuning"] = {"fp64": tun64, "fp32": s.tuning()}
        trained = False
        if p == args.headline_degree and not args.no_learned:
            log("[bench] training the learned smoother p=%d" % p)
            rep = s.train_smoother([synth.random_field_modes(5000 + k) for k in range(16)],
                                   val_modes=synth.random_field_modes(5900), epochs=args.epochs)
            res["learned_training"] = {k: v for k, v in rep.items()
                                       if k not in ("loss_first", "loss_last", "rho_plain_level",
                                                    "rho_learned_level", "accepted_level")}
            L = s.num_levels
            for k in ("loss_first", "loss_last", "rho_plain_level", "rho_learned_level", "accepted_level"):
                res["learned_training"][k] = [round(v, 5) for v in rep[k][:L]]
            trained = bool(rep["accepted"])
        s.set_rhs_field(synth.random_field_modes(2000 + p))
        forms = (("plain_fp64", igamg.EXTRAP_NONE, igamg.FP64, False),
                 ("rre_fp64", igamg.RRE, igamg.FP64, False),
                 ("ir_rre", igamg.RRE, igamg.FP32_IR, False),
                 ("chosen", igamg.RRE, igamg.FP32_IR, True))
        for name, method, prec, learned in forms:
            if name == "chosen" and not trained:
                res["chosen"] = dict(res["ir_rre"], learned=False)
                xsol[(p, "chosen")] = xsol[(p, "ir_rre")]
                continue
            steps = args.steps if name in ("chosen", "ir_rre") or p == args.headline_degree \
                else max(1, args.steps // 2)
            log("[bench] p=%d form=%s steps=%d" % (p, name, steps))
            ms, st, x = time_form(s, igamg, torch, method, prec, steps, args.warmup, learned, trained)
            res[name] = {"ms": round(ms, 3), "vcycles": st.vcycles, "restarts": st.restarts,
                         "rel_residual": st.rel_residual, "learned_fallbacks": st.learned_fallbacks,
                         "dof_updates_per_s": round(dof_updates(s, st.vcycles, 4) / (ms * 1e-3), 1)}
            res["setup_ms"] = round(st.setup_ms, 1)
            xsol[(p, name)] = x
        if p == args.headline_degree and trained:
            # held-out right-hand sides (seed 5900 decided the acceptance)
            ev = {}
            for seed in range(5901, 5910):
                s.set_rhs_field(synth.random_field_modes(seed))
                row = {}
                for tag, learned in (("learned", True), ("plain_gs", False)):
                    ms_e, st_e, _ = time_form(s, igamg, torch, igamg.RRE, igamg.FP32_IR, 1, 1, learned, True)
                    row[tag] = {"ms": round(ms_e, 3), "vcycles": st_e.vcycles,
                                "learned_fallbacks": st_e.learned_fallbacks}
                ev[str(seed)] = row
            res["learned_heldout"] = {
                "seeds": ev,
                "vcycles_learned": sum(r["learned"]["vcycles"] for r in ev.values()),
                "vcycles_plain_gs": sum(r["plain_gs"]["vcycles"] for r in ev.values()),
                "ms_learned": round(sum(r["learned"]["ms"] for r in ev.values()), 3),
                "ms_plain_gs": round(sum(r["plain_gs"]["ms"] for r in ev.values()), 3)}
            s.set_rhs_field(synth.random_field_modes(2000 + p))
        x64 = xsol[(p, "rre_fp64")]
        for name in ("ir_rre", "chosen"):
            res[name]["err_vs_fp64_rre"] = float(torch.linalg.norm(xsol[(p, name)] - x64) /
                                                 torch.linalg.norm(x64))
        res["smoother_fp64"] = smoother_roofline(s, igamg, igamg.FP64)
        res["smoother_fp32"] = smoother_roofline(s, igamg, igamg.FP32_IR)
        results[p] = res
        if p == args.headline_degree:
            headline = res
        s.close()
        for name in ("plain_fp64", "ir_rre"):
            xsol.pop((p, name), None)
        torch.cuda.empty_cache()
    if headline is None:
        headline = results[degrees[0]]
        args.headline_degree = degrees[0]

    c1 = c3 = c3x = None
    if not args.no_c1c3:
        log("[bench] unit square 64^2 p=2")
        c1 = c1_measure(igamg, torch, synth, args.steps)
        log("[bench] unit cube 128^3 p=3")
        c3, c3x = c3_measure(igamg, torch, synth, max(1, args.steps // 2))

    paper = None
    if not args.no_paper_setting:
        log("[bench] paper setting: unit square 64^2, Jacobi V(1,1)/W(1,1), p = 1..5")
        paper = paper_setting_measure(igamg, torch, synth, max(1, args.steps // 2))

    elliptic = None
    if not args.no_elliptic:
        log("[bench] full elliptic problems (Tables 13, 15)")
        elliptic = elliptic_measure(igamg, torch, max(1, args.steps // 2))

    oned = None
    if not args.no_1d:
        log("[bench] 1D model problem (Tables 1, 4)")
        oned = oned_measure(igamg, torch, max(1, args.steps // 2))

    batch = None
    if not args.no_batch:
        log("[bench] batch of 96 problems")
        batch = batch_measure(igamg, torch, synth, max(1, args.steps // 2), args.warmup)

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) p=%d" % args.headline_degree)
        xo, cpu = cpu_baseline(args.headline_degree)
        xg = xsol[(args.headline_degree, "rre_fp64")].cpu().numpy()
        xc = xsol[(args.headline_degree, "chosen")].cpu().numpy()
        cpu["gpu_fp64_rre_vs_oracle"] = float(np.linalg.norm(xg - xo) / np.linalg.norm(xo))
        cpu["gpu_chosen_vs_oracle"] = float(np.linalg.norm(xc - xo) / np.linalg.norm(xo))
        if not args.no_1d:
            cpu["poisson_1d_n64_p8"] = cpu_baseline_1d()
        if c3x is not None:
            log("[bench] cube: oracle exact discrete solution")
            c3["error_vs_oracle_exact"] = c3_oracle_error(c3x)

    hp = args.headline_degree
    detail = {"per_degree": {str(k): v for k, v in results.items()},
              "batch": batch, "unit_square_64_p2": c1, "unit_cube_128_p3": c3,
              "paper_setting_square64_jacobi": paper, "full_elliptic": elliptic,
              "poisson_1d": oned, "cpu_baseline": cpu}
    for k, v in detail.items():
        if v is not None:
            log(json.dumps({"leg": k, "result": v}))
    if args.detail_out:
        os.makedirs(os.path.dirname(os.path.abspath(args.detail_out)), exist_ok=True)
        with open(args.detail_out, "w") as f:
            json.dump(detail, f, indent=1)
    print(json.dumps(headline_line(args, hp, headline, cpu)), flush=True)


def headline_line(args, hp, headline, cpu):
    """The one compact JSON line of the run (the last line on stdout)."""
    ch, plain = headline["chosen"], headline["plain_fp64"]
    roof = {k: headline["smoother_fp32"][k] for k in ("bound", "achieved", "peak", "unit", "frac",
                                                         "traffic", "kernel", "avg_launch_us",
                                                         "bytes_per_launch")}
    cpu_short = None
    if cpu is not None:
        cpu_short = {k: cpu[k] for k in ("value", "unit", "cores", "kind", "sample", "host_cpu",
                                         "gpu_chosen_vs_oracle")}
    return {
        "metric": METRIC,
        "value": ch["ms"],
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ch["ms"],
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "quarter annulus (radii 1, 2), B-spline p=%d, 1024x1024 elements, "
                               "V(2,2) multicolour GS with the learned first pre-smoothing step, "
                               "9 levels, RRE(5), FP32 V-cycles in FP64 refinement, random-field "
                               "RHS seed %d, x0=0, tol 1e-10" % (hp, 2000 + hp),
                   "ndof": (N_EL + hp - 2) ** 2,
                   "chosen_vcycles": ch["vcycles"], "chosen_uses_learned": ch.get("learned", True),
                   "plain_fp64_ms": plain["ms"], "plain_fp64_vcycles": plain["vcycles"],
                   "rre_fp64_ms": headline["rre_fp64"]["ms"], "ir_rre_ms": headline["ir_rre"]["ms"],
                   "speedup_vs_plain_fp64": round(plain["ms"] / ch["ms"], 2),
                   "chosen_dof_updates_per_s": ch["dof_updates_per_s"],
                   "smoother_fp64_gbs": headline["smoother_fp64"]["achieved"],
                   "smoother_fp32_gbs": headline["smoother_fp32"]["achieved"],
                   "tuning_fp32": {k: headline["tuning"]["fp32"][k] for k in
                                   ("tail_items", "row_class", "learned_kernel")}
                   if "tuning" in headline else None,
                   "detail": "per-degree results and extra legs on stderr (one JSON line each)"},
        "roofline": roof,
        "cpu_baseline": cpu_short,
    }


if __name__ == "__main__":
    main()
