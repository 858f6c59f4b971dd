"""Learned smoother on the GPU: forward and gradient parity with the FP64
oracle evaluated on the same BF16-rounded weights and rounding points, training
gain measured by the true residual, and the Gauss-Seidel fallback."""
import numpy as np
import pytest
import torch

import synth
from oracle import learned as ln
from paper_2412_20205_amd import igamg

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def to_bf16_bits(a):
    f = np.asarray(ln.bf16_round(a), dtype=np.float32)
    return (f.view(np.uint32) >> 16).astype(np.uint16)


def canonical(Ws):
    W1, W2, W3 = Ws
    return np.concatenate([W1[:, 0].reshape(16, 9).ravel(), W2.reshape(16, 16, 9).ravel(),
                           W3[0].reshape(16, 9).ravel()])


def from_canonical(v):
    return [v[:144].reshape(16, 1, 3, 3), v[144:2448].reshape(16, 16, 3, 3),
            v[2448:].reshape(1, 16, 3, 3)]


@pytest.fixture(scope="module")
def solver():
    print("[case] annulus 128 p=3 learned", flush=True)
    return igamg.Solver(igamg.QUARTER_ANNULUS, 128, 3)


@pytest.mark.parametrize("level,seed", [(5, 1), (4, 2), (2, 3)])
def test_forward_matches_oracle(solver, level, seed):
    rng = np.random.default_rng(seed)
    Ws = ln.init_weights(rng)
    bits = to_bf16_bits(canonical(Ws))
    Wq = from_canonical(ln.bf16_round(canonical(Ws)))
    solver.set_smoother_weights(level, bits)
    assert np.array_equal(solver.get_smoother_weights(level), bits)
    n = int(round(solver.level_ndof(level) ** 0.5))
    z = rng.standard_normal((n, n)).astype(np.float32)
    y = torch.zeros(n * n, dtype=torch.float32, device=DEV)
    solver.smoother_forward(level, torch.tensor(z.ravel(), device=DEV), y)
    yg = y.cpu().numpy().reshape(n, n)
    yr, _ = ln.forward(z.astype(np.float64), Wq, bf16_points=True)
    err = np.linalg.norm(yg - yr) / np.linalg.norm(yr)
    print("[learned fwd] level %d n=%d rel err %.2e" % (level, n, err))
    assert err < 1e-4


@pytest.mark.parametrize("kernel", [0, 12, 28, 29])
@pytest.mark.parametrize("level,seed", [(5, 11), (3, 12)])
def test_every_inference_kernel_matches_oracle(solver, kernel, level, seed):
    """Each inference kernel the autotuner can pick (16x16-tile VALU/MFMA;
    all-MFMA with 12x12 or 28x28 tiles, 512 or 256 threads) against the
    oracle's forward pass on the same BF16 points; level 3 (11^2) is smaller
    than one tile and level 5 (131^2) leaves a ragged edge tile for each."""
    rng = np.random.default_rng(seed)
    Ws = ln.init_weights(rng)
    solver.set_smoother_weights(level, to_bf16_bits(canonical(Ws)))
    Wq = from_canonical(ln.bf16_round(canonical(Ws)))
    t = solver.tuning()
    t["learned_kernel"][level] = kernel
    solver.set_tuning(t)
    assert solver.tuning()["learned_kernel"][level] == kernel
    n = int(round(solver.level_ndof(level) ** 0.5))
    z = rng.standard_normal((n, n)).astype(np.float32)
    y = torch.zeros(n * n, dtype=torch.float32, device=DEV)
    solver.smoother_forward(level, torch.tensor(z.ravel(), device=DEV), y)
    yr, _ = ln.forward(z.astype(np.float64), Wq, bf16_points=True)
    err = np.linalg.norm(y.cpu().numpy().reshape(n, n) - yr) / np.linalg.norm(yr)
    print("[learned fwd] kernel %d level %d n=%d rel err %.2e" % (kernel, level, n, err))
    assert err < 1e-4


def test_tuning_is_validated(solver):
    t = solver.tuning()
    for field, bad in (("learned_kernel", 16), ("row_class", 2)):
        u = dict(t, **{field: list(t[field])})
        u[field][1] = bad
        with pytest.raises(igamg.IgamgError):
            solver.set_tuning(u)
    with pytest.raises(ValueError):
        solver.set_tuning(dict(t, num_levels=t["num_levels"] + 1))
    solver.set_tuning(t)
    assert solver.tuning()["learned_kernel"] == t["learned_kernel"]


@pytest.mark.parametrize("level,seed", [(5, 4), (3, 5)])
def test_gradients_match_oracle(solver, level, seed):
    rng = np.random.default_rng(seed)
    Ws = ln.init_weights(rng)
    bits = to_bf16_bits(canonical(Ws))
    Wq = from_canonical(ln.bf16_round(canonical(Ws)))
    solver.set_smoother_weights(level, bits)
    n = int(round(solver.level_ndof(level) ** 0.5))
    z = rng.standard_normal((n, n)).astype(np.float32)
    t = rng.standard_normal((n, n)).astype(np.float32)
    loss, g = solver.smoother_loss_grad(level, torch.tensor(z.ravel(), device=DEV),
                                        torch.tensor(t.ravel(), device=DEV))
    lr, gr = ln.loss_and_grads(z.astype(np.float64), t.astype(np.float64), Wq, bf16_points=True)
    assert abs(loss - lr) / lr < 1e-5
    gc = canonical(gr)
    for sl, name in ((slice(0, 144), "W1"), (slice(144, 2448), "W2"), (slice(2448, 2592), "W3")):
        err = np.linalg.norm(g[sl] - gc[sl]) / np.linalg.norm(gc[sl])
        print("[learned grad] level %d %s rel err %.2e" % (level, name, err))
        assert err < 2e-3, name


def test_training_gain_and_fallback():
    """Train on a 256^2 annulus (p = 3), keeping each level's network only if
    the cycle started on that level contracts better with it; the networks kept
    must contract better than the Gauss-Seidel sweeps they replace and the
    RRE(5) solve must reach 1e-10 by the true residual with no more V-cycles
    than without them."""
    print("[case] annulus 256 p=3 training", flush=True)
    s = igamg.Solver(igamg.QUARTER_ANNULUS, 256, 3)
    modes = [synth.random_field_modes(5000 + k) for k in range(8)]
    rep = s.train_smoother(modes, val_modes=synth.random_field_modes(5900), epochs=8, per_level_accept=1)
    print("[learned train]", {k: v for k, v in rep.items() if k not in ("loss_first", "loss_last")})
    print("[learned train] loss first", np.round(rep["loss_first"][:9], 4))
    print("[learned train] loss last ", np.round(rep["loss_last"][:9], 4))
    assert rep["levels_trained"] >= 2
    assert rep["accepted"] == 1 and rep["rho_learned"] < rep["rho_plain"]
    # per-level contraction: the cycle started on level l (levels 0..l) on the
    # validation right-hand side restricted to level l
    L = s.num_levels - 1
    top = s.tuning()["tail_top"]
    rp, rl = rep["rho_plain_level"], rep["rho_learned_level"]
    print("[learned rho per level] plain", np.round(rp[:L + 1], 4), "learned", np.round(rl[:L + 1], 4),
          "split", top)
    acc = rep["accepted_level"]
    print("[learned levels kept]", acc[:L + 1])
    assert rp[0] == 0.0 and rl[0] == 0.0
    assert rp[L] == rep["rho_plain"] and rl[L] == rep["rho_learned"]
    assert sum(acc) >= 1 and all(a in (0, 1) for a in acc)
    for l in range(1, L + 1):
        assert 0.0 < rp[l] < 1.0 and 0.0 < rl[l] < 1.0, l
        if l <= top:  # no network in a cycle that runs in the single-workgroup kernel
            assert rl[l] == rp[l] and acc[l] == 0, l
        if not any(acc[1:l + 1]):  # no network kept on levels 0..l: the same cycle
            assert rl[l] == rp[l], l
    s.set_rhs_field(synth.random_field_modes(5901))
    x = torch.zeros(s.ndof, dtype=torch.float64, device=DEV)
    st_l, _ = s.solve(x, tol=1e-10, max_restarts=100, method=igamg.RRE, q=5)
    assert s.residual(x) <= 1.0000001e-10
    s.set_learned(False)
    x0 = torch.zeros(s.ndof, dtype=torch.float64, device=DEV)
    st_p, _ = s.solve(x0, tol=1e-10, max_restarts=100, method=igamg.RRE, q=5)
    print("[learned gain] vcycles learned %d plain %d; solve ms learned %.1f plain %.1f"
          % (st_l.vcycles, st_p.vcycles, st_l.solve_ms, st_p.solve_ms))
    assert st_l.vcycles <= st_p.vcycles
    assert st_l.learned_fallbacks == 0
    # fallback: spoil the finest network (negated output layer) -> Gauss-Seidel takes over
    L = s.num_levels - 1
    w = s.get_smoother_weights(L).copy()
    w[2448:] ^= np.uint16(0x8000)
    s.set_smoother_weights(L, w)
    s.set_learned(True)
    x1 = torch.zeros(s.ndof, dtype=torch.float64, device=DEV)
    st_f, _ = s.solve(x1, tol=1e-10, max_restarts=200, method=igamg.RRE, q=5)
    print("[learned fallback] fallbacks %d vcycles %d" % (st_f.learned_fallbacks, st_f.vcycles))
    assert s.residual(x1) <= 1.0000001e-10
    assert st_f.learned_fallbacks >= 1


def test_default_training_keeps_every_trained_level():
    """Without per_level_accept every trained level (those above the
    single-workgroup split) keeps its network; the per-level contraction
    figures are reported all the same."""
    print("[case] annulus 128 p=3 training, default acceptance", flush=True)
    s = igamg.Solver(igamg.QUARTER_ANNULUS, 128, 3)
    rep = s.train_smoother([synth.random_field_modes(5000 + k) for k in range(4)],
                           val_modes=synth.random_field_modes(5900), epochs=2)
    L = s.num_levels - 1
    top = s.tuning()["tail_top"]
    print("[learned default] kept", rep["accepted_level"][:L + 1], "split", top,
          "rho", np.round(rep["rho_plain_level"][:L + 1], 4), np.round(rep["rho_learned_level"][:L + 1], 4))
    assert rep["levels_trained"] == L - top
    assert rep["accepted_level"][:L + 1] == [0] * (top + 1) + [1] * (L - top)
    for l in range(1, L + 1):
        assert 0.0 < rep["rho_plain_level"][l] < 1.0 and 0.0 < rep["rho_learned_level"][l] < 1.0
    s.close()
