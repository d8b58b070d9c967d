"""GPU parity of the learned warm start: the bf16 MFMA network kernels against the
FP64 network oracle, the per-contact features and labels against the oracle's,
training behaviour, and the learned-warm-start step against the FP64 step oracle.

Tolerances of the network comparisons.  Both sides round every GEMM operand to
bfloat16; the GPU sums the exact products in FP32, the oracle in FP64, so a
pre-activation differs by about sqrt(K) 2^-24 relative (K = 128).  A hidden
value that close to a bfloat16 rounding boundary rounds the other way on one
side (probability ~ 1e-6 / 2^-8 ~ 4e-4 per value, so a few flips per hundred
rows); a flip moves that value by one bf16 unit (2^-8 relative) and the
outputs downstream of it by up to ~2^-8 of their scale.  Outputs are therefore
checked in two parts: the bulk (99th percentile of the per-row error) against
1e-4 of the largest output, which only the FP32-versus-FP64 summation order can
reach, and the worst row against 1e-2; gradients norm-wise to 1e-2.  A dropped
term, a transposed operand or a missing ReLU mask exceeds these by orders of
magnitude in every row.
"""
import sys

import numpy as np
import pytest

from oracle import flash_oracle as O
from oracle import mlp_oracle as M
from paper_2604_17513_amd import scenes

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _F():
    from paper_2604_17513_amd import flash as F
    return F


def _torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def _net(seed):
    rng = np.random.default_rng(seed)
    parts = []
    for _, s in M.SHAPES:
        k = int(np.prod(s))
        parts.append(rng.uniform(-1, 1, k) * (np.sqrt(6.0 / s[-1]) if len(s) == 2 else 0.2))
    return np.concatenate(parts).astype(np.float32)


@pytest.mark.parametrize("n", [1, 37, 300, 140001])
def test_mlp_forward_matches_oracle(n):
    """n = 140001 needs more 32-row tiles than the persistent grid has waves (ragged last tile)."""
    torch = _torch()
    F = _F()
    _say(f"mlp forward n={n}")
    th = _net(n)
    X = np.random.default_rng(10 + n).standard_normal((n, 16)).astype(np.float32)
    m = F.Mlp(max_rows=4096, seed=0)
    m.set_params(th)
    xd = torch.from_numpy(X).cuda()
    yd = torch.empty((n, 3), dtype=torch.float32, device="cuda")
    m.forward(xd, n, yd)
    Y = yd.cpu().numpy().astype(np.float64)
    R, _ = M.forward(th.astype(np.float64), X.astype(np.float64), rounded=True)
    scale = max(np.abs(R).max(), 1e-30)
    row_err = np.abs(Y - R).max(axis=1) / scale
    p99 = np.percentile(row_err, 99)
    _say(f"  row error / max|Y|: p50 {np.median(row_err):.2e} p99 {p99:.2e} max {row_err.max():.2e}")
    assert p99 <= 1e-4
    assert row_err.max() <= 1e-2


@pytest.mark.parametrize("n", [5, 64, 333])
def test_mlp_gradient_matches_oracle(n):
    torch = _torch()
    F = _F()
    _say(f"mlp grad n={n}")
    th = _net(100 + n)
    rng = np.random.default_rng(20 + n)
    X = rng.standard_normal((n, 16)).astype(np.float32)
    T = rng.standard_normal((n, 3)).astype(np.float32)
    m = F.Mlp(max_rows=512, seed=0)
    m.set_params(th)
    g, loss = m.grad(torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda(), n)
    L, gr = M.loss_and_grad(th.astype(np.float64), X.astype(np.float64), T.astype(np.float64), rounded=True)
    rel = np.linalg.norm(g - gr) / np.linalg.norm(gr)
    _say(f"  loss gpu {loss:.6e} oracle {L:.6e}; grad rel err {rel:.2e}")
    assert abs(loss - L) <= 2e-3 * L
    assert rel <= 1e-2
    # every parameter block is exercised (a skipped layer would show here)
    off = 0
    for name, shp in M.SHAPES:
        k = int(np.prod(shp))
        blk = slice(off, off + k)
        off += k
        nb = np.linalg.norm(gr[blk])
        if nb > 0:
            assert np.linalg.norm(g[blk] - gr[blk]) <= 2e-2 * nb + 1e-6 * np.linalg.norm(gr), name


def test_mlp_training_reduces_loss_and_is_deterministic():
    torch = _torch()
    F = _F()
    rng = np.random.default_rng(7)
    n = 16384
    X = rng.standard_normal((n, 16)).astype(np.float32)
    X[:, 15] = 1.0
    teacher = _net(9).astype(np.float64)
    T, _ = M.forward(teacher, X.astype(np.float64), rounded=False)
    T = T.astype(np.float32)
    xd, td = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    runs = []
    for rep in range(2):
        m = F.Mlp(max_rows=4096, seed=3)
        m.fit_norm(xd, td, n)
        l0 = m.eval(xd, td, n)
        losses = m.train(xd, td, n, epochs=6, batch=1024, lr=2e-3, seed=5)
        l1 = m.eval(xd, td, n)
        _say(f"rep {rep}: eval loss {l0:.4e} -> {l1:.4e}; epoch losses {np.round(losses, 5).tolist()}")
        runs.append((m.params(), losses, l0, l1))
    assert runs[0][3] < 0.25 * runs[0][2]
    assert np.all(np.diff(runs[0][1]) < 0)
    assert np.array_equal(runs[0][0], runs[1][0])            # bitwise reproducible
    assert np.array_equal(runs[0][1], runs[1][1])


def test_mlp_one_adam_step_matches_oracle():
    torch = _torch()
    F = _F()
    n = 256
    rng = np.random.default_rng(11)
    X = rng.standard_normal((n, 16)).astype(np.float32)
    X[:, 15] = 1.0
    T = rng.standard_normal((n, 3)).astype(np.float32)
    th = _net(12)
    m = F.Mlp(max_rows=n, seed=0)
    m.set_params(th)
    norm = np.concatenate([np.zeros(16), np.ones(16), np.ones(3)]).astype(np.float32)
    m.set_norm(norm)
    lr = 1e-3
    m.train(torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda(), n, epochs=1, batch=n, lr=lr, seed=0)
    new = m.params().astype(np.float64)
    _, g = M.loss_and_grad(th.astype(np.float64), X.astype(np.float64), T.astype(np.float64), rounded=True)
    ref, _, _ = M.adam_step(th.astype(np.float64), g, np.zeros_like(g), np.zeros_like(g), 1, lr)
    # the first Adam step is ~lr * sign(g): compare where the gradient is well resolved
    big = np.abs(g) > 1e-2 * np.abs(g).max()
    d = np.abs(new - ref)
    _say(f"adam step: max diff on resolved entries {d[big].max() / lr:.3e} lr; {big.sum()} entries")
    assert d[big].max() <= 0.05 * lr
    assert d.max() <= 2.0 * lr * (1 + 1e-3)


def _prev_multipliers(con_prev, lam_prev, con, mu):
    """Previous-step multipliers of each contact of `con`, in its frame, projected on the cone."""
    lam = np.zeros((con.count, 3))
    has = np.zeros(con.count, bool)
    key = {(int(v), int(o)): j for j, (v, o) in enumerate(zip(con_prev.vertex, con_prev.obstacle))}
    for j, (v, o) in enumerate(zip(con.vertex, con.obstacle)):
        i = key.get((int(v), int(o)))
        if i is None:
            continue
        f = con_prev.frame[i] @ lam_prev[i]
        l = con.frame[j].T @ f
        l[0] = max(l[0], 0.0)
        t = np.hypot(l[1], l[2])
        if t > mu * l[0]:
            l[1:] *= (mu * l[0] / t) if t > 0 else 0.0
        lam[j], has[j] = l, True
    return lam, has


def test_features_and_labels_match_oracle():
    torch = _torch()
    F = _F()
    sc = scenes.squeeze_blocks(2, seed=3, hexes=4)
    oes = [O.precompute(e, sc.params.h) for e in sc.envs]
    b = F.from_scene(sc, precision=F.FLASH_FP64, max_contacts=160)
    b.ws_record(True)
    cap = 2 * 160
    fd = torch.zeros((cap, 16), dtype=torch.float32, device="cuda")
    ld = torch.zeros((cap, 3), dtype=torch.float32, device="cuda")
    prev = [None, None]
    for s in range(3):
        x0, v0 = b.get_state()
        xs, vs = b.split(x0), b.split(v0)
        obs = [b.get_obstacles(e) for e in range(2)]
        b.step(1)
        n = b.ws_collect(fd, ld, cap, 0)
        feat = fd[:n].cpu().numpy().astype(np.float64)
        lab = ld[:n].cpu().numpy().astype(np.float64)
        row = 0
        for e in range(2):
            ref = O.step(oes[e], xs[e], vs[e], obs[e], sc.params, tol=1e-12)
            con = ref.contacts
            if prev[e] is None:
                lam_p, has = np.zeros((con.count, 3)), np.zeros(con.count, bool)
            else:
                lam_p, has = _prev_multipliers(prev[e][0], prev[e][1], con, sc.envs[e].mu)
            Fo = M.features(oes[e], xs[e], vs[e], obs[e], sc.params, con, lam_p, has)
            Lo = M.labels(oes[e], sc.params, con, ref.info.get("lam_first", np.zeros((0, 3))), lam_p)
            Fg = feat[row:row + con.count]
            Lg = lab[row:row + con.count]
            row += con.count
            scale = np.maximum(np.abs(Fo).max(axis=0), 1.0)
            ferr = (np.abs(Fg - Fo) / scale).max() if con.count else 0.0
            lerr = np.abs(Lg - Lo).max() / max(np.abs(Lo).max(), 1e-30) if con.count else 0.0
            _say(f"step {s} env {e}: {con.count} contacts, feature err {ferr:.2e}, label err {lerr:.2e}")
            assert ferr <= 1e-5
            assert lerr <= 1e-5
            prev[e] = (con, ref.lam)
        assert row == n


def _train_quick(b, sc, torch, F, steps=12, epochs=8):
    """Records a short rollout of `b` and fits a network to it (GPU kernels only).

    `b` runs with the zero warm start, so every contact of every step is a
    cold-start example: the case the prediction is used for."""
    cap = b.n_envs * 320 * steps
    fd = torch.zeros((cap, 16), dtype=torch.float32, device="cuda")
    ld = torch.zeros((cap, 3), dtype=torch.float32, device="cuda")
    b.ws_record(True)
    n = 0
    for _ in range(steps):
        b.step(1)
        n = b.ws_collect(fd, ld, cap, n)
    b.ws_record(False)
    m = F.Mlp(max_rows=4096, seed=1)
    m.fit_norm(fd, ld, n)
    losses = m.train(fd, ld, n, epochs=epochs, batch=min(1024, n), lr=2e-3, seed=2)
    return m, n, losses


def test_learned_warm_start_step_matches_oracle():
    torch = _torch()
    F = _F()
    sc_train = scenes.squeeze_blocks(4, seed=21, hexes=6)
    bt = F.from_scene(sc_train, warm_start=F.FLASH_WS_ZERO)
    m, n, losses = _train_quick(bt, sc_train, torch, F)
    _say(f"trained on {n} rows, epoch losses {np.round(losses, 4).tolist()}")
    sc = scenes.squeeze_blocks(2, seed=22, hexes=6)
    oes = [O.precompute(e, sc.params.h) for e in sc.envs]
    b = F.from_scene(sc, warm_start=F.FLASH_WS_LEARNED)
    b.ws_load(m.params_bf16(), m.norm())
    picked = 0
    for s in range(16):
        if s in (3, 9, 15):
            x0, v0 = b.get_state()
            xs, vs = b.split(x0), b.split(v0)
            obs = [b.get_obstacles(e) for e in range(2)]
            b.set_state(x0, v0)          # forget the multiplier history: every contact starts cold
            b.step(1)
            x1s = b.split(b.get_state()[0])
            for e in range(2):
                ref = O.step(oes[e], xs[e], vs[e], obs[e], sc.params, tol=1e-12)
                L = np.linalg.norm(sc.envs[e].rest_x.max(0) - sc.envs[e].rest_x.min(0))
                err = np.abs(x1s[e] - ref.x).max()
                _say(f"step {s} env {e}: max|dq| {err:.3e} tol {1e-5 * max(np.abs(ref.x).max(), L):.3e}")
                assert err <= 1e-5 * max(np.abs(ref.x).max(), L)
        else:
            b.step(1)
        picked += sum(st["ws_state"] & 1 for st in b.stats())
        per, mx, its, stc = b.residual()
        assert mx <= 1e-6
    _say(f"prediction chosen in {picked} of 32 env-steps")
    assert picked >= 1


def test_learned_start_gain_on_cold_starts():
    """What the trained network gains over the method without it, measured where it is used:
    from identical mid-squeeze states with the multiplier history dropped (every contact starts
    cold), one step with the learned start and one with the plain previous-step start (which then
    has no history either).  Both solve every step to the tolerance; the Newton iterations of
    both are reported, and the learned start may not cost more than a quarter more."""
    torch = _torch()
    F = _F()
    sc_train = scenes.squeeze_blocks(4, seed=25, hexes=6)
    bt = F.from_scene(sc_train, warm_start=F.FLASH_WS_ZERO)
    m, n, losses = _train_quick(bt, sc_train, torch, F)
    sc = scenes.squeeze_blocks(4, seed=26, hexes=6)
    bl = F.from_scene(sc, warm_start=F.FLASH_WS_LEARNED)
    bl.ws_load(m.params_bf16(), m.norm())
    bp = F.from_scene(sc, warm_start=F.FLASH_WS_PREV)
    its_l = its_p = 0
    picked = 0
    for s in range(18):
        if s % 6 == 5:
            x0, v0 = bp.get_state()
            bl.set_obstacles([bp.get_obstacles(e) for e in range(sc.n_envs)])
            for b in (bl, bp):
                b.set_state(x0, v0)          # identical states and obstacles, no multiplier history
                b.residual_history(reset=True)
                b.step(1)
            for b, name in ((bl, "learned"), (bp, "plain")):
                mx, over, newton, steps = b.residual_history(reset=True, full=True)
                assert mx <= sc.params.ncp_tol and over == 0, name
                if name == "learned":
                    its_l += newton
                else:
                    its_p += newton
            picked += sum(st["ws_state"] & 1 for st in bl.stats())
        else:
            bp.step(1)
    started, restarted = bl.ws_history(reset=True)
    _say(f"ws_history: started from the prediction {started}, restarted {restarted}")
    assert started == picked
    gain = 1.0 - its_l / max(its_p, 1)
    _say(f"cold-start steps: Newton iterations learned {its_l}, plain {its_p} (gain {100 * gain:.1f}%); "
         f"prediction chosen in {picked} of 12 env-steps")
    assert picked >= 1
    assert its_l <= its_p


def test_learned_warm_start_rejects_non_finite_predictions():
    F = _F()
    sc = scenes.squeeze_blocks(2, seed=23, hexes=4)
    ref = F.from_scene(sc)
    b = F.from_scene(sc, warm_start=F.FLASH_WS_LEARNED)
    w = np.full(M.N_PARAMS, 0x7FC0, dtype=np.uint16)      # bf16 NaN everywhere
    b.ws_load(w, np.concatenate([np.zeros(16), np.ones(19)]).astype(np.float32))
    for s in range(6):
        ref.step(1)
        b.step(1)
        assert all((st["ws_state"] & 1) == 0 for st in b.stats())
        xa, xb = ref.get_state()[0], b.get_state()[0]
        assert np.array_equal(xa, xb)     # the prediction never wins, so the runs are identical
    per, mx, its, stc = b.residual()
    assert mx <= 1e-6


def test_ws_collect_capacity_error():
    torch = _torch()
    F = _F()
    sc = scenes.squeeze_blocks(2, seed=24, hexes=4)
    b = F.from_scene(sc)
    fd = torch.zeros((4, 16), dtype=torch.float32, device="cuda")
    ld = torch.zeros((4, 3), dtype=torch.float32, device="cuda")
    with pytest.raises(F.FlashError) as ei:
        b.ws_collect(fd, ld, 4, 0)
    assert ei.value.status == F.FLASH_ERR_INVALID_ARG     # recording is off
    b.ws_record(True)
    for _ in range(3):
        b.step(1)
    with pytest.raises(F.FlashError) as ei:
        b.ws_collect(fd, ld, 4, 0)
    assert ei.value.status == F.FLASH_ERR_CAPACITY
