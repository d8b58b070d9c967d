"""Pins of the FP64 network oracle (learned warm start) against facts that do not
come from the oracle itself: known bfloat16 roundings, hand-built networks with
closed-form outputs, central finite differences of the loss, the format's
precision bound for the bf16 procedure, and Adam's first step."""
import math

import numpy as np
import pytest

from oracle import mlp_oracle as M


def test_param_count():
    assert M.N_PARAMS == 35587


def test_bf16_rounding_known_values():
    # 8 significant bits: spacing 2^-7 on [1, 2)
    assert M.bf16(1.0) == 1.0
    assert M.bf16(1.0 + 2.0 ** -8) == 1.0                    # tie -> even (mantissa 0)
    assert M.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6     # tie -> even (mantissa 2)
    assert M.bf16(1.0 + 2.0 ** -8 + 2.0 ** -20) == 1.0 + 2.0 ** -7
    assert M.bf16(np.pi) == 3.140625
    assert M.bf16(0.1) == 0.10009765625
    assert M.bf16(-0.1) == -0.10009765625
    assert M.bf16(0.0) == 0.0
    assert M.bf16(65280.0) == 65280.0 and M.bf16(65408.0) == 65536.0   # tie at the top of [2^15, 2^16)
    x = np.random.default_rng(0).standard_normal(10000)
    r = M.bf16(x)
    assert np.all(np.abs(r - x) <= np.abs(x) * 2.0 ** -8 * (1 + 1e-12))
    assert np.array_equal(M.bf16(r), r)                       # idempotent


def _zero():
    return np.zeros(M.N_PARAMS)


def test_forward_bias_only_network():
    th = _zero()
    p = M.unpack(th)
    p["b4"][:] = [0.5, -2.0, 3.25]
    X = np.random.default_rng(1).standard_normal((7, 16))
    Y, _ = M.forward(th, X)
    assert np.array_equal(Y, np.tile([0.5, -2.0, 3.25], (7, 1)))


def test_forward_single_path_closed_form():
    # y0 = 2 relu(relu(relu(x0 + 0.25))); y1 = -relu(x3)... built from unit paths
    th = _zero()
    p = M.unpack(th)
    p["W1"][0, 0] = 1.0
    p["b1"][0] = 0.25
    p["W2"][0, 0] = 1.0
    p["W3"][0, 0] = 1.0
    p["W4"][0, 0] = 2.0
    p["W1"][5, 3] = 1.0
    p["W2"][7, 5] = 1.0
    p["W3"][9, 7] = 1.0
    p["W4"][1, 9] = -1.0
    X = np.zeros((4, 16))
    X[:, 0] = [-1.0, 0.5, 1.5, -0.25]
    X[:, 3] = [2.0, -1.0, 0.75, 0.0]
    Y, _ = M.forward(th, X, rounded=False)
    np.testing.assert_array_equal(Y[:, 0], 2.0 * np.maximum(X[:, 0] + 0.25, 0.0))
    np.testing.assert_array_equal(Y[:, 1], -np.maximum(X[:, 3], 0.0))
    np.testing.assert_array_equal(Y[:, 2], 0.0)


def _random_net(seed, n=9):
    rng = np.random.default_rng(seed)
    th = np.concatenate([rng.uniform(-1, 1, int(np.prod(s))) * (np.sqrt(6.0 / s[-1]) if len(s) == 2 else 0.1)
                         for _, s in M.SHAPES])
    X = rng.standard_normal((n, 16))
    T = rng.standard_normal((n, 3))
    return th, X, T


@pytest.mark.parametrize("seed", [0, 1])
def test_backprop_matches_central_differences(seed):
    th, X, T = _random_net(seed)
    L, g = M.loss_and_grad(th, X, T, rounded=False)
    assert L == pytest.approx(M.loss(th, X, T, rounded=False), rel=1e-15)
    rng = np.random.default_rng(100 + seed)
    # every bias and last-layer weight, plus random entries of every matrix
    idx = list(range(M.N_PARAMS - 3 - 384, M.N_PARAMS))
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in M.SHAPES])
    for k in range(len(M.SHAPES)):
        idx += list(rng.integers(offs[k], offs[k + 1], 40))
    eps = 1e-6
    worst = 0.0
    gmax = np.max(np.abs(g))
    for i in idx:
        tp = th.copy(); tp[i] += eps
        tm = th.copy(); tm[i] -= eps
        fd = (M.loss(tp, X, T, rounded=False) - M.loss(tm, X, T, rounded=False)) / (2 * eps)
        worst = max(worst, abs(fd - g[i]))
    # central differences: O(eps^2) truncation + rounding ~ 1e-16 / eps; ReLU kinks are avoided with probability 1
    assert worst <= 1e-8 * max(gmax, 1.0)


def test_backprop_input_gradient_sign_and_scale():
    # with one linear path, dL/db4 is the mean residual times 2/(3n) summed per column
    th, X, T = _random_net(3, n=5)
    Y, _ = M.forward(th, X, rounded=False)
    _, g = M.loss_and_grad(th, X, T, rounded=False)
    np.testing.assert_allclose(g[-3:], 2.0 * (Y - T).sum(axis=0) / Y.size, rtol=1e-14, atol=1e-16)


def test_bf16_gradient_within_format_precision():
    th, X, T = _random_net(4, n=64)
    _, g64 = M.loss_and_grad(th, X, T, rounded=False)
    _, g16 = M.loss_and_grad(th, X, T, rounded=True)
    # each product carries <= 2 * 2^-8 relative rounding per operand pair; four layers deep
    err = np.linalg.norm(g16 - g64) / np.linalg.norm(g64)
    assert err < 0.05
    assert err > 0.0   # the rounding is really applied


def test_adam_first_step_is_signed_lr():
    # with m = v = 0 and bias correction, the first step is lr * g / (|g| + eps') ~ lr * sign(g)
    rng = np.random.default_rng(5)
    th = rng.standard_normal(50)
    g = rng.standard_normal(50)
    new, m, v = M.adam_step(th, g, np.zeros(50), np.zeros(50), 1, 1e-3)
    np.testing.assert_allclose(th - new, 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_features_and_labels_of_a_resting_contact():
    """A single tet resting on the ground: gap, frame and scale features follow from the scene."""
    from paper_2604_17513_amd import scenes
    from oracle import flash_oracle as O
    sc = scenes.single_tet_scene("rest", seed=0)
    env = sc.envs[0]
    oe = O.precompute(env, sc.params.h)
    x, v = sc.x0[0], sc.v0[0]
    con = O.detect(x, v, sc.obstacles[0], sc.params)
    assert con.count >= 1
    lam = np.zeros((con.count, 3))
    F = M.features(oe, x, v, sc.obstacles[0], sc.params, con, lam, np.zeros(con.count, bool))
    dc = sc.params.contact_margin
    h = sc.params.h
    np.testing.assert_allclose(F[:, 0], con.d0 / dc, rtol=1e-15)
    # the ground normal points against gravity: (g.n) h^2 / dc = -9.81 h^2 / dc
    np.testing.assert_allclose(F[:, 13], -9.81 * h * h / dc, rtol=1e-12)
    assert np.all(F[:, 8] == 0) and np.all(F[:, 15] == 1) and np.all(F[:, 9] == env.mu)
    # m_v Gbar_vv lies in (0, 1]: A >= M makes Abar^-1 <= M^-1
    assert np.all(F[:, 10] <= 1e-12)
    lab = M.labels(oe, sc.params, con, np.ones((con.count, 3)), np.full((con.count, 3), 0.25))
    np.testing.assert_allclose(lab[:, 0], 0.75 * h * h / oe.mass[con.vertex] / dc, rtol=1e-15)
    # the first-iteration multipliers recorded by the step solve the first subproblem
    res = O.step(oe, x, v, sc.obstacles[0], sc.params)
    assert res.info["lam_first"].shape == (res.contacts.count, 3)
    assert np.all(res.info["lam_first"][:, 0] >= 0)


def test_every_feature_column_by_hand():
    """All 16 feature columns of a hand-built scene, each computed from the scene by hand.

    One tet (legs 2 cm, rho = 1000) lifted 0.5 mm above the ground with uniform velocity
    (0.1, -0.05, 0.2) m/s; vertex 1 also sits 1 mm from the -x face of a box translating at
    (-0.03, 0.01, 0.02) m/s.  Contacts, in (vertex, obstacle) order: (0, ground), (1, ground),
    (1, box), (2, ground).  Frames follow the tangent rule t1 = unit(e_k x n), k = argmin |n_i|
    (lowest on ties), t2 = n x t1: ground n = +y, t1 = +z, t2 = +x; box face n = -x, t1 = +z,
    t2 = +y.  The local stiffness column uses Abar built by polarising the element energy
    w |D_s D_m^-1|^2 (w = 2 mu_L V), not the oracle's assembly.
    """
    from paper_2604_17513_amd import scenes
    from oracle import flash_oracle as O
    h = 1.0 / 60.0
    dc = 2e-3
    L = 0.02
    rest = np.array([[0.0, 0.0, 0.0], [L, 0.0, 0.0], [0.0, 0.0, L], [0.0, L, 0.0]])
    env = scenes.EnvDesc(scenes.TET, rest, np.array([[0, 1, 2, 3]], np.int32), density=1000.0,
                         young=1e5, poisson=0.3, mu=0.6)
    params = scenes.Params(h=h, contact_margin=dc)
    x = rest + np.array([0.0, 5e-4, 0.0])
    vel = np.array([0.1, -0.05, 0.2])
    v = np.tile(vel, (4, 1))
    vb = np.array([-0.03, 0.01, 0.02])
    half = np.array([0.01, 0.05, 0.05])
    c_next = np.array([L + 1e-3 + half[0], 0.01, 0.0])          # pose at the end of the step
    bx = scenes.box(c_next - h * vb, half, vel=vb)
    obs = [scenes.ground(), bx]
    oe = O.precompute(env, h)
    con = O.detect(x, v, obs, params)
    assert list(zip(con.vertex, con.obstacle)) == [(0, 0), (1, 0), (1, 1), (2, 0)]
    lam_prev = np.array([[0.5, 0.1, -0.05], [0.3, 0.0, 0.02], [0.2, 0.01, 0.0], [0.0, 0.0, 0.0]])
    has = np.array([True, True, False, False])
    F = M.features(oe, x, v, obs, params, con, lam_prev, has)

    g = -9.81
    V = L ** 3 / 6.0
    m = 1000.0 * V / 4.0
    s = h * h / m
    # Abar by polarisation of q -> h^2 w |F(q)|^2 with F(q) = D_s(q) D_m^-1 (one coordinate)
    mu_L = 1e5 / (2.0 * 1.3)
    w = 2.0 * mu_L * V
    Dm_inv = np.linalg.inv(np.column_stack([rest[1] - rest[0], rest[2] - rest[0], rest[3] - rest[0]]))

    def energy(q):
        Ds = np.array([q[1] - q[0], q[2] - q[0], q[3] - q[0]])
        return float(np.sum((Ds @ Dm_inv) ** 2))

    E = np.eye(4)
    Abar = np.diag(np.full(4, m))
    for a in range(4):
        for b in range(4):
            Abar[a, b] += h * h * w * 0.5 * (energy(E[a] + E[b]) - energy(E[a]) - energy(E[b]))
    Ginv = np.linalg.inv(Abar)

    ground_row = lambda vtx, lp, flag, nc: [
        5e-4 / dc, (h * vel[1] + h * h * g) / dc, h * vel[1] / dc, h * vel[2] / dc, h * vel[0] / dc,
        s * lp[0] / dc, s * lp[1] / dc, s * lp[2] / dc, flag, 0.6, math.log10(m * Ginv[vtx, vtx]),
        math.log10(m / 1e-3), nc, g * h * h / dc, 0.0, 1.0]
    rel = h * vel - h * vb
    box_row = [1e-3 / dc, -h * vel[0] / dc, -rel[0] / dc, rel[2] / dc, rel[1] / dc,
               s * lam_prev[2, 0] / dc, s * lam_prev[2, 1] / dc, s * lam_prev[2, 2] / dc, 0.0, 0.6,
               math.log10(m * Ginv[1, 1]), math.log10(m / 1e-3), 2, 0.0, h * 0.03 / dc, 1.0]
    expect = np.array([ground_row(0, lam_prev[0], 1.0, 1), ground_row(1, lam_prev[1], 1.0, 2), box_row,
                       ground_row(2, lam_prev[3], 0.0, 1)])
    np.testing.assert_allclose(F, expect, rtol=1e-9, atol=1e-12)
    # the local-stiffness column is informative: Gbar_vv m_v < 1 strictly for a stiff tet
    assert np.all(F[:, 10] < -0.5)
