"""GPU parity of the bilateral attachment (supplementary: bilateral constraint for cloth control).

The capture set follows from the state at the capture step by the oracle's own rule
(grasp_update), so each checked GPU step is compared with the oracle's step from the GPU's state
with the gripper poses advanced in lockstep on the host.
"""
import sys

import numpy as np
import pytest

from oracle import flash_oracle as O
from paper_2604_17513_amd import scenes

pytestmark = pytest.mark.gpu


def _F():
    from paper_2604_17513_amd import flash as F
    return F


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _block(hexes=2, young=2e5, lift=0.3):
    rest, tets = scenes.hex_lattice(hexes, hexes, hexes, (0.05, 0.05, 0.05), (-0.025, 0.0, -0.025))
    env = scenes.EnvDesc(scenes.TET, rest, tets, density=1000.0, young=young, poisson=0.3, mu=0.5)
    return env, rest + np.array([0.0, lift, 0.0])


@pytest.mark.parametrize("precision,rel,vel", [
    ("fp64", 1e-9, (0.06, 0.05, 0.02)),      # dragged across the ground while lifted
    ("fp32", 1e-5, (0.06, 0.05, 0.02)),
    ("fp32", 1e-5, (0.0, 0.05, 0.0)),        # lifted straight up: the sheet peels off
])
def test_sheet_dragged_by_a_corner_matches_oracle(precision, rel, vel):
    """A sheet lying on the ground with one corner held by a moving gripper.  In FP32 these steps
    exercise the contact solve's stall recovery: with warm-started attachment rows a Newton run
    stalled (every backtracking line search failed) until it restarts from the zero start."""
    F = _F()
    sc = scenes.cloth_drop(n=10, side=0.2, height=0.001, seed=3)
    x0 = sc.x0[0] - np.array([0.0, 0.05, 0.0])             # just above the ground
    sc.x0[0] = x0
    sc.obstacles[0] = [scenes.ground()]
    grip = scenes.Gripper(x0[0].copy(), 1e-3, True, np.array(vel), 40)
    sc.grippers = [[grip]]
    p = sc.params
    oe = O.precompute(sc.envs[0], p.h)
    b = F.from_scene(sc, precision=F.FLASH_FP64 if precision == "fp64" else F.FLASH_FP32, max_contacts=256)
    held = O.grasp_update(x0, [grip], None)
    assert list(held[0]) == [0]
    gr = [grip]
    for s in range(24):
        if s in (0, 1, 5, 12, 23):
            x, v = b.get_state()
            obs = b.get_obstacles(0)
            b.step(1)
            x1, _ = b.get_state()
            ref = O.step(oe, x, v, obs, p, grippers=gr, held=held)
            gc = b.contacts(0)
            same = list(zip(gc["vertex"], gc["obstacle"])) == list(zip(ref.contacts.vertex, ref.contacts.obstacle))
            L = np.linalg.norm(sc.envs[0].rest_x.max(0) - sc.envs[0].rest_x.min(0))
            err = float(np.abs(x1 - ref.x).max())
            tol = rel * max(np.abs(ref.x).max(), L)
            att = gc["mode"] == 3
            st = b.stats()[0]
            _say(f"{precision} step {s}: flags {st['flags']} Newton {st['inner_iterations']} residual {st['residual']:.2e} "
                 f"rows {ref.contacts.count} (attachments {int(att.sum())}) max|dq| {err:.3e} "
                 f"(tol {tol:.3e}) held vertex at {x1[0]} target {gr[0].center + O.gripper_displacement(gr[0], p.h)}")
            assert same and att.sum() == 1 and gc["obstacle"][att][0] == F.MAX_OBSTACLES
            assert err <= tol
            r = O.contact_residual(oe, x, x1, ref.contacts, gc["lambda"], p.h)
            assert r <= 1e-6
            held = ref.held
        else:
            b.step(1)
        gr = [O.advance_gripper(g, p.h) for g in gr]
    per, mx, its, st = b.residual()
    assert mx <= p.ncp_tol


def test_carried_block_falls_freely_after_release():
    """FP64: a block held whole by a gripper moving at constant velocity translates rigidly with it
    (impulses carry the weight), and after release falls by the implicit-Euler closed form."""
    F = _F()
    env, x0 = _block()
    u = np.array([0.1, 0.2, -0.05])
    grip = scenes.Gripper(x0.mean(0), 1.0, True, u, -1)
    p = scenes.Params(lg_iterations=4)
    sc = scenes.Scene([env], [x0], [np.tile(u, (x0.shape[0], 1))], [[]], p, grippers=[[grip]])
    b = F.from_scene(sc, precision=F.FLASH_FP64, max_contacts=64)
    M = float(env.density * 0.05 ** 3)
    b.step(3)
    x3, v3 = b.get_state()
    np.testing.assert_allclose(x3, x0 + 3 * p.h * u, rtol=0, atol=1e-12)
    imp = b.contacts(0)["impulse"].sum(0)
    np.testing.assert_allclose(imp, -p.h * M * np.asarray(p.gravity), rtol=1e-9, atol=1e-13)
    rel = grip.copy()
    rel.center = grip.center + 3 * p.h * u
    rel.grasp = False
    b.set_grippers([rel], env=0)
    g = np.asarray(p.gravity)
    for k in range(1, 5):
        b.step(1)
        xk, _ = b.get_state()
        xe = x3 + k * p.h * u + p.h * p.h * g * k * (k + 1) / 2
        assert b.stats()[0]["contacts"] == 0
        np.testing.assert_allclose(xk, xe, rtol=0, atol=1e-11)


def test_hanging_block_carries_its_weight_fp32():
    F = _F()
    env, x0 = _block(young=5e5)
    top = x0[:, 1].max()
    grip = scenes.Gripper(np.array([0.0, top + 0.03, 0.0]), 0.05)
    p = scenes.Params(lg_iterations=8)
    sc = scenes.Scene([env], [x0], [np.zeros_like(x0)], [[]], p, grippers=[[grip]])
    b = F.from_scene(sc, max_contacts=64, fused_lg=True)
    b.step(120)
    x, v = b.get_state()
    c = b.contacts(0)
    M = float(env.density * 0.05 ** 3)
    assert (c["mode"] == 3).sum() == 9
    _say(f"hanging block: |v| max {np.abs(v).max():.2e}, attachment impulse {c['impulse'].sum(0)}")
    w = -p.h * M * np.asarray(p.gravity)
    # FP32 sums: the horizontal components are rounding noise on the weight's scale
    np.testing.assert_allclose(c["impulse"].sum(0), w, rtol=2e-3, atol=1e-5 * np.abs(w).max())
    per, mx, its, st = b.residual()
    assert mx <= p.ncp_tol


def test_lightweight_mode_with_attachment_matches_oracle():
    """FP64 lightweight mode (5 x 10 updates) with a corner held above the ground."""
    F = _F()
    sc = scenes.cloth_drop(n=8, side=0.2, height=0.001, seed=4, lg_iterations=5)
    x0 = sc.x0[0] - np.array([0.0, 0.05, 0.0])
    sc.x0[0] = x0
    sc.obstacles[0] = [scenes.ground()]
    grip = scenes.Gripper(x0[0].copy(), 1e-3, True, np.array([0.0, 0.1, 0.0]), -1)
    sc.grippers = [[grip]]
    sc.params.max_inner_iterations = 10
    oe = O.precompute(sc.envs[0], sc.params.h)
    b = F.from_scene(sc, precision=F.FLASH_FP64, contact_metric=F.FLASH_METRIC_LIGHTWEIGHT, inner_tol=1e-300)
    x, v = b.get_state()
    b.step(1)
    x1, _ = b.get_state()
    ref = O.step_lightweight(oe, x, v, sc.obstacles[0], sc.params, newton_iterations=10, tol=0.0,
                             grippers=[grip], held=None)
    assert ref.contacts.attach.sum() == 1
    err = float(np.abs(x1 - ref.x).max())
    _say(f"lightweight with attachment: rows {ref.contacts.count} max|dq| {err:.3e} oracle residual {ref.residual:.2e}")
    assert err <= 1e-9 * 0.3
