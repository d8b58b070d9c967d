"""Pins of the oracle's bilateral attachment (supplementary: bilateral constraint for cloth control,
Eq. 13: x_i - p_grip(t) = 0 for the grasped vertices, which join the set when the gripper is
activated within a proximity threshold and leave it on release).

* a body held whole by a gripper moving at constant velocity with g = 0 translates rigidly with it
  and its attachment impulses vanish; with gravity they carry the weight, sum P = -h M g;
* after release the body falls freely (implicit-Euler closed form);
* a block hung by its top face settles with the attachment impulses carrying its weight;
* held vertices sit at their targets (the gripper's end-of-step pose plus the capture offset);
* capture takes exactly the vertices within the radius, a vertex held by one gripper is not taken
  by another, and a grasping gripper that holds nothing captures once it reaches vertices;
* momentum balance holds with attachments.
"""
import numpy as np
import pytest

from oracle import flash_oracle as O
from paper_2604_17513_amd import scenes


def _block(hexes=2, young=2e5, lift=0.3):
    rest, tets = scenes.hex_lattice(hexes, hexes, hexes, (0.05, 0.05, 0.05), (-0.025, 0.0, -0.025))
    env = scenes.EnvDesc(scenes.TET, rest, tets, density=1000.0, young=young, poisson=0.3, mu=0.5)
    return env, rest + np.array([0.0, lift, 0.0])


def test_capture_rule_radius_order_and_retry():
    x = np.array([[0.0, 0.0, 0.0], [0.01, 0.0, 0.0], [0.02, 0.0, 0.0], [0.03, 0.0, 0.0]])
    g0 = scenes.Gripper(np.array([0.0, 0.0, 0.0]), 0.01)          # takes 0 and 1 (1 on the boundary)
    g1 = scenes.Gripper(np.array([0.015, 0.0, 0.0]), 0.0051)      # would take 1 and 2: 1 is taken
    held = O.grasp_update(x, [g0, g1], None)
    assert sorted(held[0]) == [0, 1] and sorted(held[1]) == [2]
    np.testing.assert_allclose(held[1][2], [0.005, 0.0, 0.0], atol=1e-15)
    # release of g0 frees its vertices; g1 keeps its set while grasping
    g0r = g0.copy(); g0r.grasp = False
    held2 = O.grasp_update(x, [g0r, g1], held)
    assert held2[0] == {} and sorted(held2[1]) == [2]
    # a grasping gripper out of reach holds nothing and captures when it arrives
    far = scenes.Gripper(np.array([1.0, 0.0, 0.0]), 0.005)
    assert O.grasp_update(x, [far], None) == [{}]
    near = far.copy(); near.center = np.array([0.03, 0.0, 0.001])
    assert sorted(O.grasp_update(x, [near], [{}])[0]) == [3]


def test_held_body_translates_rigidly_then_falls_freely_after_release():
    env, x0 = _block()
    p = scenes.Params(lg_iterations=4)
    oe = O.precompute(env, p.h)
    u = np.array([0.1, 0.2, -0.05])
    center = x0.mean(0)
    grip = scenes.Gripper(center, 1.0, True, u, -1)              # radius covers the whole block
    # g = 0: rigid translation with the gripper, no impulses needed after the first step
    p0 = scenes.Params(lg_iterations=4)
    p0.gravity = (0.0, 0.0, 0.0)
    x, v, held, gr = x0.copy(), np.zeros_like(x0), None, [grip]
    for n in range(1, 5):
        r = O.step(oe, x, v, [], p0, grippers=gr, held=held)
        assert r.contacts.count == x0.shape[0] and r.contacts.attach.all()
        np.testing.assert_allclose(r.x, x0 + n * p0.h * u, rtol=0, atol=1e-12)
        if n > 1:
            assert np.abs(r.impulse).max() <= 1e-10
        x, v, held, gr = r.x, r.v, r.held, r.grippers
    # with gravity: the impulses carry the weight every step of the steady motion
    x, v, held, gr = x0.copy(), np.tile(u, (x0.shape[0], 1)), None, [grip]
    M = oe.mass.sum()
    for n in range(1, 4):
        r = O.step(oe, x, v, [], p, grippers=gr, held=held)
        np.testing.assert_allclose(r.impulse.sum(0), -p.h * M * np.asarray(p.gravity), rtol=1e-9, atol=1e-13)
        np.testing.assert_allclose(r.x, x0 + n * p.h * u, rtol=0, atol=1e-12)
        x, v, held, gr = r.x, r.v, r.held, r.grippers
    # release: free fall from there (every vertex has velocity u, the body is undeformed)
    rel = gr[0].copy(); rel.grasp = False
    xs, vs, hs, gs = x.copy(), v.copy(), held, [rel]
    g = np.asarray(p.gravity)
    for k in range(1, 5):
        r = O.step(oe, xs, vs, [], p, grippers=gs, held=hs)
        assert r.contacts.count == 0 and r.held == [{}]
        xe = x + k * p.h * u + p.h * p.h * g * k * (k + 1) / 2
        np.testing.assert_allclose(r.x, xe, rtol=0, atol=1e-11)
        xs, vs, hs, gs = r.x, r.v, r.held, r.grippers


def test_block_hung_by_its_top_face_carries_its_weight():
    env, x0 = _block(young=5e5)
    p = scenes.Params(lg_iterations=8)
    oe = O.precompute(env, p.h)
    top = x0[:, 1].max()
    # 3 cm above the top face: its 9 vertices lie within 0.047 m, the next layer beyond 0.055 m
    grip = scenes.Gripper(np.array([0.0, top + 0.03, 0.0]), 0.05)
    x, v, held, gr = x0.copy(), np.zeros_like(x0), None, [grip]
    M = oe.mass.sum()
    for n in range(120):
        r = O.step(oe, x, v, [], p, grippers=gr, held=held)
        x, v, held, gr = r.x, r.v, r.held, r.grippers
    assert len(held[0]) == 9
    # held vertices at their targets; the body at rest carries its weight through them
    for vtx, off in held[0].items():
        np.testing.assert_allclose(x[vtx], grip.center + off, rtol=0, atol=1e-12)
    assert np.abs(v).max() < 1e-4
    np.testing.assert_allclose(r.impulse.sum(0), -p.h * M * np.asarray(p.gravity), rtol=2e-3, atol=1e-10)
    # the hanging block stretched: its bottom is below its rest position
    assert x[:, 1].min() < x0[:, 1].min() - 1e-6


@pytest.mark.parametrize("seed", [0, 1])
def test_momentum_balance_with_attachments_and_ground(seed):
    """A sheet dragged across the ground by one corner: sum m (v' - v) = h M g + sum P (contacts and
    attachments) at every step."""
    rng = np.random.default_rng(seed)
    sc = scenes.cloth_drop(n=8, side=0.2, height=0.001, seed=seed)
    p = sc.params
    oe = O.precompute(sc.envs[0], p.h)
    x = sc.x0[0] - np.array([0.0, 0.05, 0.0])                       # lying just above the ground
    corner = x[0].copy()
    grip = scenes.Gripper(corner, 1e-3, True, np.array([0.05, 0.04, rng.uniform(-0.02, 0.02)]), -1)
    v, held, gr, obs = np.zeros_like(x), None, [grip], [scenes.ground()]
    M = oe.mass.sum()
    for _ in range(6):
        r = O.step(oe, x, v, obs, p, grippers=gr, held=held)
        lhs = (oe.mass[:, None] * (r.v - v)).sum(0)
        rhs = p.h * M * np.asarray(p.gravity) + r.impulse.sum(0)
        np.testing.assert_allclose(lhs, rhs, rtol=1e-9, atol=1e-12)
        assert r.residual <= 1e-10
        assert r.contacts.attach.sum() == 1 and (~r.contacts.attach).sum() > 0
        x, v, held, gr, obs = r.x, r.v, r.held, r.grippers, r.obstacles


def test_held_vertex_takes_no_obstacle_rows():
    """A corner held just above the ground lies within the contact margin but gets only its
    attachment rows; its neighbours keep their ground contacts."""
    sc = scenes.cloth_drop(n=6, side=0.1, height=0.001, seed=0)
    p = sc.params
    x = sc.x0[0] - np.array([0.0, 0.05, 0.0])
    grip = scenes.Gripper(x[0].copy(), 1e-3)
    held = O.grasp_update(x, [grip], None)
    con = O.detect(x, np.zeros_like(x), [scenes.ground()], p, [grip], held)
    rows0 = [(int(o), bool(a)) for vv, o, a in zip(con.vertex, con.obstacle, con.attach) if vv == 0]
    assert rows0 == [(O.MAX_OBSTACLES, True)]
    assert (con.vertex == 1).sum() == 1 and not con.attach[con.vertex == 1][0]
    free = O.detect(x, np.zeros_like(x), [scenes.ground()], p)
    assert free.count == con.count       # the ground row of vertex 0 became its attachment row
