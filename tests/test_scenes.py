"""Host-side checks of the seeded scene recipes (no GPU): the uneven mixed batch starts with
every body clear of every moving obstacle and above the ground, so each contact the batch sees
comes from motion within the run, never from an overlap built into the initial pose; and every
cloth sheet, in every recipe, carries the cloth material, gravity and force clamp the paper
prints (fixture under tests/golden/, with its citation)."""
import json
import os

import numpy as np
import pytest

from oracle import flash_oracle as O
from paper_2604_17513_amd import scenes


@pytest.mark.parametrize("n_envs,seed", [(64, 5), (256, 6)])
def test_uneven_batch_starts_clear(n_envs, seed):
    sc = scenes.uneven_batch(n_envs, seed=seed, max_tet_vertices=1200, max_cloth_side=17)
    kinds = set()
    for e in range(n_envs):
        x = np.asarray(sc.x0[e], dtype=np.float64)
        assert x[:, 1].min() > 1e-3
        for ob in sc.obstacles[e]:
            if ob.kind == O.PLANE:
                continue
            kinds.add(ob.kind)
            _, d, _ = O._sdf_eval(ob.kind, np.asarray(ob.center, float), np.asarray(ob.rot, float),
                                  np.asarray(ob.size, float), x, 0.0)
            assert d.min() >= 4e-3, (e, ob.kind, d.min())
    assert kinds == {O.BOX, O.CAPSULE}
    elems = {d.elem for d in sc.envs}
    assert elems == {scenes.TET, scenes.TRI}


def test_cloth_recipes_use_the_papers_parameters():
    with open(os.path.join(os.path.dirname(__file__), "golden", "flash_cloth_parameters.json")) as f:
        g = json.load(f)
    c = g["cloth"]
    sheets = [scenes.cloth_drop(n=12, seed=42)]
    sheets.append(scenes.uneven_batch(32, seed=8, max_tet_vertices=1200, max_cloth_side=17))
    n_tri = 0
    for sc in sheets:
        assert tuple(sc.params.gravity) == tuple(g["gravity"])
        assert sc.params.max_force == g["maxforce"]
        for d in sc.envs:
            if d.elem != scenes.TRI:
                continue
            n_tri += 1
            assert d.young == c["young"] and d.poisson == c["poisson"] and d.bending == c["bending"]
            assert d.density == c["obj_mass"]
            assert d.thickness > 0
    assert n_tri >= 2
    # defaults that a new scene starts from
    p = scenes.Params()
    assert tuple(p.gravity) == tuple(g["gravity"]) and p.max_force == g["maxforce"]


def test_cloth_fold_grippers_take_the_near_corners():
    """Each gripper captures the near corner and its two edge neighbours (radius 1.2 spacings),
    carries them to the midline and 3 cm up over 5 s (500 steps of 0.01 s), then holds; envs are
    copies of one mesh."""
    from oracle import flash_oracle as O
    sc = scenes.cloth_fold(2, n=16, side=0.6)
    x0 = sc.x0[0]
    held = O.grasp_update(x0, sc.grippers[0], None)
    assert [len(h) for h in held] == [3, 3]
    for g in sc.grippers[0]:
        assert g.move_steps == 500
        np.testing.assert_allclose(g.lin_vel * 5.0, [0.0, 0.03, 0.3])
    assert sc.params.h == 0.01 and sc.params.lg_iterations == 5 and sc.params.max_inner_iterations == 10
    assert sc.envs[0] is sc.envs[1] and sc.envs[0].mu == 1.0
    assert np.all(x0[:, 1] == 1e-3)


def test_slab_press_has_the_large_scene_sizes():
    """100 x 9 x 100 hexes of 5 mm: 102,010 vertices and 540,000 tets; at the start the ground and the
    two pads give at most 20,000 contacts; the pads travel 6 mm (1 mm gap + 5 mm indentation) at
    2 cm/s, then hold."""
    from oracle import flash_oracle as O
    sc = scenes.slab_press(1)
    env = sc.envs[0]
    assert env.n_vertices == 102010 and env.n_elements == 540000
    con = O.detect(sc.x0[0], sc.v0[0], sc.obstacles[0], sc.params)
    assert 10201 < con.count <= 20000
    pads = sc.obstacles[0][1:]
    for p in pads:
        travel = p.move_steps * sc.params.h * -p.lin_vel[1]
        assert abs(travel - 0.006) < 0.0005
