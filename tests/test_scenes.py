"""Host-side checks of the seeded scene recipes (no GPU): the uneven mixed batch starts with
every body clear of every moving obstacle and above the ground, so each contact the batch sees
comes from motion within the run, never from an overlap built into the initial pose."""
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
