"""GPU parity of the fixed-budget lightweight mode (Alg. 1 with the inertia-only metric, Eq. 10).

The mode's result is defined by its iteration, not by convergence, so each checked GPU step is
compared with the oracle's `step_lightweight` from the same state, the same budget and the same
starting multipliers: zero after a state reset (no history), or the previous step's multipliers
re-expressed in the new frames and projected on the cone, as the GPU's warm start does.
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


def _warm_start(prev, con, mu, h):
    """The GPU's warm start: previous world force at the same (vertex, obstacle), in the new
    frame, projected on the friction cone; zero for new pairs."""
    lam = np.zeros((con.count, 3))
    if prev is None:
        return lam
    force = {(int(v), int(o)): imp / h for v, o, imp in zip(prev["vertex"], prev["obstacle"], prev["impulse"])}
    for j, (v, o) in enumerate(zip(con.vertex.tolist(), con.obstacle.tolist())):
        f = force.get((v, o))
        if f is None:
            continue
        l = con.frame[j].T @ f
        l[0] = max(l[0], 0.0)
        lt = np.hypot(l[1], l[2])
        if lt > mu * l[0]:
            l[1:] *= (mu * l[0] / lt) if lt > 0 else 0.0
        lam[j] = l
    return lam


def _check(b, sc, oes, envs, budget, rel, warm, label):
    x0, v0 = b.get_state()
    xs, vs = b.split(x0), b.split(v0)
    obs = {e: b.get_obstacles(e) for e in envs}
    prev = {e: (b.contacts(e) if warm else None) for e in envs}
    b.step(1)
    x1, _ = b.get_state()
    x1s = b.split(x1)
    worst = 0.0
    for e in envs:
        con = O.detect(xs[e], vs[e], obs[e], sc.params)
        lam0 = _warm_start(prev[e], con, sc.envs[e].mu, sc.params.h)
        ref = O.step_lightweight(oes[e], xs[e], vs[e], obs[e], sc.params, newton_iterations=budget,
                                 tol=0.0, lam_warm=lam0)
        L = np.linalg.norm(sc.envs[e].rest_x.max(0) - sc.envs[e].rest_x.min(0))
        scale = max(np.abs(ref.x).max(), L)
        err = float(np.abs(x1s[e] - ref.x).max())
        gc = b.contacts(e)
        same = list(zip(gc["vertex"], gc["obstacle"])) == list(zip(ref.contacts.vertex, ref.contacts.obstacle))
        lerr = float(np.abs(gc["lambda"] - ref.lam).max()) if same and ref.contacts.count else 0.0
        _say(f"{label} env {e}: contacts {ref.contacts.count} updates {ref.info['newton']} max|dq| {err:.3e} "
             f"(tol {rel * scale:.3e}) max|dlambda| {lerr:.3e} oracle residual {ref.residual:.2e}")
        assert same
        assert err <= rel * scale
        worst = max(worst, err / scale)
    return worst


@pytest.mark.parametrize("budget", [1, 10])
def test_lightweight_fp64_drop_cube_matches_oracle(budget):
    """The drop cube in FP64 with the paper's budgets (5 local-global iterations, 1 or 10
    multiplier updates each, no tolerance exit): every checked step from the GPU's state matches the
    oracle's lightweight step, with its warm start rebuilt from the previous GPU step."""
    F = _F()
    sc = scenes.drop_cube(seed=0, lg_iterations=5)
    sc.params.max_inner_iterations = budget
    oe = O.precompute(sc.envs[0], sc.params.h)
    b = F.from_scene(sc, precision=F.FLASH_FP64, max_contacts=128, inner_tol=1e-300,
                     contact_metric=F.FLASH_METRIC_LIGHTWEIGHT)
    checked = 0
    for s in range(30):
        if s in (0, 10, 11, 12, 13, 15, 20, 29):
            _check(b, sc, {0: oe}, [0], budget, 1e-9, warm=s > 0, label=f"budget {budget} step {s}")
            checked += 1
        else:
            b.step(1)
    st = b.stats()[0]
    assert st["inner_iterations"] <= 5 * budget
    assert checked == 8


def test_lightweight_fp32_squeeze_matches_oracle_from_reset_states():
    """FP32 squeeze blocks (6^3 hexes, 3 envs) in the lightweight mode with the paper's budget (5 x
    10): steps taken from states without multiplier history (zero start on both sides) match the
    oracle within 1e-5 relative."""
    F = _F()
    sc = scenes.squeeze_blocks(3, seed=1, hexes=6, lg_iterations=5)
    sc.params.max_inner_iterations = 10
    oes = {e: O.precompute(sc.envs[e], sc.params.h) for e in range(3)}
    b = F.from_scene(sc, contact_metric=F.FLASH_METRIC_LIGHTWEIGHT, inner_tol=1e-300)
    for s in range(16):
        if s in (2, 8, 15):
            x, v = b.get_state()
            b.set_state(x, v)                # forget the history: both sides start from zero
            _check(b, sc, oes, [0, 1, 2], 10, 1e-5, warm=False, label=f"fp32 step {s}")
        else:
            b.step(1)


def test_lightweight_fused_equals_per_phase_and_converges_to_exact():
    """The fused local-global loop gives the per-phase bits in the lightweight mode; with a large
    budget and the exact mode's tolerance, a soft block's step reaches the exact mode's step."""
    F = _F()
    sc = scenes.drop_cube(seed=4, hexes=3, young=2e4, drop_height=0.0005, jitter=0.0, lg_iterations=3)
    sc.params.max_inner_iterations = 10
    a = F.from_scene(sc, precision=F.FLASH_FP64, contact_metric=F.FLASH_METRIC_LIGHTWEIGHT)
    c = F.from_scene(sc, precision=F.FLASH_FP64, contact_metric=F.FLASH_METRIC_LIGHTWEIGHT, fused_lg=True)
    a.step(4)
    c.step(4)
    xa, va = a.get_state()
    xc, vc = c.get_state()
    assert np.array_equal(xa, xc) and np.array_equal(va, vc)
    assert np.array_equal(a.contacts()["lambda"], c.contacts()["lambda"])
    # large budget: the exact mode's step from the same state
    sc.params.max_inner_iterations = 5000
    li = F.from_scene(sc, precision=F.FLASH_FP64, contact_metric=F.FLASH_METRIC_LIGHTWEIGHT)
    ex = F.from_scene(sc, precision=F.FLASH_FP64)
    li.step(1)
    ex.step(1)
    xl, _ = li.get_state()
    xe, _ = ex.get_state()
    per, mx, its, st = li.residual()
    _say(f"large budget: max |dq| to the exact mode {np.abs(xl - xe).max():.3e}, residual {mx:.2e}, "
         f"updates {its[0]} (exact mode {ex.residual()[2][0]} Newton iterations)")
    assert mx <= 1e-11
    assert np.abs(xl - xe).max() <= 1e-9


# ---- the lightweight update from global memory (capacities beyond one CU's LDS) -------------------

def _sheet_on_ground(n, seed, grippers=0):
    sc = scenes.cloth_drop(n=n, side=0.5, height=0.001, seed=seed, lg_iterations=5)
    sc.x0[0] = sc.x0[0] - np.array([0.0, 0.05, 0.0])           # lying 1 mm above the ground
    sc.obstacles[0] = [scenes.ground()]
    sc.params.max_inner_iterations = 10
    x0 = sc.x0[0]
    if grippers:
        a = int(np.argmin(x0[:, 0] + x0[:, 2]))
        c = int(np.argmax(x0[:, 0] - x0[:, 2]))
        sc.grippers = [[scenes.Gripper(x0[a].copy(), 1e-3, True, np.array([0.03, 0.06, 0.03]), -1),
                        scenes.Gripper(x0[c].copy(), 1e-3, True, np.array([-0.03, 0.06, 0.03]), -1)]]
    return sc


@pytest.mark.parametrize("budget", [1, 10])
def test_global_update_fp64_drop_cube_matches_oracle(budget):
    """The drop cube's lightweight steps with the update forced into global memory match the
    oracle as the in-LDS update does (warm starts rebuilt from the previous GPU step)."""
    F = _F()
    sc = scenes.drop_cube(seed=0, lg_iterations=5)
    sc.params.max_inner_iterations = budget
    oe = O.precompute(sc.envs[0], sc.params.h)
    b = F.from_scene(sc, precision=F.FLASH_FP64, max_contacts=128, inner_tol=1e-300,
                     contact_metric=F.FLASH_METRIC_LIGHTWEIGHT, global_contact_solve=1)
    for s in range(30):
        if s in (0, 11, 12, 13, 20, 29):
            _check(b, sc, {0: oe}, [0], budget, 1e-9, warm=s > 0, label=f"global budget {budget} step {s}")
        else:
            b.step(1)
    assert b.stats()[0]["inner_iterations"] <= 5 * budget


def test_global_update_equals_lds_update_and_graph():
    """Same iteration in LDS and from global memory (FP64 squeeze block, tolerance exit on): the
    two routes differ by rounding only; the global route captured in a graph gives its eager bits."""
    F = _F()
    sc = scenes.squeeze_blocks(2, seed=5, hexes=5, lg_iterations=6)
    sc.params.max_inner_iterations = 10
    kw = dict(precision=F.FLASH_FP64, contact_metric=F.FLASH_METRIC_LIGHTWEIGHT)
    a = F.from_scene(sc, **kw)
    g = F.from_scene(sc, global_contact_solve=1, **kw)
    gg = F.from_scene(sc, global_contact_solve=1, use_graph=True, **kw)
    for bb in (a, g, gg):
        bb.step(12)
    xa, xg, xgg = a.get_state()[0], g.get_state()[0], gg.get_state()[0]
    _say(f"global vs LDS route after 12 steps: max |dx| {np.abs(xa - xg).max():.2e} m; updates "
         f"{a.stats()[0]['inner_iterations']} / {g.stats()[0]['inner_iterations']}")
    assert np.abs(xa - xg).max() <= 1e-10
    assert np.array_equal(xg, xgg)
    assert np.array_equal(g.contacts()["lambda"], gg.contacts()["lambda"])


def test_sheet_on_ground_beyond_lds_fp32_matches_oracle():
    """A 48 x 48 sheet lying on the ground: 2304 contacts, beyond what one CU's LDS holds, so the
    FP32 batch updates from global memory.  Steps from reset states (zero start on both sides) match
    the oracle's lightweight step with the paper's budget (5 x 10) within 1e-5 relative."""
    F = _F()
    sc = _sheet_on_ground(48, seed=2)
    oe = O.precompute(sc.envs[0], sc.params.h)
    b = F.from_scene(sc, contact_metric=F.FLASH_METRIC_LIGHTWEIGHT, max_contacts=2400, inner_tol=1e-300,
                     use_graph=True)
    for s in range(6):
        if s in (0, 4):
            x, v = b.get_state()
            b.set_state(x, v)
            _check(b, sc, {0: oe}, [0], 10, 1e-5, warm=False, label=f"sheet 48^2 fp32 step {s}")
        else:
            b.step(1)
    st = b.stats()[0]
    assert st["contacts"] == 2304 and not (st["flags"] & 4)


def test_two_grippers_lift_sheet_corners_beyond_lds_fp64():
    """Two grippers take the corners of the 48 x 48 sheet on the ground and lift them (bilateral
    attachment rows beside 2302 ground rows): FP64 steps from reset multiplier histories match the
    oracle's lightweight step with the same grippers and held sets."""
    F = _F()
    sc = _sheet_on_ground(48, seed=3, grippers=2)
    p = sc.params
    oe = O.precompute(sc.envs[0], p.h)
    b = F.from_scene(sc, precision=F.FLASH_FP64, contact_metric=F.FLASH_METRIC_LIGHTWEIGHT, max_contacts=2400,
                     inner_tol=1e-300)
    gr = list(sc.grippers[0])
    held = None
    L = np.linalg.norm(sc.envs[0].rest_x.max(0) - sc.envs[0].rest_x.min(0))
    for s in range(8):
        if s in (0, 6):
            x, v = b.get_state()
            b.set_state(x, v)
            obs = b.get_obstacles(0)
            b.step(1)
            x1, _ = b.get_state()
            ref = O.step_lightweight(oe, x, v, obs, p, newton_iterations=10, tol=0.0, grippers=gr, held=held)
            gc = b.contacts(0)
            same = list(zip(gc["vertex"], gc["obstacle"])) == list(zip(ref.contacts.vertex, ref.contacts.obstacle))
            err = float(np.abs(x1 - ref.x).max())
            _say(f"two grippers step {s}: rows {ref.contacts.count} (attachments {int(ref.contacts.attach.sum())}) "
                 f"max|dq| {err:.3e} oracle residual {ref.residual:.2e}")
            assert same and int((gc["mode"] == 3).sum()) == 2
            assert err <= 1e-9 * max(np.abs(ref.x).max(), L)
            held = ref.held
        else:
            b.step(1)
        gr = [O.advance_gripper(g, p.h) for g in gr]


def test_cloth_fold_matches_oracle_and_shares_the_inverse():
    """The folding stand-in (32 x 32 sheet on the table, two grippers carrying the near corners,
    h = 0.01, budget 5 x 10) in FP32: a step from a reset multiplier history matches the oracle's
    lightweight step with the same grippers and held sets; three identical envs share one explicit
    inverse and give the single env's bits."""
    F = _F()
    sc = scenes.cloth_fold(3, n=32)
    p = sc.params
    oe = O.precompute(sc.envs[0], p.h)
    b = F.from_scene(sc, contact_metric=F.FLASH_METRIC_LIGHTWEIGHT, max_contacts=32 * 32 + 8, inner_tol=1e-300,
                     use_graph=True)
    one = F.from_scene(scenes.cloth_fold(1, n=32), contact_metric=F.FLASH_METRIC_LIGHTWEIGHT,
                       max_contacts=32 * 32 + 8, inner_tol=1e-300)
    gr = [g.copy() for g in sc.grippers[0]]
    held = None
    L = np.linalg.norm(sc.envs[0].rest_x.max(0) - sc.envs[0].rest_x.min(0))
    for s in range(12):
        if s in (0, 10):
            x, v = b.get_state()
            b.set_state(x, v)
            xs, vs = b.split(x), b.split(v)
            xo, vo = one.get_state()
            one.set_state(xo, vo)
            obs = b.get_obstacles(0)
            b.step(1)
            one.step(1)
            x1 = b.split(b.get_state()[0])
            ref = O.step_lightweight(oe, xs[0], vs[0], obs, p, newton_iterations=10, tol=0.0, grippers=gr, held=held)
            err = float(np.abs(x1[0] - ref.x).max())
            _say(f"fold step {s}: rows {ref.contacts.count} (attachments {int(ref.contacts.attach.sum())}) "
                 f"max|dq| {err:.3e} oracle residual {ref.residual:.2e}")
            assert int(ref.contacts.attach.sum()) == 6
            assert err <= 1e-5 * max(np.abs(ref.x).max(), L)
            held = ref.held
        else:
            b.step(1)
            one.step(1)
        gr = [O.advance_gripper(g, p.h) for g in gr]
    xe = b.split(b.get_state()[0])
    assert np.array_equal(xe[0], xe[1]) and np.array_equal(xe[0], xe[2])
    assert np.array_equal(xe[0], one.get_state()[0])


def test_pressed_slab_with_large_splits_matches_oracle():
    """The large-scene recipe at reduced size (a 40 x 5 x 40-hex slab: 10,086 vertices, so each
    row split of the inverse products spans two LDS chunks) pressed by two pads, two identical envs
    sharing one inverse and its products (one workgroup reads each row for both): FP32 lightweight
    steps from a history reset match the oracle within 1e-5 relative, and both envs give the same
    bits."""
    F = _F()
    sc = scenes.slab_press(2, nx=40, ny=5, nz=40)
    p = sc.params
    oe = O.precompute(sc.envs[0], p.h)
    b = F.from_scene(sc, contact_metric=F.FLASH_METRIC_LIGHTWEIGHT, global_contact_solve=1, max_contacts=6000,
                     use_graph=True, twin_chunk=2)
    L = np.linalg.norm(sc.envs[0].rest_x.max(0) - sc.envs[0].rest_x.min(0))
    b.step(6)
    x, v = b.get_state()
    b.set_state(x, v)
    xs, vs = b.split(x), b.split(v)
    obs = b.get_obstacles(0)
    b.step(1)
    x1 = b.split(b.get_state()[0])
    ref = O.step_lightweight(oe, xs[0], vs[0], obs, p, newton_iterations=p.max_inner_iterations,
                             tol=0.25 * p.ncp_tol)
    err = float(np.abs(x1[0] - ref.x).max())
    _say(f"pressed slab: {sc.envs[0].n_vertices} vertices, contacts {ref.contacts.count}, max|dq| {err:.3e}, "
         f"oracle residual {ref.residual:.2e}")
    assert ref.contacts.count > 1681
    assert err <= 1e-5 * max(np.abs(ref.x).max(), L)
    assert np.array_equal(x1[0], x1[1])


@pytest.mark.parametrize("prec,chunk", [("fp32", 8), ("fp64", 3)])
def test_twin_chunks_give_each_env_its_own_bits(prec, chunk):
    """Ten identical slabs share one inverse and run their global-route products in chunks of
    `chunk` envs per workgroup (8 + 2, or 3 + 3 + 3 + 1).  Three of them differ in state: pads one
    hex further along x, pads pressing twice as fast, a slab starting 3 mm higher; so their contact
    rows part from the others' (rows loaded per env).  With a loose tolerance the envs' iterations
    stop at different updates (the stopped envs of a chunk skip the products).  After 8 steps every
    env holds the bits it gets in a batch of its own (one env per workgroup)."""
    F = _F()
    sc = scenes.slab_press(10, nx=12, ny=3, nz=12, hex_size=0.01)
    for ob in sc.obstacles[3][1:]:
        ob.center[0] += 0.01
    for ob in sc.obstacles[6][1:]:
        ob.lin_vel[1] *= 2.0
    sc.x0[9] = sc.x0[9] + np.array([0.0, 0.003, 0.0])
    kw = dict(precision=F.FLASH_FP64 if prec == "fp64" else F.FLASH_FP32,
              contact_metric=F.FLASH_METRIC_LIGHTWEIGHT, global_contact_solve=1, max_contacts=400, inner_tol=5e-4)
    b = F.from_scene(sc, twin_chunk=chunk, **kw)
    b.step(8)
    xb = b.split(b.get_state()[0])
    cb = [b.stats()[e]["contacts"] for e in range(10)]
    its = [b.stats()[e]["inner_iterations"] for e in range(10)]
    _say(f"twin chunks {prec}: contacts per env {cb}, updates {its}")
    v0 = b.contacts(0)["vertex"]
    assert not np.array_equal(v0, b.contacts(3)["vertex"])
    for e in range(10):
        one = scenes.Scene([sc.envs[e]], [sc.x0[e]], [sc.v0[e]], [sc.obstacles[e]], sc.params, name="one")
        bo = F.from_scene(one, **kw)
        bo.step(8)
        assert np.array_equal(bo.get_state()[0], xb[e]), e


def test_automatic_chunks_give_one_env_per_workgroup_bits():
    """32 identical 64 x 64 folding sheets: the automatic choice runs their products in chunks of
    8 envs (144 blocks per env, so 4 chunks keep 576 workgroups per product); after 6 steps in
    HIP graphs every env holds the bits of the same batch run one env per workgroup."""
    F = _F()
    sc = scenes.cloth_fold(32, n=64)
    kw = dict(contact_metric=F.FLASH_METRIC_LIGHTWEIGHT, max_contacts=64 * 64 + 8, use_graph=True)
    a = F.from_scene(sc, **kw)
    one = F.from_scene(sc, twin_chunk=1, **kw)
    a.step(6)
    one.step(6)
    xa, x1 = a.get_state()[0], one.get_state()[0]
    _say(f"automatic chunks vs one env per workgroup: max |dx| {np.abs(xa - x1).max():.1e}")
    assert np.array_equal(xa, x1)
