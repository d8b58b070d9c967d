"""GPU parity for membrane triangles with hinge bending, and for uneven batches that mix
cloth and tet environments in one launch per phase.

Same protocol as the tet parity tests: from the GPU's own start state (promoted exactly to
FP64) and obstacle poses, one GPU step and one oracle step; positions within
1e-5 * max(|q|_inf, L_env) in FP32 and 1e-9 * ... in FP64, identical contact lists, and the
oracle's NCP residual of the GPU's positions and multipliers <= 1e-6 m.
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


def _check_step(b, sc, oes, envs, rel, label):
    """One GPU step and the oracle step of `envs`: same contact list, positions within `rel` of
    the body's extent, and the oracle's NCP residual of the GPU positions and multipliers
    <= 1e-6 m."""
    x0, v0 = b.get_state()
    xs, vs = b.split(x0), b.split(v0)
    obs = {e: b.get_obstacles(e) for e in envs}
    b.step(1)
    x1s = b.split(b.get_state()[0])
    for e in envs:
        ref = O.step(oes[e], xs[e], vs[e], obs[e], sc.params, tol=1e-12)
        L = np.linalg.norm(sc.envs[e].rest_x.max(0) - sc.envs[e].rest_x.min(0))
        tol = rel * max(np.abs(ref.x).max(), L)
        err = np.abs(x1s[e] - ref.x).max()
        gc = b.contacts(e)
        same = (gc["vertex"].tolist() == ref.contacts.vertex.tolist()
                and gc["obstacle"].tolist() == ref.contacts.obstacle.tolist())
        r = O.contact_residual(oes[e], xs[e], x1s[e], ref.contacts, gc["lambda"], sc.params.h) if same else np.inf
        _say(f"{label} env {e}: {len(gc['vertex'])} contacts, max|dq| {err:.3e} (tol {tol:.3e}), residual {r:.2e}")
        assert same
        assert err <= tol
        assert r <= 1e-6


@pytest.mark.parametrize("precision,rel", [("fp64", 1e-9), ("fp32", 1e-5)])
def test_cloth_drop_matches_oracle(precision, rel):
    F = _F()
    sc = scenes.cloth_drop(n=12, seed=0)
    oes = {0: O.precompute(sc.envs[0], sc.params.h)}
    b = F.from_scene(sc, precision=F.FLASH_FP64 if precision == "fp64" else F.FLASH_FP32)
    checked = 0
    for s in range(24):
        if s in (0, 5, 6, 7, 9, 12, 17, 23):
            _check_step(b, sc, oes, [0], rel, f"{precision} step {s}")
            checked += 1
        else:
            b.step(1)
    per, mx, its, st = b.residual()
    assert mx <= 1e-6
    assert checked == 8


def test_cloth_free_flight_closed_form():
    """Rigid translation: ARAP and flat hinges exert no force, so implicit Euler gives
    x_n = x_0 + n h v_0 + h^2 g n (n + 1) / 2 exactly (up to rounding)."""
    F = _F()
    sc = scenes.cloth_drop(n=10, seed=0)
    sc.x0[0] = sc.envs[0].rest_x + np.array([0.0, 20.0, 0.0])   # far above the ground and the box
    v0 = np.tile([0.2, 0.5, -0.1], (sc.envs[0].n_vertices, 1))
    sc.v0[0] = v0
    b = F.from_scene(sc, precision=F.FLASH_FP64)
    n = 12
    b.step(n)
    x, v = b.get_state()
    h = sc.params.h
    g = np.asarray(sc.params.gravity)
    xe = sc.x0[0] + n * h * v0 + h * h * g * n * (n + 1) / 2
    ve = v0 + n * h * g
    assert np.abs(x - xe).max() <= 1e-11 * max(np.abs(xe).max(), 1.0)
    assert np.abs(v - ve).max() <= 1e-9


def test_uneven_cloth_and_tet_batch():
    """Cloth sheets and tet blocks of different sizes in one batch (one launch per phase),
    each env against the oracle, and each env bitwise equal to a batch of its own."""
    F = _F()
    parts = [scenes.cloth_drop(n=12, seed=1), scenes.drop_cube(seed=2, hexes=3, drop_height=0.002),
             scenes.cloth_drop(n=9, seed=3, bending=0.0), scenes.drop_cube(seed=4, hexes=5, drop_height=0.002)]
    envs, xs, vs, obs = [], [], [], []
    for p in parts:
        envs += p.envs; xs += p.x0; vs += p.v0; obs += p.obstacles
    sc = scenes.Scene(envs, xs, vs, obs, scenes.Params(lg_iterations=10))
    oes = {e: O.precompute(sc.envs[e], sc.params.h) for e in range(len(envs))}
    b = F.from_scene(sc)
    for s in range(10):
        if s in (2, 6, 9):
            _check_step(b, sc, oes, list(range(len(envs))), 1e-5, f"uneven step {s}")
        else:
            b.step(1)
    xb = b.split(b.get_state()[0])
    for e in (0, 3):
        one = scenes.Scene([envs[e]], [xs[e]], [vs[e]], [obs[e]], sc.params)
        b1 = F.from_scene(one)
        b1.step(10)
        assert np.array_equal(b1.get_state()[0], xb[e])


def test_autotuned_schedule_is_bitwise_identical():
    """The autotuner picks the work schedule of the explicit-inverse products by timing;
    every candidate sums each output over the same rows in the same order, so a tuned
    batch and a batch on the default schedule end in the same bits."""
    F = _F()
    parts = [scenes.cloth_drop(n=14, seed=5), scenes.drop_cube(seed=6, hexes=4, drop_height=0.002),
             scenes.cloth_drop(n=8, seed=7), scenes.drop_cube(seed=8, hexes=6, drop_height=0.002)]
    envs, xs, vs, obs = [], [], [], []
    for p in parts:
        envs += p.envs; xs += p.x0; vs += p.v0; obs += p.obstacles
    sc = scenes.Scene(envs, xs, vs, obs, scenes.Params(lg_iterations=6))
    tuned = F.from_scene(sc)
    fixed = F.from_scene(sc, fixed_schedule=True)
    tuned.step(8)
    fixed.step(8)
    it, ifx = tuned.schedule_info(), fixed.schedule_info()
    _say(f"tuned schedule {it}; fixed {ifx}")
    assert it["tuned"] and not ifx["tuned"]
    assert all(m > 0 for m in it["candidate_ms"])
    n_tiles = sum(-(-e.n_vertices // it["tile_cols"]) for e in envs)
    assert it["work_items"] == n_tiles
    assert np.array_equal(tuned.get_state()[0], fixed.get_state()[0])
    assert np.array_equal(tuned.get_state()[1], fixed.get_state()[1])


@pytest.mark.parametrize("groups", [2, 3])
def test_stream_groups_match_one_group(groups):
    """A batch split into env groups on separate streams gives the bits of one batch, and the
    ABI's per-env and all-env calls address the same envs."""
    torch = pytest.importorskip("torch")
    F = _F()
    parts = [scenes.cloth_drop(n=10, seed=9), scenes.drop_cube(seed=10, hexes=3, drop_height=0.002),
             scenes.squeeze_blocks(2, seed=11, hexes=4), scenes.cloth_drop(n=7, seed=12)]
    envs, xs, vs, obs = [], [], [], []
    for p in parts:
        envs += p.envs; xs += p.x0; vs += p.v0; obs += p.obstacles
    sc = scenes.Scene(envs, xs, vs, obs, scenes.Params(lg_iterations=6))
    one = F.from_scene(sc)
    grp = F.from_scene(sc, stream_groups=groups, use_graph=True)
    one.ws_record(True)
    grp.ws_record(True)
    for b in (one, grp):
        b.step(5)
    cap = 5 * 320
    rows = []
    for b in (one, grp):
        fd = torch.zeros((cap, 16), dtype=torch.float32, device="cuda")
        ld = torch.zeros((cap, 3), dtype=torch.float32, device="cuda")
        n = b.ws_collect(fd, ld, cap, 0)
        rows.append((n, fd[:n].cpu().numpy(), ld[:n].cpu().numpy()))
    assert rows[0][0] == rows[1][0] and np.array_equal(rows[0][1], rows[1][1]) and np.array_equal(rows[0][2], rows[1][2])
    # per-env state round trip through the groups
    x3, v3 = grp.get_state(env=3)
    assert np.array_equal(x3, one.get_state(env=3)[0])
    grp.set_state(x3, v3, env=3)
    one.set_state(x3, v3, env=3)
    for b in (one, grp):
        b.step(4)
    xo, vo = one.get_state()
    xg, vg = grp.get_state()
    assert np.array_equal(xo, xg) and np.array_equal(vo, vg)
    co, cg = one.contacts(), grp.contacts()
    for k in ("env", "vertex", "obstacle", "lambda"):
        assert np.array_equal(co[k], cg[k]), k
    for e in (0, 4):
        assert np.array_equal(one.contacts(e)["vertex"], grp.contacts(e)["vertex"])
        assert np.array_equal(np.array([o.center for o in one.get_obstacles(e)]),
                              np.array([o.center for o in grp.get_obstacles(e)]))
    so, sg = one.stats(), grp.stats()
    assert [s["contacts"] for s in so] == [s["contacts"] for s in sg]
    assert [s["residual"] for s in so] == [s["residual"] for s in sg]
    assert one.residual_history(full=True) == grp.residual_history(full=True)
    info = grp.schedule_info()
    assert info["stream_groups"] == groups


def test_uneven_batch_fp64_matches_oracle():
    """64 envs of the uneven recipe (cloth 16^2-17^2, tet blocks 500-1200 vertices, 1-3 moving
    boxes or capsules each) in FP64, grouped on 3 streams with one graph per group per step:
    sampled sheets and tet envs against the oracle at 1e-9, and every env-step of the batch at
    the NCP tolerance.  (Sheets stay within the default capacity of 320 contacts per env: a
    sheet lying on the ground touches it with every vertex.)"""
    F = _F()
    sc = scenes.uneven_batch(64, seed=5, max_tet_vertices=1200, max_cloth_side=17, lg_iterations=10)
    b = F.from_scene(sc, precision=F.FLASH_FP64, use_graph=True, stream_groups=3)
    cloth = [e for e, d in enumerate(sc.envs) if d.elem == 1]
    tets = [e for e, d in enumerate(sc.envs) if d.elem == 0]
    sample = cloth[:2] + tets[:2] + [cloth[-1], tets[-1]]
    oes = {e: O.precompute(sc.envs[e], sc.params.h) for e in sample}
    b.step(5)
    _check_step(b, sc, oes, sample, 1e-9, "uneven fp64 step 5")
    b.step(3)
    _check_step(b, sc, oes, sample, 1e-9, "uneven fp64 step 9")
    mx, over = b.residual_history(reset=True)
    _say(f"uneven fp64 64: worst residual {mx:.2e}, env-steps above tolerance {over}")
    assert mx <= sc.params.ncp_tol and over == 0


def test_uneven_batch_fp32_bench_configuration():
    """256 envs of the uneven recipe in FP32 in the batched launch configuration (3 stream
    groups, graphs, autotuned schedule): every env-step ends at the library's FP64 NCP residual
    <= 1e-6 m, no env exceeds its contact capacity, and sampled sheets and tet envs have the
    oracle's contact lists and its positions within 1e-5 relative."""
    F = _F()
    sc = scenes.uneven_batch(256, seed=6, max_tet_vertices=1200, max_cloth_side=17, lg_iterations=10)
    b = F.from_scene(sc, use_graph=True, stream_groups=3)
    cloth = [e for e, d in enumerate(sc.envs) if d.elem == 1]
    tets = [e for e, d in enumerate(sc.envs) if d.elem == 0]
    sample = cloth[:2] + tets[:2] + [cloth[-1], tets[-1]]
    oes = {e: O.precompute(sc.envs[e], sc.params.h) for e in sample}
    b.step(6)
    x0, v0 = b.get_state()
    xs, vs = b.split(x0), b.split(v0)
    obs = {e: b.get_obstacles(e) for e in sample}
    b.step(1)
    x1s = b.split(b.get_state()[0])
    for e in sample:
        ref = O.step(oes[e], xs[e], vs[e], obs[e], sc.params, tol=1e-12)
        L = np.linalg.norm(sc.envs[e].rest_x.max(0) - sc.envs[e].rest_x.min(0))
        err = np.abs(x1s[e] - ref.x).max()
        gc = b.contacts(e)
        _say(f"uneven fp32 env {e} ({'cloth' if e in cloth else 'tets'}): {len(gc['vertex'])} contacts, "
             f"max|dq| {err:.3e}")
        assert gc["vertex"].tolist() == ref.contacts.vertex.tolist()
        assert err <= 1e-5 * max(np.abs(ref.x).max(), L)
    b.step(3)
    mx, over = b.residual_history(reset=True)
    _say(f"uneven fp32 256: worst residual {mx:.2e}, env-steps above tolerance {over}")
    assert mx <= 1e-6 and over == 0
    assert not any(s_["flags"] & 4 for s_ in b.stats())
