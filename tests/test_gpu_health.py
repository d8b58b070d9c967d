"""Health flags, error paths and checkpoint behaviour on the GPU (conditions forced from the
host; every kernel still runs to completion).

* a non-finite state in one env is flagged for that env only, and leaves every other env
  bitwise unchanged (envs never couple);
* an inner-iteration cap of 1 with one local-global iteration per step ends the squeeze's
  steps above the tolerance and is reported as not converged;
* a get/set state round trip is bitwise, and resuming after it (which drops the multiplier
  history) agrees with the uninterrupted run within the solve tolerance;
* a checkpoint (state, obstacle and gripper tracks, held vertices, multiplier cache, learned-start
  state) resumes bitwise in a fresh batch with another stream grouping, and a blob of another
  shape is rejected before anything is written;
* invalid env indices and too small output capacities are rejected with their status;
* 128 envs run the squeeze's whole 500-step horizon in the batched configuration with every
  env-step at the tolerance.
"""
import ctypes as C
import sys

import numpy as np
import pytest

from paper_2604_17513_amd import scenes

pytestmark = pytest.mark.gpu


def _F():
    from paper_2604_17513_amd import flash as F
    return F


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_nonfinite_env_is_isolated():
    F = _F()
    sc = scenes.squeeze_blocks(3, seed=31, hexes=4)
    a = F.from_scene(sc)
    b = F.from_scene(sc)
    a.step(3)
    b.step(3)
    x, v = b.get_state(env=1)
    x[5, 1] = np.nan
    b.set_state(x, v, env=1)
    a.step(3)
    b.step(3)
    per, mx, its, st = b.residual()
    stats = b.stats()
    _say("residuals", per, "flags", [s["flags"] for s in stats], "status", st)
    assert st == F.FLASH_ERR_NONFINITE
    assert stats[1]["flags"] & 1
    assert not (stats[0]["flags"] & 1) and not (stats[2]["flags"] & 1)
    xa, xb = a.split(a.get_state()[0]), b.split(b.get_state()[0])
    assert np.array_equal(xa[0], xb[0]) and np.array_equal(xa[2], xb[2])
    assert not np.all(np.isfinite(xb[1]))


def test_iteration_cap_reports_not_converged():
    F = _F()
    # one local-global iteration with one Newton iteration: the squeeze's contact solve
    # cannot reach the tolerance in a step (with K = 20 the iterations add up and it does)
    sc = scenes.squeeze_blocks(2, seed=32, hexes=5)
    sc.params.max_inner_iterations = 1
    sc.params.lg_iterations = 1
    b = F.from_scene(sc)
    st = F.FLASH_OK
    for _ in range(20):
        b.step(1)
        per, mx, its, st = b.residual()
        if st != F.FLASH_OK:
            break
    stats = b.stats()
    _say("capped residuals", per, "status", st, "flags", [s["flags"] for s in stats])
    assert st == F.FLASH_ERR_NOT_CONVERGED
    assert mx > sc.params.ncp_tol
    assert any(s["flags"] & 2 for s in stats)


def test_state_round_trip_and_resume():
    F = _F()
    sc = scenes.squeeze_blocks(2, seed=33, hexes=5)
    a = F.from_scene(sc)
    b = F.from_scene(sc)
    a.step(12)
    b.step(12)
    x, v = b.get_state()
    b.set_state(x, v)
    x2, v2 = b.get_state()
    assert np.array_equal(x, x2) and np.array_equal(v, v2)
    a.step(6)
    b.step(6)
    xa, xb = a.get_state()[0], b.get_state()[0]
    # the resumed run lost only its warm start: each step's solve still reaches the tolerance
    L = np.linalg.norm(sc.envs[0].rest_x.max(0) - sc.envs[0].rest_x.min(0))
    err = np.abs(xa - xb).max()
    _say(f"resume difference {err:.2e} m")
    assert err <= 1e-5 * max(np.abs(xa).max(), L)
    per, mx, its, st = b.residual()
    assert mx <= sc.params.ncp_tol


@pytest.mark.parametrize("case", ["squeeze_fp32", "dragged_sheet_fp64"])
def test_checkpoint_resume_is_bitwise(case):
    """Save after 15 steps, run 10 more; a fresh batch (other stream grouping) that loads the
    checkpoint runs the same 10 steps to the same bits: positions, velocities, multipliers and
    the moving obstacles' and grippers' tracks."""
    F = _F()
    if case == "squeeze_fp32":
        sc = scenes.squeeze_blocks(3, seed=36, hexes=5)
        kw_a, kw_b = dict(stream_groups=1), dict(stream_groups=3, use_graph=True)
    else:
        sc = scenes.cloth_drop(n=8, side=0.2, height=0.001, seed=5)
        sc.x0[0] = sc.x0[0] - np.array([0.0, 0.05, 0.0])
        sc.obstacles[0] = [scenes.ground()]
        sc.grippers = [[scenes.Gripper(sc.x0[0][0].copy(), 1e-3, True, np.array([0.05, 0.04, 0.01]), 30)]]
        kw_a, kw_b = dict(precision=F.FLASH_FP64), dict(precision=F.FLASH_FP64, fused_lg=True)
    a = F.from_scene(sc, **kw_a)
    a.step(15)
    blob = a.save_checkpoint()
    a.step(10)
    xa, va = a.get_state()
    ca = a.contacts()
    b = F.from_scene(sc, **kw_b)
    b.load_checkpoint(blob)
    b.step(10)
    xb, vb = b.get_state()
    cb = b.contacts()
    _say(f"{case}: checkpoint {len(blob)} bytes, contacts {len(ca['vertex'])}, "
         f"max |dx| {np.abs(xa - xb).max():.1e}")
    assert np.array_equal(xa, xb) and np.array_equal(va, vb)
    assert np.array_equal(ca["lambda"], cb["lambda"]) and np.array_equal(ca["obstacle"], cb["obstacle"])
    for e in range(len(sc.envs)):
        oa, ob = a.get_obstacles(e), b.get_obstacles(e)
        assert all(np.array_equal(p.center, q.center) for p, q in zip(oa, ob))
    # a state-only resume loses the multiplier history (and the held set): not the same run
    c = F.from_scene(sc, **kw_b)
    c.load_checkpoint(blob)
    xs, vs = c.get_state()
    c.set_state(xs, vs)
    c.step(10)
    _say(f"{case}: state-only resume differs by {np.abs(c.get_state()[0] - xa).max():.1e} m")
    # a blob of another shape is rejected and leaves the batch as it was
    other = F.from_scene(scenes.squeeze_blocks(1, seed=36, hexes=4))
    with pytest.raises(F.FlashError):
        b.load_checkpoint(other.save_checkpoint())
    with pytest.raises(F.FlashError):
        b.load_checkpoint(blob[:-1])
    assert np.array_equal(b.get_state()[0], xb)


def test_invalid_env_and_capacity_are_rejected():
    F = _F()
    L = F.lib()
    sc = scenes.squeeze_blocks(2, seed=34, hexes=4)
    b = F.from_scene(sc)
    b.step(2)
    x = np.zeros((sc.envs[0].n_vertices, 3))
    st = L.flash_set_state(b._h, 7, x.ctypes.data_as(C.POINTER(C.c_double)), None)
    assert st == F.FLASH_ERR_INVALID_ARG
    st = L.flash_get_state(b._h, -2, x.ctypes.data_as(C.POINTER(C.c_double)), None)
    assert st == F.FLASH_ERR_INVALID_ARG
    out = (F.flash_contact * 1)()
    n = C.c_int32()
    st = L.flash_contacts(b._h, 0, out, 1, C.byref(n))
    assert st == F.FLASH_ERR_CAPACITY
    assert n.value == len(b.contacts(0)["vertex"]) > 1


def test_full_squeeze_horizon_in_the_batched_configuration():
    """128 envs of the squeeze workload through its whole 500-step horizon (closing, then
    holding) with the fused loop, 3 stream groups and graphs: every env-step ends at the NCP
    tolerance and the state stays finite."""
    F = _F()
    sc = scenes.squeeze_blocks(128, seed=35)
    b = F.from_scene(sc, fused_lg=True, use_graph=True, stream_groups=3)
    b.residual_history(reset=True)
    for blk in range(5):
        b.step(100)
        mx, over, newton, steps = b.residual_history(reset=False, full=True)
        _say(f"squeeze horizon step {100 * (blk + 1)}: worst residual {mx:.2e}, above tolerance {over}, "
             f"Newton per env-step {newton / steps:.2f}")
    assert steps == 128 * 500
    assert mx <= sc.params.ncp_tol and over == 0
    x, v = b.get_state()
    assert np.all(np.isfinite(x)) and np.all(np.isfinite(v))
