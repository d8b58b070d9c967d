"""The fused local-global loop (one launch per step, one workgroup per env) against the
kernel-per-phase step, through the C ABI.

Every phase of the fused loop runs the same device code on the same data as its batched
kernel, so a fused batch must give the bits of a per-phase batch: positions, velocities,
contact lists and multipliers, per-env statistics and the residual history.  Cases: the
squeeze (FP32, FP64 contact solve), cloth sheets in FP64 and FP32, an uneven mixed batch on
stream groups with graphs, the learned warm start, and a step that records training pairs
(which takes the per-phase launches).  One sampled env of the uneven batch is also checked
against the oracle, so the fused path is held to the same bar as the per-phase one.
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


def _same(a, b, label):
    xa, va = a.get_state()
    xb, vb = b.get_state()
    assert np.array_equal(xa, xb) and np.array_equal(va, vb), label
    ca, cb = a.contacts(), b.contacts()
    for k in ("env", "vertex", "obstacle", "lambda", "impulse"):
        assert np.array_equal(ca[k], cb[k]), (label, k)
    sa, sb = a.stats(), b.stats()
    for k in ("inner_iterations", "refactorizations", "contacts", "fp64_polar", "flags", "residual"):
        assert [s[k] for s in sa] == [s[k] for s in sb], (label, k)
    assert a.residual_history(reset=False, full=True) == b.residual_history(reset=False, full=True), label


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_fused_squeeze_is_bitwise_per_phase(precision):
    F = _F()
    sc = scenes.squeeze_blocks(3, seed=41, hexes=5)
    kw = {} if precision == "fp32" else {"precision": F.FLASH_FP64}
    a = F.from_scene(sc, **kw)
    b = F.from_scene(sc, fused_lg=True, **kw)
    for blk in range(3):
        a.step(4)
        b.step(4)
        _say(f"squeeze {precision} steps to {4 * blk + 4}: contacts {[s['contacts'] for s in b.stats()]}")
        _same(a, b, f"squeeze {precision} block {blk}")
    kt = b.kernel_times()
    assert "lg_fused" in kt


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_fused_cloth_is_bitwise_per_phase(precision):
    F = _F()
    sc = scenes.cloth_drop(n=12, seed=42)
    kw = {} if precision == "fp32" else {"precision": F.FLASH_FP64}
    a = F.from_scene(sc, **kw)
    b = F.from_scene(sc, fused_lg=True, **kw)
    for blk in range(4):
        a.step(5)
        b.step(5)
        _same(a, b, f"cloth {precision} block {blk}")
    _say(f"cloth {precision}: {len(b.contacts()['vertex'])} contacts after 20 steps")


def test_fused_uneven_groups_graph_and_oracle():
    """Uneven mixed batch on 3 stream groups with graphs: fused equals per-phase bitwise, and a
    sampled sheet and block match the oracle's step (1e-5 relative in FP32)."""
    F = _F()
    sc = scenes.uneven_batch(24, seed=43, max_tet_vertices=900, max_cloth_side=17, lg_iterations=10)
    a = F.from_scene(sc, use_graph=True, stream_groups=3)
    b = F.from_scene(sc, use_graph=True, stream_groups=3, fused_lg=True)
    a.step(5)
    b.step(5)
    _same(a, b, "uneven step 5")
    cloth = [e for e, d in enumerate(sc.envs) if d.elem == 1]
    tets = [e for e, d in enumerate(sc.envs) if d.elem == 0]
    sample = [cloth[0], tets[-1]]
    x0, v0 = b.get_state()
    xs, vs = b.split(x0), b.split(v0)
    obs = {e: b.get_obstacles(e) for e in sample}
    a.step(1)
    b.step(1)
    _same(a, b, "uneven step 6")
    x1s = b.split(b.get_state()[0])
    for e in sample:
        oe = O.precompute(sc.envs[e], sc.params.h)
        ref = O.step(oe, xs[e], vs[e], obs[e], sc.params, tol=1e-12)
        L = np.linalg.norm(sc.envs[e].rest_x.max(0) - sc.envs[e].rest_x.min(0))
        err = np.abs(x1s[e] - ref.x).max()
        gc = b.contacts(e)
        _say(f"fused uneven env {e}: {len(gc['vertex'])} contacts, max|dq| {err:.3e}")
        assert gc["vertex"].tolist() == ref.contacts.vertex.tolist()
        assert err <= 1e-5 * max(np.abs(ref.x).max(), L)
    b.step(4)
    mx, over = b.residual_history(reset=True)
    assert mx <= sc.params.ncp_tol and over == 0


def test_fused_learned_start_and_recording():
    """A network loaded as the learned warm start runs before the loop, so fused and per-phase
    agree bitwise with it; a recording step takes the per-phase launches and collects the same
    pairs in both batches."""
    torch = pytest.importorskip("torch")
    F = _F()
    from oracle import mlp_oracle as M
    rng = np.random.default_rng(44)
    theta = rng.normal(scale=0.05, size=M.N_PARAMS)
    w16 = (np.asarray(theta, dtype=np.float32).view(np.uint32) >> 16).astype(np.uint16)
    norm = np.zeros(35, dtype=np.float32)
    norm[16:32] = 1.0
    norm[32:35] = 1.0
    sc = scenes.squeeze_blocks(2, seed=44, hexes=4)
    a = F.from_scene(sc, warm_start=F.FLASH_WS_LEARNED)
    b = F.from_scene(sc, warm_start=F.FLASH_WS_LEARNED, fused_lg=True)
    for x in (a, b):
        x.ws_load(w16, norm)
        x.step(6)
    _same(a, b, "learned")
    cap = 2 * 320
    rows = []
    for x in (a, b):
        x.ws_record(True)
        x.step(2)
        fd = torch.zeros((cap, 16), dtype=torch.float32, device="cuda")
        ld = torch.zeros((cap, 3), dtype=torch.float32, device="cuda")
        n = x.ws_collect(fd, ld, cap, 0)
        rows.append((n, fd[:n].cpu().numpy(), ld[:n].cpu().numpy()))
        x.ws_record(False)
    assert rows[0][0] == rows[1][0] > 0
    assert np.array_equal(rows[0][1], rows[1][1]) and np.array_equal(rows[0][2], rows[1][2])
    _same(a, b, "after recording")


def test_tiny_contact_capacity_fallbacks():
    """A contact capacity of 4 (capacitance systems of at most 12 rows, too small for the staged
    16 x 16 diagonal blocks) takes the memory paths of the capacitance solves: the run stays
    finite, flags the overflow, and fused equals per-phase bitwise."""
    F = _F()
    sc = scenes.drop_cube(seed=45, hexes=3, drop_height=0.0005, jitter=0.0)
    a = F.from_scene(sc, max_contacts=4)
    b = F.from_scene(sc, max_contacts=4, fused_lg=True)
    a.step(4)
    b.step(4)
    _same(a, b, "tiny capacity")
    x = b.get_state()[0]
    st = b.stats()
    _say("tiny capacity contacts", [s_["contacts"] for s_ in st], "flags", [s_["flags"] for s_ in st])
    assert np.all(np.isfinite(x))
    assert st[0]["contacts"] == 4 and st[0]["flags"] & 4


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_largest_contact_capacity_is_bitwise_default(precision):
    """The largest contact capacity create accepts with the FP64 contact solve (330 contacts per
    env: the CU's 160 KB of LDS less the static reserve) runs full-size squeeze blocks with the
    bits of the default capacity (320): the capacity sets strides and overflow limits only, and
    these envs (about 219 contacts) reach neither.  Fused loop, 3 envs, 8 steps.  The larger
    batch is created first: creating a smaller one afterwards must not lower the LDS limit it
    launches with."""
    F = _F()
    sc = scenes.squeeze_blocks(3, seed=47)
    kw = {} if precision == "fp32" else {"precision": F.FLASH_FP64}
    b = F.from_scene(sc, fused_lg=True, max_contacts=330, **kw)
    a = F.from_scene(sc, fused_lg=True, **kw)
    a.step(8)
    b.step(8)
    st = b.stats()
    _say(f"capacity 330 {precision}: contacts {[s_['contacts'] for s_ in st]}")
    _same(a, b, f"capacity 330 {precision}")
    assert all(s_["contacts"] > 150 and not (s_["flags"] & 4) for s_ in st)


def test_fp32_contact_solve_at_its_largest_capacity():
    """An FP32 batch that solves its contacts in FP32 (contact_fp32) at the largest capacity
    create accepts for it (814 contacts per env): the drop cube through touchdown and settling
    matches the oracle's steps (same contact lists, positions within 1e-5 relative, NCP residual
    of the GPU positions and multipliers <= 1e-6 m), and the fused loop gives the bits of the
    per-phase launches."""
    F = _F()
    sc = scenes.drop_cube(seed=49)
    oes = {0: O.precompute(sc.envs[0], sc.params.h)}
    a = F.from_scene(sc, contact_fp32=True, max_contacts=814)
    b = F.from_scene(sc, contact_fp32=True, max_contacts=814, fused_lg=True)
    checked = 0
    for s in range(24):
        if s in (11, 12, 13, 16, 23):
            xg, vg = b.get_state()
            x0, v0 = b.split(xg)[0], b.split(vg)[0]
            obs = b.get_obstacles(0)
            a.step(1)
            b.step(1)
            ref = O.step(oes[0], x0, v0, obs, sc.params, tol=1e-12)
            x1 = b.split(b.get_state()[0])[0]
            L = np.linalg.norm(sc.envs[0].rest_x.max(0) - sc.envs[0].rest_x.min(0))
            err = np.abs(x1 - ref.x).max()
            gc = b.contacts(0)
            same = (gc["vertex"].tolist() == ref.contacts.vertex.tolist()
                    and gc["obstacle"].tolist() == ref.contacts.obstacle.tolist())
            r = O.contact_residual(oes[0], x0, x1, ref.contacts, gc["lambda"], sc.params.h) if same else np.inf
            _say(f"contact_fp32 step {s}: {len(gc['vertex'])} contacts, max|dq| {err:.3e}, residual {r:.2e}")
            assert same
            assert err <= 1e-5 * max(np.abs(ref.x).max(), L)
            assert r <= 1e-6
            checked += 1
        else:
            a.step(1)
            b.step(1)
        _same(a, b, f"contact_fp32 step {s}")
    assert checked == 5
    mx, over = b.residual_history(reset=True)
    assert mx <= sc.params.ncp_tol and over == 0
