"""GPU parity of batched depth ray casting (supplementary: depth simulation -- depth maps, instance
masks and point clouds cast from the simulation state) against the FP64 brute-force oracle.

Bar: instance ids equal except on the oracle's silhouettes (pixels with a neighbour of another
instance, where a rounding difference may move the edge by a pixel: the GPU's id must then be one
the oracle shows next to the pixel) and at depth ties (the surface's
and an obstacle's nearest hits within 1e-5 relative, as where a sheet lies on the table: either id is
right); depth and point cloud within 1e-5 relative (FP32 against FP64) wherever the instances agree
or tie.  The GPU renders the simulation's own
device state (read with flash_get_state_device)."""
import math
import sys

import numpy as np
import pytest

from oracle import render_oracle as RO
from paper_2604_17513_amd import scenes

pytestmark = pytest.mark.gpu


def _F():
    from paper_2604_17513_amd import flash as F
    return F


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _look_at(pos, target, fx, w, h):
    pos, target = np.asarray(pos, float), np.asarray(target, float)
    fwd = target - pos
    fwd /= np.linalg.norm(fwd)
    right = np.cross(fwd, np.array([0.0, 1.0, 0.0]))
    if np.linalg.norm(right) < 1e-9:
        right = np.array([1.0, 0.0, 0.0])
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    return {"position": pos, "rot": np.stack([right, down, fwd], axis=1), "fx": fx, "fy": fx, "cx": w / 2.0,
            "cy": h / 2.0}


def _silhouette(inst):
    """Pixels with a 4-neighbour of another instance."""
    s = np.zeros_like(inst, dtype=bool)
    s[1:, :] |= inst[1:, :] != inst[:-1, :]
    s[:-1, :] |= inst[:-1, :] != inst[1:, :]
    s[:, 1:] |= inst[:, 1:] != inst[:, :-1]
    s[:, :-1] |= inst[:, :-1] != inst[:, 1:]
    return s


def _ties(xe, tris, obs, cam, W, H):
    """Pixels where the surface's and an obstacle's nearest hits are within 1e-5 relative."""
    ds, _, _ = RO.render(xe, tris, [], cam, W, H)
    do, _, _ = RO.render(np.zeros((0, 3)), np.zeros((0, 3), int), obs, cam, W, H)
    both = (ds > 0) & (do > 0)
    return both & (np.abs(ds - do) <= 1e-5 * np.maximum(ds, do))


def _compare(label, depth, inst, pts, ref_depth, ref_inst, ref_pts, ties):
    sil = _silhouette(ref_inst)
    bad = (inst != ref_inst) & ~sil & ~ties
    agree = ((inst == ref_inst) | (ties & (inst >= 0))) & (ref_inst >= 0)
    rel = np.abs(depth - ref_depth)[agree] / ref_depth[agree]
    perr = np.linalg.norm(pts - ref_pts, axis=-1)[agree] / ref_depth[agree]
    n_sil = int(((inst != ref_inst) & sil).sum())
    _say(f"{label}: hit pixels {int((ref_inst >= 0).sum())} of {ref_inst.size}, instance mismatches on "
         f"silhouettes {n_sil}, at depth ties {int(((inst != ref_inst) & ties).sum())}, elsewhere "
         f"{int(bad.sum())}; max depth rel err {rel.max() if rel.size else 0:.2e}, "
         f"max point err / depth {perr.max() if perr.size else 0:.2e}")
    assert not bad.any()
    # a silhouette mismatch moved the edge by at most a pixel: the GPU's instance is one the oracle
    # shows within the pixel's 3 x 3 neighbourhood
    Hh, Ww = ref_inst.shape
    pad = np.pad(ref_inst, 1, constant_values=-2)
    for v, u in zip(*np.nonzero((inst != ref_inst) & sil)):
        assert inst[v, u] in pad[v:v + 3, u:u + 3], (label, v, u)
    assert rel.size == 0 or rel.max() <= 1e-5
    assert perr.size == 0 or perr.max() <= 1e-5
    assert np.all(depth[ref_inst < 0][inst[ref_inst < 0] < 0] == 0.0)


def _state_on_device(b, torch):
    n = sum(b.nv)
    x = torch.empty((3, n), dtype=torch.float32, device="cuda")
    b.get_state_device(x)
    torch.cuda.synchronize()
    return x


def test_render_deformed_sheets_and_a_squeezed_block_matches_oracle():
    """Two envs of the folding stand-in after 30 steps (sheets lifted at the corners over the table)
    and one squeezed tet block (its boundary faces, two box fingers and the ground), each seen by an
    oblique camera; depth, instances and points against the oracle."""
    import torch
    F = _F()
    fold = scenes.cloth_fold(2, n=24)
    bf = F.from_scene(fold, contact_metric=F.FLASH_METRIC_LIGHTWEIGHT, max_contacts=24 * 24 + 8)
    bf.step(30)
    sq = scenes.squeeze_blocks(1, seed=3, hexes=5)
    bs = F.from_scene(sq)
    bs.step(25)
    xf = _state_on_device(bf, torch)
    xs = _state_on_device(bs, torch)
    x = torch.cat([xf, xs], dim=1)
    envs = fold.envs + sq.envs
    obs = [bf.get_obstacles(0), bf.get_obstacles(1), bs.get_obstacles(0)]
    W, H = 96, 72
    cams = [_look_at((0.35, 0.55, -0.45), (0.0, 0.0, 0.0), 70.0, W, H),
            _look_at((-0.2, 0.7, 0.3), (0.0, 0.02, 0.0), 90.0, W, H),
            _look_at((0.25, 0.3, -0.3), (0.0, 0.05, 0.0), 80.0, W, H)]
    R = F.Renderer(envs)
    out = R.render(x, cams, W, H, obstacles=obs, points=True)
    depth, inst, pts = (out[k].cpu().numpy() for k in ("depth", "instance", "points"))
    xh = x.cpu().numpy().astype(np.float64).T
    offs = np.concatenate([[0], np.cumsum([e.n_vertices for e in envs])])
    for e, env in enumerate(envs):
        xe = xh[offs[e]:offs[e + 1]]
        tris = RO.surface_triangles(env.elem, env.elements)
        rd, ri, rp = RO.render(xe, tris, obs[e], cams[e], W, H)
        assert (ri == 0).sum() > 200 and len(set(np.unique(ri)) - {-1, 0}) >= 1
        _compare(f"env {e}", depth[e], inst[e], pts[e], rd, ri, rp, _ties(xe, tris, obs[e], cams[e], W, H))
    R.close()


def test_identical_envs_share_a_hierarchy_and_render_alike():
    """Three identical sheets at the same state and camera give bitwise equal images; one env alone
    renders the same bits as inside the batch; a near-top-down view of a flat sheet on the table gives
    the closed-form depth."""
    import torch
    F = _F()
    sc = scenes.cloth_fold(3, n=16)
    W, H = 64, 48
    cam = _look_at((0.0, 0.8, 1e-3), (0.0, 0.0, 0.0), 60.0, W, H)
    x = torch.tensor(np.concatenate(sc.x0).T.copy(), dtype=torch.float32, device="cuda")
    R = F.Renderer(sc.envs)
    out = R.render(x, [cam] * 3, W, H, obstacles=[[scenes.ground()]] * 3)
    d = out["depth"].cpu().numpy()
    i = out["instance"].cpu().numpy()
    assert np.array_equal(d[0], d[1]) and np.array_equal(d[0], d[2]) and np.array_equal(i[0], i[2])
    R1 = F.Renderer(sc.envs[:1])
    one = R1.render(x[:, :sc.envs[0].n_vertices], [cam], W, H, obstacles=[[scenes.ground()]])
    assert np.array_equal(one["depth"].cpu().numpy()[0], d[0])
    # the centre pixel sees the sheet 1 mm above the table almost straight down
    fwd = cam["rot"][:, 2]
    t_sheet = (cam["position"][1] - 1e-3) / -fwd[1]
    assert i[0, H // 2, W // 2] == 0
    assert math.isclose(d[0, H // 2, W // 2], t_sheet, rel_tol=2e-4)
    R.close()
    R1.close()


def test_render_rejects_invalid_arguments():
    import torch
    F = _F()
    sc = scenes.cloth_fold(1, n=8)
    R = F.Renderer(sc.envs)
    x = torch.tensor(sc.x0[0].T.copy(), dtype=torch.float32, device="cuda")
    cam = _look_at((0.0, 0.5, 0.01), (0.0, 0.0, 0.0), 40.0, 16, 16)
    bad = dict(cam, fx=0.0)
    with pytest.raises(F.FlashError):
        R.render(x, [bad], 16, 16)
    with pytest.raises(F.FlashError):
        R.render(x, [cam], 0, 16)
    with pytest.raises(F.FlashError):
        R.render(x, [cam], 16, 16, obstacles=[[scenes.ground()] * 5])
    R.close()
