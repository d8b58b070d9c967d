"""Pins of the ray-casting oracle (supplementary: depth simulation -- depth maps, instance masks and
point clouds cast from the simulation state), each by a route other than the oracle's own ray solve:

* a horizontal sheet under a top-down camera: coverage from back-projecting pixel centres onto its
  plane and testing the square, depth = camera height - sheet height;
* random triangles: coverage equals the 2-D point-in-triangle test of the pixel centre against the
  perspective projections of the vertices; depth equals the triangle's plane equation solved along
  the ray;
* the ground plane under an oblique camera: depth in closed form per pixel;
* a box seen face-on and a capsule seen across its axis: distances in closed form;
* occlusion: the nearer of two sheets wins, instance ids follow;
* the point cloud reprojects to the pixel centres at the reported depth;
* boundary faces of a tet lattice: every face once, each on the lattice's outer surface (faces are
  two-sided for ray casting, so their orientation is not fixed).
"""
import math

import numpy as np
import pytest

from oracle import render_oracle as R
from paper_2604_17513_amd import scenes


def _top_down(height, fx=80.0, w=48, h=40):
    # camera at (0, height, 0) looking down -y; image right = +x, image down = +z
    rot = np.array([[1.0, 0.0, 0.0], [0.0, 0.0, -1.0], [0.0, 1.0, 0.0]])
    return {"position": np.array([0.0, height, 0.0]), "rot": rot, "fx": fx, "fy": fx, "cx": w / 2.0, "cy": h / 2.0}


def test_horizontal_sheet_under_a_top_down_camera():
    cam = _top_down(0.5, fx=40.0)
    W, H = 48, 40
    rest, tris = scenes.cloth_grid(9, 0.3, (-0.15, -0.15), 0.1)
    depth, inst, pts = R.render(rest, tris, [], cam, W, H)
    u, v = np.meshgrid(np.arange(W) + 0.5, np.arange(H) + 0.5)
    dist = 0.5 - 0.1
    X = (u - cam["cx"]) / cam["fx"] * dist
    Z = (v - cam["cy"]) / cam["fy"] * dist
    inside = (np.abs(X) < 0.15 - 1e-9) & (np.abs(Z) < 0.15 - 1e-9)
    outside = (np.abs(X) > 0.15 + 1e-9) | (np.abs(Z) > 0.15 + 1e-9)
    assert inside.sum() > 100 and outside.sum() > 100
    assert np.all(inst[inside] == 0) and np.all(inst[outside] == -1)
    np.testing.assert_allclose(depth[inside], dist, rtol=0, atol=1e-12)
    assert np.all(depth[outside] == 0.0)


@pytest.mark.parametrize("seed", range(4))
def test_random_triangles_match_the_projected_2d_test_and_plane_depth(seed):
    rng = np.random.default_rng(seed)
    W, H = 32, 24
    cam = {"position": np.zeros(3), "rot": np.eye(3), "fx": 30.0, "fy": 30.0, "cx": W / 2.0, "cy": H / 2.0}
    m = 6
    x = np.concatenate([rng.uniform(-0.6, 0.6, (3 * m, 2)), rng.uniform(1.0, 3.0, (3 * m, 1))], axis=1)
    tris = np.arange(3 * m).reshape(m, 3)
    depth, inst, _ = R.render(x, tris, [], cam, W, H)
    # projections of the vertices (camera frame = world frame here)
    pu = cam["fx"] * x[:, 0] / x[:, 2] + cam["cx"]
    pv = cam["fy"] * x[:, 1] / x[:, 2] + cam["cy"]
    u, v = np.meshgrid(np.arange(W) + 0.5, np.arange(H) + 0.5)
    best = np.full((H, W), np.inf)
    margin = np.full((H, W), np.inf)
    for a, b, c in tris:
        def edge(i, j):
            return (pu[j] - pu[i]) * (v - pv[i]) - (pv[j] - pv[i]) * (u - pu[i])
        e0, e1, e2 = edge(a, b), edge(b, c), edge(c, a)
        ins = ((e0 >= 0) & (e1 >= 0) & (e2 >= 0)) | ((e0 <= 0) & (e1 <= 0) & (e2 <= 0))
        margin = np.minimum(margin, np.minimum(np.minimum(np.abs(e0), np.abs(e1)), np.abs(e2)))
        # depth from the plane through the three vertices along the pixel's ray d = (xn, yn, 1)
        n = np.cross(x[b] - x[a], x[c] - x[a])
        xn = (u - cam["cx"]) / cam["fx"]
        yn = (v - cam["cy"]) / cam["fy"]
        t = (n @ x[a]) / (n[0] * xn + n[1] * yn + n[2])
        best = np.where(ins & (t > 0) & (t < best), t, best)
    clear = margin > 1e-6
    hit = np.isfinite(best)
    assert np.array_equal((inst == 0)[clear], hit[clear])
    np.testing.assert_allclose(depth[clear & hit], best[clear & hit], rtol=1e-12, atol=0)


def test_ground_plane_under_an_oblique_camera():
    tilt = math.radians(35.0)
    # camera at height 0.8 looking along (0, -sin, cos): rotate the top-down frame by the tilt
    fwd = np.array([0.0, -math.sin(tilt), math.cos(tilt)])
    right = np.array([1.0, 0.0, 0.0])
    down = np.cross(fwd, right)
    cam = {"position": np.array([0.0, 0.8, 0.0]), "rot": np.stack([right, down, fwd], axis=1),
           "fx": 40.0, "fy": 40.0, "cx": 20.0, "cy": 15.0}
    depth, inst, _ = R.render(np.zeros((0, 3)), np.zeros((0, 3), int), [scenes.ground()], cam, 40, 30)
    u, v = np.meshgrid(np.arange(40) + 0.5, np.arange(30) + 0.5)
    dw = ((u - 20.0) / 40.0)[..., None] * right + ((v - 15.0) / 40.0)[..., None] * down + fwd
    t = np.where(dw[..., 1] < 0, 0.8 / -dw[..., 1], 0.0)
    np.testing.assert_allclose(depth, t, rtol=1e-13, atol=0)
    assert np.array_equal(inst, np.where(t > 0, 1, -1))


def test_box_face_on_and_capsule_across_its_axis():
    cam = _top_down(1.0, w=32, h=32)
    box = scenes.box((0.0, 0.2, 0.0), (0.1, 0.05, 0.1))
    depth, inst, _ = R.render(np.zeros((0, 3)), np.zeros((0, 3), int), [box], cam, 32, 32)
    assert inst[16, 16] == 1 and math.isclose(depth[16, 16], 1.0 - 0.25, rel_tol=1e-14)
    cap = scenes.Obstacle(scenes.CAPSULE, np.array([0.0, 0.3, 0.0]), np.eye(3), np.array([0.04, 0.05, 0.0]),
                          np.zeros(3), -1)
    depth, inst, _ = R.render(np.zeros((0, 3)), np.zeros((0, 3), int), [cap], cam, 32, 32)
    o, D = R.camera_rays(cam, 32, 32)
    d = D[16 * 32 + 16]
    # closed form: |(o + t d) - axis point| = r with the axis along x: solve in the (y, z) plane
    a = d[1] ** 2 + d[2] ** 2
    b = 2 * ((o[1] - 0.3) * d[1] + o[2] * d[2])
    c = (o[1] - 0.3) ** 2 + o[2] ** 2 - 0.04 ** 2
    t = (-b - math.sqrt(b * b - 4 * a * c)) / (2 * a)
    assert inst[16, 16] == 1 and math.isclose(depth[16, 16], t, rel_tol=1e-13)
    # beyond the half-length the spherical caps end the capsule
    x_end = 0.05 + 0.04
    u_end = int(cam["cx"] + cam["fx"] * x_end / (1.0 - 0.3)) + 2
    assert inst[16, u_end] == -1


def test_occlusion_order_and_point_cloud():
    cam = _top_down(0.6, w=40, h=40)
    near, tn = scenes.cloth_grid(5, 0.1, (-0.05, -0.05), 0.2)
    far, tf = scenes.cloth_grid(5, 0.2, (-0.1, -0.1), 0.1)
    x = np.concatenate([near, far])
    tris = np.concatenate([tn, tf + near.shape[0]])
    box = scenes.box((0.0, 0.02, 0.0), (0.3, 0.02, 0.3))
    depth, inst, pts = R.render(x, tris, [box], cam, 40, 40)
    assert math.isclose(depth[20, 20], 0.4, rel_tol=1e-12) and inst[20, 20] == 0      # near sheet
    assert math.isclose(depth[20, 8], 0.5, rel_tol=1e-12) and inst[20, 8] == 0        # far sheet only
    assert math.isclose(depth[0, 0], 0.56, rel_tol=1e-12) and inst[0, 0] == 1         # the box top
    # reprojection of the cloud
    hit = inst >= 0
    Rm = cam["rot"]
    pc = (pts - cam["position"]) @ Rm
    u = cam["fx"] * pc[..., 0] / pc[..., 2] + cam["cx"]
    v = cam["fy"] * pc[..., 1] / pc[..., 2] + cam["cy"]
    uu, vv = np.meshgrid(np.arange(40) + 0.5, np.arange(40) + 0.5)
    np.testing.assert_allclose(u[hit], uu[hit], atol=1e-9)
    np.testing.assert_allclose(v[hit], vv[hit], atol=1e-9)
    np.testing.assert_allclose(pc[..., 2][hit], depth[hit], rtol=1e-12)


def test_boundary_faces_of_a_tet_lattice():
    rest, tets = scenes.hex_lattice(2, 3, 2, (0.1, 0.1, 0.1), (0.0, 0.0, 0.0))
    f = R.surface_triangles(0, tets)
    # a 2 x 3 x 2 lattice of hexes, each outer quad split into 2 triangles
    assert f.shape[0] == 2 * 2 * (2 * 3 + 3 * 2 + 2 * 2)
    key = {tuple(sorted(t)) for t in f.tolist()}
    assert len(key) == f.shape[0]
    lo, hi = rest.min(0), rest.max(0)
    for t in f:
        p = rest[t]
        on = np.any([np.all(np.isclose(p[:, k], lo[k])) or np.all(np.isclose(p[:, k], hi[k])) for k in range(3)])
        assert on
    # the faces tile the outer surface: their areas add up to the box's surface area
    area = 0.5 * np.linalg.norm(np.cross(rest[f[:, 1]] - rest[f[:, 0]], rest[f[:, 2]] - rest[f[:, 0]]), axis=1).sum()
    ext = hi - lo
    assert abs(area - 2 * (ext[0] * ext[1] + ext[1] * ext[2] + ext[0] * ext[2])) < 1e-12
