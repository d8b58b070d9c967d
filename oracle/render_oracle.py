"""Oracle of batched depth ray casting (supplementary: depth simulation and perception -- depth
maps, instance segmentation masks and point clouds cast from the simulation state).

TEST INFRASTRUCTURE ONLY.  Only tests, the smoke check and the benchmark's CPU baseline may import
this module; the library never does.  It is a plain, slow, FP64 brute force: every pixel's ray is
intersected with every surface triangle and every obstacle and the nearest hit is kept.

Camera model (the reading used by both sides): a pinhole with intrinsics (fx, fy, cx, cy) in pixels,
position p and camera-to-world rotation R whose columns are the camera's x (image right), y (image
down) and z (optical axis) directions in world coordinates.  Pixel (u, v) (column, row) casts the
ray p + t R d with d = ((u + 0.5 - cx) / fx, (v + 0.5 - cy) / fy, 1): with d's third component 1 the
ray parameter t of a hit IS its depth along the optical axis.  A pixel whose ray hits nothing in
front of the camera (t > 0) has depth 0 (no return, as depth cameras report) and instance -1;
instance 0 is the env's deformable body, 1 + o is obstacle o.  The point cloud holds the world
position of each pixel's hit (zero where none).
"""
from __future__ import annotations

import numpy as np

PLANE, BOX, CAPSULE = 0, 1, 2
EDGE_BAND = 1e-9


def surface_triangles(elem_kind: int, elements: np.ndarray) -> np.ndarray:
    """The triangles a body shows to a camera: membrane triangles as they are (elem_kind 1), or the
    boundary faces of a tet mesh (faces that belong to exactly one tet, elem_kind 0)."""
    el = np.asarray(elements, dtype=np.int64)
    if elem_kind == 1:
        return el[:, :3].copy()
    faces = np.concatenate([el[:, [1, 2, 3]], el[:, [0, 3, 2]], el[:, [0, 1, 3]], el[:, [0, 2, 1]]])
    key = np.sort(faces, axis=1)
    _, inv, cnt = np.unique(key, axis=0, return_inverse=True, return_counts=True)
    return faces[cnt[inv.ravel()] == 1]


def camera_rays(cam, width: int, height: int):
    """Origin (3,) and world directions (height*width, 3) of every pixel, row-major (v, u)."""
    fx, fy, cx, cy = cam["fx"], cam["fy"], cam["cx"], cam["cy"]
    R = np.asarray(cam["rot"], dtype=np.float64).reshape(3, 3)
    u, v = np.meshgrid(np.arange(width, dtype=np.float64), np.arange(height, dtype=np.float64))
    d = np.stack([(u.ravel() + 0.5 - cx) / fx, (v.ravel() + 0.5 - cy) / fy, np.ones(width * height)], axis=1)
    return np.asarray(cam["position"], dtype=np.float64), d @ R.T


def ray_triangles(o, D, A, B, C):
    """Nearest t > 0 of each ray o + t D (D: (r, 3)) over triangles (A, B, C: (m, 3)) by the
    Moller-Trumbore solve of o + t d = A + b1 (B - A) + b2 (C - A), hit iff b1, b2 and 1 - b1 - b2
    are all >= -EDGE_BAND and t > 0: a closed band of 1e-9 in barycentric coordinates, so that a
    ray along an edge shared by two triangles hits one of them whatever the rounding (watertight),
    while a silhouette grows by a negligible 1e-9 of a triangle.  Returns t (inf where none) and
    the index of the hit triangle."""
    e1 = B - A
    e2 = C - A
    s = o - A                                  # (m, 3)
    P = np.cross(D[:, None, :], e2[None, :, :])            # (r, m, 3)
    det = np.einsum("rmk,mk->rm", P, e1)
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / det
        b1 = np.einsum("rmk,mk->rm", P, s) * inv
        Q = np.cross(s, e1)                                 # (m, 3)
        b2 = np.einsum("rk,mk->rm", D, Q) * inv
        t = np.einsum("mk,mk->m", e2, Q)[None, :] * inv
    hit = (det != 0) & (b1 >= -EDGE_BAND) & (b2 >= -EDGE_BAND) & (b1 + b2 <= 1 + EDGE_BAND) & (t > 0)
    t = np.where(hit, t, np.inf)
    k = np.argmin(t, axis=1)
    return t[np.arange(D.shape[0]), k], k


def ray_obstacle(o, D, ob) -> np.ndarray:
    """Nearest t > 0 of each ray with one obstacle (inf where none): the plane through its center
    with normal R e_y, the box with half-extents size (slab test in its frame), or the capsule of
    radius size[0] around its axis R e_x with half-length size[1]."""
    c = np.asarray(ob.center, dtype=np.float64)
    R = np.asarray(ob.rot, dtype=np.float64).reshape(3, 3)
    r = D.shape[0]
    if ob.kind == PLANE:
        n = R[:, 1]
        dn = D @ n
        with np.errstate(divide="ignore", invalid="ignore"):
            t = (c - o) @ n / dn
        return np.where((dn != 0) & (t > 0), t, np.inf)
    ol = R.T @ (o - c)
    Dl = D @ R
    if ob.kind == BOX:
        e = np.asarray(ob.size, dtype=np.float64)
        with np.errstate(divide="ignore", invalid="ignore"):
            t1 = (-e[None, :] - ol[None, :]) / Dl
            t2 = (e[None, :] - ol[None, :]) / Dl
        lo = np.where(Dl == 0, np.where(np.abs(ol[None, :]) <= e[None, :], -np.inf, np.inf), np.minimum(t1, t2))
        hi = np.where(Dl == 0, np.where(np.abs(ol[None, :]) <= e[None, :], np.inf, -np.inf), np.maximum(t1, t2))
        tn, tf = lo.max(axis=1), hi.min(axis=1)
        t = np.where(tn > 0, tn, tf)           # entering hit, or the exit hit from inside
        return np.where((tn <= tf) & (t > 0), t, np.inf)
    # capsule: nearest root over the cylinder wall and the two end spheres
    rad, half = float(ob.size[0]), float(ob.size[1])
    best = np.full(r, np.inf)
    # cylinder |(x - axis part)| = rad with x = ol + t Dl, axis e_x, |x_0| <= half
    a = Dl[:, 1] ** 2 + Dl[:, 2] ** 2
    b = 2 * (ol[1] * Dl[:, 1] + ol[2] * Dl[:, 2])
    cc = ol[1] ** 2 + ol[2] ** 2 - rad * rad
    disc = b * b - 4 * a * cc
    with np.errstate(divide="ignore", invalid="ignore"):
        for sgn in (-1.0, 1.0):
            t = (-b + sgn * np.sqrt(np.maximum(disc, 0))) / (2 * a)
            x0 = ol[0] + t * Dl[:, 0]
            ok = (a > 0) & (disc >= 0) & (t > 0) & (np.abs(x0) <= half)
            best = np.where(ok & (t < best), t, best)
    for end in (-half, half):
        oc = ol - np.array([end, 0.0, 0.0])
        bb = Dl @ oc
        dd = np.einsum("rk,rk->r", Dl, Dl)
        c2 = oc @ oc - rad * rad
        disc = bb * bb - dd * c2
        for sgn in (-1.0, 1.0):
            t = (-bb + sgn * np.sqrt(np.maximum(disc, 0))) / dd
            ok = (disc >= 0) & (t > 0)
            best = np.where(ok & (t < best), t, best)
    return best


def render(x, tris, obstacles, cam, width: int, height: int, chunk: int = 512):
    """Depth (height, width), instance (height, width) and point cloud (height, width, 3) of one env:
    surface x (n, 3) with triangles tris (m, 3), obstacles as scenes.Obstacle records."""
    x = np.asarray(x, dtype=np.float64)
    tris = np.asarray(tris, dtype=np.int64)
    o, D = camera_rays(cam, width, height)
    npx = width * height
    tbest = np.full(npx, np.inf)
    inst = np.full(npx, -1, dtype=np.int64)
    A, B, C = x[tris[:, 0]], x[tris[:, 1]], x[tris[:, 2]]
    for r0 in range(0, npx, chunk):
        sl = slice(r0, min(r0 + chunk, npx))
        if tris.shape[0]:
            t, _ = ray_triangles(o, D[sl], A, B, C)
            better = t < tbest[sl]
            tbest[sl] = np.where(better, t, tbest[sl])
            inst[sl] = np.where(better, 0, inst[sl])
    for q, ob in enumerate(obstacles):
        t = ray_obstacle(o, D, ob)
        better = t < tbest
        tbest = np.where(better, t, tbest)
        inst = np.where(better, 1 + q, inst)
    hit = np.isfinite(tbest)
    depth = np.where(hit, tbest, 0.0)
    pts = np.where(hit[:, None], o[None, :] + tbest[:, None] * D, 0.0)
    return depth.reshape(height, width), inst.reshape(height, width), pts.reshape(height, width, 3)


def silhouette_margin(x, tris, cam, width: int, height: int, chunk: int = 512) -> np.ndarray:
    """Per pixel, how far the ray passes from the edges of the triangles it hits or nearly hits: the
    smallest |barycentric coordinate| over triangles whose solve has t > 0 and all coordinates
    above -0.5 (1.0 where no triangle comes near).  Pixels with a tiny margin sit on an edge: a
    rounding difference may flip which triangle, or whether any, is hit there."""
    x = np.asarray(x, dtype=np.float64)
    tris = np.asarray(tris, dtype=np.int64)
    o, D = camera_rays(cam, width, height)
    A, B, C = x[tris[:, 0]], x[tris[:, 1]], x[tris[:, 2]]
    e1, e2 = B - A, C - A
    s = o - A
    Q = np.cross(s, e1)
    out = np.ones(width * height)
    for r0 in range(0, width * height, chunk):
        Dc = D[r0:r0 + chunk]
        P = np.cross(Dc[:, None, :], e2[None, :, :])
        det = np.einsum("rmk,mk->rm", P, e1)
        with np.errstate(divide="ignore", invalid="ignore"):
            inv = 1.0 / det
            b1 = np.einsum("rmk,mk->rm", P, s) * inv
            b2 = np.einsum("rk,mk->rm", Dc, Q) * inv
            t = np.einsum("mk,mk->m", e2, Q)[None, :] * inv
        b0 = 1 - b1 - b2
        near = (det != 0) & (t > 0) & (b0 > -0.5) & (b1 > -0.5) & (b2 > -0.5)
        m = np.minimum(np.minimum(np.abs(b0), np.abs(b1)), np.abs(b2))
        out[r0:r0 + chunk] = np.where(near, m, 1.0).min(axis=1)
    return out.reshape(height, width)
