"""Pins of the oracle's cloth precompute: membrane triangles and bending hinges.

Everything here is computed by a route that does not go through the oracle's
own rest frames: the membrane strain energy from Gram matrices of the rest and
deformed edges (frame-free), the bending term from exact dihedral angles of the
two triangle normals, masses and weights from the lattice's closed forms, and
whole-step behaviour from closed forms (rigid motion, free flight).  The
readings pinned are those of Sec. III-B (projective internal forces, Eq. 3)
for cloth: weight w = 2 mu_L A t per triangle, row-sum lumped masses
rho t A / 3 per triangle vertex, and a hinge term w_h |sum alpha_a x_a|^2 with
w_h = 3 k_b |e|^2 / (A_1 + A_2) on every interior edge.
"""
import math

import numpy as np
import pytest

from oracle import flash_oracle as O
from paper_2604_17513_amd import scenes


def _sheet(n=7, side=0.3, bending=0.2, young=3e4, poisson=0.4, thickness=1e-3, density=1000.0):
    rest, tris = scenes.cloth_grid(n, side, (-side / 2, -side / 2), 0.0)
    env = scenes.EnvDesc(scenes.TRI, rest, tris, density=density, thickness=thickness, young=young,
                         poisson=poisson, bending=bending, mu=0.5)
    return env


def _interior_edges(tris):
    """Interior edges with their two opposite vertices, found by brute force over triangle pairs."""
    out = []
    m = len(tris)
    for a in range(m):
        for b in range(a + 1, m):
            common = sorted(set(tris[a]) & set(tris[b]))
            if len(common) == 2:
                oa = [v for v in tris[a] if v not in common][0]
                ob = [v for v in tris[b] if v not in common][0]
                out.append((common[0], common[1], oa, ob))
    return out


def _dihedral(x, i0, i1, i2, i3):
    """Exact angle between the normals of triangles (i0, i1, i2) and (i0, i1, i3) of a hinge."""
    e = x[i1] - x[i0]
    n1 = np.cross(e, x[i2] - x[i0])
    n2 = np.cross(x[i3] - x[i0], e)
    # both normals point to the same side for a flat hinge; the fold is the angle between them
    s = np.dot(np.cross(n1, n2), e / np.linalg.norm(e))
    c = np.dot(n1, n2)
    return math.atan2(s, c)


def test_cloth_masses_sum_to_areal_density_times_area():
    env = _sheet(n=9, side=0.4)
    h = 1.0 / 60.0
    oe = O.precompute(env, h)
    total = env.density * env.thickness * 0.4 * 0.4
    assert math.isclose(oe.mass.sum(), total, rel_tol=1e-13)
    # each vertex carries a third of rho t A of every incident triangle; on the lattice every
    # triangle has area a^2 / 2, so m_v = rho t a^2 / 6 times the number of incident triangles
    a = 0.4 / 8
    counts = np.zeros(env.n_vertices)
    for t in env.elements:
        for vtx in t:
            counts[vtx] += 1
    np.testing.assert_allclose(oe.mass, env.density * env.thickness * a * a / 6.0 * counts, rtol=1e-13)
    # Abar 1 = m: translations carry no membrane or bending energy
    np.testing.assert_allclose(oe.Abar @ np.ones(oe.n), oe.mass, rtol=1e-11, atol=1e-18)


def test_cloth_weights_follow_the_lattice_closed_forms():
    n, side, kb = 8, 0.35, 0.2
    env = _sheet(n=n, side=side, bending=kb)
    oe = O.precompute(env, 1.0 / 60.0)
    a = side / (n - 1)
    mu_L = env.young / (2.0 * (1.0 + env.poisson))
    # membrane: w = 2 mu_L A t with A = a^2 / 2 for every lattice triangle
    np.testing.assert_allclose(oe.weight, mu_L * a * a * env.thickness, rtol=1e-13)
    # hinges: |e|^2 = a^2 on axis-aligned edges (A1 + A2 = a^2 -> w_h = 3 k_b), 2 a^2 on diagonals
    # (w_h = 6 k_b); one hinge per interior edge
    edges = _interior_edges([list(t) for t in env.elements])
    assert oe.hinge_idx.shape[0] == len(edges)
    rest = env.rest_x
    for (i0, i1, i2, i3), w in zip(oe.hinge_idx, oe.hinge_w):
        e = rest[i1] - rest[i0]
        diag = abs(abs(e[0]) - abs(e[2])) < 1e-12
        assert math.isclose(w, (6.0 if diag else 3.0) * kb, rel_tol=1e-12)


@pytest.mark.parametrize("bending", [0.0, 0.2])
def test_cloth_system_matrix_matches_frame_free_energy(bending):
    """q^T (Abar - M) q / h^2 = sum_tri w |F|^2 + sum_hinge w_h theta^2 for small out-of-plane q.

    |F|^2 is taken frame-free as tr(Ds^T Ds (Dm^T Dm)^-1) with 3x2 edge matrices, the fold angle
    theta exactly from the two triangle normals; the sheet lies in y = 0 and q moves only y.
    """
    env = _sheet(n=6, side=0.25, bending=bending)
    h = 1.0 / 60.0
    oe = O.precompute(env, h)
    rest = env.rest_x
    mu_L = env.young / (2.0 * (1.0 + env.poisson))
    rng = np.random.default_rng(11)
    eps = 1e-6
    edges = _interior_edges([list(t) for t in env.elements])
    for _ in range(3):
        qy = eps * rng.normal(size=env.n_vertices)
        lhs = (qy @ (oe.Abar @ qy) - np.sum(oe.mass * qy * qy)) / (h * h)
        x = rest.copy()
        x[:, 1] += qy
        memb = 0.0
        for t in env.elements:
            X = rest[t]
            Dm = np.column_stack([X[1] - X[0], X[2] - X[0]])
            dq = np.zeros((3, 3))
            dq[:, 1] = qy[t]
            Ds = np.column_stack([dq[1] - dq[0], dq[2] - dq[0]])
            area = 0.5 * np.linalg.norm(np.cross(Dm[:, 0], Dm[:, 1]))
            memb += 2 * mu_L * area * env.thickness * np.trace(Ds.T @ Ds @ np.linalg.inv(Dm.T @ Dm))
        bend = 0.0
        for (i0, i1, i2, i3) in edges:
            e = rest[i1] - rest[i0]
            a1 = 0.5 * np.linalg.norm(np.cross(e, rest[i2] - rest[i0]))
            a2 = 0.5 * np.linalg.norm(np.cross(e, rest[i3] - rest[i0]))
            wh = 3.0 * bending * np.dot(e, e) / (a1 + a2)
            bend += wh * _dihedral(x, i0, i1, i2, i3) ** 2
        assert math.isclose(lhs, memb + bend, rel_tol=1e-5)
        if bending > 0:
            assert bend > 0.1 * memb    # the hinge term is really exercised


def test_cloth_rigid_motion_has_no_elastic_force():
    """A rotated and translated flat sheet with g = 0 and uniform velocity moves as q = q~."""
    env = _sheet(n=7, side=0.3, bending=0.2)
    rng = np.random.default_rng(4)
    R = np.linalg.qr(rng.normal(size=(3, 3)))[0]
    if np.linalg.det(R) < 0:
        R[:, 0] = -R[:, 0]
    x0 = env.rest_x @ R.T + np.array([0.1, 2.0, -0.3])
    vel = np.tile([0.2, -0.1, 0.3], (env.n_vertices, 1))
    p = scenes.Params(lg_iterations=4)
    p.gravity = (0.0, 0.0, 0.0)
    oe = O.precompute(env, p.h)
    r = O.step(oe, x0, vel, [], p)
    assert np.max(np.abs(r.x - (x0 + p.h * vel))) <= 1e-13


def test_cloth_free_flight_closed_form():
    """x_n = x0 + n h v0 + h^2 g n(n+1)/2 for a flat sheet far from every obstacle."""
    env = _sheet(n=6, side=0.2, bending=0.2)
    p = scenes.Params(lg_iterations=3)
    oe = O.precompute(env, p.h)
    x = env.rest_x + np.array([0.0, 5.0, 0.0])
    v0 = np.tile([0.05, 0.4, -0.1], (env.n_vertices, 1))
    g = np.array(p.gravity)
    xs, v = x.copy(), v0.copy()
    for n in range(1, 6):
        r = O.step(oe, xs, v, [scenes.ground()], p)
        xs, v = r.x, r.v
        assert r.contacts.count == 0
        xe = x + n * p.h * v0 + p.h * p.h * g * n * (n + 1) / 2
        tol = 1e-12 * n * np.abs(xe).max()      # FP64 rounding of the global solves
        assert np.max(np.abs(xs - xe)) <= tol
        assert np.max(np.abs(v - (v0 + n * p.h * g))) <= 2 * tol / p.h
