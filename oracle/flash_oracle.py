"""FP64 CPU oracle of the FLASH per-timestep NCP step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call this
module; only the tests, the smoke entry and the benchmark's CPU-baseline leg do.
It shares no code with the HIP path: the only thing both sides use is the
seeded input generator module (meshes, materials, obstacle tracks).

The step follows the paper's statement of the problem:

* implicit Euler as a variational problem, predicted state
  q~ = q_h + h v_h + h^2 M^-1 f_ext                         (Sec. III, Eq. 1)
* contact-constrained dynamics with multipliers lambda      (Sec. III-A, Eq. 2)
* projective internal forces p_i = argmin w/2|p - G_i q|^2 + zeta_i(p),
  f_int = sum w_i G_i^T (p_i - G_i q)                       (Sec. III-B, Eq. 3)
* assembled system A q - b - h^2 H^T lambda = 0 with
  A = M + h^2 sum w_i G_i^T G_i,  b = M q~ + h^2 sum w_i G_i^T p_i   (Eq. 4)
* the multi-env pipeline: detect, predict, then k = 1..k_max local
  projections each followed by the contact solve and the position update
  (Alg. 1; block-diagonal batching of Eq. 11-12 means every env is solved
  independently).

Readings where the paper is silent (each is also listed in the design notes):

* constitutive projection: as-rigid-as-possible, i.e. p = closest rotation
  (tets) or closest matrix with orthonormal columns (triangles), weights
  w = 2 mu_L V (tets) and 2 mu_L A t (triangles), mu_L = E / (2 (1 + nu));
  hinge bending term with p = 0 (linearised dihedral angle, flat rest state).
* lumped masses by row sums: rho V / 4 per tet vertex, rho t A / 3 per tri vertex.
* NCP function: min-map for Signorini, Alart-Curnier proximal form for
  Coulomb with a circular cone, residual scale s = h^2 / m_v.
* momentum rows use H^T (the contact Jacobian); the non-smooth Jacobian J only
  enters linearised constraint rows.  The Delta-lambda sign is the one that
  follows from eliminating Eq. 6 (Alg. 1's form, h - J A^-1 g).
* each local-global iteration's contact subproblem is solved to convergence
  (tolerance 1e-12 m here) with the exact Delassus operator W = h^2 H A^-1 H^T,
  so the result does not depend on the inner solver or its warm start.
* contact detection: vertex against kinematic obstacle signed distance, taken
  at the obstacle's end-of-step pose, margin delta_c, evaluated in FP64 with a
  fixed operation order and squared-distance comparisons.
* first projection point q^0 = q~.

Units: SI.  lambda in newtons; impulses P = h F lambda in N s (world frame).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

TET, TRI = 0, 1
PLANE, BOX, CAPSULE = 0, 1, 2


# =============================================================================
# O0 - precompute (Sec. III-B, Eq. 3 element maps; Eq. 4 system matrix; Alg. 1,
# set-up of the per-env operators)
# =============================================================================

def tet_rest(rest_x: np.ndarray, tets: np.ndarray):
    """Rest data of linear tets.

    D_m = [X1-X0 | X2-X0 | X3-X0]; a negative det swaps local vertices 2 and 3;
    V = det D_m / 6; B = D_m^-1.  The element map is F = D_s B, which equals
    sum_a x_a gradN_a^T with gradN_a = row a-1 of B (a = 1..3) and
    gradN_0 = -sum_{a>=1} gradN_a.
    """
    tets = np.array(tets, dtype=np.int64, copy=True)
    X = rest_x[tets]                                    # (m, 4, 3)
    Dm = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=2)
    det = np.linalg.det(Dm)
    neg = det < 0
    if np.any(neg):
        tets[neg, 2], tets[neg, 3] = tets[neg, 3].copy(), tets[neg, 2].copy()
        X = rest_x[tets]
        Dm = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=2)
        det = np.linalg.det(Dm)
    B = np.linalg.inv(Dm)
    vol = det / 6.0
    grad = np.zeros((tets.shape[0], 4, 3))
    grad[:, 1:, :] = B
    grad[:, 0, :] = -B.sum(axis=1)
    return tets, B, vol, grad


def tri_rest(rest_x: np.ndarray, tris: np.ndarray):
    """Rest data of linear triangles (membrane).

    Rest frame e1 = unit(X1-X0), n = unit((X1-X0) x (X2-X0)), e2 = n x e1.
    D_m is the 2x2 matrix of rest edge coordinates in (e1, e2); B = D_m^-1;
    F = [x1-x0 | x2-x0] B (3x2); area = |det D_m| / 2.
    """
    tris = np.asarray(tris, dtype=np.int64)
    X = rest_x[tris]
    E1 = X[:, 1] - X[:, 0]
    E2 = X[:, 2] - X[:, 0]
    e1 = E1 / np.linalg.norm(E1, axis=1, keepdims=True)
    nn = np.cross(E1, E2)
    nn = nn / np.linalg.norm(nn, axis=1, keepdims=True)
    e2 = np.cross(nn, e1)
    Dm = np.empty((tris.shape[0], 2, 2))
    Dm[:, 0, 0] = np.sum(E1 * e1, axis=1)
    Dm[:, 0, 1] = np.sum(E2 * e1, axis=1)
    Dm[:, 1, 0] = np.sum(E1 * e2, axis=1)
    Dm[:, 1, 1] = np.sum(E2 * e2, axis=1)
    det = Dm[:, 0, 0] * Dm[:, 1, 1] - Dm[:, 0, 1] * Dm[:, 1, 0]
    B = np.linalg.inv(Dm)
    area = np.abs(det) / 2.0
    grad = np.zeros((tris.shape[0], 3, 2))
    grad[:, 1:, :] = B
    grad[:, 0, :] = -B.sum(axis=1)
    return tris, B, area, grad


def hinge_stencils(rest_x: np.ndarray, tris: np.ndarray):
    """Bending hinges of a flat-rest triangle mesh.

    For each interior edge (x0, x1) with opposite vertices x2, x3 the stencil
    alpha has alpha_2 = 1/d_2, alpha_3 = 1/d_3 (rest distances to the edge
    line); alpha_0, alpha_1 follow from sum alpha = 0 and sum alpha X^ = 0 in
    the pair's 2-D rest coordinates.  G_h q = sum alpha_a x_a, p_h = 0.
    Returns (idx (k,4), alpha (k,4), edge_len2 (k,), area_sum (k,)).
    """
    tris = np.asarray(tris, dtype=np.int64)
    edge_map = {}
    for t, (a, b, c) in enumerate(tris):
        for (u, v, w) in ((a, b, c), (b, c, a), (c, a, b)):
            key = (min(u, v), max(u, v))
            edge_map.setdefault(key, []).append((t, u, v, w))
    idx, alpha, elen2, asum = [], [], [], []
    for key in sorted(edge_map):
        lst = edge_map[key]
        if len(lst) != 2:
            continue
        (t0, u0, v0, w0), (t1, u1, v1, w1) = lst
        i0, i1 = key
        x0, x1, x2, x3 = rest_x[i0], rest_x[i1], rest_x[w0], rest_x[w1]
        e = x1 - x0
        L = np.linalg.norm(e)
        eh = e / L
        a2 = np.dot(x2 - x0, eh)
        a3 = np.dot(x3 - x0, eh)
        d2 = np.linalg.norm((x2 - x0) - a2 * eh)
        d3 = np.linalg.norm((x3 - x0) - a3 * eh)
        al2 = 1.0 / d2
        al3 = 1.0 / d3
        al1 = -(al2 * a2 + al3 * a3) / L
        al0 = -(al1 + al2 + al3)
        A1 = 0.5 * np.linalg.norm(np.cross(x1 - x0, x2 - x0))
        A2 = 0.5 * np.linalg.norm(np.cross(x1 - x0, x3 - x0))
        idx.append([i0, i1, w0, w1])
        alpha.append([al0, al1, al2, al3])
        elen2.append(L * L)
        asum.append(A1 + A2)
    return (np.asarray(idx, dtype=np.int64).reshape(-1, 4), np.asarray(alpha).reshape(-1, 4),
            np.asarray(elen2), np.asarray(asum))


@dataclass
class OracleEnv:
    """Per-environment constant data (masses, element maps, weights, A)."""
    elem: int
    n: int
    elements: np.ndarray
    grad: np.ndarray            # (m, k, d): gradN_a per element
    weight: np.ndarray          # (m,)
    mass: np.ndarray            # (n,)
    hinge_idx: np.ndarray
    hinge_alpha: np.ndarray
    hinge_w: np.ndarray
    Abar: sp.csc_matrix         # scalar system matrix; A = Abar (x) I3
    mu: float
    _chol: object = None
    _lu: object = None

    def solve(self, rhs: np.ndarray) -> np.ndarray:
        """A^-1 rhs for rhs of shape (n, k) (columns: coordinates or unit vectors)."""
        if self._chol is not None:
            return sla.cho_solve(self._chol, rhs)
        return self._lu.solve(rhs)


def precompute(env, h: float) -> OracleEnv:
    """Masses, element maps, weights and A = M + h^2 sum w G^T G (Eq. 4).

    G^T G for one element is [(gradN_a . gradN_b)]_{ab} (x) I3 because the map
    q -> F acts identically on every coordinate; hence A = Abar (x) I3 with a
    scalar n x n matrix Abar.
    """
    rest = np.asarray(env.rest_x, dtype=np.float64)
    n = rest.shape[0]
    mu_L = env.young / (2.0 * (1.0 + env.poisson))
    hidx = np.zeros((0, 4), dtype=np.int64)
    halpha = np.zeros((0, 4))
    hw = np.zeros(0)
    if env.elem == TET:
        elements, B, vol, grad = tet_rest(rest, env.elements)
        weight = 2.0 * mu_L * vol
        mass = np.zeros(n)
        np.add.at(mass, elements.ravel(), np.repeat(env.density * vol / 4.0, 4))
    else:
        elements, B, area, grad = tri_rest(rest, env.elements)
        weight = 2.0 * mu_L * area * env.thickness
        mass = np.zeros(n)
        np.add.at(mass, elements.ravel(), np.repeat(env.density * env.thickness * area / 3.0, 3))
        if env.bending > 0.0:
            hidx, halpha, elen2, asum = hinge_stencils(rest, elements)
            hw = 3.0 * env.bending * elen2 / asum
    k = elements.shape[1]
    rows, cols, vals = [np.arange(n)], [np.arange(n)], [mass]
    for a in range(k):
        for b in range(k):
            rows.append(elements[:, a])
            cols.append(elements[:, b])
            vals.append(h * h * weight * np.sum(grad[:, a, :] * grad[:, b, :], axis=1))
    for a in range(4):
        for b in range(4):
            if hidx.shape[0]:
                rows.append(hidx[:, a])
                cols.append(hidx[:, b])
                vals.append(h * h * hw * halpha[:, a] * halpha[:, b])
    Abar = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, n)).tocsc()
    oe = OracleEnv(env.elem, n, elements, grad, weight, mass, hidx, halpha, hw, Abar, float(env.mu))
    if n <= 4000:
        oe._chol = sla.cho_factor(Abar.toarray(), lower=True)
    else:
        oe._lu = spla.splu(Abar)
    return oe


# =============================================================================
# O1 - contact detection (Alg. 1, per-env detection step)
# =============================================================================

def obstacle_displacement(ob, h: float) -> np.ndarray:
    """Obstacle translation over the coming step: h * lin_vel while it still moves."""
    if ob.move_steps == 0:
        return np.zeros(3)
    return h * np.asarray(ob.lin_vel, dtype=np.float64)


def advance_obstacle(ob, h: float):
    """Pose at the start of the next step (kinematic track)."""
    ob = ob.copy()
    ob.center = ob.center + obstacle_displacement(ob, h)
    if ob.move_steps > 0:
        ob.move_steps -= 1
    return ob


def _sdf_eval(kind, c, R, size, x, margin):
    """Predicate, signed distance and normal at points x (k,3); fixed FP64 op order.

    Plane: d = n.(x - c), n = R[:,1].  Box: p = R^T (x - c), q = |p| - e;
    outside: d = |max(q,0)|; inside: d = max q.  Capsule: axis a = R[:,0],
    s = clamp(a.(x - c), -l, l), d = |x - c - s a| - r.  The predicate compares
    squared distances (no square root).
    """
    r0 = x[:, 0] - c[0]
    r1 = x[:, 1] - c[1]
    r2 = x[:, 2] - c[2]
    k = x.shape[0]
    if kind == PLANE:
        n = R[:, 1]
        d = (n[0] * r0 + n[1] * r1) + n[2] * r2
        pred = d < margin
        normal = np.tile(n, (k, 1))
        return pred, d, normal
    if kind == BOX:
        p = np.stack([(R[0, i] * r0 + R[1, i] * r1) + R[2, i] * r2 for i in range(3)], axis=1)
        q = np.abs(p) - size[None, :]
        outside = np.any(q > 0.0, axis=1)
        m = np.maximum(q, 0.0)
        d2 = (m[:, 0] * m[:, 0] + m[:, 1] * m[:, 1]) + m[:, 2] * m[:, 2]
        pred = np.where(outside, d2 < margin * margin, True)
        d = np.where(outside, np.sqrt(d2), np.maximum(np.maximum(q[:, 0], q[:, 1]), q[:, 2]))
        sgn = np.where(p >= 0.0, 1.0, -1.0)
        gl = m * sgn
        gw = np.stack([(R[i, 0] * gl[:, 0] + R[i, 1] * gl[:, 1]) + R[i, 2] * gl[:, 2] for i in range(3)], axis=1)
        gn = np.sqrt((gw[:, 0] * gw[:, 0] + gw[:, 1] * gw[:, 1]) + gw[:, 2] * gw[:, 2])
        with np.errstate(invalid="ignore", divide="ignore"):
            n_out = gw / gn[:, None]
        istar = np.argmax(q, axis=1)
        n_in = R[:, istar].T * sgn[np.arange(k), istar][:, None]
        normal = np.where(outside[:, None], n_out, n_in)
        return pred, d, normal
    if kind == CAPSULE:
        a = R[:, 0]
        rad, half = float(size[0]), float(size[1])
        t = (a[0] * r0 + a[1] * r1) + a[2] * r2
        s = np.clip(t, -half, half)
        w0 = r0 - s * a[0]
        w1 = r1 - s * a[1]
        w2 = r2 - s * a[2]
        d2 = (w0 * w0 + w1 * w1) + w2 * w2
        lim = rad + margin
        pred = d2 < lim * lim
        dn = np.sqrt(d2)
        d = dn - rad
        w = np.stack([w0, w1, w2], axis=1)
        with np.errstate(invalid="ignore", divide="ignore"):
            normal = np.where((dn > 0.0)[:, None], w / dn[:, None], np.tile(a, (k, 1)))
        return pred, d, normal
    raise ValueError(kind)


def tangent_frame(n: np.ndarray):
    """t1 = unit(e_k x n) with k = argmin |n_i| (lowest on ties); t2 = n x t1."""
    k = np.argmin(np.abs(n), axis=1)
    e = np.zeros_like(n)
    e[np.arange(n.shape[0]), k] = 1.0
    t1 = np.cross(e, n)
    t1 = t1 / np.sqrt((t1[:, 0] * t1[:, 0] + t1[:, 1] * t1[:, 1]) + t1[:, 2] * t1[:, 2])[:, None]
    t2 = np.cross(n, t1)
    return t1, t2


@dataclass
class Contacts:
    """Constraint rows of a step, in (vertex, obstacle) order.

    Obstacle contacts: frame columns n, t1, t2, gap d0, obstacle displacement dobs.
    Attachment rows (bilateral, supplementary Eq. 13), obstacle index MAX_OBSTACLES + gripper:
    frame I, d = target - x stored as d0 = -d[0] and dobs = d, so that the contact-frame
    quantities become Phi = Y - d with every row active and sticking (no cone)."""
    vertex: np.ndarray      # (c,) int
    obstacle: np.ndarray    # (c,) int
    frame: np.ndarray       # (c, 3, 3) columns n, t1, t2
    d0: np.ndarray          # (c,)
    dobs: np.ndarray        # (c, 3) obstacle displacement over the step
    attach: np.ndarray = field(default_factory=lambda: np.zeros(0, dtype=bool))

    def __post_init__(self):
        if self.attach.shape[0] != self.vertex.shape[0]:
            self.attach = np.zeros(self.vertex.shape[0], dtype=bool)

    @property
    def count(self) -> int:
        return int(self.vertex.shape[0])


def predicted_state(x, v, h, gravity):
    """q~ = x + h v + h^2 g  (Eq. 1 with f_ext = M g), fixed order (x + h v) + (h h) g."""
    g = np.asarray(gravity, dtype=np.float64)
    return (x + h * v) + (h * h) * g[None, :]


MAX_OBSTACLES = 4


def grasp_update(x, grippers, held):
    """Attachment sets at the start of a step (supplementary, bilateral constraint for cloth
    control): a gripper whose grasp is off holds nothing; a grasping gripper that holds no vertex
    takes every vertex within its radius of its center ((dx^2 + dy^2) + dz^2 <= r^2, FP64), with
    the offset o = x - c, except vertices already held by another gripper (lower index first).
    held: list (per gripper) of dicts vertex -> offset, or None."""
    held = [dict(hg) for hg in held] if held else [dict() for _ in grippers]
    while len(held) < len(grippers):
        held.append({})
    for g, gr in enumerate(grippers):
        if not gr.grasp:
            held[g] = {}
    for g, gr in enumerate(grippers):
        if gr.grasp and not held[g]:
            taken = set().union(*[set(hg) for hg in held]) if held else set()
            c = np.asarray(gr.center, dtype=np.float64)
            r = float(gr.radius)
            d = x - c[None, :]
            d2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
            held[g] = {int(i): d[i].copy() for i in np.nonzero(d2 <= r * r)[0] if int(i) not in taken}
    return held[:len(grippers)]


def gripper_displacement(gr, h: float) -> np.ndarray:
    return np.zeros(3) if gr.move_steps == 0 else h * np.asarray(gr.lin_vel, dtype=np.float64)


def advance_gripper(gr, h: float):
    gr = gr.copy()
    gr.center = gr.center + gripper_displacement(gr, h)
    if gr.move_steps > 0:
        gr.move_steps -= 1
    return gr


def detect(x, v, obstacles, params, grippers=None, held=None) -> Contacts:
    """Vertex-obstacle contacts and attachment rows, listed in (vertex, obstacle) order.

    A pair is a contact iff the predicate holds at x or at the predicted
    position x~, with the obstacle at its end-of-step pose.  Normal, tangents
    and gap d0 are taken at x.  A vertex held by gripper g adds an attachment
    row (obstacle index MAX_OBSTACLES + g) with target c_g(t+h) + o (the
    gripper's end-of-step pose plus the offset taken at capture), and no
    obstacle rows: its position is prescribed by the attachment (a reading;
    an obstacle row beside three equality rows on one vertex is redundant
    when the target is clear of the obstacle and contradicts it otherwise).
    """
    h = params.h
    margin = params.contact_margin
    xt = predicted_state(x, v, h, params.gravity)
    n = x.shape[0]
    hits, d0s, normals = [], [], []
    dobs = []
    for o, ob in enumerate(obstacles):
        dob = obstacle_displacement(ob, h)
        c_next = np.asarray(ob.center, dtype=np.float64) + dob
        R = np.asarray(ob.rot, dtype=np.float64)
        size = np.asarray(ob.size, dtype=np.float64)
        p0, d0, nrm = _sdf_eval(ob.kind, c_next, R, size, x, margin)
        p1, _, _ = _sdf_eval(ob.kind, c_next, R, size, xt, margin)
        hits.append(p0 | p1)
        d0s.append(d0)
        normals.append(nrm)
        dobs.append(dob)
    # a vertex held by a gripper has its position prescribed by the attachment: no obstacle rows
    held_v = set().union(*[set(hg) for hg in held]) if (grippers and held) else set()
    verts, obsi = [], []
    for vtx in range(n):
        if vtx in held_v:
            continue
        for o in range(len(obstacles)):
            if hits[o][vtx]:
                verts.append(vtx)
                obsi.append(o)
    c = len(verts)
    verts = np.asarray(verts, dtype=np.int64)
    obsi = np.asarray(obsi, dtype=np.int64)
    if c == 0:
        con = Contacts(verts, obsi, np.zeros((0, 3, 3)), np.zeros(0), np.zeros((0, 3)))
    else:
        nn = np.stack([normals[o][vv] for vv, o in zip(verts, obsi)])
        t1, t2 = tangent_frame(nn)
        frame = np.stack([nn, t1, t2], axis=2)
        d0 = np.array([d0s[o][vv] for vv, o in zip(verts, obsi)])
        dob = np.stack([dobs[o] for o in obsi])
        con = Contacts(verts, obsi, frame, d0, dob)
    if not grippers or not held or not any(held):
        return con
    # attachment rows, merged into the (vertex, obstacle) order
    rows = []
    for g, gr in enumerate(grippers):
        cn = np.asarray(gr.center, dtype=np.float64) + gripper_displacement(gr, h)
        for vtx, off in held[g].items():
            d = (cn + off) - x[vtx]
            rows.append((vtx, MAX_OBSTACLES + g, d))
    keys = [(int(a), int(b), "c", j) for j, (a, b) in enumerate(zip(con.vertex, con.obstacle))]
    keys += [(vtx, o, "a", k) for k, (vtx, o, _) in enumerate(rows)]
    keys.sort(key=lambda t: (t[0], t[1]))
    V, Ob, Fr, D0, Dob, At = [], [], [], [], [], []
    for vtx, o, kind, k in keys:
        V.append(vtx); Ob.append(o)
        if kind == "c":
            Fr.append(con.frame[k]); D0.append(con.d0[k]); Dob.append(con.dobs[k]); At.append(False)
        else:
            d = rows[k][2]
            Fr.append(np.eye(3)); D0.append(-d[0]); Dob.append(d.copy()); At.append(True)
    return Contacts(np.asarray(V, dtype=np.int64), np.asarray(Ob, dtype=np.int64), np.stack(Fr),
                    np.asarray(D0), np.stack(Dob), np.asarray(At, dtype=bool))


# =============================================================================
# O3 - local projection and assembly (Eq. 3, Eq. 4; Alg. 1, local step)
# =============================================================================

def closest_rotation(F: np.ndarray) -> np.ndarray:
    """argmin over R in SO(3) of |F - R|_F = U diag(1, 1, det(U V^T)) V^T (batched)."""
    U, S, Vt = np.linalg.svd(F)
    d = np.linalg.det(U @ Vt)
    D = np.ones((F.shape[0], 3))
    D[:, 2] = d
    return (U * D[:, None, :]) @ Vt


def closest_orthonormal_columns(F: np.ndarray) -> np.ndarray:
    """argmin over P with P^T P = I of |F - P|_F for 3x2 F: U V^T of the thin SVD."""
    U, S, Vt = np.linalg.svd(F, full_matrices=False)
    return U @ Vt


def deformation_gradients(oe: OracleEnv, q: np.ndarray) -> np.ndarray:
    """F_e = sum_a q_a gradN_a^T (the element map G_e q)."""
    xa = q[oe.elements]                                   # (m, k, 3)
    return np.einsum("mai,maj->mij", xa, oe.grad)


def project(oe: OracleEnv, q: np.ndarray) -> np.ndarray:
    """p_e = Pi_e(G_e q): closest rotation (tets) / orthonormal columns (tris)."""
    F = deformation_gradients(oe, q)
    if oe.elem == TET:
        return closest_rotation(F)
    return closest_orthonormal_columns(F)


def assemble_rhs(oe: OracleEnv, qtilde: np.ndarray, p: np.ndarray, h: float) -> np.ndarray:
    """b = M q~ + h^2 sum_e w_e G_e^T p_e, with (G_e^T p_e)_a = p_e gradN_a; hinges have p = 0."""
    b = oe.mass[:, None] * qtilde
    contrib = h * h * oe.weight[:, None, None] * np.einsum("mij,maj->mai", p, oe.grad)
    np.add.at(b, oe.elements.ravel(), contrib.reshape(-1, 3))
    return b


# =============================================================================
# O3.3 - contact subproblem (Eq. 2b, Eq. 5-9)
# =============================================================================

@dataclass
class CSP:
    """Contact subproblem data in contact space.

    Y(lambda) = y0 + W lambda holds the contact-frame displacement
    F_j^T (q_{v_j} - x_{v_j}) at each contact; W = h^2 H A^-1 H^T (exact Delassus).
    """
    y0: np.ndarray       # (3c,)
    W: np.ndarray        # (3c, 3c)
    d0: np.ndarray       # (c,)
    dob: np.ndarray      # (c, 2): T^T dobs
    s: np.ndarray        # (c,) h^2 / m_v
    mu: float
    max_force: float
    attach: np.ndarray = None   # (c,) bool: bilateral rows (Phi = Y - d, always active and sticking)

    def att(self) -> np.ndarray:
        return self.attach if self.attach is not None else np.zeros(self.d0.shape[0], dtype=bool)


def build_csp(oe: OracleEnv, x, qb, contacts: Contacts, h: float, max_force: float):
    """Exact contact-space operator for fixed A and contact set.

    q(lambda) = qb + h^2 A^-1 H^T lambda; (H^T lambda) puts F_j lambda_j at
    vertex v_j.  Columns of A^-1 = Abar^-1 (x) I3 for the contacted vertices
    come from the exact FP64 factorisation.
    """
    c = contacts.count
    uniq, inv = np.unique(contacts.vertex, return_inverse=True)
    E = np.zeros((oe.n, uniq.shape[0]))
    E[uniq, np.arange(uniq.shape[0])] = 1.0
    Gcols = oe.solve(E)                                   # (n, u): columns of Abar^-1
    Gcc = Gcols[contacts.vertex][:, inv]                  # (c, c)
    Fr = contacts.frame                                   # (c, 3, 3)
    W = h * h * np.einsum("jk,jia,kib->jakb", Gcc, Fr, Fr).reshape(3 * c, 3 * c)
    disp = qb[contacts.vertex] - x[contacts.vertex]
    y0 = np.einsum("jia,ji->ja", Fr, disp).reshape(-1)
    dob = np.einsum("jia,ji->ja", Fr, contacts.dobs)[:, 1:]
    s = h * h / oe.mass[contacts.vertex]
    return CSP(y0, W, contacts.d0.copy(), dob, s, oe.mu, max_force, contacts.attach.copy()), Gcols, inv


def ncp_function(csp: CSP, lam: np.ndarray, s: Optional[np.ndarray] = None):
    """Phi(lambda) (c,3) and the contact-frame quantities.

    Phi_n = min(C_n, s lambda_n), C_n = d0 + Y_n (Signorini, min-map).
    Phi_t = s (lambda_t - Pi_D(mu max(lambda_n,0)) (lambda_t - u_t / s)),
    u_t = Y_t - T^T dobs (Coulomb, Alart-Curnier proximal form).
    `s` overrides the proximal scale (default: the residual scale h^2 / m_v);
    every positive scale has the same zero set.
    """
    c = csp.d0.shape[0]
    Y = (csp.y0 + csp.W @ lam.reshape(-1)).reshape(c, 3)
    Cn = csp.d0 + Y[:, 0]
    ut = Y[:, 1:] - csp.dob
    if s is None:
        s = csp.s
    phi = np.zeros((c, 3))
    phi[:, 0] = np.minimum(Cn, s * lam[:, 0])
    y = lam[:, 1:] - ut / s[:, None]
    rho = csp.mu * np.maximum(lam[:, 0], 0.0)
    ny = np.linalg.norm(y, axis=1)
    proj = y.copy()
    out = ny > rho
    att = csp.att()
    out &= ~att
    with np.errstate(invalid="ignore", divide="ignore"):
        proj[out] = (rho[out] / ny[out])[:, None] * y[out]
    phi[:, 1:] = s[:, None] * (lam[:, 1:] - proj)
    # bilateral rows: Phi = Y - d (the attached vertex at its target)
    phi[att, 0] = Cn[att]
    phi[att, 1:] = ut[att]
    return phi, Cn, ut, y, rho, ny


def residual_of(phi: np.ndarray) -> float:
    """r = max_j max(|Phi_n,j|, |Phi_t,j|_2)  (metres)."""
    if phi.shape[0] == 0:
        return 0.0
    return float(np.max(np.maximum(np.abs(phi[:, 0]), np.linalg.norm(phi[:, 1:], axis=1))))


def generalized_jacobian(csp: CSP, lam: np.ndarray, s: Optional[np.ndarray] = None):
    """An element of the generalized Jacobian dPhi/dlambda (3c x 3c).

    Normal: active (C_n <= s lambda_n) -> row of W; inactive -> s e_n.
    Tangential, rho = mu max(lambda_n, 0): rho = 0 -> s I; stick (|y| <= rho)
    -> rows of W; slip -> kappa P W_t + s (I - kappa P) and -s mu y^ on the
    normal column, kappa = rho/|y|, P = I - y^ y^^T.
    """
    c = csp.d0.shape[0]
    if s is None:
        s = csp.s
    phi, Cn, ut, y, rho, ny = ncp_function(csp, lam, s)
    W = csp.W
    att = csp.att()
    Jm = np.zeros((3 * c, 3 * c))
    for j in range(c):
        rn = 3 * j
        if att[j]:                            # bilateral: rows of W, E = 0
            Jm[rn:rn + 3, :] = W[rn:rn + 3, :]
            continue
        if Cn[j] <= s[j] * lam[j, 0]:
            Jm[rn, :] = W[rn, :]
        else:
            Jm[rn, rn] = s[j]
        rt = slice(3 * j + 1, 3 * j + 3)
        if rho[j] <= 0.0:
            Jm[rt, rt] = s[j] * np.eye(2)
        elif ny[j] <= rho[j]:
            Jm[rt, :] = W[rt, :]
        else:
            yh = y[j] / ny[j]
            kap = rho[j] / ny[j]
            P = np.eye(2) - np.outer(yh, yh)
            Jm[rt, :] = kap * (P @ W[rt, :])
            Jm[rt, rt] += s[j] * (np.eye(2) - kap * P)
            Jm[rt, rn] += -s[j] * csp.mu * yh
    return Jm, phi


def solve_csp(csp: CSP, lam0: Optional[np.ndarray] = None, tol: float = 1e-12,
              max_newton: int = 200, max_pgs: int = 300, attempts: int = 20):
    """Semismooth Newton with backtracking on 1/2|Phi|^2; projected Gauss-Seidel fallback.

    Newton runs on Phi with the per-contact proximal scale s'_j = W_(j,n),(j,n)
    (Delassus diagonal), which has the same zero set as Phi with s = h^2/m_v
    but a far better conditioned switching between stick and slip; the
    stopping test and the returned residual use s = h^2 / m_v.
    Returns (lambda (c,3), residual, info dict).
    """
    c = csp.d0.shape[0]
    info = {"newton": 0, "pgs": 0, "fallback": False}
    if c == 0:
        return np.zeros((0, 3)), 0.0, info
    s_in = np.diag(csp.W)[0::3].copy()
    lam = np.zeros((c, 3)) if lam0 is None else np.array(lam0, dtype=np.float64).reshape(c, 3)
    phi, *_ = ncp_function(csp, lam)
    r = residual_of(phi)
    for attempt in range(attempts):
        for it in range(max_newton):
            if r <= tol:
                return lam, r, info
            Jm, phi = generalized_jacobian(csp, lam, s_in)
            rhs = -phi.reshape(-1)
            try:
                d = np.linalg.solve(Jm, rhs)
                if not np.all(np.isfinite(d)):
                    raise np.linalg.LinAlgError
            except np.linalg.LinAlgError:
                d = np.linalg.lstsq(Jm, rhs, rcond=None)[0]
            psi = 0.5 * float(np.dot(phi.reshape(-1), phi.reshape(-1)))
            alpha = 1.0
            accepted = False
            for _ in range(60):
                trial = np.clip(lam + alpha * d.reshape(c, 3), -csp.max_force, csp.max_force)
                ptrial, *_ = ncp_function(csp, trial, s_in)
                psit = 0.5 * float(np.dot(ptrial.reshape(-1), ptrial.reshape(-1)))
                if psit <= (1.0 - 2e-4 * alpha) * psi:
                    accepted = True
                    break
                alpha *= 0.5
            info["newton"] += 1
            if not accepted:
                break
            lam = trial
            r = residual_of(ncp_function(csp, lam)[0])
        if r <= tol:
            return lam, r, info
        # projected Gauss-Seidel on the exact W (per-contact local solves)
        info["fallback"] = True
        lam = _pgs(csp, lam, tol, max_pgs, info)
        phi, *_ = ncp_function(csp, lam)
        r = residual_of(phi)
        if r <= tol:
            return lam, r, info
    return lam, r, info


def _pgs(csp: CSP, lam, tol, max_sweeps, info):
    c = csp.d0.shape[0]
    W = csp.W
    lam = lam.copy()
    Y = csp.y0 + W @ lam.reshape(-1)
    att = csp.att()
    for sweep in range(max_sweeps):
        for j in range(c):
            i = 3 * j
            Wjj = W[i:i + 3, i:i + 3]
            if att[j]:
                # bilateral row: lambda_j <- lambda_j - W_jj^-1 (Y_j - d_j), unbounded
                r = np.array([csp.d0[j] + Y[i], Y[i + 1] - csp.dob[j, 0], Y[i + 2] - csp.dob[j, 1]])
                dl = -np.linalg.solve(Wjj, r)
                lam[j] += dl
                Y += W[:, i:i + 3] @ dl
                continue
            # normal: lambda_n <- max(0, lambda_n - C_n / W_nn)
            Cn = csp.d0[j] + Y[i]
            ln = max(0.0, lam[j, 0] - Cn / Wjj[0, 0])
            dl = ln - lam[j, 0]
            lam[j, 0] = ln
            Y += W[:, i] * dl
            # tangential: lambda_t <- Pi_D(mu lambda_n)(lambda_t - Wtt^-1 u_t)
            ut = Y[i + 1:i + 3] - csp.dob[j]
            lt = lam[j, 1:] - np.linalg.solve(Wjj[1:, 1:], ut)
            rho = csp.mu * ln
            nl = np.linalg.norm(lt)
            if nl > rho:
                lt = lt * (rho / nl) if nl > 0 else lt * 0.0
            dl = lt - lam[j, 1:]
            lam[j, 1:] = lt
            Y += W[:, i + 1:i + 3] @ dl
        info["pgs"] += 1
        if sweep % 50 == 49:
            phi, *_ = ncp_function(csp, lam)
            if residual_of(phi) <= tol:
                break
    return lam


# =============================================================================
# The step (Alg. 1 body) and its result
# =============================================================================

@dataclass
class StepResult:
    x: np.ndarray
    v: np.ndarray
    contacts: Contacts
    lam: np.ndarray          # (c,3) contact-frame multipliers (N)
    impulse: np.ndarray      # (c,3) world-frame impulses h F lambda (N s)
    residual: float
    obstacles: list
    info: dict = field(default_factory=dict)
    grippers: list = field(default_factory=list)
    held: list = field(default_factory=list)


def contact_residual(oe: OracleEnv, x, q, contacts: Contacts, lam, h: float) -> float:
    """NCP residual evaluated directly from end-of-step positions q and multipliers."""
    c = contacts.count
    if c == 0:
        return 0.0
    Fr = contacts.frame
    disp = q[contacts.vertex] - x[contacts.vertex]
    Y = np.einsum("jia,ji->ja", Fr, disp)
    Cn = contacts.d0 + Y[:, 0]
    dob = np.einsum("jia,ji->ja", Fr, contacts.dobs)[:, 1:]
    ut = Y[:, 1:] - dob
    s = h * h / oe.mass[contacts.vertex]
    phi = np.zeros((c, 3))
    phi[:, 0] = np.minimum(Cn, s * lam[:, 0])
    y = lam[:, 1:] - ut / s[:, None]
    rho = oe.mu * np.maximum(lam[:, 0], 0.0)
    ny = np.linalg.norm(y, axis=1)
    proj = y.copy()
    att = contacts.attach
    out = (ny > rho) & ~att
    proj[out] = (rho[out] / ny[out])[:, None] * y[out]
    phi[:, 1:] = s[:, None] * (lam[:, 1:] - proj)
    phi[att, 0] = Cn[att]
    phi[att, 1:] = ut[att]
    return residual_of(phi)


def step(oe: OracleEnv, x, v, obstacles, params, tol: float = 1e-12, lam_warm=None, grippers=None,
         held=None) -> StepResult:
    """One time step of one environment (Alg. 1 body, every CSP solved to `tol`).  grippers / held:
    kinematic grippers and the attachment sets they held after the previous step (see grasp_update)."""
    h = float(params.h)
    x = np.asarray(x, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    grippers = list(grippers) if grippers else []
    held = grasp_update(x, grippers, held) if grippers else []
    contacts = detect(x, v, obstacles, params, grippers, held)
    qt = predicted_state(x, v, h, params.gravity)
    q = qt.copy()
    c = contacts.count
    lam = np.zeros((c, 3)) if lam_warm is None else np.array(lam_warm, dtype=np.float64)
    info = {"newton": 0, "pgs": 0, "fallback": False, "csp_residuals": []}
    for k in range(int(params.lg_iterations)):
        p = project(oe, q)
        b = assemble_rhs(oe, qt, p, h)
        qb = oe.solve(b)
        if c:
            csp, Gcols, inv = build_csp(oe, x, qb, contacts, h, params.max_force)
            lam, r, inf = solve_csp(csp, lam, tol=tol)
            if k == 0:
                info["lam_first"] = lam.copy()
            info["newton"] += inf["newton"]
            info["pgs"] += inf["pgs"]
            info["fallback"] |= inf["fallback"]
            info["csp_residuals"].append(r)
            f = np.einsum("jia,ja->ji", contacts.frame, lam)    # world force per contact
            fu = np.zeros((Gcols.shape[1], 3))
            np.add.at(fu, inv, f)
            q = qb + h * h * (Gcols @ fu)
        else:
            q = qb
    xn = q
    vn = (q - x) / h
    impulse = h * np.einsum("jia,ja->ji", contacts.frame, lam) if c else np.zeros((0, 3))
    r = contact_residual(oe, x, q, contacts, lam, h)
    new_obs = [advance_obstacle(ob, h) for ob in obstacles]
    new_grip = [advance_gripper(gr, h) for gr in grippers]
    return StepResult(xn, vn, contacts, lam, impulse, r, new_obs, info, new_grip, held)


def rollout(oe: OracleEnv, x, v, obstacles, params, n_steps: int, tol: float = 1e-12, grippers=None):
    """n_steps consecutive steps; returns the list of StepResults."""
    out = []
    held = None
    for _ in range(n_steps):
        res = step(oe, x, v, obstacles, params, tol=tol, grippers=grippers, held=held)
        out.append(res)
        x, v, obstacles, grippers, held = res.x, res.v, res.obstacles, res.grippers, res.held
    return out


# =============================================================================
# Fixed-budget lightweight mode (Alg. 1 with the inertia-only contact metric, Eq. 10)
# =============================================================================
#
# Alg. 1 updates the multipliers once per local-global iteration with the
# lightweight Schur complement Z~ = J M^-1 J^T + E (Eq. 10) in place of the
# exact Z = J A^-1 J^T + E (Eq. 7), and recomputes the positions with the
# exact global solve (Eq. 9); the scene configuration bounds the non-smooth
# Newton iterations ("iterations") and stops them at a tolerance, and the
# parameter table sets 5 local-global and 10 linear-solver iterations.  This
# mode runs, for each of K local-global iterations, up to N such updates:
#   g = b + h^2 H^T lambda,  q_g = A^-1 g                    (global solve)
#   Phi, K, E at (q_g, lambda)                                (Eq. 5)
#   stop if r(Phi) <= tol
#   delta = -(K W~ + E)^-1 Phi,  W~ = h^2 H M^-1 H^T          (Eq. 8 with Eq. 10)
#   lambda <- clip(lambda + delta)
# and then q^k = A^-1 (b + h^2 H^T lambda) (Eq. 9).  N = 1 is Alg. 1 as
# printed.  With the positions q_g consistent with lambda, Alg. 1's increment
# (1/h^2) Z~^-1 (h - J A^-1 g) equals -(K W~ + E)^-1 Phi in these units
# (lambda in newtons, Phi in metres); Phi is evaluated exactly at q_g rather
# than through its linearisation.  No line search: the algorithm has none.
# The proximal scale is the residual scale s = h^2 / m_v, which is the
# diagonal of W~ for a vertex with one contact.  W~ couples only contacts on
# the same vertex.  The result depends on the budget and is not the converged
# step unless the iteration converges within it.

def contact_blocks(Y, lam, d0, dob, s, mu, attach=None):
    """Phi (c,3) and the generalized-Jacobian blocks of each contact at contact-frame displacement
    Y (c,3) and multipliers lam (c,3): K_j = dPhi_j/dY_j, E_j = dPhi_j/dlambda_j (3x3 each), with
    the min-map normal and Alart-Curnier tangential parts at proximal scale s (c,); bilateral rows
    (attach) have Phi = Y - d, K = I, E = 0."""
    c = Y.shape[0]
    phi = np.zeros((c, 3))
    Kb = np.zeros((c, 3, 3))
    Eb = np.zeros((c, 3, 3))
    for j in range(c):
        cn = d0[j] + Y[j, 0]
        ut = Y[j, 1:] - dob[j]
        sj = s[j]
        if attach is not None and attach[j]:
            phi[j, 0] = cn
            phi[j, 1:] = ut
            Kb[j] = np.eye(3)
            continue
        if cn <= sj * lam[j, 0]:              # normal active: Phi_n = C_n
            phi[j, 0] = cn
            Kb[j, 0, 0] = 1.0
        else:                                 # inactive: Phi_n = s lambda_n
            phi[j, 0] = sj * lam[j, 0]
            Eb[j, 0, 0] = sj
        y = lam[j, 1:] - ut / sj
        rho = mu * max(lam[j, 0], 0.0)
        ny = float(np.linalg.norm(y))
        if rho <= 0.0:                        # no friction force available: Phi_t = s lambda_t
            phi[j, 1:] = sj * lam[j, 1:]
            Eb[j, 1:, 1:] = sj * np.eye(2)
        elif ny <= rho:                       # stick: Phi_t = u_t
            phi[j, 1:] = ut
            Kb[j, 1:, 1:] = np.eye(2)
        else:                                 # slip
            yh = y / ny
            kap = rho / ny
            P = np.eye(2) - np.outer(yh, yh)
            phi[j, 1:] = sj * (lam[j, 1:] - rho * yh)
            Kb[j, 1:, 1:] = kap * P
            Eb[j, 1:, 1:] = sj * (np.eye(2) - kap * P)
            Eb[j, 1:, 0] = -sj * mu * yh
    return phi, Kb, Eb


def inertia_metric(oe: OracleEnv, contacts: Contacts, h: float):
    """W~ = h^2 H M^-1 H^T in contact frames (3c x 3c, scipy sparse): (h^2 / m_v) F_j^T F_k for
    contacts j, k on the same vertex v, zero otherwise (Eq. 10's inertia-only metric; M is diagonal,
    so only contacts of one vertex couple)."""
    c = contacts.count
    rows, cols, vals = [], [], []
    by_vertex = {}
    for j in range(c):
        by_vertex.setdefault(int(contacts.vertex[j]), []).append(j)
    ii, jj = np.meshgrid(np.arange(3), np.arange(3), indexing="ij")
    for vtx, idx in by_vertex.items():
        for j in idx:
            for k in idx:
                blk = h * h / oe.mass[vtx] * (contacts.frame[j].T @ contacts.frame[k])
                rows.append(3 * j + ii.ravel())
                cols.append(3 * k + jj.ravel())
                vals.append(blk.ravel())
    if not rows:
        return sp.csr_matrix((3 * c, 3 * c))
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(3 * c, 3 * c))


def _contact_force_field(oe: OracleEnv, contacts: Contacts, lam):
    """H^T lambda as per-vertex world forces (n, 3)."""
    f = np.zeros((oe.n, 3))
    if contacts.count:
        np.add.at(f, contacts.vertex, np.einsum("jia,ja->ji", contacts.frame, lam))
    return f


def step_lightweight(oe: OracleEnv, x, v, obstacles, params, newton_iterations: int, tol: float = 0.0,
                     lam_warm=None, grippers=None, held=None, progress=None) -> StepResult:
    """One time step in the fixed-budget lightweight mode described above (K = params.lg_iterations,
    N = newton_iterations).  info['newton'] counts the multiplier updates, info['lam_history'] holds
    the multipliers after each update.  progress (optional) is called with the index of each finished
    local-global iteration (large scenes take minutes)."""
    h = float(params.h)
    x = np.asarray(x, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    grippers = list(grippers) if grippers else []
    held = grasp_update(x, grippers, held) if grippers else []
    contacts = detect(x, v, obstacles, params, grippers, held)
    qt = predicted_state(x, v, h, params.gravity)
    q = qt.copy()
    c = contacts.count
    lam = np.zeros((c, 3)) if lam_warm is None else np.array(lam_warm, dtype=np.float64).reshape(c, 3)
    s = h * h / oe.mass[contacts.vertex] if c else np.zeros(0)
    Fr = contacts.frame
    dob = np.einsum("jia,ji->ja", Fr, contacts.dobs)[:, 1:] if c else np.zeros((0, 2))
    Wt = inertia_metric(oe, contacts, h)
    # Z~ = K W~ + E couples only the contacts of one vertex (W~ does): the vertex groups and their
    # W~ blocks, fixed over the step
    groups = {}
    for j in range(c):
        groups.setdefault(int(contacts.vertex[j]), []).append(j)
    blocks = []
    for idx in groups.values():
        rows = np.array([3 * j + a for j in idx for a in range(3)])
        blocks.append((np.array(idx), Wt[rows][:, rows].toarray()))
    info = {"newton": 0, "lam_history": [], "csp_residuals": []}
    for k in range(int(params.lg_iterations)):
        p = project(oe, q)
        b = assemble_rhs(oe, qt, p, h)
        if c:
            for it in range(int(newton_iterations)):
                qg = oe.solve(b + h * h * _contact_force_field(oe, contacts, lam))
                Y = np.einsum("jia,ji->ja", Fr, qg[contacts.vertex] - x[contacts.vertex])
                phi, Kb, Eb = contact_blocks(Y, lam, contacts.d0, dob, s, oe.mu, contacts.attach)
                r = residual_of(phi)
                if r <= tol:
                    break
                # Z~ delta = -Phi, one vertex block at a time
                delta = np.zeros((c, 3))
                for idx, Wb in blocks:
                    m = len(idx)
                    Zb = sla.block_diag(*Kb[idx]) @ Wb + sla.block_diag(*Eb[idx])
                    delta[idx] = np.linalg.solve(Zb, -phi[idx].reshape(3 * m)).reshape(m, 3)
                lam = np.clip(lam + delta, -params.max_force, params.max_force)
                info["newton"] += 1
                info["lam_history"].append(lam.copy())
            info["csp_residuals"].append(r)
        q = oe.solve(b + h * h * _contact_force_field(oe, contacts, lam))
        if progress is not None:
            progress(k)
    xn = q
    vn = (q - x) / h
    impulse = h * np.einsum("jia,ja->ji", Fr, lam) if c else np.zeros((0, 3))
    r = contact_residual(oe, x, q, contacts, lam, h)
    new_obs = [advance_obstacle(ob, h) for ob in obstacles]
    new_grip = [advance_gripper(gr, h) for gr in grippers]
    return StepResult(xn, vn, contacts, lam, impulse, r, new_obs, info, new_grip, held)
