"""Seeded synthetic scene generators (inputs only).

This module builds meshes, materials, initial states and kinematic obstacle
tracks.  It performs none of the simulation method's arithmetic (no masses,
no element maps, no system matrices, no contact geometry): both the HIP path
and the FP64 oracle consume what it returns.

Shapes follow the workloads the FLASH paper uses its solver for: volumetric
blocks squeezed by fingers and dropped on the ground, and cloth sheets
(Sec. IV-A, Fig. 3; cloth material of the FLASH parameter table).  The paper's
own meshes (scanned garments, towels) are not available, so seeded lattices
stand in for them.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field
from typing import List

import numpy as np

TET = 0
TRI = 1

PLANE = 0
BOX = 1
CAPSULE = 2

MAX_OBSTACLES = 4


@dataclass
class EnvDesc:
    """One environment: a single deformable body (tet block or cloth sheet)."""
    elem: int
    rest_x: np.ndarray          # (n_vertices, 3) float64, metres
    elements: np.ndarray        # (n_elements, 4) tets or (n_elements, 3) tris, int32
    density: float = 1000.0     # kg/m^3
    thickness: float = 1e-3     # m, TRI only
    young: float = 1e5          # Pa
    poisson: float = 0.3
    bending: float = 0.0        # TRI only (hinge stiffness)
    mu: float = 0.5             # Coulomb coefficient against every obstacle

    @property
    def n_vertices(self) -> int:
        return int(self.rest_x.shape[0])

    @property
    def n_elements(self) -> int:
        return int(self.elements.shape[0])


@dataclass
class Obstacle:
    """Kinematic obstacle.  Pose is the pose at the start of the next step.

    kind: PLANE (normal = rot @ +y, passes through center), BOX (half extents
    in size), CAPSULE (size = (radius, half_length, 0), axis = rot @ +x).
    The obstacle translates by h*lin_vel per step for move_steps steps
    (negative: forever), then holds.
    """
    kind: int
    center: np.ndarray
    rot: np.ndarray             # (3, 3) world-from-local rotation
    size: np.ndarray
    lin_vel: np.ndarray
    move_steps: int = -1

    def copy(self) -> "Obstacle":
        return Obstacle(self.kind, self.center.copy(), self.rot.copy(), self.size.copy(),
                        self.lin_vel.copy(), int(self.move_steps))


@dataclass
class Gripper:
    """Kinematic gripper (end effector) for bilateral attachment.

    center is the pose at the start of the next step; it translates by h*lin_vel per step for
    move_steps steps (negative: forever), then holds.  While `grasp` is on and the gripper holds
    no vertex, the vertices within `radius` of its center are attached to it; turning `grasp`
    off releases them.
    """
    center: np.ndarray
    radius: float
    grasp: bool = True
    lin_vel: np.ndarray = field(default_factory=lambda: np.zeros(3))
    move_steps: int = -1

    def copy(self) -> "Gripper":
        return Gripper(np.array(self.center, float), float(self.radius), bool(self.grasp),
                       np.array(self.lin_vel, float), int(self.move_steps))


MAX_GRIPPERS = 2


@dataclass
class Params:
    h: float = 1.0 / 60.0
    gravity: tuple = (0.0, -9.81, 0.0)
    lg_iterations: int = 20
    max_inner_iterations: int = 50
    ncp_tol: float = 1e-6
    contact_margin: float = 2e-3
    max_force: float = 1e10


@dataclass
class Scene:
    envs: List[EnvDesc]
    x0: List[np.ndarray]                # per env (n_v, 3) float64
    v0: List[np.ndarray]
    obstacles: List[List[Obstacle]]     # per env
    params: Params
    name: str = ""
    meta: dict = field(default_factory=dict)
    grippers: List[List[Gripper]] = field(default_factory=list)   # per env (may be empty)

    @property
    def n_envs(self) -> int:
        return len(self.envs)


# ----------------------------------------------------------------------------
# meshes
# ----------------------------------------------------------------------------

def hex_lattice(nx: int, ny: int, nz: int, size, origin):
    """Box lattice of nx*ny*nz hexes, each split into 6 Kuhn tets.

    Vertices are in lexicographic (i, j, k) order, index
    i*(ny+1)*(nz+1) + j*(nz+1) + k, with i along x, j along y, k along z.
    Each hex is cut into the 6 tets that share its main diagonal.
    """
    sx, sy, sz = (float(s) for s in size)
    ox, oy, oz = (float(o) for o in origin)
    xs = ox + sx * np.arange(nx + 1) / nx
    ys = oy + sy * np.arange(ny + 1) / ny
    zs = oz + sz * np.arange(nz + 1) / nz
    X, Y, Z = np.meshgrid(xs, ys, zs, indexing="ij")
    rest = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1).astype(np.float64)

    def vid(i, j, k):
        return (i * (ny + 1) + j) * (nz + 1) + k

    perms = list(itertools.permutations(range(3)))
    tets = []
    for i in range(nx):
        for j in range(ny):
            for k in range(nz):
                base = np.array([i, j, k])
                for p in perms:
                    c0 = base.copy()
                    c1 = c0.copy(); c1[p[0]] += 1
                    c2 = c1.copy(); c2[p[1]] += 1
                    c3 = base + 1
                    tets.append([vid(*c0), vid(*c1), vid(*c2), vid(*c3)])
    return rest, np.asarray(tets, dtype=np.int32)


def cloth_grid(n: int, side: float, origin, y: float):
    """n*n vertex sheet in the xz-plane at height y, alternating diagonals."""
    ox, oz = float(origin[0]), float(origin[1])
    t = side * np.arange(n) / (n - 1)
    X, Z = np.meshgrid(ox + t, oz + t, indexing="ij")
    rest = np.stack([X.ravel(), np.full(n * n, float(y)), Z.ravel()], axis=1)
    tris = []
    for i in range(n - 1):
        for k in range(n - 1):
            a = i * n + k
            b = (i + 1) * n + k
            c = (i + 1) * n + k + 1
            d = i * n + k + 1
            if (i + k) % 2 == 0:
                tris += [[a, b, c], [a, c, d]]
            else:
                tris += [[a, b, d], [b, c, d]]
    return rest.astype(np.float64), np.asarray(tris, dtype=np.int32)


# ----------------------------------------------------------------------------
# obstacles
# ----------------------------------------------------------------------------

def ground(height: float = 0.0) -> Obstacle:
    return Obstacle(PLANE, np.array([0.0, height, 0.0]), np.eye(3), np.zeros(3), np.zeros(3), -1)


def tilted_plane(angle: float) -> Obstacle:
    """Plane through the origin, rotated by `angle` about +z (normal leans toward -x)."""
    c, s = math.cos(angle), math.sin(angle)
    rot = np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])
    return Obstacle(PLANE, np.zeros(3), rot, np.zeros(3), np.zeros(3), -1)


def box(center, half, vel=(0.0, 0.0, 0.0), move_steps=-1, rot=None) -> Obstacle:
    return Obstacle(BOX, np.asarray(center, float), np.eye(3) if rot is None else np.asarray(rot, float),
                    np.asarray(half, float), np.asarray(vel, float), int(move_steps))


def capsule(center, radius, half_length, vel=(0.0, 0.0, 0.0), move_steps=-1, rot=None) -> Obstacle:
    return Obstacle(CAPSULE, np.asarray(center, float), np.eye(3) if rot is None else np.asarray(rot, float),
                    np.array([radius, half_length, 0.0]), np.asarray(vel, float), int(move_steps))


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniform random rotation from a normalised Gaussian quaternion."""
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


# ----------------------------------------------------------------------------
# scenes
# ----------------------------------------------------------------------------

def drop_cube(seed: int = 0, hexes: int = 4, edge: float = 0.1, drop_height: float = 0.2,
              young: float = 1e5, poisson: float = 0.3, density: float = 1000.0, mu: float = 0.5,
              jitter: float = 1e-3, lg_iterations: int = 20) -> Scene:
    """Single cube of hexes^3 hexes dropped onto the ground (125 vertices / 384 tets at hexes=4).

    The bottom face starts at y = drop_height; initial positions (not the rest
    shape) are jittered by U(-jitter, jitter) per coordinate.
    """
    rng = np.random.default_rng(seed)
    rest, tets = hex_lattice(hexes, hexes, hexes, (edge, edge, edge), (-edge / 2, 0.0, -edge / 2))
    x0 = rest + np.array([0.0, drop_height, 0.0])
    x0 = x0 + rng.uniform(-jitter, jitter, size=x0.shape)
    env = EnvDesc(TET, rest, tets, density=density, young=young, poisson=poisson, mu=mu)
    params = Params(lg_iterations=lg_iterations)
    return Scene([env], [x0], [np.zeros_like(x0)], [[ground()]], params, name="drop_cube")


def squeeze_blocks(n_envs: int, seed: int = 0, hexes: int = 10, edge: float = 0.1,
                   lg_iterations: int = 20, start_gap: float = 1e-3, indent: float = 1e-2,
                   close_speed: float = 0.02, h: float = 1.0 / 60.0) -> Scene:
    """Blocks resting on the ground, squeezed by two kinematic box fingers.

    Per env: E ~ U(5e4, 5e5) Pa, nu ~ U(0.30, 0.45), mu ~ U(0.3, 0.8).  Fingers
    (half extents 0.02 x 0.03 x 0.03 m) sit on the +-x faces at mid height with
    `start_gap`, close at `close_speed` each until `indent`, then hold.
    """
    rng = np.random.default_rng(seed)
    rest, tets = hex_lattice(hexes, hexes, hexes, (edge, edge, edge), (-edge / 2, 0.0, -edge / 2))
    travel = start_gap + indent
    move_steps = int(round(travel / (close_speed * h)))
    half = np.array([0.02, 0.03, 0.03])
    envs, xs, vs, obs = [], [], [], []
    for _ in range(n_envs):
        E = float(rng.uniform(5e4, 5e5))
        nu = float(rng.uniform(0.30, 0.45))
        mu = float(rng.uniform(0.3, 0.8))
        envs.append(EnvDesc(TET, rest, tets, density=1000.0, young=E, poisson=nu, mu=mu))
        xs.append(rest.copy())
        vs.append(np.zeros_like(rest))
        cx = edge / 2 + start_gap + half[0]
        cy = edge / 2
        obs.append([ground(),
                    box((cx, cy, 0.0), half, (-close_speed, 0.0, 0.0), move_steps),
                    box((-cx, cy, 0.0), half, (close_speed, 0.0, 0.0), move_steps)])
    params = Params(h=h, lg_iterations=lg_iterations)
    return Scene(envs, xs, vs, obs, params, name="squeeze_blocks",
                 meta={"hexes": hexes, "move_steps": move_steps})


def incline_block(mu: float, angle_deg: float = 30.0, young: float = 1e8, hexes: int = 2,
                  edge: float = 0.05, lg_iterations: int = 5) -> Scene:
    """Stiff block resting on a plane tilted by angle_deg (friction threshold test)."""
    ang = math.radians(angle_deg)
    rest, tets = hex_lattice(hexes, hexes, hexes, (edge, edge, edge), (-edge / 2, 0.0, -edge / 2))
    c, s = math.cos(ang), math.sin(ang)
    rot = np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])
    x0 = rest @ rot.T
    env = EnvDesc(TET, rest, tets, density=1000.0, young=young, poisson=0.3, mu=mu)
    params = Params(lg_iterations=lg_iterations)
    return Scene([env], [x0], [np.zeros_like(x0)], [[tilted_plane(ang)]], params, name="incline")


def cloth_drop(n: int = 16, side: float = 0.5, height: float = 0.05, seed: int = 0,
               bending: float = 0.2, lg_iterations: int = 10) -> Scene:
    """Cloth sheet (FLASH cloth material: E=3e4, nu=0.4, bending 0.2) over a box."""
    rng = np.random.default_rng(seed)
    rest, tris = cloth_grid(n, side, (-side / 2, -side / 2), 0.0)
    top = 0.05
    x0 = rest + np.array([0.0, top + height, 0.0])
    x0[:, 1] += rng.uniform(-1e-4, 1e-4, size=n * n)
    env = EnvDesc(TRI, rest, tris, density=1000.0, thickness=1e-3, young=3e4, poisson=0.4,
                  bending=bending, mu=0.5)
    obs = [ground(), box((0.0, top / 2, 0.0), (0.08, top / 2, 0.08))]
    params = Params(lg_iterations=lg_iterations)
    return Scene([env], [x0], [np.zeros_like(x0)], [obs], params, name="cloth_drop")


def cloth_fold(n_envs: int = 1, n: int = 64, side: float = 0.6, lg_iterations: int = 5,
               inner_iterations: int = 10, fold_time: float = 5.0, lift: float = 0.03) -> Scene:
    """Cloth-folding stand-in for the paper's garment-folding throughput scene (Sec. V, Table II).

    A square sheet of n x n vertices (side metres, FLASH cloth material: E 3e4, nu 0.4, bending
    0.2, 1 mm thick, 1000 kg/m^3) lies 1 mm above a table (the ground plane, Coulomb mu = 1.0 as in
    the paper's folding scene); h = 0.01 s.  Two grippers grasp the near corners (capture radius
    1.2 vertex spacings: the corner and its two edge neighbours) and carry them at constant
    velocity across to the sheet's midline and `lift` metres up over `fold_time` seconds, then
    hold: a quasi-static fold of the near half over the far half.  Every env is the same copy (the
    paper's throughput comparison steps copies of one scene).  Solver budget: lg_iterations local-
    global iterations, inner_iterations multiplier updates each (the paper's 5 and 10)."""
    rest, tris = cloth_grid(n, side, (-side / 2, -side / 2), 0.0)
    x0 = rest + np.array([0.0, 1e-3, 0.0])
    env = EnvDesc(TRI, rest, tris, density=1000.0, thickness=1e-3, young=3e4, poisson=0.4, bending=0.2, mu=1.0)
    params = Params(h=0.01, lg_iterations=lg_iterations, max_inner_iterations=inner_iterations)
    steps = int(round(fold_time / params.h))
    vel = np.array([0.0, lift / fold_time, 0.5 * side / fold_time])
    r = 1.2 * side / (n - 1)
    near = [int(np.argmin(x0[:, 0] + x0[:, 2])), int(np.argmax(x0[:, 0] - x0[:, 2]))]
    grips = [Gripper(x0[i].copy(), r, True, vel.copy(), steps) for i in near]
    envs = [env] * n_envs
    return Scene(envs, [x0.copy() for _ in range(n_envs)], [np.zeros_like(x0) for _ in range(n_envs)],
                 [[ground()] for _ in range(n_envs)], params, name="cloth_fold",
                 grippers=[[g.copy() for g in grips] for _ in range(n_envs)])


def slab_press(n_envs: int = 64, nx: int = 100, ny: int = 9, nz: int = 100, hex_size: float = 0.005,
               press_speed: float = 0.02, indent: float = 0.005, lg_iterations: int = 10,
               inner_iterations: int = 10) -> Scene:
    """The large-scene recipe (about 100k vertices, 540k tets, at most 20k contacts per env).

    A slab of nx x ny x nz hexes of hex_size (0.5 x 0.045 x 0.5 m at the defaults: 102,010 vertices,
    540,000 tets; E 1e5 Pa, nu 0.3, 1000 kg/m^3, mu 0.5) rests 1 mm above the ground.  Two box finger
    pads, each covering a little under half of the top face (their x half-extent is a quarter of the
    slab minus 1.5 hexes, so that with the ground contacts every env stays at or below 20,000
    contacts), start 1 mm above it and press down at press_speed until they are `indent` into the
    slab, then hold.  h = 1/60 s; budget lg_iterations x inner_iterations; every env the same copy."""
    sx, sy, sz = nx * hex_size, ny * hex_size, nz * hex_size
    rest, tets = hex_lattice(nx, ny, nz, (sx, sy, sz), (-sx / 2, 0.0, -sz / 2))
    x0 = rest + np.array([0.0, 1e-3, 0.0])
    env = EnvDesc(TET, rest, tets, density=1000.0, young=1e5, poisson=0.3, mu=0.5)
    top = sy + 1e-3
    half = (sx / 4 - 1.5 * hex_size, 0.01, sz / 2 - 0.5 * hex_size)
    steps = int(round((1e-3 + indent) / press_speed * 60.0))
    def obstacles():
        return [ground()] + [box((c * sx / 4, top + 1e-3 + half[1], 0.0), half, vel=(0.0, -press_speed, 0.0),
                                 move_steps=steps) for c in (-1.0, 1.0)]
    params = Params(lg_iterations=lg_iterations, max_inner_iterations=inner_iterations)
    return Scene([env] * n_envs, [x0.copy() for _ in range(n_envs)], [np.zeros_like(x0) for _ in range(n_envs)],
                 [obstacles() for _ in range(n_envs)], params, name="slab_press")


def single_tet_scene(kind: str = "ground", seed: int = 0, tang_speed: float = 0.2) -> Scene:
    """Tiny scenes for brute-force enumeration of contact modes (1-3 contacts)."""
    rng = np.random.default_rng(seed)
    rest = np.array([[0.0, 0.0, 0.0], [0.02, 0.0, 0.0], [0.0, 0.0, 0.02], [0.0, 0.02, 0.0]])
    tets = np.array([[0, 1, 2, 3]], dtype=np.int32)
    x0 = rest.copy()
    x0[:, 1] += 0.0005
    v0 = np.zeros_like(x0)
    v0[:, 0] = rng.uniform(-tang_speed, tang_speed)
    v0[:, 2] = rng.uniform(-tang_speed, tang_speed)
    v0[:, 1] = -0.05
    env = EnvDesc(TET, rest, tets, density=1000.0, young=float(rng.uniform(2e4, 2e5)), poisson=0.3,
                  mu=float(rng.uniform(0.1, 0.9)))
    params = Params(lg_iterations=2)
    return Scene([env], [x0], [v0], [[ground()]], params, name="single_tet")


def uneven_batch(n_envs: int, seed: int = 0, max_tet_vertices: int = 8000, max_cloth_side: int = 48,
                 lg_iterations: int = 10) -> Scene:
    """Mixed batch of cloth sheets and tet blocks with log-uniform sizes.

    Per env (seeded): a cloth sheet of n x n vertices, n = round(exp U(ln 16, ln max_cloth_side)),
    or a tet block of about exp U(ln 500, ln max_tet_vertices) vertices, realised as a lattice of
    a x b x c hexes with aspect ratios in [1, 2] and E ~ U(5e4, 5e5); resting 2 mm above the ground
    (blocks) or 5 cm above it (cloth), with 1-3 kinematic boxes or capsules (2-10 cm) at random
    poses above the body moving at |v| <= 5 cm/s for 30 steps, plus the ground.  Per env
    mu ~ U(0.3, 0.8).  Every obstacle starts clear of the body whatever its rotation: its centre
    sits 0.9 of its size (a rotated cube reaches sqrt(3)/2 of its side below its centre, a capsule
    of radius size/4 and half-length size/2 three quarters) plus 5-25 mm above the body's top.
    Contact solves may take up to 100 Newton iterations (a sheet lying flat on the ground couples
    all its n^2 contacts; 50 left one of 122,880 env-steps of a 4096-env batch at its cap).
    """
    rng = np.random.default_rng(seed)
    envs, xs, vs, obs = [], [], [], []
    for _ in range(n_envs):
        if rng.random() < 0.5:
            n = int(round(np.exp(rng.uniform(np.log(16), np.log(max_cloth_side)))))
            side = 0.01 * n
            rest, tris = cloth_grid(n, side, (-side / 2, -side / 2), 0.0)
            x0 = rest + np.array([0.0, 0.05, 0.0])
            env = EnvDesc(TRI, rest, tris, density=1000.0, thickness=1e-3, young=3e4, poisson=0.4,
                          bending=0.2, mu=float(rng.uniform(0.3, 0.8)))
            top = 0.05
        else:
            nv = float(np.exp(rng.uniform(np.log(500), np.log(max_tet_vertices))))
            r = rng.uniform(1.0, 2.0, size=3)
            k = (nv / np.prod(r)) ** (1.0 / 3.0)
            nx, ny, nz = (max(2, int(round(k * ri)) - 1) for ri in r)
            h = 0.01
            rest, tets = hex_lattice(nx, ny, nz, (nx * h, ny * h, nz * h), (-nx * h / 2, 0.0, -nz * h / 2))
            x0 = rest + np.array([0.0, 0.002, 0.0])
            env = EnvDesc(TET, rest, tets, density=1000.0, young=float(rng.uniform(5e4, 5e5)),
                          poisson=float(rng.uniform(0.30, 0.45)), mu=float(rng.uniform(0.3, 0.8)))
            top = ny * h + 0.002
        lst = [ground()]
        for _ in range(int(rng.integers(1, 4))):
            size = rng.uniform(0.02, 0.10)
            c = np.array([rng.uniform(-0.1, 0.1), top + 0.9 * size + rng.uniform(0.005, 0.025),
                          rng.uniform(-0.1, 0.1)])
            d = rng.normal(size=3)
            vel = d / np.linalg.norm(d) * rng.uniform(0.0, 0.05)
            if rng.random() < 0.5:
                lst.append(box(c, (size / 2,) * 3, vel=vel, move_steps=30, rot=random_rotation(rng)))
            else:
                lst.append(capsule(c, size / 4, size / 2, vel=vel, move_steps=30, rot=random_rotation(rng)))
        envs.append(env); xs.append(x0); vs.append(np.zeros_like(x0)); obs.append(lst)
    return Scene(envs, xs, vs, obs, Params(lg_iterations=lg_iterations, max_inner_iterations=100),
                 name="uneven_batch")
