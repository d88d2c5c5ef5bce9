"""Seeded synthetic scene generators.

Both the FP64 oracle and the HIP solver consume the scenes built here.  The
module only builds geometry and parameters (tet meshes from voxels, analytic
obstacles, pin groups, material constants); it holds none of the solver's
arithmetic.  Every generator takes an explicit seed and draws from
``numpy.random.default_rng(seed)``.

Mesh recipes
------------
* voxel grids split into 5 tets per voxel with alternating parity (conforming
  face diagonals) or 6 tets per voxel (Kuhn split along the main diagonal);
* a 2D star profile r(theta) = R (1 + 0.35 cos 5 theta + smooth seeded noise)
  voxelised and extruded (the teaser-scale "gingerbread" stand-in);
* a 40x10x10-node bar (twist/compression sweep);
* seeded voxel blobs (unions of spheres) sized to a target node count;
* a small cube (drop, incline and conveyor tests; moving planes).

Obstacle encoding (``Obstacle.type``):
  0 half-space  geom = [px,py,pz, nx,ny,nz]           solid where n.(x-p) < 0
  1 box         geom = [cx,cy,cz, hx,hy,hz]           axis-aligned solid box
  2 cylinder    geom = [ax,ay,az, bx,by,bz, radius]   capped cylinder, axis a->b
  3 binding     geom = [px,py,pz, cx,cy,cz, e, node]  bilateral row c . x_node = c . p
                                                      with compliance e (0: hard)
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

MODEL_ARAP, MODEL_COROT, MODEL_SNH, MODEL_MR = 0, 1, 2, 3
OBST_HALFSPACE, OBST_BOX, OBST_CYLINDER, OBST_BINDING = 0, 1, 2, 3


@dataclasses.dataclass
class Obstacle:
    type: int
    geom: np.ndarray          # float64[10], unused tail is zero
    mu: float
    vel: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(3))

    @staticmethod
    def make(type_: int, geom, mu: float, vel=(0.0, 0.0, 0.0)) -> "Obstacle":
        g = np.zeros(10)
        g[: len(geom)] = np.asarray(geom, dtype=np.float64)
        return Obstacle(int(type_), g, float(mu), np.asarray(vel, dtype=np.float64))


@dataclasses.dataclass
class Scene:
    """A complete simulation input.  Node and tet arrays are in the caller's order."""
    name: str
    rest: np.ndarray                      # (n,3) float64 rest positions
    tets: np.ndarray                      # (m,4) int32, positively oriented
    model: int                            # default material model
    E: float
    nu: float
    rho: float
    h: float
    gravity: np.ndarray                   # (3,)
    obstacles: List[Obstacle]
    margin: float                         # collision margin (m)
    iters: int                            # local-global iterations per frame
    cr_iters: int
    frames: int
    init_pos: Optional[np.ndarray] = None  # (n,3) or None -> rest
    init_vel: Optional[np.ndarray] = None  # (n,3) or None -> zero
    pin_nodes: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(0, np.int32))
    pin_group: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(0, np.int32))
    pin_lin_vel: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros((0, 3)))
    pin_ang_vel: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros((0, 3)))
    pin_pivot: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros((0, 3)))
    pin_weight_scale: float = 1.0
    tet_model: Optional[np.ndarray] = None  # (m,) int32 per-tet override
    tet_E: Optional[np.ndarray] = None
    tet_nu: Optional[np.ndarray] = None
    self_contact: bool = False              # vertex-triangle contact rows between surface parts
    self_mu: float = 0.0                    # their friction coefficient

    @property
    def n(self) -> int:
        return int(self.rest.shape[0])

    @property
    def m(self) -> int:
        return int(self.tets.shape[0])

    def q0(self) -> np.ndarray:
        return (self.rest if self.init_pos is None else self.init_pos).copy()

    def v0(self) -> np.ndarray:
        return np.zeros_like(self.rest) if self.init_vel is None else self.init_vel.copy()


# ---------------------------------------------------------------------------
# voxel -> tet meshes
# ---------------------------------------------------------------------------
_EVEN = [(0, 0, 0), (1, 1, 0), (1, 0, 1), (0, 1, 1)]
_ODD = [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 1)]


def _nbrs(c, pool):
    return [p for p in pool if sum(abs(a - b) for a, b in zip(c, p)) == 1]


def _five_split(parity: int):
    centre, corners = (_EVEN, _ODD) if parity == 0 else (_ODD, _EVEN)
    tets = [list(centre)]
    for c in corners:
        tets.append([c] + _nbrs(c, centre))
    return tets


def _six_split():
    tets = []
    for perm in [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]:
        p = [0, 0, 0]
        path = [tuple(p)]
        for ax in perm:
            p[ax] = 1
            path.append(tuple(p))
        tets.append(path)
    return tets


def voxel_mesh(occ: np.ndarray, voxel: float, split: int = 5, origin=(0.0, 0.0, 0.0)):
    """Tet mesh of the occupied voxels ``occ[i,j,k]``; only used nodes are kept."""
    occ = np.asarray(occ, dtype=bool)
    nx, ny, nz = occ.shape
    vid = -np.ones((nx + 1, ny + 1, nz + 1), dtype=np.int64)
    ii, jj, kk = np.nonzero(occ)
    for dx in (0, 1):
        for dy in (0, 1):
            for dz in (0, 1):
                vid[ii + dx, jj + dy, kk + dz] = 1
    used = np.argwhere(vid > 0)                      # lexicographic (i,j,k)
    vid[used[:, 0], used[:, 1], used[:, 2]] = np.arange(len(used))
    rest = used.astype(np.float64) * voxel + np.asarray(origin, dtype=np.float64)
    patterns = {0: _five_split(0), 1: _five_split(1)} if split == 5 else {0: _six_split(), 1: _six_split()}
    tets = []
    for i, j, k in zip(ii, jj, kk):
        for t in patterns[(i + j + k) % 2]:
            tets.append([vid[i + c[0], j + c[1], k + c[2]] for c in t])
    tets = np.asarray(tets, dtype=np.int64)
    # orient positively
    e1 = rest[tets[:, 1]] - rest[tets[:, 0]]
    e2 = rest[tets[:, 2]] - rest[tets[:, 0]]
    e3 = rest[tets[:, 3]] - rest[tets[:, 0]]
    vol = np.einsum("ij,ij->i", np.cross(e1, e2), e3)
    flip = vol < 0
    tets[flip, 1], tets[flip, 2] = tets[flip, 2].copy(), tets[flip, 1].copy()
    return rest, tets.astype(np.int32)


def _mean_edge(rest, tets):
    e = []
    for a in range(4):
        for b in range(a + 1, 4):
            e.append(np.linalg.norm(rest[tets[:, a]] - rest[tets[:, b]], axis=1))
    return float(np.mean(np.concatenate(e)))


# ---------------------------------------------------------------------------
# scenes
# ---------------------------------------------------------------------------
def cube_drop(seed: int = 0, model: int = MODEL_COROT, nodes: int = 5, edge: float = 0.1,
              height: float = 0.05, mu: float = 0.5, E: float = 1e5, nu: float = 0.3,
              frames: int = 60, iters: int = 5, cr_iters: int = 10) -> Scene:
    """5x5x5-node cube (0.1 m edge, 320 tets) dropped from 0.05 m onto z=0."""
    rng = np.random.default_rng(seed)
    nv = nodes - 1
    voxel = edge / nv
    rest, tets = voxel_mesh(np.ones((nv, nv, nv), bool), voxel, split=5)
    init = rest + np.array([0.0, 0.0, height])
    init = init + rng.uniform(-0.01 * edge, 0.01 * edge, size=init.shape)
    ground = Obstacle.make(OBST_HALFSPACE, [0, 0, 0, 0, 0, 1], mu)
    return Scene("cube_drop", rest, tets, model, E, nu, 1000.0, 1.0 / 60.0,
                 np.array([0.0, 0.0, -9.81]), [ground], 0.25 * voxel, iters, cr_iters, frames,
                 init_pos=init)


def fork_clap(seed: int = 0, mu: float = 0.0, speed: float = 0.6, voxel: float = 0.025, depth: int = 2,
              height: int = 4, gap: int = 1, model: int = MODEL_COROT, E: float = 1e5, nu: float = 0.3,
              frames: int = 20, iters: int = 5, cr_iters: int = 10) -> Scene:
    """Self-contact: a U-shaped body (two prongs of 2 x depth voxels and `height` voxels on a
    one-voxel base, `gap` voxels apart) whose prongs swing toward each other, with speeds
    growing linearly with height (+x for the left prong, -x for the right), no gravity and
    no obstacle: the prongs' inner faces meet through vertex-triangle self-contact rows.
    The initial velocity field is mirror-symmetric, so the total momentum is zero; a
    seeded perturbation of 0.5% of a voxel breaks exact symmetry of the positions."""
    rng = np.random.default_rng(seed)
    nx = 4 + gap
    occ = np.zeros((nx, depth, height + 1), bool)
    occ[:, :, 0] = True
    occ[:2, :, 1:] = True
    occ[2 + gap:, :, 1:] = True
    rest, tets = voxel_mesh(occ, voxel, split=5)
    init = rest + rng.uniform(-0.005 * voxel, 0.005 * voxel, size=rest.shape)
    vel = np.zeros_like(rest)
    xm = 0.5 * nx * voxel
    lift = np.clip(rest[:, 2] / (height * voxel + voxel), 0.0, 1.0)
    vel[:, 0] = np.where(rest[:, 0] < xm, speed, -speed) * lift
    vel[np.isclose(rest[:, 0], xm), 0] = 0.0
    return Scene("fork_clap", rest, tets, model, E, nu, 1000.0, 0.01, np.zeros(3), [], 0.25 * voxel, iters,
                 cr_iters, frames, init_pos=init, init_vel=vel, self_contact=True, self_mu=mu)


def cube_on_obstacle(kind: str, seed: int = 0, mu: float = 0.5, frames: int = 40) -> Scene:
    """The 5x5x5-node drop cube (0.1 m, x, y in [0, 0.1]) falling onto a slab or a capped
    cylinder instead of the ground plane (App. A's analytic partners), placed so that
    every branch of their distance functions holds contacts:
    * "slab": a box whose top face is z = 0 and whose +x side face is at x = 0.07, so the
      cube lands across the slab's edge (inside points, the edge and the side face);
    * "cylinder_side": a horizontal capped cylinder along y, radius 0.03, top line z = 0
      at x = 0.05, its cap at y = 0.097, just inside the cube's last node row (curved
      side, cap and rim);
    * "cylinder_cap": a vertical capped cylinder of radius 0.046 under the cube's centre,
      its upper cap at z = 0 (the cap face, and its rim edge just inside the cube's edge
      midpoints; the cube's corners overhang)."""
    sc = cube_drop(seed, mu=mu, frames=frames)
    if kind == "slab":
        ob = Obstacle.make(OBST_BOX, [0.0, 0.05, -0.02, 0.07, 0.2, 0.02], mu)
    elif kind == "cylinder_side":
        ob = Obstacle.make(OBST_CYLINDER, [0.05, -0.2, -0.03, 0.05, 0.097, -0.03, 0.03], mu)
    elif kind == "cylinder_cap":
        ob = Obstacle.make(OBST_CYLINDER, [0.05, 0.05, -0.3, 0.05, 0.05, 0.0, 0.046], mu)
    else:
        raise ValueError(kind)
    sc.name = f"cube_on_{kind}"
    sc.obstacles = [ob]
    return sc


def incline_block(mu: float, theta_deg: float = 10.0, nodes: int = 4, edge: float = 0.1,
                  E: float = 1e8, nu: float = 0.3, model: int = MODEL_COROT, h: float = 0.01,
                  frames: int = 60, iters: int = 10, cr_iters: int = 24,
                  slide_speed: float = 0.0) -> Scene:
    """Stiff block resting on a plane inclined by ``theta_deg``.

    The slope is represented by tilting gravity: the plane stays z=0 and gravity is
    rotated by theta about the y axis, so the downhill direction is +x.  The block
    sticks iff mu > tan(theta).  It starts in exact contact, at rest (or sliding
    downhill at ``slide_speed``).
    """
    nv = nodes - 1
    voxel = edge / nv
    rest, tets = voxel_mesh(np.ones((nv, nv, nv), bool), voxel, split=5)
    th = math.radians(theta_deg)
    g = 9.81 * np.array([math.sin(th), 0.0, -math.cos(th)])
    ground = Obstacle.make(OBST_HALFSPACE, [0, 0, 0, 0, 0, 1], mu)
    vel = np.zeros_like(rest)
    vel[:, 0] = slide_speed
    return Scene("incline", rest, tets, model, E, nu, 1000.0, h, g, [ground], 0.25 * voxel,
                 iters, cr_iters, frames, init_pos=rest.copy(), init_vel=vel)


def conveyor_block(mu: float = 0.8, belt=(0.2, 0.0, 0.0), nodes: int = 3, edge: float = 0.1, E: float = 1e5,
                   nu: float = 0.3, model: int = MODEL_COROT, h: float = 0.01, frames: int = 40,
                   iters: int = 10, cr_iters: int = 24) -> Scene:
    """Block at rest on the plane z=0 whose surface moves with velocity ``belt`` (a
    conveyor: the obstacle velocity enters the friction rows).  Static friction carries
    the block up to belt speed when mu g is large enough."""
    nv = nodes - 1
    voxel = edge / nv
    rest, tets = voxel_mesh(np.ones((nv, nv, nv), bool), voxel, split=5)
    ground = Obstacle.make(OBST_HALFSPACE, [0, 0, 0, 0, 0, 1], mu, vel=belt)
    return Scene("conveyor", rest, tets, model, E, nu, 1000.0, h, np.array([0.0, 0.0, -9.81]), [ground],
                 0.25 * voxel, iters, cr_iters, frames, init_pos=rest.copy())


def moving_plane(z: float, mu: float = 0.5, vel=(0.0, 0.0, 0.0)) -> Obstacle:
    """The half-space below z (normal +z), moving with ``vel`` (geometry updated by the
    caller every frame)."""
    return Obstacle.make(OBST_HALFSPACE, [0, 0, z, 0, 0, 1], mu, vel=vel)


def hanging_block(e_z: float = 0.0, nodes: int = 3, edge: float = 0.1, E: float = 1e5, nu: float = 0.3,
                  model: int = MODEL_COROT, h: float = 0.01, frames: int = 40, iters: int = 10,
                  cr_iters: int = 24, swing: float = 0.0) -> Scene:
    """Block hanging from its top corner by bilateral (binding) rows: along x and y hard,
    along z with compliance e_z (0: a hard point anchor, > 0: a vertical spring of
    stiffness 1/e_z).  swing: initial sideways speed of every node (m/s)."""
    nv = nodes - 1
    voxel = edge / nv
    rest, tets = voxel_mesh(np.ones((nv, nv, nv), bool), voxel, split=5)
    top = int(np.argmax(rest @ np.array([1.0, 1.0, 1.0])))
    p = rest[top]
    binds = [Obstacle.make(OBST_BINDING, [p[0], p[1], p[2], 1, 0, 0, 0.0, top], 0.0),
             Obstacle.make(OBST_BINDING, [p[0], p[1], p[2], 0, 1, 0, 0.0, top], 0.0),
             Obstacle.make(OBST_BINDING, [p[0], p[1], p[2], 0, 0, 1, e_z, top], 0.0)]
    vel = np.zeros_like(rest)
    vel[:, 1] = swing
    return Scene("hanging", rest, tets, model, E, nu, 1000.0, h, np.array([0.0, 0.0, -9.81]), binds,
                 0.25 * voxel, iters, cr_iters, frames, init_pos=rest.copy(), init_vel=vel)


def free_block(seed: int = 0, model: int = MODEL_SNH, nodes: int = 4, edge: float = 0.1,
               E: float = 1e5, nu: float = 0.3, gravity=(0.0, 0.0, -9.81), h: float = 0.01,
               spin: float = 0.0) -> Scene:
    """Contact-free block with seeded perturbed initial state (momentum tests)."""
    rng = np.random.default_rng(seed)
    nv = nodes - 1
    voxel = edge / nv
    rest, tets = voxel_mesh(np.ones((nv, nv, nv), bool), voxel, split=5)
    init = rest + rng.uniform(-0.05 * voxel, 0.05 * voxel, size=rest.shape)
    vel = rng.normal(0.0, 0.1, size=rest.shape)
    if spin:
        c = rest.mean(0)
        vel += spin * np.cross(np.array([0.0, 0.0, 1.0]), rest - c)
    return Scene("free_block", rest, tets, model, E, nu, 1000.0, h, np.asarray(gravity, float), [],
                 0.25 * voxel, 5, 10, 10, init_pos=init, init_vel=vel)


def twist_bar(seed: int = 0, model: int = MODEL_SNH, E: float = 1e6, nu: float = 0.4,
              mu: float = 0.2, nodes=(40, 10, 10), voxel: float = 0.01, frames: int = 400,
              iters: int = 10, cr_iters: int = 10, h: float = 0.01, turns: float = 1.0,
              press: float = 0.2, ground: bool = True) -> Scene:
    """40x10x10-node bar; end caps rotate +-turns*360 deg over ``frames`` while pressed
    ``press`` x height into the plane z=0 (5 tets per voxel); ground=False drops the plane
    (the twisting test of the global-step comparison has no contact)."""
    rng = np.random.default_rng(seed)
    nvx, nvy, nvz = nodes[0] - 1, nodes[1] - 1, nodes[2] - 1
    rest, tets = voxel_mesh(np.ones((nvx, nvy, nvz), bool), voxel, split=5)
    height = nvz * voxel
    rest = rest + np.array([0.0, -0.5 * nvy * voxel, 0.0])
    init = rest + np.array([0.0, 0.0, 0.25 * voxel]) + rng.uniform(-1e-5, 1e-5, rest.shape)
    xmin, xmax = rest[:, 0].min(), rest[:, 0].max()
    left = np.nonzero(np.isclose(rest[:, 0], xmin))[0]
    right = np.nonzero(np.isclose(rest[:, 0], xmax))[0]
    pins = np.concatenate([left, right]).astype(np.int32)
    group = np.concatenate([np.zeros(len(left)), np.ones(len(right))]).astype(np.int32)
    T = frames * h
    w = 2.0 * math.pi * turns / T
    vz = -press * height / T
    cz = 0.25 * voxel + 0.5 * height
    lin = np.array([[0.0, 0.0, vz], [0.0, 0.0, vz]])
    ang = np.array([[-w, 0.0, 0.0], [w, 0.0, 0.0]])
    piv = np.array([[xmin, 0.0, cz], [xmax, 0.0, cz]])
    ground_plane = Obstacle.make(OBST_HALFSPACE, [0, 0, 0, 0, 0, 1], mu)
    return Scene("twist_bar", rest, tets, model, E, nu, 1000.0, h, np.array([0.0, 0.0, -9.81]),
                 [ground_plane] if ground else [], 0.25 * voxel, iters, cr_iters, frames, init_pos=init,
                 pin_nodes=pins, pin_group=group, pin_lin_vel=lin, pin_ang_vel=ang, pin_pivot=piv)


def _star_occupancy(R: float, layers: int, coeffs, phases):
    half = int(math.ceil(R * 1.6)) + 2
    xs = np.arange(-half, half) + 0.5
    X, Y = np.meshgrid(xs, xs, indexing="ij")
    th = np.arctan2(Y, X)
    r = R * (1.0 + 0.35 * np.cos(5.0 * th))
    for k, (a, p) in enumerate(zip(coeffs, phases)):
        r = r + R * a * np.cos((k + 2) * th + p)
    inside = np.hypot(X, Y) < r
    return np.repeat(inside[:, :, None], layers, axis=2)


def star_profile_mesh(seed: int, target=(19300, 19700), layers: int = 15, voxel: float = 0.01,
                      split: int = 5):
    """Extruded seeded star voxelised to a node count inside ``target``."""
    rng = np.random.default_rng(seed)
    coeffs = rng.uniform(-0.03, 0.03, size=7)
    phases = rng.uniform(0, 2 * math.pi, size=7)
    lo, hi = 5.0, 60.0
    best = None
    for _ in range(60):
        R = 0.5 * (lo + hi)
        occ = _star_occupancy(R, layers, coeffs, phases)
        # node count of the voxel set without building the mesh
        nx, ny, nz = occ.shape
        v = np.zeros((nx + 1, ny + 1, nz + 1), bool)
        for dx in (0, 1):
            for dy in (0, 1):
                for dz in (0, 1):
                    v[dx:nx + dx, dy:ny + dy, dz:nz + dz] |= occ
        n = int(v.sum())
        best = (R, occ)
        if n < target[0]:
            lo = R
        elif n > target[1]:
            hi = R
        else:
            break
    R, occ = best
    nx, ny, _ = occ.shape
    rest, tets = voxel_mesh(occ, voxel, split=split,
                            origin=(-0.5 * nx * voxel, -0.5 * ny * voxel, 0.0))
    return rest, tets


def teaser_scene(seed: int = 0, contacts: int = 800, model: int = MODEL_SNH, E: float = 1e6,
                 nu: float = 0.45, mu: float = 0.3, iters: int = 5, cr_iters: int = 10,
                 frames: int = 300, h: float = 0.01, split: int = 5,
                 target=(19300, 19700), drop_speed: float = 0.1) -> Scene:
    """Teaser-scale scene (~19.5k nodes, 58.5k DoFs).

    A seeded extruded star moving down at ``drop_speed`` reaches a slightly tilted
    seeded ground plane; the tip of the +x arm is a pinned handle pulled at 0.5 m/s
    towards a gap between two seeded static capped cylinders.  The plane offset is
    placed so that the collision predicate (min of the signed distance at q_t and at
    the predicted state, compared with the margin) selects exactly ``contacts`` nodes
    at frame 0.
    """
    rng = np.random.default_rng(1000 + seed)
    voxel = 0.01
    rest, tets = star_profile_mesh(seed, target=target, voxel=voxel, split=split)
    margin = 0.25 * voxel
    g = np.array([0.0, 0.0, -9.81])
    # predicted state x + h v + h^2 g; the plane offset lies between the c-th and
    # (c+1)-th lowest predicted node, and the tilt (seeded direction) is sized so that
    # the selected nodes span margin + h |v|: the lowest node then just touches the
    # plane at q_t and the predicted state penetrates by up to h |v|
    vel = np.zeros_like(rest)
    vel[:, 2] = -drop_speed
    pred = rest + h * vel + h * h * g
    ang = rng.uniform(0.0, 2.0 * math.pi)
    want = margin + h * drop_speed

    def plane(mag):
        nv = np.array([mag * math.cos(ang), mag * math.sin(ang), 1.0])
        nv /= np.linalg.norm(nv)
        sv = np.sort(pred @ nv)
        return nv, sv

    lo, hi = 0.0, 0.5
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        _, sv = plane(mid)
        if sv[contacts - 1] - sv[0] < want:
            lo = mid
        else:
            hi = mid
    nrm, s = plane(hi)
    off = 0.5 * (s[contacts - 1] + s[contacts]) - margin
    ground = Obstacle.make(OBST_HALFSPACE, list(nrm * off) + list(nrm), mu)
    # handle: tip of the +x arm
    xmax = rest[:, 0].max()
    handle = np.nonzero(rest[:, 0] > xmax - 0.03)[0].astype(np.int32)
    # two cylinders forming a gap ahead of the handle (vertical axes)
    ywidth = rest[:, 1].max() - rest[:, 1].min()
    gap = ywidth * rng.uniform(0.35, 0.5)
    rad = 0.03
    cx = xmax + rng.uniform(0.05, 0.10)
    zlo, zhi = -0.1, rest[:, 2].max() + 0.1
    cyl1 = Obstacle.make(OBST_CYLINDER, [cx, 0.5 * gap + rad, zlo, cx, 0.5 * gap + rad, zhi, rad], mu)
    cyl2 = Obstacle.make(OBST_CYLINDER, [cx, -0.5 * gap - rad, zlo, cx, -0.5 * gap - rad, zhi, rad], mu)
    return Scene("teaser", rest, tets, model, E, nu, 1000.0, h, g, [ground, cyl1, cyl2], margin,
                 iters, cr_iters, frames, init_pos=rest.copy(), init_vel=vel,
                 pin_nodes=handle, pin_group=np.zeros(len(handle), np.int32),
                 pin_lin_vel=np.array([[0.5, 0.0, 0.0]]), pin_ang_vel=np.zeros((1, 3)),
                 pin_pivot=np.zeros((1, 3)))


def blob_scene(seed: int, target_nodes: int, model: int, E: float, mu: float, contacts: int,
               nu: float = 0.4, iters: int = 5, cr_iters: int = 10, h: float = 0.01) -> Scene:
    """Seeded voxel blob (union of 3-6 spheres) with about ``target_nodes`` nodes resting on
    a tilted plane that gives exactly ``contacts`` contacts at frame 0."""
    rng = np.random.default_rng(seed)
    ns = int(rng.integers(3, 7))
    cen = rng.uniform(-0.6, 0.6, size=(ns, 3))
    rad = rng.uniform(0.6, 1.0, size=ns)

    def occ_at(res):
        xs = (np.arange(-2 * res, 2 * res) + 0.5) / res
        X, Y, Z = np.meshgrid(xs, xs, xs, indexing="ij")
        o = np.zeros(X.shape, bool)
        for c, r in zip(cen, rad):
            o |= (X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2 < r * r
        return o

    def count(o):
        nx, ny, nz = o.shape
        v = np.zeros((nx + 1, ny + 1, nz + 1), bool)
        for dx in (0, 1):
            for dy in (0, 1):
                for dz in (0, 1):
                    v[dx:nx + dx, dy:ny + dy, dz:nz + dz] |= o
        return int(v.sum())

    lo, hi = 1.0, 40.0
    occ = None
    for _ in range(40):
        res = 0.5 * (lo + hi)
        o = occ_at(res)
        c = count(o)
        occ = o
        if c < 0.95 * target_nodes:
            lo = res
        elif c > 1.05 * target_nodes:
            hi = res
        else:
            break
    voxel = 0.01
    rest, tets = voxel_mesh(occ, voxel, split=5)
    rest = rest - rest.mean(0)
    rest[:, 2] -= rest[:, 2].min()
    margin = 0.25 * voxel
    g = np.array([0.0, 0.0, -9.81])
    obst = []
    contacts = min(contacts, len(rest) - 1)
    if contacts > 0:
        tilt = rng.uniform(-0.05, 0.05, size=2)
        nrm = np.array([tilt[0], tilt[1], 1.0])
        nrm /= np.linalg.norm(nrm)
        pred = rest + h * h * g
        s = np.sort(pred @ nrm)
        off = 0.5 * (s[contacts - 1] + s[contacts]) - margin
        obst.append(Obstacle.make(OBST_HALFSPACE, list(nrm * off) + list(nrm), mu))
    return Scene(f"blob{seed}", rest, tets, model, E, nu, 1000.0, h, g, obst, margin, iters,
                 cr_iters, 60, init_pos=rest.copy())


def batch_scenes(seed: int = 0, count: int = 64, lo: int = 200, hi: int = 20000):
    """``count`` blobs with node counts log-uniform in [lo, hi], mixed corotated / stable
    Neo-Hookean, E log-uniform in [1e4, 1e7], 0-800 plane contacts, mu ~ U(0.1, 0.9)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        nodes = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        model = MODEL_COROT if rng.uniform() < 0.5 else MODEL_SNH
        E = float(math.exp(rng.uniform(math.log(1e4), math.log(1e7))))
        mu = float(rng.uniform(0.1, 0.9))
        c = int(rng.integers(0, 801))
        out.append(blob_scene(10_000 * (seed + 1) + i, nodes, model, E, mu, min(c, nodes // 4)))
    return out


def mean_edge_length(scene: Scene) -> float:
    return _mean_edge(scene.rest, scene.tets)
