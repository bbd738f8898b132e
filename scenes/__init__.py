"""Seeded synthetic workloads for the DiffCloth hot path.

This module only *describes inputs*: node positions, triangles, the spring
list of a regular triangulation, per-spring stiffness draws, masses,
obstacles, attachment targets, time-step settings and loss targets.  It holds
none of the method's arithmetic (no rest lengths, no bending stencils, no
system matrix, no projections, no contact law), so both the FP64 oracle and
the GPU library can consume it without sharing any method code.

Conventions (the paper simulates with y as the height axis, Sec. 7 Dress):
  * y is up, gravity (0, -9.8, 0), ground plane y = 0 with normal +y.
  * Regular grids split cell (i, j) along the (i, j)-(i+1, j+1) diagonal;
    node (i, j) has index i * n + j.
  * Springs are the unique triangle edges, each stored as (a, b) with a < b
    and the list sorted lexicographically.
  * A cloth of side 1 m weighs 0.1 kg, spread evenly over its nodes.
All randomness goes through ``numpy.random.default_rng(seed)``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

PLANE = 0
SPHERE = 1
MESH = 2

GRAVITY = (0.0, -9.8, 0.0)
AREAL_DENSITY = 0.1          # kg per m^2 (0.1 kg over a 1 m x 1 m square cloth)
ATTACH_WEIGHT = 1.0e5        # N/m, attachment (pin / driven ring) constraint weight
BEND_WEIGHT = 1.0e-2         # quadratic bending weight


@dataclasses.dataclass
class Obstacle:
    kind: int                       # PLANE or SPHERE
    point: tuple                    # plane: a point on it; sphere: centre
    normal: tuple = (0.0, 1.0, 0.0) # plane normal (unit); unused for spheres
    radius: float = 0.0             # sphere radius
    mu: float = 0.5                 # Coulomb friction coefficient
    verts: Optional[np.ndarray] = None   # MESH: (nv, 3) vertices
    tris: Optional[np.ndarray] = None    # MESH: (nt, 3) int32, outward normal by (v1-v0) x (v2-v0)


@dataclasses.dataclass
class Scene:
    name: str
    X: np.ndarray                   # (m, 3) float64 rest = initial positions
    tris: np.ndarray                # (nt, 3) int32
    edges: np.ndarray               # (E, 2) int32, a < b, lexicographic
    edge_stiffness: np.ndarray      # (E,) float64, N/m
    node_mass: np.ndarray           # (m,) float64, kg
    v0: np.ndarray                  # (m, 3) float64 initial velocities
    h: float = 1.0 / 120.0
    steps: int = 60
    pd_iters: int = 20
    gravity: tuple = GRAVITY
    bend_weight: float = BEND_WEIGHT
    attach: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(0, np.int32))
    attach_weight: float = ATTACH_WEIGHT
    attach_omega: float = 0.0       # targets rotate about attach_axis through attach_center
    attach_axis: tuple = (0.0, 1.0, 0.0)
    attach_center: tuple = (0.0, 0.0, 0.0)
    obstacles: List[Obstacle] = dataclasses.field(default_factory=list)
    # Optional stiffness regions: spring e uses edge_stiffness[e] * region_scale[edge_region[e]],
    # the bending constraint centred at node j uses bend_weight * region_scale[bend_region[j]].
    edge_region: Optional[np.ndarray] = None
    bend_region: Optional[np.ndarray] = None
    region_scale: Optional[np.ndarray] = None
    # Optional external force besides gravity: node j receives force_scale[n] * force[j]
    # (newtons) during step n (force_scale None: 1 at every step).
    force: Optional[np.ndarray] = None           # (m, 3)
    force_scale: Optional[np.ndarray] = None     # (steps,)
    # Node-node self-collision: thickness d (m; 0 = off), detection radius on the
    # predictor (m; 0 = the thickness) and friction coefficient.
    self_thickness: float = 0.0
    self_radius: float = 0.0
    self_mu: float = 0.0
    # Loss description (inputs only; each side evaluates it itself).
    loss: str = "centroid"          # "centroid" | "apex"
    target: Optional[np.ndarray] = None          # centroid target (3,)
    waist_nodes: Optional[np.ndarray] = None     # apex loss: top ring
    hem_nodes: Optional[np.ndarray] = None       # apex loss: bottom ring
    seed: int = 0

    @property
    def n_nodes(self) -> int:
        return int(self.X.shape[0])

    @property
    def dof(self) -> int:
        return 3 * self.n_nodes


# --------------------------------------------------------------------------- meshes

def _sorted_unique_pairs(pairs: np.ndarray) -> np.ndarray:
    pairs = np.sort(np.asarray(pairs, dtype=np.int64), axis=1)
    pairs = np.unique(pairs, axis=0)           # unique rows, lexicographic
    return pairs.astype(np.int32)


def grid_mesh(n: int, side: float = 1.0, origin=(0.0, 0.0, 0.0)):
    """Regular n x n node grid in the xz-plane at height origin[1]."""
    if n < 2:
        raise ValueError("grid needs at least 2 x 2 nodes")
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    X = np.zeros((n * n, 3))
    X[:, 0] = origin[0] + side * i.ravel() / (n - 1)
    X[:, 1] = origin[1]
    X[:, 2] = origin[2] + side * j.ravel() / (n - 1)
    ci, cj = np.meshgrid(np.arange(n - 1), np.arange(n - 1), indexing="ij")
    a = (ci * n + cj).ravel()
    b = ((ci + 1) * n + cj).ravel()
    c = (ci * n + cj + 1).ravel()
    d = ((ci + 1) * n + cj + 1).ravel()
    tris = np.concatenate([np.stack([a, b, d], 1), np.stack([a, d, c], 1)]).astype(np.int32)
    pairs = np.concatenate([np.stack([a, b], 1), np.stack([a, c], 1), np.stack([a, d], 1),
                            np.stack([b, d], 1), np.stack([c, d], 1)])
    return X, tris, _sorted_unique_pairs(pairs)


def frustum_mesh(n_around: int, n_rings: int, r_top: float, r_bottom: float,
                 slant: float, y_top: float):
    """Open cone frustum (skirt): ring 0 is the waist, ring n_rings-1 the hem.
    Node (ring i, sector k) has index i * n_around + k; the seam is periodic."""
    drop = math.sqrt(slant * slant - (r_bottom - r_top) ** 2)
    X = np.zeros((n_rings * n_around, 3))
    for i in range(n_rings):
        t = i / (n_rings - 1)
        r = r_top + (r_bottom - r_top) * t
        y = y_top - drop * t
        th = 2.0 * np.pi * np.arange(n_around) / n_around
        X[i * n_around:(i + 1) * n_around, 0] = r * np.cos(th)
        X[i * n_around:(i + 1) * n_around, 1] = y
        X[i * n_around:(i + 1) * n_around, 2] = r * np.sin(th)
    ri, k = np.meshgrid(np.arange(n_rings - 1), np.arange(n_around), indexing="ij")
    k1 = (k + 1) % n_around
    a = (ri * n_around + k).ravel()
    b = ((ri + 1) * n_around + k).ravel()
    c = (ri * n_around + k1).ravel()
    d = ((ri + 1) * n_around + k1).ravel()
    tris = np.concatenate([np.stack([a, b, d], 1), np.stack([a, d, c], 1)]).astype(np.int32)
    pairs = np.concatenate([np.stack([a, b], 1), np.stack([a, c], 1), np.stack([a, d], 1),
                            np.stack([b, d], 1), np.stack([c, d], 1)])
    return X, tris, _sorted_unique_pairs(pairs)


def _log_uniform(rng, lo, hi, size=None):
    return np.exp(rng.uniform(math.log(lo), math.log(hi), size))


def _centroid_target(rng, X):
    return X.mean(axis=0) + rng.normal(0.0, 0.1, 3)


def icosphere(center, radius: float, level: int):
    """Triangulated sphere: an icosahedron subdivided ``level`` times (each
    triangle into four), vertices pushed onto the sphere; outward winding.
    20 * 4**level triangles."""
    t = (1.0 + math.sqrt(5.0)) / 2.0
    V = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    F = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4), (11, 10, 2),
         (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5), (2, 4, 11),
         (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    V = [np.asarray(v, float) / np.linalg.norm(v) for v in V]
    for _ in range(level):
        mid = {}

        def midpoint(a, b):
            key = (min(a, b), max(a, b))
            if key not in mid:
                m = V[a] + V[b]
                V.append(m / np.linalg.norm(m))
                mid[key] = len(V) - 1
            return mid[key]
        F2 = []
        for a, b, c in F:
            ab, bc, ca = midpoint(a, b), midpoint(b, c), midpoint(c, a)
            F2 += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        F = F2
    verts = np.asarray(center, float) + radius * np.stack(V)
    tris = np.asarray(F, np.int32)
    # outward winding: (v1 - v0) x (v2 - v0) points away from the centre
    nrm = np.cross(verts[tris[:, 1]] - verts[tris[:, 0]], verts[tris[:, 2]] - verts[tris[:, 0]])
    flip = np.sum(nrm * (verts[tris[:, 0]] - np.asarray(center, float)), axis=1) < 0
    tris[flip] = tris[flip][:, [0, 2, 1]]
    return verts, tris


def mesh_obstacle(verts, tris, mu: float) -> Obstacle:
    return Obstacle(MESH, (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 0.0, mu, np.asarray(verts, float),
                    np.asarray(tris, np.int32))


def discretized_sphere_drop(seed: int = 0, n: int = 40, steps: int = 200, level: int = 2) -> Scene:
    """The sphere drop onto a triangulated sphere (icosphere, 20 * 4**level
    triangles) of the same centre and radius (the discretized-sphere study)."""
    s = c2_sphere_drop(seed, n, steps)
    o = s.obstacles[0]
    V, T = icosphere(o.point, o.radius, level)
    s.obstacles = [mesh_obstacle(V, T, o.mu)]
    s.name = f"mesh_sphere_drop{n}x{n}_L{level}"
    return s


# --------------------------------------------------------------------------- workloads

def c1_napkin(seed: int = 0, n: int = 10, steps: int = 60) -> Scene:
    """Plain method, FP64: 10 x 10 square cloth, 1 m side, 0.2 m above a ground
    plane (mu 0.5), springs 1e3 N/m, bending 1e-2, 0.1 kg, two corners pinned."""
    rng = np.random.default_rng(seed)
    X, tris, edges = grid_mesh(n, 1.0, (0.0, 0.2, 0.0))
    m = X.shape[0]
    return Scene(
        name=f"napkin{n}x{n}_plane", X=X, tris=tris, edges=edges,
        edge_stiffness=np.full(edges.shape[0], 1.0e3),
        node_mass=np.full(m, AREAL_DENSITY / m), v0=np.zeros((m, 3)),
        steps=steps, attach=np.array([0, (n - 1) * n], np.int32),
        obstacles=[Obstacle(PLANE, (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 0.0, 0.5)],
        target=_centroid_target(rng, X), seed=seed)


def c2_sphere_drop(seed: int = 0, n: int = 40, steps: int = 200) -> Scene:
    """40 x 40 square cloth (4800 DoF), side 1 m, dropped from 0.3 m above the
    top of a sphere of radius 0.25 m; per-spring stiffness log-uniform in
    [5e2, 5e3] N/m, mu uniform in [0.2, 0.8]."""
    rng = np.random.default_rng(seed)
    X, tris, edges = grid_mesh(n, 1.0, (-0.5, 0.55, -0.5))
    m = X.shape[0]
    k = _log_uniform(rng, 5.0e2, 5.0e3, edges.shape[0])
    mu = float(rng.uniform(0.2, 0.8))
    return Scene(
        name=f"sphere_drop{n}x{n}", X=X, tris=tris, edges=edges, edge_stiffness=k,
        node_mass=np.full(m, AREAL_DENSITY / m), v0=np.zeros((m, 3)), steps=steps,
        obstacles=[Obstacle(SPHERE, (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 0.25, mu)],
        target=_centroid_target(rng, X), seed=seed)


def wind_napkin(seed: int = 0, n: int = 24, steps: int = 200, h: float = 1.0 / 90.0) -> Scene:
    """Hanging napkin under a synthetic wind (the Wind benchmark's setting:
    h = 1/90 s, 200 steps): n x n square cloth, 1 m side, hanging in the
    xy-plane from its two top corners; every node receives the force
    s_n * d * m_j / mean(m) with d a seeded 3-vector (|d| ~ 0.3 m_j g) and the
    gust profile s_n = 0.5 [sin(omega t_{n+1} + phase) + 1] (the T-shirt wind
    model), omega and phase seeded; no obstacle."""
    rng = np.random.default_rng(seed)
    Xg, tris, edges = grid_mesh(n, 1.0, (0.0, 0.0, 0.0))
    X = np.stack([Xg[:, 0], 1.0 - Xg[:, 2], np.zeros(Xg.shape[0])], axis=1)
    m = X.shape[0]
    mass = np.full(m, AREAL_DENSITY / m)
    d = rng.normal(0.0, 1.0, 3)
    d[2] = abs(d[2]) + 1.0                   # blowing mostly through the cloth
    d *= 0.3 * 9.8 * mass[0] / np.linalg.norm(d)
    omega = float(rng.uniform(2.0, 8.0))
    phase = float(rng.uniform(0.0, 2.0 * math.pi))
    t1 = (np.arange(steps) + 1) * h
    return Scene(
        name=f"wind{n}x{n}", X=X, tris=tris, edges=edges,
        edge_stiffness=_log_uniform(rng, 5.0e2, 5.0e3, edges.shape[0]),
        node_mass=mass, v0=np.zeros((m, 3)), steps=steps, h=h,
        attach=np.array([0, (n - 1) * n], np.int32),
        force=np.tile(d, (m, 1)), force_scale=0.5 * (np.sin(omega * t1 + phase) + 1.0),
        target=_centroid_target(rng, X), seed=seed)


def flying_napkin(seed: int = 0, n: int = 10, steps: int = 60) -> Scene:
    """The napkin above the ground plane with a time-invariant external force on
    every node (3 n^2 force variables; the Flying Napkin control problem):
    forces normal with deviation 0.3 m_j g per component, no pins."""
    s = c1_napkin(seed, n, steps)
    rng = np.random.default_rng(seed + 1000)
    s.name = f"flying_napkin{n}x{n}"
    s.attach = np.zeros(0, np.int32)
    s.force = rng.normal(0.0, 0.3 * 9.8, (s.n_nodes, 3)) * s.node_mass[:, None]
    return s


def c3_skirt(seed: int = 0, n_around: int = 40, n_rings: int = 91, steps: int = 125,
             omega: float = 4.0) -> Scene:
    """Procedural skirt: open frustum, waist radius 0.12 m, hem radius 0.30 m,
    slant length 0.6 m; the waist ring is attached to targets rotating about
    the vertical axis at ``omega`` rad/s.  Four stiffness regions:
    {upper, lower} half x {stretch, bend}.  Loss: final apex angle."""
    X, tris, edges = frustum_mesh(n_around, n_rings, 0.12, 0.30, 0.6, 1.0)
    m = X.shape[0]
    ring = np.arange(m) // n_around
    half = (n_rings - 1) / 2.0
    upper_node = ring < half
    edge_upper = (ring[edges[:, 0]] + ring[edges[:, 1]]) < 2 * half
    area = math.pi * (0.12 + 0.30) * 0.6
    return Scene(
        name=f"skirt{n_around}x{n_rings}", X=X, tris=tris, edges=edges,
        edge_stiffness=np.full(edges.shape[0], 1.0e3),
        node_mass=np.full(m, AREAL_DENSITY * area / m), v0=np.zeros((m, 3)),
        steps=steps, bend_weight=1.0e-1,
        attach=np.arange(n_around, dtype=np.int32), attach_omega=omega,
        attach_axis=(0.0, 1.0, 0.0), attach_center=(0.0, 1.0, 0.0),
        edge_region=np.where(edge_upper, 0, 1).astype(np.int32),
        bend_region=np.where(upper_node, 2, 3).astype(np.int32),
        region_scale=np.ones(4), loss="apex",
        waist_nodes=np.arange(n_around, dtype=np.int32),
        hem_nodes=np.arange((n_rings - 1) * n_around, n_rings * n_around, dtype=np.int32),
        seed=seed)


def mixed_grid(rng, n: int, steps: int, k: float, mu: float, sphere: bool) -> Scene:
    """One rollout of the mixed-size batches: an n x n, 1 m cloth either dropped
    onto the sphere of the sphere-drop workload or hung from two corners above
    the ground plane of the napkin workload."""
    if sphere:
        X, tris, edges = grid_mesh(n, 1.0, (-0.5, 0.55, -0.5))
        obst = [Obstacle(SPHERE, (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 0.25, mu)]
        attach = np.zeros(0, np.int32)
    else:
        X, tris, edges = grid_mesh(n, 1.0, (0.0, 0.2, 0.0))
        obst = [Obstacle(PLANE, (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 0.0, mu)]
        attach = np.array([0, (n - 1) * n], np.int32)
    m = X.shape[0]
    return Scene(
        name=f"{'sphere' if sphere else 'plane'}{n}x{n}", X=X, tris=tris, edges=edges,
        edge_stiffness=np.full(edges.shape[0], k), node_mass=np.full(m, AREAL_DENSITY / m),
        v0=np.zeros((m, 3)), steps=steps, attach=attach, obstacles=obst,
        target=_centroid_target(rng, X))


def c4_batch(seed: int = 0, count: int = 64, steps: int = 150, n_lo: int = 16,
             n_hi: int = 64) -> List[Scene]:
    """64 independent rollouts of uneven size: grids from 16 x 16 to 64 x 64
    nodes, each with its own stiffness (log-uniform [5e2, 5e3]), mu (uniform
    [0.1, 0.9]) and a sphere or plane obstacle."""
    rng = np.random.default_rng(seed)
    out = []
    for r in range(count):
        n = int(rng.integers(n_lo, n_hi + 1))
        k = float(_log_uniform(rng, 5.0e2, 5.0e3))
        mu = float(rng.uniform(0.1, 0.9))
        sphere = bool(rng.integers(0, 2))
        s = mixed_grid(rng, n, steps, k, mu, sphere)
        s.seed = seed * 1000 + r
        out.append(s)
    return out


def c5_requests(seed: int = 0, count: int = 500, n_lo: int = 20, n_hi: int = 100,
                steps_lo: int = 100, steps_hi: int = 300):
    """Serving stream: request sizes round(exp(U[ln 20, ln 100])) nodes per side,
    steps uniform in [100, 300], obstacle sphere or plane; material fixed per
    size (1e3 N/m springs, mu 0.5) so a factor can be cached per topology.
    Returns a list of (n, steps, sphere) tuples; arrival times are drawn by the
    serving driver from its own seeded Poisson process."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        steps = int(rng.integers(steps_lo, steps_hi + 1))
        sphere = bool(rng.integers(0, 2))
        out.append((n, steps, sphere))
    return out


def request_scene(n: int, steps: int, sphere: bool, seed: int = 0) -> Scene:
    rng = np.random.default_rng(seed)
    s = mixed_grid(rng, n, steps, 1.0e3, 0.5, sphere)
    s.seed = seed
    return s


def stacked_sheets(n: int = 6, steps: int = 12, gap: float = 0.012, shift: float = 0.1,
                   k: float = 200.0, self_mu: float = 0.5, seed: int = 0,
                   v0_top=(0.08, -0.5, 0.03), h: float = 1.0 / 120.0, ground: bool = False,
                   pinned: bool = True) -> Scene:
    """Two aligned n x n sheets (spacing 2 cm): the bottom one pinned at its
    four corners 0.3 m above the ground plane, the top one hanging gap metres
    above it, shifted by shift grid spacings along x and z and moving at v0_top
    (plus noise).  Node masses vary by +-30 % so that pairs have unequal
    masses.  Self-collision thickness 0.6 grid spacings, detection radius 1.5
    times that (pairs at rest at the thickness stay detected).  ground: the bottom
    sheet lies 2 mm above the plane instead, unpinned; pinned=False: no pins
    (both sheets fly free)."""
    rng = np.random.default_rng(seed)
    a = 0.02
    side = a * (n - 1)
    y0 = 0.002 if ground else 0.3
    Xb, tris, edges = grid_mesh(n, side, (0.0, y0, 0.0))
    Xt = Xb + np.array([shift * a, gap, shift * a])
    mb = Xb.shape[0]
    X = np.concatenate([Xb, Xt]) + rng.normal(0.0, 2e-4, (2 * mb, 3))
    tris2 = np.concatenate([tris, tris + mb]).astype(np.int32)
    edges2 = np.concatenate([edges, edges + mb]).astype(np.int32)
    m = 2 * mb
    v0 = np.zeros((m, 3))
    v0[mb:] = np.asarray(v0_top, float) + 0.05 * rng.normal(0.0, 1.0, (mb, 3))
    mass = AREAL_DENSITY * side * side / mb * np.exp(rng.uniform(-0.3, 0.3, m)) + 1e-4
    attach = (np.array([0, n - 1, n * (n - 1), n * n - 1], np.int32) if pinned and not ground
              else np.zeros(0, np.int32))
    return Scene(
        name=f"stacked{n}x{n}", X=X, tris=tris2, edges=edges2,
        edge_stiffness=k * np.exp(rng.uniform(-0.3, 0.3, edges2.shape[0])),
        node_mass=mass, v0=v0, steps=steps, h=h, attach=attach,
        obstacles=[Obstacle(PLANE, (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 0.0, 0.4)],
        self_thickness=0.6 * a, self_radius=0.9 * a, self_mu=self_mu, target=_centroid_target(rng, X), seed=seed)


def tiny_scene(n: int = 3, steps: int = 10, obstacle: Optional[str] = "plane",
               k: float = 50.0, mu: float = 0.4, seed: int = 0, height: float = 0.02,
               pins: bool = False, bend: float = BEND_WEIGHT, h: float = 1.0 / 120.0,
               v0_scale: float = 0.0) -> Scene:
    """Small cloths for brute-force checks (finite differences, direct Jacobians)."""
    rng = np.random.default_rng(seed)
    side = 0.1 * (n - 1)
    if obstacle == "sphere":
        X, tris, edges = grid_mesh(n, side, (-side / 2, 0.25 + height, -side / 2))
        obst = [Obstacle(SPHERE, (0.01, 0.0, -0.015), (0.0, 1.0, 0.0), 0.25, mu)]
    else:
        X, tris, edges = grid_mesh(n, side, (0.0, height, 0.0))
        obst = [] if obstacle is None else [
            Obstacle(PLANE, (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 0.0, mu)]
    m = X.shape[0]
    X = X + rng.normal(0.0, 1e-3, X.shape)        # break symmetry
    v0 = v0_scale * rng.normal(0.0, 1.0, (m, 3))
    return Scene(
        name=f"tiny{n}x{n}_{obstacle}", X=X, tris=tris, edges=edges,
        edge_stiffness=k * np.exp(rng.uniform(-0.3, 0.3, edges.shape[0])),
        node_mass=np.full(m, AREAL_DENSITY * side * side / m + 1e-3), v0=v0, steps=steps, h=h,
        bend_weight=bend, attach=np.array([0, (n - 1) * n], np.int32) if pins else np.zeros(0, np.int32),
        obstacles=obst, target=_centroid_target(rng, X), seed=seed)
