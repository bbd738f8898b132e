"""FP64 CPU oracle of the DiffCloth hot path (Projective Dynamics with dry
frictional contact, forward and adjoint).

TEST INFRASTRUCTURE ONLY.  This module is the plain, slow, obviously correct
reference that the GPU library is checked against.  Only the test suite, the
smoke check and the CPU-baseline leg of the benchmark may import it; the
product path never calls it.  It shares no code with the GPU library: it
reads the seeded inputs of ``scenes`` and implements every step itself with
NumPy / SciPy in float64.

Layout: positions, velocities and gradients are (m, 3) arrays (node-major);
3m-vectors, where needed for sparse algebra, interleave xyz per node.

Readings of the paper taken here (the paper is silent or ambiguous on them):
  * Contact iteration (Sec. 3.2, the per-node decoupled iteration of Ly et al.):
    one global solve with the prefactored P per PD iteration, with the current
    contact impulses on the right-hand side, followed by one per-node contact
    update that uses the decoupled node response h/m_j (the same fixed point).
  * Contact detection on the inertial predictor y, contact frame and gap taken
    at x_n; Signorini applies to the gap-corrected normal velocity u_N + phi/h.
  * Tie-breaks: take off iff a > 0, stick iff |u_T| <= mu(-a); obstacle is
    argmin phi with ties to the lowest index; phi(y) = 0 counts as contact.
  * Contact adjoint: differentiate the converged state through the per-node
    closed-form contact map (blocks T_j); this is the block-diagonal, per-node
    contact Jacobian of Sec. 4.2 and reduces to the DiffPD adjoint without contact.
  * Springs: p = L0 q/|q| with the given stiffness as weight; quadratic bending:
    one constraint per interior vertex with a cotangent-Laplacian stencil l,
    p = rho0 l(x)/|l(x)|, rho0 = |l(X)|, p = 0 when rho0 = 0; attachments
    p = target(t).
  * Degenerate |q| < 1e-12 rho: use the rest direction and a zero projection Jacobian.
  * Initial guess per step: v^0 = v_n + h g, contact impulses 0, or (warm
    start) the previous step's impulses on the nodes of the contact set.
  * Backward projections re-evaluated at x_{n+1} = x_n + h v_{n+1}.
  * Node-node self-collision (Sec. 4.2, Extensions): pairs found on the
    predictor y among nodes outside the obstacle contact set (each node in at
    most one contact); the pair's normal is the direction of x_i - x_j at x_n,
    its gap |x_i - x_j| - d, the law acts on the relative velocity with the
    pair's reduced mass, and the pair's impulse is +f on i and -f on j.  The
    adjoint takes T with two-node blocks in the mass-weighted form M T M^{-1}.
Every function cites the passage it follows.  Parity is pinned by the
``-m "not gpu"`` tests in ``tests/test_oracle_pins.py``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

FREE, TAKEOFF, STICK, SLIP = 0, 1, 2, 3
PLANE, SPHERE, MESH = 0, 1, 2
FACE, VERTEX, EDGE = 0, 1, 2
DEGENERATE_REL = 1e-12


# =========================================================================== constraints

def triangle_edges(tris: np.ndarray) -> np.ndarray:
    """Unique undirected triangle edges (a < b), sorted lexicographically."""
    t = np.asarray(tris, dtype=np.int64)
    e = np.concatenate([t[:, [0, 1]], t[:, [1, 2]], t[:, [2, 0]]])
    e = np.sort(e, axis=1)
    return np.unique(e, axis=0).astype(np.int64)


def cotangent_bending_stencils(X: np.ndarray, tris: np.ndarray):
    """Quadratic bending constraints (Bouaziz et al. material, Sec. 3.1): one
    per interior vertex b, with A_b x = sum_k c_bk (x_k - x_b) and c_bk the
    cotangent weight (cot alpha + cot beta) / 2 of edge (b, k).
    Returns (centers, stencil matrix L (nb x m))."""
    m = X.shape[0]
    t = np.asarray(tris, dtype=np.int64)
    W = {}
    count = {}
    for tri in t:
        for r in range(3):
            i, j, k = tri[r], tri[(r + 1) % 3], tri[(r + 2) % 3]
            # angle at k, opposite edge (i, j)
            u = X[i] - X[k]
            v = X[j] - X[k]
            cot = float(np.dot(u, v) / np.linalg.norm(np.cross(u, v)))
            key = (min(i, j), max(i, j))
            W[key] = W.get(key, 0.0) + 0.5 * cot
            count[key] = count.get(key, 0) + 1
    boundary = np.zeros(m, bool)
    for (a, b), c in count.items():
        if c == 1:
            boundary[a] = True
            boundary[b] = True
    centers = [b for b in range(m) if not boundary[b]]
    nbrs = {b: {} for b in centers}
    for (a, b), w in W.items():
        if a in nbrs:
            nbrs[a][b] = w
        if b in nbrs:
            nbrs[b][a] = w
    rows, cols, vals = [], [], []
    for r, b in enumerate(centers):
        tot = 0.0
        for k, w in nbrs[b].items():
            rows.append(r); cols.append(k); vals.append(w)
            tot += w
        rows.append(r); cols.append(b); vals.append(-tot)
    L = sp.csr_matrix((vals, (rows, cols)), shape=(len(centers), m))
    return np.array(centers, dtype=np.int64), L


def rotation(axis, angle: float) -> np.ndarray:
    a = np.asarray(axis, float)
    a = a / np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + math.sin(angle) * K + (1 - math.cos(angle)) * (K @ K)


@dataclasses.dataclass
class Contact:
    """Per-step contact record (Sec. 3.2: contact set, local frames, modes)."""
    nodes: np.ndarray       # (C,) node ids in the contact set
    obstacle: np.ndarray    # (C,) obstacle index
    normal: np.ndarray      # (C, 3) contact normal at x_n
    gap: np.ndarray         # (C,) signed distance at x_n
    mu: np.ndarray          # (C,)
    ubar: np.ndarray        # (C, 3) free velocity of the last contact update
    impulse: np.ndarray     # (C, 3) h J^T r, world frame
    mode: np.ndarray        # (C,) TAKEOFF / STICK / SLIP


@dataclasses.dataclass
class SelfContact:
    """Per-step node-node contact record (Sec. 4.2, Extensions: a row of J
    with two node blocks, the normal along the pair's relative position)."""
    i: np.ndarray           # (S,) lower node id of each pair
    j: np.ndarray           # (S,) higher node id
    normal: np.ndarray      # (S, 3) (x_i - x_j) / |x_i - x_j| at x_n
    gap: np.ndarray         # (S,) |x_i - x_j| - d at x_n
    dist: np.ndarray        # (S,) |x_i - x_j| at x_n
    mred: np.ndarray        # (S,) reduced mass m_i m_j / (m_i + m_j)
    ubar: np.ndarray        # (S, 3) free relative velocity of the last contact update
    impulse: np.ndarray     # (S, 3) impulse on node i (node j receives its negative)
    mode: np.ndarray        # (S,) TAKEOFF / STICK / SLIP


def no_self_contact() -> SelfContact:
    z = np.zeros(0, np.int64)
    return SelfContact(z, z, np.zeros((0, 3)), np.zeros(0), np.zeros(0), np.zeros(0),
                       np.zeros((0, 3)), np.zeros((0, 3)), np.zeros(0, np.int8))


@dataclasses.dataclass
class StepRecord:
    x0: np.ndarray          # x_n
    v0: np.ndarray          # v_n
    x1: np.ndarray          # x_{n+1}
    v1: np.ndarray          # v_{n+1}
    contact: Contact
    iters: int
    pairs: Optional[SelfContact] = None     # node-node contacts (None: none)


class Model:
    """Constraint set, masses and the prefactored global matrix (Sec. 3.1,
    eqn pd_global): P = M + h^2 sum_i w_i A_i^T A_i, with A_i = a_i^T (x) I_3 for
    springs and bending, and the node selector for attachments, so that
    P = P_s (x) I_3 with the scalar m x m matrix P_s."""

    def __init__(self, scene, edge_stiffness=None, bend_weight=None, region_scale=None,
                 mu=None, h=None, force=None, force_scale=None, self_mu=None):
        self.scene = scene
        self.X = np.asarray(scene.X, float)
        self.m = self.X.shape[0]
        self.h = float(scene.h if h is None else h)
        self.g = np.asarray(scene.gravity, float)
        self.mass = np.asarray(scene.node_mass, float)
        F = scene.force if force is None else force
        self.force = np.zeros((self.m, 3)) if F is None else np.asarray(F, float).reshape(self.m, 3)
        fs = scene.force_scale if force_scale is None else force_scale
        self.force_scale = None if fs is None else np.asarray(fs, float)
        edges = np.asarray(scene.edges if scene.edges is not None else triangle_edges(scene.tris),
                           np.int64)
        self.edges = edges
        E = edges.shape[0]
        k = np.asarray(scene.edge_stiffness if edge_stiffness is None else edge_stiffness, float)
        wb = float(scene.bend_weight if bend_weight is None else bend_weight)
        rs = scene.region_scale if region_scale is None else region_scale
        self.region_scale = None if rs is None else np.asarray(rs, float)
        # springs: a_e = e_a - e_b
        S = sp.csr_matrix((np.concatenate([np.ones(E), -np.ones(E)]),
                           (np.concatenate([np.arange(E), np.arange(E)]),
                            np.concatenate([edges[:, 0], edges[:, 1]]))), shape=(E, self.m))
        centers, Lb = cotangent_bending_stencils(self.X, scene.tris)
        self.bend_centers = centers
        nb = centers.shape[0]
        self.A = sp.vstack([S, Lb]).tocsr()                      # (nc, m)
        self.n_spring, self.n_bend = E, nb
        self.nc = E + nb
        base_w = np.concatenate([k, np.full(nb, wb)])
        self.base_w = base_w
        if self.region_scale is not None:
            reg = np.concatenate([np.asarray(scene.edge_region, np.int64),
                                  np.asarray(scene.bend_region, np.int64)[centers]])
            self.region = reg
            self.w = base_w * self.region_scale[reg]
        else:
            self.region = None
            self.w = base_w.copy()
        q_rest = self.A @ self.X
        self.rho = np.linalg.norm(q_rest, axis=1)
        # flat bending: a rest Laplacian below 1e-10 of sum_k |c_bk||X_k - X_b| has no target
        Lc = Lb.tocoo()
        terms = np.abs(Lc.data) * np.linalg.norm(self.X[Lc.col] - self.X[centers[Lc.row]], axis=1)
        mag = np.zeros(nb)
        np.add.at(mag, Lc.row, terms)
        flat = self.rho[E:] <= 1e-10 * mag
        self.rho[E:][flat] = 0.0
        rd = np.zeros_like(q_rest)
        ok = self.rho > 0
        rd[ok] = q_rest[ok] / self.rho[ok, None]
        self.rest_dir = rd
        self.attach = np.asarray(scene.attach, np.int64)
        self.w_att = float(scene.attach_weight)
        self.obstacles = list(scene.obstacles)
        if mu is not None:
            self.obstacles = [dataclasses.replace(o, mu=float(mu_o))
                              for o, mu_o in zip(self.obstacles, np.atleast_1d(mu))]
        h2 = self.h * self.h
        Patt = sp.csr_matrix((np.full(len(self.attach), self.w_att),
                              (self.attach, self.attach)), shape=(self.m, self.m))
        self.K_s = (self.A.T @ sp.diags(self.w) @ self.A + Patt).tocsr()   # sum w A^T A (scalar)
        self.P_s = (sp.diags(self.mass) + h2 * self.K_s).tocsc()
        self.lu = spla.splu(self.P_s)                            # "prefactorized" P
        # node-node self-collision: thickness d (0: off) and friction coefficient;
        # nodes that share a constraint stencil never form a pair
        self.self_d = float(getattr(scene, "self_thickness", 0.0) or 0.0)
        self.self_r = float(getattr(scene, "self_radius", 0.0) or 0.0) or self.self_d
        self.self_mu = float(getattr(scene, "self_mu", 0.0) if self_mu is None else self_mu)
        self._shared = None

    def shares_stencil(self) -> np.ndarray:
        """(m, m) bool: nodes i, j appear together in a spring or bending stencil."""
        if self._shared is None:
            Aa = abs(self.A)
            self._shared = (Aa.T @ Aa).toarray() != 0
        return self._shared

    # ----------------------------------------------------------------- helpers
    def force_at(self, n: int) -> np.ndarray:
        """External force besides gravity during step n: s_n F (part of f_ext in
        eqn implicit_v; a time-invariant field F scaled per step)."""
        s = 1.0 if self.force_scale is None else float(self.force_scale[n])
        return s * self.force

    def external_accel(self, n: int) -> np.ndarray:
        """M^{-1} f_ext during step n: gravity plus the external force."""
        return self.g + self.force_at(n) / self.mass[:, None]

    def attach_targets(self, t: float) -> np.ndarray:
        sc = self.scene
        R = rotation(sc.attach_axis, sc.attach_omega * t)
        c = np.asarray(sc.attach_center, float)
        return (self.X[self.attach] - c) @ R.T + c

    def solve_P(self, rhs: np.ndarray) -> np.ndarray:
        """Global step: back-substitution with the prefactored P (eqn pd_global)."""
        return self.lu.solve(rhs)

    # ----------------------------------------------------------------- obstacles
    def signed_distance(self, o, x: np.ndarray) -> np.ndarray:
        if o.kind == PLANE:
            return (x - np.asarray(o.point)) @ np.asarray(o.normal, float)
        if o.kind == MESH:
            return mesh_query(o, x)[0]
        d = x - np.asarray(o.point, float)
        return np.linalg.norm(d, axis=1) - o.radius

    def normal_at(self, o, x: np.ndarray) -> np.ndarray:
        if o.kind == PLANE:
            return np.tile(np.asarray(o.normal, float), (x.shape[0], 1))
        if o.kind == MESH:
            return mesh_query(o, x)[1]
        d = x - np.asarray(o.point, float)
        return d / np.linalg.norm(d, axis=1)[:, None]


# =========================================================================== triangle-mesh obstacles

def closest_point_on_triangle(p, a, b, c):
    """Closest point of triangle abc to each point p (Voronoi-region tests of
    Ericson, Real-Time Collision Detection, Sec. 5.1.5), vectorised over rows:
    p, a, b, c are (N, 3).  Returns the point (N, 3), the region (FACE, VERTEX
    or EDGE) and, for EDGE, the unit edge direction (N, 3; zeros otherwise).
    The region tests run in the order vertex a, vertex b, edge ab, vertex c,
    edge ac, edge bc, face; the first that holds decides."""
    dot = lambda u, v: np.sum(u * v, axis=1)
    ab, ac, ap = b - a, c - a, p - a
    d1, d2 = dot(ab, ap), dot(ac, ap)
    bp = p - b
    d3, d4 = dot(ab, bp), dot(ac, bp)
    cp = p - c
    d5, d6 = dot(ab, cp), dot(ac, cp)
    vc = d1 * d4 - d3 * d2
    vb = d5 * d2 - d1 * d6
    va = d3 * d6 - d5 * d4
    N = p.shape[0]
    q = np.zeros((N, 3))
    region = np.full(N, -1, np.int8)
    e = np.zeros((N, 3))
    undecided = np.ones(N, bool)

    def take(mask, point, reg, edge=None):
        sel = undecided & mask
        q[sel] = point[sel]
        region[sel] = reg
        if edge is not None:
            e[sel] = edge[sel] / np.linalg.norm(edge[sel], axis=1)[:, None]
        undecided[sel] = False

    with np.errstate(divide="ignore", invalid="ignore"):
        take((d1 <= 0) & (d2 <= 0), a, VERTEX)
        take((d3 >= 0) & (d4 <= d3), b, VERTEX)
        take((vc <= 0) & (d1 >= 0) & (d3 <= 0), a + (d1 / (d1 - d3))[:, None] * ab, EDGE, ab)
        take((d6 >= 0) & (d5 <= d6), c, VERTEX)
        take((vb <= 0) & (d2 >= 0) & (d6 <= 0), a + (d2 / (d2 - d6))[:, None] * ac, EDGE, ac)
        take((va <= 0) & (d4 - d3 >= 0) & (d5 - d6 >= 0),
             b + ((d4 - d3) / ((d4 - d3) + (d5 - d6)))[:, None] * (c - b), EDGE, c - b)
        den = va + vb + vc
        take(np.ones(N, bool), a + (vb / den)[:, None] * ab + (vc / den)[:, None] * ac, FACE)
    return q, region, e


def mesh_query(o, x: np.ndarray):
    """Signed distance and contact normal of points x (N, 3) to a triangle-mesh
    obstacle (Sec. 5.1, the discretized sphere; reading): the closest triangle
    (ties to the lowest index); on its face phi = n_t.(x - a) and n = n_t, the
    unit face normal of (v1 - v0) x (v2 - v0); on an edge or vertex with closest
    point c, r = |x - c|, s = sign(n_t.(x - c)) (+1 at 0), phi = s r and
    n = s (x - c) / r (n = n_t when r = 0).  Returns phi (N,), n (N, 3), the
    region (N,) and the unit edge direction (N, 3) of EDGE regions."""
    V = np.asarray(o.verts, float)
    Tr = np.asarray(o.tris, np.int64)
    x = np.atleast_2d(np.asarray(x, float))
    N, T = x.shape[0], Tr.shape[0]
    A, B, C = V[Tr[:, 0]], V[Tr[:, 1]], V[Tr[:, 2]]
    nt = np.cross(B - A, C - A)
    nt /= np.linalg.norm(nt, axis=1)[:, None]
    P = np.repeat(x, T, axis=0)
    q, reg, e = closest_point_on_triangle(P, np.tile(A, (N, 1)), np.tile(B, (N, 1)), np.tile(C, (N, 1)))
    ntr = np.tile(nt, (N, 1))
    face_d = np.sum(ntr * (P - np.tile(A, (N, 1))), axis=1)
    dist = np.where(reg == FACE, np.abs(face_d), np.linalg.norm(P - q, axis=1)).reshape(N, T)
    best = np.argmin(dist, axis=1)                 # ties -> lowest triangle index
    k = np.arange(N) * T + best
    phi = np.zeros(N)
    n = np.zeros((N, 3))
    region = reg[k]
    edge = e[k]
    for i in range(N):
        j = k[i]
        if region[i] == FACE:
            phi[i] = face_d[j]
            n[i] = ntr[j]
        else:
            d = P[j] - q[j]
            r = math.sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2])
            sgn = 1.0 if ntr[j, 0] * d[0] + ntr[j, 1] * d[1] + ntr[j, 2] * d[2] >= 0.0 else -1.0
            if r > 0.0:
                phi[i] = sgn * r
                n[i] = sgn * d / r
            else:
                n[i] = ntr[j]
    return phi, n, region, edge


# =========================================================================== forward

def inertial_predictor(model: Model, x: np.ndarray, v: np.ndarray, n: int = 0) -> np.ndarray:
    """y = x_n + h v_n + h^2 M^{-1} f_ext with f_ext = M g + s_n F (eqn implicit_energy)."""
    return x + model.h * v + model.h ** 2 * model.external_accel(n)


def detect_contacts(model: Model, x: np.ndarray, y: np.ndarray):
    """Contact set on the predictor y; explicit frame and gap at x_n (Sec. 3.2:
    J_n depends on the state entering the step; Sec. 4.2 Extensions: the normal
    of a curved obstacle is taken where the contact occurs)."""
    if not model.obstacles:
        z = np.zeros(0, np.int64)
        return z, z, np.zeros((0, 3)), np.zeros(0), np.zeros(0)
    phis = np.stack([model.signed_distance(o, y) for o in model.obstacles], axis=1)
    ostar = np.argmin(phis, axis=1)                 # ties -> lowest index
    phimin = phis[np.arange(model.m), ostar]
    nodes = np.nonzero(phimin <= 0.0)[0]
    obst = ostar[nodes]
    normal = np.zeros((nodes.size, 3))
    gap = np.zeros(nodes.size)
    mu = np.zeros(nodes.size)
    for oi, o in enumerate(model.obstacles):
        sel = obst == oi
        if np.any(sel):
            xs = x[nodes[sel]]
            normal[sel] = model.normal_at(o, xs)
            gap[sel] = model.signed_distance(o, xs)
            mu[sel] = o.mu
    return nodes, obst, normal, gap, mu


def detect_self_pairs(model: Model, x: np.ndarray, y: np.ndarray, busy: np.ndarray,
                      f_prev: Optional[np.ndarray] = None) -> SelfContact:
    """Node-node contact set on the predictor y (Sec. 4.2, Extensions; reading).
    Node i's candidates are the nodes j != i that share no constraint stencil
    with i, are both outside the obstacle contact set (busy), have x_i != x_j
    and |y_i - y_j| <= r, the detection radius (r >= d; squared distances
    compared, summed over x, y, z in that order); its partner is its nearest candidate, ties to the lowest
    index; i and j form a pair when each is the other's partner.  The pair's
    frame is taken at x_n (as for obstacles): normal (x_i - x_j)/|x_i - x_j|
    for i < j, gap |x_i - x_j| - d.  Its impulse starts from zero, or (warm
    start) from node i's impulse at the end of the previous step."""
    d = model.self_d
    if d <= 0.0:
        return no_self_contact()
    m = model.m

    def sq(P):
        D = P[:, None, :] - P[None, :, :]
        return D[..., 0] * D[..., 0] + D[..., 1] * D[..., 1] + D[..., 2] * D[..., 2]

    rr = model.self_r
    d2 = sq(y)
    ok = (d2 <= rr * rr) & (sq(x) > 0.0) & ~model.shares_stencil()
    ok &= ~busy[:, None] & ~busy[None, :]
    np.fill_diagonal(ok, False)
    d2 = np.where(ok, d2, np.inf)
    nn = np.argmin(d2, axis=1)                                 # ties -> lowest index
    nn[~np.isfinite(d2[np.arange(m), nn])] = -1
    i = np.nonzero((nn > np.arange(m)) & (nn[np.maximum(nn, 0)] == np.arange(m)))[0]
    j = nn[i]
    S = i.size
    sc = no_self_contact()
    if S == 0:
        return sc
    e = x[i] - x[j]
    r = np.sqrt(e[:, 0] * e[:, 0] + e[:, 1] * e[:, 1] + e[:, 2] * e[:, 2])
    mi, mj = model.mass[i], model.mass[j]
    f0 = np.zeros((S, 3)) if f_prev is None else np.asarray(f_prev, float)[i].copy()
    return SelfContact(i, j, e / r[:, None], r - d, r, mi * mj / (mi + mj), np.zeros((S, 3)), f0,
                       np.full(S, TAKEOFF, np.int8))


def local_projection(model: Model, x: np.ndarray):
    """Local step (eqn pd_project): p_i = argmin over M_i of |A_i x - p|.
    Springs/bending: the sphere of radius rho_i; returns (p, q = A x)."""
    q = model.A @ x
    nq = np.linalg.norm(q, axis=1)
    p = np.zeros_like(q)
    act = model.rho > 0
    deg = act & (nq < DEGENERATE_REL * np.maximum(model.rho, 1e-300))
    ok = act & ~deg
    p[ok] = model.rho[ok, None] * q[ok] / nq[ok, None]
    p[deg] = model.rho[deg, None] * model.rest_dir[deg]
    return p, q


def constant_rhs(model: Model, x: np.ndarray, v: np.ndarray, t1: float, n: int = 0) -> np.ndarray:
    """b_hat minus the parts that change inside the step (eqn pd_velocity):
    (b(p) - P x_n)/h = M v_n + h f_ext - (P - M) x_n / h + h sum_att w t_j(t_{n+1})
    + h sum_i w_i A_i^T p_i with f_ext = M g + s_n F, of which the last sum is
    added per iteration."""
    h = model.h
    r = model.mass[:, None] * v + h * (model.mass[:, None] * model.g + model.force_at(n))
    r -= h * (model.K_s @ x)
    if model.attach.size:
        np.add.at(r, model.attach, h * model.w_att * model.attach_targets(t1))
    return r


def signorini_coulomb(ubar, n, phi, mu, h, mass):
    """Per-node Signorini-Coulomb update (eqn contact_all) for nodes whose
    velocity responds to their impulse f as v = ubar + f/m (decoupled nodes, the
    mass-splitting of eqn ly_et_al_govrningEq).  With an isotropic node
    response the law has a closed form; the normal uses the gap-corrected
    velocity u_N + phi/h.  Vectorised over nodes: ubar, n (C, 3); phi, mu,
    mass (C,).  Returns v, f (C, 3) and the mode (TAKEOFF/STICK/SLIP)."""
    ubar = np.atleast_2d(np.asarray(ubar, float))
    n = np.atleast_2d(np.asarray(n, float))
    phi = np.atleast_1d(np.asarray(phi, float))
    mu = np.atleast_1d(np.asarray(mu, float))
    mass = np.atleast_1d(np.asarray(mass, float))
    un = np.sum(n * ubar, axis=1)
    a = un + phi / h
    ut = ubar - un[:, None] * n
    tau = np.linalg.norm(ut, axis=1)
    takeoff = a > 0.0
    stick = ~takeoff & (tau <= mu * (-a))
    slip = ~takeoff & ~stick
    v = ubar.copy()
    vn = -(phi / h)[:, None] * n
    v[stick] = vn[stick]
    that = np.zeros_like(ut)
    that[slip] = ut[slip] / tau[slip, None]
    v[slip] = vn[slip] + ut[slip] + (mu * a)[slip, None] * that[slip]
    f = mass[:, None] * (v - ubar)
    f[takeoff] = 0.0
    mode = np.where(takeoff, TAKEOFF, np.where(stick, STICK, SLIP)).astype(np.int8)
    return v, f, mode


def forward_step(model: Model, x: np.ndarray, v: np.ndarray, n: int, iters: Optional[int] = None,
                 tol: Optional[float] = None, max_iters: int = 100000, energy_log=None,
                 f_prev: Optional[np.ndarray] = None):
    """One implicit-Euler step with dry frictional contact (eqn
    implicit_with_contact) solved by PD local/global iterations (Sec. 3.1) with
    contact impulses on the right-hand side (eqn pd_velocity_with_contact) and a
    per-node Signorini-Coulomb update after each global step.

    f_prev (m, 3): warm start of the contact iteration (Sec. 4.2, Convergence,
    as a remedy for slow forward convergence): every node of this step's
    contact set starts from its impulse at the end of the previous step
    (zero for nodes that were not in contact), instead of from zero.  The
    iteration's fixed point does not depend on its start."""
    h = model.h
    t1 = (n + 1) * h
    y = inertial_predictor(model, x, v, n)
    nodes, obst, normal, gap, mu = detect_contacts(model, x, y)
    C = nodes.size
    busy = np.zeros(model.m, bool)
    busy[nodes] = True
    ps = detect_self_pairs(model, x, y, busy, f_prev)          # node-node contacts
    S = ps.i.size
    pf = ps.impulse
    bhat0 = constant_rhs(model, x, v, t1, n)
    vk = v + h * model.external_accel(n)                      # v^0: x^0 = y
    f = np.zeros((C, 3)) if f_prev is None else np.asarray(f_prev, float)[nodes].copy()
    ubar = np.zeros((C, 3))
    mode = np.full(C, TAKEOFF, np.int8)
    K = model.scene.pd_iters if iters is None else iters
    k = 0
    while True:
        xk = x + h * vk
        p, _ = local_projection(model, xk)                    # local step
        rhs = bhat0 + h * (model.A.T @ (model.w[:, None] * p))
        if C:
            np.add.at(rhs, nodes, f)                          # h J^T r
        if S:                                                 # pair rows: +f on i, -f on j
            np.add.at(rhs, ps.i, pf)
            np.add.at(rhs, ps.j, -pf)
        vnew = model.solve_P(rhs)                             # global step
        df = 0.0
        if C:                                                 # contact update per node
            ubar = vnew[nodes] - f / model.mass[nodes, None]
            vc, fn, mode = signorini_coulomb(ubar, normal, gap, mu, h, model.mass[nodes])
            df = np.max(np.abs(fn - f) / model.mass[nodes, None])
            f = fn
            vnew[nodes] = vc
        if S:                                                 # contact update per pair
            mi, mj = model.mass[ps.i, None], model.mass[ps.j, None]
            ubi = vnew[ps.i] - pf / mi                        # free velocities of both nodes
            ubj = vnew[ps.j] + pf / mj
            urel = ubi - ubj                                  # relative response f / m_ij
            _, fn, ps.mode = signorini_coulomb(urel, ps.normal, ps.gap, np.full(S, model.self_mu), h, ps.mred)
            df = max(df, np.max(np.abs(fn - pf) / mi), np.max(np.abs(fn - pf) / mj))
            pf = fn
            ps.ubar = urel
            vnew[ps.i] = ubi + fn / mi
            vnew[ps.j] = ubj - fn / mj
        k += 1
        # the iterate is the pair (v, impulses): a contact node held by the
        # contact update keeps its velocity while its impulse still changes
        dv = max(np.max(np.abs(vnew - vk)) if vk.size else 0.0, df)
        vk = vnew
        if energy_log is not None:
            energy_log.append(implicit_energy(model, x + h * vk, y, t1))
        if tol is None:
            if k >= K:
                break
        elif dv <= tol or k >= max_iters:
            break
    x1 = x + h * vk
    ps.impulse = pf
    return StepRecord(x.copy(), v.copy(), x1, vk.copy(),
                      Contact(nodes, obst, normal, gap, mu, ubar, f, mode), k, ps)


def step_impulses(model: Model, rec: StepRecord) -> np.ndarray:
    """Per-node impulses (m, 3) at the end of a recorded step (zero off contact)."""
    f = np.zeros((model.m, 3))
    f[rec.contact.nodes] = rec.contact.impulse
    if rec.pairs is not None and rec.pairs.i.size:
        f[rec.pairs.i] = rec.pairs.impulse
        f[rec.pairs.j] = -rec.pairs.impulse
    return f


def rollout(model: Model, x0=None, v0=None, steps: Optional[int] = None, iters=None, tol=None,
            warm_start: bool = False, max_iters: int = 100000):
    """Forward simulation over T steps; returns the list of step records.
    warm_start: each step's contact iteration starts from the previous step's
    impulses (see forward_step)."""
    x = np.asarray(model.X if x0 is None else x0, float).copy()
    v = np.asarray(model.scene.v0 if v0 is None else v0, float).copy()
    T = model.scene.steps if steps is None else steps
    recs = []
    fp = None
    for n in range(T):
        r = forward_step(model, x, v, n, iters=iters, tol=tol, max_iters=max_iters,
                         f_prev=fp if warm_start else None)
        recs.append(r)
        x, v = r.x1, r.v1
        fp = step_impulses(model, r)
    return recs


def elastic_energy(model: Model, x: np.ndarray, t: float) -> float:
    """W(x) = sum_i min_p w_i/2 |A_i x - p|^2 (eqn pd_energy)."""
    p, q = local_projection(model, x)
    W = 0.5 * float(np.sum(model.w * np.sum((q - p) ** 2, axis=1)))
    if model.attach.size:
        d = x[model.attach] - model.attach_targets(t)
        W += 0.5 * model.w_att * float(np.sum(d * d))
    return W


def implicit_energy(model: Model, x: np.ndarray, y: np.ndarray, t: Optional[float] = None) -> float:
    """g(x) = (1/2h^2)(x-y)^T M (x-y) + W(x) (eqn implicit_energy)."""
    if t is None:
        t = 0.0
    d = x - y
    return 0.5 / model.h ** 2 * float(np.sum(model.mass[:, None] * d * d)) + elastic_energy(model, x, t)


# =========================================================================== backward

def projection_jacobian_blocks(model: Model, x: np.ndarray):
    """dp_i/d(A_i x) for the sphere projections: (rho/|q|)(I - qhat qhat^T), zero for
    rho = 0 and for degenerate q (Sec. 4.1, the DiffPD Hessian term)."""
    q = model.A @ x
    nq = np.linalg.norm(q, axis=1)
    act = model.rho > 0
    ok = act & (nq >= DEGENERATE_REL * np.maximum(model.rho, 1e-300))
    J = np.zeros((model.nc, 3, 3))
    qh = np.zeros_like(q)
    qh[ok] = q[ok] / nq[ok, None]
    s = np.zeros(model.nc)
    s[ok] = model.rho[ok] / nq[ok]
    J[ok] = s[ok, None, None] * (np.eye(3)[None] - qh[ok, :, None] * qh[ok, None, :])
    return J


def _kron3(Ms: sp.spmatrix) -> sp.csr_matrix:
    return sp.kron(Ms, sp.eye(3), format="csr")


def _blockdiag3(blocks: np.ndarray) -> sp.csr_matrix:
    nb = blocks.shape[0]
    r = (3 * np.arange(nb)[:, None, None] + np.arange(3)[None, :, None]) * np.ones((1, 1, 3), int)
    c = (3 * np.arange(nb)[:, None, None] + np.arange(3)[None, None, :]) * np.ones((1, 3, 1), int)
    return sp.csr_matrix((blocks.ravel(), (r.ravel(), c.ravel())), shape=(3 * nb, 3 * nb))


def delta_P(model: Model, x: np.ndarray) -> sp.csr_matrix:
    """Delta P = h^2 sum_i w_i A_i^T dp_i*/dx at x (eqn adjoint_pd), 3m x 3m."""
    J = projection_jacobian_blocks(model, x)
    At = _kron3(model.A)                                      # (3nc, 3m)
    D = _blockdiag3(model.h ** 2 * model.w[:, None, None] * J)
    return (At.T @ D @ At).tocsr()


def sc_jacobian_blocks(ubar, normal, gap, mu, mode, h: float):
    """T = d v / d ubar of the closed-form contact update (eqn contact_all) per
    contact: identity for take-off, zero for stick, (1-s)Pi + s t t^T + mu t n^T
    for slip, with Pi = I - n n^T, t the unit free tangential velocity and
    s = mu(-a)/|u_T|.  Vectorised: ubar, normal (C, 3); gap, mu, mode (C,)."""
    C = mode.size
    T = np.zeros((C, 3, 3))
    T[mode == TAKEOFF] = np.eye(3)
    sl = mode == SLIP
    if np.any(sl):
        n = normal[sl]
        ub = ubar[sl]
        un = np.sum(n * ub, axis=1)
        ut = ub - un[:, None] * n
        tau = np.linalg.norm(ut, axis=1)
        t = ut / tau[:, None]
        a = un + gap[sl] / h
        m_ = mu[sl]
        s = m_ * (-a) / tau
        Pi = np.eye(3)[None] - n[:, :, None] * n[:, None, :]
        T[sl] = ((1 - s)[:, None, None] * Pi + s[:, None, None] * t[:, :, None] * t[:, None, :]
                 + m_[:, None, None] * t[:, :, None] * n[:, None, :])
    return T


def contact_jacobian_blocks(contact: Contact, h: float):
    """T_j = d v_j / d ubar_j of the obstacle contacts (see sc_jacobian_blocks)."""
    return sc_jacobian_blocks(contact.ubar, contact.normal, contact.gap, contact.mu, contact.mode, h)


def step_contact_jacobian(model: Model, rec: StepRecord) -> sp.csr_matrix:
    """T = d v / d ubar of the step's whole contact update (3m x 3m): identity
    off contact, the per-node blocks of the obstacle contacts, and for a pair
    (i, j) with relative block T_r and D = T_r - I the two-node block
    [[I + a_i D, -a_i D], [-a_j D, I + a_j D]], a_i = m_ij / m_i, since
    v_i = ubar_i + f/m_i, v_j = ubar_j - f/m_j with f = m_ij (u - ubar_i + ubar_j)."""
    m = model.m
    h = model.h
    Tb = np.tile(np.eye(3), (m, 1, 1))
    if rec.contact.nodes.size:
        Tb[rec.contact.nodes] = contact_jacobian_blocks(rec.contact, h)
    T = _blockdiag3(Tb).tolil()
    ps = rec.pairs
    if ps is not None and ps.i.size:
        D = sc_jacobian_blocks(ps.ubar, ps.normal, ps.gap, np.full(ps.i.size, model.self_mu), ps.mode, h)
        D = D - np.eye(3)[None]
        for q in range(ps.i.size):
            i, j = int(ps.i[q]), int(ps.j[q])
            ai, aj = ps.mred[q] / model.mass[i], ps.mred[q] / model.mass[j]
            for (r, c, blk) in ((i, i, np.eye(3) + ai * D[q]), (i, j, -ai * D[q]),
                                (j, i, -aj * D[q]), (j, j, np.eye(3) + aj * D[q])):
                T[3 * r:3 * r + 3, 3 * c:3 * c + 3] = blk
    return T.tocsr()


def frame_gradients(lam, normal, gap, ubar, mu, mode, h: float):
    """For active contacts (stick / slip) with multipliers lam = M zeta (a pair:
    m_ij (zeta_i - zeta_j)): lam^T dv/dphi, (dv/dn)^T lam (ubar and the gap held
    fixed) and lam^T dv/dmu of the closed-form update, v = -(phi/h) n (stick),
    -(phi/h) n + u_T + mu a t (slip).  Returns (C,), (C, 3), (C,)."""
    I3 = np.eye(3)[None]
    nrm, phi, ub = normal, gap, ubar
    un = np.sum(nrm * ub, axis=1)
    a = un + phi / h
    ut = ub - un[:, None] * nrm
    tau = np.linalg.norm(ut, axis=1)
    sl = mode == SLIP
    t = np.zeros_like(ut)
    t[sl] = ut[sl] / tau[sl, None]
    # d v / d phi: stick -n/h, slip (-n + mu t)/h
    dv_dphi = (-nrm + (mu * sl)[:, None] * t) / h
    # d v / d n (ubar, phi held fixed)
    dv_dn = -(phi / h)[:, None, None] * I3 * np.ones((mode.size, 1, 1))
    dmu = np.zeros(mode.size)
    if np.any(sl):
        nn, ubs, ts, taus, As, mus = nrm[sl], ub[sl], t[sl], tau[sl], a[sl], mu[sl]
        dut_dn = -un[sl][:, None, None] * I3 - nn[:, :, None] * ubs[:, None, :]
        dt_dut = (I3 - ts[:, :, None] * ts[:, None, :]) / taus[:, None, None]
        dv_dn[sl] += (dut_dn + mus[:, None, None] * ts[:, :, None] * ubs[:, None, :]
                      + (mus * As)[:, None, None] * np.einsum('cij,cjk->cik', dt_dut, dut_dn))
        dmu[sl] = np.sum(lam[sl] * ts, axis=1) * As
    dphi = np.sum(lam * dv_dphi, axis=1)
    dn = np.einsum('cji,cj->ci', dv_dn, lam)                  # (dv/dn)^T lambda
    return dphi, dn, dmu


def backward_step(model: Model, rec: StepRecord, gx: np.ndarray, gv: np.ndarray,
                  n: int, direct: bool = True, iter_tol: float = 1e-12, iter_max: int = 100000):
    """Adjoint of one step (Sec. 4.2, eqns adjoint_vv, adjoint_v, ppr_adjoint):
    given dL/dx_{n+1} and dL/dv_{n+1}, solve (M + H Tc^T) zeta = gbar with
    H = h^2 Hess W(x_{n+1}) = P - M - Delta P and Tc = M T M^{-1} (T = dv/dubar
    of the contact update; Tc = T when T is block diagonal per node), and
    return dL/dx_n, dL/dv_n and the parameter gradients of this step.

    Why Tc: the converged step satisfies M ubar + h grad W(x_n + h v) = c with
    v = V(ubar), so dL/dc = (M + H T)^{-T} T^T gbar = Tc^T zeta.  The plain
    definition of the adjoint is the direct solve (the paper's ground truth);
    ``direct=False`` runs the paper's iteration P zeta^{k+1} = (Delta P +
    Delta R) zeta^k + gbar instead.  dmu holds one entry per obstacle, then
    (with self-collision on) the self-friction coefficient's."""
    h = model.h
    m = model.m
    x1 = rec.x1
    gbar = gv + h * gx                                        # x_{n+1} = x_n + h v_{n+1}
    dP = delta_P(model, x1)
    PmM = _kron3(h * h * model.K_s)
    Hm = (PmM - dP).tocsr()                                   # h^2 Hess W(x_{n+1})
    Mk = sp.diags(np.repeat(model.mass, 3))
    Minv = sp.diags(1.0 / np.repeat(model.mass, 3))
    T = step_contact_jacobian(model, rec)
    TT = (Mk @ T @ Minv).T.tocsr()                            # Tc^T
    Aadj = (Mk + Hm @ TT).tocsc()
    gb = gbar.reshape(-1)
    if direct:
        zeta = spla.splu(Aadj).solve(gb)
        iters = 0
    else:
        zeta, iters = adjoint_fixed_point(model, Hm, dP, TT, gb, iter_tol, iter_max)
    z = TT @ zeta
    dv = (Mk @ z).reshape(m, 3)
    dx = gx - (Hm @ z).reshape(m, 3) / h
    zeta3 = zeta.reshape(m, 3)
    z3 = z.reshape(m, 3)
    # parameter gradients: dc/dw_i = h A_i^T (p_i - q_i) at x_{n+1}
    p, q = local_projection(model, x1)
    Az = model.A @ z3
    dw = h * np.sum(Az * (p - q), axis=1)
    self_on = model.self_d > 0
    dmu = np.zeros(len(model.obstacles) + (1 if self_on else 0))
    ct = rec.contact
    act = ct.mode != TAKEOFF
    if np.any(act):
        j = ct.nodes[act]
        nrm = ct.normal[act]
        lam = model.mass[j, None] * zeta3[j]                  # lambda = M zeta
        dphi, dn, dmu_c = frame_gradients(lam, nrm, ct.gap[act], ct.ubar[act], ct.mu[act], ct.mode[act], h)
        np.add.at(dmu, ct.obstacle[act], dmu_c)
        np.add.at(dx, j, dphi[:, None] * nrm)                 # grad phi = n (plane, sphere)
        for oi, o in enumerate(model.obstacles):
            if o.kind == MESH:
                # dn/dx of the frame at x_n: 0 on a face, (I - n n^T)/phi at a
                # vertex, (I - n n^T - e e^T)/phi on an edge (the closest point
                # slides along it); phi = 0 exactly: taken as a face
                so = np.nonzero(ct.obstacle[act] == oi)[0]
                if so.size == 0:
                    continue
                phim, nm, regm, em = mesh_query(o, rec.x0[j[so]])
                for q_, i_ in enumerate(so):
                    if regm[q_] == FACE or phim[q_] == 0.0:
                        continue
                    dni = dn[i_]
                    g = dni - (nm[q_] @ dni) * nm[q_]
                    if regm[q_] == EDGE:
                        g = g - (em[q_] @ dni) * em[q_]
                    dx[j[i_]] += g / phim[q_]
                continue
            if o.kind != SPHERE:
                continue
            so = ct.obstacle[act] == oi
            if not np.any(so):
                continue
            r = np.linalg.norm(rec.x0[j[so]] - np.asarray(o.point, float), axis=1)
            ns = nrm[so]
            dns = dn[so]
            proj = dns - np.sum(ns * dns, axis=1)[:, None] * ns   # (I - n n^T) dn
            np.add.at(dx, j[so], proj / r[:, None])
    ps = rec.pairs
    if ps is not None and ps.i.size and np.any(ps.mode != TAKEOFF):
        # pairs: v_i, v_j move by +-(m_ij/m) du, so the multiplier of the relative
        # update is m_ij (zeta_i - zeta_j); phi = |x_i - x_j| - d and
        # n = (x_i - x_j)/|x_i - x_j| give d phi/dx_i = n, dn/dx_i = (I - n n^T)/r,
        # and the negatives for x_j
        a_ = ps.mode != TAKEOFF
        i, j = ps.i[a_], ps.j[a_]
        nrm = ps.normal[a_]
        lam = ps.mred[a_, None] * (zeta3[i] - zeta3[j])
        dphi, dn, dmu_c = frame_gradients(lam, nrm, ps.gap[a_], ps.ubar[a_],
                                          np.full(i.size, model.self_mu), ps.mode[a_], h)
        g = dphi[:, None] * nrm + (dn - np.sum(nrm * dn, axis=1)[:, None] * nrm) / ps.dist[a_, None]
        np.add.at(dx, i, g)
        np.add.at(dx, j, -g)
        dmu[-1] += np.sum(dmu_c)
    return dx, dv, dw, dmu, iters


def adjoint_fixed_point(model: Model, Hm, dP, TT, gbar, tol, max_iters):
    """Paper's iteration for the contact adjoint (eqn ppr_adjoint): with the
    prefactored P, zeta^{k+1} = P^{-1}[gbar + Delta P z^k + (P - M)(zeta^k - z^k)],
    z^k = T^T zeta^k, which at its fixed point solves (M + H T^T) zeta = gbar."""
    m = model.m
    PmM = _kron3(model.h ** 2 * model.K_s)
    zeta = np.zeros_like(gbar)
    for k in range(1, max_iters + 1):
        z = TT @ zeta
        r = gbar + dP @ z + PmM @ (zeta - z)
        zn = model.solve_P(r.reshape(m, 3)).reshape(-1)
        d = np.max(np.abs(zn - zeta))
        zeta = zn
        if d <= tol * max(np.max(np.abs(zeta)), 1e-300):
            return zeta, k
    return zeta, max_iters


@dataclasses.dataclass
class Gradients:
    dx0: np.ndarray
    dv0: np.ndarray
    dw: np.ndarray          # per constraint: springs first, then bending
    dmu: np.ndarray         # per obstacle, then self-friction (with self-collision on)
    dregion: Optional[np.ndarray] = None
    dforce: Optional[np.ndarray] = None         # (m, 3) dL/dF
    dforce_scale: Optional[np.ndarray] = None   # (T,) dL/ds_n

    @property
    def dk_spring(self):
        return self.dw


def force_gradients_of_step(model: Model, n: int, dL_dvn: np.ndarray):
    """Step n's share of dL/dF and dL/ds_n from dL/dv_n = M z_n: the external
    force enters b_hat as h s_n F, next to M v_n, so dL/df_ext,n = h z_n."""
    hz = model.h * dL_dvn / model.mass[:, None]
    s = 1.0 if model.force_scale is None else float(model.force_scale[n])
    return s * hz, float(np.sum(model.force * hz))


def backward(model: Model, recs: List[StepRecord], dL_dxT: np.ndarray, dL_dvT=None,
             dL_dx_steps=None, direct: bool = True) -> Gradients:
    """Backpropagation through the whole rollout (Sec. 4.1, eqn adjoint): the
    per-step adjoints chained from the last step to the first.

    External force: v_n and f_ext,n enter step n only through b_hat (as M v_n
    and h f_ext,n; eqn pd_velocity) and through the predictor and the initial
    guess, which the adjoint of the converged step does not see, so
    dL/df_ext,n = h M^{-1} dL/dv_n = h z_n.  With f_ext,n = s_n F this gives
    dL/dF = h sum_n s_n z_n and dL/ds_n = h F . z_n."""
    gx = np.asarray(dL_dxT, float).copy()
    if dL_dx_steps is not None:                               # a per-step loss term on x_T as well
        gx = gx + dL_dx_steps[len(recs)]
    gv = np.zeros_like(gx) if dL_dvT is None else np.asarray(dL_dvT, float).copy()
    dw = np.zeros(model.nc)
    dmu = np.zeros(len(model.obstacles) + (1 if model.self_d > 0 else 0))
    T = len(recs)
    dF = np.zeros((model.m, 3))
    ds = np.zeros(T)
    for n in range(T - 1, -1, -1):
        dx, dv, dwn, dmun, _ = backward_step(model, recs[n], gx, gv, n, direct=direct)
        dw += dwn
        dmu += dmun
        dFn, ds[n] = force_gradients_of_step(model, n, dv)
        dF += dFn
        gx, gv = dx, dv
        if dL_dx_steps is not None:
            gx = gx + dL_dx_steps[n]
    dregion = None
    if model.region is not None:
        dregion = np.zeros(model.region_scale.size)
        np.add.at(dregion, model.region, dw * model.base_w)
    return Gradients(gx, gv, dw, dmu, dregion, dF, ds)


# =========================================================================== losses

def centroid_loss(model: Model, x: np.ndarray, target: np.ndarray):
    """Squared distance of the centroid to a target; returns (L, dL/dx)."""
    c = x.mean(axis=0)
    d = c - target
    return float(d @ d), np.tile(2.0 * d / x.shape[0], (x.shape[0], 1))


def apex_angle_loss(x: np.ndarray, waist: np.ndarray, hem: np.ndarray):
    """Apex angle 2 atan(mean hem radius / (mean waist y - mean hem y)) of a
    skirt about the vertical axis; returns (angle, d angle / dx)."""
    rh = np.sqrt(x[hem, 0] ** 2 + x[hem, 2] ** 2)
    R = rh.mean()
    Hh = x[waist, 1].mean() - x[hem, 1].mean()
    ang = 2.0 * math.atan2(R, Hh)
    den = R * R + Hh * Hh
    dR = 2.0 * Hh / den
    dH = -2.0 * R / den
    g = np.zeros_like(x)
    g[hem, 0] += dR * x[hem, 0] / rh / hem.size
    g[hem, 2] += dR * x[hem, 2] / rh / hem.size
    g[waist, 1] += dH / waist.size
    g[hem, 1] -= dH / hem.size
    return ang, g
