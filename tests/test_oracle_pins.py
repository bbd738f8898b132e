"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed
forms (free fall, rest state, rigid motions, textbook friction cases, the
sliding-particle trajectory), invariants (monotone PD energy, the
Signorini-Coulomb conditions, continuity in mu), brute-force assemblies and
central finite differences on tiny meshes, so that a dropped term, a wrong
sign or index, or a transposed operand fails at least one of them.
"""
import math
import os

import numpy as np
import pytest

import scenes
from oracle import diffcloth_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------------ helpers

def particle_scene(points, obstacles, v0, steps=1, h=1.0 / 120.0, mass=1e-3):
    """Independent particles: a grid mesh with zero spring and bending weights."""
    pts = np.asarray(points, float)
    n = int(round(math.sqrt(pts.shape[0])))
    assert n * n == pts.shape[0]
    _, tris, edges = scenes.grid_mesh(n)
    return scenes.Scene(
        name="particles", X=pts, tris=tris, edges=edges,
        edge_stiffness=np.zeros(edges.shape[0]), node_mass=np.full(pts.shape[0], mass),
        v0=np.asarray(v0, float) * np.ones_like(pts), h=h, steps=steps, bend_weight=0.0,
        obstacles=obstacles)


def dense_constraint_rows(model):
    """Explicit A_i (3 x 3m) of every spring/bending constraint, built from the
    edge list and the stencil coefficients (eqn pd_project)."""
    rows = []
    A = model.A.tocsr()
    for i in range(model.nc):
        Ai = np.zeros((3, 3 * model.m))
        for p in range(A.indptr[i], A.indptr[i + 1]):
            k = A.indices[p]
            Ai[:, 3 * k:3 * k + 3] += A.data[p] * np.eye(3)
        rows.append(Ai)
    return rows


def converged_loss(scene, tol=1e-13, **kw):
    """Converged rollout and L = centroid loss + a seeded linear functional of x_T
    (the latter makes L sensitive to the cloth's deformation)."""
    x0 = kw.pop("x0", None)
    v0 = kw.pop("v0", None)
    model = O.Model(scene, **kw)
    recs = O.rollout(model, x0=x0, v0=v0, tol=tol)
    L, g = O.centroid_loss(model, recs[-1].x1, scene.target)
    c = np.random.default_rng(1234).normal(size=g.shape)
    return model, recs, L + float(np.sum(c * recs[-1].x1)), g + c


def modes_of(recs):
    return [tuple(r.contact.nodes.tolist()) + tuple(r.contact.mode.tolist()) for r in recs]


# ------------------------------------------------------------------ constraint set

def test_edges_match_triangle_edges():
    for sc in (scenes.c1_napkin(0), scenes.tiny_scene(4), scenes.c3_skirt(0, 8, 6)):
        e = O.triangle_edges(sc.tris)
        assert np.array_equal(e, sc.edges.astype(np.int64))


def test_cotangent_stencil_on_regular_grid_is_five_point():
    # cot 45 deg = 1 on the axis edges, cot 90 deg = 0 on the diagonals
    X, tris, _ = scenes.grid_mesh(5, 0.4)
    centers, L = O.cotangent_bending_stencils(X, tris)
    assert sorted(centers.tolist()) == [i * 5 + j for i in range(1, 4) for j in range(1, 4)]
    L = L.toarray()
    for r, b in enumerate(centers):
        i, j = divmod(int(b), 5)
        expect = np.zeros(25)
        for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1)):
            expect[(i + di) * 5 + (j + dj)] = 1.0
        expect[b] = -4.0
        assert np.allclose(L[r], expect, atol=1e-12)


def test_global_matrix_matches_bruteforce_assembly():
    sc = scenes.tiny_scene(4, pins=True, seed=3)
    model = O.Model(sc)
    h = model.h
    P = np.diag(np.repeat(model.mass, 3))
    for w, Ai in zip(model.w, dense_constraint_rows(model)):
        P += h * h * w * Ai.T @ Ai
    for j in model.attach:
        Aj = np.zeros((3, 3 * model.m))
        Aj[:, 3 * j:3 * j + 3] = np.eye(3)
        P += h * h * model.w_att * Aj.T @ Aj
    P_or = np.kron(model.P_s.toarray(), np.eye(3))
    assert np.allclose(P_or, P, rtol=1e-13, atol=1e-15)
    # global solve: residual and agreement with a dense solve of the brute-force P
    rng = np.random.default_rng(0)
    rhs = rng.normal(size=(model.m, 3))
    v = model.solve_P(rhs)
    assert np.linalg.norm(P @ v.ravel() - rhs.ravel()) <= 1e-13 * np.linalg.norm(rhs)
    assert np.allclose(v.ravel(), np.linalg.solve(P, rhs.ravel()), rtol=1e-12, atol=1e-14)


def test_projection_of_rigid_motion_is_identity():
    sc = scenes.tiny_scene(4, seed=5)     # noisy rest shape: curved bending active
    model = O.Model(sc)
    R = O.rotation((0.3, 1.0, -0.2), 0.7)
    x = sc.X @ R.T + np.array([0.4, -1.0, 2.0])
    p, q = O.local_projection(model, x)
    act = model.rho > 0
    assert act.sum() > model.n_spring          # bending constraints are curved here
    assert np.allclose(p[act], q[act], rtol=0, atol=1e-14)
    assert np.allclose(np.linalg.norm(p[act], axis=1), model.rho[act], rtol=1e-14)


# ------------------------------------------------------------------ forward closed forms

def test_free_fall_is_exact():
    sc = scenes.tiny_scene(4, steps=12, obstacle=None, seed=2)
    vel = np.array([0.3, 0.5, -0.2])
    sc.v0 = np.tile(vel, (sc.n_nodes, 1))
    model = O.Model(sc)
    recs = O.rollout(model)
    T, h, g = sc.steps, sc.h, np.asarray(sc.gravity)
    expect = sc.X + T * h * vel + h * h * g * T * (T + 1) / 2
    assert np.allclose(recs[-1].x1, expect, rtol=0, atol=1e-12)
    # per step: x_{n+1} = x_n + h v_n + h^2 g
    for r in recs:
        assert np.allclose(r.x1, r.x0 + h * r.v0 + h * h * g, rtol=0, atol=1e-13)


def test_rest_state_stays_still():
    sc = scenes.tiny_scene(4, steps=10, obstacle=None, pins=True, seed=4)
    sc.gravity = (0.0, 0.0, 0.0)
    model = O.Model(sc)
    recs = O.rollout(model)
    assert np.max(np.abs(recs[-1].x1 - sc.X)) <= 1e-12


def test_pd_energy_decreases_monotonically():
    sc = scenes.c1_napkin(0, steps=6)
    sc.obstacles = []
    model = O.Model(sc)
    x, v = sc.X.copy(), sc.v0.copy()
    checked = 0
    for n in range(sc.steps):
        log = []
        r = O.forward_step(model, x, v, n, iters=40, energy_log=log)
        e = np.array(log)
        assert np.all(e[1:] <= e[:-1] * (1 + 1e-12) + 1e-15), (n, np.max(np.diff(e)))
        checked += e.size
        x, v = r.x1, r.v1
    assert checked == 6 * 40


def test_converged_step_satisfies_implicit_euler():
    sc = scenes.tiny_scene(4, steps=3, obstacle=None, pins=True, seed=7)
    model = O.Model(sc)
    recs = O.rollout(model, tol=1e-14, steps=3)
    rows = dense_constraint_rows(model)
    for n, r in enumerate(recs):
        x = r.x1
        y = O.inertial_predictor(model, r.x0, r.v0)
        p, _ = O.local_projection(model, x)
        grad = np.zeros(3 * model.m)
        for i, Ai in enumerate(rows):
            grad += model.w[i] * Ai.T @ (Ai @ x.ravel() - p[i])
        tgt = model.attach_targets((n + 1) * model.h)
        for c, j in enumerate(model.attach):
            grad[3 * j:3 * j + 3] += model.w_att * (x[j] - tgt[c])
        res = (model.mass[:, None] * (x - y)).ravel() / model.h ** 2 + grad
        scale = np.abs(grad).max()
        assert np.abs(res).max() <= 1e-8 * scale


# ------------------------------------------------------------------ contact law

def test_signorini_coulomb_conditions_hold():
    rng = np.random.default_rng(11)
    C = 4000
    n = rng.normal(size=(C, 3))
    n /= np.linalg.norm(n, axis=1)[:, None]
    ub = rng.normal(size=(C, 3))
    phi = rng.uniform(-0.01, 0.01, C)
    mu = rng.uniform(0.0, 1.5, C)
    mass = rng.uniform(1e-4, 1e-2, C)
    h = 1.0 / 120.0
    v, f, mode = O.signorini_coulomb(ub, n, phi, mu, h, mass)
    assert set(np.unique(mode)) == {O.TAKEOFF, O.STICK, O.SLIP}
    assert np.allclose(v, ub + f / mass[:, None], rtol=0, atol=1e-14)   # v = ubar + W f
    r = f / h
    rN = np.sum(r * n, axis=1)
    rT = r - rN[:, None] * n
    vN = np.sum(v * n, axis=1)
    vT = v - vN[:, None] * n
    uN = vN + phi / h                                           # gap-corrected normal velocity
    assert np.all(rN >= -1e-12 * np.abs(r).max(axis=1))
    assert np.all(np.linalg.norm(rT, axis=1) <= mu * rN * (1 + 1e-12) + 1e-13)
    to, st, sl = mode == O.TAKEOFF, mode == O.STICK, mode == O.SLIP
    assert np.all(r[to] == 0.0) and np.all(uN[to] > 0)
    assert np.allclose(vT[st], 0.0, atol=1e-14) and np.allclose(uN[st], 0.0, atol=1e-12)
    assert np.allclose(uN[sl], 0.0, atol=1e-12)
    assert np.allclose(np.linalg.norm(rT[sl], axis=1), mu[sl] * rN[sl], rtol=1e-12)
    assert np.all(np.sum(rT[sl] * vT[sl], axis=1) <= 1e-15)
    cross = np.cross(rT[sl], vT[sl])
    assert np.allclose(cross, 0.0, atol=1e-12 * np.abs(rT[sl]).max() * np.abs(vT[sl]).max())


def test_friction_special_cases():
    rng = np.random.default_rng(12)
    C = 2000
    n = np.tile([0.0, 1.0, 0.0], (C, 1))
    ub = rng.normal(size=(C, 3))
    ub[:, 1] = -np.abs(ub[:, 1])
    phi = np.zeros(C)
    mass = np.ones(C)
    _, _, mode0 = O.signorini_coulomb(ub, n, phi, np.zeros(C), 0.01, mass)
    assert np.all(mode0 == O.SLIP)                   # mu = 0: no stick unless u_T = 0
    ub2 = ub.copy()
    ub2[:10, [0, 2]] = 0.0
    _, _, m2 = O.signorini_coulomb(ub2, n, phi, np.zeros(C), 0.01, mass)
    assert np.all(m2[:10] == O.STICK)
    _, _, mbig = O.signorini_coulomb(ub, n, phi, np.full(C, 1e6), 0.01, mass)
    assert np.all(mbig == O.STICK)                   # huge mu: every pressed node sticks


def _inclined(theta, mu, steps=1, v0=(0.0, 0.0, 0.0)):
    nrm = np.array([-math.sin(theta), math.cos(theta), 0.0])
    tang = np.array([math.cos(theta), math.sin(theta), 0.0])
    pts = np.array([a * tang + b * np.array([0.0, 0.0, 1.0]) for a in (0.0, 0.3) for b in (0.0, 0.3)])
    sc = particle_scene(pts, [scenes.Obstacle(scenes.PLANE, (0, 0, 0), tuple(nrm), 0.0, mu)],
                        v0, steps=steps)
    return sc, nrm, tang


def test_inclined_plane_textbook_cases():
    rows = np.loadtxt(os.path.join(GOLDEN, "inclined_plane.txt"))
    for theta_deg, mu, expect in rows:
        sc, nrm, tang = _inclined(math.radians(theta_deg), mu)
        recs = O.rollout(O.Model(sc))
        assert np.all(recs[0].contact.mode == int(expect)), (theta_deg, mu)
        if int(expect) == O.STICK:
            assert np.allclose(recs[0].x1, sc.X, atol=1e-15)
        else:
            # slides along the slope with a = g (sin - mu cos), stays on the plane
            g = 9.8
            acc = g * (math.sin(math.radians(theta_deg)) - mu * math.cos(math.radians(theta_deg)))
            h = sc.h
            assert np.allclose((recs[0].x1 - sc.X) @ nrm, 0.0, atol=1e-15)
            assert np.allclose((recs[0].x1 - sc.X) @ tang, -h * h * acc, rtol=1e-12)


def test_sliding_particle_decelerates_then_sticks():
    mu, h, g = 0.3, 1.0 / 120.0, 9.8
    vx = 0.05
    pts = np.array([[a, 0.0, b] for a in (0.0, 0.5) for b in (0.0, 0.5)])
    sc = particle_scene(pts, [scenes.Obstacle(scenes.PLANE, (0, 0, 0), (0, 1, 0), 0.0, mu)],
                        (vx, 0.0, 0.0), steps=30, h=h)
    recs = O.rollout(O.Model(sc))
    v = vx
    for r in recs:
        if v > mu * g * h:
            v = v - mu * g * h
            md = O.SLIP
        else:
            v = 0.0
            md = O.STICK
        assert np.all(r.contact.mode == md)
        assert np.allclose(r.v1[:, 0], v, atol=1e-14)
        assert np.allclose(r.v1[:, 1], 0.0, atol=1e-15)


def test_landing_stops_on_the_surface():
    # falls from 1 cm, lands exactly on the linearised surface on the contact step
    pts = np.array([[a, 0.01, b] for a in (0.0, 0.5) for b in (0.0, 0.5)])
    sc = particle_scene(pts, [scenes.Obstacle(scenes.PLANE, (0, 0, 0), (0, 1, 0), 0.0, 0.5)],
                        (0.0, -0.9, 0.0), steps=3)
    recs = O.rollout(O.Model(sc))
    first = next(i for i, r in enumerate(recs) if r.contact.nodes.size)
    r = recs[first]
    assert np.all(r.contact.mode == O.STICK)
    assert np.allclose(r.x1[:, 1], 0.0, atol=1e-15)


def test_sphere_polar_angle_stick_criterion():
    # a particle resting on a sphere at polar angle theta sticks iff tan(theta) <= mu
    for theta, mu, expect in ((0.4, 0.5, O.STICK), (0.4, 0.4, O.SLIP), (0.9, 1.3, O.STICK),
                              (0.9, 1.2, O.SLIP)):
        R = 0.5
        pts = np.array([[R * math.sin(theta + d) * math.cos(psi), R * math.cos(theta + d),
                         R * math.sin(theta + d) * math.sin(psi)]
                        for d in (0.0, 1e-3) for psi in (0.0, 1e-2)])
        sc = particle_scene(pts, [scenes.Obstacle(scenes.SPHERE, (0, 0, 0), (0, 1, 0), R, mu)],
                            (0.0, 0.0, 0.0))
        recs = O.rollout(O.Model(sc))
        assert np.all(recs[0].contact.mode == expect), (theta, mu)


def test_velocities_continuous_in_mu():
    # branch switches stick <-> slip <-> take-off do not create jumps (Sec. 5.1)
    sc = scenes.tiny_scene(4, steps=12, obstacle="sphere", seed=8, height=0.002, v0_scale=0.3)
    mus = np.linspace(0.0, 0.6, 121)
    finals = []
    for mu in mus:
        recs = O.rollout(O.Model(sc, mu=[mu]))
        finals.append(recs[-1].v1.ravel())
    finals = np.array(finals)
    d = np.abs(np.diff(finals, axis=0)).max(axis=1)
    assert d.max() <= 12 * np.median(d) + 1e-12


# ------------------------------------------------------------------ adjoint

def test_adjoint_fixed_point_equals_direct_solve():
    # the paper's iteration converges to the direct solve (its ground truth)
    rng = np.random.default_rng(21)
    for obst in ("plane", "sphere", None):
        sc = scenes.tiny_scene(4, steps=6, obstacle=obst, seed=9, height=0.003, v0_scale=0.05)
        model, recs, L, g = converged_loss(sc, tol=1e-13)
        for n in range(len(recs)):
            gx = rng.normal(size=g.shape)
            gv = rng.normal(size=g.shape)
            d = O.backward_step(model, recs[n], gx, gv, n, direct=True)
            it = O.backward_step(model, recs[n], gx, gv, n, direct=False, iter_tol=1e-14)
            for a, b in zip(d[:4], it[:4]):
                if a.size:
                    assert np.allclose(a, b, rtol=1e-9, atol=1e-10 * np.abs(a).max())


def test_no_contact_step_jacobian_matches_finite_differences():
    sc = scenes.tiny_scene(3, steps=1, obstacle=None, seed=10, v0_scale=0.2)
    model = O.Model(sc)
    r = O.forward_step(model, sc.X, sc.v0, 0, tol=1e-14, max_iters=5000)
    m3 = 3 * model.m
    Jx = np.zeros((m3, m3))
    for i in range(m3):
        e = np.zeros(m3)
        e[i] = 1.0
        dx, dv, *_ = O.backward_step(model, r, e.reshape(-1, 3), np.zeros((model.m, 3)), 0)
        Jx[i] = dx.ravel()                       # row i: d x1_i / d x0
    eps = 1e-6
    for j in range(0, m3, 4):
        xp = sc.X.copy().ravel(); xp[j] += eps
        xm = sc.X.copy().ravel(); xm[j] -= eps
        rp = O.forward_step(model, xp.reshape(-1, 3), sc.v0, 0, tol=1e-14, max_iters=5000)
        rm = O.forward_step(model, xm.reshape(-1, 3), sc.v0, 0, tol=1e-14, max_iters=5000)
        fd = (rp.x1 - rm.x1).ravel() / (2 * eps)
        assert np.allclose(Jx[:, j], fd, rtol=1e-6, atol=1e-7)


def test_linear_system_whole_trajectory_jacobian():
    # attachments + flat bending, no springs: the step is affine, so dL/dv0 is a
    # product of the per-step matrices v_{n+1} = P^-1 (M v_n + ... - (P-M) x_n / h)
    X, tris, edges = scenes.grid_mesh(4, 0.3, (0.0, 0.5, 0.0))
    sc = scenes.Scene(name="lin", X=X, tris=tris, edges=edges,
                      edge_stiffness=np.zeros(edges.shape[0]), node_mass=np.full(16, 2e-3),
                      v0=np.zeros((16, 3)), steps=8, bend_weight=0.5,
                      attach=np.array([0, 3], np.int32), obstacles=[],
                      target=np.array([0.1, 0.2, 0.3]))
    model = O.Model(sc)
    recs = O.rollout(model)
    L, g = O.centroid_loss(model, recs[-1].x1, sc.target)
    G = O.backward(model, recs, g)
    P = np.kron(model.P_s.toarray(), np.eye(3))
    Mk = np.diag(np.repeat(model.mass, 3))
    h = model.h
    Pinv = np.linalg.inv(P)
    A_v = Pinv @ Mk                          # d v_{n+1} / d v_n
    A_x = -Pinv @ (P - Mk) / h               # d v_{n+1} / d x_n
    # state s = (x, v): x' = x + h v', v' = A_x x + A_v v + c
    Ms = np.block([[np.eye(len(Mk)) + h * A_x, h * A_v], [A_x, A_v]])
    J = np.linalg.matrix_power(Ms, sc.steps)
    gs = np.concatenate([g.ravel(), np.zeros(g.size)])
    back = J.T @ gs
    assert np.allclose(G.dx0.ravel(), back[:g.size], rtol=1e-10, atol=1e-13)
    assert np.allclose(G.dv0.ravel(), back[g.size:], rtol=1e-10, atol=1e-13)


def test_sliding_particle_gradients_closed_form():
    mu, h, g, T = 0.2, 1.0 / 120.0, 9.8, 10
    vx = 1.0                                  # keeps sliding for all T steps
    pts = np.array([[a, 0.0, b] for a in (0.0, 0.5) for b in (0.0, 0.5)])
    sc = particle_scene(pts, [scenes.Obstacle(scenes.PLANE, (0, 0, 0), (0, 1, 0), 0.0, mu)],
                        (vx, 0.0, 0.0), steps=T, h=h)
    model = O.Model(sc)
    recs = O.rollout(model)
    assert all(np.all(r.contact.mode == O.SLIP) for r in recs)
    x_T = recs[-1].x1
    assert np.allclose(x_T[:, 0], pts[:, 0] + T * h * vx - mu * g * h * h * T * (T + 1) / 2, rtol=1e-13)
    # L = sum of final x coordinates
    gl = np.zeros_like(x_T)
    gl[:, 0] = 1.0
    G = O.backward(model, recs, gl)
    npart = pts.shape[0]
    assert np.isclose(G.dmu[0], -npart * g * h * h * T * (T + 1) / 2, rtol=1e-10)
    assert np.allclose(G.dv0[:, 0], T * h, rtol=1e-10)
    assert np.allclose(G.dx0[:, 0], 1.0, rtol=1e-10)
    # gap at the first step: x_1 = x_0 + h(v0 - mu(g h - delta/h)) along x
    assert np.allclose(G.dx0[:, 1], mu, rtol=1e-10)


@pytest.mark.parametrize("obst", ["plane", "sphere", None])
def test_gradients_match_central_finite_differences(obst):
    sc = scenes.tiny_scene(3, steps=8, obstacle=obst, k=50.0, mu=0.4, seed=1, height=0.005,
                           v0_scale=0.05, bend=0.02)
    model, recs, L, g = converged_loss(sc)
    G = O.backward(model, recs, g)
    base_modes = modes_of(recs)
    rng = np.random.default_rng(0)
    checks = 0

    def fd(eps, **kw):
        _, rp, Lp, _ = converged_loss(sc, **{k: v[0] for k, v in kw.items()})
        _, rm, Lm, _ = converged_loss(sc, **{k: v[1] for k, v in kw.items()})
        if modes_of(rp) != base_modes or modes_of(rm) != base_modes:
            return None
        return (Lp - Lm) / (2 * eps)

    d = rng.normal(size=sc.X.shape)
    e = 1e-6
    val = fd(e, x0=(sc.X + e * d, sc.X - e * d))
    if val is not None:
        assert abs(val - np.sum(G.dx0 * d)) <= 1e-5 * abs(val) + 1e-12
        checks += 1
    d = rng.normal(size=sc.X.shape)
    val = fd(e, v0=(sc.v0 + e * d, sc.v0 - e * d))
    if val is not None:
        assert abs(val - np.sum(G.dv0 * d)) <= 1e-5 * abs(val) + 1e-12
        checks += 1
    # per-spring stiffness and the bending weight (a relative step of 1e-4)
    k = sc.edge_stiffness
    d = rng.normal(size=k.shape) * k
    e = 1e-4
    val = fd(e, edge_stiffness=(k + e * d, k - e * d))
    if val is not None:
        ad = np.sum(G.dw[:model.n_spring] * d)
        assert abs(val - ad) <= 1e-4 * abs(val) + 1e-14, (val, ad)
        checks += 1
    wb = sc.bend_weight
    val = fd(e * wb, bend_weight=(wb * (1 + e), wb * (1 - e)))
    if val is not None:
        ad = np.sum(G.dw[model.n_spring:])
        assert abs(val - ad) <= 1e-4 * abs(val) + 1e-14, (val, ad)
        checks += 1
    if obst is not None:
        mu = sc.obstacles[0].mu
        e = 1e-5
        val = fd(e, mu=([mu + e], [mu - e]))
        if val is not None:
            assert abs(val - G.dmu[0]) <= 1e-5 * abs(val) + 1e-10, (val, G.dmu[0])
            checks += 1
    assert checks >= 3


# ------------------------------------------------------------------ losses, regions, per-step terms

def test_apex_angle_of_a_cone_and_its_gradient():
    # rest skirt: a frustum whose hem nodes lie on a circle of radius 0.30 m
    sc = scenes.c3_skirt(0, n_around=10, n_rings=5, steps=1)
    x = sc.X
    r_hem = np.sqrt(x[sc.hem_nodes, 0] ** 2 + x[sc.hem_nodes, 2] ** 2).mean()
    height = x[sc.waist_nodes, 1].mean() - x[sc.hem_nodes, 1].mean()
    ang, g = O.apex_angle_loss(x, sc.waist_nodes, sc.hem_nodes)
    assert np.isclose(ang, 2 * np.arctan(r_hem / height), rtol=1e-14)
    assert np.isclose(np.tan(ang / 2), 0.30 / height, rtol=1e-12)      # hem nodes on the 0.30 m circle
    rng = np.random.default_rng(3)
    xp = x + rng.normal(0, 0.01, x.shape)
    _, g = O.apex_angle_loss(xp, sc.waist_nodes, sc.hem_nodes)
    for _ in range(5):
        d = rng.normal(size=x.shape)
        e = 1e-6
        fd = (O.apex_angle_loss(xp + e * d, sc.waist_nodes, sc.hem_nodes)[0]
              - O.apex_angle_loss(xp - e * d, sc.waist_nodes, sc.hem_nodes)[0]) / (2 * e)
        assert abs(fd - np.sum(g * d)) <= 1e-8 * abs(fd) + 1e-12


def test_region_gradients_match_finite_differences():
    # skirt with rotating waist attachments (no contact), converged steps
    sc = scenes.c3_skirt(0, n_around=6, n_rings=4, steps=4, omega=4.0)
    sc.edge_stiffness = np.full(sc.edges.shape[0], 20.0)
    sc.node_mass = sc.node_mass * 50.0

    def run(rs):
        model = O.Model(sc, region_scale=np.asarray(rs, float))
        recs = O.rollout(model, tol=1e-14)
        ang, g = O.apex_angle_loss(recs[-1].x1, sc.waist_nodes, sc.hem_nodes)
        return model, recs, ang, g

    rs0 = np.array([1.0, 0.8, 1.2, 0.9])
    model, recs, ang, g = run(rs0)
    G = O.backward(model, recs, g)
    assert G.dregion.shape == (4,)
    for r in range(4):
        e = 1e-5 * rs0[r]
        up, dn = rs0.copy(), rs0.copy()
        up[r] += e
        dn[r] -= e
        fd = (run(up)[2] - run(dn)[2]) / (2 * e)
        assert abs(fd - G.dregion[r]) <= 1e-5 * abs(fd) + 1e-9, (r, fd, G.dregion[r])


def test_per_step_loss_terms_match_finite_differences():
    # L = sum_n c_n . x_n over n = 0..T, including the final state
    sc = scenes.tiny_scene(3, steps=5, obstacle=None, k=50.0, seed=4, v0_scale=0.05)
    cs = np.random.default_rng(5).normal(size=(sc.steps + 1,) + sc.X.shape)

    def loss(v0):
        model = O.Model(sc)
        recs = O.rollout(model, v0=v0, tol=1e-14)
        traj = np.stack([recs[0].x0] + [r.x1 for r in recs])
        return model, recs, float(np.sum(cs * traj))

    model, recs, _ = loss(sc.v0)
    G = O.backward(model, recs, np.zeros_like(sc.X), dL_dx_steps=cs)
    assert np.allclose(G.dx0, cs[0] + O.backward(model, recs, np.zeros_like(sc.X),
                                                 dL_dx_steps=np.concatenate([0 * cs[:1], cs[1:]])).dx0)
    d = np.random.default_rng(6).normal(size=sc.X.shape)
    e = 1e-6
    fd = (loss(sc.v0 + e * d)[2] - loss(sc.v0 - e * d)[2]) / (2 * e)
    assert abs(fd - np.sum(G.dv0 * d)) <= 1e-6 * abs(fd) + 1e-12


# ------------------------------------------------------------------ external force (wind) parameters

def _uniform_accel_scene(seed, steps=9):
    # no pins, no obstacle, uniform masses: a force proportional to each node's mass
    # moves the rest shape rigidly (every constraint stays at its rest value)
    sc = scenes.tiny_scene(4, steps=steps, obstacle=None, seed=seed)
    rng = np.random.default_rng(seed)
    d = rng.normal(size=3)
    sc.force = sc.node_mass[:, None] * d[None, :]
    sc.force_scale = rng.uniform(0.2, 1.5, steps)
    return sc, d


def test_uniform_external_force_translates_rigidly():
    sc, d = _uniform_accel_scene(21)
    recs = O.rollout(O.Model(sc))
    T, h, g, s = sc.steps, sc.h, np.asarray(sc.gravity), sc.force_scale
    # v_{k+1} = v_k + h (g + s_k d), x_T = x_0 + h sum_k v_{k+1}
    acc = np.cumsum(s)                                      # sum_{n <= k} s_n
    expect = sc.X + h * h * (g * T * (T + 1) / 2 + d * np.sum(acc))
    assert np.allclose(recs[-1].x1, expect, rtol=0, atol=1e-12)


def test_external_force_gradients_closed_form():
    # centroid loss of a rigid translation: x_T shifts by h^2 (T - n) d per unit of
    # s_n, and by h^2 sum_n s_n (T - n) e per unit of a force m_j e on every node
    sc, d = _uniform_accel_scene(22)
    model = O.Model(sc)
    recs = O.rollout(model)
    L, g = O.centroid_loss(model, recs[-1].x1, sc.target)
    G = O.backward(model, recs, g)
    T, h = sc.steps, sc.h
    c = recs[-1].x1.mean(axis=0) - sc.target
    n = np.arange(T)
    expect_ds = 2.0 * float(c @ d) * h * h * (T - n)
    assert np.allclose(G.dforce_scale, expect_ds, rtol=1e-9, atol=1e-15)
    for e in np.eye(3):
        got = float(np.sum(G.dforce * (sc.node_mass[:, None] * e[None, :])))
        want = 2.0 * float(c @ e) * h * h * float(np.sum(sc.force_scale * (T - n)))
        assert abs(got - want) <= 1e-9 * abs(want) + 1e-15, (got, want)


@pytest.mark.parametrize("obst", ["plane", "sphere", None])
def test_external_force_gradients_match_finite_differences(obst):
    sc = scenes.tiny_scene(3, steps=8, obstacle=obst, k=50.0, mu=0.4, seed=3, height=0.005,
                           v0_scale=0.05, bend=0.02, pins=obst is None)
    rng = np.random.default_rng(7)
    F0 = rng.normal(0.0, 0.5 * 9.8, (sc.n_nodes, 3)) * sc.node_mass[:, None]
    s0 = rng.uniform(0.3, 1.2, sc.steps)
    model, recs, L, g = converged_loss(sc, force=F0, force_scale=s0)
    G = O.backward(model, recs, g)
    assert G.dforce.shape == (sc.n_nodes, 3) and G.dforce_scale.shape == (sc.steps,)
    base_modes = modes_of(recs)
    checks = 0

    def fd(eps, **kw):
        _, rp, Lp, _ = converged_loss(sc, **{k: v[0] for k, v in kw.items()})
        _, rm, Lm, _ = converged_loss(sc, **{k: v[1] for k, v in kw.items()})
        if modes_of(rp) != base_modes or modes_of(rm) != base_modes:
            return None
        return (Lp - Lm) / (2 * eps)

    for _ in range(2):
        dF = rng.normal(size=F0.shape) * sc.node_mass[:, None]
        e = 1e-3
        val = fd(e, force=(F0 + e * dF, F0 - e * dF), force_scale=(s0, s0))
        if val is not None:
            ad = float(np.sum(G.dforce * dF))
            assert abs(val - ad) <= 1e-5 * abs(val) + 1e-12, (val, ad)
            checks += 1
    for n in (0, 3, sc.steps - 1):
        e = 1e-5
        up, dn = s0.copy(), s0.copy()
        up[n] += e
        dn[n] -= e
        val = fd(e, force=(F0, F0), force_scale=(up, dn))
        if val is not None:
            assert abs(val - G.dforce_scale[n]) <= 1e-5 * abs(val) + 1e-12, (n, val, G.dforce_scale[n])
            checks += 1
    assert checks >= 3


# ------------------------------------------------------------------ triangle-mesh obstacles

def _segment_closest(p, a, b):
    t = np.clip(np.dot(p - a, b - a) / np.dot(b - a, b - a), 0.0, 1.0)
    return a + t * (b - a)


def test_closest_point_on_triangle_against_feature_enumeration():
    # the exact distance from the candidates of a quadratic program over the
    # triangle: the plane projection when it falls inside, else the three edges
    rng = np.random.default_rng(11)
    for _ in range(300):
        a, b, c = rng.normal(size=(3, 3))
        p = rng.normal(size=3) * 2.0
        q, reg, e = O.closest_point_on_triangle(p[None], a[None], b[None], c[None])
        nrm = np.cross(b - a, c - a)
        nrm /= np.linalg.norm(nrm)
        proj = p - np.dot(p - a, nrm) * nrm
        # barycentric coordinates of the projection
        M = np.stack([b - a, c - a], axis=1)
        uv = np.linalg.lstsq(M, proj - a, rcond=None)[0]
        inside = uv[0] >= 0 and uv[1] >= 0 and uv.sum() <= 1
        cands = [proj] if inside else [_segment_closest(p, a, b), _segment_closest(p, b, c),
                                       _segment_closest(p, a, c)]
        best = min(np.linalg.norm(p - x) for x in cands)
        assert abs(np.linalg.norm(p - q[0]) - best) <= 1e-12 * (1 + best)
        assert (reg[0] == O.FACE) == inside
        if reg[0] == O.EDGE:                        # p - q is perpendicular to the edge
            assert abs(np.dot(p - q[0], e[0])) <= 1e-12 * (1 + np.linalg.norm(p - q[0]))


def test_triangulated_plane_equals_the_plane():
    sc = scenes.tiny_scene(4, steps=14, obstacle="plane", seed=12, height=0.004, v0_scale=0.1, mu=0.3)
    L = 10.0
    V = np.array([[-L, 0.0, -L], [L, 0.0, -L], [L, 0.0, L], [-L, 0.0, L]])
    T = np.array([[0, 3, 2], [0, 2, 1]], np.int32)           # normals +y
    sm = scenes.tiny_scene(4, steps=14, obstacle="plane", seed=12, height=0.004, v0_scale=0.1, mu=0.3)
    sm.obstacles = [scenes.mesh_obstacle(V, T, 0.3)]
    a = O.Model(sc)
    b = O.Model(sm)
    ra, rb = O.rollout(a), O.rollout(b)
    assert modes_of(ra) == modes_of(rb) and any(r.contact.nodes.size for r in ra)
    assert np.array_equal(ra[-1].x1, rb[-1].x1)
    _, g = O.centroid_loss(a, ra[-1].x1, sc.target)
    Ga, Gb = O.backward(a, ra, g), O.backward(b, rb, g)
    for u, v in ((Ga.dx0, Gb.dx0), (Ga.dv0, Gb.dv0), (Ga.dw, Gb.dw), (Ga.dmu, Gb.dmu)):
        assert np.array_equal(u, v)


def test_icosphere_distance_brackets_the_sphere():
    # the icosphere is inscribed in its sphere: outside points are at least as
    # far from it as from the sphere, and at most the sagitta farther
    V, T = scenes.icosphere((0.1, -0.2, 0.05), 0.3, 2)
    o = scenes.mesh_obstacle(V, T, 0.5)
    rng = np.random.default_rng(13)
    d = rng.normal(size=(400, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    x = np.asarray((0.1, -0.2, 0.05)) + d * rng.uniform(0.31, 0.6, (400, 1))
    phi, n, reg, _ = O.mesh_query(o, x)
    ps = np.linalg.norm(x - np.asarray((0.1, -0.2, 0.05)), axis=1) - 0.3
    # sagitta: largest distance from the sphere to a face plane inside it
    A, B, C = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    nt = np.cross(B - A, C - A)
    nt /= np.linalg.norm(nt, axis=1)[:, None]
    sag = 0.3 - np.min(np.abs(np.sum(nt * (A - np.asarray((0.1, -0.2, 0.05))), axis=1)))
    assert np.all(phi >= ps - 1e-12) and np.all(phi <= ps + sag + 1e-12)
    assert np.allclose(np.linalg.norm(n, axis=1), 1.0, atol=1e-14)
    assert set(np.unique(reg)) >= {O.FACE}


def test_mesh_obstacle_gradients_match_finite_differences():
    # a coarse icosphere (80 triangles) under a small cloth: contacts on faces,
    # edges and vertices, each with its own frame derivative
    sc = scenes.tiny_scene(3, steps=8, obstacle="sphere", k=50.0, mu=0.4, seed=14, height=0.004,
                           v0_scale=0.05, bend=0.02)
    o = sc.obstacles[0]
    V, T = scenes.icosphere(o.point, o.radius, 1)
    sc.obstacles = [scenes.mesh_obstacle(V, T, o.mu)]
    model, recs, L, g = converged_loss(sc)
    regions = set()
    for r in recs:
        act = r.contact.mode != O.TAKEOFF
        if np.any(act):
            regions |= set(O.mesh_query(sc.obstacles[0], r.x0[r.contact.nodes[act]])[2].tolist())
    assert len(regions) >= 2, regions                 # not only faces
    G = O.backward(model, recs, g)
    base_modes = modes_of(recs)
    rng = np.random.default_rng(15)
    checks = 0

    def fd(eps, **kw):
        _, rp, Lp, _ = converged_loss(sc, **{k: v[0] for k, v in kw.items()})
        _, rm, Lm, _ = converged_loss(sc, **{k: v[1] for k, v in kw.items()})
        if modes_of(rp) != base_modes or modes_of(rm) != base_modes:
            return None
        return (Lp - Lm) / (2 * eps)

    for _ in range(2):
        d = rng.normal(size=sc.X.shape)
        e = 1e-6
        val = fd(e, x0=(sc.X + e * d, sc.X - e * d))
        if val is not None:
            assert abs(val - np.sum(G.dx0 * d)) <= 1e-5 * abs(val) + 1e-12, (val, np.sum(G.dx0 * d))
            checks += 1
    d = rng.normal(size=sc.X.shape)
    val = fd(1e-6, v0=(sc.v0 + 1e-6 * d, sc.v0 - 1e-6 * d))
    if val is not None:
        assert abs(val - np.sum(G.dv0 * d)) <= 1e-5 * abs(val) + 1e-12
        checks += 1
    mu = sc.obstacles[0].mu
    val = fd(1e-5, mu=([mu + 1e-5], [mu - 1e-5]))
    if val is not None:
        assert abs(val - G.dmu[0]) <= 1e-5 * abs(val) + 1e-10, (val, G.dmu[0])
        checks += 1
    assert checks >= 3


# ------------------------------------------------------------------ warm-started contact impulses

def _is_contact_fixed_point(model, rec, n):
    """The recorded (v_{n+1}, impulses) solve the step's equations: the global
    momentum balance P v = b(p(x_n + h v)) + f (eqn pd_velocity_with_contact),
    and at every contact node the Signorini-Coulomb law (eqn contact_all):
    one more contact update from the recorded state changes nothing."""
    h = model.h
    ct = rec.contact
    b0 = O.constant_rhs(model, rec.x0, rec.v0, (n + 1) * h, n)
    p, _ = O.local_projection(model, rec.x1)
    rhs = b0 + h * (model.A.T @ (model.w[:, None] * p))
    np.add.at(rhs, ct.nodes, ct.impulse)
    v = model.solve_P(rhs)
    scale = np.abs(rec.v1).max() + 1e-3
    if np.abs(v - rec.v1).max() > 1e-9 * scale:
        return False
    if ct.nodes.size == 0:
        return True
    ub = v[ct.nodes] - ct.impulse / model.mass[ct.nodes, None]
    vc, f, md = O.signorini_coulomb(ub, ct.normal, ct.gap, ct.mu, h, model.mass[ct.nodes])
    return (np.abs(vc - rec.v1[ct.nodes]).max() <= 1e-9 * scale and np.array_equal(md, ct.mode))


@pytest.mark.parametrize("obst,n,steps,height", [("sphere", 4, 12, 0.004), ("plane", 5, 8, 0.0005)])
def test_warm_start_keeps_the_converged_state(obst, n, steps, height):
    # starting each step's contact iteration from the previous step's impulses
    # changes where the iteration starts, not its fixed point: converged
    # rollouts agree to the tolerance, with the same modes, and every
    # converged step solves the step's equations.  (On the plane the cloth
    # settles with every node in contact; a stopping rule on the velocities
    # alone stops there while the impulses still change -- every velocity is
    # held by the contact update -- and fails the fixed-point check.)
    sc = scenes.tiny_scene(n, steps=steps, obstacle=obst, seed=5, height=height, v0_scale=0.05, k=50.0)
    model = O.Model(sc)
    cold = O.rollout(model, tol=1e-13)
    warm = O.rollout(model, tol=1e-13, warm_start=True)
    assert any(r.contact.nodes.size for r in cold)
    for k, (a, b) in enumerate(zip(cold, warm)):
        assert np.abs(a.x1 - b.x1).max() <= 1e-11
        assert np.array_equal(a.contact.nodes, b.contact.nodes)
        assert np.array_equal(a.contact.mode, b.contact.mode)
        assert _is_contact_fixed_point(model, a, k) and _is_contact_fixed_point(model, b, k)


def test_warm_start_starts_from_the_previous_impulses():
    # one PD iteration per step: with warm start the first global solve of
    # step n already carries step n-1's impulses, so a cloth lying at rest on
    # the ground (every node supporting its own weight, f_j = m_j g h) is
    # exactly still after its first step; from zero impulses the single
    # iteration leaves the free-fall velocity in the global solve
    pts = np.array([[a, 0.0, b] for a in (0.0, 0.2, 0.4) for b in (0.0, 0.2, 0.4)])
    sc = particle_scene(pts, [scenes.Obstacle(scenes.PLANE, (0, 0, 0), (0, 1, 0), 0.0, 0.5)], (0.0, 0.0, 0.0),
                        steps=4)
    sc.edge_stiffness[:] = 100.0                    # springs at rest length
    model = O.Model(sc)
    warm = O.rollout(model, iters=1, warm_start=True)
    for r in warm:
        assert np.all(r.contact.mode == O.STICK)
        mgh = sc.node_mass[:, None] * 9.8 * sc.h
        assert np.allclose(r.contact.impulse, np.array([0.0, 1.0, 0.0]) * mgh, rtol=1e-12, atol=1e-12 * mgh.max())
        assert np.abs(r.v1).max() <= 1e-15
    # the cold iteration's impulse comes from the free velocity of that one
    # solve; the warm one adds the previous impulse on the right-hand side
    # first, so its free velocity u = v - f/m equals the cold one exactly
    cold = O.rollout(model, iters=1)
    for a, b in zip(cold[1:], warm[1:]):
        assert np.allclose(a.contact.ubar, b.contact.ubar, rtol=1e-12, atol=1e-12 * np.abs(a.contact.ubar).max())


# ------------------------------------------------------------------ node-node self-collision

def free_particles(X, v0, mass, d, radius, mu, h=0.01, steps=1):
    """Particles with no springs or bending, node-node contact on."""
    X = np.asarray(X, float)
    return scenes.Scene(
        name="pair", X=X, tris=np.zeros((0, 3), np.int32), edges=np.zeros((0, 2), np.int32),
        edge_stiffness=np.zeros(0), node_mass=np.asarray(mass, float), v0=np.asarray(v0, float), h=h,
        steps=steps, bend_weight=0.0, self_thickness=d, self_radius=radius, self_mu=mu)


def test_two_particle_pair_closed_form():
    # P = M: one global solve is exact, so two PD iterations reach the fixed point
    rows = [ln.split() for ln in open(os.path.join(GOLDEN, "two_particle_pair.txt"))
            if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        mu = float(r[1])
        v0 = np.array(r[2:8], float).reshape(2, 3)
        want = np.array(r[8:14], float).reshape(2, 3)
        sc = free_particles([[0, 0.105, 0], [0, 0, 0]], v0, [1.0, 3.0], 0.1, 0.15, mu)
        rec = O.forward_step(O.Model(sc), sc.X, v0, 0, iters=3)
        assert rec.pairs.i.tolist() == [0] and rec.pairs.j.tolist() == [1], r[0]
        assert int(rec.pairs.mode[0]) == int(r[14]), r[0]
        assert np.allclose(rec.v1, want, rtol=0, atol=1e-12), (r[0], rec.v1, want)


def test_pairs_are_mutual_nearest_outside_stencils_and_obstacle_contacts():
    # brute force over a tiny configuration: three particles on a line (B is
    # nearest to both A and C, A-B the closer pair), a fourth one far away, and
    # a cloth whose own nodes are close but share stencils
    sc = free_particles([[0, 0, 0], [0.03, 0, 0], [0.07, 0, 0], [1, 0, 0]], np.zeros((4, 3)),
                        [1.0, 1.0, 1.0, 1.0], 0.05, 0.08, 0.3)
    rec = O.forward_step(O.Model(sc), sc.X, sc.v0, 0, iters=2)
    assert list(zip(rec.pairs.i.tolist(), rec.pairs.j.tolist())) == [(0, 1)]
    for kw in (dict(), dict(pinned=False, shift=0.0), dict(ground=True)):
        sc = scenes.stacked_sheets(n=4, **kw)
        model = O.Model(sc)
        x, v = sc.X, sc.v0
        for n in range(3):
            rec = O.forward_step(model, x, v, n)
            y = O.inertial_predictor(model, x, v, n)
            busy = set(rec.contact.nodes.tolist())
            shared = model.shares_stencil()
            m = model.m
            nearest = []
            for i in range(m):
                best, bj = None, -1
                for j in range(m):
                    if j == i or i in busy or j in busy or shared[i, j] or np.all(x[i] == x[j]):
                        continue
                    dd = sum((y[i, c] - y[j, c]) ** 2 for c in range(3))
                    if dd <= model.self_r ** 2 and (best is None or dd < best):
                        best, bj = dd, j
                nearest.append(bj)
            want = [(i, nearest[i]) for i in range(m) if nearest[i] > i and nearest[nearest[i]] == i]
            assert list(zip(rec.pairs.i.tolist(), rec.pairs.j.tolist())) == want, (kw, n)
            if kw.get("ground") and n > 0:
                assert rec.contact.nodes.size > 0
            x, v = rec.x1, rec.v1


def test_pair_impulses_conserve_momentum_and_hold_the_thickness():
    # free sheets (no pins, no obstacle contact): springs and pair impulses are
    # internal, so total momentum changes by h sum m g per step; a pair in stick
    # or slip ends each converged step at normal separation d
    sc = scenes.stacked_sheets(n=4, steps=6, pinned=False)
    model = O.Model(sc)
    recs = O.rollout(model, tol=1e-12, max_iters=50000)
    modes = np.concatenate([r.pairs.mode for r in recs])
    assert {1, 2, 3} <= set(modes.tolist())                    # take-off, stick and slip all occur
    M = model.mass[:, None]
    dp_want = model.h * np.sum(model.mass) * np.asarray(model.g)
    for r in recs:
        dp = np.sum(M * r.v1, axis=0) - np.sum(M * r.v0, axis=0)
        assert np.allclose(dp, dp_want, rtol=0, atol=1e-12 * np.sum(M)), (dp, dp_want)
        ps = r.pairs
        act = ps.mode != O.TAKEOFF
        sep = np.sum(ps.normal * (r.x1[ps.i] - r.x1[ps.j]), axis=1)
        assert np.allclose(sep[act], model.self_d, rtol=0, atol=1e-12)
        assert np.all(sep[~act] >= model.self_d - 1e-12)


def test_self_collision_off_changes_nothing():
    sc = scenes.stacked_sheets(n=4, steps=3)
    on = O.rollout(O.Model(sc))
    sc.self_thickness = 0.0
    off = O.rollout(O.Model(sc))
    assert sum(r.pairs.i.size for r in on) > 0 and sum(r.pairs.i.size for r in off) == 0
    sc2 = scenes.tiny_scene(3, steps=4, obstacle="plane", height=0.005)
    a = O.rollout(O.Model(sc2))
    assert all(r.pairs.i.size == 0 for r in a)


def test_self_adjoint_fixed_point_equals_direct_solve():
    sc = scenes.stacked_sheets(n=4, steps=4, pinned=False)
    model = O.Model(sc)
    recs = O.rollout(model, tol=1e-12, max_iters=50000)
    rng = np.random.default_rng(3)
    for n in range(len(recs)):
        assert recs[n].pairs.i.size > 0
        gx, gv = rng.normal(size=(2, model.m, 3))
        d = O.backward_step(model, recs[n], gx, gv, n, direct=True)
        it = O.backward_step(model, recs[n], gx, gv, n, direct=False, iter_tol=1e-14)
        for a, b in zip(d[:4], it[:4]):
            assert np.allclose(a, b, rtol=1e-8, atol=1e-10 * max(1.0, np.abs(a).max()))


def self_modes_of(recs):
    return [tuple(r.pairs.i.tolist()) + tuple(r.pairs.j.tolist()) + tuple(r.pairs.mode.tolist())
            + tuple(r.contact.nodes.tolist()) + tuple(r.contact.mode.tolist()) for r in recs]


@pytest.mark.parametrize("seed", [0, 1])
def test_self_collision_gradients_match_central_finite_differences(seed):
    # the top sheet lands on the pinned one: pairs in slip, then stick; steps
    # of 1e-7 keep the central differences clear of the nearest mode boundary
    sc = scenes.stacked_sheets(n=3, steps=4, k=50.0, seed=seed)
    model, recs, L, g = converged_loss(sc, tol=1e-13)
    assert sum(int(np.sum(r.pairs.mode != O.TAKEOFF)) for r in recs) > 0
    G = O.backward(model, recs, g)
    base = self_modes_of(recs)
    rng = np.random.default_rng(5)

    def fd(eps, **kw):
        _, rp, Lp, _ = converged_loss(sc, tol=1e-13, **{k: v[0] for k, v in kw.items()})
        _, rm, Lm, _ = converged_loss(sc, tol=1e-13, **{k: v[1] for k, v in kw.items()})
        assert self_modes_of(rp) == base and self_modes_of(rm) == base
        return (Lp - Lm) / (2 * eps)

    e = 1e-7
    d = rng.normal(size=sc.X.shape)
    val = fd(e, x0=(sc.X + e * d, sc.X - e * d))
    assert abs(val - np.sum(G.dx0 * d)) <= 1e-5 * abs(val) + 1e-12, (val, np.sum(G.dx0 * d))
    d = rng.normal(size=sc.X.shape)
    val = fd(e, v0=(sc.v0 + e * d, sc.v0 - e * d))
    assert abs(val - np.sum(G.dv0 * d)) <= 1e-5 * abs(val) + 1e-12, (val, np.sum(G.dv0 * d))
    k = sc.edge_stiffness
    d = rng.normal(size=k.shape) * k
    e = 1e-4
    val = fd(e, edge_stiffness=(k + e * d, k - e * d))
    ad = np.sum(G.dw[:model.n_spring] * d)
    assert abs(val - ad) <= 1e-4 * abs(val) + 1e-14, (val, ad)
    e = 1e-6
    mu = sc.self_mu
    val = fd(e, self_mu=(mu + e, mu - e))
    assert abs(val - G.dmu[-1]) <= 1e-5 * abs(val) + 1e-10, (val, G.dmu[-1])
