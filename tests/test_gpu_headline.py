"""The benchmark's own configurations against the FP64 oracle.

Sphere drop 40 x 40 (4800 DoF), 200 steps, mixed precision, direct adjoint:
the kernel instantiation the benchmark times (float32 local step, float64
solves and contact).  Every step is redone by the oracle from the GPU's
recorded state, so the comparison measures one step's arithmetic and not the
divergence of two rollouts:

* positions within 1e-6 m (the float32 projection p = L0 q/|q| rounds at
  6e-8 relative, 1.5e-9 m on a 2.6 cm spring; through h w ~ 40 N/m per spring
  and P ~ 1 kg/s that is ~1e-8 m per PD iteration, measured 3e-8 m per step);
* contact modes identical except near ties, which are reported: a node whose
  FP64 decision margin (|phi(y)| for detection, |a| for take-off,
  |tau - mu(-a)| for stick / slip) is within 1e-6 m/s of zero in the
  oracle's own state may decide either way under a 1e-7 m/s velocity change;
* the adjoint step (sim_adjoint_step) against the oracle's direct solve at
  the GPU's recorded state, sampled steps: relative error within
  100 eps32 kappa_1(A), with A = M + H T^T and kappa_1 estimated from the
  oracle's factor (float32 rounding of the projection Jacobians and of K_s
  in the operator, 6e-8 relative per entry, amplified by the condition).

A batch with a 48 x 48 member (whose vectors do not all fit in LDS) and a
served request are compared with the oracle in float64.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import scenes
from oracle import diffcloth_oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
EPS32 = 2.0 ** -24


def _rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def _modes(model, rec):
    md = np.zeros(model.m, np.uint8)
    md[rec.contact.nodes] = rec.contact.mode
    return md


def _margins(model, rec, x0, v0, n):
    """Per node the oracle's smallest FP64 decision margin at step n (inf off contact)."""
    h = model.h
    y = O.inertial_predictor(model, x0, v0, n)
    phis = np.stack([model.signed_distance(o, y) for o in model.obstacles], axis=1)
    marg = np.abs(phis.min(axis=1)) / h                 # detection, in velocity units
    ct = rec.contact
    if ct.nodes.size:
        un = np.sum(ct.normal * ct.ubar, axis=1)
        a = un + ct.gap / h
        tau = np.linalg.norm(ct.ubar - un[:, None] * ct.normal, axis=1)
        marg[ct.nodes] = np.minimum(marg[ct.nodes], np.minimum(np.abs(a), np.abs(tau - ct.mu * (-a))))
    return marg


def _kappa1(model, rec):
    """kappa_1 of the step's adjoint matrix M + H T^T, estimated (Hager / Higham)."""
    h = model.h
    m = model.m
    Hm = (O._kron3(h * h * model.K_s) - O.delta_P(model, rec.x1)).tocsr()
    Tb = np.tile(np.eye(3), (m, 1, 1))
    if rec.contact.nodes.size:
        Tb[rec.contact.nodes] = O.contact_jacobian_blocks(rec.contact, h)
    A = (sp.diags(np.repeat(model.mass, 3)) + Hm @ O._blockdiag3(np.transpose(Tb, (0, 2, 1)))).tocsc()
    lu = spla.splu(A)
    inv = spla.LinearOperator(A.shape, matvec=lu.solve, rmatvec=lambda b: lu.solve(b, trans="T"))
    return spla.norm(A, 1) * spla.onenormest(inv)


def test_headline_mixed_40x40_every_step_from_gpu_state():
    from paper_2106_05306_amd.sim import Sim
    sc = scenes.c2_sphere_drop(0)
    model = O.Model(sc)
    # the benchmark's solver settings (its refinement stops at a backward error of 1e-4)
    sim = Sim.from_scene(sc, device=DEV, precision="mixed", adj_solver="direct", adj_tol=1e-4, adj_max_iters=10)
    st = sim.stats()
    # the benchmark's instantiation: the multi-workgroup forward, the adjoint's LDS placement
    assert st["fwd_workgroups"] > 1 and st["lds_flags_bwd"] == 1
    sim.forward(sc.steps)
    xs, vs = zip(*[sim.state(n) for n in range(sc.steps + 1)])
    xs = [x.cpu().numpy() for x in xs]
    vs = [v.cpu().numpy() for v in vs]
    worst, ties, mism = 0.0, 0, 0
    recs = []
    for n in range(sc.steps):
        rec = O.forward_step(model, xs[n], vs[n], n)
        recs.append(rec)
        worst = max(worst, np.abs(xs[n + 1] - rec.x1).max())
        md_g, md_o = sim.modes(n), _modes(model, rec)
        marg = _margins(model, rec, xs[n], vs[n], n)
        bad = np.nonzero(md_g != md_o)[0]
        mism += bad.size
        assert np.all(marg[bad] <= 1e-6), (n, bad[marg[bad] > 1e-6], marg[bad])
        ties += int(np.sum(marg <= 1e-6))
    print(f"headline 40x40 mixed: max one-step position error {worst:.2e} m, "
          f"{mism} mode mismatches among {ties} near-tie node-steps", flush=True)
    assert worst <= 1e-6
    rng = np.random.default_rng(0)
    for n in (5, 31, 34, 40, 60, 100, 150, 199):
        rec = recs[n]
        at_gpu = O.StepRecord(xs[n], vs[n], xs[n + 1], vs[n + 1], rec.contact, rec.iters)
        gx, gv = rng.normal(size=(2, sc.n_nodes, 3))
        out = sim.adjoint_step(n, torch.tensor(gx, device=DEV), torch.tensor(gv, device=DEV))
        assert out["status"] >= 0, (n, out["status"])
        dx, dv, dw, dmu, _ = O.backward_step(model, at_gpu, gx, gv, n)
        kappa = _kappa1(model, at_gpu)
        e = max(_rel(out["dx0"].cpu().numpy(), dx), _rel(out["dv0"].cpu().numpy(), dv))
        bound = 100 * EPS32 * kappa
        print(f"step {n}: adjoint rel err {e:.2e}, kappa_1 {kappa:.2e}, bound {bound:.2e}", flush=True)
        assert e <= bound, (n, e, bound)


def test_batch_with_a_48x48_member_matches_oracle():
    from paper_2106_05306_amd.sim import Sim, batch_backward, batch_forward
    rng = np.random.default_rng(4)
    batch = [scenes.mixed_grid(rng, 48, 10, 2.0e3, 0.4, True), scenes.mixed_grid(rng, 16, 10, 8.0e2, 0.7, False),
             scenes.mixed_grid(rng, 23, 10, 1.5e3, 0.3, True)]
    for sc in batch:                        # released 1 cm above the obstacle: contact within the 10 steps
        sc.X = sc.X - np.array([0.0, 0.29 if sc.obstacles[0].kind == scenes.SPHERE else 0.19, 0.0])
    sims = [Sim.from_scene(sc, device=DEV, precision="fp64", adj_solver="direct", adj_tol=1e-12, adj_max_iters=10)
            for sc in batch]
    assert sims[0].stats()["lds_flags_fwd"] != 7                    # the large member does not fit whole
    seeds = [np.random.default_rng(9 + i).normal(size=(sc.n_nodes, 3)) for i, sc in enumerate(batch)]
    outs = batch_forward(sims, [sc.steps for sc in batch])
    grads = batch_backward(sims, [torch.tensor(g, device=DEV) for g in seeds])
    for sc, s, (xT, _), g, seed in zip(batch, sims, outs, grads, seeds):
        model = O.Model(sc)
        recs = O.rollout(model)
        assert np.abs(xT.cpu().numpy() - recs[-1].x1).max() <= 1e-9
        for n, r in enumerate(recs):
            assert np.array_equal(s.modes(n), _modes(model, r)), (sc.name, n)
        assert sum(r.contact.nodes.size for r in recs) > 0
        G = O.backward(model, recs, seed)
        for key, ref in (("dx0", G.dx0), ("dv0", G.dv0), ("dw_edge", G.dw[:model.n_spring]), ("dmu", G.dmu)):
            assert _rel(g[key].cpu().numpy(), ref) <= 1e-6, (sc.name, key, _rel(g[key].cpu().numpy(), ref))


def test_served_requests_match_oracle():
    # requests served by continuous batching next to each other (chunks of a
    # few steps joining and leaving the launches) give the oracle's gradients
    # (float64), including a request whose cached handle last served another
    # material of the same topology
    from paper_2106_05306_amd.serve import Request, Server

    def make(rid, n, steps, sphere, k=1.0e3, mu=0.5):
        def f():
            sc = scenes.request_scene(n, steps, sphere, seed=rid)
            sc.X = sc.X - np.array([0.0, 0.29 if sphere else 0.19, 0.0])   # contact within the first steps
            sc.edge_stiffness = np.full_like(sc.edge_stiffness, k)
            for o in sc.obstacles:
                o.mu = mu
            return sc
        return f
    spec = [(14, 12, True, 1.0e3, 0.5), (9, 16, False, 1.0e3, 0.5), (12, 10, True, 1.0e3, 0.5),
            (14, 9, True, 2.5e3, 0.3)]
    reqs = [Request(rid, (n, sphere), steps, 0.01 * rid, make(rid, n, steps, sphere, k, mu))
            for rid, (n, steps, sphere, k, mu) in enumerate(spec)]
    srv = Server(DEV, keep_grads=True, round_ms=0.5, max_chunk=4, precision="fp64", adj_solver="direct",
                 adj_tol=1e-12, adj_max_iters=10)
    res = {r.rid: r for r in srv.run(reqs)}
    res2 = {r.rid: r for r in srv.run(list(reversed(reqs)))}    # second pass from the handle cache
    assert srv.stats["cache_hits"] >= len(spec)
    for rid, req in enumerate(reqs):
        sc = req.make_scene()
        model = O.Model(sc)
        recs = O.rollout(model)
        L, g = O.centroid_loss(model, recs[-1].x1, sc.target)
        assert sum(r.contact.nodes.size for r in recs) > 0
        G = O.backward(model, recs, g)
        for r in (res[rid], res2[rid]):
            assert r.status == 0, (rid, r.status)
            for key, ref in (("dx0", G.dx0), ("dv0", G.dv0), ("dw_edge", G.dw[:model.n_spring]), ("dmu", G.dmu)):
                assert _rel(r.grads[key].cpu().numpy(), ref) <= 1e-6, (rid, key)
    srv.close()
