"""GPU (gfx950) parity of the HIP path against the FP64 oracle, through the C ABI.

Tolerances: positions max |x_gpu - x_oracle| <= 1e-6 m (cloths are ~1 m)
in float64 mode, contact modes identical at every step, gradients
|g_gpu - g_oracle|_2 <= 1e-4 |g_oracle|_2 per parameter group.  The oracle
solves each adjoint directly; the GPU iterates (the paper's fixed point), so
its tolerance is set tight (1e-12) for parity runs.
"""
import numpy as np
import pytest

import scenes
from oracle import diffcloth_oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _sim(sc, **kw):
    from paper_2106_05306_amd.sim import Sim
    kw.setdefault("adj_tol", 1e-12)
    kw.setdefault("adj_max_iters", 3000)
    return Sim.from_scene(sc, device=DEV, **kw)


def _oracle(sc, tol=None, **mkw):
    model = O.Model(sc, **mkw)
    recs = O.rollout(model, tol=tol)
    traj = np.stack([recs[0].x0] + [r.x1 for r in recs])
    return model, recs, traj


def _modes(model, rec):
    md = np.zeros(model.m, np.uint8)
    md[rec.contact.nodes] = rec.contact.mode
    return md


def _rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def _check_forward(sim, model, recs, traj, tol=1e-6):
    _, _, tg = sim.forward(len(recs), trajectory=True)
    err = np.abs(tg.cpu().numpy() - traj).max()
    assert err <= tol, f"positions differ by {err}"
    for n, r in enumerate(recs):
        assert np.array_equal(sim.modes(n), _modes(model, r)), f"modes differ at step {n}"
    return err


def _check_grads(sim, model, recs, tol=1e-4, seed_gv=False):
    L, g = O.centroid_loss(model, recs[-1].x1, model.scene.target)
    c = np.random.default_rng(7).normal(size=g.shape)
    g = g + c                                         # deformation-sensitive seed
    gv = np.random.default_rng(8).normal(size=g.shape) if seed_gv else None
    G = O.backward(model, recs, g, dL_dvT=gv)
    out = sim.backward(torch.tensor(g, device=DEV), None if gv is None else torch.tensor(gv, device=DEV))
    assert out["status"] >= 0
    errs = {"dx0": _rel(out["dx0"].cpu().numpy(), G.dx0), "dv0": _rel(out["dv0"].cpu().numpy(), G.dv0),
            "dw_edge": _rel(out["dw_edge"].cpu().numpy(), G.dw[:model.n_spring])}
    if model.n_bend:
        dwb = np.zeros(model.m)
        dwb[model.bend_centers] = G.dw[model.n_spring:]
        errs["dw_bend"] = _rel(out["dw_bend"].cpu().numpy(), dwb)
    if model.obstacles:
        errs["dmu"] = _rel(out["dmu"].cpu().numpy(), G.dmu)
    for k, e in errs.items():
        assert e <= tol, f"{k} differs by {e}"
    return errs, out, G


def test_napkin_forward_and_gradients_fp64():
    sc = scenes.c1_napkin(0)
    model, recs, traj = _oracle(sc)
    sim = _sim(sc, precision="fp64")
    err = _check_forward(sim, model, recs, traj)
    errs, _, _ = _check_grads(sim, model, recs)
    print("napkin fp64: pos err", err, "grad errs", errs)


@pytest.mark.parametrize("obst,pins,seed", [("plane", False, 1), ("sphere", False, 2), (None, True, 3),
                                            ("plane", True, 4)])
def test_tiny_scenes_fp64(obst, pins, seed):
    sc = scenes.tiny_scene(5, steps=15, obstacle=obst, pins=pins, seed=seed, height=0.01, v0_scale=0.1, k=200.0)
    model, recs, traj = _oracle(sc)
    sim = _sim(sc, precision="fp64")
    _check_forward(sim, model, recs, traj, tol=1e-9)
    _check_grads(sim, model, recs, tol=1e-6, seed_gv=True)


def test_converge_mode_matches_oracle():
    sc = scenes.tiny_scene(4, steps=6, obstacle="sphere", seed=5, height=0.004, v0_scale=0.05, k=50.0)
    model, recs, traj = _oracle(sc, tol=1e-12)
    sim = _sim(sc, precision="fp64", fwd_tol=1e-12, fwd_max_iters=100000)
    _check_forward(sim, model, recs, traj, tol=1e-9)
    _check_grads(sim, model, recs, tol=1e-6)


def test_skirt_region_gradients():
    sc = scenes.c3_skirt(0, n_around=12, n_rings=14, steps=10)
    model, recs, traj = _oracle(sc)
    sim = _sim(sc, precision="fp64")
    _check_forward(sim, model, recs, traj, tol=1e-8)
    ang, g = O.apex_angle_loss(recs[-1].x1, sc.waist_nodes, sc.hem_nodes)
    G = O.backward(model, recs, g)
    out = sim.backward(torch.tensor(g, device=DEV))
    assert _rel(out["dregion"].cpu().numpy(), G.dregion) <= 1e-6
    assert _rel(out["dx0"].cpu().numpy(), G.dx0) <= 1e-6


def test_mixed_precision_error_is_small():
    # every step of the mixed-precision rollout redone by the FP64 oracle from
    # the GPU's recorded state (whole 20-iteration rollouts drift apart): the
    # float32 projection rounds at 6e-8 relative (1.5e-9 m on a 2.6 cm spring
    # of the napkin's 11 cm ones: 7e-9 m), amplified by h w / P per PD
    # iteration, ~1e-8 m per step; the bound is 1e-6 m as on the 40 x 40 headline
    sc = scenes.c1_napkin(0)
    model = O.Model(sc)
    sim = _sim(sc, precision="mixed")
    _, _, tg = sim.forward(sc.steps, trajectory=True)
    xs = tg.cpu().numpy()
    vs = [sim.state(n)[1].cpu().numpy() for n in range(sc.steps)]
    worst = 0.0
    for n in range(sc.steps):
        rec = O.forward_step(model, xs[n], vs[n], n)
        worst = max(worst, np.abs(rec.x1 - xs[n + 1]).max())
    print("napkin mixed precision: max one-step position error vs FP64 oracle", worst)
    assert worst <= 1e-6


def test_checkpointing_is_bitwise_identical():
    sc = scenes.c1_napkin(0, steps=30)
    g = torch.randn(sc.n_nodes, 3, dtype=torch.float64, generator=torch.Generator().manual_seed(3)).to(DEV)
    outs = []
    for k in (0, 7):
        sim = _sim(sc, precision="fp64", checkpoint_every=k, adj_tol=1e-10, adj_max_iters=300)
        xT, vT, _ = sim.forward(sc.steps)
        outs.append((xT, sim.backward(g)))
    assert torch.equal(outs[0][0], outs[1][0])
    for key in ("dx0", "dv0", "dw_edge", "dmu"):
        assert torch.equal(outs[0][1][key], outs[1][1][key]), key


def test_rerun_is_deterministic():
    sc = scenes.c2_sphere_drop(0, n=20, steps=40)
    sim = _sim(sc, precision="mixed", adj_tol=1e-8, adj_max_iters=300)
    g = torch.ones(sc.n_nodes, 3, dtype=torch.float64, device=DEV)
    a = sim.forward(sc.steps)[0].clone()
    ga = sim.backward(g)
    b = sim.forward(sc.steps)[0].clone()
    gb = sim.backward(g)
    assert torch.equal(a, b)
    for key in ("dx0", "dv0", "dw_edge", "dmu"):
        assert torch.equal(ga[key], gb[key]), key


def test_batch_matches_single_launches():
    from paper_2106_05306_amd.sim import batch_backward, batch_forward
    batch = scenes.c4_batch(seed=1, count=4, steps=12, n_lo=6, n_hi=14)
    singles, sims = [], []
    for sc in batch:
        s = _sim(sc, precision="fp64", adj_tol=1e-10, adj_max_iters=300)
        xT, vT, _ = s.forward(sc.steps)
        gseed = torch.ones(sc.n_nodes, 3, dtype=torch.float64, device=DEV)
        singles.append((xT.clone(), s.backward(gseed)))
        sims.append(_sim(sc, precision="fp64", adj_tol=1e-10, adj_max_iters=300))
    outs = batch_forward(sims, [sc.steps for sc in batch])
    grads = batch_backward(sims, [torch.ones(sc.n_nodes, 3, dtype=torch.float64, device=DEV) for sc in batch])
    for (xT, g1), (xb, _), g2 in zip(singles, outs, grads):
        assert torch.equal(xT, xb)
        for key in ("dx0", "dv0", "dw_edge", "dmu"):
            assert torch.equal(g1[key], g2[key]), key


def test_sphere_drop_forward_fp64_first_steps():
    sc = scenes.c2_sphere_drop(0, steps=60)
    model, recs, traj = _oracle(sc)
    sim = _sim(sc, precision="fp64")
    err = _check_forward(sim, model, recs, traj)
    print("sphere drop 40x40, 60 steps fp64: pos err", err)


def test_sphere_drop_adjoint_steps_from_gpu_state():
    # The per-step adjoint map is linear in its seeds.  The oracle steps from
    # the GPU's recorded state (so both linearise at the same point) and the
    # two adjoints are compared on random seeds.  Steps whose adjoint system
    # the GPU solver reports as not converged (near-singular systems of the
    # 20-iteration forward) are checked with the direct solve on a second
    # handle with the same recorded rollout (its forward is bitwise the same).
    sc = scenes.c2_sphere_drop(0, steps=200)
    model = O.Model(sc)
    sim = _sim(sc, precision="fp64", adj_max_iters=6000)
    sim.forward(sc.steps)
    simd = _sim(sc, precision="fp64", adj_solver="direct", adj_tol=1e-12, adj_max_iters=10)
    simd.forward(sc.steps)
    direct_checked = 0
    rng = np.random.default_rng(0)
    checked = 0
    for n in (5, 20, 28, 31, 35, 60, 120, 199):
        x, v = sim.state(n)
        rec = O.forward_step(model, x.cpu().numpy(), v.cpu().numpy(), n)
        x1, _ = sim.state(n + 1)
        assert np.abs(x1.cpu().numpy() - rec.x1).max() <= 1e-9, n
        assert np.array_equal(sim.modes(n), _modes(model, rec)), n
        gx, gv = rng.normal(size=(2, sc.n_nodes, 3))
        out = sim.adjoint_step(n, torch.tensor(gx, device=DEV), torch.tensor(gv, device=DEV))
        if out["status"] == 2:                           # SIM_WADJ_NOCONV: the direct solve instead
            print(f"step {n}: iterative adjoint did not converge, checked with the direct solve", flush=True)
            out = simd.adjoint_step(n, torch.tensor(gx, device=DEV), torch.tensor(gv, device=DEV))
            assert out["status"] in (0, 1), (n, out["status"])
            direct_checked += 1
        dx, dv, dw, dmu, _ = O.backward_step(model, rec, gx, gv, n)
        print(f"step {n}: adjoint rel err {_rel(out['dx0'].cpu().numpy(), dx):.2e}", flush=True)
        assert _rel(out["dx0"].cpu().numpy(), dx) <= 1e-6, n
        assert _rel(out["dv0"].cpu().numpy(), dv) <= 1e-6, n
        # springs at rest length (free fall) give weight gradients at rounding level: absolute floor
        ddw = np.linalg.norm(out["dw_edge"].cpu().numpy() - dw[:model.n_spring])
        assert ddw <= 1e-5 * np.linalg.norm(dw[:model.n_spring]) + 1e-12, n
        checked += 1
    assert checked == 8
    print(f"{8 - direct_checked} steps by the iterative solve, {direct_checked} by the direct solve", flush=True)


# ------------------------------------------------------------------ direct adjoint (per-step factorisation)

def test_direct_adjoint_napkin_fp64():
    sc = scenes.c1_napkin(0)
    model, recs, traj = _oracle(sc)
    sim = _sim(sc, precision="fp64", adj_solver="direct")
    _check_forward(sim, model, recs, traj)
    errs, out, _ = _check_grads(sim, model, recs, tol=1e-6)
    assert out["status"] == 0
    print("napkin direct adjoint: grad errs", errs, "solves", sim.stats()["adj_iters_total"])


@pytest.mark.parametrize("obst,pins,seed", [("plane", False, 1), ("sphere", False, 2), (None, True, 3)])
def test_direct_adjoint_tiny_scenes(obst, pins, seed):
    sc = scenes.tiny_scene(5, steps=15, obstacle=obst, pins=pins, seed=seed, height=0.01, v0_scale=0.1, k=200.0)
    model, recs, traj = _oracle(sc)
    sim = _sim(sc, precision="fp64", adj_solver="direct")
    _check_forward(sim, model, recs, traj, tol=1e-9)
    _check_grads(sim, model, recs, tol=1e-8, seed_gv=True)


def test_direct_adjoint_skirt_regions_with_checkpoints():
    sc = scenes.c3_skirt(0, n_around=12, n_rings=14, steps=10)
    model, recs, traj = _oracle(sc)
    sim = _sim(sc, precision="fp64", adj_solver="direct", checkpoint_every=4)
    sim.forward(sc.steps)
    ang, g = O.apex_angle_loss(recs[-1].x1, sc.waist_nodes, sc.hem_nodes)
    G = O.backward(model, recs, g)
    out = sim.backward(torch.tensor(g, device=DEV))
    assert _rel(out["dregion"].cpu().numpy(), G.dregion) <= 1e-6
    assert _rel(out["dx0"].cpu().numpy(), G.dx0) <= 1e-6


def test_direct_adjoint_sphere_drop_every_step_converges():
    # at 40x40 the iterative adjoint misses its tolerance on most steps; the
    # direct solve matches the oracle's direct solve on every sampled step
    sc = scenes.c2_sphere_drop(0, steps=200)
    model = O.Model(sc)
    sim = _sim(sc, precision="fp64", adj_solver="direct", adj_max_iters=10)
    sim.forward(sc.steps)
    rng = np.random.default_rng(0)
    for n in (5, 28, 35, 60, 120, 199):
        x, v = sim.state(n)
        rec = O.forward_step(model, x.cpu().numpy(), v.cpu().numpy(), n)
        gx, gv = rng.normal(size=(2, sc.n_nodes, 3))
        out = sim.adjoint_step(n, torch.tensor(gx, device=DEV), torch.tensor(gv, device=DEV))
        assert out["status"] == 0, n
        dx, dv, dw, dmu, _ = O.backward_step(model, rec, gx, gv, n)
        e = (_rel(out["dx0"].cpu().numpy(), dx), _rel(out["dv0"].cpu().numpy(), dv))
        print(f"step {n}: direct adjoint rel err dx {e[0]:.2e} dv {e[1]:.2e}", flush=True)
        assert max(e) <= 1e-6, n
        ddw = np.linalg.norm(out["dw_edge"].cpu().numpy() - dw[:model.n_spring])
        assert ddw <= 1e-5 * np.linalg.norm(dw[:model.n_spring]) + 1e-12, n


def test_direct_adjoint_batch_and_checkpoint_are_bitwise():
    from paper_2106_05306_amd.sim import batch_backward, batch_forward
    batch = scenes.c4_batch(seed=2, count=3, steps=10, n_lo=6, n_hi=12)
    singles, sims = [], []
    for sc in batch:
        s = _sim(sc, precision="fp64", adj_solver="direct", adj_tol=1e-10, adj_max_iters=10)
        s.forward(sc.steps)
        gseed = torch.ones(sc.n_nodes, 3, dtype=torch.float64, device=DEV)
        singles.append(s.backward(gseed))
        c = _sim(sc, precision="fp64", adj_solver="direct", adj_tol=1e-10, adj_max_iters=10, checkpoint_every=3)
        c.forward(sc.steps)
        gc = c.backward(gseed)
        w = _sim(sc, precision="fp64", adj_solver="direct", adj_tol=1e-10, adj_max_iters=10, adj_window=4)
        w.forward(sc.steps)
        gw = w.backward(gseed)
        w.trim()                                    # records released: a new rollout works as before
        w.forward(sc.steps)
        gw2 = w.backward(gseed)
        for key in ("dx0", "dv0", "dw_edge", "dmu"):
            assert torch.equal(singles[-1][key], gc[key]), key
            assert torch.equal(singles[-1][key], gw[key]), key
            assert torch.equal(singles[-1][key], gw2[key]), key
        sims.append(_sim(sc, precision="fp64", adj_solver="direct", adj_tol=1e-10, adj_max_iters=10))
    batch_forward(sims, [sc.steps for sc in batch])
    grads = batch_backward(sims, [torch.ones(sc.n_nodes, 3, dtype=torch.float64, device=DEV) for sc in batch])
    for g1, g2 in zip(singles, grads):
        for key in ("dx0", "dv0", "dw_edge", "dmu"):
            assert torch.equal(g1[key], g2[key]), key


def test_direct_adjoint_factorisation_overlap_is_bitwise(monkeypatch):
    # the step factorisations run on a second stream while the forward pass is
    # still running (chunked forward launches); results equal the serial path
    sc = scenes.c1_napkin(0)
    sc.steps = 40
    gseed = torch.ones(sc.n_nodes, 3, dtype=torch.float64, device=DEV)
    res = {}
    for overlap in ("0", "1"):
        monkeypatch.setenv("DIFFCLOTH_FACTOR_OVERLAP", overlap)
        s = _sim(sc, precision="fp64", adj_solver="direct", adj_tol=1e-10, adj_max_iters=10)
        xT, vT, _ = s.forward(sc.steps)
        assert s.stats()["fwd_launches"] == (1 if overlap == "0" else 4)   # chunks end at 20, 30, 35, 40
        g1 = s.backward(gseed)
        g2 = s.backward(2.0 * gseed)              # the factors are reused
        s.set_state(None, None)
        s.forward(sc.steps)                        # a second rollout refactors
        g3 = s.backward(gseed)
        n = 17
        a = s.adjoint_step(n, gseed, gseed)        # replaces slot 0 with step n's factor
        g4 = s.backward(gseed)                     # and the full backward factors again
        res[overlap] = (xT, vT, g1, g2, g3, a, g4)
        s.close()
    r0, r1 = res["0"], res["1"]
    assert torch.equal(r0[0], r1[0]) and torch.equal(r0[1], r1[1])
    for k in range(2, 7):
        for key in ("dx0", "dv0", "dw_edge", "dmu"):
            assert torch.equal(r0[k][key], r1[k][key]), (k, key)
    for key in ("dx0", "dv0"):                     # linear in the seed
        assert torch.allclose(r1[2][key] * 2.0, r1[3][key], rtol=1e-12, atol=0.0), key


def test_direct_adjoint_prefetch_workgroups_change_nothing(monkeypatch):
    # the prefetch workgroups of a single-handle adjoint launch only read; the
    # gradients with and without them are identical
    sc = scenes.c2_sphere_drop(0, n=24, steps=30)
    gseed = torch.ones(sc.n_nodes, 3, dtype=torch.float64, device=DEV)
    s = _sim(sc, precision="mixed", adj_solver="direct", adj_tol=1e-8, adj_max_iters=10)
    s.forward(sc.steps)
    out = {}
    for h in ("0", "4", "7"):
        monkeypatch.setenv("DIFFCLOTH_ADJ_HELPERS", h)
        out[h] = s.backward(gseed)
    for key in ("dx0", "dv0", "dw_edge", "dmu"):
        assert torch.equal(out["0"][key], out["4"][key]), key
        assert torch.equal(out["0"][key], out["7"][key]), key


def test_forward_prefetch_workgroups_change_nothing(monkeypatch):
    # forward prefetch workgroups (forced on a small mesh, alone and in a
    # batched launch) only read: the trajectories are identical
    from paper_2106_05306_amd.sim import batch_forward
    sc = scenes.c2_sphere_drop(0, n=16, steps=12)
    outs = {}
    for h in ("0", "3"):
        monkeypatch.setenv("DIFFCLOTH_FWD_HELPERS", h)
        s = _sim(sc, precision="mixed", adj_solver="direct")
        _, _, traj = s.forward(sc.steps, trajectory=True)
        b = [_sim(c, precision="mixed", adj_solver="direct") for c in scenes.c4_batch(seed=1, count=3, steps=8, n_lo=6, n_hi=12)]
        batch_forward(b, [8, 8, 8])
        outs[h] = (traj, [bb.state(8)[0] for bb in b])
    assert torch.equal(outs["0"][0], outs["3"][0])
    for x0, x3 in zip(outs["0"][1], outs["3"][1]):
        assert torch.equal(x0, x3)
