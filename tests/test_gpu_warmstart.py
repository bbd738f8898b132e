"""Warm-started contact impulses and the converged forward on the GPU, against the oracle.

* warm start at a fixed iteration count: positions, contact modes and
  gradients as the oracle's warm-started rollout (float64: positions 1e-9 m,
  gradients 1e-6 relative per group);
* the tolerance-terminated forward (iterate (v, impulses) to a tolerance),
  cold and warm, as the oracle's; its stop rule includes the impulses;
* a whole sphere-drop rollout converged at every step: the chained gradient
  of the centroid loss equals the oracle's to 1e-4 per parameter group (the
  bar for gradients), and it is finite;
* replays are bitwise: checkpoint segments carry the impulses, chunked
  forward launches and batched launches continue them, the allocation-free
  forward starts from zero impulses as sim_forward does.
"""
import numpy as np
import pytest

import scenes
from oracle import diffcloth_oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
KEYS = ("dx0", "dv0", "dw_edge", "dmu")


def _rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def _modes(model, rec):
    md = np.zeros(model.m, np.uint8)
    md[rec.contact.nodes] = rec.contact.mode
    return md


def _sim(sc, **kw):
    from paper_2106_05306_amd.sim import Sim
    kw.setdefault("adj_tol", 1e-12)
    kw.setdefault("adj_max_iters", 10)
    kw.setdefault("adj_solver", "direct")
    return Sim.from_scene(sc, device=DEV, **kw)


def _compare(sc, sim, model, recs, pos_tol, grad_tol, seed=3):
    _, _, traj = sim.forward(len(recs), trajectory=True)
    ref = np.stack([recs[0].x0] + [r.x1 for r in recs])
    err = np.abs(traj.cpu().numpy() - ref).max()
    assert err <= pos_tol, err
    for n, r in enumerate(recs):
        assert np.array_equal(sim.modes(n), _modes(model, r)), n
    L, g = O.centroid_loss(model, recs[-1].x1, sc.target)
    g = g + np.random.default_rng(seed).normal(size=g.shape) * np.abs(g).max()
    G = O.backward(model, recs, g)
    out = sim.backward(torch.tensor(g, device=DEV))
    assert out["status"] == 0, out["status"]
    ref_g = dict(dx0=G.dx0, dv0=G.dv0, dw_edge=G.dw[:model.n_spring], dmu=G.dmu)
    errs = {k: _rel(out[k].cpu().numpy(), ref_g[k]) for k in KEYS if ref_g[k].size}
    for k, e in errs.items():
        assert np.all(np.isfinite(out[k].cpu().numpy())), k
        assert e <= grad_tol, (k, e)
    return err, errs


@pytest.mark.parametrize("make", [lambda: scenes.c1_napkin(0, steps=60),
                                  lambda: scenes.tiny_scene(5, steps=15, obstacle="sphere", seed=2, height=0.01,
                                                            v0_scale=0.1, k=200.0)])
def test_warm_start_fixed_iterations_matches_oracle(make):
    sc = make()
    model = O.Model(sc)
    recs = O.rollout(model, warm_start=True)
    cold = O.rollout(model)
    assert any(np.abs(a.x1 - b.x1).max() > 1e-9 for a, b in zip(recs, cold))   # warm start changes a K-step result
    sim = _sim(sc, precision="fp64", warm_start=True)
    err, errs = _compare(sc, sim, model, recs, 1e-9, 1e-6)
    print("warm start K=20:", sc.name, "pos err", err, "grad errs", errs)


@pytest.mark.parametrize("warm", [False, True])
def test_converged_forward_matches_oracle(warm):
    # a cloth landing and settling on a plane: every node ends in contact, where
    # a stop rule on the velocities alone would stop early
    sc = scenes.tiny_scene(5, steps=8, obstacle="plane", seed=5, height=0.0005, v0_scale=0.05, k=50.0)
    model = O.Model(sc)
    recs = O.rollout(model, tol=1e-12, warm_start=warm)
    sim = _sim(sc, precision="fp64", fwd_tol=1e-12, fwd_max_iters=200000, warm_start=warm)
    err, errs = _compare(sc, sim, model, recs, 1e-9, 1e-6)
    its = [sim.step_stats(n)["pd_iters"] for n in range(sc.steps)]
    assert its == [r.iters for r in recs] or max(abs(a - b.iters) for a, b in zip(its, recs)) <= 2
    print("converged forward, warm", warm, "pos err", err, "grad errs", errs, "iters", its)


def test_whole_sphere_drop_rollout_gradient_converged():
    # the sphere drop of the benchmark at 8 x 8 nodes, released 3 cm above the
    # sphere: every step iterated to 1e-9 m/s (warm-started; 9 000 - 25 000 PD
    # iterations per contact step), then the chained adjoint over all 24 steps
    sc = scenes.c2_sphere_drop(0, n=8, steps=24)
    sc.X = sc.X - np.array([0.0, 0.27, 0.0])
    model = O.Model(sc)
    recs = O.rollout(model, tol=1e-9, warm_start=True)
    assert sum(r.contact.nodes.size for r in recs) > 0
    sim = _sim(sc, precision="fp64", fwd_tol=1e-9, fwd_max_iters=200000, warm_start=True)
    err, errs = _compare(sc, sim, model, recs, 1e-7, 1e-4)
    st = sim.stats()
    print("8x8 sphere drop converged: pos err", err, "grad errs", errs, "modes", st["mode_counts"],
          "max iters", st["fwd_iters_max"])


def test_warm_start_replays_are_bitwise(monkeypatch):
    from paper_2106_05306_amd.sim import batch_backward, batch_forward
    sc = scenes.c2_sphere_drop(0, n=14, steps=40)
    g = torch.tensor(np.random.default_rng(5).normal(size=(sc.n_nodes, 3)), device=DEV)
    res = {}
    for name, kw in (("plain", {}), ("ckpt", dict(checkpoint_every=7)), ("window", dict(adj_window=6))):
        s = _sim(sc, precision="mixed", warm_start=True, adj_tol=1e-10, **kw)
        xT, vT, _ = s.forward(sc.steps)
        res[name] = (xT.clone(), s.backward(g))
        s.close()
    monkeypatch.setenv("DIFFCLOTH_FACTOR_OVERLAP", "0")
    s = _sim(sc, precision="mixed", warm_start=True, adj_tol=1e-10)
    xT, _, _ = s.forward(sc.steps)
    res["one launch"] = (xT.clone(), s.backward(g))
    xa = torch.empty_like(xT)
    va = torch.empty_like(xT)
    s.forward_noalloc(sc.steps, xa, va)
    torch.cuda.synchronize()
    assert torch.equal(xa, xT)
    s.close()
    b = [_sim(sc, precision="mixed", warm_start=True, adj_tol=1e-10) for _ in range(2)]
    outs = batch_forward(b, [sc.steps, sc.steps])
    grads = batch_backward(b, [g, g])
    res["batch"] = (outs[1][0], grads[1])
    for name, (x, gr) in res.items():
        assert torch.equal(x, res["plain"][0]), name
        for k in KEYS:
            assert torch.equal(gr[k], res["plain"][1][k]), (name, k)
