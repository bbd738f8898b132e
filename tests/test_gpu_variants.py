"""Every kernel variant the product runs, against the FP64 oracle.

The forward and adjoint kernels are instantiated per LDS placement (which of
the PD iterates / solve vectors, the solve's update buffer and the positions
live in LDS instead of HBM), per adjoint solver and per obstacle kind; large
meshes (the skirt, big batch members and served meshes) run the placements
with data in HBM.  ``DIFFCLOTH_LDS`` restricts the placement, so every
variant runs here on small meshes:

* float64: positions within 1e-9 m of the oracle, identical contact modes and
  gradients within 1e-6 of the oracle's (relative, per parameter group);
* every placement gives bitwise the same result as every other (the placement
  only moves data), in float64 and in mixed precision.
"""
import numpy as np
import pytest

import scenes
from oracle import diffcloth_oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
KEYS = ("dx0", "dv0", "dw_edge", "dw_bend", "dmu")


def _rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def _modes(model, rec):
    md = np.zeros(model.m, np.uint8)
    md[rec.contact.nodes] = rec.contact.mode
    return md


def _run(sc, monkeypatch, mask, statuses=(0,), **kw):
    from paper_2106_05306_amd.sim import Sim
    monkeypatch.setenv("DIFFCLOTH_LDS", str(mask))
    sim = Sim.from_scene(sc, device=DEV, **kw)
    st = sim.stats()
    assert st["lds_flags_fwd"] == mask, (st["lds_flags_fwd"], mask)
    assert st["lds_flags_bwd"] == (mask & 3), (st["lds_flags_bwd"], mask)
    _, _, traj = sim.forward(sc.steps, trajectory=True)
    modes = np.stack([sim.modes(n) for n in range(sc.steps)])
    g = torch.tensor(_seed(sc), device=DEV)
    out = sim.backward(g)
    assert out["status"] in statuses, out["status"]
    res = {k: out[k].cpu().numpy() for k in KEYS}
    sim.close()
    return traj.cpu().numpy(), modes, res


def _seed(sc):
    return np.random.default_rng(11).normal(size=(sc.n_nodes, 3))


def _oracle(sc):
    model = O.Model(sc)
    recs = O.rollout(model)
    traj = np.stack([recs[0].x0] + [r.x1 for r in recs])
    modes = np.stack([_modes(model, r) for r in recs])
    G = O.backward(model, recs, _seed(sc))
    dwb = np.zeros(model.m)
    dwb[model.bend_centers] = G.dw[model.n_spring:]
    ref = dict(dx0=G.dx0, dv0=G.dv0, dw_edge=G.dw[:model.n_spring], dw_bend=dwb, dmu=G.dmu)
    return traj, modes, ref


@pytest.mark.parametrize("solver", ["iterative", "direct"])
@pytest.mark.parametrize("obstacle", ["sphere", "mesh"])
def test_every_lds_placement_matches_oracle_fp64(monkeypatch, solver, obstacle):
    sc = scenes.tiny_scene(5, steps=12, obstacle="sphere", seed=21, height=0.01, v0_scale=0.1, k=200.0)
    if obstacle == "mesh":
        o = sc.obstacles[0]
        V, T = scenes.icosphere(o.point, o.radius, 2)
        sc.obstacles = [scenes.mesh_obstacle(V, T, o.mu)]
    traj_o, modes_o, ref = _oracle(sc)
    first = None
    for mask in range(8):
        traj, modes, res = _run(sc, monkeypatch, mask, precision="fp64", adj_solver=solver, adj_tol=1e-12,
                                adj_max_iters=3000 if solver == "iterative" else 10)
        err = np.abs(traj - traj_o).max()
        assert err <= 1e-9, (mask, err)
        assert np.array_equal(modes, modes_o), mask
        for k in KEYS:
            assert _rel(res[k], ref[k]) <= 1e-6, (mask, k, _rel(res[k], ref[k]))
        if first is None:
            first = (traj, modes, res)
        else:
            assert np.array_equal(traj, first[0]), mask
            for k in KEYS:
                assert np.array_equal(res[k], first[2][k]), (mask, k)


@pytest.mark.parametrize("solver", ["iterative", "direct"])
def test_every_lds_placement_is_bitwise_in_mixed_precision(monkeypatch, solver):
    sc = scenes.c2_sphere_drop(0, n=12, steps=40)
    first = None
    for mask in range(8):
        # (the 20-iteration forward leaves some adjoint systems that the
        # iterative solver does not bring to 1e-10: a warning, same in every variant)
        traj, modes, res = _run(sc, monkeypatch, mask, statuses=(0, 1, 2), precision="mixed", adj_solver=solver,
                                adj_tol=1e-10, adj_max_iters=3000 if solver == "iterative" else 10)
        if first is None:
            first = (traj, modes, res)
            continue
        assert np.array_equal(traj, first[0]), mask
        assert np.array_equal(modes, first[1]), mask
        for k in KEYS:
            assert np.array_equal(res[k], first[2][k]), (mask, k)


def test_batched_launch_with_data_in_hbm_matches_oracle(monkeypatch):
    # a batch whose placement keeps everything in HBM (as the batches of large
    # members run) against the oracle, member by member
    from paper_2106_05306_amd.sim import Sim, batch_backward, batch_forward
    monkeypatch.setenv("DIFFCLOTH_LDS", "0")
    batch = scenes.c4_batch(seed=3, count=3, steps=10, n_lo=5, n_hi=9)
    sims = [Sim.from_scene(sc, device=DEV, precision="fp64", adj_solver="direct", adj_tol=1e-12, adj_max_iters=10)
            for sc in batch]
    outs = batch_forward(sims, [sc.steps for sc in batch])
    grads = batch_backward(sims, [torch.tensor(_seed(sc), device=DEV) for sc in batch])
    for sc, (xT, _), g in zip(batch, outs, grads):
        traj_o, modes_o, ref = _oracle(sc)
        assert np.abs(xT.cpu().numpy() - traj_o[-1]).max() <= 1e-9
        for k in KEYS:
            assert _rel(g[k].cpu().numpy(), ref[k]) <= 1e-6, k
