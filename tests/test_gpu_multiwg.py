"""The multi-workgroup forward kernel (one handle on up to 16 workgroups of
one XCD: whole subtrees of the elimination tree per workgroup, the root
supernode shared) against the single-workgroup kernel and the oracle.

Every node, row and work item is computed with the single-workgroup kernel's
arithmetic (same items, team sizes and summation orders; which workgroup takes
which run of the root's row pairs, and whether it reads them from L2 or from
its LDS copy, changes no sum), so trajectories,
records and gradients are bitwise equal; the float64 run also matches the
oracle.  A barrier that waits longer than its limit gives up (a limit of 0
ticks from the host forces it): the launch returns SIM_ESYNC and the kernel
exits normally.
"""
import numpy as np
import pytest

import scenes
from oracle import diffcloth_oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
KEYS = ("dx0", "dv0", "dw_edge", "dmu")


def _run(sc, monkeypatch, wgs, steps=None, **kw):
    from paper_2106_05306_amd.sim import Sim
    monkeypatch.setenv("DIFFCLOTH_FWD_WGS", str(wgs))
    kw.setdefault("adj_solver", "direct")
    kw.setdefault("adj_tol", 1e-10)
    kw.setdefault("adj_max_iters", 10)
    s = Sim.from_scene(sc, device=DEV, **kw)
    steps = steps or sc.steps
    _, _, traj = s.forward(steps, trajectory=True)
    st = s.stats()
    g = s.backward(torch.tensor(np.random.default_rng(2).normal(size=(sc.n_nodes, 3)), device=DEV))
    info = [s.step_stats(n) for n in range(steps)]
    modes = [s.modes(n) for n in range(0, steps, max(1, steps // 7))]
    s.close()
    return traj, g, st, info, modes


@pytest.mark.parametrize("n,prec,kw", [(40, "mixed", {}), (24, "fp64", {}), (40, "mixed", dict(warm_start=True)),
                                       (30, "fp64", dict(checkpoint_every=9))])
def test_multi_workgroup_forward_is_bitwise(monkeypatch, n, prec, kw):
    sc = scenes.c2_sphere_drop(0, n=n, steps=45)
    a = _run(sc, monkeypatch, 1, precision=prec, **kw)
    b = _run(sc, monkeypatch, 16, precision=prec, **kw)
    print(f"{n}x{n} {prec} {kw}: forward {a[2]['fwd_ms']:.1f} ms on one workgroup, {b[2]['fwd_ms']:.1f} ms on several",
          flush=True)
    assert torch.equal(a[0], b[0])
    for k in KEYS:
        assert torch.equal(a[1][k], b[1][k]), k
    assert a[3] == b[3]
    for x, y in zip(a[4], b[4]):
        assert np.array_equal(x, y)
    assert a[2]["mode_counts"] == b[2]["mode_counts"]


@pytest.mark.parametrize("n,threads,root_lds", [(24, "1024", "1"), (40, "256", "1"), (40, "1024", "0")])
def test_multi_workgroup_forward_with_vectors_in_hbm_is_bitwise(monkeypatch, n, threads, root_lds):
    # the variant for subtrees whose vectors do not fit LDS (large meshes): the
    # solve runs in place in the iterate buffer, which swaps every PD iteration;
    # also fewer threads per workgroup (timing only), and each workgroup's run
    # of the root's stored inverse read from L2 instead of its LDS copy
    sc = scenes.c2_sphere_drop(0, n=n, steps=30)
    a = _run(sc, monkeypatch, 1, precision="mixed")
    monkeypatch.setenv("DIFFCLOTH_MW_LDS", "0")
    monkeypatch.setenv("DIFFCLOTH_MW_THREADS", threads)
    monkeypatch.setenv("DIFFCLOTH_MW_ROOT_LDS", root_lds)
    b = _run(sc, monkeypatch, 16, precision="mixed")
    assert b[2]["fwd_workgroups"] > 1
    assert torch.equal(a[0], b[0])
    for k in KEYS:
        assert torch.equal(a[1][k], b[1][k]), k
    assert a[3] == b[3]


def test_multi_workgroup_converged_forward_matches_oracle(monkeypatch):
    # tolerance-terminated forward: the stop decision is a maximum over all
    # workgroups' nodes, taken identically by every workgroup
    sc = scenes.c2_sphere_drop(0, n=8, steps=24)
    sc.X = sc.X - np.array([0.0, 0.27, 0.0])
    model = O.Model(sc)
    recs = O.rollout(model, tol=1e-9, warm_start=True)
    a = _run(sc, monkeypatch, 1, precision="fp64", fwd_tol=1e-9, fwd_max_iters=200000, warm_start=True)
    b = _run(sc, monkeypatch, 16, precision="fp64", fwd_tol=1e-9, fwd_max_iters=200000, warm_start=True)
    assert torch.equal(a[0], b[0])
    ref = np.stack([recs[0].x0] + [r.x1 for r in recs])
    assert np.abs(b[0].cpu().numpy() - ref).max() <= 1e-7
    assert [q["pd_iters"] for q in b[3]] == [q["pd_iters"] for q in a[3]]


def test_multi_workgroup_barrier_gives_up_when_told(monkeypatch):
    # the host withholds one workgroup (it returns at once), so the others'
    # first barrier never completes: each wait ends at its 1 ms limit, every
    # workgroup returns, and the call reports SIM_ESYNC
    from paper_2106_05306_amd import _binding as B
    from paper_2106_05306_amd.sim import Sim
    sc = scenes.c2_sphere_drop(0, n=40, steps=4)
    monkeypatch.setenv("DIFFCLOTH_FWD_WGS", "16")
    monkeypatch.setenv("DIFFCLOTH_MW_SPIN", "100000")
    monkeypatch.setenv("DIFFCLOTH_MW_TEST_ABSENT", "1")
    s = Sim.from_scene(sc, device=DEV, precision="mixed")
    with pytest.raises(B.SimError) as e:
        s.forward(sc.steps)
    assert e.value.code == B.SIM_ESYNC
    s.close()
    monkeypatch.delenv("DIFFCLOTH_MW_SPIN")
    monkeypatch.delenv("DIFFCLOTH_MW_TEST_ABSENT")
    s = Sim.from_scene(sc, device=DEV, precision="mixed")
    xT, _, _ = s.forward(sc.steps)
    assert torch.isfinite(xT).all()
    s.close()
