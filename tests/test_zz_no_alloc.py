"""The allocation-free forward (sim_forward_noalloc) through the C ABI.

It must give bitwise the x_T and v_T of sim_forward on the same handle (the
same kernels run; only where their work memory lives differs), allocate
nothing (the handle's allocator callback is not called and its device bytes
do not change), leave the recorded rollout alone, and work again right after
on a smaller handle (the device scratch keeps the previous call's contents).
"""
import ctypes

import numpy as np
import pytest

import scenes

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _pair(sc, **kw):
    from paper_2106_05306_amd.sim import Sim
    s = Sim.from_scene(sc, device=DEV, **kw)
    xT, vT, _ = s.forward(sc.steps)
    return s, xT.clone(), vT.clone()


def _noalloc(s, steps):
    from paper_2106_05306_amd import _binding as B
    xT = torch.full((s.m, 3), float("nan"), dtype=torch.float64, device=DEV)
    vT = torch.full((s.m, 3), float("nan"), dtype=torch.float64, device=DEV)
    live = len(s._alloc.live)
    dev_bytes = s.stats()["device_bytes"]
    code = B.lib().sim_forward_noalloc(s.h, int(steps), ctypes.c_void_p(xT.data_ptr()), ctypes.c_void_p(vT.data_ptr()))
    assert code == 0, code
    torch.cuda.synchronize()
    assert len(s._alloc.live) == live
    assert s.stats()["device_bytes"] == dev_bytes
    return xT, vT


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_forward_equals_forward_twice_second_smaller(precision):
    big = scenes.c2_sphere_drop(0, n=24, steps=30)
    small = scenes.c1_napkin(0, steps=25)
    s1, x1, v1 = _pair(big, precision=precision)
    s2, x2, v2 = _pair(small, precision=precision)
    assert s2.noalloc_scratch_bytes() < s1.noalloc_scratch_bytes()
    ref_x12 = s1.state(12)[0].clone()
    a_x, a_v = _noalloc(s1, big.steps)
    assert torch.equal(a_x, x1) and torch.equal(a_v, v1)
    b_x, b_v = _noalloc(s2, small.steps)            # second call, smaller input
    assert torch.equal(b_x, x2) and torch.equal(b_v, v2)
    assert torch.equal(s1.state(12)[0], ref_x12)     # the recorded rollout is untouched
    s1.close()
    s2.close()


def test_noalloc_forward_with_checkpointed_and_mesh_handles():
    # a handle with a triangle-mesh obstacle (its own kernel variant) and
    # fewer steps than its last recorded rollout
    sc = scenes.discretized_sphere_drop(0, n=12, steps=20, level=1)
    s, xT, vT = _pair(sc, precision="fp64", checkpoint_every=6)
    a_x, a_v = _noalloc(s, sc.steps)
    assert torch.equal(a_x, xT) and torch.equal(a_v, vT)
    s.close()


def test_noalloc_rejects_meshes_beyond_the_scratch():
    from paper_2106_05306_amd import _binding as B
    from paper_2106_05306_amd.sim import Sim
    sc = scenes.mixed_grid(np.random.default_rng(0), 200, 2, 1e3, 0.5, False)
    s = Sim.from_scene(sc, device=DEV, precision="fp64")
    assert s.noalloc_scratch_bytes() > 16 << 20
    xT = torch.empty((s.m, 3), dtype=torch.float64, device=DEV)
    vT = torch.empty_like(xT)
    code = B.lib().sim_forward_noalloc(s.h, 2, ctypes.c_void_p(xT.data_ptr()), ctypes.c_void_p(vT.data_ptr()))
    assert code == B.SIM_ESCRATCH
    s.close()
