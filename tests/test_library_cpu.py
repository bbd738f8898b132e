"""CPU-side checks of the HIP library: it loads, exports every symbol the
public header declares, and its host setup (constraints, PD matrix,
nested-dissection ordering, supernodal Cholesky) matches the oracle's
independently assembled matrix.  No kernel is launched."""
import os
import re

import numpy as np
import pytest

import scenes
from oracle import diffcloth_oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2106_05306_amd import _binding as B
    return B, B.lib()


def test_library_exports_every_declared_symbol():
    B, L = _lib()
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"^\s*(?:int64_t|int|void|const char)\s*\*?\s*(sim_\w+)\s*\(", txt, re.M))
    assert {"sim_create", "sim_forward", "sim_backward", "sim_destroy"} <= names
    for n in sorted(names):
        assert hasattr(L, n), n


def test_header_is_plain_c():
    # the boundary is a C ABI: the header compiles as C99 on its own, with
    # every struct's size and field offsets as the binding's ctypes mirrors expect
    import shutil
    import subprocess
    import tempfile
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    from paper_2106_05306_amd import _binding as B
    inc = os.path.join(ROOT, "include")
    import ctypes
    pairs = list(zip(("sim_obstacle_t", "sim_mesh_t", "sim_params_t", "sim_grads_t", "sim_stats_t"),
                     (B.SimObstacle, B.SimMesh, B.SimParams, B.SimGrads, B.SimStats)))
    body = ""
    expect = []
    for cname, py in pairs:
        body += f'  printf("%zu\\n", sizeof({cname}));\n'
        expect.append(ctypes.sizeof(py))
        for fname, _ in py._fields_:             # every field at the offset the mirror uses
            body += f'  printf("%zu\\n", offsetof({cname}, {fname}));\n'
            expect.append(getattr(py, fname).offset)
    src = ("#include <stdio.h>\n#include <stddef.h>\n#include \"diffcloth.h\"\nint main(void) {\n" + body +
           "  return 0;\n}\n")
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write(src)
        subprocess.run([gcc, "-std=c99", "-Wall", "-Werror", "-I", inc, c, "-o", exe], check=True)
        sizes = [int(v) for v in subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()]
    assert sizes == expect


def test_error_strings():
    B, L = _lib()
    for code in (0, -1, -2, -3, -4, -5, -6, -7, 1, 2, 3):
        assert L.sim_strerror(code) != b"unknown code", code


@pytest.mark.parametrize("make", [lambda: scenes.c1_napkin(0), lambda: scenes.tiny_scene(5, pins=True, seed=3),
                                  lambda: scenes.c2_sphere_drop(0, n=24), lambda: scenes.c3_skirt(0, 12, 14)])
def test_host_factor_matches_oracle_matrix(make):
    from paper_2106_05306_amd import sim as S
    sc = make()
    st, perm, L = S.analyze(max_dense=2000, **S.scene_kwargs(sc))
    model = O.Model(sc)
    assert sorted(perm.tolist()) == list(range(sc.n_nodes))
    Pp = model.P_s.toarray()[np.ix_(perm, perm)]
    assert np.allclose(np.tril(L), L)
    assert np.abs(L @ L.T - Pp).max() <= 1e-13 * np.abs(Pp).max()
    assert st["n_edges"] == model.n_spring and st["n_bend"] == model.n_bend
    assert st["n_constraints_active"] == int(np.sum(model.rho > 0))


def test_host_rejects_bad_inputs():
    from paper_2106_05306_amd import sim as S
    from paper_2106_05306_amd import _binding as B
    sc = scenes.tiny_scene(3)
    kw = S.scene_kwargs(sc)
    bad_mass = dict(kw, node_mass=np.zeros(sc.n_nodes))
    with pytest.raises(B.SimError) as e:
        S.analyze(**bad_mass)
    assert e.value.code == B.SIM_ENOTSPD
    bad_x = dict(kw, X=np.full_like(sc.X, np.nan))
    with pytest.raises(B.SimError) as e:
        S.analyze(**bad_x)
    assert e.value.code == B.SIM_ENONFINITE
    bad_tri = dict(kw, tris=np.array([[0, 1, 99]]))
    with pytest.raises(B.SimError) as e:
        S.analyze(**bad_tri)
    assert e.value.code == B.SIM_EINVAL
    # self-collision: finite non-negative parameters, and only with the iterative adjoint
    S.analyze(**dict(kw, self_thickness=0.01, self_radius=0.02, self_mu=0.3))
    for bad in (dict(self_thickness=-0.01), dict(self_thickness=0.01, self_mu=np.nan),
                dict(self_thickness=0.01, self_radius=-1.0), dict(self_thickness=0.01, adj_solver="direct")):
        with pytest.raises(B.SimError) as e:
            S.analyze(**dict(kw, **bad))
        assert e.value.code == B.SIM_EINVAL, bad


def test_host_checks_mesh_obstacles():
    from paper_2106_05306_amd import sim as S
    from paper_2106_05306_amd import _binding as B
    sc = scenes.tiny_scene(3, obstacle="sphere")
    V, T = scenes.icosphere((0.0, 0.0, 0.0), 0.25, 1)
    ok = dict(type=B.SIM_MESH, p=(0, 0, 0), mu=0.4, verts=V, tris=T)
    S.analyze(**S.scene_kwargs(sc, obstacles=[ok]))                  # accepted
    for bad in (dict(ok, tris=np.where(T == 3, 999, T)),               # vertex index out of range
                dict(ok, tris=np.array([[0, 1, 1]], np.int32)),        # degenerate triangle
                dict(ok, verts=np.where(V == V[0, 0], np.nan, V)),     # non-finite vertex
                dict(ok, tris=np.zeros((0, 3), np.int32))):            # no triangles
        with pytest.raises(B.SimError) as e:
            S.analyze(**S.scene_kwargs(sc, obstacles=[bad]))
        assert e.value.code == B.SIM_EINVAL


def test_null_handles_are_rejected_without_a_gpu():
    # argument checks run before any device work
    import ctypes
    B, L = _lib()
    assert L.sim_set_material(None, None, None, None, None) == B.SIM_EINVAL
    assert L.sim_set_external_force(None, None, 0, None) == B.SIM_EINVAL
    assert L.sim_job_forward(None, 10) == B.SIM_EINVAL
    assert L.sim_job_backward(None, None, None) == B.SIM_EINVAL
    assert L.sim_job_grads(None, None) == B.SIM_EINVAL
    assert L.sim_batch_advance(None, 0, None, None, None) == B.SIM_EINVAL
    assert L.sim_forward(None, 5, None, None, None) == B.SIM_EINVAL
    assert L.sim_backward(None, None, None, None, None) == B.SIM_EINVAL
    one = (ctypes.c_void_p * 1)(None)
    steps = (ctypes.c_int32 * 1)(3)
    assert L.sim_batch_advance(one, 1, steps, None, None) == B.SIM_EINVAL


def test_ordering_merges_top_separators():
    # the elimination tree of a 40 x 40 grid with its top separators merged
    # into one supernode is shallower than without, and both orders give
    # L L^T = P_s[perm][:, perm]
    import os
    from paper_2106_05306_amd.sim import analyze, scene_kwargs
    sc = scenes.c2_sphere_drop(0, n=12, steps=2)
    st, perm, L = analyze(leaf_size=8, max_dense=200, **scene_kwargs(sc))
    model = O.Model(sc)
    P = model.P_s.toarray()[perm][:, perm]
    assert sorted(perm.tolist()) == list(range(sc.n_nodes))
    assert np.allclose(L @ L.T, P, rtol=1e-12, atol=1e-14 * np.abs(P).max())
    os.environ["DIFFCLOTH_MERGE"] = "0"
    try:
        st0, perm0, L0 = analyze(leaf_size=8, max_dense=200, **scene_kwargs(sc))
    finally:
        del os.environ["DIFFCLOTH_MERGE"]
    P0 = model.P_s.toarray()[perm0][:, perm0]
    assert np.allclose(L0 @ L0.T, P0, rtol=1e-12, atol=1e-14 * np.abs(P0).max())
    assert st["n_levels"] < st0["n_levels"]


def test_plans_are_host_only_and_build_on_threads():
    # the host part of a handle needs no GPU (none here) and distinct plans
    # build concurrently; errors come back as from sim_create
    import concurrent.futures
    from paper_2106_05306_amd import sim as S
    from paper_2106_05306_amd import _binding as B
    scs = [scenes.request_scene(n, 10, bool(n % 2), seed=n) for n in (12, 17, 23, 30, 12, 17)]
    with concurrent.futures.ThreadPoolExecutor(max_workers=4) as ex:
        plans = list(ex.map(S.Plan.from_scene, scs))
    assert all(p.h for p in plans)
    for p in plans:
        p.close()
        assert p.h is None
    with pytest.raises(B.SimError) as e:
        S.Plan.from_scene(scs[0], bend_weight=-1.0)
    assert e.value.code == B.SIM_EINVAL
