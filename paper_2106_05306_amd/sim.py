"""Python front end of the C ABI: one ``Sim`` per cloth handle.

PyTorch provides device memory (the handle's allocations come from the
caching allocator through a callback) and the stream; every step of the
simulation and of its adjoint runs in the HIP kernels of libdiffcloth.so.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np
import torch

from . import _binding as B


class _TorchAllocator:
    """Device allocations for the library, owned by PyTorch tensors."""

    def __init__(self, device):
        self.device = device
        self.live = {}
        self.c_alloc = B.ALLOC_FN(self._alloc)
        self.c_free = B.FREE_FN(self._free)

    def _alloc(self, nbytes, ctx):
        try:
            t = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        except RuntimeError:
            return None
        p = t.data_ptr()
        self.live[p] = t
        return p

    def _free(self, ptr, ctx):
        self.live.pop(ptr, None)


def _dptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _arr(a, dtype):
    return np.ascontiguousarray(np.asarray(a, dtype=dtype))


def build_structs(X, tris, node_mass, edge_stiffness, *, edges=None, h=1.0 / 120.0, pd_iters=20, fwd_tol=0.0,
                  fwd_max_iters=0, gravity=(0.0, -9.8, 0.0), bend_weight=1e-2, attach=(), attach_weight=1e5,
                  attach_omega=0.0, attach_axis=(0.0, 1.0, 0.0), attach_center=(0.0, 0.0, 0.0),
                  obstacles: Sequence[dict] = (), edge_region=None, bend_region=None, region_scale=None,
                  precision="fp64", adj_tol=1e-10, adj_max_iters=500, checkpoint_every=0, adj_restart=0,
                  adj_solver="iterative", adj_window=0, warm_start=False, self_thickness=0.0, self_radius=0.0,
                  self_mu=0.0):
    """Marshal a mesh and its parameters into the C structs; returns
    (SimMesh, SimParams, keep-alive dict of the numpy arrays they point to)."""
    k = {}
    X = _arr(X, np.float64).reshape(-1, 3)
    tris = _arr(tris, np.int32).reshape(-1, 3)
    k["X"], k["tris"] = X, tris
    mesh = B.SimMesh()
    mesh.n_nodes = X.shape[0]
    mesh.X = X.ctypes.data_as(B.c_double_p)
    mesh.n_tris = tris.shape[0]
    mesh.tris = tris.ctypes.data_as(B.c_int32_p)
    if edges is not None:
        k["edges"] = _arr(edges, np.int32).reshape(-1, 2)
        mesh.n_edges = k["edges"].shape[0]
        mesh.edges = k["edges"].ctypes.data_as(B.c_int32_p)
    k["attach"] = _arr(attach, np.int32).reshape(-1)
    mesh.n_attach = k["attach"].size
    mesh.attach = k["attach"].ctypes.data_as(B.c_int32_p)
    mesh.attach_omega = attach_omega
    mesh.attach_axis[:] = list(attach_axis)
    mesh.attach_center[:] = list(attach_center)
    p = B.SimParams()
    p.h = h
    p.pd_iters = pd_iters
    p.fwd_tol = fwd_tol
    p.fwd_max_iters = fwd_max_iters
    p.gravity[:] = list(gravity)
    k["mass"] = _arr(node_mass, np.float64)
    p.node_mass = k["mass"].ctypes.data_as(B.c_double_p)
    k["k"] = _arr(edge_stiffness, np.float64)
    p.edge_stiffness = k["k"].ctypes.data_as(B.c_double_p)
    p.bend_weight = bend_weight
    p.attach_weight = attach_weight
    if region_scale is not None:
        k["er"] = _arr(edge_region, np.int32)
        k["br"] = _arr(bend_region, np.int32)
        k["rs"] = _arr(region_scale, np.float64)
        p.edge_region = k["er"].ctypes.data_as(B.c_int32_p)
        p.bend_region = k["br"].ctypes.data_as(B.c_int32_p)
        p.region_scale = k["rs"].ctypes.data_as(B.c_double_p)
        p.n_regions = k["rs"].size
    obs = (B.SimObstacle * max(1, len(obstacles)))()
    for i, o in enumerate(obstacles):
        obs[i].type = o["type"]
        obs[i].p[:] = list(o["p"])
        obs[i].n[:] = list(o.get("n", (0.0, 1.0, 0.0)))
        obs[i].radius = o.get("radius", 0.0)
        obs[i].mu = o["mu"]
        if o.get("verts") is not None:          # triangle mesh (copied by sim_create)
            k[f"ov{i}"] = _arr(o["verts"], np.float64).reshape(-1)
            k[f"ot{i}"] = _arr(o["tris"], np.int32).reshape(-1)
            obs[i].n_verts = k[f"ov{i}"].size // 3
            obs[i].n_tris = k[f"ot{i}"].size // 3
            obs[i].verts = k[f"ov{i}"].ctypes.data_as(B.c_double_p)
            obs[i].tris = k[f"ot{i}"].ctypes.data_as(B.c_int32_p)
    k["obs"] = obs
    p.n_obstacles = len(obstacles)
    p.obstacles = obs
    p.precision = {"fp64": B.SIM_FP64, "mixed": B.SIM_MIXED}[precision]
    p.adj_tol = adj_tol
    p.adj_max_iters = adj_max_iters
    p.checkpoint_every = checkpoint_every
    p.adj_restart = adj_restart
    p.adj_solver = {"iterative": B.SIM_ADJ_ITERATIVE, "direct": B.SIM_ADJ_DIRECT}[adj_solver]
    p.adj_window = adj_window
    p.warm_start = 1 if warm_start else 0
    p.self_thickness = self_thickness
    p.self_radius = self_radius
    p.self_mu = self_mu
    return mesh, p, k


def scene_kwargs(scene, **kw):
    """Keyword arguments of build_structs / Sim for an object carrying the
    workload fields (X, tris, edges, node_mass, edge_stiffness, obstacles, ...)."""
    obstacles = [dict(type=o.kind, p=o.point, n=o.normal, radius=o.radius, mu=o.mu,
                      verts=getattr(o, "verts", None), tris=getattr(o, "tris", None)) for o in scene.obstacles]
    args = dict(X=scene.X, tris=scene.tris, node_mass=scene.node_mass, edge_stiffness=scene.edge_stiffness,
                edges=scene.edges, h=scene.h, pd_iters=scene.pd_iters, gravity=scene.gravity,
                bend_weight=scene.bend_weight, attach=scene.attach, attach_weight=scene.attach_weight,
                attach_omega=scene.attach_omega, attach_axis=scene.attach_axis, attach_center=scene.attach_center,
                obstacles=obstacles)
    if getattr(scene, "self_thickness", 0.0):
        args.update(self_thickness=scene.self_thickness, self_radius=scene.self_radius, self_mu=scene.self_mu)
    if scene.region_scale is not None:
        args.update(edge_region=scene.edge_region, bend_region=scene.bend_region, region_scale=scene.region_scale)
    args.update(kw)
    return args


def analyze(leaf_size=32, max_dense=0, **kw):
    """Host-only analysis (no GPU): sizes, elimination order and, for small
    meshes, the dense Cholesky factor of the permuted PD matrix."""
    mesh, p, keep = build_structs(**kw)
    st = B.SimStats()
    m = mesh.n_nodes
    perm = np.zeros(m, np.int32)
    L = np.zeros((m, m)) if max_dense and m <= max_dense else None
    B.check(B.lib().sim_analyze(ctypes.byref(mesh), ctypes.byref(p), leaf_size, ctypes.byref(st),
                                perm.ctypes.data_as(B.c_int32_p),
                                None if L is None else L.ctypes.data_as(B.c_double_p), max_dense), "sim_analyze")
    return {name: getattr(st, name) for name, _ in B.SimStats._fields_}, perm, L


class Plan:
    """The host part of a handle (``sim_plan_create``: constraint tables, PD
    matrix, ordering, Cholesky factor) built without any GPU call, so it may
    run on a worker thread; ``Sim.from_plan`` turns it into a handle."""

    def __init__(self, X, tris, node_mass, edge_stiffness, **kw):
        self.kw = kw
        self._mesh, self._params, self._keep = build_structs(X, tris, node_mass, edge_stiffness, **kw)
        out = ctypes.c_void_p()
        B.check(B.lib().sim_plan_create(ctypes.byref(self._mesh), ctypes.byref(self._params), ctypes.byref(out)),
                "sim_plan_create")
        self.h = out

    @classmethod
    def from_scene(cls, scene, **kw):
        a = scene_kwargs(scene, **kw)
        return cls(a.pop("X"), a.pop("tris"), a.pop("node_mass"), a.pop("edge_stiffness"), **a)

    def close(self):
        if getattr(self, "h", None):
            B.lib().sim_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()


class Sim:
    """A cloth handle: mesh + parameters -> factorised PD system on the GPU."""

    def __init__(self, X, tris, node_mass, edge_stiffness, *, device="cuda",
                 stream: Optional[torch.cuda.Stream] = None, plan: Optional[Plan] = None, **kw):
        self.device = torch.device(device)
        self.stream = stream or torch.cuda.current_stream(self.device)
        self._alloc = _TorchAllocator(self.device)
        if plan is not None:
            kw = plan.kw
            mesh, p, self._keep = plan._mesh, plan._params, dict(plan._keep)
        else:
            mesh, p, self._keep = build_structs(X, tris, node_mass, edge_stiffness, **kw)
        self.m = mesh.n_nodes
        self.n_regions = int(p.n_regions)
        self._gen = 0                       # bumped by every call that replaces the recorded rollout
        self.edge_region = None if kw.get("edge_region") is None else np.asarray(kw["edge_region"], np.int64)
        self.bend_region = None if kw.get("bend_region") is None else np.asarray(kw["bend_region"], np.int64)
        self.region_scale = None if kw.get("region_scale") is None else np.asarray(kw["region_scale"], np.float64)
        self.n_obstacles = int(p.n_obstacles)
        self.precision = kw.get("precision", "fp64")
        self._mesh, self._params = mesh, p
        h_out = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            if plan is not None:
                B.check(B.lib().sim_create_from_plan(plan.h, ctypes.c_void_p(self.stream.cuda_stream),
                                                     self._alloc.c_alloc, self._alloc.c_free, None,
                                                     ctypes.byref(h_out)), "sim_create_from_plan")
                plan.h = None                   # taken over by the handle
            else:
                B.check(B.lib().sim_create(ctypes.byref(mesh), ctypes.byref(p),
                                           ctypes.c_void_p(self.stream.cuda_stream), self._alloc.c_alloc,
                                           self._alloc.c_free, None, ctypes.byref(h_out)), "sim_create")
        self.h = h_out
        st = self.stats()
        self.n_edges = st["n_edges"]
        self.T = -1

    # ------------------------------------------------------------------ construction helpers
    @classmethod
    def from_plan(cls, plan: Plan, device="cuda", stream: Optional[torch.cuda.Stream] = None):
        """The handle of a host plan (its device part; the plan is used up)."""
        return cls(None, None, None, None, device=device, stream=stream, plan=plan)

    @classmethod
    def from_scene(cls, scene, **kw):
        """Build from an object carrying the workload fields (see scene_kwargs)."""
        a = scene_kwargs(scene, **kw)
        sim = cls(a.pop("X"), a.pop("tris"), a.pop("node_mass"), a.pop("edge_stiffness"), **a)
        v0 = np.asarray(getattr(scene, "v0", None) if getattr(scene, "v0", None) is not None else 0.0)
        if np.any(v0 != 0):
            sim.set_state(None, torch.as_tensor(np.broadcast_to(v0, (sim.m, 3)).copy(), dtype=torch.float64))
        if getattr(scene, "force", None) is not None:
            sim.set_external_force(torch.as_tensor(np.asarray(scene.force, np.float64)),
                                   getattr(scene, "force_scale", None))
        return sim

    # ------------------------------------------------------------------ calls
    def _vec(self):
        return torch.empty((self.m, 3), dtype=torch.float64, device=self.device)

    def set_state(self, x0: Optional[torch.Tensor] = None, v0: Optional[torch.Tensor] = None):
        x0 = None if x0 is None else x0.to(self.device, torch.float64).contiguous()
        v0 = None if v0 is None else v0.to(self.device, torch.float64).contiguous()
        self._keep["x0"], self._keep["v0"] = x0, v0
        B.check(B.lib().sim_set_state(self.h, _dptr(x0), _dptr(v0)), "sim_set_state")
        self.T = -1
        self._gen += 1

    def set_material(self, edge_stiffness=None, bend_weight=None, region_scale=None, mu=None):
        """New constraint weights / friction (host values; None = keep); refactors P."""
        def host(a, n):
            if a is None:
                return None, None
            a = np.ascontiguousarray(np.asarray(a.detach().cpu() if torch.is_tensor(a) else a,
                                                dtype=np.float64).reshape(-1))
            if n > 0 and a.size != n:          # (n = 0: the library rejects the argument)
                raise ValueError(f"expected {n} values, got {a.size}")
            return a, a.ctypes.data_as(B.c_double_p)
        k, kp = host(edge_stiffness, self.n_edges)
        b, bp = host(bend_weight, 1)
        r, rp = host(region_scale, self.n_regions)
        u, up = host(mu, self.n_obstacles)
        B.check(B.lib().sim_set_material(self.h, kp, bp, rp, up), "sim_set_material")
        if r is not None:
            self.region_scale = r.copy()
        self.T = -1
        self._gen += 1

    def set_external_force(self, force: Optional[torch.Tensor] = None, scale=None):
        """External force besides gravity: node j receives scale[n] * force[j]
        (newtons) during step n (scale None: 1 at every step; force None:
        remove).  The backward pass then returns dforce (m, 3) and dforce_scale (T,)."""
        f = None if force is None else force.to(self.device, torch.float64).reshape(self.m, 3).contiguous()
        sc = None
        if f is not None and scale is not None:
            sc = np.ascontiguousarray(np.asarray(scale.detach().cpu() if torch.is_tensor(scale) else scale,
                                                 dtype=np.float64).reshape(-1))
        self._keep["force"] = f
        B.check(B.lib().sim_set_external_force(self.h, _dptr(f), 0 if sc is None else sc.size,
                                               None if sc is None else sc.ctypes.data_as(B.c_double_p)),
                "sim_set_external_force")
        self.T = -1
        self._gen += 1

    def forward(self, n_steps: int, trajectory: bool = False):
        xT, vT = self._vec(), self._vec()
        traj = torch.empty((n_steps + 1, self.m, 3), dtype=torch.float64, device=self.device) if trajectory else None
        B.check(B.lib().sim_forward(self.h, n_steps, _dptr(traj), _dptr(xT), _dptr(vT)), "sim_forward")
        self.T = n_steps
        self._gen += 1
        return xT, vT, traj

    def forward_noalloc(self, n_steps: int, xT: torch.Tensor, vT: torch.Tensor):
        """sim_forward_noalloc: x_T, v_T into the caller's (n, 3) float64 tensors;
        the library allocates nothing and records no rollout."""
        for t in (xT, vT):
            if t.dtype != torch.float64 or not t.is_contiguous() or t.numel() != 3 * self.m or t.device != self.device:
                raise ValueError("x_T / v_T must be contiguous float64 device tensors of n_nodes x 3")
        B.check(B.lib().sim_forward_noalloc(self.h, int(n_steps), _dptr(xT), _dptr(vT)), "sim_forward_noalloc")

    def noalloc_scratch_bytes(self) -> int:
        return int(B.lib().sim_noalloc_scratch_bytes(self.h))

    def _grads(self):
        g = dict(dx0=self._vec(), dv0=self._vec(),
                 dw_edge=torch.zeros(max(self.n_edges, 1), dtype=torch.float64, device=self.device),
                 dw_bend=torch.zeros(self.m, dtype=torch.float64, device=self.device),
                 dregion=torch.zeros(max(self.n_regions, 1), dtype=torch.float64, device=self.device),
                 dmu=torch.zeros(max(self.n_obstacles, 1), dtype=torch.float64, device=self.device),
                 dforce=self._vec(),
                 dforce_scale=torch.zeros(max(self.T, 1), dtype=torch.float64, device=self.device),
                 dmu_self=torch.zeros(1, dtype=torch.float64, device=self.device))
        s = B.SimGrads(*[ctypes.c_void_p(g[k].data_ptr()) for k in ("dx0", "dv0", "dw_edge", "dw_bend", "dregion",
                                                                     "dmu", "dforce", "dforce_scale", "dmu_self")])
        return g, s

    def backward(self, dL_dxT: torch.Tensor, dL_dvT: Optional[torch.Tensor] = None,
                 dL_dx_steps: Optional[torch.Tensor] = None):
        g, s = self._grads()
        a = dL_dxT.to(self.device, torch.float64).contiguous()
        b = None if dL_dvT is None else dL_dvT.to(self.device, torch.float64).contiguous()
        c = None if dL_dx_steps is None else dL_dx_steps.to(self.device, torch.float64).contiguous()
        code = B.check(B.lib().sim_backward(self.h, _dptr(a), _dptr(b), _dptr(c), ctypes.byref(s)), "sim_backward")
        g["status"] = code
        return self._trim(g)

    def adjoint_step(self, n: int, gx: torch.Tensor, gv: torch.Tensor):
        g, s = self._grads()
        gx = gx.to(self.device, torch.float64).contiguous()
        gv = gv.to(self.device, torch.float64).contiguous()
        code = B.check(B.lib().sim_adjoint_step(self.h, n, _dptr(gx), _dptr(gv), _dptr(g["dx0"]), _dptr(g["dv0"]),
                                                ctypes.byref(s)), "sim_adjoint_step")
        g["status"] = code
        return self._trim(g)

    def trim(self):
        """Release the device memory held only for a rollout (records, step factors)."""
        B.check(B.lib().sim_trim(self.h), "sim_trim")
        self.T = -1
        self._gen += 1

    # ------------------------------------------------------------------ continuous batching
    def job_forward(self, n_steps: int):
        """Arm a forward pass of n_steps (run by batch_advance)."""
        B.check(B.lib().sim_job_forward(self.h, int(n_steps)), "sim_job_forward")
        self.T = -1
        self._job_T = int(n_steps)
        self._gen += 1

    def job_backward(self, dL_dxT: torch.Tensor, dL_dvT: Optional[torch.Tensor] = None):
        """Arm the backward pass of the finished forward pass."""
        a = dL_dxT.to(self.device, torch.float64).contiguous()
        b = None if dL_dvT is None else dL_dvT.to(self.device, torch.float64).contiguous()
        self._keep["job_seed"] = (a, b)
        self.T = self._job_T
        B.check(B.lib().sim_job_backward(self.h, _dptr(a), _dptr(b)), "sim_job_backward")

    def job_grads(self):
        g, s = self._grads()
        g["status"] = B.check(B.lib().sim_job_grads(self.h, ctypes.byref(s)), "sim_job_grads")
        return self._trim(g)

    def _trim(self, g):
        g["dw_edge"] = g["dw_edge"][:self.n_edges]
        g["dregion"] = g["dregion"][:self.n_regions]
        g["dmu"] = g["dmu"][:self.n_obstacles]
        g["dforce_scale"] = g["dforce_scale"][:max(self.T, 0)]
        return g

    def state(self, n: int):
        """Recorded (x_n, v_n) of the last forward pass."""
        x, v = self._vec(), self._vec()
        B.check(B.lib().sim_state(self.h, n, _dptr(x), _dptr(v)), "sim_state")
        return x, v

    def modes(self, n: int) -> np.ndarray:
        out = np.zeros(self.m, np.uint8)
        B.check(B.lib().sim_modes(self.h, n, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))), "sim_modes")
        return out

    def self_pairs(self, n: int) -> np.ndarray:
        """Node-node contact partner of every node at recorded step n (-1: none)."""
        out = np.zeros(self.m, np.int32)
        B.check(B.lib().sim_self_pairs(self.h, n, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))),
                "sim_self_pairs")
        return out

    def stats(self) -> dict:
        st = B.SimStats()
        B.check(B.lib().sim_stats(self.h, ctypes.byref(st)), "sim_stats")
        d = {name: getattr(st, name) for name, _ in B.SimStats._fields_}
        d["mode_counts"] = list(d["mode_counts"])
        return d

    def step_stats(self, n: int) -> dict:
        """PD iterations and contact-mode counts of recorded step n."""
        out = (ctypes.c_int32 * 4)()
        B.check(B.lib().sim_step_stats(self.h, int(n), out), "sim_step_stats")
        return dict(pd_iters=out[0], takeoff=out[1], stick=out[2], slip=out[3])

    def close(self):
        if getattr(self, "h", None):
            B.lib().sim_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_forward(sims: Sequence[Sim], n_steps: Sequence[int]):
    """One persistent launch over independent handles (one workgroup each)."""
    n = len(sims)
    hs = (ctypes.c_void_p * n)(*[s.h for s in sims])
    st = (ctypes.c_int32 * n)(*n_steps)
    outs = [(s._vec(), s._vec()) for s in sims]
    xs = (ctypes.c_void_p * n)(*[o[0].data_ptr() for o in outs])
    vs = (ctypes.c_void_p * n)(*[o[1].data_ptr() for o in outs])
    B.check(B.lib().sim_batch_forward(hs, n, st, xs, vs), "sim_batch_forward")
    for s, T in zip(sims, n_steps):
        s.T = T
        s._gen += 1
    return outs


def batch_backward(sims: Sequence[Sim], dL_dxT: Sequence[torch.Tensor]):
    n = len(sims)
    hs = (ctypes.c_void_p * n)(*[s.h for s in sims])
    seeds = [g.to(s.device, torch.float64).contiguous() for s, g in zip(sims, dL_dxT)]
    ds = (ctypes.c_void_p * n)(*[g.data_ptr() for g in seeds])
    gs, structs = zip(*[s._grads() for s in sims])
    arr = (B.SimGrads * n)(*structs)
    code = B.check(B.lib().sim_batch_backward(hs, n, ds, arr), "sim_batch_backward")
    out = []
    for s, g in zip(sims, gs):
        g["status"] = code
        out.append(s._trim(g))
    return out


def batch_advance(sims: Sequence[Sim], steps: Sequence[int], backward_stream: Optional[torch.cuda.Stream] = None):
    """Advance every handle's armed phase by up to steps[i] steps (forward chunks
    in one launch, backward chunks in another on backward_stream); returns the
    steps left in each handle's phase."""
    n = len(sims)
    hs = (ctypes.c_void_p * n)(*[s.h for s in sims])
    st = (ctypes.c_int32 * n)(*[int(k) for k in steps])
    left = (ctypes.c_int32 * n)()
    bs = None if backward_stream is None else ctypes.c_void_p(backward_stream.cuda_stream)
    B.check(B.lib().sim_batch_advance(hs, n, st, bs, left), "sim_batch_advance")
    return list(left)
