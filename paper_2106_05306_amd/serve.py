"""Serving forward + gradient rollout requests by continuous batching.

Each request is one cloth rollout on a mesh of its own size: the forward
simulation, then the adjoint pass back to the initial state (gradients of a
centroid loss with respect to the initial state, stiffness and friction).

The server
  * admits a request when the device memory it needs fits the HBM budget
    (handles in flight plus idle cached handles; idle handles are evicted,
    least recently used first, to make room);
  * caches handles per mesh topology: a handle holds the factorised PD matrix
    of its mesh and material, so a request whose topology is cached skips the
    setup (ordering, factorisation, device tables);
  * prepares the handle of a request whose topology is not cached on worker
    threads: the host part (constraint tables, ordering, Cholesky
    factorisation: ``Plan``) makes no GPU call, so rounds of the requests
    already admitted keep running meanwhile; the device part (uploads) runs
    on the serving thread between rounds, so no two threads drive the GPU.
    The request is admitted at the first round after its plan is ready
    (requests behind it whose handles are ready go first), while a request
    waiting for memory holds back the ones behind it;
  * runs rounds: one ``batch_advance`` call advances every admitted request by
    a chunk of steps of its current phase (forward chunks in one persistent
    launch, adjoint chunks in another on a second stream), chunks sized so
    that a round takes about ``round_ms``; requests that arrive during a round
    join at the next one, and finished ones leave.

``run_sequential`` serves the same requests one at a time with the same
kernels (``sim_forward`` + ``sim_backward``), the plain GPU baseline.
"""
from __future__ import annotations

import collections
import concurrent.futures
import dataclasses
import time
from typing import Callable, Dict, List, Optional

import numpy as np
import torch

from .sim import Plan, Sim, batch_advance


@dataclasses.dataclass
class Request:
    rid: int
    key: tuple                      # mesh topology: requests with equal keys can share a handle
    steps: int
    arrival: float                  # seconds after the start of the run
    make_scene: Callable[[], object]


@dataclasses.dataclass
class Result:
    rid: int
    arrival: float
    admitted: float
    finished: float
    status: int
    grads: Optional[dict] = None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def _start(sim: Sim, scene):
    """The request's initial velocity and external force on a handle that may
    come from the cache (it keeps neither from its previous request)."""
    v0 = None if scene is None else getattr(scene, "v0", None)
    if v0 is not None and (np.asarray(v0) != 0).any():
        sim.set_state(None, torch.as_tensor(np.asarray(v0), dtype=torch.float64))
    else:
        sim.set_state(None, None)
    f = None if scene is None else getattr(scene, "force", None)
    if f is not None:
        sim.set_external_force(torch.as_tensor(np.asarray(f), dtype=torch.float64),
                               getattr(scene, "force_scale", None))
    elif sim._keep.get("force") is not None:
        sim.set_external_force(None)


def centroid_seed(scene, xT: torch.Tensor) -> torch.Tensor:
    """dL/dx_T of L = |centroid(x_T) - target|^2."""
    target = torch.as_tensor(scene.target, dtype=torch.float64, device=xT.device)
    d = xT.mean(dim=0) - target
    return (2.0 / xT.shape[0]) * d.expand_as(xT).contiguous()


def step_cost_ms(m: int, backward: bool) -> float:
    """Rough time of one step (forward: K = 20 PD iterations) for m nodes; only
    used to size the chunks of a round."""
    return 0.2 + 0.35 * m / 1000.0 if backward else 20 * (0.06 + 0.04 * m / 1000.0)


def _material(scene):
    """What a cached handle's factor and friction depend on besides the topology."""
    return (np.asarray(scene.edge_stiffness, np.float64).tobytes(), float(scene.bend_weight),
            np.asarray(scene.region_scale if scene.region_scale is not None else [], np.float64).tobytes(),
            tuple(float(o.mu) for o in scene.obstacles))


class _Handle:
    def __init__(self, sim: Sim, key, material=None):
        self.sim = sim
        self.key = key
        self.material = material
        self.last_used = 0.0
        self.base_bytes = sim.stats()["device_bytes"]

    def match(self, scene):
        """Give the handle the request's material (stiffness, bending weight,
        region scales, friction) if the handle last served another one."""
        mat = _material(scene)
        if mat != self.material:
            self.sim.set_material(edge_stiffness=scene.edge_stiffness, bend_weight=scene.bend_weight,
                                  region_scale=scene.region_scale, mu=[o.mu for o in scene.obstacles])
            self.material = mat

    def need_bytes(self, steps: int, window: int) -> int:
        """Device bytes of a rollout of `steps` steps whose adjoint runs in
        chunks of `window` steps (tables + records + step factors)."""
        st = self.sim.stats()
        m = st["n_nodes"]
        records = (steps + 1) * m * 48 + steps * m * 26
        factors = window * (st["adj_factor_bytes"] + 8 * (9 * m + 4 * st["n_constraints_active"] + 64))
        return self.base_bytes + records + factors


class Server:
    def __init__(self, device="cuda:0", hbm_budget_bytes: int = 64 << 30, round_ms: float = 40.0,
                 max_chunk: int = 64, keep_grads: bool = False, on_done: Optional[Callable] = None,
                 builders: int = 2, **sim_kw):
        self.device = torch.device(device)
        self.budget = int(hbm_budget_bytes)
        self.round_ms = round_ms
        self.max_chunk = max_chunk
        self.keep_grads = keep_grads
        self.on_done = on_done              # called with every finished Result (progress reporting)
        self.sim_kw = dict(sim_kw)
        self.pool: Dict[tuple, List[_Handle]] = collections.defaultdict(list)
        self.stream = torch.cuda.current_stream(self.device)   # every handle's stream (batched launches)
        self.bstream = torch.cuda.Stream(device=self.device)
        self.stats = collections.Counter()
        self.builder = concurrent.futures.ThreadPoolExecutor(max_workers=max(1, builders)) if builders else None
        self.orphans: List[concurrent.futures.Future] = []    # builds whose request took a cached handle

    def _chunk(self, m: int, backward: bool, steps: int) -> int:
        """Steps of one round for a rollout of m nodes (about round_ms of work)."""
        k = int(self.round_ms / step_cost_ms(m, backward))
        return max(1, min(k, self.max_chunk, steps))

    # ------------------------------------------------------------------ handles
    def _idle(self):
        return [h for hs in self.pool.values() for h in hs]

    def _used_bytes(self, busy):
        return sum(h.sim.stats()["device_bytes"] for h in self._idle()) + sum(b for _, b in busy)

    def _evict(self, need, busy) -> bool:
        idle = sorted(self._idle(), key=lambda h: h.last_used)
        while self._used_bytes(busy) + need > self.budget and idle:
            h = idle.pop(0)
            self.pool[h.key].remove(h)
            h.sim.close()
            self.stats["evicted"] += 1
        return self._used_bytes(busy) + need <= self.budget

    def _build(self, key, scene) -> _Handle:
        return _Handle(Sim.from_scene(scene, device=self.device, stream=self.stream, **self.sim_kw), key,
                       _material(scene))

    def _plan(self, key, scene):
        """Host part of a handle (worker thread: no GPU call)."""
        return key, Plan.from_scene(scene, **self.sim_kw), _material(scene)

    def _finish(self, planned) -> _Handle:
        """Device part of a planned handle (serving thread)."""
        key, plan, material = planned
        return _Handle(Sim.from_plan(plan, device=self.device, stream=self.stream), key, material)

    def _take_idle(self, key, scene):
        if self.pool[key]:
            self.stats["cache_hits"] += 1
            h = self.pool[key].pop()
            h.match(scene)
            return h
        return None

    def _acquire(self, req: Request, scene):
        h = self._take_idle(req.key, scene)
        if h is not None:
            return h
        self.stats["cache_misses"] += 1
        return self._build(req.key, scene)

    def _adopt_orphans(self):
        keep = []
        for f in self.orphans:
            if f.done():
                h = self._finish(f.result())
                self.pool[h.key].append(h)
            else:
                keep.append(f)
        self.orphans = keep

    # ------------------------------------------------------------------ serving
    def run(self, requests: List[Request]) -> List[Result]:
        queue = collections.deque(sorted(requests, key=lambda r: r.arrival))
        waiting = []                 # arrived, not admitted: [req, scene, handle or None, build future or None]
        active = []                  # [req, scene, handle, phase, bytes, admitted]
        results = []
        t0 = time.perf_counter()
        clock = lambda: time.perf_counter() - t0
        while queue or waiting or active:
            now = clock()
            while queue and queue[0].arrival <= now:
                req = queue.popleft()
                scene = req.make_scene()
                h = self._take_idle(req.key, scene)
                fut = None
                if h is None:
                    self.stats["cache_misses"] += 1
                    if self.builder is None:
                        h = self._build(req.key, scene)
                    else:
                        fut = self.builder.submit(self._plan, req.key, scene)
                waiting.append([req, scene, h, fut])
            self._adopt_orphans()
            # admission in arrival order: a request whose handle is still being
            # built lets the ones behind it pass; one waiting for memory does not
            still, blocked = [], False
            for item in waiting:
                req, scene, h, fut = item
                if not blocked and h is None:
                    h = self._take_idle(req.key, scene)     # a handle freed meanwhile
                    if h is not None:
                        if fut is not None:
                            self.orphans.append(fut)
                    elif fut is not None and fut.done():
                        h = self._finish(fut.result())
                    if h is not None:
                        item[2], item[3] = h, None
                if blocked or h is None:
                    still.append(item)
                    continue
                need = h.need_bytes(req.steps, self._chunk(h.sim.m, True, req.steps))
                busy = [(a[2], a[4]) for a in active]
                if not self._evict(need, busy) and active:
                    blocked = True                          # wait for memory to free up
                    self.pool[req.key].append(h)            # (counted as idle meanwhile)
                    item[2] = None
                    still.append(item)
                    continue
                _start(h.sim, scene)
                h.sim.job_forward(req.steps)
                active.append([req, scene, h, "fwd", need, clock()])
            waiting = still
            if not active:
                nxt = queue[0].arrival - clock() if queue else 0.05
                time.sleep(max(0.0, min(nxt, 0.005 if waiting else 0.05)))
                continue
            steps = [self._chunk(h.sim.m, phase == "bwd", req.steps) for req, scene, h, phase, _, _ in active]
            left = batch_advance([a[2].sim for a in active], steps, self.bstream)
            self.stats["rounds"] += 1
            keep = []
            for a, rem in zip(active, left):
                req, scene, h, phase, need, adm = a
                if rem > 0:
                    keep.append(a)
                elif phase == "fwd":
                    xT, _ = h.sim.state(req.steps)
                    h.sim.job_backward(centroid_seed(scene, xT))
                    a[3] = "bwd"
                    keep.append(a)
                else:
                    g = h.sim.job_grads()
                    if g["status"] == 3:            # gradients overflowed: served, reported
                        self.stats["nonfinite"] += 1
                    h.last_used = clock()
                    results.append(Result(req.rid, req.arrival, adm, clock(), int(g["status"]),
                                          g if self.keep_grads else None))
                    h.sim.trim()                    # an idle handle keeps only its tables and factor
                    self.pool[req.key].append(h)
                    if self.on_done:
                        self.on_done(results[-1])
            active = keep
        for f in self.orphans:
            f.result()
        self._adopt_orphans()
        return results

    def run_sequential(self, requests: List[Request]) -> List[Result]:
        """The same requests one at a time (same kernels, same handle cache)."""
        results = []
        t0 = time.perf_counter()
        clock = lambda: time.perf_counter() - t0
        for req in sorted(requests, key=lambda r: r.arrival):
            wait = req.arrival - clock()
            if wait > 0:
                time.sleep(wait)
            adm = clock()
            scene = req.make_scene()
            h = self._acquire(req, scene)
            self._evict(h.need_bytes(req.steps, req.steps), [])
            _start(h.sim, scene)
            xT, _, _ = h.sim.forward(req.steps)
            g = h.sim.backward(centroid_seed(scene, xT))
            torch.cuda.synchronize(self.device)
            h.last_used = clock()
            results.append(Result(req.rid, req.arrival, adm, clock(), int(g["status"]),
                                  g if self.keep_grads else None))
            h.sim.trim()
            self.pool[req.key].append(h)
            if self.on_done:
                self.on_done(results[-1])
        return results

    def close(self):
        for f in self.orphans:
            f.result()
        self._adopt_orphans()
        if self.builder is not None:
            self.builder.shutdown(wait=True)
        for h in self._idle():
            h.sim.close()
        self.pool.clear()


def latency_summary(results: List[Result]) -> dict:
    import numpy as np
    lat = np.array([r.latency for r in results])
    span = max(r.finished for r in results) - min(r.arrival for r in results)
    return {"requests": len(results), "rollouts_per_s": len(results) / span, "makespan_s": span,
            "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean())}
