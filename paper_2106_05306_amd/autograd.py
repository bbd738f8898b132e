"""A whole rollout as one differentiable PyTorch operation.

``rollout`` runs the forward simulation in the HIP kernels and records the
trajectory (or its checkpoints) in the handle; its backward runs the adjoint
pass of the paper (Sec. 4) in the HIP kernels and maps the handle's gradients
to the inputs:

  x0, v0          dL/dx_0, dL/dv_0 (the adjoint's final state gradients);
  edge_stiffness  dL/dk_e = dL/dw_e * s_r(e): spring e has weight
                  w_e = k_e * s_r(e) with s the region scales (1 without regions);
  bend_weight     dL/dw_b summed over the bending constraints, each scaled by
                  its region scale;
  region_scale    dL/ds_r = sum over the constraints c of region r of
                  dL/dw_c * (base weight of c);
  mu              dL/dmu per obstacle;
  force           dL/dF of the external force field (m, 3);
  force_scale     dL/ds_n of its per-step multipliers (T,): node j receives
                  force_scale[n] * force[j] during step n (Sec. 3.1, f_ext).
                  A parametric wind model (a gust profile, a direction, per-node
                  coefficients) is written in PyTorch on top of these two and
                  its parameters' gradients follow by autograd.

Material inputs (stiffness, bending weight, region scales, friction) are sent
to the handle with ``Sim.set_material`` before the forward pass, which
refactors the PD matrix on the handle's ordering.
"""
from __future__ import annotations

from typing import Optional

import numpy as np
import torch

from .sim import Sim


def _host(t):
    return None if t is None else t.detach().to("cpu", torch.float64).numpy()


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, sim: Sim, n_steps: int, trajectory: bool, x0, v0, edge_stiffness, bend_weight, region_scale,
                mu, force, force_scale):
        if any(t is not None for t in (edge_stiffness, bend_weight, region_scale, mu)):
            sim.set_material(_host(edge_stiffness), _host(bend_weight), _host(region_scale), _host(mu))
        if force is not None:
            sim.set_external_force(force.detach(), _host(force_scale))
        elif force_scale is not None:
            raise ValueError("force_scale needs a force field")
        sim.set_state(None if x0 is None else x0.detach(), None if v0 is None else v0.detach())
        xT, vT, traj = sim.forward(n_steps, trajectory=trajectory)
        ctx.sim = sim
        ctx.gen = sim._gen
        ctx.trajectory = trajectory
        ins = (x0, v0, edge_stiffness, bend_weight, region_scale, mu, force, force_scale)
        ctx.has = [t is not None for t in ins]
        ctx.dtypes = [None if t is None else (t.dtype, t.device) for t in ins]
        if trajectory:
            return xT, vT, traj
        return xT, vT

    @staticmethod
    def backward(ctx, *grads):
        sim: Sim = ctx.sim
        if sim._gen != ctx.gen:
            raise RuntimeError("the handle ran another rollout after this one was recorded; "
                               "use one handle per live graph")
        gxT, gvT = grads[0], grads[1]
        gsteps = grads[2] if ctx.trajectory else None
        z = torch.zeros((sim.m, 3), dtype=torch.float64, device=sim.device)
        out = sim.backward(z if gxT is None else gxT, gvT, gsteps)
        if out["status"] == 3:                  # SIM_WADJ_NONFINITE
            raise FloatingPointError("the rollout's adjoint overflowed (non-finite gradients); the forward "
                                     "steps are probably far from converged (raise pd_iters or set fwd_tol)")
        res = [None] * 8
        if ctx.has[0]:
            res[0] = out["dx0"]
        if ctx.has[1]:
            res[1] = out["dv0"]
        scale_e = scale_b = None
        if sim.region_scale is not None:
            rs = torch.as_tensor(sim.region_scale, dtype=torch.float64, device=sim.device)
            scale_e = rs[torch.as_tensor(sim.edge_region, device=sim.device)]
            scale_b = rs[torch.as_tensor(sim.bend_region, device=sim.device)]
        if ctx.has[2]:
            res[2] = out["dw_edge"] * (1.0 if scale_e is None else scale_e)
        if ctx.has[3]:
            res[3] = (out["dw_bend"] * (1.0 if scale_b is None else scale_b)).sum().reshape(1)
        if ctx.has[4]:
            res[4] = out["dregion"]
        if ctx.has[5]:
            res[5] = out["dmu"]
        if ctx.has[6]:
            res[6] = out["dforce"]
        if ctx.has[7]:
            res[7] = out["dforce_scale"]
        for i, (r, dd) in enumerate(zip(res, ctx.dtypes)):
            if r is not None:
                res[i] = r.to(dtype=dd[0], device=dd[1])
        ctx.status = out["status"]
        return (None, None, None, *res)


def rollout(sim: Sim, n_steps: int, x0: Optional[torch.Tensor] = None, v0: Optional[torch.Tensor] = None, *,
            edge_stiffness: Optional[torch.Tensor] = None, bend_weight: Optional[torch.Tensor] = None,
            region_scale: Optional[torch.Tensor] = None, mu: Optional[torch.Tensor] = None,
            force: Optional[torch.Tensor] = None, force_scale: Optional[torch.Tensor] = None,
            trajectory: bool = False):
    """Differentiable rollout of ``n_steps`` from (x0, v0) (None: rest shape,
    zero velocity).  Returns (x_T, v_T) or, with ``trajectory``, (x_T, v_T,
    x_0..x_T).  ``bend_weight`` is a one-element tensor.  The handle keeps
    one recorded rollout: back-propagate before running it again."""
    return _Rollout.apply(sim, int(n_steps), bool(trajectory), x0, v0, edge_stiffness, bend_weight, region_scale,
                          mu, force, force_scale)
