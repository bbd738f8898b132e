"""MI355X (gfx950) implementation of the DiffCloth hot path.

Projective Dynamics cloth with dry frictional contact, forward and adjoint,
as HIP kernels behind the C ABI in include/diffcloth.h.  The Python layer
only marshals arguments; PyTorch provides device memory and streams.
"""
from ._binding import (MODE_FREE, MODE_SLIP, MODE_STICK, MODE_TAKEOFF, SIM_FP64, SIM_MIXED, SIM_PLANE, SIM_SPHERE,
                       SimError, lib)

__all__ = ["lib", "SimError", "Sim", "batch_forward", "batch_backward", "rollout", "SIM_PLANE", "SIM_SPHERE", "SIM_FP64",
           "SIM_MIXED", "MODE_FREE", "MODE_TAKEOFF", "MODE_STICK", "MODE_SLIP"]


def __getattr__(name):
    # torch-dependent front end, imported on first use
    if name in ("Sim", "batch_forward", "batch_backward"):
        from . import sim as _sim
        return getattr(_sim, name)
    if name == "rollout":
        from .autograd import rollout
        return rollout
    raise AttributeError(name)
