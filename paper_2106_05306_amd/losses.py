"""Losses of the workloads, in PyTorch (differentiated by autograd up to the
rollout's final state)."""
import torch


def centroid_distance2(x: torch.Tensor, target: torch.Tensor) -> torch.Tensor:
    """Squared distance of the node centroid of x [m, 3] to a target point."""
    d = x.mean(dim=0) - target
    return (d * d).sum()


def apex_angle(x: torch.Tensor, waist: torch.Tensor, hem: torch.Tensor) -> torch.Tensor:
    """Apex angle of a skirt about the vertical (y) axis: twice the angle
    whose tangent is the mean hem radius over the height of the mean waist
    above the mean hem."""
    r = torch.sqrt(x[hem, 0] ** 2 + x[hem, 2] ** 2).mean()
    height = x[waist, 1].mean() - x[hem, 1].mean()
    return 2.0 * torch.atan2(r, height)
