"""torch.autograd bridge for the interaction matrix's misregistration derivative.

``interaction_matrix(theta, ifs, wfs)`` builds the IM [n_act][2N] with the HIP
fused build; its backward pass is the hand-written vector-Jacobian-product
kernel (``synim_im_vjp``), which returns dL/dtheta for theta = (shift_x,
shift_y, rot, mag) without materialising the Jacobian.  theta is a CPU float64
tensor of 4 (the map is composed on the host in FP64); the IF stack is not
differentiated.
"""
from __future__ import annotations

import torch

from . import affine_from_misreg, im_build, im_vjp


class InteractionMatrix(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, ifs, wfs, kappa):
        if theta.device.type != "cpu" or theta.numel() != 4:
            raise ValueError("theta must be a CPU tensor of 4 values")
        H, W = wfs.shape
        A, dA = affine_from_misreg(theta.detach().double().tolist(), ifs.shape[1], ifs.shape[2],
                                   H, W, kappa)
        ctx.geom = (ifs, wfs, A, dA)
        ctx.theta_meta = (theta.dtype, theta.device)
        return im_build(ifs, A, wfs)

    @staticmethod
    def backward(ctx, grad_im):
        ifs, wfs, A, dA = ctx.geom
        g = im_vjp(ifs, A, dA, wfs, grad_im.detach().float().contiguous())
        dtype, device = ctx.theta_meta
        return g.to(device=device, dtype=dtype), None, None, None


def interaction_matrix(theta, ifs, wfs, kappa: float = 1.0):
    """IM [n_act][2N] as a differentiable function of theta (CPU float64 [4])."""
    return InteractionMatrix.apply(theta, ifs, wfs, float(kappa))
