"""torch.autograd bridge for the rollout adjoint (pi_rollout_adjoint).

J = PI2RHAdjoint.apply(u_nom, centre, metric, prob, model) returns the mean
rollout cost with the noise held fixed; J.backward() yields dJ/du_nom,
dJ/dcentre and dJ/dmetric.  The library computes J and all three gradients in
one fused forward + reverse pass, so the forward saves the gradients and the
backward only scales them by the incoming gradient.  (pi_rollout_adjoint also
takes that seed, gJ, as a device scalar; it is unknown when autograd's forward
runs the fused pass, so here the scaling happens in backward.)
"""
from __future__ import annotations

import copy

import torch

from . import DeviceModel, DeviceProblem, rollout_adjoint


class PI2RHAdjoint(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u_nom, centre, metric, prob: DeviceProblem, model: DeviceModel, ckpt_every=0):
        m = copy.copy(model)
        m.centre = centre.detach().contiguous()
        m.metric = metric.detach().contiguous()
        J, gu, gc, gD = rollout_adjoint(prob, m, u_nom=u_nom.detach().contiguous(),
                                        ckpt_every=int(ckpt_every))
        ctx.save_for_backward(gu, gc, gD)
        return J.reshape(())

    @staticmethod
    def backward(ctx, gJ):
        gu, gc, gD = ctx.saved_tensors
        return (gJ.to(gu.dtype) * gu, gJ.to(gc.dtype) * gc, gJ.to(gD.dtype) * gD, None, None, None)
