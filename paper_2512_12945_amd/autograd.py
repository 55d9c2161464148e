"""torch.autograd.Function over the library's map loss and its hand-written
backward (include/slimvdb.h: slim_integrate_rays, slim_map_loss,
slim_backward_rays).  Argument marshalling only; the forward integration, the
loss and the gradients all run in the library's HIP kernels."""
from __future__ import annotations

import torch

from . import slimvdb as sv


class MapLoss(torch.autograd.Function):
    """Loss of a closed-set map integrated from F frames of rays.

    forward(ranges (F, N), logits (F, N, K), dirs (F, N, 3), poses [F x 4x4],
            gmap, keys (M, 3) int32, labels (M,) int32, samples (S, 3), alpha0)
    resets `gmap`, integrates the frames in order, and returns the scalar loss
    (cross-entropy of the Dirichlet predictive at the true class, averaged over
    the map's voxels, plus the mean |D| at the surface samples).  `keys` must be
    all voxels the frames create (from an extract of the same inputs).  The
    backward gives dL/dranges and dL/dlogits.
    """

    @staticmethod
    def forward(ctx, ranges, logits, dirs, poses, gmap, keys, labels, samples, alpha0=1.0):
        gmap.reset()
        for f in range(ranges.shape[0]):
            gmap.integrate_rays(ranges[f], dirs[f], poses[f], logits[f], sv.IN_LOGIT_F32)
        out = gmap.loss(keys, labels, samples, alpha0)
        ctx.gmap = gmap
        ctx.poses = poses
        ctx.save_for_backward(ranges, logits, dirs)
        ctx.mark_non_differentiable(out)
        return out[0].clone(), out

    @staticmethod
    def backward(ctx, g_loss, g_terms):
        ranges, logits, dirs = ctx.saved_tensors
        grad_logits = torch.empty_like(logits)
        grad_ranges = torch.empty_like(ranges)
        scale = g_loss.detach().reshape(1).to(torch.float32).contiguous()
        for f in range(ranges.shape[0]):
            ctx.gmap.backward_rays(ranges[f], dirs[f], ctx.poses[f], logits[f], grad_logits[f], grad_ranges[f],
                                   grad_scale=scale)
        return grad_ranges, grad_logits, None, None, None, None, None, None, None


def map_loss(ranges, logits, dirs, poses, gmap, keys, labels, samples, alpha0=1.0):
    """Scalar loss with gradients w.r.t. ranges and logits (see MapLoss)."""
    loss, _ = MapLoss.apply(ranges, logits, dirs, poses, gmap, keys, labels, samples, alpha0)
    return loss
