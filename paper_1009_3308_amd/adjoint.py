"""Gradients through a trajectory of NDF_p steps (eq. (ode_disc)) with checkpoints.

`trajectory(sphere, alpha0, forcing, nsteps)` runs nsteps of nse_step from the
history [alpha0, 0, ..., 0] and returns the final state as a torch tensor that
takes part in autograd. Its backward pass is the discrete adjoint: the
history is kept only every `checkpoint_every` steps during the forward run;
each segment is recomputed forward from its checkpoint into a trajectory
buffer (nse_step_trajectory, which keeps every intermediate history in place),
then swept backward over that buffer (nse_step_adjoint_trajectory). Both
replay captured graphs for the fixed-coefficient steps, and one buffer serves
every segment. Every step and every adjoint step runs in the HIP library; this
module only schedules the segments and keeps the checkpoints.

Gradients follow torch's convention for complex tensors and a real loss,
dL/dRe + i dL/dIm, which is the vector-Jacobian product on the stored
(re, im) doubles that the library computes.
"""
from __future__ import annotations

import torch


class _Trajectory(torch.autograd.Function):
    @staticmethod
    def forward(ctx, alpha0, sphere, forcing, nsteps, step0, every):
        hist = sphere.new_history()
        hist[0] = alpha0.detach()
        checkpoints = []
        for s in range(0, nsteps, every):
            n = min(every, nsteps - s)
            checkpoints.append((s, n, hist.clone()))
            sphere.step(hist, forcing, step0 + s, n)
        ctx.sphere, ctx.forcing, ctx.step0 = sphere, forcing, step0
        ctx.checkpoints = checkpoints
        return hist[0].clone()

    @staticmethod
    def backward(ctx, grad_final):
        sphere, forcing, step0 = ctx.sphere, ctx.forcing, ctx.step0
        hist_bar = sphere.new_history()
        hist_bar[0] = grad_final
        trajs = {}
        for s, n, start in reversed(ctx.checkpoints):
            if n not in trajs:
                trajs[n] = sphere.new_trajectory(n)
            tr = trajs[n]
            tr[n:] = start
            sphere.step_trajectory(tr, forcing, step0 + s, n)
            sphere.step_adjoint_trajectory(tr, forcing, step0 + s, n, hist_bar)
        ctx.checkpoints = None
        return hist_bar[0].clone(), None, None, None, None, None


def trajectory(sphere, alpha0, forcing, nsteps: int, step0: int = 0,
               checkpoint_every: int = 20):
    """Final state after nsteps NDF_p steps from [alpha0, 0, ...], differentiable in alpha0.

    Requires a context built with newton_iters == 1 (the library rejects the
    step adjoint otherwise). The forcing is held fixed (not differentiated).
    """
    if nsteps < 1:
        raise ValueError("nsteps must be >= 1")
    if checkpoint_every < 1:
        raise ValueError("checkpoint_every must be >= 1")
    return _Trajectory.apply(alpha0, sphere, forcing, int(nsteps), int(step0),
                             int(checkpoint_every))
