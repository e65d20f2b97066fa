"""torch.autograd.Function over N time steps with checkpoint/recompute.

Forward: from the rest state, run N steps of the library's forward kernels,
keeping the raw population state every K steps (device tensors) while the
library records the objective's terms; return J (FP64).  Backward: for each
K-step segment in reverse, the library restores the segment's checkpoint,
recomputes it onto a K+1-buffer tape and runs the hand-written adjoint
kernels backwards through it; the FP64 gradients with respect to the velocity
inlet's Fourier coefficients and the Brinkman field come back scaled by the
incoming gradient of J.  Memory: ceil(N/K) checkpoints plus K+1 tape buffers.
With K = 0 every state of the forward stays on the device instead (N + 1
population buffers) and the backward needs no recomputation; the gradients are
the same bits.  That record is kept only when a gradient is wanted; it is freed
by the backward, or by the handle's next forward, or by `lb.record_end()` when
the result is dropped without a backward.
"""

import dataclasses

import numpy as np
import torch


def _with_coefficients(io, theta):
    H = len(getattr(io, "cos", ()))
    th = [float(x) for x in theta]
    return dataclasses.replace(io, mean=th[0], cos=tuple(th[1:1 + H]), sin=tuple(th[1 + H:]))


class LBAdjointFn(torch.autograd.Function):
    """J = LBAdjointFn.apply(theta, alpha, lb, inlet, steps, K).

    theta: FP64 tensor [1 + 2H], the (mean, cos_1..H, sin_1..H) coefficients of
    velocity iolet `inlet`; alpha: tensor [N] (caller site order), the Brinkman
    field; lb: an `LB` handle with an objective set (`LB.set_objective`).
    """

    @staticmethod
    def forward(ctx, theta, alpha, lb, inlet, steps, K):
        th = theta.detach().to("cpu", torch.float64).numpy()
        lb.set_iolet(inlet, _with_coefficients(lb.iolets[inlet], th))
        lb.set_alpha(alpha.detach().to("cpu", torch.float32).numpy())
        lb.record_end()
        lb.set_deviations(torch.zeros((lb.q, lb.n), dtype=torch.float32, device="cuda"), t=0)
        checkpoints = []
        wanted = any(ctx.needs_input_grad[:2])
        if not wanted:
            lb.step(steps)
        elif K == 0:
            lb.record(steps)
            lb.step(steps)
        else:
            for t0 in range(0, steps, K):
                checkpoints.append((t0, min(K, steps - t0), lb.get_state()[0].clone()))
                lb.step(min(K, steps - t0))
        J, _, _ = lb.objective_value()
        ctx.lb, ctx.inlet, ctx.K, ctx.checkpoints = lb, inlet, K, checkpoints
        ctx.alpha_meta = (alpha.dtype, alpha.device)
        ctx.theta_meta = (theta.dtype, theta.device)
        return torch.tensor(J, dtype=torch.float64)

    @staticmethod
    def backward(ctx, gJ):
        lb = ctx.lb
        if ctx.K == 0:
            lb.adjoint_begin(1)
            lb.adjoint_recorded()
            dth, da = lb.adjoint_grads()
            lb.record_end()
        else:
            lb.adjoint_begin(ctx.K)
            lb.adjoint_run(ctx.checkpoints)
            dth, da = lb.adjoint_grads()
        g = float(gJ)
        dtheta = torch.from_numpy(dth[ctx.inlet] * g).to(dtype=ctx.theta_meta[0],
                                                          device=ctx.theta_meta[1])
        dalpha = torch.from_numpy(np.asarray(da) * g).to(dtype=ctx.alpha_meta[0],
                                                          device=ctx.alpha_meta[1])
        return dtheta, dalpha, None, None, None, None
