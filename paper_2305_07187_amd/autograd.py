"""torch.autograd.Function over the adjoint entry points of the C ABI.

SpringIsingRelaxedEnergy.apply(J, x0, p0, dt_sched, zeta_sched, ckpt_every)
returns the relaxed end-energy (1/R) sum_r -1/2 q_r^T J q_r of the final
positions after len(dt_sched) paper-order steps from (x0, p0); its backward
supplies gradients for dt_sched and zeta_sched only.  The forward runs the
checkpointed forward half in the HIP library and keeps the context (its
checkpoints and the seed of the reverse sweep) on the autograd node; the
reverse sweep runs only when backward is called, and the context is released
there.  When neither schedule requires a gradient the forward releases it at
once.
"""
from __future__ import annotations

import torch

from . import spring_ising as si


class SpringIsingRelaxedEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, J, x0, p0, dt_sched, zeta_sched, ckpt_every=100):
        S = int(dt_sched.numel())
        model = si.SpringIsing(J.detach().float().contiguous(), x0.detach().float().contiguous(),
                               None if p0 is None else p0.detach().float().contiguous(),
                               total_steps=S)
        keep = False
        try:
            model.set_schedule(dt_sched.detach().float().contiguous(),
                               zeta_sched.detach().float().contiguous())
            loss = model.relaxed_energy_forward(ckpt_every)
            torch.cuda.current_stream().synchronize()
            keep = ctx.needs_input_grad[3] or ctx.needs_input_grad[4]
        finally:
            if not keep:
                model.close()
        ctx.model = model if keep else None
        ctx.dtypes = (dt_sched.dtype, zeta_sched.dtype)
        return loss[0]

    @staticmethod
    def backward(ctx, grad_out):
        model, ctx.model = ctx.model, None
        if model is None:
            raise RuntimeError("SpringIsingRelaxedEnergy: backward called twice, or the "
                               "schedules did not require gradients")
        try:
            g_dt, g_z = model.relaxed_energy_backward()
        finally:
            model.close()  # waits for the context's stream
        gd = (grad_out.to(torch.float64) * g_dt).to(ctx.dtypes[0])
        gz = (grad_out.to(torch.float64) * g_z).to(ctx.dtypes[1])
        return None, None, None, gd, gz, None


def relaxed_energy(J, x0, p0, dt_sched, zeta_sched, ckpt_every=100):
    return SpringIsingRelaxedEnergy.apply(J, x0, p0, dt_sched, zeta_sched, ckpt_every)
