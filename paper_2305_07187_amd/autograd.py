"""torch.autograd.Function over the adjoint entry point of the C ABI.

SpringIsingRelaxedEnergy.apply(J, x0, p0, dt_sched, zeta_sched, ckpt_every)
returns the relaxed end-energy (1/R) sum_r -1/2 q_r^T J q_r of the final
positions after len(dt_sched) paper-order steps from (x0, p0); its backward
supplies gradients for dt_sched and zeta_sched only.  The HIP library
computes the loss and both gradients in one call (checkpointed reverse
sweep) when the forward runs; backward scales them by the incoming grad.
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
        try:
            model.set_schedule(dt_sched.detach().float().contiguous(),
                               zeta_sched.detach().float().contiguous())
            loss, g_dt, g_z = model.relaxed_energy_grad(ckpt_every)
            torch.cuda.current_stream().synchronize()
        finally:
            model.close()
        ctx.save_for_backward(g_dt, g_z)
        ctx.dtypes = (dt_sched.dtype, zeta_sched.dtype)
        return loss[0]

    @staticmethod
    def backward(ctx, grad_out):
        g_dt, g_z = ctx.saved_tensors
        gd = (grad_out.to(torch.float64) * g_dt).to(ctx.dtypes[0])
        gz = (grad_out.to(torch.float64) * g_z).to(ctx.dtypes[1])
        return None, None, None, gd, gz, None


def relaxed_energy(J, x0, p0, dt_sched, zeta_sched, ckpt_every=100):
    return SpringIsingRelaxedEnergy.apply(J, x0, p0, dt_sched, zeta_sched, ckpt_every)
