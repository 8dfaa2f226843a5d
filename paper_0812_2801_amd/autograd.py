"""torch.autograd.Function over the library's checkpointed adjoint.

``DipoleObjective.apply(ctrl, dv_coarse, system, psi0, every)`` runs the
frozen-ion AETRS trajectory on the GPU with field amplitudes ``ctrl[n]``
(float64, one per step) and the static potential interpolated from
``dv_coarse`` (an m^3 float64 grid), and returns the final dipole
J = h^3 sum (x - L/2) rho(T).  Its backward pass is the library's
hand-written adjoint: the trajectory is recomputed segment by segment from
checkpoints taken every ``every`` steps, and each step is reversed by
``me_adjoint_step``.  Gradients flow to ``ctrl`` and ``dv_coarse``.
"""
from __future__ import annotations

import torch


class DipoleObjective(torch.autograd.Function):
    @staticmethod
    def forward(ctx, ctrl, dv_coarse, system, psi0, every: int = 10):
        s = system
        n_steps = int(ctrl.shape[0])
        eps = [float(x) for x in ctrl.detach().cpu().tolist()]
        s.set_static_potential_coarse(dv_coarse.detach())
        s.set_state(psi0)
        ckpts = []
        for n in range(n_steps):
            if n % every == 0:
                buf = s.new_checkpoint()
                s.save_checkpoint(buf)
                ckpts.append(buf)
            s.step(ctrl=eps[n])
        J = s.dipole()
        ctx.system = s
        ctx.eps = eps
        ctx.ckpts = ckpts
        ctx.every = every
        ctx.m = int(dv_coarse.shape[0])
        ctx.dv_device = dv_coarse.device
        return torch.tensor(J, dtype=torch.float64)

    @staticmethod
    def backward(ctx, gJ):
        s = ctx.system
        eps, every = ctx.eps, ctx.every
        n_steps = len(eps)
        g_eps = torch.zeros(n_steps, dtype=torch.float64)
        s.adjoint_begin()
        seg_bufs = [s.new_checkpoint() for _ in range(min(every, n_steps))]
        for seg in range(len(ctx.ckpts) - 1, -1, -1):
            n0 = seg * every
            n1 = min(n0 + every, n_steps)
            # recompute the segment, keeping the state at the start of each step
            s.load_checkpoint(ctx.ckpts[seg])
            for n in range(n0, n1):
                s.save_checkpoint(seg_bufs[n - n0])
                if n + 1 < n1:
                    s.step(ctrl=eps[n])
            for n in range(n1 - 1, n0 - 1, -1):
                s.load_checkpoint(seg_bufs[n - n0])
                g_eps[n] = s.adjoint_step(eps[n])
        g_v = s.adjoint_grad_v(ctx.m).to(ctx.dv_device)
        g = float(gJ)
        return g * g_eps, g * g_v, None, None, None
