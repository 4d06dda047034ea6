"""Differentiable rollout of the Runge-Kutta solver for a probe objective.

``LesRollout.apply(f, Q0, solver, nsteps, dt, i_f, i_p, p_inf, mode)``
returns the time-integrated squared pressure fluctuation on the probe plane
i = i_p,

    J = sum_{n=1..nsteps} dt * sum_{j,k} (p(Q^n)_{i_p, j, k} - p_inf)^2,

for a constant source f (shape (5, nk, nj), device, float64) on the plane
i = i_f and the initial state Q0 (library layout).  The backward pass runs
the hand-written adjoint kernels through the C ABI (les_probe_objective with
a Qbar accumulation, les_adjoint_step) and returns dJ/df and dJ/dQ0.

Checkpointing: mode "stages" keeps the five stage inputs of every step on the
device (5 x 5 fields per step); mode "steps" keeps only Q^n per step and
recomputes the stage inputs of each step just before its adjoint.  dt is held
fixed over the rollout (it is not differentiated).

Only argument marshalling happens here; all arithmetic runs in the HIP
kernels of liblesmi.so.
"""
from __future__ import annotations

import torch


class LesRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f, Q0, solver, nsteps, dt, i_f, i_p, p_inf, mode="stages"):
        if mode not in ("stages", "steps"):
            raise ValueError("mode must be 'stages' or 'steps'")
        fe = solver.fe
        f = f.detach().contiguous()
        solver.set_forcing(f, i_f)
        Q = Q0.detach().clone()
        J = torch.zeros(1, dtype=torch.float64, device=Q.device)
        saved = []
        for _ in range(int(nsteps)):
            if mode == "stages":
                ck = torch.empty(25 * fe, dtype=torch.float64, device=Q.device)
                solver.rk_step(Q, dt, ckpt=ck)
                saved.append(ck)
            else:
                saved.append(Q.clone())
                solver.rk_step(Q, dt)
            solver.probe_objective(Q, i_p, p_inf, dt, J)
        ctx.solver, ctx.nsteps, ctx.dt, ctx.i_f, ctx.i_p, ctx.p_inf, ctx.mode = solver, int(nsteps), dt, i_f, i_p, p_inf, mode
        ctx.saved = saved
        ctx.Q_final = Q
        ctx.f = f
        return J[0].clone()

    @staticmethod
    def backward(ctx, Jbar):
        s = ctx.solver
        fe = s.fe
        dev = ctx.Q_final.device
        Qbar = torch.zeros(5 * fe, dtype=torch.float64, device=dev)
        fbar = torch.zeros_like(ctx.f)
        scratch = torch.zeros(1, dtype=torch.float64, device=dev)
        s.set_forcing(ctx.f, ctx.i_f)
        ck = None if ctx.mode == "stages" else torch.empty(25 * fe, dtype=torch.float64, device=dev)
        for n in range(ctx.nsteps, 0, -1):
            # the objective term of Q^n
            if n == ctx.nsteps:
                Qn = ctx.Q_final
            elif ctx.mode == "stages":
                Qn = ctx.saved[n][0:5 * fe]  # stage input Q^(0) of step n+1
            else:
                Qn = ctx.saved[n]
            s.probe_objective(Qn, ctx.i_p, ctx.p_inf, ctx.dt, scratch, Qbar)
            # reverse step n (from Q^{n-1})
            if ctx.mode == "stages":
                stages = ctx.saved[n - 1]
            else:
                Qs = ctx.saved[n - 1].clone()
                s.rk_step(Qs, ctx.dt, ckpt=ck)
                stages = ck
            s.adjoint_step(stages, ctx.dt, Qbar, fbar)
        g = Jbar.to(torch.float64)
        return fbar * g, Qbar * g, None, None, None, None, None, None, None


def objective(solver, f, Q0, nsteps, dt, i_f, i_p, p_inf):
    """J without gradient bookkeeping (for finite differences)."""
    solver.set_forcing(f.contiguous(), i_f)
    Q = Q0.clone()
    J = torch.zeros(1, dtype=torch.float64, device=Q.device)
    for _ in range(int(nsteps)):
        solver.rk_step(Q, dt)
        solver.probe_objective(Q, i_p, p_inf, dt, J)
    return float(J.item())
