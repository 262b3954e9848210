"""Differentiable SSP-RK3 rollout through the library.

DGRollout.apply(U0, solver, dt, nsteps, checkpoint) returns U_N after nsteps
Shu-Osher SSP-RK3 steps of the fused stage; its backward is the hand-written
discrete adjoint (dg_rk_stage_adjoint), three launches per step in reverse.

Checkpointing:
  "stages": every stage state (U^n, U1, U2) of every step is kept on the
            device; the backward pass only runs adjoint stages.
  "steps":  only U^n of every step is kept; the backward pass recomputes U1
            and U2 of a step from U^n (two forward stages) before its adjoint
            stages.
dt is a fixed float (not differentiated).  Only the initial state receives a
gradient.
"""

import torch


class DGRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U0, solver, dt, nsteps, checkpoint="stages"):
        if checkpoint not in ("stages", "steps"):
            raise ValueError("checkpoint must be 'stages' or 'steps'")
        U = U0.detach().clone().contiguous()
        saved = []
        for _ in range(int(nsteps)):
            U1, U2 = solver.empty(), solver.empty()
            Un = U.clone()
            solver.ssprk3_step(U, dt, U1, U2)
            saved.append((Un, U1, U2) if checkpoint == "stages" else (Un,))
        ctx.solver, ctx.dt, ctx.saved_states, ctx.checkpoint = solver, float(dt), saved, checkpoint
        return U

    @staticmethod
    def backward(ctx, gU):
        s, dt = ctx.solver, ctx.dt
        # lam and nxt swap roles every step and the reverse sweep writes into
        # nxt: both are the binding's own buffers, never the caller's gradient
        lam = gU.to(s.dtype, copy=True).contiguous()
        nxt = s.empty()
        acc, mu2, mu1 = s.empty(), s.empty(), s.empty()
        for st in reversed(ctx.saved_states):
            if ctx.checkpoint == "stages":
                states = st
            else:
                Un = st[0]
                U1, U2 = s.empty(), s.empty()
                s.rk_stage(None, Un, U1, 0.0, 1.0, dt)
                s.rk_stage(Un, U1, U2, 0.75, 0.25, 0.25 * dt)
                states = (Un, U1, U2)
            s.ssprk3_step_adjoint(states, dt, lam, nxt, acc, mu2, mu1)
            lam, nxt = nxt, lam
        ctx.saved_states = None
        return lam, None, None, None, None
