"""Oracle adjoint: reverse-mode differentiation of the oracle itself.

The discrete adjoint of L and of the Shu-Osher stage is obtained by
torch.autograd through the plain operator (no hand-written transposes), so it
is an independent check of a hand-written adjoint.  Kinks follow one fixed
convention: d max(x, y) goes to x when x >= y, d|x| = +1 when x >= 0 (both are
written with torch.where in the operator).

Pinned by: the dot-product identity <lam, J v> = <J^T lam, v> with J v from
forward-mode (torch.func.jvp), and central finite differences of the rollout
loss (tests/test_oracle_adjoint.py).
"""

import torch

from .timestep import SSPRK33, kinetic_energy


def rhs_vjp(op, U, lam):
    """(dL/dU)^T lam at U."""
    U = U.detach().clone().requires_grad_(True)
    out = op.rhs(U)
    (g,) = torch.autograd.grad(out, U, grad_outputs=lam)
    return g


def rhs_jvp(op, U, v):
    """(dL/dU) v at U (forward mode)."""
    _, jv = torch.func.jvp(op.rhs, (U,), (v,))
    return jv


def rk_stage_vjp(op, Uk, lam_out, a, b, c_dt):
    """Adjoint of U_out = a U0 + b Uk + c_dt L(Uk):
    returns (lam_k, lam_0) = (b lam + c_dt (dL/dU)^T lam, a lam)."""
    return b * lam_out + c_dt * rhs_vjp(op, Uk, lam_out), a * lam_out


def rollout(op, U0, dt, nsteps):
    U = U0
    for _ in range(nsteps):
        Un = U
        for (a, b, c) in SSPRK33:
            U = a * Un + b * U + c * dt * op.rhs(U)
    return U


def loss(op, U0, dt, nsteps):
    """Kinetic energy (summed over the batch) after nsteps SSP-RK3 steps."""
    return kinetic_energy(op, rollout(op, U0, dt, nsteps))


def loss_grad(op, U0, dt, nsteps):
    U0 = U0.detach().clone().requires_grad_(True)
    val = loss(op, U0, dt, nsteps)
    (g,) = torch.autograd.grad(val, U0)
    return float(val), g
