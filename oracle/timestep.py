"""Time stepping and reductions (SSP-RK Time Discretization appendix).

* Shu-Osher stage  U^(i) = a U0 + b U^(k) + c_dt L(U^(k)).
* "SSP-RK3" is read as the three-stage third-order method of Shu and Osher
  (SSP coefficient 1): (a, b, c) = (0, 1, 1), (3/4, 1/4, 1/4), (1/3, 2/3, 2/3),
  with c multiplied by dt.
* Time step (reading of the CFL bound): dt = CFL * h_min / ((2N+1) lam_max),
  lam_max = max over nodes of |u| + a, computed once from U^0; the parabolic
  bound dt_D = CFL * h_min^2 / ((2N+1)^2 nu_max), nu_max = max(mu/rho,
  mu/(Pr rho)), is combined by min.
* Integrals: sum_e J_e sum_i w_i U_i per variable and batch member, and the
  kinetic energy sum J w |m|^2/(2 rho), accumulated with math.fsum over
  per-element partials.
"""

import math

import numpy as np
import torch

SSPRK33 = ((0.0, 1.0, 1.0), (0.75, 0.25, 0.25), (1.0 / 3.0, 2.0 / 3.0, 2.0 / 3.0))


def rk_stage(op, U0, Uk, a, b, c_dt):
    return a * U0 + b * Uk + c_dt * op.rhs(Uk)


def ssprk33_step(op, U, dt):
    U1 = rk_stage(op, U, U, 0.0, 1.0, dt)
    U2 = rk_stage(op, U, U1, 0.75, 0.25, 0.25 * dt)
    return rk_stage(op, U, U2, 1.0 / 3.0, 2.0 / 3.0, 2.0 / 3.0 * dt)


def dt_cfl(op, U, cfl):
    N = op.N
    hmin = op.mesh.hmin()
    dt = cfl * hmin / ((2 * N + 1) * op.lam_max(U))
    if op.viscous is not None:
        P = op.phys.prims(U)
        mu, pr = op.viscous["mu"], op.viscous["prandtl"]
        nu = torch.maximum(mu / P["rho"], mu / (pr * P["rho"]))
        dtd = cfl * hmin ** 2 / ((2 * N + 1) ** 2 * float(nu.max()))
        dt = min(dt, dtd)
    return dt


def tensor_weights(op):
    """W_i = prod over directions of the 1-D weights, shape (n, .., n)."""
    w = op.w
    Wt = w
    for _ in range(op.dim - 1):
        Wt = Wt.unsqueeze(0) * w.reshape((-1,) + (1,) * Wt.dim())
    return Wt


def integrals(op, U, with_ke=True):
    """(B, nv+1) array: per-variable sum J w U and the kinetic energy (the last
    column is left 0 when with_ke is False, e.g. for a right-hand side)."""
    Wt = tensor_weights(op)
    J = op.J
    B, nv, E = U.shape[:3]
    out = np.zeros((B, nv + 1))
    red = tuple(range(1, 1 + op.dim))
    for b in range(B):
        for v in range(nv):
            per_el = (J.reshape(-1, *([1] * op.dim)) * Wt * U[b, v]).sum(dim=red)
            out[b, v] = math.fsum(per_el.tolist())
        if not with_ke:
            continue
        P = op.phys.prims(U[b:b + 1])
        ke = 0.5 * sum(P["m"][d] * P["u"][d] for d in range(op.dim))[0]
        per_el = (J.reshape(-1, *([1] * op.dim)) * Wt * ke).sum(dim=red)
        out[b, nv] = math.fsum(per_el.tolist())
    return out


def kinetic_energy(op, U):
    """Differentiable sum_b sum J w |m|^2/(2 rho) (loss of the adjoint case)."""
    Wt = tensor_weights(op)
    J = op.J.reshape((1, -1) + (1,) * op.dim)
    rho = U[:, 0]
    m2 = sum(U[:, 1 + d] ** 2 for d in range(op.dim))
    return (J * Wt * 0.5 * m2 / rho).sum()
