"""Pins of the oracle adjoint: the dot-product identity against forward-mode
derivatives, and central finite differences of the rollout loss."""

import math

import numpy as np
import pytest
import torch

import dginputs as di
from oracle import adjoint
from oracle.dgsem import Operator
from oracle.mesh import cartesian_mesh
from oracle.physics import Euler
from oracle.timestep import dt_cfl


def small_op(dim):
    if dim == 2:
        m = cartesian_mesh(2, 3, (3, 3), (0, 0), (2 * math.pi, 2 * math.pi))
    else:
        m = cartesian_mesh(3, 2, (2, 2, 2), (0, 0, 0), (2 * math.pi,) * 3)
    return Operator(m, Euler(dim))


def state(op, B=2):
    X = op.mesh.coords()
    base = di.random_euler(X, op.mesh.lo, op.mesh.hi)
    return torch.tensor(np.stack([di.perturb_density(base, b) for b in range(B)]))


@pytest.mark.parametrize("dim", [2, 3])
def test_dot_product_identity(dim):
    op = small_op(dim)
    U = state(op)
    g = torch.Generator().manual_seed(3)
    lam = torch.randn(U.shape, generator=g, dtype=torch.float64)
    v = torch.randn(U.shape, generator=g, dtype=torch.float64)
    Jv = adjoint.rhs_jvp(op, U, v)
    JTl = adjoint.rhs_vjp(op, U, lam)
    a = float((lam * Jv).sum())
    b = float((JTl * v).sum())
    assert abs(a - b) <= 1e-12 * (abs(a) + abs(b))


def test_rollout_gradient_central_differences():
    op = small_op(3)
    U0 = state(op)
    dt = dt_cfl(op, U0, 0.5)
    nsteps = 3
    val, g = adjoint.loss_grad(op, U0, dt, nsteps)
    gen = torch.Generator().manual_seed(9)
    for _ in range(3):
        d = torch.randn(U0.shape, generator=gen, dtype=torch.float64)
        d = d / d.norm()
        eps = 1e-5 * float(U0.norm())
        with torch.no_grad():
            fp = float(adjoint.loss(op, U0 + eps * d, dt, nsteps))
            fm = float(adjoint.loss(op, U0 - eps * d, dt, nsteps))
        fd = (fp - fm) / (2 * eps)
        ad = float((g * d).sum())
        assert abs(fd - ad) <= 1e-6 * abs(ad), (fd, ad)
