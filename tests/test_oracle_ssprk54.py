"""Pins of the oracle's SSPRK54 table and positivity floor against what the
mathematics fixes: the fourth-order conditions of the Butcher tableau that
the Shu-Osher coefficients define, consistency (rows of alpha sum to 1,
alpha and beta non-negative), the SSP coefficient the paper quotes (1.508),
fourth-order convergence on a nonlinear ODE with a closed-form solution,
conservation and free stream through a DG step, and the floor's defining
properties."""

import math

import numpy as np
import pytest
import torch

import dginputs as di
from oracle.dgsem import Operator
from oracle.mesh import cartesian_mesh
from oracle.physics import Euler
from oracle.ssprk54 import ALPHA, BETA, STAGES, positivity_floor, ssprk54_step
from oracle.timestep import integrals

G = 1.4


def butcher():
    """A (5x5, stage k's derivative in stage i's value), b, c from the
    Shu-Osher form: U^(i) = U^n + dt sum_j A_ij L(U^(j)) with
    A_ij = sum_k alpha_ik A_kj + beta_ij."""
    A = np.zeros((STAGES + 1, STAGES))
    for i in range(1, STAGES + 1):
        for j in range(STAGES):
            A[i, j] = sum(ALPHA.get((i, k), 0.0) * A[k, j] for k in range(i)) + BETA.get((i, j), 0.0)
    b = A[STAGES].copy()
    A = A[:STAGES]
    return A, b, A.sum(axis=1)


def test_fourth_order_conditions():
    A, b, c = butcher()
    Ac = A @ c
    conds = {
        "b": (b.sum(), 1.0),
        "bc": (b @ c, 1 / 2),
        "bc2": (b @ c ** 2, 1 / 3),
        "bAc": (b @ Ac, 1 / 6),
        "bc3": (b @ c ** 3, 1 / 4),
        "bcAc": (b @ (c * Ac), 1 / 8),
        "bAc2": (b @ (A @ c ** 2), 1 / 12),
        "bAAc": (b @ (A @ Ac), 1 / 24),
    }
    for name, (got, want) in conds.items():
        assert abs(got - want) < 1e-13, (name, got, want)
    # explicit: strictly lower triangular
    assert np.allclose(np.triu(A), 0.0)
    # and not fifth order (the tableau is not accidentally a different method)
    assert abs(b @ c ** 4 - 1 / 5) > 1e-4


def test_consistency_and_ssp_coefficient():
    for i in range(1, STAGES + 1):
        assert abs(sum(ALPHA.get((i, k), 0.0) for k in range(i)) - 1.0) < 2e-15
    assert all(v >= 0 for v in ALPHA.values()) and all(v > 0 for v in BETA.values())
    ssp = min(ALPHA.get(key, 0.0) / v for key, v in BETA.items())
    assert abs(ssp - 1.508) < 5e-4, ssp


class _Cubic:
    """y' = -y^3, y(t) = (2t + y0^-2)^(-1/2)."""

    def rhs(self, y):
        return -y ** 3


def test_fourth_order_convergence_on_nonlinear_ode():
    y0 = torch.tensor([0.5, 1.0, 2.0], dtype=torch.float64)
    T = 1.0
    exact = (2 * T + y0 ** -2) ** -0.5
    errs = []
    for nsteps in (10, 20, 40):
        y, dt = y0.clone(), T / nsteps
        for _ in range(nsteps):
            y = ssprk54_step(_Cubic(), y, dt)
        errs.append(float((y - exact).abs().max()))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(3.7 < o < 4.5 for o in orders), (errs, orders)


def test_dg_step_conserves_and_keeps_free_stream():
    m = cartesian_mesh(2, 3, (6, 5), (-5, -5), (5, 5))
    op = Operator(m, Euler(2))
    U = torch.tensor(di.vortex(m.coords(), 0.0))[None]
    U1 = ssprk54_step(op, U, 0.05)
    I0, I1 = integrals(op, U, with_ke=False), integrals(op, U1, with_ke=False)
    assert np.abs(I1[:, :-1] - I0[:, :-1]).max() < 1e-12 * np.abs(I0[:, :-1]).max()
    c = torch.ones_like(U)
    c[:, 1] = 0.3
    c[:, 2] = -0.2
    c[:, 3] = 2.5 + 0.5 * (0.09 + 0.04)
    assert float((ssprk54_step(op, c, 0.05) - c).abs().max()) < 1e-13


def _pressure(U):
    m = U[:, 1:-1]
    return (G - 1) * (U[:, -1] - 0.5 * (m * m).sum(1) / U[:, 0])


def test_floor_leaves_admissible_states_untouched():
    rng = np.random.default_rng(0)
    n = 1000
    rho = rng.uniform(0.1, 2.0, n)
    vel = [rng.uniform(-1, 1, n) for _ in range(3)]
    p = rng.uniform(0.1, 2.0, n)
    U = torch.tensor(di.conserved_from_primitive(rho, vel, p, G))[None]
    assert torch.equal(positivity_floor(U, G, 1e-6, 5e-7), U)


def test_floor_enforces_the_bounds_and_nothing_else():
    rng = np.random.default_rng(1)
    n = 4000
    U = torch.tensor(rng.uniform(-1.0, 1.0, (1, 5, n)))
    U[:, 0] = torch.where(torch.tensor(rng.uniform(size=n) < 0.5), U[:, 0].abs() + 0.01, U[:, 0])
    rmin, pmin = 1e-3, 2e-3
    F = positivity_floor(U, G, rmin, pmin)
    assert torch.equal(F[:, 1:4], U[:, 1:4])                        # momentum untouched
    assert bool((F[:, 0] >= rmin).all())
    assert torch.equal(F[:, 0], torch.clamp(U[:, 0], min=rmin))
    pF = _pressure(F)
    assert bool((pF >= pmin * (1 - 1e-9)).all())
    low = _pressure(torch.cat([F[:, :1], U[:, 1:]], 1)) < pmin     # pressure below at the floored density
    assert bool(low.any()) and bool((~low).any())
    assert torch.allclose(pF[low], torch.full_like(pF[low], pmin), rtol=1e-9, atol=0)
    assert torch.equal(F[:, 4][~low], U[:, 4][~low])                 # energy raised only where needed
    FF = positivity_floor(F, G, rmin, pmin)
    assert torch.allclose(FF, F, rtol=1e-14, atol=1e-300)


def test_floored_step_equals_plain_step_on_admissible_flow():
    m = cartesian_mesh(2, 3, (6, 5), (-5, -5), (5, 5))
    op = Operator(m, Euler(2))
    U = torch.tensor(di.vortex(m.coords(), 0.0))[None]
    assert torch.equal(ssprk54_step(op, U, 0.05, floor=(1e-6, 5e-7)), ssprk54_step(op, U, 0.05))
