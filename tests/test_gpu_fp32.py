"""Accuracy statement of the FP32 form against the CPU FP64 oracle.

Two errors are stated for the right-hand side, per variable and norm-wise:
  * arithmetic: the FP32 kernel against the oracle evaluated at the same
    (float-rounded) state -- what the kernel's own arithmetic costs
    (target 1e-5);
  * end to end: against the oracle at the original double state, which adds
    the quantisation of the state to float storage.
The state after 100 SSP-RK3 steps is compared with the oracle's FP64 run
(target 1e-4)."""

import math

import numpy as np
import pytest
import torch

import dginputs as di
from oracle.timestep import ssprk33_step, dt_cfl
from helpers import make_pair, to_gpu, from_gpu, rel_err, rel_err_floor, flux_scale, smooth_euler_state

pytestmark = pytest.mark.gpu


def statement(op, s, U, name, floor=None):
    Uq = U.float().double()
    got = from_gpu(op, s.rhs(to_gpu(s, Uq)))
    err = (lambda a, b: rel_err(a, b)) if floor is None else (lambda a, b: rel_err_floor(a, b, floor))
    e_arith = err(got, op.rhs(Uq))
    e_total = err(got, op.rhs(U))
    print(f"FP32 RHS {name}: arithmetic {e_arith:.3e}, end to end {e_total:.3e}")
    return e_arith, e_total


def test_fp32_rhs_euler_workload():
    p = di.PRESETS["euler3d"]
    op, s = make_pair(3, 3, p["nel"], p["lo"], p["hi"], precision="f32")
    a, t = statement(op, s, smooth_euler_state(op), "3-D Euler 32^3 N=3")
    assert a < 1e-5
    assert t < 1e-4


def test_fp32_state_after_100_steps():
    p = di.PRESETS["euler3d"]
    op, s = make_pair(3, 3, (8, 8, 8), p["lo"], p["hi"], precision="f32")
    U = smooth_euler_state(op)
    dt = dt_cfl(op, U, p["cfl"])
    Ug = to_gpu(s, U)
    for _ in range(100):
        U = ssprk33_step(op, U, dt)
        s.ssprk3_step(Ug, dt)
    err = rel_err(from_gpu(op, Ug), U)
    print(f"FP32 state error after 100 SSP-RK3 steps (3-D Euler 8^3 N=3): {err:.3e}")
    assert err < 1e-4


def test_fp32_rhs_navier_stokes():
    p = di.PRESETS["tgv3d"]
    op, s = make_pair(3, 4, (8, 8, 8), p["lo"], p["hi"], physics="navier_stokes", precision="f32",
                      mu=p["mu"], prandtl=p["prandtl"])
    U = torch.tensor(di.taylor_green(op.mesh.coords(), mach=p["mach"]))[None]
    # Mach 0.1: the mean pressure sits in the momentum and energy fluxes;
    # errors are stated relative to the flux scale where the result is small
    a, t = statement(op, s, U, "Navier-Stokes TGV 8^3 N=4", floor=1e-4 * flux_scale(op, U))
    assert a < 1e-5


def test_fp32_rhs_reacting():
    P = di.PRESETS["air5_2d"]
    mech = di.air5_mechanism(P["mech_seed"])
    op, s = make_pair(2, 3, (16, 16), P["lo"], P["hi"], physics="reacting", precision="f32",
                      patch=((6, 6), (10, 10)), mech=mech)
    U = torch.tensor(di.reacting_state(op.mesh.coords(), P["lo"], P["hi"], mech))[None]
    a, t = statement(op, s, U, "reacting 2-D 16^2+patch", floor=1e-4 * flux_scale(op, U))
    assert a < 1e-5
