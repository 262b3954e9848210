"""Accuracy statement of the FP32 form against the CPU FP64 oracle.

Three numbers are stated for the right-hand side, per variable and norm-wise:
  * arithmetic: the FP32 kernel against the oracle evaluated at the same
    (float-rounded) state -- what the kernel's own arithmetic costs
    (target 1e-5, asserted);
  * quantisation floor: the oracle at the float-rounded state against the
    oracle at the double state -- what storing the state in float costs any
    implementation (the derivative sums amplify the 6e-8 rounding of the
    state by about (2/h) ||D|| |U| / |L|);
  * end to end: the kernel against the oracle at the double state, asserted
    at the target above that floor (at most floor + 1e-5).
The state after 100 SSP-RK3 steps is compared with the oracle's FP64 run
(target 1e-4)."""

import math
import os

import numpy as np
import pytest
import torch

import dginputs as di
from oracle.timestep import ssprk33_step, dt_cfl
from helpers import make_pair, to_gpu, from_gpu, rel_err, rel_err_floor, flux_scale, smooth_euler_state

pytestmark = pytest.mark.gpu
TARGET = 1e-5
LONG = os.environ.get("DG_LONG", "0") == "1"


def statement(op, s, U, name, floor=None):
    Uq = U.float().double()
    got = from_gpu(op, s.rhs(to_gpu(s, Uq)))
    err = (lambda a, b: rel_err(a, b)) if floor is None else (lambda a, b: rel_err_floor(a, b, floor))
    ref_q, ref = op.rhs(Uq), op.rhs(U)
    e_arith = err(got, ref_q)
    e_quant = err(ref_q, ref)
    e_total = err(got, ref)
    print(f"FP32 RHS {name}: arithmetic {e_arith:.3e}, quantisation floor {e_quant:.3e}, "
          f"end to end {e_total:.3e}", flush=True)
    assert e_arith < TARGET
    assert e_total <= e_quant + TARGET
    return e_arith, e_quant, e_total


def test_fp32_rhs_euler_workload():
    p = di.PRESETS["euler3d"]
    op, s = make_pair(3, 3, p["nel"], p["lo"], p["hi"], precision="f32")
    statement(op, s, smooth_euler_state(op), "3-D Euler 32^3 N=3")


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
    statement(op, s, U, "Navier-Stokes TGV 8^3 N=4", floor=1e-4 * flux_scale(op, U))


def test_fp32_rhs_reacting():
    P = di.PRESETS["air5_2d"]
    mech = di.preset_mechanism(P)
    op, s = make_pair(2, 3, (16, 16), P["lo"], P["hi"], physics="reacting", precision="f32",
                      patch=((6, 6), (10, 10)), mech=mech)
    U = torch.tensor(di.reacting_state(op.mesh.coords(), P["lo"], P["hi"], mech))[None]
    statement(op, s, U, "reacting 2-D 16^2+patch", floor=1e-4 * flux_scale(op, U))


@pytest.mark.skipif(not LONG, reason="full-length run (minutes of CPU oracle time): set DG_LONG=1")
def test_full_length_euler_workload_100_steps():
    """The 3-D Euler workload at its full size and length: 32^3, N = 3,
    100 SSP-RK3 steps at CFL 0.5, the library in FP64 and in the FP32 form
    against the oracle's FP64 run.  FP64: each of the 300 stages may differ
    by a few units in the last place of U (the right-hand side's own bound
    times dt is far below that), and the smooth flow does not amplify them:
    at most 1e-12.  FP32: the stated 1e-4."""
    p = di.PRESETS["euler3d"]
    op, s64 = make_pair(3, 3, p["nel"], p["lo"], p["hi"])
    _, s32 = make_pair(3, 3, p["nel"], p["lo"], p["hi"], precision="f32")
    U = smooth_euler_state(op)
    dt = dt_cfl(op, U, p["cfl"])
    g64, g32 = to_gpu(s64, U), to_gpu(s32, U)
    for k in range(100):
        U = ssprk33_step(op, U, dt)
        s64.ssprk3_step(g64, dt)
        s32.ssprk3_step(g32, dt)
        if k % 20 == 19:
            print(f"step {k + 1}: FP64 {rel_err(from_gpu(op, g64), U):.3e}, "
                  f"FP32 {rel_err(from_gpu(op, g32), U):.3e}", flush=True)
    e64, e32 = rel_err(from_gpu(op, g64), U), rel_err(from_gpu(op, g32), U)
    print(f"32^3 N=3 after 100 steps: FP64 {e64:.3e}, FP32 {e32:.3e}", flush=True)
    assert e64 < 1e-12
    assert e32 < 1e-4
    assert s64.status()["nonphysical"] == 0 and s32.status()["nonphysical"] == 0
