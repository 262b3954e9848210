"""GPU parity of the Navier-Stokes (BR1) stage against the CPU FP64 oracle:
small meshes at N = 2, 3, 4 (ragged last workgroup), the full Taylor-Green
workload (16^3, N = 4), conservation, and the TGV viscous-dissipation identity
evaluated from the library's own right-hand sides."""

import math
import os

import numpy as np
import pytest
import torch

import dginputs as di
from oracle.timestep import rk_stage, tensor_weights
from helpers import (make_pair, to_gpu, from_gpu, rel_err, flux_scale, random_euler_state, rounding_spread,
                     spread_err, SPREAD_FACTOR)

pytestmark = pytest.mark.gpu
TWO_PI = 2 * math.pi
P = di.PRESETS["tgv3d"]


@pytest.mark.parametrize("N", [2, 3, 4])
def test_ns_rhs_parity_small(N):
    op, s = make_pair(3, N, (3, 4, 3), (0, 0, 0), (1.0, 1.2, 0.9), physics="navier_stokes",
                      mu=2e-2, prandtl=0.72)
    U = random_euler_state(op, 40 + N)
    ref = op.rhs(U)
    got = from_gpu(op, s.rhs(to_gpu(s, U)))
    assert rel_err(got, ref) < 1e-12


def test_ns_stage_parity_full_workload():
    op, s = make_pair(3, P["N"], P["nel"], P["lo"], P["hi"], physics="navier_stokes",
                      mu=P["mu"], prandtl=P["prandtl"])
    U = torch.tensor(di.taylor_green(op.mesh.coords(), mach=P["mach"]))[None]
    Ug = to_gpu(s, U)
    dt = s.dt_cfl(Ug, P["cfl"])
    # At Mach 0.1 the momentum and energy fluxes carry the mean pressure,
    # 700 times its variation, and the density rate of the initial state is
    # 1e-5 of the density flux: the right-hand side is a small difference of
    # large terms.  The bound is the oracle's own rounding spread at this
    # state (mirror images and axis relabellings: every sum in another
    # order), times SPREAD_FACTOR, where that exceeds 1e-12 of the result.
    ref, spread = rounding_spread(op.rhs, U, P["nel"], [(0,), (1,), (2,)], cycles=True)
    dU = s.rhs(Ug)
    err = spread_err(from_gpu(op, dU), ref, spread)
    print(f"TGV 16^3 N=4 BR1 rhs: spread {spread.numpy()}, err/bound {err:.3f}", flush=True)
    assert err < 1.0
    out = s.empty()
    s.rk_stage(None, Ug, out, 0.0, 1.0, dt)
    ref_stage = rk_stage(op, U, U, 0.0, 1.0, dt)
    # the stage adds dt L to U: its own rounding (half a unit of U) plus dt
    # times the right-hand side's bound
    floor = dt * SPREAD_FACTOR * spread + 2.0 ** -52 * U.reshape(1, 5, -1).abs().amax(dim=(0, 2))
    assert spread_err(from_gpu(op, out), ref_stage, floor / SPREAD_FACTOR) < 1.0
    # Conservation: the volume integrals of the momentum components telescope
    # to zero only up to rounding of the flux differences, whose size is the
    # flux scale times the domain volume, not the (small) integral of |dU|.
    I = s.integrals(dU)[:, :-1]
    vol = float(np.prod(np.subtract(P["hi"], P["lo"])))
    scale = np.maximum(s.integrals(dU.abs())[:, :-1], vol * flux_scale(op, U).numpy()[None])
    assert np.abs(I / scale).max() < 1e-13


def test_tgv_viscous_dissipation_on_gpu():
    """dE_k/dt of the viscous part at t = 0 equals -3/4 mu (rho = 1)."""
    from paper_2605_26388_amd import Solver
    nel = (8, 8, 8)
    ns = Solver(3, 4, nel, P["lo"], P["hi"], physics="navier_stokes", mu=P["mu"], prandtl=P["prandtl"])
    eu = Solver(3, 4, nel, P["lo"], P["hi"], physics="euler")
    X = ns.node_coords().cpu().numpy()
    U = torch.tensor(di.taylor_green(X, mach=P["mach"]))[None].to(ns.device).contiguous()
    dv = ns.rhs(U) - eu.rhs(U)          # viscous part of L(U)
    vel = U[:, 1:4] / U[:, 0:1]
    rate = (vel * dv[:, 1:4]).sum(1, keepdim=True)                     # u . d(m)/dt
    zero = torch.zeros_like(rate)
    tmp = torch.cat([rate, zero, zero, zero, torch.ones_like(rate)], 1).contiguous()
    # integrate u . dm/dt with the library's quadrature (first column)
    val = eu.integrals(tmp)[0, 0] / TWO_PI ** 3
    assert abs(val / (-0.75 * P["mu"]) - 1.0) < 1e-2
    assert float(dv[:, 0].abs().max()) < 1e-12


@pytest.mark.skipif(os.environ.get("DG_LONG", "0") != "1",
                    reason="full-length run (minutes of CPU oracle time): set DG_LONG=1")
def test_full_length_tgv_200_steps():
    """The Taylor-Green workload at its full size and length: 16^3, N = 4,
    200 SSP-RK3 steps, the library in FP64 and in the FP32 form against the
    oracle's FP64 run.  FP64: each of the 600 stages adds at most dt times
    the right-hand side's bound (16 oracle rounding spreads, about 1e-11 of
    the flux scale) plus a few units in the last place of U: 1e-10 of each
    variable's norm covers the run.  FP32: the stated 1e-4.  The momentum is
    measured as one vector (its z component starts at zero).  The workload
    states no CFL; it runs at 0.25 (at 0.5 the 3-D N = 4 operator is not
    stable under SSP-RK3)."""
    from oracle.timestep import ssprk33_step
    op, s64 = make_pair(3, P["N"], P["nel"], P["lo"], P["hi"], physics="navier_stokes",
                        mu=P["mu"], prandtl=P["prandtl"])
    _, s32 = make_pair(3, P["N"], P["nel"], P["lo"], P["hi"], physics="navier_stokes", precision="f32",
                       mu=P["mu"], prandtl=P["prandtl"])
    U = torch.tensor(di.taylor_green(op.mesh.coords(), mach=P["mach"]))[None]
    g64, g32 = to_gpu(s64, U), to_gpu(s32, U)
    dt = s64.dt_cfl(g64, P["cfl"])

    def err(got, ref):
        # norm-wise per variable; the momentum is one vector, its components
        # measured against the largest component's norm (m_z starts at zero)
        d = (got - ref).reshape(5, -1).abs().amax(dim=1)
        n = ref.reshape(5, -1).abs().amax(dim=1)
        n[1:4] = n[1:4].max()
        return float((d / n).max())

    for k in range(200):
        U = ssprk33_step(op, U, dt)
        s64.ssprk3_step(g64, dt)
        s32.ssprk3_step(g32, dt)
        if k % 50 == 49:
            print(f"step {k + 1}: FP64 {err(from_gpu(op, g64), U):.3e}, FP32 {err(from_gpu(op, g32), U):.3e} "
                  f"(per component: FP32 {rel_err(from_gpu(op, g32), U):.3e})", flush=True)
    e64, e32 = err(from_gpu(op, g64), U), err(from_gpu(op, g32), U)
    print(f"TGV 16^3 N=4 after 200 steps: FP64 {e64:.3e}, FP32 {e32:.3e}", flush=True)
    assert e64 < 1e-10
    assert e32 < 1e-4
