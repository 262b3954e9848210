"""GPU parity of the reacting-flow path: the 2-D reacting Euler stage with the
2:1 mortar patch, the chemistry source (mode 0) and the implicit source substep
(mode 1), and one Strang step, against the CPU FP64 oracle on the full
reacting workload (64^2 + refined 16^2 block, N=3, 5-species air)."""

import math
import os

import numpy as np
import pytest
import torch

import dginputs as di
from oracle import chem
from oracle.ssprk54 import ssprk54_step
from oracle.timestep import rk_stage, ssprk33_step, dt_cfl
from helpers import make_pair, to_gpu, from_gpu, rel_err

pytestmark = pytest.mark.gpu
P = di.PRESETS["air5_2d"]


def workload(nel=None, patch=None, moving=True):
    mech = di.preset_mechanism(P)
    nel = nel or P["nel"]
    patch = patch or (P["patch_lo"], P["patch_hi"])
    op, s = make_pair(2, 3, nel, P["lo"], P["hi"], physics="reacting", patch=patch, mech=mech)
    X = op.mesh.coords()
    U = torch.tensor(di.reacting_state(X, P["lo"], P["hi"], mech))[None]
    if moving:  # a smooth velocity field so every flux column is exercised
        rho = U[:, :5].sum(1)
        Xt = torch.tensor(X)
        u = 300.0 * torch.sin(math.pi * Xt[1])[None]
        v = 200.0 * torch.cos(math.pi * Xt[0])[None]
        U[:, 5] = rho * u
        U[:, 6] = rho * v
        U[:, 7] = U[:, 7] + 0.5 * rho * (u * u + v * v)
    return mech, op, s, U


def test_reacting_rhs_parity_small_and_conservative():
    mech, op, s, U = workload(nel=(10, 8), patch=((3, 2), (7, 5)))
    ref = op.rhs(U)
    dU = s.rhs(to_gpu(s, U))
    assert rel_err(from_gpu(op, dU), ref) < 1e-12
    I = s.integrals(dU)[:, :-1]
    scale = s.integrals(dU.abs())[:, :-1]
    assert np.abs(I / scale).max() < 1e-13


def test_reacting_stage_parity_full_workload():
    mech, op, s, U = workload()
    Ug = to_gpu(s, U)
    dt = s.dt_cfl(Ug, P["cfl"])
    assert abs(dt / dt_cfl(op, U, P["cfl"]) - 1.0) < 1e-13
    out = s.empty()
    s.rk_stage(None, Ug, out, 0.0, 1.0, dt)
    ref = rk_stage(op, U, U, 0.0, 1.0, dt)
    assert rel_err(from_gpu(op, out), ref) < 1e-12
    assert s.status()["nonphysical"] == 0


def test_source_mode0_parity_and_invariants():
    mech, op, s, U = workload(moving=False)
    Ug = to_gpu(s, U)
    out = torch.zeros_like(Ug)
    s.source_chem(Ug, out, 0.0, 0)
    ref = chem.source(mech, 2, U)
    got = from_gpu(op, out)
    # species rows against the oracle, per species norm-wise
    assert rel_err(got[:, :5], ref[:, :5]) < 1e-12
    assert float(got[:, 5:].abs().max()) == 0.0
    w = got[0, :5]
    assert float(w.sum(0).abs().max()) <= 1e-14 * float(w.abs().max())


def test_source_mode0_accumulates_in_place():
    mech, op, s, U = workload(nel=(8, 8), patch=((2, 2), (4, 4)))
    Ug = to_gpu(s, U)
    ref = U + chem.source(mech, 2, U)
    s.source_chem(Ug, Ug, 0.0, 0)
    assert rel_err(from_gpu(op, Ug), ref) < 1e-12


def test_implicit_substep_parity_full_workload():
    mech, op, s, U = workload(moving=False)
    Ug = to_gpu(s, U)
    dt = s.dt_cfl(Ug, P["cfl"])
    out = s.empty()
    s.status(reset=True)
    s.source_chem(Ug, out, 0.5 * dt, 1)
    st = s.status(reset=True)
    ref, info = chem.implicit_substep(mech, 2, U, 0.5 * dt)
    assert info["unconverged"] == 0
    assert st["newton_unconverged"] == 0 and st["nonphysical"] == 0
    got = from_gpu(op, out)
    rho = U[:, :5].sum(1, keepdim=True)
    assert float(((got[:, :5] - ref[:, :5]).abs() / rho).max()) < 1e-11
    # momentum and energy are copied bit for bit
    assert torch.equal(out[:, 5:], Ug[:, 5:])
    # the nodes that needed the continuation in h ran up to 25 iterations on
    # each of its 41 levels after the first 25
    print(f"implicit substep: oracle continued {info['continued']} nodes, max iterations oracle "
          f"{int(info['iters'].max())} library {st['newton_iters_max']}", flush=True)
    assert info["continued"] > 0
    assert st["newton_iters_max"] <= 25 * 42


def test_implicit_substep_fp32_in_place():
    """The two-pass implicit substep with a float state (double arithmetic)
    and in place (out = U) on the full workload: the species against the
    oracle at the float-rounded state to the float rounding of the output,
    the continued nodes included; momentum and energy untouched."""
    mech = di.preset_mechanism(P)
    op, s = make_pair(2, 3, P["nel"], P["lo"], P["hi"], physics="reacting", patch=(P["patch_lo"], P["patch_hi"]),
                      mech=mech, precision="f32")
    U = torch.tensor(di.reacting_state(op.mesh.coords(), P["lo"], P["hi"], mech))[None].float().double()
    Ug = to_gpu(s, U)
    h = 0.5 * dt_cfl(op, U, P["cfl"])
    s.status(reset=True)
    s.source_chem(Ug, Ug, h, 1)
    st = s.status(reset=True)
    ref, info = chem.implicit_substep(mech, 2, U, h)
    assert info["continued"] > 0 and info["unconverged"] == 0
    assert st["newton_unconverged"] == 0 and st["nonphysical"] == 0
    got = from_gpu(op, Ug)
    rho = U[:, :5].sum(1, keepdim=True)
    err = float(((got[:, :5] - ref[:, :5]).abs() / rho).max())
    print(f"FP32 implicit substep in place: species {err:.3e} of rho", flush=True)
    assert err < 2e-7
    assert torch.equal(got[:, 5:], U[:, 5:])


def test_strang_step_matches_oracle():
    """Two Strang steps S_{dt/2} T_dt S_{dt/2} on the full reacting workload
    (quiescent initial state, dt at CFL 0.5; the implicit substeps converge
    everywhere, a few per cent of the nodes through the continuation in h)."""
    mech, op, s, U = workload(moving=False)
    Ug = to_gpu(s, U)
    dt = s.dt_cfl(Ug, P["cfl"])
    for _ in range(2):
        U, i1 = chem.implicit_substep(mech, 2, U, 0.5 * dt)
        U = ssprk33_step(op, U, dt)
        U, i2 = chem.implicit_substep(mech, 2, U, 0.5 * dt)
        assert i1["unconverged"] == 0 and i2["unconverged"] == 0
        s.strang_step(Ug, dt)
    got = from_gpu(op, Ug)
    rho = U[:, :5].sum(1, keepdim=True)
    assert float(((got[:, :5] - U[:, :5]).abs() / rho).max()) < 1e-10
    assert rel_err(got[:, 5:], U[:, 5:]) < 1e-10
    st = s.status()
    assert st["newton_unconverged"] == 0 and st["nonphysical"] == 0


def test_strang_step_with_ssprk54_matches_oracle():
    """The paper's Strang step: the transport step T_dt taken with SSPRK54
    (at its larger SSP step, 1.508 x the SSP-RK3 CFL step), two steps on the
    full reacting workload against the oracle's SSPRK54 on the reacting
    operator, with the mortar patch and a moving state."""
    mech, op, s, U = workload()
    Ug = to_gpu(s, U)
    dt = 1.508 * s.dt_cfl(Ug, P["cfl"])
    t1, t2, t3 = s.empty(), s.empty(), s.empty()
    for _ in range(2):
        U, i1 = chem.implicit_substep(mech, 2, U, 0.5 * dt)
        U = ssprk54_step(op, U, dt)
        U, i2 = chem.implicit_substep(mech, 2, U, 0.5 * dt)
        assert i1["unconverged"] == 0 and i2["unconverged"] == 0
        s.strang_step(Ug, dt, t1, t2, t3, transport="ssprk54")
    got = from_gpu(op, Ug)
    rho = U[:, :5].sum(1, keepdim=True)
    err_y = float(((got[:, :5] - U[:, :5]).abs() / rho).max())
    err_m = rel_err(got[:, 5:], U[:, 5:])
    print(f"Strang with SSPRK54, two steps: species {err_y:.3e}, momentum/energy {err_m:.3e}", flush=True)
    assert err_y < 1e-10
    assert err_m < 1e-10
    st = s.status()
    assert st["newton_unconverged"] == 0 and st["nonphysical"] == 0


@pytest.mark.skipif(os.environ.get("DG_LONG", "0") != "1",
                    reason="full-length run (minutes of CPU oracle time): set DG_LONG=1")
def test_full_length_50_strang_steps():
    """The reacting workload at its full length: 50 Strang steps (SSP-RK3
    transport at CFL 0.5, implicit source half steps) on the full mesh with a
    moving state, against the oracle.  Every substep converges on both sides;
    species to 1e-10 of the density, momentum and energy to 1e-10 norm-wise."""
    mech, op, s, U = workload()
    Ug = to_gpu(s, U)
    dt = s.dt_cfl(Ug, P["cfl"])
    t1, t2 = s.empty(), s.empty()
    for k in range(50):
        U, i1 = chem.implicit_substep(mech, 2, U, 0.5 * dt)
        U = ssprk33_step(op, U, dt)
        U, i2 = chem.implicit_substep(mech, 2, U, 0.5 * dt)
        assert i1["unconverged"] == 0 and i2["unconverged"] == 0
        s.strang_step(Ug, dt, t1, t2)
        if k % 10 == 9:
            got = from_gpu(op, Ug)
            rho = U[:, :5].sum(1, keepdim=True)
            print(f"Strang step {k + 1}: species {float(((got[:, :5] - U[:, :5]).abs() / rho).max()):.3e}, "
                  f"momentum/energy {rel_err(got[:, 5:], U[:, 5:]):.3e}", flush=True)
    got = from_gpu(op, Ug)
    rho = U[:, :5].sum(1, keepdim=True)
    assert float(((got[:, :5] - U[:, :5]).abs() / rho).max()) < 1e-10
    assert rel_err(got[:, 5:], U[:, 5:]) < 1e-10
    st = s.status()
    assert st["newton_unconverged"] == 0 and st["nonphysical"] == 0
