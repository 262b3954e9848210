"""GPU parity of the two-temperature reacting path against the oracle: the
2-D stage with the E_v column and the 2:1 mortar patch, the source (mode 0:
species rows and the E_v row with Landau-Teller relaxation and the
vibrational energy of the produced molecules), the implicit substep on
(rho_s, E_v) (mode 1), and Strang steps, on the two-temperature version of
the reacting workload (64^2 + refined 16^2 block, N = 3, 5-species air)."""

import math

import numpy as np
import pytest
import torch

import dginputs as di
from oracle import twotemp
from oracle.timestep import rk_stage, ssprk33_step, dt_cfl
from helpers import make_pair, to_gpu, from_gpu, rel_err

pytestmark = pytest.mark.gpu
P = di.PRESETS["air5_2t_2d"]


def workload(nel=None, patch=None, u0=250.0):
    mech = di.preset_mechanism(P)
    vib = di.air5_vibration(mech)
    nel = nel or P["nel"]
    patch = patch or (P["patch_lo"], P["patch_hi"])
    op, s = make_pair(2, 3, nel, P["lo"], P["hi"], physics="reacting_2t", patch=patch, mech=mech, vib=vib)
    U = torch.tensor(di.reacting2t_state(op.mesh.coords(), P["lo"], P["hi"], mech, vib, u0=u0))[None]
    return mech, vib, op, s, U


def test_2t_rhs_parity_small_and_conservative():
    mech, vib, op, s, U = workload(nel=(10, 8), patch=((3, 2), (7, 5)))
    ref = op.rhs(U)
    dU = s.rhs(to_gpu(s, U))
    assert rel_err(from_gpu(op, dU), ref) < 1e-12
    I = s.integrals(dU)[:, :-1]
    scale = s.integrals(dU.abs())[:, :-1]
    assert np.abs(I / scale).max() < 1e-13


def test_2t_stage_parity_full_workload():
    mech, vib, op, s, U = workload()
    Ug = to_gpu(s, U)
    dt = s.dt_cfl(Ug, P["cfl"])
    assert abs(dt / dt_cfl(op, U, P["cfl"]) - 1.0) < 1e-13
    out = s.empty()
    s.rk_stage(None, Ug, out, 0.0, 1.0, dt)
    ref = rk_stage(op, U, U, 0.0, 1.0, dt)
    assert rel_err(from_gpu(op, out), ref) < 1e-12
    assert s.status()["nonphysical"] == 0


def test_2t_source_mode0_parity():
    mech, vib, op, s, U = workload(u0=0.0)
    Ug = to_gpu(s, U)
    out = torch.zeros_like(Ug)
    s.source_chem(Ug, out, 0.0, 0)
    ref = twotemp.source(op.phys, U)
    got = from_gpu(op, out)
    assert rel_err(got[:, :5], ref[:, :5]) < 1e-12
    assert rel_err(got[:, 8:], ref[:, 8:]) < 1e-12
    assert float(got[:, 5:8].abs().max()) == 0.0
    # accumulates in place
    U2 = to_gpu(s, U)
    s.source_chem(U2, U2, 0.0, 0)
    assert rel_err(from_gpu(op, U2), U + ref) < 1e-12


def test_2t_implicit_substep_parity_full_workload():
    mech, vib, op, s, U = workload(u0=0.0)
    Ug = to_gpu(s, U)
    dt = s.dt_cfl(Ug, P["cfl"])
    out = s.empty()
    s.status(reset=True)
    s.source_chem(Ug, out, 0.5 * dt, 1)
    st = s.status(reset=True)
    ref, info = twotemp.implicit_substep(op.phys, U, 0.5 * dt)
    assert info["unconverged"] == 0
    assert st["newton_unconverged"] == 0 and st["nonphysical"] == 0
    assert st["newton_iters_max"] == int(info["iters"].max())
    got = from_gpu(op, out)
    rho = U[:, :5].sum(1, keepdim=True)
    assert float(((got[:, :5] - ref[:, :5]).abs() / rho).max()) < 1e-11
    assert rel_err(got[:, 8:], ref[:, 8:]) < 1e-11
    assert torch.equal(out[:, 5:8], Ug[:, 5:8])                   # momentum and E copied


def test_2t_strang_steps_match_oracle():
    """Two Strang steps on the full workload at its CFL step, where every node
    converges within a dozen Newton iterations.  (At a few times that step
    single stiff nodes need tens of iterations and their Newton path depends
    on rounding, so iteration counts are not comparable there.)"""
    mech, vib, op, s, U = workload()
    Ug = to_gpu(s, U)
    dt = s.dt_cfl(Ug, P["cfl"])
    for _ in range(2):
        U, i1 = twotemp.implicit_substep(op.phys, U, 0.5 * dt)
        U = ssprk33_step(op, U, dt)
        U, i2 = twotemp.implicit_substep(op.phys, U, 0.5 * dt)
        assert i1["unconverged"] == 0 and i2["unconverged"] == 0
        s.strang_step(Ug, dt)
    got = from_gpu(op, Ug)
    rho = U[:, :5].sum(1, keepdim=True)
    assert float(((got[:, :5] - U[:, :5]).abs() / rho).max()) < 1e-10
    assert rel_err(got[:, 5:], U[:, 5:]) < 1e-10
    st = s.status()
    assert st["newton_unconverged"] == 0 and st["nonphysical"] == 0
