"""GPU parity of the SSPRK54 path (dg_rk_stage_dual, dg_ssprk54_step) and of
the per-stage positivity floor against the oracle: the dual stage's two
combinations (in place and out of place, Euler 2-D/3-D incl. mortars,
Navier-Stokes, FP32), whole SSPRK54 steps (standard and split volume
integrals, Navier-Stokes, batches, the full 32^3 workload), the floor on
stage outputs with the count of floored nodes, and the argument checks."""

import math

import numpy as np
import pytest
import torch

import dginputs as di
from oracle.ssprk54 import positivity_floor, ssprk54_step
from oracle.timestep import rk_stage
from helpers import (make_pair, to_gpu, from_gpu, rel_err, rel_err_floor, flux_scale, random_euler_state,
                     smooth_euler_state)

pytestmark = pytest.mark.gpu
TOL64 = 1e-12
TWO_PI = 2 * math.pi


@pytest.mark.parametrize("dim,patch", [(3, None), (2, ((2, 2), (5, 4)))])
def test_dual_stage_parity(dim, patch):
    nel = (5, 4, 3) if dim == 3 else (8, 7)
    lo, hi = (0.0,) * dim, (1.0, 1.3, 0.9)[:dim]
    op, s = make_pair(dim, 3, nel, lo, hi, batch=2, patch=patch)
    U0 = random_euler_state(op, 1, B=2)
    Uk = random_euler_state(op, 2, B=2)
    V = random_euler_state(op, 3, B=2)
    a, b, c, a2, b2, c2 = 0.178, 0.822, 0.0054, 0.517, 0.096, 0.00064
    ref1 = rk_stage(op, U0, Uk, a, b, c)
    ref2 = rk_stage(op, V, Uk, a2, b2, c2)
    o1, o2 = s.empty(), s.empty()
    s.rk_stage_dual(to_gpu(s, U0), to_gpu(s, Uk), o1, a, b, c, to_gpu(s, V), o2, a2, b2, c2)
    assert rel_err(from_gpu(op, o1), ref1) < TOL64
    assert rel_err(from_gpu(op, o2), ref2) < TOL64
    # in place on U0 and on V (the SSPRK54 use)
    g0, gv = to_gpu(s, U0), to_gpu(s, V)
    s.rk_stage_dual(g0, to_gpu(s, Uk), g0, a, b, c, gv, gv, a2, b2, c2)
    assert rel_err(from_gpu(op, g0), ref1) < TOL64
    assert rel_err(from_gpu(op, gv), ref2) < TOL64
    # a2 = 0: V is not read
    o1, o2 = s.empty(), s.empty()
    s.rk_stage_dual(None, to_gpu(s, Uk), o1, 0.0, 1.0, c, None, o2, 0.0, b2, c2)
    assert rel_err(from_gpu(op, o2), rk_stage(op, Uk, Uk, 0.0, b2, c2)) < TOL64


def test_dual_stage_navier_stokes_and_f32():
    p = di.PRESETS["tgv3d"]
    op, s = make_pair(3, 3, (4, 4, 3), p["lo"], p["hi"], physics="navier_stokes", mu=p["mu"],
                      prandtl=p["prandtl"])
    X = op.mesh.coords()
    U = torch.tensor(di.taylor_green(X, mach=p["mach"]))[None]
    V = smooth_euler_state(op)
    ref1 = rk_stage(op, U, U, 0.0, 1.0, 1e-3)
    ref2 = rk_stage(op, V, U, 0.5, 0.25, 2e-4)
    o1, o2 = s.empty(), s.empty()
    s.rk_stage_dual(None, to_gpu(s, U), o1, 0.0, 1.0, 1e-3, to_gpu(s, V), o2, 0.5, 0.25, 2e-4)
    floor = flux_scale(op, U) * 1e-3 * 1e-3
    assert rel_err_floor(from_gpu(op, o1), ref1, floor) < TOL64
    assert rel_err_floor(from_gpu(op, o2), ref2, floor) < TOL64
    op, s = make_pair(3, 3, (5, 4, 3), (0, 0, 0), (TWO_PI,) * 3, precision="f32")
    U = smooth_euler_state(op)
    Ug = to_gpu(s, U)
    Uq = from_gpu(op, Ug)
    o1, o2 = s.empty(), s.empty()
    s.rk_stage_dual(Ug, Ug, o1, 0.25, 0.75, 0.01, Ug, o2, 0.5, 0.5, 0.003)
    assert rel_err(from_gpu(op, o1), rk_stage(op, Uq, Uq, 0.25, 0.75, 0.01)) < 1e-6
    assert rel_err(from_gpu(op, o2), rk_stage(op, Uq, Uq, 0.5, 0.5, 0.003)) < 1e-6


def test_dual_stage_argument_checks():
    from paper_2605_26388_amd._abi import DGError, DG_ERR_ARG
    op, s = make_pair(3, 2, (2, 2, 2), (0, 0, 0), (1, 1, 1))
    U = to_gpu(s, random_euler_state(op, 1))
    o = s.empty()
    for args in ((U, U, o, 0.5, 0.5, 0.1, U, U, 0.5, 0.5, 0.1),       # Wout aliases Uk
                 (U, U, o, 0.5, 0.5, 0.1, U, o, 0.5, 0.5, 0.1),       # outputs overlap
                 (None, U, o, 0.5, 0.5, 0.1, U, s.empty(), 0.5, 0.5, 0.1)):
        with pytest.raises((DGError, ValueError)) as e:
            s.rk_stage_dual(*args)
        if isinstance(e.value, DGError):
            assert e.value.code == DG_ERR_ARG


@pytest.mark.parametrize("volume", ["standard", "split"])
@pytest.mark.parametrize("dim", [2, 3])
def test_ssprk54_step_parity(dim, volume):
    nel = (6, 5) if dim == 2 else (4, 3, 3)
    lo, hi = (0.0,) * dim, (TWO_PI,) * dim
    op, s = make_pair(dim, 3, nel, lo, hi, batch=2, volume=volume)
    U = smooth_euler_state(op, B=2)
    Ug = to_gpu(s, U)
    dt = s.dt_cfl(Ug, 1.0)   # SSP coefficient 1.5: CFL 1 is inside its bound
    ref = ssprk54_step(op, U, dt)
    s.ssprk54_step(Ug, dt)
    assert rel_err(from_gpu(op, Ug), ref) < TOL64


def test_ssprk54_step_parity_mortar_and_navier_stokes():
    op, s = make_pair(2, 3, (10, 8), (-5, -5), (5, 5), patch=((3, 2), (7, 5)))
    U = torch.tensor(di.vortex(op.mesh.coords(), 0.0))[None]
    Ug = to_gpu(s, U)
    dt = s.dt_cfl(Ug, 1.0)
    ref = ssprk54_step(op, U, dt)
    s.ssprk54_step(Ug, dt)
    assert rel_err(from_gpu(op, Ug), ref) < TOL64
    p = di.PRESETS["tgv3d"]
    op, s = make_pair(3, 4, (3, 3, 3), p["lo"], p["hi"], physics="navier_stokes", mu=p["mu"], prandtl=p["prandtl"])
    U = torch.tensor(di.taylor_green(op.mesh.coords(), mach=p["mach"]))[None]
    Ug = to_gpu(s, U)
    dt = s.dt_cfl(Ug, 1.0)
    ref = ssprk54_step(op, U, dt)
    s.ssprk54_step(Ug, dt)
    assert rel_err(from_gpu(op, Ug), ref) < TOL64


def test_ssprk54_full_size_workload():
    """32^3, N = 3 smooth random state, CFL 0.75, the benchmark's launch shape."""
    p = di.PRESETS["euler3d"]
    op, s = make_pair(3, 3, p["nel"], p["lo"], p["hi"])
    U = smooth_euler_state(op)
    Ug = to_gpu(s, U)
    dt = s.dt_cfl(Ug, 0.75)
    ref = ssprk54_step(op, U, dt)
    t1, t2, t3 = s.empty(), s.empty(), s.empty()
    s.ssprk54_step(Ug, dt, t1, t2, t3)
    assert rel_err(from_gpu(op, Ug), ref) < TOL64
    # the step conserves (periodic box)
    I0 = s.integrals(to_gpu(s, U))
    I1 = s.integrals(Ug)
    assert np.abs(I1[:, :-1] - I0[:, :-1]).max() < 1e-12 * np.abs(I0[:, :-1]).max()


def _near_vacuum_state(op, seed, B=1):
    """Smooth flow with a sprinkle of nodes at very low density and pressure
    and strong velocity, so that a stage drives some nodes below the floor."""
    U = smooth_euler_state(op, B=B).clone()
    rng = np.random.default_rng(seed)
    flat = U.reshape(B, op.phys.nv, -1)
    idx = torch.tensor(rng.choice(flat.shape[-1], size=flat.shape[-1] // 25, replace=False))
    rho = 1e-5
    flat[:, 0, idx] = rho
    flat[:, 1:-1, idx] = 0.0
    flat[:, 1, idx] = rho * 2.0                    # velocity (2, 0, 0)
    flat[:, -1, idx] = 1e-6 / 0.4 + 0.5 * rho * 4.0  # p = 1e-6
    return flat.reshape(U.shape)


@pytest.mark.parametrize("physics", ["euler", "navier_stokes"])
def test_positivity_floor_on_stage_outputs(physics):
    rmin, pmin = 1e-6, 5e-7
    kw = dict(mu=1e-3, prandtl=0.72) if physics == "navier_stokes" else {}
    op, s = make_pair(3, 3, (4, 4, 3), (0, 0, 0), (TWO_PI,) * 3, physics=physics, **kw)
    from paper_2605_26388_amd import Solver
    sf = Solver(3, 3, (4, 4, 3), (0, 0, 0), (TWO_PI,) * 3, physics=physics, rho_floor=rmin, p_floor=pmin, **kw)
    U = _near_vacuum_state(op, 7)
    Ug = to_gpu(sf, U)
    dt = 2e-3
    raw = rk_stage(op, U, U, 0.0, 1.0, dt)
    ref = positivity_floor(raw, 1.4, rmin, pmin)
    nfloored = int((ref != raw).any(dim=1).sum())
    assert nfloored > 0
    sf.status(reset=True)
    out = sf.empty()
    sf.rk_stage(None, Ug, out, 0.0, 1.0, dt)
    got = from_gpu(op, out)
    assert rel_err(got, ref) < TOL64
    assert sf.status()["floored"] == nfloored
    # dg_rhs is never floored, and a context without floors leaves the stage alone
    assert rel_err(from_gpu(op, sf.rhs(Ug)), op.rhs(U)) < TOL64
    out0 = s.empty()
    s.rk_stage(None, to_gpu(s, U), out0, 0.0, 1.0, dt)
    assert rel_err(from_gpu(op, out0), raw) < TOL64
    assert s.status()["floored"] == 0


def test_positivity_floor_fp32_form():
    """FP32 form: the stage combination in float, the floor itself in double,
    the result rounded to float.  The floored output matches the oracle's
    floored FP64 stage at the same (float) state to the form's accuracy, and
    the bounds hold up to float rounding."""
    rmin, pmin = 1e-6, 5e-7
    op, _ = make_pair(3, 3, (4, 4, 3), (0, 0, 0), (TWO_PI,) * 3)
    from paper_2605_26388_amd import Solver
    sf = Solver(3, 3, (4, 4, 3), (0, 0, 0), (TWO_PI,) * 3, precision="f32", rho_floor=rmin, p_floor=pmin)
    U = _near_vacuum_state(op, 7).float().double()
    dt = 2e-3
    raw = rk_stage(op, U, U, 0.0, 1.0, dt)
    ref = positivity_floor(raw, 1.4, rmin, pmin)
    nfloored = int((ref != raw).any(dim=1).sum())
    assert nfloored > 0
    sf.status(reset=True)
    out = sf.empty()
    sf.rk_stage(None, to_gpu(sf, U), out, 0.0, 1.0, dt)
    got = from_gpu(op, out)
    err = rel_err(got, ref)
    print(f"FP32 floored stage error: {err:.3e}; floored {sf.status()['floored']} (oracle {nfloored})")
    assert err < 1e-5
    assert abs(sf.status()["floored"] - nfloored) <= max(1, nfloored // 100)
    P = op.phys.prims(got)
    assert float(P["rho"].min()) >= rmin * (1 - 2.0 ** -23)
    slack = 8 * 2.0 ** -24 * 0.4 * P["E"].abs()
    assert bool((P["p"] >= pmin - slack).all())


def test_floored_ssprk54_step():
    rmin, pmin = 1e-6, 5e-7
    op, _ = make_pair(3, 3, (4, 3, 3), (0, 0, 0), (TWO_PI,) * 3)
    from paper_2605_26388_amd import Solver
    s = Solver(3, 3, (4, 3, 3), (0, 0, 0), (TWO_PI,) * 3, batch=2, rho_floor=rmin, p_floor=pmin)
    U = _near_vacuum_state(op, 9, B=2)
    Ug = to_gpu(s, U)
    dt = 1e-3
    ref = ssprk54_step(op, U, dt, floor=(rmin, pmin))
    s.ssprk54_step(Ug, dt)
    assert rel_err(from_gpu(op, Ug), ref) < TOL64
    assert s.status()["floored"] > 0
    # the bounds hold up to the rounding of E: where the clipped density
    # leaves a large kinetic energy, p = (gamma-1)(E - ke) cancels
    P = op.phys.prims(from_gpu(op, Ug))
    assert float(P["rho"].min()) >= rmin
    slack = 8 * 2.0 ** -52 * 0.4 * P["E"].abs()
    assert bool((P["p"] >= pmin - slack).all())
