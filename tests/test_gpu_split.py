"""GPU parity of the split-form stage (entropy-conservative volume integral
with Ranocha's two-point flux, Rusanov interfaces) against the oracle's
SplitOperator: every degree in 2-D and 3-D on rough states (partner states
far apart: the kernel's exact log-mean path), smooth states (the series
path only), a mix of both inside one wavefront, batched Shu-Osher stages,
the 2:1 mortar mesh, the FP32 form and the full 32^3 workload, plus free
stream, conservation and the unsupported combinations."""

import math

import numpy as np
import pytest
import torch

import dginputs as di
from oracle.timestep import rk_stage
from helpers import (make_pair, to_gpu, from_gpu, rel_err, random_euler_state, smooth_euler_state, rounding_spread,
                     spread_err, SPREAD_FACTOR)

pytestmark = pytest.mark.gpu
TOL64 = 1e-12
TWO_PI = 2 * math.pi


@pytest.mark.parametrize("dim,N", [(2, 1), (2, 2), (2, 3), (2, 4), (2, 5), (2, 6), (2, 7),
                                   (3, 1), (3, 2), (3, 3), (3, 4), (3, 5), (3, 6), (3, 7)])
def test_split_rhs_parity_all_degrees_rough(dim, N):
    nel = (7, 5) if dim == 2 else (5, 3, 3)
    lo, hi = (0.0,) * dim, (1.0, 1.3, 0.9)[:dim]
    op, s = make_pair(dim, N, nel, lo, hi, volume="split")
    U = random_euler_state(op, 300 + N)   # rho, p uniform in [0.5, 1.5]: most pairs far apart
    ref = op.rhs(U)
    got = from_gpu(op, s.rhs(to_gpu(s, U)))
    assert rel_err(got, ref) < TOL64


@pytest.mark.parametrize("dim,N", [(2, 3), (2, 5), (3, 2), (3, 3), (3, 4)])
def test_split_rhs_parity_smooth(dim, N):
    """Smooth state with 2 % density variation: every pair of every line
    within the log-mean series' range (u below 3e-4), the series path only."""
    nel = (9, 7) if dim == 2 else (5, 4, 3)
    lo, hi = (0.0,) * dim, (TWO_PI,) * dim
    op, s = make_pair(dim, N, nel, lo, hi, volume="split")
    U = torch.tensor(di.random_euler(op.mesh.coords(), lo, hi, drho=0.02))[None]
    ref = op.rhs(U)
    got = from_gpu(op, s.rhs(to_gpu(s, U)))
    assert rel_err(got, ref) < TOL64


def test_split_mixed_paths_within_a_wavefront():
    """A smooth state with isolated density and pressure spikes: inside one
    element some lanes take the exact log-mean path and the others do not."""
    op, s = make_pair(3, 3, (4, 4, 3), (0, 0, 0), (TWO_PI,) * 3, volume="split")
    U = smooth_euler_state(op)
    rng = np.random.default_rng(5)
    flat = U.reshape(1, 5, -1).clone()
    idx = torch.tensor(rng.choice(flat.shape[-1], size=flat.shape[-1] // 40, replace=False))
    flat[:, 0, idx] *= 1.6        # rho up by 60 %: velocity kept, so scale momentum too
    flat[:, 1:4, idx] *= 1.6
    flat[:, 4, idx] *= 1.3        # energy (and so p) up
    U = flat.reshape(U.shape)
    ref = op.rhs(U)
    got = from_gpu(op, s.rhs(to_gpu(s, U)))
    assert rel_err(got, ref) < TOL64


@pytest.mark.parametrize("dim", [2, 3])
def test_split_rk_stage_parity_batched(dim):
    nel = (6, 9) if dim == 2 else (4, 5, 3)
    lo, hi = (0.0,) * dim, (TWO_PI,) * dim
    op, s = make_pair(dim, 3, nel, lo, hi, batch=3, volume="split")
    U0 = smooth_euler_state(op, B=3)
    Uk = random_euler_state(op, 17, B=3)
    for (a, b, c) in ((0.0, 1.0, 0.01), (0.75, 0.25, 0.0025), (1 / 3, 2 / 3, 0.02 / 3)):
        ref = rk_stage(op, U0, Uk, a, b, c)
        out = s.empty()
        s.rk_stage(to_gpu(s, U0), to_gpu(s, Uk), out, a, b, c)
        assert rel_err(from_gpu(op, out), ref) < TOL64


def test_split_mortar_mesh_parity_and_conservation():
    op, s = make_pair(2, 3, (10, 8), (-5, -5), (5, 5), patch=((3, 2), (7, 5)), volume="split")
    U = torch.tensor(di.vortex(op.mesh.coords(), 0.0))[None]
    U = U + 0.05 * random_euler_state(op, 3)
    ref = op.rhs(U)
    dU = s.rhs(to_gpu(s, U))
    assert rel_err(from_gpu(op, dU), ref) < TOL64
    I = s.integrals(dU)
    scale = s.integrals(dU.abs())
    assert np.abs(I[:, :-1] / scale[:, :-1]).max() < 1e-13


def test_split_f32_parity():
    """FP32 storage: the oracle at the state the kernel reads; the pair
    fluxes are evaluated in double, so only the float output rounding and
    the float neighbour data remain."""
    op, s = make_pair(3, 3, (6, 5, 4), (0, 0, 0), (TWO_PI,) * 3, precision="f32", volume="split")
    U = smooth_euler_state(op)
    Ug = to_gpu(s, U)
    ref = op.rhs(from_gpu(op, Ug))
    got = from_gpu(op, s.rhs(Ug))
    assert rel_err(got, ref) < 1e-6


def test_split_full_size_workload_parity():
    """3-D Euler 32^3, N = 3, smooth random state: the launch shape the
    benchmark times.  dU/dt itself (mode 0) against the oracle, within 1e-12
    of each variable's norm or SPREAD_FACTOR times the oracle's own rounding
    spread at this state (mirror images and axis relabellings), whichever is
    larger; then the stage built on it."""
    p = di.PRESETS["euler3d"]
    op, s = make_pair(3, 3, p["nel"], p["lo"], p["hi"], volume="split")
    U = smooth_euler_state(op)
    Ug = to_gpu(s, U)
    ref, spread = rounding_spread(op.rhs, U, p["nel"], [(0,), (1,), (2,)], cycles=True)
    err = spread_err(from_gpu(op, s.rhs(Ug)), ref, spread)
    print(f"split 32^3 rhs: spread {spread.numpy()}, err/bound {err:.3f}", flush=True)
    assert err < 1.0
    dt = s.dt_cfl(Ug, p["cfl"])
    out = s.empty()
    s.rk_stage(None, Ug, out, 0.0, 1.0, dt)
    ref_stage = U + dt * ref
    assert rel_err(from_gpu(op, out), ref_stage) < TOL64


@pytest.mark.parametrize("nx,nz", [(5, 2), (5, 4), (64, 4)])
def test_split_block_orders_batched(nx, nz):
    """3-D meshes whose z-count selects the element-block orders of the
    stage kernel (groups of 2 and 4 whole z-planes taken z fastest; 64
    columns cut into tiles of 16), with a batch of 2, through the pairwise
    split sweep."""
    op, s = make_pair(3, 3, (nx, 3, nz), (0, 0, 0), (TWO_PI,) * 3, batch=2, volume="split")
    U = torch.cat([smooth_euler_state(op), random_euler_state(op, 40 + nz)])
    ref = op.rhs(U)
    got = from_gpu(op, s.rhs(to_gpu(s, U)))
    assert rel_err(got, ref) < TOL64


def test_split_free_stream_and_conservation_large():
    """64^3 at N = 3: a constant state gives dU/dt = 0 to rounding and a
    rough state a conservative right-hand side."""
    from paper_2605_26388_amd import Solver
    p = di.PRESETS["euler3d_L"]
    s = Solver(3, 3, p["nel"], p["lo"], p["hi"], volume="split")
    U = s.empty()
    U[:, 0] = 1.0
    U[:, 1] = 0.3
    U[:, 2] = -0.2
    U[:, 3] = 0.1
    U[:, 4] = 2.5 + 0.5 * (0.09 + 0.04 + 0.01)
    dU = s.rhs(U)
    assert float(dU.abs().max()) < 1e-13 * 3 * 9.1 * 2 / (TWO_PI / 64)
    g = torch.Generator(device=s.device).manual_seed(3)
    U[:, 0] += 0.2 * torch.rand(U[:, 0].shape, generator=g, device=s.device, dtype=U.dtype)
    dU = s.rhs(U)
    I = s.integrals(dU)
    scale = s.integrals(dU.abs())
    assert np.abs(I[:, :-1] / scale[:, :-1]).max() < 1e-12
    assert s.status()["nonphysical"] == 0


def test_split_rejected_where_unsupported():
    from paper_2605_26388_amd import Solver
    from paper_2605_26388_amd._abi import DGError, DG_ERR_UNSUPPORTED
    s = Solver(3, 3, (2, 2, 2), (0, 0, 0), (1, 1, 1), volume="split")
    U = s.empty()
    U.fill_(1.0)
    U[:, 4] = 2.5
    with pytest.raises(DGError) as e:
        s.rhs_adjoint(U, s.empty())
    assert e.value.code == DG_ERR_UNSUPPORTED
    with pytest.raises(DGError) as e:
        Solver(2, 3, (4, 4), (0, 0), (1, 1), physics="reacting", mech=di.preset_mechanism(di.PRESETS["air5_2d"]),
               volume="split")
    assert e.value.code == DG_ERR_UNSUPPORTED


@pytest.mark.parametrize("N", [2, 3, 4])
def test_split_navier_stokes_rhs_parity_small(N):
    """Split form with the BR1 viscous terms (the paper's Taylor-Green
    setting) on a rough state, N = 2, 3, 4 (one- and two-wave elements)."""
    op, s = make_pair(3, N, (3, 4, 3), (0, 0, 0), (1.0, 1.2, 0.9), physics="navier_stokes",
                      mu=2e-2, prandtl=0.72, volume="split")
    U = random_euler_state(op, 70 + N)
    ref = op.rhs(U)
    got = from_gpu(op, s.rhs(to_gpu(s, U)))
    assert rel_err(got, ref) < TOL64


def test_split_navier_stokes_tgv_full_workload():
    """The Taylor-Green workload (16^3, N = 4) with the split form: dU/dt
    within 1e-12 of each variable's norm or 16 oracle rounding spreads, the
    stage built on it, and conservation."""
    P = di.PRESETS["tgv3d"]
    op, s = make_pair(3, P["N"], P["nel"], P["lo"], P["hi"], physics="navier_stokes", mu=P["mu"],
                      prandtl=P["prandtl"], volume="split")
    U = torch.tensor(di.taylor_green(op.mesh.coords(), mach=P["mach"]))[None]
    Ug = to_gpu(s, U)
    ref, spread = rounding_spread(op.rhs, U, P["nel"], [(0,), (1,), (2,)], cycles=True)
    dU = s.rhs(Ug)
    err = spread_err(from_gpu(op, dU), ref, spread)
    print(f"split + BR1 TGV 16^3 N=4: spread {spread.numpy()}, err/bound {err:.3f}", flush=True)
    assert err < 1.0
    dt = s.dt_cfl(Ug, P["cfl"])
    out = s.empty()
    s.rk_stage(None, Ug, out, 0.0, 1.0, dt)
    # the stage adds dt L to U (whose z-momentum is zero): its rounding plus
    # dt times the right-hand side's bound
    floor = dt * SPREAD_FACTOR * spread + 2.0 ** -52 * U.reshape(1, 5, -1).abs().amax(dim=(0, 2))
    assert spread_err(from_gpu(op, out), U + dt * ref, floor / SPREAD_FACTOR) < 1.0
    I = s.integrals(dU)[:, :-1]
    vol = float(np.prod(np.subtract(P["hi"], P["lo"])))
    from helpers import flux_scale
    scale = np.maximum(s.integrals(dU.abs())[:, :-1], vol * flux_scale(op, U).numpy()[None])
    assert np.abs(I / scale).max() < 1e-13
    assert s.status()["nonphysical"] == 0
