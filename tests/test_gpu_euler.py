"""GPU parity of the fused Euler stage (dg_rhs / dg_rk_stage) against the CPU
FP64 oracle: element by element on small meshes (several workgroups and a
ragged tail), every supported degree, batches, the 2:1 mortar mesh, the full
32^3 workload, and the invariants (free stream, conservation, determinism,
complete output coverage, non-physical state flagging, argument errors)."""

import math

import numpy as np
import pytest
import torch

import dginputs as di
from oracle.timestep import rk_stage, ssprk33_step, integrals
from helpers import make_pair, to_gpu, from_gpu, rel_err, random_euler_state, smooth_euler_state

pytestmark = pytest.mark.gpu
TOL64 = 1e-12
TWO_PI = 2 * math.pi


@pytest.mark.parametrize("dim,N", [(2, 1), (2, 2), (2, 3), (2, 4), (2, 5), (2, 6), (2, 7),
                                   (3, 1), (3, 2), (3, 3), (3, 4), (3, 5), (3, 6), (3, 7)])
def test_rhs_parity_all_degrees(dim, N):
    nel = (7, 5) if dim == 2 else (5, 3, 3)   # element counts leave a ragged last workgroup
    lo = (0.0,) * dim
    hi = (1.0, 1.3, 0.9)[:dim]
    op, s = make_pair(dim, N, nel, lo, hi)
    U = random_euler_state(op, 100 + N)
    ref = op.rhs(U)
    got = from_gpu(op, s.rhs(to_gpu(s, U)))
    assert rel_err(got, ref) < TOL64


@pytest.mark.parametrize("N,nel", [(3, (3, 2, 2)), (3, (2, 3, 6)), (3, (3, 3, 4)), (3, (2, 2, 8)), (5, (3, 2, 2)),
                                   (4, (2, 3, 4)), (3, (64, 2, 4)), (3, (128, 3, 2))])
def test_rhs_parity_block_orders(N, nel):
    """3-D meshes whose z-count selects each order of the element blocks
    (groups of 2 or 4 z-planes taken z fastest; plain order for odd counts is
    covered above; 64 and 128 columns in x cut the groups into tiles of 16
    columns), batched so that a group boundary falls between members."""
    op, s = make_pair(3, N, nel, (0.0, 0.0, 0.0), (1.0, 0.8, 1.2), batch=2)
    U = random_euler_state(op, 40 + N, B=2)
    ref = op.rhs(U)
    got = from_gpu(op, s.rhs(to_gpu(s, U)))
    assert rel_err(got, ref) < TOL64


def _tile4(X, n16=16):
    """A (B, nv, E, Np) state of a 16^3 mesh repeated 4 times along each
    element axis (lexicographic element order, x fastest)."""
    B, nv, _, Np = X.shape
    Y = X.reshape(B, nv, n16, n16, n16, Np).repeat(1, 1, 4, 4, 4, 1)
    return Y.reshape(B, nv, -1, Np).contiguous()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_64cubed_as_tiled_16cubed(precision):
    """64^3, N = 3: states beyond the 256 MiB Infinity Cache, where the stage
    kernel takes the non-temporal cache policy for U0 and the output and
    cuts the element groups into tiles of 16 columns.  A state that repeats
    a 16^3 state 4 times along each axis, on a box 4 times as long (the same
    element sizes, the same arithmetic per element), must give the 16^3
    right-hand side and stage output repeated, bit for bit; the 16^3 FP64
    right-hand side itself is checked against the oracle."""
    from paper_2605_26388_amd import Solver
    op, s16 = make_pair(3, 3, (16, 16, 16), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), precision=precision)
    U = random_euler_state(op, 77)
    U0 = random_euler_state(op, 78)
    g16, g016 = to_gpu(s16, U), to_gpu(s16, U0)
    d16 = s16.rhs(g16)
    if precision == "f64":
        assert rel_err(from_gpu(op, d16), op.rhs(U)) < TOL64
    o16 = s16.empty()
    s16.rk_stage(g016, g16, o16, 0.75, 0.25, 0.0025)
    d16, o16 = d16.cpu(), o16.cpu()
    del g16, g016
    s16.close()
    s64 = Solver(3, 3, (64, 64, 64), (0.0, 0.0, 0.0), (4.0, 4.0, 4.0), precision=precision)
    g64 = _tile4(U.reshape(1, 5, 4096, 64)).to(s64.device, s64.dtype)
    g064 = _tile4(U0.reshape(1, 5, 4096, 64)).to(s64.device, s64.dtype)
    d64 = s64.rhs(g64)
    assert torch.equal(d64.cpu(), _tile4(d16))
    del d64
    o64 = s64.empty()
    s64.rk_stage(g064, g64, o64, 0.75, 0.25, 0.0025)
    assert torch.equal(o64.cpu(), _tile4(o16))
    assert s64.status()["nonphysical"] == 0
    s64.close()


@pytest.mark.parametrize("dim", [2, 3])
def test_rk_stage_parity_batched(dim):
    nel = (6, 9) if dim == 2 else (4, 5, 3)
    lo, hi = (0.0,) * dim, (TWO_PI,) * dim
    op, s = make_pair(dim, 3, nel, lo, hi, batch=3)
    U0 = smooth_euler_state(op, B=3)
    Uk = random_euler_state(op, 7, B=3)
    for (a, b, c) in ((0.0, 1.0, 0.01), (0.75, 0.25, 0.0025), (1 / 3, 2 / 3, 0.02 / 3)):
        ref = rk_stage(op, U0, Uk, a, b, c)
        out = s.empty()
        s.rk_stage(to_gpu(s, U0), to_gpu(s, Uk), out, a, b, c)
        assert rel_err(from_gpu(op, out), ref) < TOL64


def test_rk_stage_in_place_on_U0():
    op, s = make_pair(3, 3, (3, 4, 3), (0, 0, 0), (1, 1, 1))
    U0 = random_euler_state(op, 1)
    Uk = random_euler_state(op, 2)
    ref = rk_stage(op, U0, Uk, 1 / 3, 2 / 3, 0.01)
    g0 = to_gpu(s, U0)
    s.rk_stage(g0, to_gpu(s, Uk), g0, 1 / 3, 2 / 3, 0.01)
    assert rel_err(from_gpu(op, g0), ref) < TOL64


def test_mortar_mesh_parity_and_conservation():
    op, s = make_pair(2, 3, (10, 8), (-5, -5), (5, 5), patch=((3, 2), (7, 5)))
    U = torch.tensor(di.vortex(op.mesh.coords(), 0.0))[None]
    U = U + 0.05 * random_euler_state(op, 3)  # rough on top of smooth
    ref = op.rhs(U)
    dU = s.rhs(to_gpu(s, U))
    assert rel_err(from_gpu(op, dU), ref) < TOL64
    I = s.integrals(dU)
    scale = s.integrals(dU.abs())
    assert np.abs(I[:, :-1] / scale[:, :-1]).max() < 1e-13


def test_full_size_workload_parity():
    """3-D Euler 32^3, N=3 smooth random state, the benchmark's launch shape."""
    p = di.PRESETS["euler3d"]
    op, s = make_pair(3, 3, p["nel"], p["lo"], p["hi"])
    U = smooth_euler_state(op)
    ref = op.rhs(U)
    Ug = to_gpu(s, U)
    got = from_gpu(op, s.rhs(Ug))
    assert rel_err(got, ref) < TOL64
    dt = s.dt_cfl(Ug, p["cfl"])
    out = s.empty()
    s.rk_stage(None, Ug, out, 0.0, 1.0, dt)
    refs = rk_stage(op, U, U, 0.0, 1.0, dt)
    assert rel_err(from_gpu(op, out), refs) < TOL64


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_stage_parity_large_batched_mesh(precision):
    """17x16x16 elements at N=3 with a batch of 2 (8704 workgroups, more than
    the device holds at once): the Shu-Osher stage with distinct U0 per
    member, in both precisions, against the oracle at the state the kernel
    reads."""
    op, s = make_pair(3, 3, (17, 16, 16), (0, 0, 0), (TWO_PI,) * 3, batch=2, precision=precision)
    U = smooth_euler_state(op, B=2)
    U0 = smooth_euler_state(op, B=2).flip(0).contiguous()
    Ug, U0g = to_gpu(s, U), to_gpu(s, U0)
    out = s.empty()
    dt = 1e-3
    s.rk_stage(U0g, Ug, out, 0.75, 0.25, 0.25 * dt)
    # the oracle at the state the kernel actually reads
    Uq = from_gpu(op, Ug)
    U0q = from_gpu(op, U0g)
    ref = rk_stage(op, U0q, Uq, 0.75, 0.25, 0.25 * dt)
    tol = TOL64 if precision == "f64" else 1e-6
    assert rel_err(from_gpu(op, out), ref) < tol


def test_large_workload_invariants():
    """64^3: free stream is preserved and the RHS is conservative."""
    p = di.PRESETS["euler3d_L"]
    from paper_2605_26388_amd import Solver
    s = Solver(3, 3, p["nel"], p["lo"], p["hi"])
    U = s.empty()
    U[:, 0] = 1.0
    U[:, 1] = 0.3
    U[:, 2] = -0.2
    U[:, 3] = 0.1
    U[:, 4] = 2.5 + 0.5 * (0.09 + 0.04 + 0.01)
    dU = s.rhs(U)
    assert float(dU.abs().max()) < 1e-13 * 3 * 9.1 * 2 / (TWO_PI / 64)
    # conservation on a smooth state built from the library's own coordinates
    X = s.node_coords().cpu().numpy()
    Us = torch.tensor(di.random_euler(X, p["lo"], p["hi"]))[None].to(s.device).contiguous()
    dU = s.rhs(Us)
    I = s.integrals(dU)
    scale = s.integrals(dU.abs())
    assert np.abs(I[:, :-1] / np.maximum(scale[:, :-1], 1e-300)).max() < 1e-13
    st = s.status()
    assert st["nonphysical"] == 0


def test_determinism_and_full_coverage():
    op, s = make_pair(3, 4, (3, 5, 2), (0, 0, 0), (1, 2, 1))
    U = random_euler_state(op, 5)
    Ug = to_gpu(s, U)
    a = torch.full(s.shape, float("nan"), dtype=s.dtype, device=s.device)
    b = torch.full(s.shape, float("nan"), dtype=s.dtype, device=s.device)
    s.rhs(Ug, a)
    s.rhs(Ug, b)
    assert not torch.isnan(a).any()
    assert torch.equal(a, b)


def test_nonphysical_flagged_and_reported():
    op, s = make_pair(3, 2, (3, 3, 3), (0, 0, 0), (1, 1, 1))
    U = random_euler_state(op, 9)
    U[0, 0, 13, 1, 2, 0] = -0.5          # negative density at element 13
    s.status(reset=True)
    s.rhs(to_gpu(s, U))
    st = s.status(reset=True)
    assert st["nonphysical"] == 1
    assert st["first_bad"] == 13 * 27 + (1 * 9 + 2 * 3 + 0)
    assert s.status()["nonphysical"] == 0


def test_argument_errors():
    from paper_2605_26388_amd import DGError
    op, s = make_pair(2, 3, (3, 3), (0, 0), (1, 1))
    U = to_gpu(s, random_euler_state(op, 1))
    with pytest.raises(DGError):
        s.rk_stage(None, U, U, 0.0, 1.0, 0.1)     # Uout aliases Uk
    with pytest.raises(DGError):
        s.rhs(U, U)
    with pytest.raises(ValueError):
        s.rhs(U.float())


def test_integrals_and_dt_match_oracle():
    from oracle.timestep import dt_cfl
    op, s = make_pair(2, 3, (8, 8), (-5, -5), (5, 5), batch=2)
    U = torch.cat([torch.tensor(di.vortex(op.mesh.coords(), 0.0))[None],
                   torch.tensor(di.vortex(op.mesh.coords(), 1.0))[None]])
    Ug = to_gpu(s, U)
    I = s.integrals(Ug)
    Iref = integrals(op, U)
    assert np.abs(I - Iref).max() <= 1e-13 * np.abs(Iref).max()
    assert abs(s.dt_cfl(Ug, 0.5) / dt_cfl(op, U, 0.5) - 1) < 1e-14
    X = s.node_coords().cpu().numpy().reshape((2, op.mesh.E) + (4, 4))
    assert np.abs(X - op.mesh.coords()).max() < 1e-14


def test_vortex_run_matches_oracle():
    """The 2-D vortex workload (8^2, N=3): 20 SSP-RK3 steps at CFL 0.5."""
    p = di.PRESETS["vortex2d"]
    op, s = make_pair(2, 3, p["nel"], p["lo"], p["hi"])
    U = torch.tensor(di.vortex(op.mesh.coords(), 0.0))[None]
    Ug = to_gpu(s, U)
    dt = s.dt_cfl(Ug, p["cfl"])
    for _ in range(p["steps"]):
        U = ssprk33_step(op, U, dt)
        s.ssprk3_step(Ug, dt)
    assert rel_err(from_gpu(op, Ug), U) < TOL64
    # density error against the exact translated vortex is the discretisation's
    ex = torch.tensor(di.vortex(op.mesh.coords(), p["steps"] * dt))[None]
    got = from_gpu(op, Ug)
    assert float((got[0, 0] - ex[0, 0]).abs().max()) < 5e-2   # 8^2 elements, h = 1.25


def _tile2(X, n16=16):
    """A (B, nv, E, Np) state of a 16^3 mesh repeated twice along each element
    axis (lexicographic element order, x fastest)."""
    B, nv, _, Np = X.shape
    Y = X.reshape(B, nv, n16, n16, n16, Np).repeat(1, 1, 2, 2, 2, 1)
    return Y.reshape(B, nv, -1, Np).contiguous()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_dual_stage_32cubed_as_tiled_16cubed(precision):
    """The dual stage (two combinations of one L(U_k), SSPRK54's fourth stage)
    at 32^3, N = 3, reading V: there the FP64 stage's five 84 MB streams exceed
    the 256 MiB Infinity Cache, so the kernel takes the non-temporal policy,
    and V is loaded at entry.  A state that repeats a 16^3 state twice along
    each axis, on a box twice as long (the same element sizes and arithmetic
    per element), must give both 16^3 outputs repeated, bit for bit; the 16^3
    outputs themselves are checked against the oracle's stage."""
    from paper_2605_26388_amd import Solver
    op, s16 = make_pair(3, 3, (16, 16, 16), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), precision=precision)
    U, U0, V = (random_euler_state(op, sd) for sd in (81, 82, 83))
    a, b, c, a2, b2, c2 = 0.4, 0.6, 0.003, 0.3, 0.5, 0.002
    g16, g016, gv16 = to_gpu(s16, U), to_gpu(s16, U0), to_gpu(s16, V)
    o16, w16 = s16.empty(), s16.empty()
    s16.rk_stage_dual(g016, g16, o16, a, b, c, gv16, w16, a2, b2, c2)
    if precision == "f64":
        Uq = from_gpu(op, g16)
        L = op.rhs(Uq)
        assert rel_err(from_gpu(op, o16), a * from_gpu(op, g016) + b * Uq + c * L) < TOL64
        assert rel_err(from_gpu(op, w16), a2 * from_gpu(op, gv16) + b2 * Uq + c2 * L) < TOL64
    o16, w16 = o16.cpu(), w16.cpu()
    s16.close()
    s32 = Solver(3, 3, (32, 32, 32), (0.0, 0.0, 0.0), (2.0, 2.0, 2.0), precision=precision)
    t = lambda X: _tile2(X.reshape(1, 5, 4096, 64)).to(s32.device, s32.dtype)
    o32, w32 = s32.empty(), s32.empty()
    s32.rk_stage_dual(t(U0), t(U), o32, a, b, c, t(V), w32, a2, b2, c2)
    assert torch.equal(o32.cpu(), _tile2(o16))
    assert torch.equal(w32.cpu(), _tile2(w16))
    assert s32.status()["nonphysical"] == 0
    s32.close()
